// NTT / iNTT kernels and launchers (see ntt_core.h for the decomposition).
#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "ntt_core.h"

namespace he {

// Rounds IDX..NR-1 of a pass, forward order (integer or FP64 arithmetic;
// the FP64 rounds of pass 2 build their twiddles from two table factors).
template <class P, int IDX, bool FT = P::PASS_NO == 2, class T, class TW, class Q>
__device__ __forceinline__ void rounds_fwd(T* lds, int tid, int wg, const TW* tw, const TW* twp, Q q, Q qinv) {
  if constexpr (IDX < P::NR) {
    if constexpr (IDX > 0) __syncthreads();
    if constexpr (std::is_same<T, double>::value)
      P::template round_f64<P::rbits(IDX), FT>(lds, tid, wg, P::rstart(IDX), tw, twp, q, qinv);
    else
      P::template round<P::rbits(IDX)>(lds, tid, wg, P::rstart(IDX), tw, twp, q);
    rounds_fwd<P, IDX + 1, FT>(lds, tid, wg, tw, twp, q, qinv);
  }
}
// Rounds IDX..0 of a pass, inverse order.
template <class P, int IDX, class T, class TW, class Q>
__device__ __forceinline__ void rounds_inv(T* lds, int tid, int wg, const TW* tw, const TW* twp, Q q, Q qinv) {
  if constexpr (IDX >= 0) {
    if constexpr (std::is_same<T, double>::value)
      P::template round_f64<P::rbits(IDX), P::PASS_NO == 2>(lds, tid, wg, P::rstart(IDX), tw, twp, q, qinv);
    else
      P::template round<P::rbits(IDX)>(lds, tid, wg, P::rstart(IDX), tw, twp, q);
    if constexpr (IDX > 0) {
      __syncthreads();
      rounds_inv<P, IDX - 1>(lds, tid, wg, tw, twp, q, qinv);
    }
  }
}

// Final store of one residue: plain, or (EPI, last forward pass) the fused
// ModDown epilogue of NttEpi for q-limb i, coefficient k, batch z.
template <bool EPI, int LOGN>
__device__ __forceinline__ void ntt_store(uint64_t* a, int k, uint64_t v, const NttEpi& epi, int i, int z,
                                          uint64_t q) {
  if constexpr (!EPI) {
    a[k] = v;
  } else {
    const size_t off = (size_t)i << LOGN;
    const bool batched = epi.out_base != nullptr || epi.tab != nullptr;
    const bool gather = batched ? (z & 1) == 0 : z == 0;  // the polynomial c0 is added to
    const uint64_t* add =
        batched ? (gather && epi.add_base ? epi.add_base + (epi.items ? epi.items[z >> 1] * epi.add_item : 0) : nullptr)
                : epi.add[z];
    uint64_t* out = epi.tab ? epi.tab->out[z] : batched ? epi.out_base + z * epi.out_bs : epi.out[z];
    const uint32_t g = epi.tab ? epi.tab->g[z >> 1] : epi.g;
    uint64_t x = 0;
    if (add) x = add[off + (gather && g != 1 ? automorph_src(k, g, LOGN) : (uint32_t)k)];
    out[off + k] = moddown_elem(epi.u[z * epi.u_bs + off + k], v, x, epi.pinv[i], epi.pinv[epi.level + i], q);
  }
}

// grid: x = tile within limb, y = batch, z = limb index in `map` (so the
// workgroups of one modulus are adjacent and share its twiddles in L2)
template <int LOGN, int PASS, bool INV, int LOG_EPT, int LOG_TILE, bool EPI>
__global__ __launch_bounds__((NttPass<LOGN, PASS, INV, LOG_EPT, LOG_TILE>::THREADS)) void ntt_pass_kernel(
    const uint64_t* src, size_t src_bs, uint64_t* data, size_t batch_stride, LimbMap map,
    const uint64_t* __restrict__ tw_all, const uint64_t* __restrict__ twp_all, const double* __restrict__ dtw_all,
    const double* __restrict__ dtwq_all, const ModInfo* __restrict__ mods, NttEpi epi) {
  static_assert(!EPI || (PASS == 2 && !INV), "the ModDown epilogue follows the last forward pass");
  using P = NttPass<LOGN, PASS, INV, LOG_EPT, LOG_TILE>;
  __shared__ uint64_t lds[P::LDS_WORDS];
  // Workgroups are dispatched round-robin over the 8 XCDs by linear id; with
  // WG_PER_LIMB a multiple of 8 the XCD is blockIdx.x mod 8.  A pass-1 tile
  // reads short row segments, so give each XCD a contiguous run of column
  // groups: neighbouring segments then meet in the same L2 instead of being
  // fetched separately by two XCDs.
  constexpr int W = P::WG_PER_LIMB;
  const int wg = (PASS == 1 && W % 8 == 0) ? (int)(blockIdx.x % 8) * (W / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
  const int limb = blockIdx.z;  // limb-major grid: the batch index varies faster
  const int bz = blockIdx.y;
  const int tid = threadIdx.x;
  // block-uniform: keep the limb's modulus and position (and so every base
  // address) in scalar registers, so loads and stores use 32-bit lane offsets
  const int m = __builtin_amdgcn_readfirstlane(map.mod[limb]);
  const int pos = __builtin_amdgcn_readfirstlane(map.pos[limb]);
  const uint64_t* ain = src + bz * src_bs + (size_t)pos * P::N;
  uint64_t* a = data + bz * batch_stride + (size_t)pos * P::N;
  const ModInfo mi = mods[m];
  const uint64_t q = mi.q;
  if (mi.k <= 50) {
    // FP64 path (exact doubles, full-rate FMA products); the branch is uniform per workgroup
    double* dl = reinterpret_cast<double*>(lds);
    const double* dtw = dtw_all + (size_t)m * P::N;
    const double* dtwq = dtwq_all + (size_t)m * P::N;
    const double dq = (double)q, dqinv = mi.dqinv;
    // inputs: canonical residues, or the raw intermediate of the other pass
    for (int e = tid; e < P::TILE; e += P::THREADS) {
      int g, k;
      P::tile_elem(e, g, k);
      dl[P::lidx(g, k)] = P::load_f64(ain[P::gidx(wg, g, k)]);
    }
    __syncthreads();
    if (!INV) rounds_fwd<P, 0, PASS == 2 && !EPI>(dl, tid, wg, dtw, dtwq, dq, dqinv);
    else rounds_inv<P, P::NR - 1>(dl, tid, wg, dtw, dtwq, dq, dqinv);
    __syncthreads();
    if constexpr (EPI) {
      // fused ModDown epilogue in centred FP64: v (|v| < 4.25q) is the transform's
      // value before canonicalisation; |u - v| < 6q, the product is below 2q and
      // adding the canonical c0 term stays below 3q, so one canonicalisation ends it
      const size_t off = (size_t)pos << LOGN;
      const double pw = bits_to_f64(epi.pinv[2 * epi.level + pos]);
      const double pwq = bits_to_f64(epi.pinv[3 * epi.level + pos]);
      const bool batched = epi.out_base != nullptr || epi.tab != nullptr;
      const bool gather = batched ? (bz & 1) == 0 : bz == 0;  // the polynomial c0 is added to
      const uint64_t* add =
          batched ? (gather && epi.add_base ? epi.add_base + (epi.items ? epi.items[bz >> 1] * epi.add_item : 0)
                                            : nullptr)
                  : epi.add[bz];
      const uint64_t* u = epi.u + bz * epi.u_bs + off;
      uint64_t* o = (epi.tab ? epi.tab->out[bz] : batched ? epi.out_base + bz * epi.out_bs : epi.out[bz]) + off;
      const uint32_t gal = epi.tab ? epi.tab->g[bz >> 1] : epi.g;  // (g is the tile loop's index below)
      if (!(add && gather && gal != 1)) {
        for (int e = tid; e < P::TILE; e += P::THREADS) {
          int g, k;
          P::tile_elem(e, g, k);
          const int kk = P::gidx(wg, g, k);
          const double r = mul_f64_c(u52_to_f64(u[kk]) - dl[P::lidx(g, k)], pw, pwq, dq);
          double x = 0.0;
          if (add) x = u52_to_f64(add[off + kk]);
          o[kk] = f64_to_u52(canon_f64(r + x, dqinv, dq));
        }
      } else {
        // c0 through phi_g: the pass-2 tile is the aligned block [wg TILE,
        // (wg + 1) TILE), which phi_g maps onto one aligned block, so that
        // block is read coalesced into the LDS (after the transform's values
        // have moved to registers) and permuted there
        constexpr int EPT = P::TILE / P::THREADS;
        double vv[EPT];
#pragma unroll
        for (int i = 0; i < EPT; i++) {
          int g, k;
          P::tile_elem(tid + i * P::THREADS, g, k);
          vv[i] = dl[P::lidx(g, k)];
        }
        __syncthreads();
        const uint32_t base = (uint32_t)wg * P::TILE;
        const uint32_t s0 = automorph_src(base, gal, LOGN) & ~(uint32_t)(P::TILE - 1);
        uint64_t* lu = reinterpret_cast<uint64_t*>(dl);
        for (int e = tid; e < P::TILE; e += P::THREADS) lu[e] = add[off + s0 + e];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < EPT; i++) {
          const uint32_t kk = base + tid + i * P::THREADS;
          const double r = mul_f64_c(u52_to_f64(u[kk]) - vv[i], pw, pwq, dq);
          const double x = u52_to_f64(lu[automorph_src(kk, gal, LOGN) - s0]);
          o[kk] = f64_to_u52(canon_f64(r + x, dqinv, dq));
        }
      }
    } else {
      // the inverse transform's N^{-1}, or a conversion's finishing constant
      double fw = mi.dninv, fwq = mi.dninvq;
      if (INV && PASS == 1 && epi.fin) {
        fw = bits_to_f64(epi.fin[4 * m + 2]);
        fwq = bits_to_f64(epi.fin[4 * m + 3]);
      }
      for (int e = tid; e < P::TILE; e += P::THREADS) {
        int g, k;
        P::tile_elem(e, g, k);
        a[P::gidx(wg, g, k)] = P::finish_f64(dl[P::lidx(g, k)], fw, fwq, dq, dqinv);
      }
    }
    return;
  }
  const uint64_t* tw = tw_all + (size_t)m * P::N;
  const uint64_t* twp = twp_all + (size_t)m * P::N;
  for (int e = tid; e < P::TILE; e += P::THREADS) {
    int g, k;
    P::tile_elem(e, g, k);
    lds[P::lidx(g, k)] = ain[P::gidx(wg, g, k)];
  }
  __syncthreads();
  if (!INV) rounds_fwd<P, 0>(lds, tid, wg, tw, twp, q, q);
  else rounds_inv<P, P::NR - 1>(lds, tid, wg, tw, twp, q, q);
  __syncthreads();
  uint64_t fw = mi.ninv, fwp = mi.ninv_p;
  if (INV && PASS == 1 && epi.fin) {
    fw = epi.fin[4 * m];
    fwp = epi.fin[4 * m + 1];
  }
  for (int e = tid; e < P::TILE; e += P::THREADS) {
    int g, k;
    P::tile_elem(e, g, k);
    ntt_store<EPI, LOGN>(a, P::gidx(wg, g, k), P::finish(lds[P::lidx(g, k)], fw, fwp, q), epi, pos, bz, q);
  }
}

// Word at element offset idx (below 2^29) of a uniform base: the byte offset
// is formed in 32 bits, so the access takes a scalar base and a 32-bit lane
// offset instead of a 64-bit address per lane.
__device__ __forceinline__ uint64_t ld_at(const uint64_t* base, uint32_t idx) {
  return *reinterpret_cast<const uint64_t*>(reinterpret_cast<const char*>(base) + (uint32_t)(idx << 3));
}
__device__ __forceinline__ void st_at(uint64_t* base, uint32_t idx, uint64_t v) {
  *reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(base) + (uint32_t)(idx << 3)) = v;
}

// Forward column rounds of two tiles side by side (the second only when
// `two`, uniform over the workgroup): one barrier per round serves both.
template <class P, int IDX>
__device__ __forceinline__ void rounds_fwd2_f64(double* a, double* b, bool two, int tid, int wg, const double* twa,
                                                const double* twqa, double qa, double qia, const double* twb,
                                                const double* twqb, double qb, double qib) {
  if constexpr (IDX < P::NR) {
    if constexpr (IDX > 0) __syncthreads();
    P::template round_f64<P::rbits(IDX), false>(a, tid, wg, P::rstart(IDX), twa, twqa, qa, qia);
    if (two) P::template round_f64<P::rbits(IDX), false>(b, tid, wg, P::rstart(IDX), twb, twqb, qb, qib);
    rounds_fwd2_f64<P, IDX + 1>(a, b, two, tid, wg, twa, twqa, qa, qia, twb, twqb, qb, qib);
  }
}

// Basis conversion fused into the forward column pass (pass 1) of its
// outputs (ConvDesc).  Workgroup (x, y, z) owns column tile x, output group
// y and batch z.  Every thread first loads all input parts at the tile
// positions it owns when a tile is staged (one round of loads in flight,
// kept in registers: NP parts x EPT residues).  An FP64 group (outputs below
// 2^50) then takes its outputs two at a time: the centred sums of both go
// into two LDS tiles, the forward column rounds of both run between the same
// barriers, and both pass-1 intermediates (the form the second pass reads)
// are stored.  An integer group (outputs of 51 bits and more; descriptors
// list them first) takes its outputs one at a time with 128-bit
// accumulators.  The workgroups of one column tile sit on one XCD (the XCD
// is the linear workgroup id mod 8, i.e. blockIdx.x mod 8 since the tile
// count is a multiple of 8), so a tile's inputs are fetched from HBM once
// and re-read from that XCD's L2 by its other output groups.
template <int LOGN, int LOG_EPT, int LOG_TILE, int NP>
__global__ __launch_bounds__((NttPass<LOGN, 1, false, LOG_EPT, LOG_TILE>::THREADS))
__attribute__((amdgpu_waves_per_eu(4))) void k_conv_fwd1(
    const uint64_t* __restrict__ in, size_t in_bs, uint64_t* __restrict__ out, size_t out_bs,
    const ConvDesc* __restrict__ descs, int zdiv, int group, const uint64_t* __restrict__ tw_all,
    const uint64_t* __restrict__ twp_all, const double* __restrict__ dtw_all, const double* __restrict__ dtwq_all,
    const ModInfo* __restrict__ mods) {
  using P = NttPass<LOGN, 1, false, LOG_EPT, LOG_TILE>;
  constexpr int EPT = P::TILE / P::THREADS;
  __shared__ uint64_t lds[2][P::LDS_WORDS];
  // the M - 1 twiddles (and quotients) of the column transform of each tile's
  // modulus, staged once per output instead of gathered from L2 every round
  __shared__ double s_tw[2][2][P::M];
  // the group's conversion constants, staged once (read with uniform
  // addresses, i.e. broadcast)
  __shared__ uint64_t s_cst[CONV_MAX_GROUP * 2 * 2 * MAX_BCONV_IN];
  constexpr int W = P::WG_PER_LIMB;
  const int wg = (W % 8 == 0) ? (int)(blockIdx.x % 8) * (W / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
  const int z = blockIdx.z;
  const ConvDesc& d = descs[z % zdiv];
  // descriptor fields are uniform: keep them (and so every base address) in
  // scalar registers, so that loads and stores take 32-bit lane offsets
  const int nout = __builtin_amdgcn_readfirstlane(d.nout);
  const int np = __builtin_amdgcn_readfirstlane(d.nparts);
  const int nint = __builtin_amdgcn_readfirstlane(d.nint);
  // group y: integer outputs [y group, ..) while y < ceil(nint / group), then FP64 ones
  const int gint = (nint + group - 1) / group;
  const int y = blockIdx.y;
  const bool fp = y >= gint;
  const int p0 = fp ? nint + (y - gint) * group : y * group;
  const int p1 = min(p0 + group, fp ? nout : nint);
  if (p0 >= p1) return;  // uniform over the workgroup
  const uint64_t* src = in + (size_t)(z / zdiv) * in_bs;
  uint64_t* dst = out + (size_t)z * out_bs;
  const int tid = threadIdx.x;
  {
    const uint64_t* c0 = d.cst + (size_t)p0 * np * 2;
    for (int t = tid; t < (p1 - p0) * np * 2; t += P::THREADS) s_cst[t] = c0[t];
  }
  int gi[EPT], li[EPT];
#pragma unroll
  for (int j = 0; j < EPT; j++) {
    int g, k;
    P::tile_elem(tid + j * P::THREADS, g, k);
    gi[j] = P::gidx(wg, g, k);
    li[j] = P::lidx(g, k);
  }
  if (fp) {
    __syncthreads();  // s_cst
    double x[NP][EPT];
#pragma unroll
    for (int v = 0; v < NP; v++) {
      if (v < np) {
        const uint64_t* sp = src + ((size_t)__builtin_amdgcn_readfirstlane(d.part_pos[v]) << LOGN);
        double pa, pb;
        conv_part_ab(__builtin_amdgcn_readfirstlane(d.part_kind[v]), pa, pb);
#pragma unroll
        for (int j = 0; j < EPT; j++) x[v][j] = conv_part(ld_at(sp, gi[j]), pa, pb);
      } else {
#pragma unroll
        for (int j = 0; j < EPT; j++) x[v][j] = 0.0;
      }
    }
    for (int p = p0; p < p1; p += 2) {
      const bool two = p + 1 < p1;
      const int ma = __builtin_amdgcn_readfirstlane(d.out_mod[p]);
      const int mb = __builtin_amdgcn_readfirstlane(d.out_mod[two ? p + 1 : p]);
      const ModInfo& mia = mods[ma];
      const ModInfo& mib = mods[mb];
      const double qa = (double)mia.q, qb = (double)mib.q;
      double* la = reinterpret_cast<double*>(lds[0]);
      double* lb = reinterpret_cast<double*>(lds[1]);
      for (int t = tid; t < P::M; t += P::THREADS) {
        s_tw[0][0][t] = dtw_all[((size_t)ma << LOGN) + t];
        s_tw[0][1][t] = dtwq_all[((size_t)ma << LOGN) + t];
        s_tw[1][0][t] = dtw_all[((size_t)mb << LOGN) + t];
        s_tw[1][1][t] = dtwq_all[((size_t)mb << LOGN) + t];
      }
      const uint64_t* ca = s_cst + (p - p0) * np * 2;
#pragma unroll
      for (int j = 0; j < EPT; j++) {
        double xs[NP];
#pragma unroll
        for (int v = 0; v < NP; v++) xs[v] = x[v][j];
        la[li[j]] = conv_sum_f64<NP>(xs, np, ca, qa, mia.dqinv);
      }
      if (two) {
        const uint64_t* cb = ca + np * 2;
#pragma unroll
        for (int j = 0; j < EPT; j++) {
          double xs[NP];
#pragma unroll
          for (int v = 0; v < NP; v++) xs[v] = x[v][j];
          lb[li[j]] = conv_sum_f64<NP>(xs, np, cb, qb, mib.dqinv);
        }
      }
      __syncthreads();
      rounds_fwd2_f64<P, 0>(la, lb, two, tid, wg, s_tw[0][0], s_tw[0][1], qa, mia.dqinv, s_tw[1][0], s_tw[1][1], qb,
                            mib.dqinv);
      __syncthreads();
      uint64_t* oa = dst + ((size_t)__builtin_amdgcn_readfirstlane(d.out_pos[p]) << LOGN);
#pragma unroll
      for (int j = 0; j < EPT; j++) st_at(oa, gi[j], f64_to_bits(la[li[j]]));
      if (two) {
        uint64_t* ob = dst + ((size_t)__builtin_amdgcn_readfirstlane(d.out_pos[p + 1]) << LOGN);
#pragma unroll
        for (int j = 0; j < EPT; j++) st_at(ob, gi[j], f64_to_bits(lb[li[j]]));
      }
      __syncthreads();  // the tiles are rewritten by the next pair
    }
    return;
  }
  // integer outputs (rare: at most a few per conversion) re-read the parts
  // from L2 instead of keeping them in registers next to the FP64 path's copy
  __syncthreads();  // s_cst
  for (int p = p0; p < p1; p++) {
    const int m = __builtin_amdgcn_readfirstlane(d.out_mod[p]);
    const ModInfo mi = mods[m];
    const uint64_t q = mi.q;
    const uint64_t* cst = s_cst + (p - p0) * np * 2;
    uint64_t* il = lds[0];
    U128 acc[EPT];
#pragma unroll
    for (int j = 0; j < EPT; j++) acc[j] = U128{0, 0};
    for (int v = 0; v < np; v++) {
      const uint64_t* sp = src + ((size_t)__builtin_amdgcn_readfirstlane(d.part_pos[v]) << LOGN);
      double pa, pb;
      conv_part_ab(__builtin_amdgcn_readfirstlane(d.part_kind[v]), pa, pb);
#pragma unroll
      for (int j = 0; j < EPT; j++) conv_mac_int(acc[j], conv_part(ld_at(sp, gi[j]), pa, pb), cst[2 * v], q);
    }
#pragma unroll
    for (int j = 0; j < EPT; j++) il[li[j]] = mont_redc(acc[j], q, mi.qinv);
    __syncthreads();
    rounds_fwd<P, 0>(il, tid, wg, tw_all + ((size_t)m << LOGN), twp_all + ((size_t)m << LOGN), q, q);
    __syncthreads();
    uint64_t* o_ = dst + ((size_t)__builtin_amdgcn_readfirstlane(d.out_pos[p]) << LOGN);
#pragma unroll
    for (int j = 0; j < EPT; j++) st_at(o_, gi[j], il[li[j]]);
    __syncthreads();
  }
}

// Forward rounds IDX..NR-1 run by the waves with `act` set; every wave of
// the workgroup passes the same barriers.
template <class P, int IDX, class T, class TW, class Q>
__device__ __forceinline__ void rounds_fwd_if(bool act, T* lds, int tid, int wg, const TW* tw, const TW* twp, Q q,
                                              Q qinv) {
  if constexpr (IDX < P::NR) {
    if constexpr (IDX > 0) __syncthreads();
    if (act) {
      if constexpr (std::is_same<T, double>::value)
        P::template round_f64<P::rbits(IDX), P::PASS_NO == 2>(lds, tid, wg, P::rstart(IDX), tw, twp, q, qinv);
      else
        P::template round<P::rbits(IDX)>(lds, tid, wg, P::rstart(IDX), tw, twp, q);
    }
    rounds_fwd_if<P, IDX + 1>(act, lds, tid, wg, tw, twp, q, qinv);
  }
}

// Key-switch inner product fused into the last forward pass of ModUp (one
// key switch, so one automorphism and one key).  Workgroup (x, z) owns output
// tile x of ext limb map[z]: phi_g maps aligned blocks of TILE positions onto
// aligned blocks, so the values it needs form one source tile.  The
// workgroup has one group of P::THREADS threads (whole waves) per digit d,
// each with its own LDS tile: group d loads digit d's source tile and
// finishes its transform (the own digit's limb is c1 itself, already in NTT
// form, and is only loaded); then every thread accumulates
// e_d[src(k)] * key_d[j][pos][k] over the digits for both key polynomials j
// in 128-bit registers.  The extended digits never return to HBM.
// Inverse rounds NR-1..0 run by the waves with `act` set; every wave of the
// workgroup passes the same barriers.
template <class P, int IDX, class T, class TW, class Q>
__device__ __forceinline__ void rounds_inv_if(bool act, T* lds, int tid, int wg, const TW* tw, const TW* twp, Q q,
                                              Q qinv) {
  if constexpr (IDX >= 0) {
    if (act) {
      if constexpr (std::is_same<T, double>::value)
        P::template round_f64<P::rbits(IDX), P::PASS_NO == 2>(lds, tid, wg, P::rstart(IDX), tw, twp, q, qinv);
      else
        P::template round<P::rbits(IDX)>(lds, tid, wg, P::rstart(IDX), tw, twp, q);
    }
    if constexpr (IDX > 0) {
      __syncthreads();
      rounds_inv_if<P, IDX - 1>(act, lds, tid, wg, tw, twp, q, qinv);
    }
  }
}

template <int LOGN, int LOG_EPT, int LOG_TILE, int DN>
__global__ __launch_bounds__((DN * NttPass<LOGN, 2, false, LOG_EPT, LOG_TILE>::THREADS)) void ntt_ip_kernel(LimbMap map, const uint64_t* __restrict__ tw_all,
                                                          const uint64_t* __restrict__ twp_all,
                                                          const double* __restrict__ dtw_all,
                                                          const double* __restrict__ dtwq_all,
                                                          const uint64_t* __restrict__ itw_all,
                                                          const uint64_t* __restrict__ itwp_all,
                                                          const double* __restrict__ ditw_all,
                                                          const double* __restrict__ ditwq_all,
                                                          const ModInfo* __restrict__ mods, NttIp ip) {
  using P = NttPass<LOGN, 2, false, LOG_EPT, LOG_TILE>;
  using PI = NttPass<LOGN, 2, true, LOG_EPT, LOG_TILE>;
  static_assert(P::THREADS % 64 == 0, "digit groups of whole waves");
  static_assert(LOG_EPT <= 3 && DN <= 4, "the FP64 inner-product bounds assume three-stage rounds, four digits");
  constexpr int NTHR = DN * P::THREADS;
  constexpr int IT = (P::TILE + NTHR - 1) / NTHR;  // outputs per thread
  extern __shared__ uint64_t lds_all[];  // [max(dnum, 2)][P::LDS_WORDS]
  const int tid = threadIdx.x;
  const int d = tid / P::THREADS;       // wave-uniform
  const int t = tid - d * P::THREADS;
  const int m = __builtin_amdgcn_readfirstlane(map.mod[blockIdx.z]);
  const int pos = __builtin_amdgcn_readfirstlane(map.pos[blockIdx.z]);
  const ModInfo mi = mods[m];
  const uint64_t q = mi.q;
  const uint32_t out0 = blockIdx.x * P::TILE;
  const uint32_t src0 = automorph_src(out0, ip.g, LOGN) & ~(uint32_t)(P::TILE - 1);
  const int swg = (int)(src0 / P::TILE);
  const size_t off = (size_t)pos << LOGN;
  const bool own = pos < ip.level && pos / ip.alpha == d;
  const bool load_only = own || ip.ext_ntt;  // already in NTT form
  const uint64_t* ain = own ? ip.c1 + off : ip.ext + d * ip.ext_ds + off;
  uint64_t* lds = lds_all + d * P::LDS_WORDS;
  const bool f64 = mi.k <= 50;  // uniform over the workgroup
  const uint64_t* key = ip.key + ((size_t)m << LOGN) + out0;
  if (f64) {
    double* dl = reinterpret_cast<double*>(lds);
    for (int e = t; e < P::TILE; e += P::THREADS) {
      int g, k;
      P::tile_elem(e, g, k);
      const uint64_t w = ain[P::gidx(swg, g, k)];
      dl[P::lidx(g, k)] = load_only ? u52_to_f64(w) : P::load_f64(w);
    }
    __syncthreads();
    rounds_fwd_if<P, 0>(!load_only, dl, t, swg, dtw_all + (size_t)m * P::N, dtwq_all + (size_t)m * P::N, (double)q,
                        mi.dqinv);
  } else {
    for (int e = t; e < P::TILE; e += P::THREADS) {
      int g, k;
      P::tile_elem(e, g, k);
      lds[P::lidx(g, k)] = ain[P::gidx(swg, g, k)];
    }
    __syncthreads();
    rounds_fwd_if<P, 0>(!load_only, lds, t, swg, tw_all + (size_t)m * P::N, twp_all + (size_t)m * P::N, q, q);
  }
  __syncthreads();
  uint64_t* u = ip.u + off + out0;
  // special-prime limbs continue with the inverse pass 2 of ModDown
  const bool pinv2 = DN >= 2 && ip.p_inv2 && pos >= ip.level;
  uint64_t r0[IT], r1[IT];
#pragma unroll
  for (int it = 0; it < IT; it++) {
    const int e = tid + it * NTHR;
    if (e >= P::TILE) break;
    const uint32_t k = out0 + e;
    const int sl = (int)((ip.g == 1 ? k : automorph_src(k, ip.g, LOGN)) - src0);
    const int li = P::lidx(sl / P::M, sl % P::M);
    uint64_t k0[DN], k1[DN];
#pragma unroll
    for (int j = 0; j < DN; j++) {
      k0[j] = key[j * ip.key_ds + e];
      k1[j] = key[j * ip.key_ds + ip.key_ps + e];
    }
    if (f64) {
      // centred FP64: the digits' values (|v| < 2.9q after rounds of at most
      // three stages, or canonical for the own digit) times the Montgomery-form
      // key words (< q, exact as doubles; quotient estimates fl(k fl(1/q)),
      // off by at most 1.5 |v| 2^-52 < 1.09) are below 1.6q each, the sum over
      // at most four digits below 6.4q; one more product by 2^-64 mod q
      // removes the Montgomery factor and leaves |x| < 2.9q for canon_f64
      const double dq = (double)q, qi = mi.dqinv;
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int j = 0; j < DN; j++) {
        const double v = bits_to_f64(lds_all[j * P::LDS_WORDS + li]);
        const double w0 = u52_to_f64(k0[j]), w1 = u52_to_f64(k1[j]);
        a0 += mul_f64_c(v, w0, w0 * qi, dq);
        a1 += mul_f64_c(v, w1, w1 * qi, dq);
      }
      r0[it] = f64_to_u52(canon_f64(mul_f64_c(a0, mi.drinv, mi.drinvq, dq), qi, dq));
      r1[it] = f64_to_u52(canon_f64(mul_f64_c(a1, mi.drinv, mi.drinvq, dq), qi, dq));
    } else {
      U128 a0{0, 0}, a1{0, 0};
#pragma unroll
      for (int j = 0; j < DN; j++) {
        const uint64_t v = P::finish(lds_all[j * P::LDS_WORDS + li], 0, 0, q);
        add_wide(a0, mul_wide(v, k0[j]));
        add_wide(a1, mul_wide(v, k1[j]));
      }
      r0[it] = mont_redc(a0, q, mi.qinv);
      r1[it] = mont_redc(a1, q, mi.qinv);
    }
    if (!pinv2) {
      u[e] = r0[it];
      u[ip.u_ps + e] = r1[it];
    }
  }
  if (!pinv2) return;  // uniform over the workgroup
  // u_0 and u_1 of this tile into regions 0 and 1 (natural order), then
  // groups 0 and 1 run the inverse pass-2 rounds and store the intermediate
  __syncthreads();
#pragma unroll
  for (int it = 0; it < IT; it++) {
    const int e = tid + it * NTHR;
    if (e >= P::TILE) break;
    const int li = PI::lidx(e / PI::M, e % PI::M);
    lds_all[li] = f64 ? f64_to_bits(u52_to_f64(r0[it])) : r0[it];
    lds_all[PI::LDS_WORDS + li] = f64 ? f64_to_bits(u52_to_f64(r1[it])) : r1[it];
  }
  __syncthreads();
  const bool act = d < 2;
  const int wg = blockIdx.x;
  if (f64)
    rounds_inv_if<PI, PI::NR - 1>(act, reinterpret_cast<double*>(lds), t, wg, ditw_all + (size_t)m * P::N,
                                  ditwq_all + (size_t)m * P::N, (double)q, mi.dqinv);
  else
    rounds_inv_if<PI, PI::NR - 1>(act, lds, t, wg, itw_all + (size_t)m * P::N, itwp_all + (size_t)m * P::N, q, q);
  __syncthreads();
  if (act) {
    uint64_t* o = ip.u + d * ip.u_ps + off;
    for (int e = t; e < PI::TILE; e += PI::THREADS) {
      int g, k;
      PI::tile_elem(e, g, k);
      const uint64_t v = lds[PI::lidx(g, k)];
      o[PI::gidx(wg, g, k)] = f64 ? PI::finish_f64(bits_to_f64(v), 0, 0, (double)q, mi.dqinv) : PI::finish(v, 0, 0, q);
    }
  }
}

// passes: bit 0 = pass 1, bit 1 = pass 2 (a forward pass 2 alone reads `data`,
// an inverse pass 1 alone reads `data` too)
template <int LOGN, int LOG_EPT, int LOG_TILE>
static int ntt_launch_v(Ctx* c, const uint64_t* src, size_t src_bs, uint64_t* data, size_t batch_stride,
                        int nbatch, const LimbMap& map, bool inverse, hipStream_t s, const NttEpi* epi = nullptr,
                        int passes = 3, const uint64_t* fin = nullptr) {
  using P1 = NttPass<LOGN, 1, false, LOG_EPT, LOG_TILE>;
  using P2 = NttPass<LOGN, 2, false, LOG_EPT, LOG_TILE>;
  constexpr int T = P1::THREADS;
  dim3 g1(P1::WG_PER_LIMB, nbatch, map.n), g2(P2::WG_PER_LIMB, nbatch, map.n);
  const double limbs = (double)map.n * nbatch, N = (double)P1::N;
  const double bytes = 16.0 * N * limbs;  // one read + one write of every residue per pass
  const double mm1 = N / 2 * P1::LM * limbs, mm2 = N / 2 * P2::LM * limbs;
  // ALU-ideal time per modular product, by the arithmetic of each limb's prime
  double per_mm = 0.0;
  if (c->prof_on) {
    int nf = 0;
    for (int i = 0; i < map.n; i++) nf += c->hmod[map.mod[i]].k <= 50;
    per_mm = ((double)nf / PEAK_MODMUL_F64 + (double)(map.n - nf) / PEAK_MODMUL_INT) / map.n;
  }
  const NttEpi none{};
  if (!inverse) {
    if (passes & 1) {
      ProfScope ps(c, "ntt_fwd_pass1", s, bytes, mm1, mm1 * per_mm);
      ntt_pass_kernel<LOGN, 1, false, LOG_EPT, LOG_TILE, false><<<g1, T, 0, s>>>(
          src, src_bs, data, batch_stride, map, c->d_tw, c->d_twp, c->d_dtw, c->d_dtwq, c->d_mod, none);
    }
    if (!(passes & 2)) {
    } else if (epi) {
      // + u read, out write instead of y write, add_0 / add_1 reads
      const double eb = bytes + 8.0 * N * limbs * (1 + (epi->add[0] ? 0.5 : 0) + (epi->add[1] ? 0.5 : 0));
      ProfScope ps(c, "ntt_fwd_pass2_moddown", s, eb, mm2 + N * limbs, mm2 * per_mm + N * limbs / PEAK_MODMUL_INT);
      ntt_pass_kernel<LOGN, 2, false, LOG_EPT, LOG_TILE, true><<<g2, T, 0, s>>>(
          data, batch_stride, data, batch_stride, map, c->d_tw, c->d_twp, c->d_dtw, c->d_dtwq, c->d_mod, *epi);
    } else {
      ProfScope ps(c, "ntt_fwd_pass2", s, bytes, mm2, mm2 * per_mm);
      ntt_pass_kernel<LOGN, 2, false, LOG_EPT, LOG_TILE, false><<<g2, T, 0, s>>>(
          data, batch_stride, data, batch_stride, map, c->d_tw, c->d_twp, c->d_dtw, c->d_dtwq, c->d_mod, none);
    }
  } else {
    if (passes & 2) {
      ProfScope ps(c, "ntt_inv_pass2", s, bytes, mm2, mm2 * per_mm);
      ntt_pass_kernel<LOGN, 2, true, LOG_EPT, LOG_TILE, false><<<g2, T, 0, s>>>(
          src, src_bs, data, batch_stride, map, c->d_itw, c->d_itwp, c->d_ditw, c->d_ditwq, c->d_mod, none);
    }
    if (passes & 1) {
      NttEpi e1{};
      e1.fin = fin;
      ProfScope ps(c, fin ? "ntt_inv_pass1_conv" : "ntt_inv_pass1", s, bytes, mm1 + N * limbs, (mm1 + N * limbs) * per_mm);
      ntt_pass_kernel<LOGN, 1, true, LOG_EPT, LOG_TILE, false><<<g1, T, 0, s>>>(
          data, batch_stride, data, batch_stride, map, c->d_itw, c->d_itwp, c->d_ditw, c->d_ditwq, c->d_mod, e1);
    }
  }
  HE_HIP(hipGetLastError());
  return HE_OK;
}

// Variants: (tile, residues per thread) = (4096, 4), (4096, 8), (4096, 16),
// (2048, 4), (2048, 8).  Smaller tiles and fewer residues per thread give
// more workgroups and waves for small limb batches; large tiles with more
// residues per thread need fewer LDS rounds and coalesce better.  The best
// variant per batch-size bucket is measured at context creation
// (ntt_autotune).
static const int kNttLogTile[NTT_VARIANTS] = {12, 12, 12, 11, 11};
static const int kNttLogEpt[NTT_VARIANTS] = {2, 3, 4, 2, 3};

static int ntt_bucket(int limbs) { return limbs <= 8 ? 0 : limbs <= 16 ? 1 : limbs <= 32 ? 2 : 3; }

template <int LOGN>
static int ntt_launch_var(Ctx* c, int var, const uint64_t* src, size_t src_bs, uint64_t* data, size_t batch_stride,
                          int nbatch, const LimbMap& map, bool inverse, hipStream_t s, const NttEpi* epi = nullptr,
                          int passes = 3, const uint64_t* fin = nullptr) {
  switch (var) {
    case 0: return ntt_launch_v<LOGN, 2, 12>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s, epi, passes, fin);
    case 1: return ntt_launch_v<LOGN, 3, 12>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s, epi, passes, fin);
    case 3: return ntt_launch_v<LOGN, 2, 11>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s, epi, passes, fin);
    case 4: return ntt_launch_v<LOGN, 3, 11>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s, epi, passes, fin);
    default: return ntt_launch_v<LOGN, 4, 12>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s, epi, passes, fin);
  }
}

// Limbs of one modulus are transformed back to back (the order of
// independent limb transforms is free), so that its twiddle tables are
// fetched once and then served from L2; the slower integer-path limbs (primes
// of 51 bits and more) go first so that they do not form the launch's tail.
static LimbMap by_modulus(const Ctx* c, const LimbMap& m) {
  LimbMap r = m;
  int idx[MAXJ];
  for (int i = 0; i < m.n; i++) idx[i] = i;
  auto key = [&](int i) { return (c->hmod[m.mod[i]].k <= 50 ? 256 : 0) + (int)m.mod[i]; };
  std::stable_sort(idx, idx + m.n, [&](int a, int b) { return key(a) < key(b); });
  for (int i = 0; i < m.n; i++) {
    r.pos[i] = m.pos[idx[i]];
    r.mod[i] = m.mod[idx[i]];
  }
  return r;
}

template <int LOGN>
static int ntt_launch_n(Ctx* c, const uint64_t* src, size_t src_bs, uint64_t* data, size_t batch_stride,
                        int nbatch, const LimbMap& map, bool inverse, hipStream_t s, const NttEpi* epi = nullptr,
                        int passes = 3, const uint64_t* fin = nullptr) {
  return ntt_launch_var<LOGN>(c, c->ntt_var[ntt_bucket(map.n * nbatch)], src, src_bs, data, batch_stride, nbatch,
                              by_modulus(c, map), inverse, s, epi, passes, fin);
}

template <int LOGN>
static int ntt_probe(Ctx* c, int var, const LimbMap& m, hipStream_t s) {
  int rc;
  if ((rc = ntt_launch_var<LOGN>(c, var, c->ws, 0, c->ws, 0, 1, m, false, s))) return rc;
  return ntt_launch_var<LOGN>(c, var, c->ws, 0, c->ws, 0, 1, m, true, s);
}

// Autotuner: time a forward + inverse transform of 8, 16, 32 and 64 limbs
// (the context's own moduli, in its workspace) with each variant and keep the
// fastest per bucket; larger batches use the 64-limb choice.
void ntt_variant_shape(int v, int* tile, int* per_thread) {
  *tile = 1 << kNttLogTile[v];
  *per_thread = 1 << kNttLogEpt[v];
}

int ntt_autotune(Ctx* c) {
  const int probes[4] = {8, 16, 32, 64};
  const size_t N = c->n;
  const int cap = (int)(c->ws_words / N);
  hipStream_t s;
  HE_HIP(hipStreamCreate(&s));
  hipEvent_t e0, e1;
  HE_HIP(hipEventCreate(&e0));
  HE_HIP(hipEventCreate(&e1));
  HE_HIP(hipMemsetAsync(c->ws, 0, c->ws_words * 8, s));
  for (int pi = 0; pi < 4; pi++) {
    const int limbs = std::min(probes[pi], std::min(cap, MAXJ));
    LimbMap m{};
    m.n = limbs;
    for (int i = 0; i < limbs; i++) {
      m.pos[i] = (uint16_t)i;
      m.mod[i] = (uint8_t)(i % (c->L + c->K));
    }
    float best = 1e30f;
    for (int v = 0; v < NTT_VARIANTS; v++) {
      auto run = [&]() -> int {
        switch (c->log_n) {
          case 16: return ntt_probe<16>(c, v, m, s);
          case 14: return ntt_probe<14>(c, v, m, s);
          default: return ntt_probe<12>(c, v, m, s);
        }
      };
      int rc;
      if ((rc = run())) return rc;  // warm-up
      HE_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 5; r++)
        if ((rc = run())) return rc;
      HE_HIP(hipEventRecord(e1, s));
      HE_HIP(hipEventSynchronize(e1));
      float ms = 0;
      HE_HIP(hipEventElapsedTime(&ms, e0, e1));
      const float us = ms * 1e3f / 5;
      c->ntt_tune_us[v][pi] = us;
      if (us < best) {
        best = us;
        c->ntt_var[pi] = v;
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  HE_HIP(hipStreamSynchronize(s));
  hipStreamDestroy(s);
  return HE_OK;
}

int ntt_launch_strided(Ctx* c, const uint64_t* src, size_t src_bs, uint64_t* data, size_t batch_stride, int nbatch,
                       const LimbMap& map, bool inverse, hipStream_t s) {
  if (map.n <= 0 || nbatch <= 0) return HE_OK;
  if (nbatch > 65535) return set_error(HE_EINVAL, "NTT batch too large for one launch");
  switch (c->log_n) {
    case 12: return ntt_launch_n<12>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s);
    case 14: return ntt_launch_n<14>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s);
    case 16: return ntt_launch_n<16>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s);
  }
  return set_error(HE_EINVAL, "unsupported ring degree");
}

int ntt_launch_moddown(Ctx* c, const uint64_t* y, size_t y_bs, const LimbMap& map, const NttEpi& epi, hipStream_t s,
                       int nbatch, int passes) {
  if (map.n <= 0 || nbatch <= 0) return HE_OK;
  if (nbatch > 65535) return set_error(HE_EINVAL, "NTT batch too large for one launch");
  // the transform runs in place on y (its scratch); results go to epi.out
  uint64_t* yy = const_cast<uint64_t*>(y);
  switch (c->log_n) {
    case 12: return ntt_launch_n<12>(c, yy, y_bs, yy, y_bs, nbatch, map, false, s, &epi, passes);
    case 14: return ntt_launch_n<14>(c, yy, y_bs, yy, y_bs, nbatch, map, false, s, &epi, passes);
    case 16: return ntt_launch_n<16>(c, yy, y_bs, yy, y_bs, nbatch, map, false, s, &epi, passes);
  }
  return set_error(HE_EINVAL, "unsupported ring degree");
}

int ntt_launch_conv_in(Ctx* c, const uint64_t* src, size_t src_bs, uint64_t* data, size_t batch_stride, int nbatch,
                       const LimbMap& map, const uint64_t* fin, int passes, hipStream_t s) {
  if (map.n <= 0 || nbatch <= 0) return HE_OK;
  if (nbatch > 65535) return set_error(HE_EINVAL, "NTT batch too large for one launch");
  switch (c->log_n) {
    case 12: return ntt_launch_n<12>(c, src, src_bs, data, batch_stride, nbatch, map, true, s, nullptr, passes, fin);
    case 14: return ntt_launch_n<14>(c, src, src_bs, data, batch_stride, nbatch, map, true, s, nullptr, passes, fin);
    case 16: return ntt_launch_n<16>(c, src, src_bs, data, batch_stride, nbatch, map, true, s, nullptr, passes, fin);
  }
  return set_error(HE_EINVAL, "unsupported ring degree");
}

int rescale_launch(Ctx* c, const uint64_t* in, size_t in_bs, uint64_t* out, size_t out_bs, int npolys, int l,
                   uint64_t* T, uint64_t* Y, hipStream_t s) {
  if (l < 2 || npolys <= 0) return set_error(HE_EINVAL, "bad rescale");
  const int t = l - 1;
  const size_t N = c->n;
  int rc;
  // top limbs to coefficient form (a one-input conversion needs no factor
  // beyond N^{-1})
  if ((rc = ntt_launch_conv_in(c, in + (size_t)t * N, in_bs, T, N, npolys, range_map(0, 1, t), nullptr, 3, s)))
    return rc;
  if ((rc = conv_fwd1_launch(c, c->rsconv[l], T, N, Y, (size_t)t * N, npolys, 1, c->conv_target[1], "conv_fwd1_rescale",
                             s)))
    return rc;
  NttEpi epi{};
  epi.u = in;
  epi.u_bs = in_bs;
  epi.pinv = c->d_rescale[l];
  epi.g = 1;
  epi.level = t;
  epi.out_base = out;
  epi.out_bs = out_bs;
  return ntt_launch_moddown(c, Y, (size_t)t * N, range_map(0, t, 0), epi, s, npolys, 2);
}

// Conversion kernel shape: 1024-residue column tiles, 4 residues per thread
// (4 LDS rounds of 2 stages at N = 2^16); the parts of an input coefficient
// stay in registers, so the kernel is instantiated per part count bucket.
constexpr int CONV_LOG_EPT = 2, CONV_LOG_TILE = 10;

template <int LOGN, int NP>
static void conv_fwd1_go(Ctx* c, const ConvSet& set, const uint64_t* in, size_t in_bs, uint64_t* out, size_t out_bs,
                         int nz, int zdiv, int group, int ngroups, hipStream_t s) {
  using P = NttPass<LOGN, 1, false, CONV_LOG_EPT, CONV_LOG_TILE>;
  const dim3 grid(P::WG_PER_LIMB, ngroups, nz);
  k_conv_fwd1<LOGN, CONV_LOG_EPT, CONV_LOG_TILE, NP><<<grid, P::THREADS, 0, s>>>(
      in, in_bs, out, out_bs, set.d, zdiv, group, c->d_tw, c->d_twp, c->d_dtw, c->d_dtwq, c->d_mod);
}

template <int LOGN>
static int conv_fwd1_n(Ctx* c, const ConvSet& set, const uint64_t* in, size_t in_bs, uint64_t* out, size_t out_bs,
                       int nz, int zdiv, int group, int ngroups, hipStream_t s) {
  const int np = set.max_parts;
  if (np <= 2) conv_fwd1_go<LOGN, 2>(c, set, in, in_bs, out, out_bs, nz, zdiv, group, ngroups, s);
  else if (np <= 4) conv_fwd1_go<LOGN, 4>(c, set, in, in_bs, out, out_bs, nz, zdiv, group, ngroups, s);
  else if (np <= 6) conv_fwd1_go<LOGN, 6>(c, set, in, in_bs, out, out_bs, nz, zdiv, group, ngroups, s);
  else if (np <= 9) conv_fwd1_go<LOGN, 9>(c, set, in, in_bs, out, out_bs, nz, zdiv, group, ngroups, s);
  else if (np <= 12) conv_fwd1_go<LOGN, 12>(c, set, in, in_bs, out, out_bs, nz, zdiv, group, ngroups, s);
  else conv_fwd1_go<LOGN, 2 * MAX_BCONV_IN>(c, set, in, in_bs, out, out_bs, nz, zdiv, group, ngroups, s);
  HE_HIP(hipGetLastError());
  return HE_OK;
}

int conv_fwd1_launch(Ctx* c, const ConvSet& set, const uint64_t* in, size_t in_bs, uint64_t* out, size_t out_bs,
                     int nz, int zdiv, int target, const char* name, hipStream_t s) {
  if (nz <= 0 || set.count <= 0) return HE_OK;
  if (nz > 65535) return set_error(HE_EINVAL, "conversion batch too large for one launch");
  const size_t N = c->n;
  const int tiles = (int)(N >> CONV_LOG_TILE);
  // outputs per group: few enough for about `target` workgroups when the
  // batch is small, at most CONV_MAX_GROUP
  const int want = std::max(1, (target + tiles * nz - 1) / (tiles * nz));
  const int group = std::min(CONV_MAX_GROUP, std::max(1, (set.max_out + want - 1) / want));
  int ngroups = 0;
  for (int t = 0; t < set.count; t++) {
    const int ni = set.nint[t], nf = set.nout[t] - ni;
    ngroups = std::max(ngroups, (ni + group - 1) / group + (nf + group - 1) / group);
  }
  const double items = (double)nz / zdiv;
  const double outs = (double)nz * set.max_out;  // upper bound on the output limbs written
  const int l1 = (c->log_n + 1) / 2;
  ProfScope ps(c, name, s, 8.0 * N * (items * set.max_in * set.count + outs),
               (double)N * outs * (set.max_parts + l1 / 2.0),
               (double)N * outs * (set.max_parts + l1 / 2.0) / PEAK_MODMUL_F64);
  switch (c->log_n) {
    case 12: return conv_fwd1_n<12>(c, set, in, in_bs, out, out_bs, nz, zdiv, group, ngroups, s);
    case 14: return conv_fwd1_n<14>(c, set, in, in_bs, out, out_bs, nz, zdiv, group, ngroups, s);
    case 16: return conv_fwd1_n<16>(c, set, in, in_bs, out, out_bs, nz, zdiv, group, ngroups, s);
  }
  return set_error(HE_EINVAL, "unsupported ring degree");
}

// Workgroup targets tried by conv_autotune (the conversion kernel is
// latency-bound: fewer, longer workgroups re-read less, more of them overlap
// better; the balance depends on the ring and the conversion's shape).
static const int kConvTargets[4] = {512, 768, 1024, 1536};

int conv_autotune(Ctx* c) {
  const int l = c->L;
  const size_t N = c->n, E = (size_t)(l + c->K);
  WS w = ws_layout(c, c->ws);
  hipStream_t s;
  HE_HIP(hipStreamCreate(&s));
  hipEvent_t e0, e1;
  HE_HIP(hipEventCreate(&e0));
  HE_HIP(hipEventCreate(&e1));
  HE_HIP(hipMemsetAsync(c->ws, 0, c->ws_words * 8, s));
  for (int kind = 0; kind < 2; kind++) {
    const ConvSet& set = kind == 0 ? c->modup[l] : c->moddown[l];
    auto run = [&](int target) -> int {
      if (kind == 0) return conv_fwd1_launch(c, set, w.coeff, 0, w.ext, E * N, set.count, set.count, target, "tune", s);
      return conv_fwd1_launch(c, set, w.u, E * N, w.y, (size_t)l * N, 2, 1, target, "tune", s);
    };
    float best = 1e30f;
    for (int t = 0; t < 4; t++) {
      int rc;
      if ((rc = run(kConvTargets[t]))) return rc;  // warm-up
      HE_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 5; r++)
        if ((rc = run(kConvTargets[t]))) return rc;
      HE_HIP(hipEventRecord(e1, s));
      HE_HIP(hipEventSynchronize(e1));
      float ms = 0;
      HE_HIP(hipEventElapsedTime(&ms, e0, e1));
      const float us = ms * 1e3f / 5;
      c->conv_tune_us[kind][t] = us;
      if (us < best) {
        best = us;
        c->conv_target[kind] = kConvTargets[t];
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  HE_HIP(hipStreamSynchronize(s));
  hipStreamDestroy(s);
  return HE_OK;
}

// ModUp's forward transform with the key inner product fused into its last
// pass: pass 1 over every converted limb (`conv`, ext-relative positions),
// then ntt_ip_kernel over the E = level + K output limbs (`outs`).
template <int LOGN, int LOG_EPT, int LOG_TILE, int LOG_EPT_IP, int LOG_TILE_IP>
static int ntt_ip_launch_v(Ctx* c, uint64_t* ext, const LimbMap& conv, const LimbMap& outs, const NttIp& ip,
                           hipStream_t s) {
  using P1 = NttPass<LOGN, 1, false, LOG_EPT, LOG_TILE>;
  using P2 = NttPass<LOGN, 2, false, LOG_EPT_IP, LOG_TILE_IP>;
  const double N = (double)P1::N;
  double nf = 0, nconv_f = 0;
  if (c->prof_on) {
    for (int i = 0; i < conv.n; i++) nconv_f += c->hmod[conv.mod[i]].k <= 50;
    for (int i = 0; i < outs.n; i++) nf += c->hmod[outs.mod[i]].k <= 50;
  }
  if (!ip.ext_ntt && !ip.ext_p1) {
    const double mm = N / 2 * P1::LM * conv.n;
    ProfScope ps(c, "ntt_fwd_pass1", s, 16.0 * N * conv.n, mm,
                 N / 2 * P1::LM * (nconv_f / PEAK_MODMUL_F64 + (conv.n - nconv_f) / PEAK_MODMUL_INT));
    ntt_pass_kernel<LOGN, 1, false, LOG_EPT, LOG_TILE, false><<<dim3(P1::WG_PER_LIMB, 1, conv.n), P1::THREADS, 0, s>>>(
        ext, 0, ext, 0, conv, c->d_tw, c->d_twp, c->d_dtw, c->d_dtwq, c->d_mod, NttEpi{});
  }
  {
    // reads: converted limbs, own limbs of c1, 2 dnum key limbs per output limb; writes: 2 output limbs
    const double own = ip.level;
    const double bytes = 8.0 * N * (conv.n + own + 2.0 * ip.dnum * outs.n + 2.0 * outs.n);
    const double fwd = ip.ext_ntt ? 0.0 : 1.0;  // forward pass 2 of the converted limbs
    const double mm_ntt = fwd * N / 2 * P2::LM * conv.n, mm_ip = 2.0 * ip.dnum * N * outs.n;
    const double ideal =
        fwd * N / 2 * P2::LM * (nconv_f / PEAK_MODMUL_F64 + (conv.n - nconv_f) / PEAK_MODMUL_INT) +
        mm_ip / PEAK_MODMUL_INT;
    ProfScope ps(c, ip.ext_ntt ? "ks_inner_product_tile" : "ntt_fwd_pass2_ip", s, bytes, mm_ntt + mm_ip, ideal);
    const dim3 grid(P2::WG_PER_LIMB, 1, outs.n);
    const size_t lds = (size_t)std::max(ip.dnum, 2) * P2::LDS_WORDS * 8;
    const dim3 blk(ip.dnum * P2::THREADS);
#define HE_IP_LAUNCH(D)                                                                                           \
  ntt_ip_kernel<LOGN, LOG_EPT_IP, LOG_TILE_IP, D><<<grid, blk, lds, s>>>(outs, c->d_tw, c->d_twp, c->d_dtw, c->d_dtwq, \
                                                                   c->d_itw, c->d_itwp, c->d_ditw, c->d_ditwq,   \
                                                                   c->d_mod, ip)
    switch (ip.dnum) {
      case 1: HE_IP_LAUNCH(1); break;
      case 2: HE_IP_LAUNCH(2); break;
      case 3: HE_IP_LAUNCH(3); break;
      default: HE_IP_LAUNCH(4); break;
    }
#undef HE_IP_LAUNCH
  }
  HE_HIP(hipGetLastError());
  return HE_OK;
}

// The fused kernel runs one group of P::THREADS threads per digit with 8
// residues per thread, on output tiles of 2^IP_LOG_TILE positions: smaller
// tiles than pass 1's (whose row segments need the width) give smaller
// workgroups, more of them resident per CU and a shorter tail.
constexpr int IP_LOG_EPT = 3, IP_LOG_TILE = 9;
template <int LOGN>
static int ntt_ip_launch_n(Ctx* c, uint64_t* ext, const LimbMap& conv, const LimbMap& outs, const NttIp& ip,
                           hipStream_t s) {
  LimbMap om = by_modulus(c, outs);
  if (ip.p_inv2) {
    // the special-prime workgroups carry the extra inverse pass: start them first
    LimbMap r = om;
    int n = 0;
    for (int pass = 0; pass < 2; pass++)
      for (int i = 0; i < om.n; i++)
        if ((om.pos[i] >= ip.level) == (pass == 0)) {
          r.pos[n] = om.pos[i];
          r.mod[n] = om.mod[i];
          n++;
        }
    om = r;
  }
  return ntt_ip_launch_v<LOGN, 3, 11, IP_LOG_EPT, IP_LOG_TILE>(c, ext, by_modulus(c, conv), om, ip, s);
}

bool ntt_ip_supported(const Ctx* c, int dnum) {
  size_t words = 0;
  switch (c->log_n) {
    case 12: words = NttPass<12, 2, false, IP_LOG_EPT, IP_LOG_TILE>::LDS_WORDS; break;
    case 14: words = NttPass<14, 2, false, IP_LOG_EPT, IP_LOG_TILE>::LDS_WORDS; break;
    case 16: words = NttPass<16, 2, false, IP_LOG_EPT, IP_LOG_TILE>::LDS_WORDS; break;
    default: return false;
  }
  return dnum >= 1 && dnum <= NTT_IP_MAXD && (size_t)std::max(dnum, 2) * words * 8 <= c->lds_per_block;
}

int ntt_launch_modup_ip(Ctx* c, uint64_t* ext, const LimbMap& conv, const LimbMap& outs, const NttIp& ip,
                        hipStream_t s) {
  if (conv.n <= 0 || outs.n <= 0) return HE_OK;
  switch (c->log_n) {
    case 12: return ntt_ip_launch_n<12>(c, ext, conv, outs, ip, s);
    case 14: return ntt_ip_launch_n<14>(c, ext, conv, outs, ip, s);
    case 16: return ntt_ip_launch_n<16>(c, ext, conv, outs, ip, s);
  }
  return set_error(HE_EINVAL, "unsupported ring degree");
}

int ntt_launch_pass(Ctx* c, const uint64_t* src, size_t src_bs, uint64_t* data, size_t batch_stride, int nbatch,
                    const LimbMap& map, bool inverse, int pass, hipStream_t s) {
  if (map.n <= 0 || nbatch <= 0) return HE_OK;
  const int passes = pass == 1 ? 1 : 2;
  switch (c->log_n) {
    case 12: return ntt_launch_n<12>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s, nullptr, passes);
    case 14: return ntt_launch_n<14>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s, nullptr, passes);
    case 16: return ntt_launch_n<16>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s, nullptr, passes);
  }
  return set_error(HE_EINVAL, "unsupported ring degree");
}

int ntt_launch_from(Ctx* c, const uint64_t* src, uint64_t* data, size_t batch_stride, int nbatch, const LimbMap& map,
                    bool inverse, hipStream_t s) {
  return ntt_launch_strided(c, src, batch_stride, data, batch_stride, nbatch, map, inverse, s);
}

int ntt_launch(Ctx* c, uint64_t* data, size_t batch_stride, int nbatch, const LimbMap& map, bool inverse,
               hipStream_t s) {
  return ntt_launch_from(c, data, data, batch_stride, nbatch, map, inverse, s);
}

}  // namespace he

using namespace he;

extern "C" int he_ntt(he_ctx* h, uint64_t* poly, int n_limbs, int first_limb, int inverse, he_stream stream) {
  if (!h || !poly) return set_error(HE_EINVAL, "null argument");
  Ctx* c = &h->c;
  if (n_limbs < 0 || first_limb < 0 || first_limb + n_limbs > c->L + c->K)
    return set_error(HE_EINVAL, "limb range outside the moduli");
  return ntt_launch(c, poly, 0, 1, range_map(0, n_limbs, first_limb), inverse != 0, (hipStream_t)stream);
}
