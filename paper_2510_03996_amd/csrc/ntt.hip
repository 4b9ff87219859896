// NTT / iNTT kernels and launchers (see ntt_core.h for the decomposition).
#include <algorithm>
#include <type_traits>

#include "internal.h"
#include "ntt_core.h"

namespace he {

// Rounds IDX..NR-1 of a pass, forward order (integer or FP64 arithmetic).
template <class P, int IDX, class T, class TW, class Q>
__device__ __forceinline__ void rounds_fwd(T* lds, int tid, int wg, const TW* tw, const TW* twp, Q q, Q qinv) {
  if constexpr (IDX < P::NR) {
    if constexpr (IDX > 0) __syncthreads();
    if constexpr (std::is_same<T, double>::value)
      P::template round_f64<P::rbits(IDX)>(lds, tid, wg, P::rstart(IDX), tw, twp, q, qinv);
    else
      P::template round<P::rbits(IDX)>(lds, tid, wg, P::rstart(IDX), tw, twp, q);
    rounds_fwd<P, IDX + 1>(lds, tid, wg, tw, twp, q, qinv);
  }
}
// Rounds IDX..0 of a pass, inverse order.
template <class P, int IDX, class T, class TW, class Q>
__device__ __forceinline__ void rounds_inv(T* lds, int tid, int wg, const TW* tw, const TW* twp, Q q, Q qinv) {
  if constexpr (IDX >= 0) {
    if constexpr (std::is_same<T, double>::value)
      P::template round_f64<P::rbits(IDX)>(lds, tid, wg, P::rstart(IDX), tw, twp, q, qinv);
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
    const uint64_t* add = epi.add[z];
    uint64_t x = 0;
    if (add) x = add[off + (z == 0 && epi.g != 1 ? automorph_src(k, epi.g, LOGN) : (uint32_t)k)];
    epi.out[z][off + k] =
        moddown_elem(epi.u[z * epi.u_bs + off + k], v, x, epi.pinv[i], epi.pinv[epi.level + i], q);
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
    if (!INV) rounds_fwd<P, 0>(dl, tid, wg, dtw, dtwq, dq, dqinv);
    else rounds_inv<P, P::NR - 1>(dl, tid, wg, dtw, dtwq, dq, dqinv);
    __syncthreads();
    if constexpr (EPI) {
      // fused ModDown epilogue in centred FP64: v (|v| < 4.2q) is the transform's
      // value before canonicalisation; |u - v| < 6q, the product is below 2q and
      // adding the canonical c0 term stays below 3q, so one canonicalisation ends it
      const size_t off = (size_t)pos << LOGN;
      const double pw = bits_to_f64(epi.pinv[2 * epi.level + pos]);
      const double pwq = bits_to_f64(epi.pinv[3 * epi.level + pos]);
      const uint64_t* add = epi.add[bz];
      const uint64_t* u = epi.u + bz * epi.u_bs + off;
      uint64_t* o = epi.out[bz] + off;
      for (int e = tid; e < P::TILE; e += P::THREADS) {
        int g, k;
        P::tile_elem(e, g, k);
        const int kk = P::gidx(wg, g, k);
        const double r = mul_f64_c(u52_to_f64(u[kk]) - dl[P::lidx(g, k)], pw, pwq, dq);
        double x = 0.0;
        if (add) x = u52_to_f64(add[off + (bz == 0 && epi.g != 1 ? automorph_src(kk, epi.g, LOGN) : (uint32_t)kk)]);
        o[kk] = f64_to_u52(canon_f64(r + x, dqinv, dq));
      }
    } else {
      for (int e = tid; e < P::TILE; e += P::THREADS) {
        int g, k;
        P::tile_elem(e, g, k);
        a[P::gidx(wg, g, k)] = P::finish_f64(dl[P::lidx(g, k)], mi.dninv, mi.dninvq, dq, dqinv);
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
  for (int e = tid; e < P::TILE; e += P::THREADS) {
    int g, k;
    P::tile_elem(e, g, k);
    ntt_store<EPI, LOGN>(a, P::gidx(wg, g, k), P::finish(lds[P::lidx(g, k)], mi.ninv, mi.ninv_p, q), epi,
                         pos, bz, q);
  }
}

template <int LOGN, int LOG_EPT, int LOG_TILE>
static int ntt_launch_v(Ctx* c, const uint64_t* src, size_t src_bs, uint64_t* data, size_t batch_stride,
                        int nbatch, const LimbMap& map, bool inverse, hipStream_t s, const NttEpi* epi = nullptr) {
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
    {
      ProfScope ps(c, "ntt_fwd_pass1", s, bytes, mm1, mm1 * per_mm);
      ntt_pass_kernel<LOGN, 1, false, LOG_EPT, LOG_TILE, false><<<g1, T, 0, s>>>(
          src, src_bs, data, batch_stride, map, c->d_tw, c->d_twp, c->d_dtw, c->d_dtwq, c->d_mod, none);
    }
    if (epi) {
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
    {
      ProfScope ps(c, "ntt_inv_pass2", s, bytes, mm2, mm2 * per_mm);
      ntt_pass_kernel<LOGN, 2, true, LOG_EPT, LOG_TILE, false><<<g2, T, 0, s>>>(
          src, src_bs, data, batch_stride, map, c->d_itw, c->d_itwp, c->d_ditw, c->d_ditwq, c->d_mod, none);
    }
    ProfScope ps(c, "ntt_inv_pass1", s, bytes, mm1 + N * limbs, (mm1 + N * limbs) * per_mm);
    ntt_pass_kernel<LOGN, 1, true, LOG_EPT, LOG_TILE, false><<<g1, T, 0, s>>>(
        data, batch_stride, data, batch_stride, map, c->d_itw, c->d_itwp, c->d_ditw, c->d_ditwq, c->d_mod, none);
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
                          int nbatch, const LimbMap& map, bool inverse, hipStream_t s, const NttEpi* epi = nullptr) {
  switch (var) {
    case 0: return ntt_launch_v<LOGN, 2, 12>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s, epi);
    case 1: return ntt_launch_v<LOGN, 3, 12>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s, epi);
    case 3: return ntt_launch_v<LOGN, 2, 11>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s, epi);
    case 4: return ntt_launch_v<LOGN, 3, 11>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s, epi);
    default: return ntt_launch_v<LOGN, 4, 12>(c, src, src_bs, data, batch_stride, nbatch, map, inverse, s, epi);
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
                        int nbatch, const LimbMap& map, bool inverse, hipStream_t s, const NttEpi* epi = nullptr) {
  return ntt_launch_var<LOGN>(c, c->ntt_var[ntt_bucket(map.n * nbatch)], src, src_bs, data, batch_stride, nbatch,
                              by_modulus(c, map), inverse, s, epi);
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

int ntt_launch_moddown(Ctx* c, const uint64_t* y, size_t y_bs, const LimbMap& map, const NttEpi& epi, hipStream_t s) {
  if (map.n <= 0) return HE_OK;
  // the transform runs in place on y (its scratch); results go to epi.out
  uint64_t* yy = const_cast<uint64_t*>(y);
  switch (c->log_n) {
    case 12: return ntt_launch_n<12>(c, yy, y_bs, yy, y_bs, 2, map, false, s, &epi);
    case 14: return ntt_launch_n<14>(c, yy, y_bs, yy, y_bs, 2, map, false, s, &epi);
    case 16: return ntt_launch_n<16>(c, yy, y_bs, yy, y_bs, 2, map, false, s, &epi);
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
