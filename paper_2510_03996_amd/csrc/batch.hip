// Batched hoisted-rotation multiply-accumulate over many ciphertexts.
//
// Work item (ciphertext i, output o):
//   out[i,o] = RS( sum_t pool[idx(i,o,t)] (.) Rot_{r_{i,t}}(in_i) )
// which is the shape of every convolution / pooling stage of the paper's
// layers (rotated copies of one input, each multiplied by a plaintext and
// summed) and of the batched key-switching workload.
//
// Batched schedule (one stream, optionally captured once in a hipGraph):
//   1. ModUp of every input at once (inverse NTT, conversion fused into the
//      forward column pass, forward row pass);
//   2. key-major key switching: for each distinct rotation key, ONE inner-
//      product launch loads each key residue once and applies it to every
//      ciphertext that uses that key (the key is read from HBM once per
//      batch instead of once per rotation), then one batched ModDown for all
//      of that key's rotations;
//   3. the plaintext pool centred once (k_pool_centre), then one fused MAC
//      launch for all outputs: each thread keeps a group of outputs'
//      accumulators in registers and streams the item's rotated copies once
//      per group (centred FP64 products for the primes below 2^50, 128-bit
//      products otherwise);
//   4. rescale of all outputs in chunks (a ModDown by the top prime).
// The result is bit-identical to the per-op path (he_rotate_hoisted,
// he_mul_plain, he_rescale), which he_batch_run_plain executes for
// comparison: every step is the same exact modular arithmetic.
#include <algorithm>
#include <map>
#include <vector>

#include "internal.h"

namespace he {

constexpr int BATCH_NMAX = 64;  // rotations per ciphertext in one batch

// ---------------------------------------------------------------- kernels
// Inner product of one key with the extended digits of every pair using it.
// grid: x = 256-coefficient tile, y = extended limb.  Pair p uses input
// item[p].  phi_g maps an aligned block of 256 NTT indices onto an aligned
// block (the bit reversal puts the block's varying low bits on top, where
// g (2 brv(j) + 1) mod 2N leaves the low bits alone), so each digit's source
// block is read coalesced into LDS and permuted there instead of gathered
// from HBM.  The next pair's blocks are loaded while the current pair is
// accumulated (two LDS buffers, one barrier per pair).  Primes below 2^50:
// centred FP64 products of the canonical digit values with the
// Montgomery-form key words (each below 1.6q, the sum over at most four
// digits below 6.4q) and one product by 2^-64 mod q; the others: 128-bit
// products and one REDC.  Both give the canonical residue.
template <int DN>
__global__ __launch_bounds__(256) void k_ip_multi(const uint64_t* __restrict__ ext_all, size_t ext_item,
                                                  const uint64_t* __restrict__ in_all, size_t in_item, int level,
                                                  int K, int alpha, const uint64_t* __restrict__ key,
                                                  size_t key_digit_stride, size_t key_poly_stride, int L, uint32_t g,
                                                  int logn, const ModInfo* __restrict__ mods,
                                                  const int32_t* __restrict__ items, int npairs,
                                                  uint64_t* __restrict__ u_all) {
  constexpr int dnum = DN;
  __shared__ uint64_t sh[2][DN][256];
  const size_t n = (size_t)1 << logn;
  const int tid = threadIdx.x;
  const uint32_t k = blockIdx.x * 256 + tid;
  const int pos = blockIdx.y;
  const int E = level + K;
  const int mod = pos < level ? pos : L + (pos - level);
  const ModInfo mi = mods[mod];
  const uint32_t src = g == 1 ? k : automorph_src(k, g, logn);
  const uint32_t s0 = src & ~255u;  // the source block, the same for the whole workgroup
  const int sl = (int)(src & 255u);
  const bool f64 = mi.k <= 50;
  const double dq = (double)mi.q, qi = mi.dqinv;
  uint64_t kb[DN], ka[DN];
#pragma unroll
  for (int j = 0; j < dnum; j++) {
    const uint64_t* kj = key + j * key_digit_stride + (size_t)mod * n + k;
    kb[j] = kj[0];
    ka[j] = kj[key_poly_stride];
  }
  const int own = pos < level ? pos / alpha : -1;
  const size_t En = (size_t)E * n;
  uint64_t cur[DN];
  auto gload = [&](int p) {
    const int it = items[p];
    const uint64_t* c1 = in_all + it * in_item + (size_t)level * n;
    const uint64_t* ext = ext_all + it * ext_item;
#pragma unroll
    for (int j = 0; j < dnum; j++) {
      const uint64_t* sp = j == own ? c1 : ext + j * En;
      cur[j] = sp[(size_t)pos * n + s0 + tid];
    }
  };
  if (npairs > 0) gload(0);
  for (int p = 0; p < npairs; p++) {
    const int b = p & 1;
#pragma unroll
    for (int j = 0; j < dnum; j++) sh[b][j][tid] = cur[j];
    __syncthreads();
    if (p + 1 < npairs) gload(p + 1);
    uint64_t* u = u_all + (size_t)p * 2 * En + (size_t)pos * n + k;
    if (f64) {
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int j = 0; j < dnum; j++) {
        const double v = u52_to_f64(sh[b][j][sl]);
        const double w0 = u52_to_f64(kb[j]), w1 = u52_to_f64(ka[j]);
        a0 += mul_f64_c(v, w0, w0 * qi, dq);
        a1 += mul_f64_c(v, w1, w1 * qi, dq);
      }
      u[0] = f64_to_u52(canon_f64(mul_f64_c(a0, mi.drinv, mi.drinvq, dq), qi, dq));
      u[En] = f64_to_u52(canon_f64(mul_f64_c(a1, mi.drinv, mi.drinvq, dq), qi, dq));
    } else {
      U128 a0{0, 0}, a1{0, 0};
#pragma unroll
      for (int j = 0; j < dnum; j++) {
        const uint64_t e = sh[b][j][sl];
        add_wide(a0, mul_wide(e, kb[j]));
        add_wide(a1, mul_wide(e, ka[j]));
      }
      u[0] = mont_redc(a0, mi.q, mi.qinv);
      u[En] = mont_redc(a1, mi.q, mi.qinv);
    }
  }
}

static int ip_multi_launch(int dn, dim3 grid, hipStream_t s, const uint64_t* ext, size_t ext_item, const uint64_t* in,
                           size_t in_item, int l, int K, int alpha, const uint64_t* key, size_t kds, size_t kps, int L,
                           uint32_t g, int logn, const ModInfo* mods, const int32_t* items, int npairs, uint64_t* u) {
  switch (dn) {
#define HE_IPM(D) \
  case D:         \
    k_ip_multi<D><<<grid, 256, 0, s>>>(ext, ext_item, in, in_item, l, K, alpha, key, kds, kps, L, g, logn, mods, items, \
                                       npairs, u);                                                                    \
    break;
    HE_IPM(1) HE_IPM(2) HE_IPM(3) HE_IPM(4) HE_IPM(5) HE_IPM(6) HE_IPM(7) HE_IPM(8)
#undef HE_IPM
    default:
      return set_error(HE_EINVAL, "too many key-switching digits");
  }
  return HE_OK;
}

// The plaintext pool as the MAC consumes it, once per run: limbs below 2^50
// as the bits of their centred double (|p| <= q/2), the others unchanged.
// grid: (N / 256, limbs, pool entries); pool_c is [entry][level][N].
__global__ __launch_bounds__(256) void k_pool_centre(const uint64_t* __restrict__ pool, size_t pool_stride,
                                                     uint64_t* __restrict__ pool_c, int level, int logn,
                                                     const ModInfo* __restrict__ mods) {
  const size_t n = (size_t)1 << logn;
  const size_t k = (size_t)blockIdx.x * 256 + threadIdx.x;
  const int limb = blockIdx.y;
  const ModInfo mi = mods[limb];
  const uint64_t v = pool[(size_t)blockIdx.z * pool_stride + (size_t)limb * n + k];
  pool_c[((size_t)blockIdx.z * level + limb) * n + k] =
      mi.k <= 50 ? f64_to_bits(centre_f64(u52_to_f64(v), mi.dqinv, (double)mi.q)) : v;
}

// out[i,o] (unrescaled) for every item: grid (items, tiles of 256
// coefficients, limbs of one arithmetic path x polynomial groups), the
// (item, tile) of a workgroup decoded from its linear id as below; the limb
// is limbs[blockIdx.z / (3 - PS)].  A thread keeps OG outputs' accumulators
// of PS polynomials (both, or the one blockIdx.z selects) in registers and
// streams the item's rotated copies once per group of OG outputs; every
// (output, rotation) plaintext residue is read once (from the pool as
// k_pool_centre leaves it, stride level N per entry, mostly from L2: all
// items of a tile run on one XCD in a row).  WIDE instantiations take the
// primes above 2^50 (integer products), the others the primes below 2^50
// (centred FP64 products); each path is its own launch, so each gets the
// registers (and occupancy) its accumulators need.
template <int OG, int PS, bool WIDE>
__global__ __launch_bounds__(256) void k_mac_multi(const uint64_t* __restrict__ rot_all, int level, int logn,
                                                   const ModInfo* __restrict__ mods,
                                                   const int32_t* __restrict__ rot_off,
                                                   const int32_t* __restrict__ rot_idx,
                                                   const int32_t* __restrict__ out_off,
                                                   const int32_t* __restrict__ pt_off,
                                                   const int32_t* __restrict__ pt_index,
                                                   const uint64_t* __restrict__ pool_c,
                                                   const int32_t* __restrict__ limbs,
                                                   uint64_t* __restrict__ mac_all) {
  const size_t n = (size_t)1 << logn;
  // Workgroups go round-robin to the 8 XCDs by linear id (x fastest; gridDim.y,
  // the tile count, is a multiple of 8).  Give each XCD whole coefficient
  // tiles, every item of a tile in a row, so that the plaintext pool's slice
  // of a tile is fetched into that XCD's L2 once and reused by all items.
  const int lin = blockIdx.x + gridDim.x * blockIdx.y;
  const int xcd = lin & 7, r = lin >> 3;
  const int it = r % (int)gridDim.x;
  const size_t k = (size_t)((r / (int)gridDim.x) * 8 + xcd) * 256 + threadIdx.x;
  const int limb = limbs[PS == 2 ? (int)blockIdx.z : (int)blockIdx.z >> 1];
  const int z0 = PS == 2 ? 0 : (int)blockIdx.z & 1;  // first polynomial of this workgroup
  const ModInfo mi = mods[limb];
  const uint64_t q2 = 2 * mi.q;
  const size_t ln = (size_t)level * n;
  const int r0 = rot_off[it], nr = rot_off[it + 1] - r0;
  const int o0 = out_off[it], no = out_off[it + 1] - o0;
  const int32_t* pix = pt_index + pt_off[it];
  const uint64_t* poolk = pool_c + (size_t)limb * n + k;
  const size_t zoff = (size_t)z0 * ln + (size_t)limb * n + k;
  if (!WIDE) {
    // Primes below 2^50: centred FP64 products (mul_f64_c with the quotient
    // estimate p fl(1/q), off by less than 0.1 for |x|, |p| <= q/2 + 1, so
    // every product is exact and below 0.6 q in magnitude).  The sums are
    // re-centred after every eighth term and so stay below 5.3 q < 2^53.
    const double dq = (double)mi.q, dqi = mi.dqinv;
    for (int og = 0; og < no; og += OG) {
      const int cnt = no - og < OG ? no - og : OG;
      double a[OG][PS];
#pragma unroll
      for (int u = 0; u < OG; u++)
#pragma unroll
        for (int z = 0; z < PS; z++) a[u][z] = 0.0;
      // term t's rotated residues and plaintext residues are loaded while
      // term t - 1 is being accumulated (register double buffering), so the
      // HBM and L2 latencies overlap the FP64 work
      uint64_t xr[PS], pr[OG];
      auto load = [&](int t, uint64_t* xv, uint64_t* pv) {
        const uint64_t* rc = rot_all + (size_t)rot_idx[r0 + t] * 2 * ln + zoff;
#pragma unroll
        for (int z = 0; z < PS; z++) xv[z] = rc[z * ln];
        const int32_t* pt = pix + og * nr + t;
#pragma unroll
        for (int u = 0; u < OG; u++) pv[u] = u < cnt ? poolk[(size_t)pt[u * nr] * ln] : 0;
      };
      load(0, xr, pr);
      for (int t = 0; t < nr; t++) {
        uint64_t xn[PS], pn[OG];
        if (t + 1 < nr) load(t + 1, xn, pn);
        double x[PS];
#pragma unroll
        for (int z = 0; z < PS; z++) x[z] = centre_f64(u52_to_f64(xr[z]), dqi, dq);
#pragma unroll
        for (int u = 0; u < OG; u++) {
          if (u < cnt) {
            const double p = bits_to_f64(pr[u]);
            const double pq = p * dqi;
#pragma unroll
            for (int z = 0; z < PS; z++) {
              a[u][z] += mul_f64_c(x[z], p, pq, dq);
              if ((t & 7) == 7) a[u][z] = centre_f64(a[u][z], dqi, dq);
            }
          }
        }
        if (t + 1 < nr) {
#pragma unroll
          for (int z = 0; z < PS; z++) xr[z] = xn[z];
#pragma unroll
          for (int u = 0; u < OG; u++) pr[u] = pn[u];
        }
      }
#pragma unroll
      for (int u = 0; u < OG; u++) {
        if (u < cnt) {
          uint64_t* dst = mac_all + (size_t)(o0 + og + u) * 2 * ln + zoff;
#pragma unroll
          for (int z = 0; z < PS; z++) dst[z * ln] = f64_to_u52(canon_f64(a[u][z], dqi, dq));
        }
      }
    }
    return;
  }
  // Primes above 2^50: 128-bit products; accumulators stay below 4 q 2^64 by
  // subtracting 2 q 2^64 (a multiple of q) after every second term; two
  // REDCs give the canonical residue.
  for (int og = 0; og < no; og += OG) {
    const int cnt = no - og < OG ? no - og : OG;
    U128 a[OG][PS];
#pragma unroll
    for (int u = 0; u < OG; u++)
#pragma unroll
      for (int z = 0; z < PS; z++) a[u][z] = U128{0, 0};
    for (int t = 0; t < nr; t++) {
      const uint64_t* rc = rot_all + (size_t)rot_idx[r0 + t] * 2 * ln + zoff;
      uint64_t x[PS];
#pragma unroll
      for (int z = 0; z < PS; z++) x[z] = rc[z * ln];
#pragma unroll
      for (int u = 0; u < OG; u++) {
        if (u < cnt) {
          const uint64_t p = poolk[(size_t)pix[(og + u) * nr + t] * ln];
#pragma unroll
          for (int z = 0; z < PS; z++) {
            add_wide(a[u][z], mul_wide(p, x[z]));
            if ((t & 1) && a[u][z].hi >= q2) a[u][z].hi -= q2;
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < OG; u++) {
      if (u < cnt) {
        uint64_t* dst = mac_all + (size_t)(o0 + og + u) * 2 * ln + zoff;
#pragma unroll
        for (int z = 0; z < PS; z++) {
          U128 v = a[u][z];
          if (v.hi >= q2) v.hi -= q2;
          if (v.hi >= mi.q) v.hi -= mi.q;
          dst[z * ln] = mont_redc(mul_wide(mont_redc(v, mi.q, mi.qinv), mi.r2), mi.q, mi.qinv);
        }
      }
    }
  }
}

// MAC variants (outputs per register group, polynomials per workgroup)
constexpr int MAC_VARIANTS = 5;
constexpr int MAC_OG[MAC_VARIANTS] = {4, 8, 16, 16, 32};
constexpr int MAC_PS[MAC_VARIANTS] = {2, 2, 2, 1, 1};
constexpr int MAC_DEFAULT = 2;

// FP64 limbs with variant v, then the integer limbs (8 outputs, both
// polynomials per workgroup)
static void launch_mac(int v, int B, int tiles, int l, hipStream_t s, const uint64_t* rot, int logn,
                       const ModInfo* mods, const int32_t* ro, const int32_t* ri, const int32_t* oo, const int32_t* po,
                       const int32_t* pi, const uint64_t* pool_c, const int32_t* limbs_f, int nf,
                       const int32_t* limbs_i, int ni, uint64_t* mac) {
  if (nf > 0) {
    const dim3 grid(B, tiles, nf * (3 - MAC_PS[v]));
#define HE_MAC(i, OG, PS) \
  case i:                 \
    k_mac_multi<OG, PS, false><<<grid, 256, 0, s>>>(rot, l, logn, mods, ro, ri, oo, po, pi, pool_c, limbs_f, mac); \
    break;
    switch (v) {
      HE_MAC(0, 4, 2)
      HE_MAC(1, 8, 2)
      HE_MAC(2, 16, 2)
      HE_MAC(3, 16, 1)
      default:
      HE_MAC(4, 32, 1)
    }
#undef HE_MAC
  }
  if (ni > 0)
    k_mac_multi<8, 2, true><<<dim3(B, tiles, ni), 256, 0, s>>>(rot, l, logn, mods, ro, ri, oo, po, pi, pool_c, limbs_i,
                                                               mac);
}

// ---------------------------------------------------------------- plan
struct KeyGroup {
  int32_t rot;        // rotation amount (normalised)
  uint32_t g;         // Galois element
  const uint64_t* key;
  int npairs;
  int first_pair;     // index of its first pair in rot_all (key-major order)
  int32_t* d_items;   // device: item of each pair
};

struct Batch {
  Ctx* c = nullptr;
  he_ctx* h = nullptr;
  int B = 0, level = 0, npool = 0, pool_level = 0;
  double in_scale = 0, pt_scale = 0;
  const uint64_t* in = nullptr;
  const uint64_t* pool = nullptr;
  uint64_t* out = nullptr;
  std::vector<int32_t> n_rot, n_out, rots, pt_index;  // host copies
  std::vector<int32_t> rot_off, out_off, pt_off;
  int total_pairs = 0, total_out = 0, max_group = 0;
  std::vector<KeyGroup> groups;
  // device tables
  int32_t *d_rot_off = nullptr, *d_rot_idx = nullptr, *d_out_off = nullptr, *d_pt_off = nullptr,
          *d_pt_index = nullptr;
  // device workspaces
  uint64_t *coeff = nullptr, *ext = nullptr, *u = nullptr, *y = nullptr, *rot = nullptr, *mac = nullptr,
           *rs_T = nullptr, *rs_R = nullptr, *pool_c = nullptr;
  int32_t *d_limbs_f = nullptr, *d_limbs_i = nullptr;  // limbs of the MAC's FP64 / integer paths
  int n_limbs_f = 0, n_limbs_i = 0;
  int rs_chunk = 0;
  int mac_v = MAC_DEFAULT;  // MAC variant (register grouping; autotuned)
  int nmax = 0;    // largest rotation set
  std::vector<void*> allocs;
  std::vector<int32_t> locked;  // keys held resident for the batch
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_graph = false;
  float tuned_ms[MAC_VARIANTS] = {0, 0, 0, 0, 0};
  double out_scale = 0;
};

template <class T>
static int balloc(Batch* b, T** p, size_t count) {
  void* v = nullptr;
  hipError_t e = hipMalloc(&v, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) return set_error(HE_ENOMEM, std::string("batch workspace: ") + hipGetErrorString(e));
  b->allocs.push_back(v);
  *p = (T*)v;
  return HE_OK;
}

static void batch_free(Batch* b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  for (void* p : b->allocs) hipFree(p);
  b->allocs.clear();
  for (int32_t id : b->locked) key_lock(b->c, id, -1);
  b->locked.clear();
}

// ---------------------------------------------------------------- execution
static int run_batched(Batch* b, hipStream_t s) {
  Ctx* c = b->c;
  const size_t N = c->n;
  const int l = b->level, K = c->K, L = c->L, dn = c->dnum(l);
  const size_t E = (size_t)(l + K), ln = (size_t)l * N, in_item = 2 * ln;
  const size_t ext_item = (size_t)dn * E * N;
  int rc;
  // 1. ModUp of every input: inverse transform into the conversion inputs,
  // conversion + forward pass 1, forward pass 2
  if ((rc = ntt_launch_conv_in(c, b->in + ln, in_item, b->coeff, ln, b->B, range_map(0, l, 0), c->d_fin[l], 3, s)))
    return rc;
  {
    const ConvSet& set = c->modup[l];
    if ((rc = conv_fwd1_launch(c, set, b->coeff, ln, b->ext, E * N, b->B * set.count, set.count, c->conv_target[0],
                               "conv_fwd1_modup", s)))
      return rc;
  }
  if ((rc = ntt_launch_pass(c, b->ext, ext_item, b->ext, ext_item, b->B, c->modup_ntt[l], false, 2, s))) return rc;
  // 2. key-major key switching
  const size_t kps = (size_t)(L + K) * N;
  for (const KeyGroup& gk : b->groups) {
    {
      ProfScope ps(c, "ks_inner_product_multi", s, 8.0 * N * E * (2.0 * dn + gk.npairs * (dn + 2.0)),
                   2.0 * dn * E * N * gk.npairs);
      if ((rc = ip_multi_launch(dn, dim3(N / 256, E), s, b->ext, ext_item, b->in, in_item, l, K, c->alpha, gk.key,
                                2 * kps, kps, L, gk.g, c->log_n, c->d_mod, gk.d_items, gk.npairs, b->u)))
        return rc;
      HE_HIP(hipGetLastError());
    }
    const int z = 2 * gk.npairs;
    if ((rc = ntt_launch_conv_in(c, b->u, E * N, b->u, E * N, z, range_map(l, K, L), c->d_fin[l], 3, s))) return rc;
    if ((rc = conv_fwd1_launch(c, c->moddown[l], b->u, E * N, b->y, ln, z, 1, c->conv_target[1], "conv_fwd1_moddown",
                               s)))
      return rc;
    // back to NTT form with the ModDown combine in the last pass: rotated copy
    // z = 2 pair + poly = add + (u - y) P^{-1}, add = phi_g(c0 of the pair's item) for poly 0
    NttEpi epi{};
    epi.u = b->u;
    epi.u_bs = E * N;
    epi.pinv = c->d_pinv[l];
    epi.g = gk.g;
    epi.level = l;
    epi.items = gk.d_items;
    epi.add_base = b->in;
    epi.add_item = in_item;
    epi.out_base = b->rot + (size_t)gk.first_pair * 2 * ln;
    epi.out_bs = ln;
    if ((rc = ntt_launch_moddown(c, b->y, ln, range_map(0, l, 0), epi, s, z, 2))) return rc;
  }
  // 3. fused multiply-accumulate of every output
  {
    double terms = 0;
    for (int i = 0; i < b->B; i++) terms += (double)b->n_rot[i] * b->n_out[i];
    int nf = 0;  // limbs on the FP64 path
    for (int i = 0; i < l; i++) nf += c->hmod[i].k <= 50;
    {
      ProfScope pc(c, "pool_centre", s, 16.0 * N * l * b->npool, 0);
      k_pool_centre<<<dim3(N / 256, l, b->npool), 256, 0, s>>>(b->pool, (size_t)b->pool_level * N, b->pool_c, l,
                                                               c->log_n, c->d_mod);
      HE_HIP(hipGetLastError());
    }
    ProfScope ps(c, "mac_multi", s, 8.0 * N * l * (2.0 * b->total_pairs + terms + 2.0 * b->total_out), 2.0 * N * l * terms,
                 2.0 * N * terms * (nf / PEAK_MODMUL_F64 + (l - nf) / PEAK_MODMUL_INT));
    launch_mac(b->mac_v, b->B, (int)(N / 256), l, s, b->rot, c->log_n, c->d_mod, b->d_rot_off, b->d_rot_idx,
               b->d_out_off, b->d_pt_off, b->d_pt_index, b->pool_c, b->d_limbs_f, b->n_limbs_f, b->d_limbs_i,
               b->n_limbs_i, b->mac);
    HE_HIP(hipGetLastError());
  }
  // 4. rescale every output (chunks of rs_chunk ciphertexts = 2 rs_chunk
  // polynomials): a ModDown by q_{l-1} whose epilogue writes the outputs
  const int t = l - 1;
  for (int o0 = 0; o0 < b->total_out; o0 += b->rs_chunk) {
    const int cnt = std::min(b->rs_chunk, b->total_out - o0);
    if ((rc = rescale_launch(c, b->mac + (size_t)o0 * 2 * ln, ln, b->out + (size_t)o0 * 2 * t * N, (size_t)t * N,
                             2 * cnt, l, b->rs_T, b->rs_R, s)))
      return rc;
  }
  return HE_OK;
}

}  // namespace he

using namespace he;

struct he_batch {
  Batch b;
};

extern "C" {

int he_batch_create(he_ctx* h, const he_batch_desc* d, int flags, he_batch** out) {
  if (!h || !d || !out) return set_error(HE_EINVAL, "null argument");
  *out = nullptr;
  Ctx* c = &h->c;
  if (d->n_items < 1 || d->level < 2 || d->level > c->L || !d->in || !d->out || !d->pool || d->n_pool < 1 ||
      d->pool_level < d->level || !d->n_rot || !d->n_out || !d->rots || !d->pt_index)
    return set_error(HE_EINVAL, "bad batch description");
  he_batch* hb = new he_batch();
  Batch* b = &hb->b;
  b->c = c;
  b->h = h;
  b->B = d->n_items;
  b->level = d->level;
  b->in = d->in;
  b->out = d->out;
  b->pool = d->pool;
  b->npool = d->n_pool;
  b->pool_level = d->pool_level;
  b->in_scale = d->in_scale;
  b->pt_scale = d->pt_scale;
  b->use_graph = (flags & HE_BATCH_GRAPH) != 0;
  auto fail = [&](int rc) {
    batch_free(b);
    delete hb;
    return rc;
  };
  // host tables
  b->rot_off.assign(b->B + 1, 0);
  b->out_off.assign(b->B + 1, 0);
  b->pt_off.assign(b->B + 1, 0);
  for (int i = 0; i < b->B; i++) {
    const int nr = d->n_rot[i], no = d->n_out[i];
    if (nr < 1 || nr > BATCH_NMAX || no < 1) return fail(set_error(HE_EINVAL, "each item needs 1..64 rotations and >= 1 output"));
    b->n_rot.push_back(nr);
    b->n_out.push_back(no);
    b->rot_off[i + 1] = b->rot_off[i] + nr;
    b->out_off[i + 1] = b->out_off[i] + no;
    b->pt_off[i + 1] = b->pt_off[i] + nr * no;
  }
  b->total_pairs = b->rot_off[b->B];
  b->total_out = b->out_off[b->B];
  b->rots.assign(d->rots, d->rots + b->total_pairs);
  b->pt_index.assign(d->pt_index, d->pt_index + b->pt_off[b->B]);
  for (int32_t x : b->pt_index)
    if (x < 0 || x >= b->npool) return fail(set_error(HE_EINVAL, "plaintext index outside the pool"));
  // key groups (key-major order of all (item, rotation) pairs)
  std::map<int32_t, std::vector<std::pair<int, int>>> by_key;  // rot -> (item, t)
  for (int i = 0; i < b->B; i++) {
    std::vector<int32_t> seen;
    for (int t = 0; t < b->n_rot[i]; t++) {
      int32_t r = norm_key_id(c, b->rots[b->rot_off[i] + t]);
      if (r == 0) return fail(set_error(HE_EINVAL, "rotation by 0 is not a key switch"));
      for (int32_t x : seen)
        if (x == r) return fail(set_error(HE_EINVAL, "rotation amounts of an item must be distinct"));
      seen.push_back(r);
      if (!key_known(c, r)) return fail(set_error(HE_ENOKEY, "rotation key " + std::to_string(r) + " not resident"));
      by_key[r].push_back({i, t});
    }
  }
  std::vector<int32_t> rot_idx(b->total_pairs);
  int gp = 0;
  int rc;
  for (auto& kv : by_key) {
    KeyGroup g;
    g.rot = kv.first;
    g.g = galois_elt(c, kv.first);
    // the batch captures the key's device address: load it now and hold it
    // resident until the batch is destroyed
    g.key = key_acquire(c, kv.first, nullptr);
    if (!g.key) return fail(HE_ENOMEM);
    key_lock(c, kv.first, 1);
    b->locked.push_back(kv.first);
    g.npairs = (int)kv.second.size();
    g.first_pair = gp;
    std::vector<int32_t> items;
    for (auto& it : kv.second) {
      items.push_back(it.first);
      rot_idx[b->rot_off[it.first] + it.second] = gp++;
    }
    if ((rc = balloc(b, &g.d_items, items.size()))) return fail(rc);
    HE_HIP(hipMemcpy(g.d_items, items.data(), items.size() * 4, hipMemcpyHostToDevice));
    b->max_group = std::max(b->max_group, g.npairs);
    b->groups.push_back(g);
  }
  // keys loaded for the batch (on the null stream) must be complete before any
  // stream runs it: its kernels read the captured addresses without a wait
  if (hipStreamSynchronize(nullptr) != hipSuccess) return fail(set_error(HE_EHIP, "key load failed"));
  // device tables
  auto up = [&](int32_t** dst, const std::vector<int32_t>& v) -> int {
    int r = balloc(b, dst, v.size());
    if (r) return r;
    HE_HIP(hipMemcpy(*dst, v.data(), v.size() * 4, hipMemcpyHostToDevice));
    return HE_OK;
  };
  std::vector<int32_t> lf, li;  // the MAC's limbs by arithmetic path
  for (int i = 0; i < b->level; i++) (c->hmod[i].k <= 50 ? lf : li).push_back(i);
  b->n_limbs_f = (int)lf.size();
  b->n_limbs_i = (int)li.size();
  if ((rc = up(&b->d_rot_off, b->rot_off)) || (rc = up(&b->d_rot_idx, rot_idx)) || (rc = up(&b->d_out_off, b->out_off)) ||
      (rc = up(&b->d_pt_off, b->pt_off)) || (rc = up(&b->d_pt_index, b->pt_index)) || (rc = up(&b->d_limbs_f, lf)) ||
      (rc = up(&b->d_limbs_i, li)))
    return fail(rc);
  // workspaces
  const size_t N = c->n, l = b->level, K = c->K, dn = c->dnum(b->level), E = l + K;
  b->rs_chunk = std::min(b->total_out, 128);
  if ((rc = balloc(b, &b->coeff, (size_t)b->B * l * N)) || (rc = balloc(b, &b->ext, (size_t)b->B * dn * E * N)) ||
      (rc = balloc(b, &b->u, (size_t)b->max_group * 2 * E * N)) || (rc = balloc(b, &b->y, (size_t)b->max_group * 2 * l * N)) ||
      (rc = balloc(b, &b->rot, (size_t)b->total_pairs * 2 * l * N)) ||
      (rc = balloc(b, &b->mac, (size_t)b->total_out * 2 * l * N)) || (rc = balloc(b, &b->rs_T, (size_t)2 * b->rs_chunk * N)) ||
      (rc = balloc(b, &b->rs_R, (size_t)2 * b->rs_chunk * (l - 1) * N)) ||
      (rc = balloc(b, &b->pool_c, (size_t)b->npool * l * N)))
    return fail(rc);
  for (int x : b->n_rot) b->nmax = std::max(b->nmax, x);
  b->mac_v = (flags & HE_BATCH_MAC4) ? 0 : MAC_DEFAULT;
  const int sel = (flags >> 8) & 15;  // HE_BATCH_MAC_SELECT(v) = (v + 1) << 8
  if (sel > MAC_VARIANTS) return fail(set_error(HE_EINVAL, "unknown MAC variant"));
  if (sel) b->mac_v = sel - 1;
  if ((flags & HE_BATCH_TUNE) && !sel) {
    // time every register grouping of the fused MAC on this batch's shapes
    // (workspace contents are irrelevant to the timing) and keep the fastest
    hipStream_t ts;
    HE_HIP(hipStreamCreate(&ts));
    hipEvent_t e0, e1;
    HE_HIP(hipEventCreate(&e0));
    HE_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    k_pool_centre<<<dim3(N / 256, l, b->npool), 256, 0, ts>>>(b->pool, (size_t)b->pool_level * N, b->pool_c, l,
                                                              c->log_n, c->d_mod);
    HE_HIP(hipGetLastError());
    for (int v = 0; v < MAC_VARIANTS; v++) {
      launch_mac(v, b->B, (int)(N / 256), l, ts, b->rot, c->log_n, c->d_mod, b->d_rot_off, b->d_rot_idx,
                 b->d_out_off, b->d_pt_off, b->d_pt_index, b->pool_c, b->d_limbs_f, b->n_limbs_f, b->d_limbs_i,
                 b->n_limbs_i, b->mac);
      HE_HIP(hipEventRecord(e0, ts));
      launch_mac(v, b->B, (int)(N / 256), l, ts, b->rot, c->log_n, c->d_mod, b->d_rot_off, b->d_rot_idx,
                 b->d_out_off, b->d_pt_off, b->d_pt_index, b->pool_c, b->d_limbs_f, b->n_limbs_f, b->d_limbs_i,
                 b->n_limbs_i, b->mac);
      HE_HIP(hipEventRecord(e1, ts));
      HE_HIP(hipEventSynchronize(e1));
      float ms = 0;
      HE_HIP(hipEventElapsedTime(&ms, e0, e1));
      b->tuned_ms[v] = ms;
      if (ms < best) {
        best = ms;
        b->mac_v = v;
      }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipStreamDestroy(ts);
  }
  b->out_scale = b->in_scale * b->pt_scale / (double)c->mod[b->level - 1];
  *out = hb;
  return HE_OK;
}

int he_batch_run(he_batch* hb, he_stream st) {
  if (!hb) return set_error(HE_EINVAL, "null batch");
  Batch* b = &hb->b;
  hipStream_t s = (hipStream_t)st;
  HE_HIP(hipSetDevice(b->c->device));
  if (!b->use_graph || b->c->prof_on) return run_batched(b, s);
  if (!b->exec) {
    if (!s) return set_error(HE_EINVAL, "graph capture needs a non-default stream");
    HE_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = run_batched(b, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (rc) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
    b->graph = g;
    HE_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  }
  HE_HIP(hipGraphLaunch(b->exec, s));
  return HE_OK;
}

int he_batch_run_plain(he_batch* hb, he_stream st) {
  if (!hb) return set_error(HE_EINVAL, "null batch");
  Batch* b = &hb->b;
  Ctx* c = b->c;
  he_ctx* h = b->h;
  const size_t N = c->n, l = b->level;
  // temporaries: the rotated copies of one input and one accumulator
  int nmax = 0;
  for (int x : b->n_rot) nmax = std::max(nmax, x);
  Lane* lane = lane_for(c, (hipStream_t)st);
  if (!lane) return HE_ENOMEM;
  std::vector<uint64_t*> tmp;
  auto cleanup = [&]() {
    for (uint64_t* p : tmp) lane->ct_pool.push_back(p);
  };
  for (int i = 0; i < nmax + 1; i++) {
    uint64_t* p = lane_ct_get(c, lane);
    if (!p) {
      cleanup();
      return HE_ENOMEM;
    }
    tmp.push_back(p);
  }
  std::vector<he_ct> rot(nmax);
  int rc = HE_OK;
  for (int i = 0; i < b->B && !rc; i++) {
    const int nr = b->n_rot[i];
    he_ct in{const_cast<uint64_t*>(b->in) + (size_t)i * 2 * l * N, (int32_t)l, (int32_t)l, b->in_scale};
    for (int t = 0; t < nr; t++) rot[t] = he_ct{tmp[t], 0, c->L, 0};
    rc = he_rotate_hoisted(h, &in, b->rots.data() + b->rot_off[i], nr, rot.data(), st);
    he_ct acc{tmp[nmax], 0, c->L, 0};
    for (int o = 0; o < b->n_out[i] && !rc; o++) {
      for (int t = 0; t < nr && !rc; t++) {
        const int32_t pi = b->pt_index[b->pt_off[i] + o * nr + t];
        he_pt pt{b->pool + (size_t)pi * b->pool_level * N, b->pool_level, b->pt_scale};
        rc = he_mul_plain(h, &rot[t], &pt, &acc, t > 0, st);
      }
      he_ct dst{b->out + (size_t)(b->out_off[i] + o) * 2 * (l - 1) * N, 0, (int32_t)(l - 1), 0};
      if (!rc) rc = he_rescale(h, &acc, &dst, st);
    }
  }
  cleanup();
  return rc;
}

int he_batch_info(const he_batch* hb, int32_t* total_rotations, int32_t* total_outputs, int32_t* distinct_keys,
                  double* out_scale) {
  if (!hb) return set_error(HE_EINVAL, "null batch");
  const Batch* b = &hb->b;
  if (total_rotations) *total_rotations = b->total_pairs;
  if (total_outputs) *total_outputs = b->total_out;
  if (distinct_keys) *distinct_keys = (int32_t)b->groups.size();
  if (out_scale) *out_scale = b->out_scale;
  return HE_OK;
}

int he_batch_tuning(const he_batch* hb, int32_t* outputs_per_group, int32_t* polys_per_group, float* ms,
                    int32_t cap) {
  if (!hb) return set_error(HE_EINVAL, "null batch");
  if (ms && cap < MAC_VARIANTS) return set_error(HE_EINVAL, "ms needs HE_BATCH_MAC_VARIANTS entries");
  if (outputs_per_group) *outputs_per_group = MAC_OG[hb->b.mac_v];
  if (polys_per_group) *polys_per_group = MAC_PS[hb->b.mac_v];
  if (ms)
    for (int v = 0; v < MAC_VARIANTS; v++) ms[v] = hb->b.tuned_ms[v];
  return HE_OK;
}

int he_batch_destroy(he_batch* hb) {
  if (!hb) return HE_OK;
  hipDeviceSynchronize();
  batch_free(&hb->b);
  delete hb;
  return HE_OK;
}

}  // extern "C"
