// Hybrid key switching (ModUp -> key inner product -> ModDown), rotations,
// hoisted rotations and relinearization.
//
// Pinned formula for every key switch (one formula for plain and hoisted
// rotations): digits of c1 are basis-extended once (ModUp), the Galois
// automorphism phi_g is applied to the extended digits as an NTT-form index
// gather fused into the inner-product load, then ModDown.
#include <mutex>
#include <string>

#include "internal.h"

namespace he {

// ---------------------------------------------------------------- kernels
__global__ __launch_bounds__(256) void k_ip(const uint64_t* __restrict__ ext, size_t ext_stride,
                                            const uint64_t* __restrict__ c1, int alpha, int dnum,
                                            const uint64_t* __restrict__ key, size_t key_digit_stride,
                                            size_t key_poly_stride, int level, int L, uint32_t g, int logn,
                                            const ModInfo* __restrict__ mods, uint64_t* __restrict__ u,
                                            size_t u_poly_stride) {
  const size_t n = (size_t)1 << logn;
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  const int pos = blockIdx.y;
  const int mod = pos < level ? pos : L + (pos - level);
  const uint32_t src = g == 1 ? k : automorph_src(k, g, logn);
  ip_elem(ext, ext_stride, pos < level ? c1 : nullptr, alpha, dnum, key, key_digit_stride, key_poly_stride, pos,
          mod, n, k, src, mods[mod], u, u, u_poly_stride);
}

// Inner products of one input's extended digits with several keys (a
// hoisted set): grid x = 256-coefficient *source* block, y = extended limb;
// the workgroup loops over the nz rotations of the round (key tab.key[z],
// Galois element tab.g[z], its inverse tab.ginv[z]; the table is a kernel
// argument), writing u_z = u + z 2 (level+K) N, [2][level+K][N].  phi_g maps
// an aligned block of 256 NTT indices onto an aligned block, so the digits'
// source block is read once, coalesced, into LDS and serves every rotation:
// for rotation z the workgroup writes the output block whose sources form
// its block (the block of phi_{g^-1}(s0)), gathering from LDS; the key words
// and outputs of that block are coalesced, and the next rotation's key
// words are loaded while the current one is accumulated.
// Primes below 2^50: centred FP64 products with the Montgomery-form key
// words and one product by 2^-64 mod q; the others: 128-bit products and one
// REDC (the same canonical residue).
template <int DN>
__global__ __launch_bounds__(256) void k_ip_set(const uint64_t* __restrict__ ext, const uint64_t* __restrict__ c1,
                                                int level, int K, int alpha, const SetTab tab, int nz,
                                                size_t key_digit_stride, size_t key_poly_stride, int L, int logn,
                                                const ModInfo* __restrict__ mods, uint64_t* __restrict__ u_all) {
  __shared__ uint64_t sh[DN][256];
  const size_t n = (size_t)1 << logn;
  const int tid = threadIdx.x;
  const uint32_t s0 = blockIdx.x * 256;  // this workgroup's source block
  const int pos = blockIdx.y;
  const int E = level + K;
  const size_t En = (size_t)E * n;
  const int mod = pos < level ? pos : L + (pos - level);
  const ModInfo mi = mods[mod];
  const int own = pos < level ? pos / alpha : -1;
  const bool f64 = mi.k <= 50;
  const double dq = (double)mi.q, qi = mi.dqinv;
#pragma unroll
  for (int j = 0; j < DN; j++) {
    const uint64_t* sp = j == own ? c1 : ext + j * En;
    sh[j][tid] = sp[(size_t)pos * n + s0 + tid];
  }
  // rotation z: this thread's output position k (in the output block of s0)
  // and the LDS slot of its source; its key words
  uint64_t kb[DN], ka[DN], nkb[DN], nka[DN];
  uint32_t kk = 0, nkk = 0;
  int sl = 0, nsl = 0;
  auto kload = [&](int z, uint64_t* b, uint64_t* a, uint32_t& kout, int& slot) {
    const uint32_t g = tab.g[z];
    const uint32_t o0 = g == 1 ? s0 : (automorph_src(s0, tab.ginv[z], logn) & ~255u);
    const uint32_t k = o0 + tid;
    slot = (int)((g == 1 ? k : automorph_src(k, g, logn)) - s0);
    kout = k;
    const uint64_t* key = tab.key[z];
#pragma unroll
    for (int j = 0; j < DN; j++) {
      const uint64_t* kj = key + j * key_digit_stride + (size_t)mod * n + k;
      b[j] = kj[0];
      a[j] = kj[key_poly_stride];
    }
  };
  kload(0, kb, ka, kk, sl);
  __syncthreads();  // sh
  // unrolled over the table, so that its entries (kernel arguments) are read
  // with constant indices
#pragma unroll
  for (int z = 0; z < SET_MAX; z++) {
    if (z >= nz) break;
    if (z + 1 < nz) kload(z + 1, nkb, nka, nkk, nsl);
    uint64_t* u = u_all + (size_t)z * 2 * En + (size_t)pos * n + kk;
    if (f64) {
      double a0 = 0.0, a1 = 0.0;
#pragma unroll
      for (int j = 0; j < DN; j++) {
        const double v = u52_to_f64(sh[j][sl]);
        const double w0 = u52_to_f64(kb[j]), w1 = u52_to_f64(ka[j]);
        a0 += mul_f64_c(v, w0, w0 * qi, dq);
        a1 += mul_f64_c(v, w1, w1 * qi, dq);
      }
      u[0] = f64_to_u52(canon_f64(mul_f64_c(a0, mi.drinv, mi.drinvq, dq), qi, dq));
      u[En] = f64_to_u52(canon_f64(mul_f64_c(a1, mi.drinv, mi.drinvq, dq), qi, dq));
    } else {
      U128 a0{0, 0}, a1{0, 0};
#pragma unroll
      for (int j = 0; j < DN; j++) {
        const uint64_t e = sh[j][sl];
        add_wide(a0, mul_wide(e, kb[j]));
        add_wide(a1, mul_wide(e, ka[j]));
      }
      u[0] = mont_redc(a0, mi.q, mi.qinv);
      u[En] = mont_redc(a1, mi.q, mi.qinv);
    }
    if (z + 1 < nz) {
#pragma unroll
      for (int j = 0; j < DN; j++) {
        kb[j] = nkb[j];
        ka[j] = nka[j];
      }
      kk = nkk;
      sl = nsl;
    }
  }
}

__global__ void k_set_tab(SetTab t, SetTab* dst) {
  if (threadIdx.x == 0) *dst = t;
}

// x -> x 2^64 mod q on every limb of a [dnum][2][L+K][N] key
__global__ __launch_bounds__(256) void k_to_mont(uint64_t* key, int M, int logn, const ModInfo* __restrict__ mods) {
  const size_t n = (size_t)1 << logn;
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int limb = blockIdx.y;  // over dnum*2*M
  const ModInfo mi = mods[limb % M];
  uint64_t* p = key + (size_t)limb * n + k;
  *p = mont_redc(mul_wide(*p % mi.q, mi.r2), mi.q, mi.qinv);
}

// ---------------------------------------------------------------- building blocks
// ModUp up to the forward column pass: the inverse transform of c1's digits
// (NTT form, `level` limbs) finishes with N^{-1} (Q_j/q_i)^{-1}, so it writes
// the conversion inputs t_i into w.coeff; one launch then converts every
// digit to its other limbs (Q_l \ Q_j) u P and runs their forward pass 1,
// writing digit j's limbs to w.ext + j (level+K) N (the digit's own limbs stay
// in c1).
static int ks_modup_convert(Ctx* c, const WS& w, const uint64_t* c1, int level, hipStream_t s) {
  const size_t N = c->n;
  const size_t E = (size_t)(level + c->K);
  int rc;
  if ((rc = ntt_launch_conv_in(c, c1, 0, w.coeff, 0, 1, range_map(0, level, 0), c->d_fin[level], 3, s))) return rc;
  const ConvSet& set = c->modup[level];
  return conv_fwd1_launch(c, set, w.coeff, 0, w.ext, E * N, set.count, set.count, c->conv_target[0],
                          "conv_fwd1_modup", s);
}

// ModUp: the extended digits in NTT form in w.ext
int ks_modup(Ctx* c, const WS& w, const uint64_t* c1, int level, hipStream_t s) {
  int rc;
  if ((rc = ks_modup_convert(c, w, c1, level, s))) return rc;
  return ntt_launch_pass(c, w.ext, 0, w.ext, 0, 1, c->modup_ntt[level], false, 2, s);
}

// ModDown of w.u (both polynomials) and the final additions
// (p_inv2: the special-prime limbs of w.u are already after inverse pass 2).
// The inverse transform of the special limbs writes the conversion inputs,
// the conversion writes forward pass 1 of the Q limbs into w.y, and the last
// forward pass applies (u - y) P^{-1} + add.
static int ks_moddown(Ctx* c, const WS& w, int level, uint32_t g, const uint64_t* add0, const uint64_t* add1,
                      uint64_t* out0, uint64_t* out1, hipStream_t s, bool p_inv2 = false) {
  const size_t N = c->n;
  const int K = c->K, L = c->L;
  const size_t E = (size_t)(level + K);
  int rc;
  if ((rc = ntt_launch_conv_in(c, w.u, E * N, w.u, E * N, 2, range_map(level, K, L), c->d_fin[level], p_inv2 ? 1 : 3,
                               s)))
    return rc;
  if ((rc = conv_fwd1_launch(c, c->moddown[level], w.u, E * N, w.y, (size_t)level * N, 2, 1, c->conv_target[1],
                              "conv_fwd1_moddown", s)))
    return rc;
  NttEpi epi{};
  epi.u = w.u;
  epi.u_bs = E * N;
  epi.add[0] = add0;
  epi.add[1] = add1;
  epi.out[0] = out0;
  epi.out[1] = out1;
  epi.pinv = c->d_pinv[level];
  epi.g = g;
  epi.level = level;
  return ntt_launch_moddown(c, w.y, (size_t)level * N, range_map(0, level, 0), epi, s, 2, 2);
}

int ks_apply(Ctx* c, const WS& w, const uint64_t* c1, int level, const uint64_t* key, uint32_t g,
             const uint64_t* add0, const uint64_t* add1, uint64_t* out0, uint64_t* out1, hipStream_t s) {
  const size_t N = c->n;
  const int K = c->K, L = c->L;
  const size_t E = (size_t)(level + K);
  const size_t kps = (size_t)(L + K) * N;  // key poly stride
  const int dn = c->dnum(level);
  if (ntt_ip_supported(c, dn)) {
    // tile-wise inner product (the fused kernel with the digits already in NTT
    // form), which also runs ModDown's inverse pass 2 on the special limbs
    NttIp ip{};
    ip.ext = w.ext;
    ip.ext_ds = E * N;
    ip.c1 = c1;
    ip.key = key;
    ip.key_ds = 2 * kps;
    ip.key_ps = kps;
    ip.u = w.u;
    ip.u_ps = E * N;
    ip.alpha = c->alpha;
    ip.dnum = dn;
    ip.level = level;
    ip.g = g;
    ip.p_inv2 = dn >= 2;
    ip.ext_ntt = 1;
    int rc;
    if ((rc = ntt_launch_modup_ip(c, w.ext, c->modup_ntt[level], ext_map(c, level), ip, s))) return rc;
    return ks_moddown(c, w, level, g, add0, add1, out0, out1, s, ip.p_inv2 != 0);
  }
  {
    ProfScope ps(c, "ks_inner_product", s, 8.0 * N * E * (3.0 * dn + 2), 2.0 * dn * E * N);
    k_ip<<<dim3(N / 256, E), 256, 0, s>>>(w.ext, E * N, c1, c->alpha, dn, key, 2 * kps, kps, level, L, g,
                                          c->log_n, c->d_mod, w.u, E * N);
  }
  HE_HIP(hipGetLastError());
  return ks_moddown(c, w, level, g, add0, add1, out0, out1, s);
}

// The key switches of a hoisted set whose extended digits are in w.ext: up
// to SET_MAX rotations per round of one inner-product launch and one batched
// ModDown (inverse transform of the special limbs, conversion fused with the
// forward column pass, forward row pass writing c0 through phi_g plus
// (u - y) P^{-1} to each rotation's outputs).  keys[i], g[i], outs[2 i],
// outs[2 i + 1] per rotation; the keys must stay resident for the rounds.
static int ks_set(Ctx* c, Lane* lane, const WS& w, const uint64_t* c0, const uint64_t* c1, int level,
                  const std::vector<const uint64_t*>& keys, const std::vector<uint32_t>& gs,
                  const std::vector<uint64_t*>& outs, hipStream_t s) {
  const size_t N = c->n;
  const int K = c->K, L = c->L, dn = c->dnum(level);
  const size_t E = (size_t)(level + K), Etop = (size_t)(L + K);
  const size_t kps = (size_t)(L + K) * N;
  if (!lane->set_ws) {
    void* v = nullptr;
    if (hipMalloc(&v, (size_t)SET_MAX * 2 * (Etop + L) * N * 8) != hipSuccess)
      return set_error(HE_ENOMEM, "hoisted-set workspace allocation failed");
    lane->set_ws = (uint64_t*)v;
    if (hipMalloc(&v, sizeof(SetTab)) != hipSuccess) return set_error(HE_ENOMEM, "hoisted-set table allocation failed");
    lane->set_tab = (SetTab*)v;
  }
  uint64_t* U = lane->set_ws;                               // [SET_MAX][2][E][N]
  uint64_t* Y = lane->set_ws + (size_t)SET_MAX * 2 * Etop * N;  // [SET_MAX][2][level][N]
  int rc;
  for (size_t r0 = 0; r0 < keys.size(); r0 += SET_MAX) {
    const int nc = (int)std::min<size_t>(SET_MAX, keys.size() - r0);
    SetTab t{};
    for (int i = 0; i < nc; i++) {
      t.key[i] = keys[r0 + i];
      t.g[i] = gs[r0 + i];
      // g^-1 mod 2N: the odd residues mod 2N have exponent N/2, so g^-1 = g^(N/2 - 1)
      uint64_t inv = 1, b = gs[r0 + i], e = N / 2 - 1;
      const uint64_t m2 = 2 * N;
      for (; e; e >>= 1, b = b * b % m2)
        if (e & 1) inv = inv * b % m2;
      if (inv * gs[r0 + i] % m2 != 1) return set_error(HE_EINVAL, "Galois element without an inverse");
      t.ginv[i] = (uint32_t)inv;
      t.out[2 * i] = outs[2 * (r0 + i)];
      t.out[2 * i + 1] = outs[2 * (r0 + i) + 1];
    }
    k_set_tab<<<1, 64, 0, s>>>(t, lane->set_tab);
    HE_HIP(hipGetLastError());
    {
      ProfScope ps(c, "ks_inner_product_set", s, 8.0 * N * E * nc * (3.0 * dn + 2), 2.0 * dn * E * N * nc);
      const dim3 grid(N / 256, E);
      switch (dn) {
#define HE_IPS(D)                                                                                                  \
  case D:                                                                                                          \
    k_ip_set<D><<<grid, 256, 0, s>>>(w.ext, c1, level, K, c->alpha, t, nc, 2 * kps, kps, L, c->log_n, c->d_mod,   \
                                     U);                                                                           \
    break;
        HE_IPS(1) HE_IPS(2) HE_IPS(3) HE_IPS(4) HE_IPS(5) HE_IPS(6) HE_IPS(7) HE_IPS(8)
#undef HE_IPS
        default:
          return set_error(HE_EINVAL, "too many key-switching digits");
      }
      HE_HIP(hipGetLastError());
    }
    const int z = 2 * nc;
    if ((rc = ntt_launch_conv_in(c, U, E * N, U, E * N, z, range_map(level, K, L), c->d_fin[level], 3, s))) return rc;
    if ((rc = conv_fwd1_launch(c, c->moddown[level], U, E * N, Y, (size_t)level * N, z, 1, c->conv_target[1],
                               "conv_fwd1_moddown", s)))
      return rc;
    NttEpi epi{};
    epi.u = U;
    epi.u_bs = E * N;
    epi.pinv = c->d_pinv[level];
    epi.level = level;
    epi.g = 1;
    epi.add_base = c0;
    epi.tab = lane->set_tab;  // batched mode, the outputs and Galois elements from the table
    if ((rc = ntt_launch_moddown(c, Y, (size_t)level * N, range_map(0, level, 0), epi, s, z, 2))) return rc;
  }
  return HE_OK;
}

int ks_single(Ctx* c, const WS& w, const uint64_t* c1, int level, const uint64_t* key, uint32_t g,
              const uint64_t* add0, const uint64_t* add1, uint64_t* out0, uint64_t* out1, hipStream_t s) {
  const size_t N = c->n;
  const int K = c->K, L = c->L;
  const size_t E = (size_t)(level + K);
  const size_t kps = (size_t)(L + K) * N;
  int rc;
  if (!ntt_ip_supported(c, c->dnum(level))) {
    if ((rc = ks_modup(c, w, c1, level, s))) return rc;
    return ks_apply(c, w, c1, level, key, g, add0, add1, out0, out1, s);
  }
  if ((rc = ks_modup_convert(c, w, c1, level, s))) return rc;
  NttIp ip{};
  ip.ext_p1 = 1;
  ip.ext = w.ext;
  ip.ext_ds = E * N;
  ip.c1 = c1;
  ip.key = key;
  ip.key_ds = 2 * kps;
  ip.key_ps = kps;
  ip.u = w.u;
  ip.u_ps = E * N;
  ip.alpha = c->alpha;
  ip.dnum = c->dnum(level);
  ip.level = level;
  ip.g = g;
  ip.p_inv2 = ip.dnum >= 2;
  if ((rc = ntt_launch_modup_ip(c, w.ext, c->modup_ntt[level], ext_map(c, level), ip, s))) return rc;
  return ks_moddown(c, w, level, g, add0, add1, out0, out1, s, ip.p_inv2 != 0);
}




}  // namespace he

using namespace he;

extern "C" {



int he_rotate_hoisted(he_ctx* h, const he_ct* in, const int32_t* r, int n, he_ct* outs, he_stream st) {
  if (!h || !r || !outs || n < 0) return set_error(HE_EINVAL, "null argument");
  Ctx* c = &h->c;
  int rc;
  if ((rc = check_ct(c, in, "in"))) return rc;
  const int l = in->level;
  const size_t N = c->n;
  int nks = 0;  // rotations that need a key switch
  for (int t = 0; t < n; t++) {
    if ((rc = check_out(c, &outs[t], l))) return rc;
    if (outs[t].data == in->data) return set_error(HE_EINVAL, "output aliases the input");
    for (int u = 0; u < t; u++)  // outputs may be written from different streams
      if (outs[u].data == outs[t].data) return set_error(HE_EINVAL, "two outputs share a buffer");
    if (norm_key_id(c, r[t]) != 0) {
      nks++;
      if (!key_known(c, r[t])) return set_error(HE_ENOKEY, "rotation key " + std::to_string(r[t]) + " not resident");
    }
  }
  hipStream_t s = (hipStream_t)st;
  Lane* lane = lane_for(c, s);
  if (!lane) return HE_ENOMEM;
  WS w = ws_layout(c, lane->ws);
  const uint64_t* c0 = in->data;
  const uint64_t* c1 = in->data + (size_t)in->cap * N;
  // one key switch: the inner product is fused into ModUp's last NTT pass;
  // several: one ModUp shared by all of them (hoisting)
  if (nks > 1 && (rc = ks_modup(c, w, c1, l, s))) return rc;
  // several key switches with resident keys: batched, SET_MAX rotations per
  // inner-product launch and per ModDown launch chain, on the caller's stream
  bool batched = nks >= HOIST_SET_MIN;
  for (int t = 0; t < n && batched; t++)
    if (norm_key_id(c, r[t]) != 0 && !key_resident_only(c, r[t])) batched = false;
  if (batched) {
    std::vector<const uint64_t*> keys;
    std::vector<uint32_t> gs;
    std::vector<uint64_t*> os;
    for (int t = 0; t < n; t++) {
      he_ct& o = outs[t];
      uint64_t* o0 = o.data;
      uint64_t* o1 = o.data + (size_t)o.cap * N;
      if (norm_key_id(c, r[t]) == 0) {
        if (hipMemcpyAsync(o0, c0, (size_t)l * N * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(o1, c1, (size_t)l * N * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
          return set_error(HE_EHIP, "copy of an identity rotation failed");
      } else {
        const uint64_t* key = key_acquire(c, r[t], s);
        if (!key) return HE_ENOMEM;
        keys.push_back(key);
        gs.push_back(galois_elt(c, r[t]));
        os.push_back(o0);
        os.push_back(o1);
      }
      o.level = l;
      o.scale = in->scale;
    }
    // rounds of SET_MAX key switches alternate over the caller's stream and
    // helper streams (each with its own lane), which start after the ModUp
    const int rounds = (int)((keys.size() + SET_MAX - 1) / SET_MAX);
    const int K = std::max(1, std::min(std::min(c->streams_for_ring(), 8), rounds));
    hipStream_t hs[8] = {s};
    Lane* lk[8] = {lane};
    if (K > 1) {
      if ((rc = aux_streams_for(c, s, K - 1, hs + 1))) return rc;
      for (int k = 1; k < K; k++)
        if (!(lk[k] = lane_for(c, hs[k]))) return HE_ENOMEM;
      if ((rc = stream_fork(s, hs + 1, K - 1))) return rc;
    }
    for (int i = 0; i < rounds && rc == HE_OK; i++) {
      const size_t a = (size_t)i * SET_MAX, b = std::min(keys.size(), a + SET_MAX);
      std::vector<const uint64_t*> kr(keys.begin() + a, keys.begin() + b);
      std::vector<uint32_t> gr(gs.begin() + a, gs.begin() + b);
      std::vector<uint64_t*> orr(os.begin() + 2 * a, os.begin() + 2 * b);
      rc = ks_set(c, lk[i % K], w, c0, c1, l, kr, gr, orr, hs[i % K]);
    }
    if (K > 1) {
      const int jr = stream_join(s, hs + 1, K - 1);  // also on an error path: the helpers read the workspace
      if (rc == HE_OK) rc = jr;
    }
    return rc;
  }
  // several: key switch j (inner product + ModDown) on the caller's stream or
  // on helper stream j mod K of it, each helper with its own lane's
  // workspace and the caller's extended digits; the helpers start after the
  // ModUp and the caller's stream waits for them before returning
  const int K = nks > 1 ? std::max(1, std::min(std::min(c->streams_for_ring(), 8), nks)) : 1;
  hipStream_t hs[8] = {s};
  WS wk[8] = {w};
  if (K > 1) {
    if ((rc = aux_streams_for(c, s, K - 1, hs + 1))) return rc;
    for (int k = 1; k < K; k++) {
      Lane* lk = lane_for(c, hs[k]);
      if (!lk) return HE_ENOMEM;
      wk[k] = ws_layout(c, lk->ws);
      wk[k].ext = w.ext;
    }
    if ((rc = stream_fork(s, hs + 1, K - 1))) return rc;
  }
  int j = 0;
  for (int t = 0; t < n && rc == HE_OK; t++) {
    he_ct& o = outs[t];
    uint64_t* o0 = o.data;
    uint64_t* o1 = o.data + (size_t)o.cap * N;
    if (norm_key_id(c, r[t]) == 0) {
      if (hipMemcpyAsync(o0, c0, (size_t)l * N * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
          hipMemcpyAsync(o1, c1, (size_t)l * N * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
        rc = set_error(HE_EHIP, "copy of an identity rotation failed");
    } else {
      const int k = j++ % K;
      const uint64_t* key = key_acquire(c, r[t], hs[k]);
      if (!key) {
        rc = HE_ENOMEM;
        break;
      }
      rc = nks == 1 ? ks_single(c, wk[k], c1, l, key, galois_elt(c, r[t]), c0, nullptr, o0, o1, hs[k])
                    : ks_apply(c, wk[k], c1, l, key, galois_elt(c, r[t]), c0, nullptr, o0, o1, hs[k]);
      if (rc == HE_OK) key_note_use(c, r[t], hs[k]);
    }
    o.level = l;
    o.scale = in->scale;
  }
  if (K > 1) {
    const int jr = stream_join(s, hs + 1, K - 1);  // also on an error path: the helpers read the workspace
    if (rc == HE_OK) rc = jr;
  }
  return rc;
}

int he_rotate(he_ctx* h, const he_ct* in, int32_t r, he_ct* out, he_stream st) {
  return he_rotate_hoisted(h, in, &r, 1, out, st);
}

}  // extern "C"

// ---------------------------------------------------------------- rotation without allocation
// he_rotate_noalloc runs the same key switch as he_rotate (ks_single), with
// its workspace in this static device array instead of a lane's allocation.
// Each GPU the library runs on holds its own copy until the process ends; in
// host code `scratch` only names the symbol, so its device address is looked
// up once per device (hipGetSymbolAddress, with that device current) and
// that address is what kernels receive.
namespace he {
constexpr size_t NOALLOC_SCRATCH_WORDS = HE_NOALLOC_SCRATCH_BYTES / 8;
static __device__ __align__(256) uint64_t scratch[NOALLOC_SCRATCH_WORDS];
constexpr int NOALLOC_MAX_DEVICES = 64;
static uint64_t* g_scratch[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

// device address of `scratch` on the current device (nullptr with the error set)
static uint64_t* scratch_ptr(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) {
    set_error(HE_EINVAL, "device index out of range for the static workspace");
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
      return nullptr;
    }
    g_scratch[device] = (uint64_t*)p;
  }
  return g_scratch[device];
}
}  // namespace he

extern "C" {

int he_rotate_noalloc(he_ctx* h, const he_ct* in, int32_t r, he_ct* out, he_stream st) {
  if (!h || !out) return set_error(HE_EINVAL, "null argument");
  Ctx* c = &h->c;
  int rc;
  if ((rc = check_ct(c, in, "in")) || (rc = check_out(c, out, in->level))) return rc;
  if (out->data == in->data) return set_error(HE_EINVAL, "output aliases the input");
  if (c->prof_on) return set_error(HE_EINVAL, "profiling is on (it creates events): not available here");
  const int l = in->level;
  const size_t N = c->n;
  hipStream_t s = (hipStream_t)st;
  const uint64_t* c0 = in->data;
  const uint64_t* c1 = in->data + (size_t)in->cap * N;
  uint64_t* o0 = out->data;
  uint64_t* o1 = out->data + (size_t)out->cap * N;
  out->level = l;
  out->scale = in->scale;
  if (norm_key_id(c, r) == 0) {
    if (hipMemcpyAsync(o0, c0, (size_t)l * N * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(o1, c1, (size_t)l * N * 8, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return set_error(HE_EHIP, "copy of an identity rotation failed");
    return HE_OK;
  }
  // the key must already be in device memory and never evicted (uploaded with
  // he_key_upload): loading or tracking a host-backed key allocates
  auto it = c->keys.find(norm_key_id(c, r));
  if (it == c->keys.end() || !it->second.dev || it->second.host)
    return set_error(HE_ENOKEY, "rotation key " + std::to_string(r) + " is not a resident (uploaded) key");
  // workspace of one key switch at level l, packed: coeff [l], ext [dnum][l+K],
  // u [2][l+K], y [2][l] limbs
  const size_t E = (size_t)(l + c->K);
  const size_t need = N * ((size_t)l + (size_t)c->dnum(l) * E + 2 * E + 2 * (size_t)l);
  if (need > NOALLOC_SCRATCH_WORDS)
    return set_error(HE_EINVAL, "key switch needs " + std::to_string(need * 8) + " bytes of workspace, more than the " +
                                    std::to_string(HE_NOALLOC_SCRATCH_BYTES) + "-byte static workspace");
  int cur = 0;
  HE_HIP(hipGetDevice(&cur));
  if (cur != c->device) HE_HIP(hipSetDevice(c->device));
  uint64_t* base = scratch_ptr(c->device);
  if (!base) {
    if (cur != c->device) hipSetDevice(cur);
    return HE_EHIP;
  }
  WS w{};
  w.coeff = base;
  w.ext = w.coeff + (size_t)l * N;
  w.u = w.ext + (size_t)c->dnum(l) * E * N;
  w.y = w.u + 2 * E * N;
  rc = ks_single(c, w, c1, l, it->second.dev, galois_elt(c, r), c0, nullptr, o0, o1, s);
  if (cur != c->device) hipSetDevice(cur);
  return rc;
}

int he_relin(he_ctx* h, const uint64_t* d, int level, double scale, he_ct* out, he_stream st) {
  if (!h || !d) return set_error(HE_EINVAL, "null argument");
  Ctx* c = &h->c;
  int rc;
  if (level < 1 || level > c->L) return set_error(HE_EINVAL, "bad level");
  if ((rc = check_out(c, out, level))) return rc;
  if (!key_known(c, HE_KEY_RELIN)) return set_error(HE_ENOKEY, "relinearization key not resident");
  hipStream_t s = (hipStream_t)st;
  const size_t N = c->n;
  Lane* lane = lane_for(c, s);
  if (!lane) return HE_ENOMEM;
  WS w = ws_layout(c, lane->ws);
  const uint64_t* d0 = d;
  const uint64_t* d1 = d + (size_t)level * N;
  const uint64_t* d2 = d + 2 * (size_t)level * N;
  const uint64_t* key = key_acquire(c, HE_KEY_RELIN, s);
  if (!key) return HE_ENOMEM;
  if ((rc = ks_single(c, w, d2, level, key, 1, d0, d1, out->data, out->data + (size_t)out->cap * N, s))) return rc;
  key_note_use(c, HE_KEY_RELIN, s);
  out->level = level;
  out->scale = scale;
  return HE_OK;
}

}  // extern "C"

namespace he {
// (a0 b0, a0 b1 + a1 b0, a1 b1) into d [3][l][N]
__global__ __launch_bounds__(256) void k_tensor(const uint64_t* __restrict__ a, size_t aps,
                                                const uint64_t* __restrict__ b, size_t bps, uint64_t* __restrict__ d,
                                                int level, int logn, const ModInfo* __restrict__ mods) {
  const size_t n = (size_t)1 << logn;
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  const ModInfo mi = mods[i];
  const uint64_t a0 = a[i * n + j], a1 = a[aps + i * n + j];
  const uint64_t b0 = b[i * n + j], b1 = b[bps + i * n + j];
  const uint64_t m0 = mul_mod(a0, b1, mi), m1 = mul_mod(a1, b0, mi);
  d[i * n + j] = mul_mod(a0, b0, mi);
  d[((size_t)level + i) * n + j] = add_mod(m0, m1, mi.q);
  d[(2 * (size_t)level + i) * n + j] = mul_mod(a1, b1, mi);
}
}  // namespace he

extern "C" int he_mul_relin(he_ctx* h, const he_ct* a, const he_ct* b, he_ct* out, he_stream st) {
  if (!h) return set_error(HE_EINVAL, "null context");
  Ctx* c = &h->c;
  int rc;
  if ((rc = check_ct(c, a, "a")) || (rc = check_ct(c, b, "b"))) return rc;
  if (a->level != b->level) return set_error(HE_ELEVEL, "operands at different levels");
  const int l = a->level;
  if ((rc = check_out(c, out, l))) return rc;
  const size_t N = c->n;
  hipStream_t s = (hipStream_t)st;
  Lane* lane = lane_for(c, s);
  if (!lane) return HE_ENOMEM;
  WS w = ws_layout(c, lane->ws);
  {
    ProfScope ps(c, "tensor", s, 8.0 * N * l * 7, 4.0 * N * l);
    k_tensor<<<dim3(N / 256, l), 256, 0, s>>>(a->data, a->cap * N, b->data, b->cap * N, w.t3, l, c->log_n, c->d_mod);
  }
  HE_HIP(hipGetLastError());
  return he_relin(h, w.t3, l, a->scale * b->scale, out, st);
}
