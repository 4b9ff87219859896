// Hybrid key switching (ModUp -> key inner product -> ModDown), rotations,
// hoisted rotations, relinearization, and the resident key store.
//
// Pinned formula for every key switch (one formula for plain and hoisted
// rotations): digits of c1 are basis-extended once (ModUp), the Galois
// automorphism phi_g is applied to the extended digits as an NTT-form index
// gather fused into the inner-product load, then ModDown.
#include "internal.h"

namespace he {

// ---------------------------------------------------------------- kernels
// Basis conversion on the int8 matrix cores (see BConvDesc).  One wave owns
// 32 coefficients: lane l loads t_i for i = 2 s + l / 32 (the B operand of
// K-step s is exactly its 8 digit bytes), then every 4-output row tile takes
// nsteps MFMAs and an epilogue that turns 8 int32 digit sums per output
// into a residue.  grid: x = 128-coefficient block (4 waves), y = chunk of
// BCONV_TILES_Y row tiles, z = batch: descriptor descs[z % zdiv], input
// in + (z / zdiv) in_bs, output out + z out_bs.
typedef int32_t v16i __attribute__((ext_vector_type(16)));

__global__ __launch_bounds__(256) void k_bconv(const uint64_t* __restrict__ in, size_t in_bs,
                                               uint64_t* __restrict__ out, size_t out_bs,
                                               const BConvDesc* __restrict__ descs, int zdiv,
                                               const ModInfo* __restrict__ mods, int logn) {
  // constants of this block's row tiles, staged once per workgroup
  __shared__ uint64_t s_frag[BCONV_TILES_Y * (MAX_BCONV_IN / 2) * 64];
  __shared__ uint64_t s_ep[BCONV_TILES_Y * 4 * BCONV_EPW];
  __shared__ uint32_t s_pos[BCONV_TILES_Y * 4];
  const size_t n = (size_t)1 << logn;
  const int lane = threadIdx.x & 63;
  const int half = lane >> 5;
  const size_t k = ((size_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 32 + (lane & 31);
  const int z = blockIdx.z;
  const BConvDesc& d = descs[z % zdiv];
  const int g0 = blockIdx.y * BCONV_TILES_Y;
  if (g0 >= d.ngroups) return;  // uniform over the block
  const int g1 = min(g0 + BCONV_TILES_Y, d.ngroups);
  const int nin = d.nin, nsteps = d.nsteps;
  const uint64_t* src = in + (z / zdiv) * in_bs;
  uint64_t* dst = out + z * out_bs;
  uint64_t x[MAX_BCONV_IN / 2];
#pragma unroll
  for (int s = 0; s < MAX_BCONV_IN / 2; s++) {
    const int i = 2 * s + half;
    x[s] = i < nin ? src[(size_t)d.in_pos[i] * n + k] : 0;
  }
  {
    const uint64_t* __restrict__ fr = d.frag + (size_t)g0 * nsteps * 64;
    const int nf = (g1 - g0) * nsteps * 64;
    for (int e = threadIdx.x; e < nf; e += 256) s_frag[e] = fr[e];
    const int p0 = 4 * g0, np = min(4 * g1, d.nout) - p0;
    for (int e = threadIdx.x; e < BCONV_EPW * np; e += 256) s_ep[e] = d.ep[BCONV_EPW * p0 + e];
    for (int e = threadIdx.x; e < np; e += 256) s_pos[e] = (uint32_t)d.out_pos[p0 + e];
  }
  long bf[MAX_BCONV_IN / 2];
#pragma unroll
  for (int s = 0; s < MAX_BCONV_IN / 2; s++) {
    const int i = 2 * s + half;
    uint64_t t = 0;
    if (i < nin) t = mul_shoup(x[s], d.tab[i], d.tab[nin + i], mods[d.in_mod[i]].q);
    bf[s] = (long)sdigits(t);
  }
  __syncthreads();
  const int np = min(4 * g1, d.nout) - 4 * g0;
  for (int g = 0; g < g1 - g0; g++) {
    const uint64_t* fr = s_frag + g * nsteps * 64 + lane;
    v16i acc = {};
#pragma unroll
    for (int s = 0; s < MAX_BCONV_IN / 2; s++)
      if (s < nsteps) acc = __builtin_amdgcn_mfma_i32_32x32x16_i8((long)fr[s * 64], bf[s], acc, 0, 0, 0);
#pragma unroll
    for (int mm = 0; mm < 2; mm++) {
      const int p = 4 * g + 2 * half + mm;
      if (p < np) {
        int32_t a8[8];
#pragma unroll
        for (int b = 0; b < 8; b++) a8[b] = acc[8 * mm + b];
        dst[(size_t)s_pos[p] * n + k] = bconv_out(a8, s_ep + BCONV_EPW * p);
      }
    }
  }
}

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
// Digits of c1 (NTT form, `level` limbs) basis-extended to Q_l u P: the
// digits' own limbs stay in c1; every other limb of digit j is written to
// w.ext + j (level+K) N in NTT form.
// iNTT of c1's digits and their basis conversion (coefficient form) into w.ext
static int ks_modup_convert(Ctx* c, const WS& w, const uint64_t* c1, int level, hipStream_t s) {
  const size_t N = c->n;
  const size_t E = (size_t)(level + c->K);
  int rc;
  if ((rc = ntt_launch_from(c, c1, w.coeff, 0, 1, range_map(0, level, 0), true, s))) return rc;
  const BConvSet& set = c->modup[level];
  {
    const double mm = (double)N * level * (1 + set.max_out);  // t_i products + MACs (upper bound)
    ProfScope ps(c, "bconv_modup", s, 8.0 * N * (level + (double)set.count * set.max_out), mm,
                 bconv_ideal_s((double)N, set.count, c->alpha, set.max_out));
    dim3 grid(N / 128, bconv_tiles_y(set), set.count);
    k_bconv<<<grid, 256, 0, s>>>(w.coeff, 0, w.ext, E * N, set.d, set.count, c->d_mod, c->log_n);
  }
  HE_HIP(hipGetLastError());
  return HE_OK;
}

int ks_modup(Ctx* c, const WS& w, const uint64_t* c1, int level, hipStream_t s) {
  int rc;
  if ((rc = ks_modup_convert(c, w, c1, level, s))) return rc;
  return ntt_launch(c, w.ext, 0, 1, c->modup_ntt[level], false, s);
}

// ModDown of w.u (both polynomials) and the final additions
// (p_inv2: the special-prime limbs of w.u are already after inverse pass 2)
static int ks_moddown(Ctx* c, const WS& w, int level, uint32_t g, const uint64_t* add0, const uint64_t* add1,
                      uint64_t* out0, uint64_t* out1, hipStream_t s, bool p_inv2 = false) {
  const size_t N = c->n;
  const int K = c->K, L = c->L;
  const size_t E = (size_t)(level + K);
  int rc;
  // ModDown of u0 and u1: P limbs to coefficient form, convert to Q_l, back to NTT form
  if (p_inv2)
    rc = ntt_launch_pass(c, w.u, E * N, w.u, E * N, 2, range_map(level, K, L), true, 1, s);
  else
    rc = ntt_launch(c, w.u, E * N, 2, range_map(level, K, L), true, s);
  if (rc) return rc;
  const BConvSet& set = c->moddown[level];
  {
    ProfScope ps(c, "bconv_moddown", s, 16.0 * N * (K + level), 2.0 * N * K * (1 + level),
                 bconv_ideal_s((double)N, 2, K, level));
    dim3 grid(N / 128, bconv_tiles_y(set), 2);
    k_bconv<<<grid, 256, 0, s>>>(w.u, E * N, w.y, (size_t)level * N, set.d, 1, c->d_mod, c->log_n);
  }
  HE_HIP(hipGetLastError());
  // back to NTT form with the ModDown epilogue fused into the last pass
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
  if ((rc = ntt_launch_moddown(c, w.y, (size_t)level * N, range_map(0, level, 0), epi, s))) return rc;
  HE_HIP(hipGetLastError());
  return HE_OK;
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
