// Exact ring operations on ciphertexts: add / sub / pt-ct multiply(-accumulate),
// rescale, level drop.  One thread per residue, limb-major coalesced access.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace he {

// out[k][i][j] = a[k][i][j] (+/-) b[k][i][j]   (k = poly, i = limb, j = coefficient)
__global__ __launch_bounds__(256) void k_addsub(const uint64_t* __restrict__ a, size_t aps,
                                                const uint64_t* __restrict__ b, size_t bps, uint64_t* out,
                                                size_t ops, int npoly_b, int logn, const ModInfo* __restrict__ mods,
                                                int sub) {
  const size_t n = (size_t)1 << logn;
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y, k = blockIdx.z;
  const uint64_t q = mods[i].q;
  const uint64_t x = a[k * aps + i * n + j];
  uint64_t r = x;
  if (k < npoly_b) {
    const uint64_t y = b[k * bps + i * n + j];
    r = sub ? sub_mod(x, y, q) : add_mod(x, y, q);
  }
  out[k * ops + i * n + j] = r;
}

// out[k][i][j] (+)= in[k][i][j] * pt[i][j]
__global__ __launch_bounds__(256) void k_mul_plain(const uint64_t* in, size_t ips, const uint64_t* __restrict__ pt,
                                                   uint64_t* out, size_t ops, int logn,
                                                   const ModInfo* __restrict__ mods, int accumulate) {
  const size_t n = (size_t)1 << logn;
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y, k = blockIdx.z;
  const ModInfo mi = mods[i];
  uint64_t r = mul_mod(in[k * ips + i * n + j], pt[i * n + j], mi);
  if (accumulate) r = add_mod(r, out[k * ops + i * n + j], mi.q);
  out[k * ops + i * n + j] = r;
}

// out[k][i][j] (+)= sum_t ct_t[k][i][j] * pt_t[i][j] for up to MAC_LIST_MAX
// terms in one pass (each product reduced, then added)
constexpr int MAC_LIST_MAX = 16;
struct MacList {
  const uint64_t* ct[MAC_LIST_MAX];
  const uint64_t* pt[MAC_LIST_MAX];
  uint64_t ps[MAC_LIST_MAX];  // polynomial stride of ct_t (words)
  int n;
};
// (both polynomials per thread: each plaintext word is read once)
__global__ __launch_bounds__(256) void k_mac_list(MacList ml, uint64_t* out, size_t ops, int logn,
                                                  const ModInfo* __restrict__ mods, int accumulate) {
  const size_t n = (size_t)1 << logn;
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  const ModInfo mi = mods[i];
  const size_t off = i * n + j;
  uint64_t r0 = accumulate ? out[off] : 0, r1 = accumulate ? out[ops + off] : 0;
  for (int t = 0; t < ml.n; t++) {
    const uint64_t p = ml.pt[t][off];
    r0 = add_mod(r0, mul_mod(ml.ct[t][off], p, mi), mi.q);
    r1 = add_mod(r1, mul_mod(ml.ct[t][ml.ps[t] + off], p, mi), mi.q);
  }
  out[off] = r0;
  out[ops + off] = r1;
}

// per-limb scalar constants (Shoup pairs) for constant-polynomial plaintexts
struct Scalars {
  uint64_t w[64];
  uint64_t wp[64];
};

// mode 0: out[k][i][j] = in[k][i][j] * w_i;  mode 1: out[0] = in[0] + w_i, out[1] = in[1]
__global__ __launch_bounds__(256) void k_scalar(const uint64_t* in, size_t ips, uint64_t* out, size_t ops, int logn,
                                                const ModInfo* __restrict__ mods, Scalars sc, int mode) {
  const size_t n = (size_t)1 << logn;
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y, k = blockIdx.z;
  const uint64_t q = mods[i].q;
  const uint64_t x = in[k * ips + i * n + j];
  uint64_t r;
  if (mode == 0) r = mul_shoup(x, sc.w[i], sc.wp[i], q);
  else r = k == 0 ? add_mod(x, sc.w[i], q) : x;
  out[k * ops + i * n + j] = r;
}

// out[k][i][j] = in[k][i][j] * (+-w_i), w_i = psi_i^(N/2): the NTT values of
// sign X^(N/2) are sign w_i on the first half of the positions (bit-reversed
// index with top bit 0, i.e. odd exponent 2 brv(j) + 1 = 1 mod 4) and
// -sign w_i on the second half
__global__ __launch_bounds__(256) void k_mul_i(const uint64_t* in, size_t ips, uint64_t* out, size_t ops, int logn,
                                               const ModInfo* __restrict__ mods, Scalars sc, int sign) {
  const size_t n = (size_t)1 << logn;
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y, k = blockIdx.z;
  const uint64_t q = mods[i].q;
  const uint64_t r = mul_shoup(in[k * ips + i * n + j], sc.w[i], sc.wp[i], q);
  const bool neg = (j >= n / 2) != (sign < 0);
  out[k * ops + i * n + j] = neg && r ? q - r : r;
}

// ModRaise lift: limb 0 of each polynomial holds coefficients a in [0, q_0);
// limb i >= 1 gets a mod q_i, or (a - q_0) mod q_i when a > (q_0 - 1)/2
__global__ __launch_bounds__(256) void k_lift(uint64_t* data, size_t ps, int logn, const ModInfo* __restrict__ mods) {
  const size_t n = (size_t)1 << logn;
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y + 1, k = blockIdx.z;
  const ModInfo mi = mods[i];
  const uint64_t q0 = mods[0].q;
  const uint64_t a = data[k * ps + j];
  uint64_t r = reduce_word(a, mi);
  if (a > (q0 >> 1)) r = sub_mod(r, reduce_word(q0, mi), mi.q);
  data[k * ps + i * n + j] = r;
}

// out[k][i][j] = sum_t ct_t[k][i][j] * (v_t mod q_i) for up to CONST_LIST_MAX
// terms (v_t signed integers: the constants llround(c_t * scale_t)), one pass
struct ConstList {
  const uint64_t* ct[CONST_LIST_MAX];
  uint64_t ps[CONST_LIST_MAX];  // polynomial stride of ct_t (words)
  int64_t v[CONST_LIST_MAX];
  int n;
};
__global__ __launch_bounds__(256) void k_mac_const(ConstList cl, uint64_t* out, size_t ops, int logn,
                                                   const ModInfo* __restrict__ mods) {
  const size_t n = (size_t)1 << logn;
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y, k = blockIdx.z;
  const ModInfo mi = mods[i];
  const size_t off = i * n + j;
  uint64_t r = 0;
  for (int t = 0; t < cl.n; t++) {
    const int64_t v = cl.v[t];
    const uint64_t a = v >= 0 ? (uint64_t)v : (uint64_t)(-(v + 1)) + 1;  // |v|
    uint64_t m = reduce_word(a, mi);
    if (v < 0 && m) m = mi.q - m;
    r = add_mod(r, mul_mod(cl.ct[t][k * cl.ps[t] + off], m, mi), mi.q);
  }
  out[k * ops + off] = r;
}

int const_value(double v, double scale, int64_t* out) {
  const double x = v * scale;
  if (!(std::fabs(x) < 9.0e18)) return set_error(HE_EINVAL, "constant times scale does not fit 64 bits");
  *out = (int64_t)llround(x);
  return HE_OK;
}

int mac_const_launch(Ctx* c, const he_ct* cts, const int64_t* vals, int n, he_ct* out, hipStream_t s) {
  if (n < 1) return set_error(HE_EINVAL, "empty constant product sum");
  const int l = cts[0].level;
  const size_t N = c->n;
  for (int t = 0; t < n; t++)
    if (cts[t].level != l) return set_error(HE_ELEVEL, "terms at different levels");
  if (out->cap < l) return set_error(HE_EINVAL, "out: capacity too small");
  if (n > CONST_LIST_MAX) return set_error(HE_EINVAL, "too many terms for one constant product sum");
  ProfScope ps(c, "mac_const", s, 8.0 * N * l * 2.0 * (n + 1), 2.0 * N * l * n);
  ConstList cl{};
  cl.n = n;
  for (int t = 0; t < n; t++) {
    cl.ct[t] = cts[t].data;
    cl.ps[t] = (uint64_t)cts[t].cap * N;
    cl.v[t] = vals[t];
  }
  k_mac_const<<<dim3((unsigned)(N / 256), l, 2), 256, 0, s>>>(cl, out->data, out->cap * N, c->log_n, c->d_mod);
  HE_HIP(hipGetLastError());
  out->level = l;
  return HE_OK;
}

// llround(c * scale) reduced into every active limb (ties away from zero)
static int const_residues(const Ctx* c, double v, double scale, int level, Scalars* sc) {
  int64_t r64 = 0;
  int rc;
  if ((rc = const_value(v, scale, &r64))) return rc;
  const long long r = r64;
  for (int i = 0; i < level; i++) {
    const uint64_t q = c->mod[i];
    uint64_t m = r >= 0 ? (uint64_t)r % q : (q - ((uint64_t)(-(r + 1)) + 1) % q) % q;
    sc->w[i] = m;
    sc->wp[i] = (uint64_t)(((unsigned __int128)m << 64) / q);
  }
  return HE_OK;
}

int check_ct(const Ctx* c, const he_ct* x, const char* what) {
  if (!x || !x->data) return set_error(HE_EINVAL, std::string(what) + ": null ciphertext");
  if (x->level < 1 || x->level > c->L || x->cap < x->level)
    return set_error(HE_EINVAL, std::string(what) + ": bad level/capacity");
  return HE_OK;
}

// outputs: only the buffer and its capacity matter (level/scale are written)
int check_out(const Ctx* c, const he_ct* x, int need_level) {
  if (!x || !x->data) return set_error(HE_EINVAL, "out: null ciphertext");
  if (x->cap < need_level || x->cap > c->L) return set_error(HE_EINVAL, "out: capacity too small");
  return HE_OK;
}

static dim3 grid_for(const Ctx* c, int limbs, int polys) { return dim3(c->n / 256, limbs, polys); }

}  // namespace he

using namespace he;

static int addsub(he_ctx* h, const he_ct* a, const he_ct* b, he_ct* out, he_stream s, int sub) {
  if (!h) return set_error(HE_EINVAL, "null context");
  Ctx* c = &h->c;
  int rc;
  if ((rc = check_ct(c, a, "a")) || (rc = check_ct(c, b, "b")) || (rc = check_out(c, out, a->level))) return rc;
  if (a->level != b->level) return set_error(HE_ELEVEL, "operands at different levels");
  if (a->scale != b->scale) return set_error(HE_ESCALE, "operands at different scales");
  const size_t N = c->n;
  ProfScope ps(c, "add_sub", (hipStream_t)s, 48.0 * N * a->level, 0);
  k_addsub<<<grid_for(c, a->level, 2), 256, 0, (hipStream_t)s>>>(a->data, a->cap * N, b->data, b->cap * N,
                                                                   out->data, out->cap * N, 2, c->log_n, c->d_mod,
                                                                   sub);
  HE_HIP(hipGetLastError());
  out->level = a->level;
  out->scale = a->scale;
  return HE_OK;
}

extern "C" {

int he_mac_plain(he_ctx* h, const he_ct* cts, const he_pt* pts, int n, he_ct* out, int accumulate, he_stream st) {
  if (!h || !cts || !pts || !out) return set_error(HE_EINVAL, "null argument");
  if (n < 1) return set_error(HE_EINVAL, "empty product sum");
  Ctx* c = &h->c;
  int rc;
  const int l = cts[0].level;
  double sc = 0.0;
  for (int t = 0; t < n; t++) {
    if ((rc = check_ct(c, &cts[t], "cts"))) return rc;
    if (!pts[t].data) return set_error(HE_EINVAL, "null plaintext");
    if (cts[t].level != l) return set_error(HE_ELEVEL, "terms at different levels");
    if (pts[t].level < l) return set_error(HE_ELEVEL, "plaintext has fewer limbs than the ciphertext");
    const double st_ = cts[t].scale * pts[t].scale;
    if (t > 0 && st_ != sc) return set_error(HE_ESCALE, "terms at different scales");
    sc = st_;
    if (cts[t].data == out->data) return set_error(HE_EINVAL, "output aliases a term");
  }
  if ((rc = check_out(c, out, l))) return rc;
  if (accumulate) {
    if (out->level != l) return set_error(HE_ELEVEL, "accumulator at a different level");
    if (out->scale != sc) return set_error(HE_ESCALE, "accumulator scale differs");
  }
  const size_t N = c->n;
  ProfScope ps(c, "mac_plain", (hipStream_t)st, 8.0 * N * l * (3.0 * n + (accumulate ? 4 : 2)), 2.0 * N * l * n);
  for (int t0 = 0; t0 < n; t0 += MAC_LIST_MAX) {
    MacList ml{};
    ml.n = std::min(MAC_LIST_MAX, n - t0);
    for (int t = 0; t < ml.n; t++) {
      ml.ct[t] = cts[t0 + t].data;
      ml.pt[t] = pts[t0 + t].data;
      ml.ps[t] = (uint64_t)cts[t0 + t].cap * N;
    }
    k_mac_list<<<grid_for(c, l, 1), 256, 0, (hipStream_t)st>>>(ml, out->data, out->cap * N, c->log_n, c->d_mod,
                                                               (accumulate || t0 > 0) ? 1 : 0);
    HE_HIP(hipGetLastError());
  }
  out->level = l;
  out->scale = sc;
  return HE_OK;
}

int he_mul_i(he_ctx* h, const he_ct* in, int sign, he_ct* out, he_stream st) {
  if (!h) return set_error(HE_EINVAL, "null context");
  Ctx* c = &h->c;
  int rc;
  if ((rc = check_ct(c, in, "in")) || (rc = check_out(c, out, in->level))) return rc;
  if (sign != 1 && sign != -1) return set_error(HE_EINVAL, "sign must be +1 or -1");
  if (out->data == in->data && out->cap != in->cap) return set_error(HE_EINVAL, "in-place product needs equal capacity");
  Scalars sc;
  for (int i = 0; i < in->level; i++) {
    sc.w[i] = omega4(c, i);
    sc.wp[i] = (uint64_t)(((unsigned __int128)sc.w[i] << 64) / c->mod[i]);
  }
  const size_t N = c->n;
  ProfScope ps(c, "mul_i", (hipStream_t)st, 32.0 * N * in->level, 2.0 * N * in->level);
  k_mul_i<<<grid_for(c, in->level, 2), 256, 0, (hipStream_t)st>>>(in->data, in->cap * N, out->data, out->cap * N,
                                                                   c->log_n, c->d_mod, sc, sign);
  HE_HIP(hipGetLastError());
  out->level = in->level;
  out->scale = in->scale;
  return HE_OK;
}

int he_mod_raise(he_ctx* h, const he_ct* in, int level, he_ct* out, he_stream st) {
  if (!h) return set_error(HE_EINVAL, "null context");
  Ctx* c = &h->c;
  int rc;
  if ((rc = check_ct(c, in, "in"))) return rc;
  if (level < 1 || level > c->L) return set_error(HE_ELEVEL, "raise level out of range");
  if ((rc = check_out(c, out, level))) return rc;
  if (out->data == in->data) return set_error(HE_EINVAL, "ModRaise output aliases the input");
  hipStream_t s = (hipStream_t)st;
  const size_t N = c->n;
  ProfScope ps(c, "mod_raise", s, 8.0 * N * 2 * (1 + level), 0);
  // limb 0 of both polynomials to coefficient form in out's limb 0
  if ((rc = ntt_launch_strided(c, in->data, in->cap * N, out->data, out->cap * N, 2, range_map(0, 1, 0), true, s)))
    return rc;
  if (level > 1) {
    k_lift<<<dim3((unsigned)(N / 256), level - 1, 2), 256, 0, s>>>(out->data, out->cap * N, c->log_n, c->d_mod);
    HE_HIP(hipGetLastError());
  }
  if ((rc = ntt_launch(c, out->data, out->cap * N, 2, range_map(0, level, 0), false, s))) return rc;
  out->level = level;
  out->scale = in->scale;
  return HE_OK;
}

int he_add(he_ctx* h, const he_ct* a, const he_ct* b, he_ct* out, he_stream s) { return addsub(h, a, b, out, s, 0); }
int he_sub(he_ctx* h, const he_ct* a, const he_ct* b, he_ct* out, he_stream s) { return addsub(h, a, b, out, s, 1); }

int he_add_plain(he_ctx* h, const he_ct* a, const he_pt* pt, he_ct* out, he_stream s) {
  if (!h || !pt || !pt->data) return set_error(HE_EINVAL, "null argument");
  Ctx* c = &h->c;
  int rc;
  if ((rc = check_ct(c, a, "a")) || (rc = check_out(c, out, a->level))) return rc;
  if (pt->level < a->level) return set_error(HE_ELEVEL, "plaintext has fewer limbs than the ciphertext");
  if (pt->scale != a->scale) return set_error(HE_ESCALE, "plaintext scale differs");
  const size_t N = c->n;
  // poly 0 gets + pt; poly 1 is copied (npoly_b = 1)
  k_addsub<<<grid_for(c, a->level, 2), 256, 0, (hipStream_t)s>>>(a->data, a->cap * N, pt->data, 0, out->data,
                                                                   out->cap * N, 1, c->log_n, c->d_mod, 0);
  HE_HIP(hipGetLastError());
  out->level = a->level;
  out->scale = a->scale;
  return HE_OK;
}

int he_mul_plain(he_ctx* h, const he_ct* in, const he_pt* pt, he_ct* out, int accumulate, he_stream s) {
  if (!h || !pt || !pt->data) return set_error(HE_EINVAL, "null argument");
  Ctx* c = &h->c;
  int rc;
  if ((rc = check_ct(c, in, "in")) || (rc = check_out(c, out, in->level))) return rc;
  if (pt->level < in->level) return set_error(HE_ELEVEL, "plaintext has fewer limbs than the ciphertext");
  const double sc = in->scale * pt->scale;
  if (accumulate) {
    if (out->data == in->data) return set_error(HE_EINVAL, "accumulate output aliases the input");
    if (out->level != in->level) return set_error(HE_ELEVEL, "accumulator at a different level");
    if (out->scale != sc) return set_error(HE_ESCALE, "accumulator scale differs");
  }
  const size_t N = c->n;
  ProfScope ps(c, "mul_plain", (hipStream_t)s, 8.0 * N * in->level * (accumulate ? 7 : 5), 2.0 * N * in->level);
  k_mul_plain<<<grid_for(c, in->level, 2), 256, 0, (hipStream_t)s>>>(in->data, in->cap * N, pt->data, out->data,
                                                                      out->cap * N, c->log_n, c->d_mod,
                                                                      accumulate ? 1 : 0);
  HE_HIP(hipGetLastError());
  out->level = in->level;
  out->scale = sc;
  return HE_OK;
}

int he_rescale(he_ctx* h, const he_ct* in, he_ct* out, he_stream st) {
  if (!h) return set_error(HE_EINVAL, "null context");
  Ctx* c = &h->c;
  int rc;
  if ((rc = check_ct(c, in, "in"))) return rc;
  const int l = in->level, t = l - 1;
  if (l < 2) return set_error(HE_ELEVEL, "cannot rescale at level 1");
  if ((rc = check_out(c, out, t))) return rc;
  if (out->data == in->data && out->cap != in->cap) return set_error(HE_EINVAL, "in-place rescale needs equal capacity");
  hipStream_t s = (hipStream_t)st;
  const size_t N = c->n;
  Lane* lane = lane_for(c, s);
  if (!lane) return HE_ENOMEM;
  WS w = ws_layout(c, lane->ws);
  // T = w.y: [2][N] top limbs in coefficient form; w.rs: [2][t][N] converted
  if ((rc = rescale_launch(c, in->data, in->cap * N, out->data, out->cap * N, 2, l, w.y, w.rs, s))) return rc;
  out->level = t;
  out->scale = in->scale / (double)c->mod[t];
  return HE_OK;
}

int he_mul_const(he_ctx* h, const he_ct* in, double v, double scale, he_ct* out, he_stream st) {
  if (!h) return set_error(HE_EINVAL, "null context");
  Ctx* c = &h->c;
  int rc;
  if ((rc = check_ct(c, in, "in")) || (rc = check_out(c, out, in->level))) return rc;
  Scalars sc;
  if ((rc = const_residues(c, v, scale, in->level, &sc))) return rc;
  const size_t N = c->n;
  ProfScope ps(c, "mul_const", (hipStream_t)st, 32.0 * N * in->level, 2.0 * N * in->level);
  k_scalar<<<grid_for(c, in->level, 2), 256, 0, (hipStream_t)st>>>(in->data, in->cap * N, out->data, out->cap * N,
                                                                     c->log_n, c->d_mod, sc, 0);
  HE_HIP(hipGetLastError());
  out->level = in->level;
  out->scale = in->scale * scale;
  return HE_OK;
}

int he_add_const(he_ctx* h, const he_ct* in, double v, he_ct* out, he_stream st) {
  if (!h) return set_error(HE_EINVAL, "null context");
  Ctx* c = &h->c;
  int rc;
  if ((rc = check_ct(c, in, "in")) || (rc = check_out(c, out, in->level))) return rc;
  Scalars sc;
  if ((rc = const_residues(c, v, in->scale, in->level, &sc))) return rc;
  const size_t N = c->n;
  k_scalar<<<grid_for(c, in->level, 2), 256, 0, (hipStream_t)st>>>(in->data, in->cap * N, out->data, out->cap * N,
                                                                     c->log_n, c->d_mod, sc, 1);
  HE_HIP(hipGetLastError());
  out->level = in->level;
  out->scale = in->scale;
  return HE_OK;
}

int he_drop_level(he_ctx* h, const he_ct* in, int level, he_ct* out, he_stream st) {
  if (!h) return set_error(HE_EINVAL, "null context");
  Ctx* c = &h->c;
  int rc;
  if ((rc = check_ct(c, in, "in"))) return rc;
  if (level < 1 || level > in->level) return set_error(HE_ELEVEL, "target level out of range");
  if ((rc = check_out(c, out, level))) return rc;
  const size_t N = c->n;
  if (out->data != in->data || out->cap != in->cap) {
    if (out->data == in->data) return set_error(HE_EINVAL, "in-place drop needs equal capacity");
    for (int k = 0; k < 2; k++)
      HE_HIP(hipMemcpyAsync(out->data + k * (size_t)out->cap * N, in->data + k * (size_t)in->cap * N,
                            (size_t)level * N * 8, hipMemcpyDeviceToDevice, (hipStream_t)st));
  }
  out->level = level;
  out->scale = in->scale;
  return HE_OK;
}

}  // extern "C"
