// Per-element bodies of the non-NTT kernels (host+device so that a whole key
// switch can be emulated on the CPU with the kernels' own arithmetic).
#pragma once
#include "modarith.h"

namespace he {

constexpr int MAX_BCONV_IN = 8;    // Montgomery accumulator bound: nin * 2^61 * p < p 2^64
constexpr int MAX_BCONV_OUT = 64;
constexpr int MAXJ = 128;          // limb jobs in one batched launch
constexpr int MAX_DIGITS = 8;      // key-switching digits (dnum)

// Which limbs of a [limbs][N] array a kernel touches and their moduli.
struct LimbMap {
  int32_t n;
  uint16_t pos[MAXJ];  // limb position inside the array
  uint8_t mod[MAXJ];   // modulus index (0..L-1 q_i, L.. p_k)
};

// Device-resident description of one fast basis conversion:
// input limbs (position, modulus) -> output limbs, constants at `tab`:
// [nin] w, [nin] w' (Shoup pair of (Qin/q_i)^{-1} mod q_i), then
// [nin][nout] (Qin/q_i mod p) * 2^64 mod p (Montgomery form).
struct BConvDesc {
  int32_t nin, nout;
  int32_t in_pos[MAX_BCONV_IN], in_mod[MAX_BCONV_IN];
  int32_t out_pos[MAX_BCONV_OUT], out_mod[MAX_BCONV_OUT];
  const uint64_t* tab;
};

HE_HD uint32_t bitrev_n(uint32_t x, int logn) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __brev(x) >> (32 - logn);
#else
  uint32_t r = 0;
  for (int i = 0; i < logn; i++) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
#endif
}

// NTT-form Galois automorphism phi_g: out[j] = in[src(j)] with
// src(j) = brv(((g (2 brv(j) + 1)) mod 2N - 1) / 2).
HE_HD uint32_t automorph_src(uint32_t j, uint32_t g, int logn) {
  const uint32_t mask2n = (2u << logn) - 1;
  uint32_t e = (uint32_t)(((uint64_t)g * (2u * bitrev_n(j, logn) + 1u)) & mask2n);
  return bitrev_n((e - 1u) >> 1, logn);
}

// Fast basis conversion of coefficient k (floor type):
//   t_i = [x_i * (Qin/q_i)^{-1}]_{q_i},  y_p = sum_i t_i [Qin/q_i]_p mod p,
// computed for the outputs p in [p0, p1).
HE_HD void bconv_elem(const uint64_t* in, uint64_t* out, size_t n, size_t k, const BConvDesc& d, int p0, int p1,
                      const ModInfo* mods) {
  const int nin = d.nin, nout = d.nout;
  const uint64_t* tab = d.tab;
  uint64_t t[MAX_BCONV_IN];
  for (int i = 0; i < nin; i++) {
    const uint64_t q = mods[d.in_mod[i]].q;
    t[i] = mul_shoup(in[(size_t)d.in_pos[i] * n + k], tab[i], tab[nin + i], q);
  }
  const uint64_t* c = tab + 2 * nin;
  if (p1 > nout) p1 = nout;
  for (int p = p0; p < p1; p++) {
    const ModInfo& mp = mods[d.out_mod[p]];
    U128 acc{0, 0};
    for (int i = 0; i < nin; i++) add_wide(acc, mul_wide(t[i], c[i * nout + p]));
    out[(size_t)d.out_pos[p] * n + k] = mont_redc(acc, mp.q, mp.qinv);
  }
}

// Key inner product for extended limb `pos` (modulus mi), coefficient k:
//   u0 = sum_j phi_g(ext_j)[k] * b_j,  u1 = sum_j phi_g(ext_j)[k] * a_j,
// keys in Montgomery form so one REDC per output gives the plain product.
// The limbs of digit j's own moduli are not copied into ext_j: they are read
// from the NTT-form source polynomial c1 directly.
HE_HD void ip_elem(const uint64_t* ext, size_t ext_stride, const uint64_t* c1, int alpha, int dnum,
                   const uint64_t* key, size_t key_digit_stride, size_t key_poly_stride, int pos, int keylimb,
                   size_t n, size_t k, uint32_t src, const ModInfo& mi, uint64_t* u0, uint64_t* u1,
                   size_t u_poly_stride) {
  U128 a0{0, 0}, a1{0, 0};
  const int own = pos / alpha;  // digit whose own limb this is (if pos < level)
  for (int j = 0; j < dnum; j++) {
    const uint64_t* srcp = (j == own && c1) ? c1 : ext + j * ext_stride;
    const uint64_t e = srcp[(size_t)pos * n + src];
    const uint64_t* kj = key + j * key_digit_stride + (size_t)keylimb * n + k;
    add_wide(a0, mul_wide(e, kj[0]));
    add_wide(a1, mul_wide(e, kj[key_poly_stride]));
  }
  u0[(size_t)pos * n + k] = mont_redc(a0, mi.q, mi.qinv);
  u1[u_poly_stride + (size_t)pos * n + k] = mont_redc(a1, mi.q, mi.qinv);
}

// ModDown epilogue on limb i (q_i), coefficient k:
//   out = add + (u - y) * P^{-1} mod q_i
HE_HD uint64_t moddown_elem(uint64_t u, uint64_t y, uint64_t add, uint64_t pinv, uint64_t pinvp, uint64_t q) {
  return add_mod(add, mul_shoup(sub_mod(u, y, q), pinv, pinvp, q), q);
}

// Rescale epilogue: (c - r) * q_t^{-1} mod q_i
HE_HD uint64_t rescale_elem(uint64_t c, uint64_t r, uint64_t w, uint64_t wp, uint64_t q) {
  return mul_shoup(sub_mod(c, r, q), w, wp, q);
}

// x mod q for any x < 2^64 (x < q^2 holds for every prime >= 2^32 used here;
// smaller moduli fall back to the % operator)
HE_HD uint64_t reduce_word(uint64_t x, const ModInfo& m) {
  if (m.k > 32) return barrett_reduce(U128{x, 0}, m.q, m.mu, m.k);
  return x % m.q;
}

}  // namespace he
