// Per-element bodies of the non-NTT kernels (host+device so that a whole key
// switch can be emulated on the CPU with the kernels' own arithmetic).
#pragma once
#include "modarith.h"

namespace he {

constexpr int MAX_BCONV_IN = 10;   // input limbs of one conversion (alpha and K)
constexpr int MAX_BCONV_OUT = 64;
constexpr int CONV_MAX_GROUP = 16;  // outputs of one conversion workgroup
constexpr int MAXJ = 128;          // limb jobs in one batched launch
constexpr int MAX_DIGITS = 8;      // key-switching digits (dnum)

// Which limbs of a [limbs][N] array a kernel touches and their moduli.
struct LimbMap {
  int32_t n;
  uint16_t pos[MAXJ];  // limb position inside the array
  uint8_t mod[MAXJ];   // modulus index (0..L-1 q_i, L.. p_k)
};

// Device-resident description of one fast basis conversion (floor type)
//   t_i = [x_i (Qin/q_i)^{-1}]_{q_i},  y_p = sum_i t_i [Qin/q_i]_p  mod p
// as the forward column pass of the outputs consumes it.  The inputs arrive
// as t_i already: the inverse transform that produces them multiplies by
// N^{-1} (Qin/q_i)^{-1} instead of N^{-1} (see conv_fin_fill).  The sum runs
// on the vector ALUs over "parts": an input below 2^50 is one part (an exact
// double); a wider one is two, its low 32 bits and the rest, with constants
// [Qin/q_i]_p and [Qin/q_i 2^32]_p.  For an output prime below 2^50 every
// term is one centred FP64 product (mul_f64_c with a centred constant,
// |term| <= 0.625 p) and the sum is re-centred every 8 terms; other outputs
// accumulate exact 128-bit products with constants in Montgomery form and
// end with one REDC.
//   part_pos[v]: input limb of part v; part_kind[v]: 0 whole value, 1 low
//     32 bits, 2 bits 32 and up
//   cst: [nout][nparts][2] words; FP64 output: centred constant and
//     fl(constant / p) as double bits; integer output: constant 2^64 mod p, 0
struct ConvDesc {
  int32_t nin, nparts, nout;
  int32_t nint;  // outputs of 51 bits and more, listed first
  int32_t in_pos[MAX_BCONV_IN], in_mod[MAX_BCONV_IN];
  int32_t part_pos[2 * MAX_BCONV_IN], part_kind[2 * MAX_BCONV_IN];
  int32_t out_pos[MAX_BCONV_OUT], out_mod[MAX_BCONV_OUT];
  const uint64_t* cst;
};

// Value of part `kind` of an input word w (canonical, below 2^61), exact
// and without a branch: with lo, hi the 32-bit halves, a whole value below
// 2^50 is hi 2^32 + lo, the low part lo, the high part hi.  conv_part_ab
// gives the weights (a, b) of hi and lo for a kind.
HE_HD void conv_part_ab(int kind, double& a, double& b) {
  a = kind == 0 ? 4294967296.0 : kind == 2 ? 1.0 : 0.0;
  b = kind == 2 ? 0.0 : 1.0;
}
HE_HD double conv_part(uint64_t w, double a, double b) {
  return fma((double)(uint32_t)(w >> 32), a, (double)(uint32_t)w * b);
}

// Outputs modulo primes of at most 50 bits take the FP64 sum; inputs below
// 2^50 are one part.
HE_HD bool conv_out_f64(int kbits) { return kbits <= 50; }
HE_HD bool conv_in_narrow(int kbits) { return kbits <= 50; }

// FP64 outputs (|x_v| < 2^50, centred constants |c| <= p/2 with
// cq = fl(c/p)): each centred product mul_f64_c(x_v, c, cq, p) is exact and
// below 0.625 p in magnitude (the quotient estimate is off by at most 1/8),
// eight of them stay below 5 p < 2^53, and re-centring after every eighth
// keeps the running sum exact; the sum is an integer-valued double congruent
// to y_p with magnitude below 5.5 p (not canonical: the column pass that
// consumes it re-centres first).
// Integer outputs: x_v (c_v 2^64 mod p), each product below 2^52 2^61,
// accumulated in 128 bits and kept below p 2^64 by one conditional
// subtraction of p 2^64 per term; one REDC then gives the canonical y_p.
HE_HD void conv_mac_int(U128& acc, double x, uint64_t c_mont, uint64_t p) {
  add_wide(acc, mul_wide(f64_to_u52(x), c_mont));
  if (acc.hi >= p) acc.hi -= p;
}
// One output from the parts x[0..nparts) of a coefficient, nparts <= NP
// (the loops unroll over NP so x stays in registers); cst = the output's
// [nparts][2] constants.
template <int NP>
HE_HD double conv_sum_f64(const double* x, int nparts, const uint64_t* cst, double p, double pinv) {
  double acc = 0.0;
#pragma unroll
  for (int v = 0; v < NP; v++) {
    if (v < nparts) {
      acc += mul_f64_c(x[v], bits_to_f64(cst[2 * v]), bits_to_f64(cst[2 * v + 1]), p);
      if ((v & 7) == 7) acc = centre_f64(acc, pinv, p);
    }
  }
  return acc;
}
template <int NP>
HE_HD uint64_t conv_sum_int(const double* x, int nparts, const uint64_t* cst, uint64_t p, uint64_t pinv64) {
  U128 acc{0, 0};
#pragma unroll
  for (int v = 0; v < NP; v++)
    if (v < nparts) conv_mac_int(acc, x[v], cst[2 * v], p);
  return mont_redc(acc, p, pinv64);
}

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

// x mod q for any x < 2^64 (x < q^2 holds for every prime >= 2^32 used here;
// smaller moduli fall back to the % operator)
HE_HD uint64_t reduce_word(uint64_t x, const ModInfo& m) {
  if (m.k > 32) return barrett_reduce(U128{x, 0}, m.q, m.mu, m.k);
  return x % m.q;
}

}  // namespace he
