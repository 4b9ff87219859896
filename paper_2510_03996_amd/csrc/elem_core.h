// Per-element bodies of the non-NTT kernels (host+device so that a whole key
// switch can be emulated on the CPU with the kernels' own arithmetic).
#pragma once
#include "modarith.h"

namespace he {

constexpr int MAX_BCONV_IN = 10;   // input limbs of one conversion (alpha and K)
constexpr int MAX_BCONV_OUT = 64;
constexpr int MAXJ = 128;          // limb jobs in one batched launch
constexpr int MAX_DIGITS = 8;      // key-switching digits (dnum)
constexpr int BCONV_EPW = 5;       // epilogue words per basis-conversion output

// Which limbs of a [limbs][N] array a kernel touches and their moduli.
struct LimbMap {
  int32_t n;
  uint16_t pos[MAXJ];  // limb position inside the array
  uint8_t mod[MAXJ];   // modulus index (0..L-1 q_i, L.. p_k)
};

// Device-resident description of one fast basis conversion (floor type):
//   t_i = [x_i (Qin/q_i)^{-1}]_{q_i},  y_p = sum_i t_i [Qin/q_i]_p  mod p.
// The sum is an integer matrix product evaluated on the int8 matrix cores:
// every t_i is split into 8 signed base-256 digits d_{i,a}, and the constant
// C_{i,a,p} = [Qin/q_i]_p 2^64 256^a mod p (Montgomery form) into 8 signed
// digits e_{i,a,p,b}, so
//   2^64 sum_i t_i [Qin/q_i]_p == sum_b 256^b sum_{i,a} d_{i,a} e_{i,a,p,b}  (mod p)
// with an inner sum of at most 80 products of magnitude <= 2^14 (exact in
// int32); one Montgomery reduction of the digit-weighted sum gives y_p.
// One 32x32x16 MFMA covers two input limbs (K = 2 x 8 digits) for 32
// coefficients (columns) and four outputs x 8 digits b (rows).
// Outputs modulo a prime below 2^50 instead use C_{i,a,p} = [Qin/q_i]_p
// 256^a mod p (no Montgomery factor) and an FP64 epilogue (bconv_combine_f64),
// which needs no 64-bit integer multiplies.
//   tab:  [nin] w, [nin] w'   Shoup pair of (Qin/q_i)^{-1} mod q_i
//   frag: [ngroups][nsteps][64] A-operand fragments (8 signed digit bytes per
//         lane, laid out as the instruction reads them)
//   ep:   [nout][BCONV_EPW] per output modulus (bconv_ep_fill): Montgomery
//         outputs hold the 128-bit offset M = p 2^k in [2^77, 2^78) (low
//         word, high word), p, p^{-1} mod 2^64, 0; FP64 outputs hold the
//         doubles 2^32 mod p, fl((2^32 mod p) / p), p, fl(1/p) (as bits), 1
struct BConvDesc {
  int32_t nin, nout;
  int32_t nsteps, ngroups;  // ceil(nin / 2) K-steps, ceil(nout / 4) row tiles
  int32_t in_pos[MAX_BCONV_IN], in_mod[MAX_BCONV_IN];
  int32_t out_pos[MAX_BCONV_OUT], out_mod[MAX_BCONV_OUT];
  const uint64_t* tab;
  const uint64_t* frag;
  const uint64_t* ep;
};

// Balanced base-256 digits of v < 2^61, packed as 8 int8 bytes: byte a is
// d_a in [-128, 127] with v = sum_a d_a 256^a (the top digit is <= 33).
HE_HD uint64_t sdigits(uint64_t v) {
  constexpr uint64_t H = 0x0080808080808080ull;
  return (v + H) ^ H;
}
HE_HD int sdigit(uint64_t v, int a) { return (int)(int8_t)(uint8_t)(sdigits(v) >> (8 * a)); }

// Row r of a 32-row accumulator tile holds output m (0..3) of the tile and
// digit weight b (0..7).  The 32x32 int32 accumulator gives lane l the rows
// (reg & 3) + 4 (l / 32) + 8 (reg / 4), so with this assignment lane l owns
// all eight b of outputs 2 (l / 32) and 2 (l / 32) + 1 in registers
// 0..7 and 8..15.
HE_HD void bconv_row(int row, int& m, int& b) {
  const int h = (row >> 2) & 1;
  const int reg = (row & 3) + 4 * (row >> 3);
  m = 2 * h + (reg >> 3);
  b = reg & 7;
}

// REDC(M + sum_b 256^b acc[b]) for |acc[b]| <= 80 2^14 < 2^20.33 (ten input
// limbs): the weighted sum has magnitude < 2^76.34, so with M = p 2^k in
// [2^77, 2^78) the argument lies in (0, 2^78.3) < p 2^64 and the result is
// canonical.
HE_HD uint64_t bconv_combine(const int32_t* acc, const uint64_t* ep) {
  const int64_t lo = (int64_t)acc[0] + (int64_t)acc[1] * 256 + (int64_t)acc[2] * 65536 + (int64_t)acc[3] * 16777216;
  const int64_t hi = (int64_t)acc[4] + (int64_t)acc[5] * 256 + (int64_t)acc[6] * 65536 + (int64_t)acc[7] * 16777216;
  const __int128 t = (__int128)hi * ((__int128)1 << 32) + lo + (__int128)(((unsigned __int128)ep[1] << 64) | ep[0]);
  return mont_redc(U128{(uint64_t)t, (uint64_t)((unsigned __int128)t >> 64)}, ep[2], ep[3]);
}

// Outputs modulo primes of at most 50 bits take the FP64 epilogue.
HE_HD bool bconv_out_f64(int kbits) { return kbits <= 50; }

// FP64 epilogue: V = sum_b 256^b acc[b] = lo + 2^32 hi with
// lo = sum_{b<4} 256^b acc[b] and hi = sum_{b>=4} 256^(b-4) acc[b].  Pairs
// acc[2c] + 256 acc[2c+1] stay below 2^28.34 (int32), lo and hi below
// 2^44.35, so both are exact doubles.  hi (2^32 mod p) is reduced with the
// centred product (|hi| 2^-52 < 2^-7.6, so the result is below 0.51 p in
// magnitude and exact), lo is added (an integer below 2^53) and one floor
// estimate with fl(1/p) plus a correction either way leaves V mod p.
HE_HD uint64_t bconv_combine_f64(const int32_t* acc, const uint64_t* ep) {
  const int32_t p0 = acc[0] + acc[1] * 256, p1 = acc[2] + acc[3] * 256;
  const int32_t p2 = acc[4] + acc[5] * 256, p3 = acc[6] + acc[7] * 256;
  const double lo = fma((double)p1, 65536.0, (double)p0);
  const double hi = fma((double)p3, 65536.0, (double)p2);
  const double p = bits_to_f64(ep[2]);
  const double v = mul_f64_c(hi, bits_to_f64(ep[0]), bits_to_f64(ep[1]), p) + lo;
  return f64_to_u52(canon_f64(v, bits_to_f64(ep[3]), p));
}

HE_HD uint64_t bconv_out(const int32_t* acc, const uint64_t* ep) {
  return ep[4] ? bconv_combine_f64(acc, ep) : bconv_combine(acc, ep);
}

// (host) Epilogue record of one output modulus po (kbits bits, pinv64 = po^{-1} mod 2^64).
inline void bconv_ep_fill(uint64_t po, int kbits, uint64_t pinv64, uint64_t* ep) {
  if (bconv_out_f64(kbits)) {
    const uint64_t c32 = (uint64_t)(((unsigned __int128)1 << 32) % po);
    ep[0] = f64_to_bits((double)c32);
    ep[1] = f64_to_bits((double)c32 / (double)po);
    ep[2] = f64_to_bits((double)po);
    ep[3] = f64_to_bits(1.0 / (double)po);
    ep[4] = 1;
    return;
  }
  int kshift = 0;
  while (((unsigned __int128)po << kshift) < ((unsigned __int128)1 << 77)) kshift++;
  const unsigned __int128 M = (unsigned __int128)po << kshift;
  ep[0] = (uint64_t)M;
  ep[1] = (uint64_t)(M >> 64);
  ep[2] = po;
  ep[3] = pinv64;
  ep[4] = 0;
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
