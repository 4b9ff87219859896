// Word-size modular arithmetic for primes q < 2^61 on gfx950.
//
// Integer-ALU only (no MFMA: a 64-bit modular product is not a floating-point
// contraction).  Three reductions are used:
//   * Shoup multiplication by a constant w with companion w' = floor(w 2^64 / q)
//     (NTT twiddles, BConv input factors, q^{-1}, P^{-1});
//   * Montgomery reduction of a 128-bit accumulator (key inner product, BConv
//     sums) with constants stored premultiplied by 2^64 mod q;
//   * Barrett reduction of a full 128-bit product for ct (.) pt products where
//     neither operand is a precomputed constant.
// All results are canonical residues in [0, q): any exact reduction yields the
// same integers, which is what makes the GPU bit-identical to a plain `%`.
#pragma once
#include <stdint.h>

#include <math.h>
#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define HE_HD __host__ __device__ __forceinline__
#else
#define HE_HD inline  // plain host build (CPU emulation of kernel index math)
#endif

namespace he {

HE_HD uint64_t mulhi(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

struct U128 {
  uint64_t lo, hi;
};

HE_HD U128 mul_wide(uint64_t a, uint64_t b) { return U128{a * b, mulhi(a, b)}; }

HE_HD void add_wide(U128& acc, U128 x) {
  uint64_t lo = acc.lo + x.lo;
  acc.hi += x.hi + (lo < x.lo ? 1 : 0);
  acc.lo = lo;
}

HE_HD uint64_t add_mod(uint64_t a, uint64_t b, uint64_t q) {
  uint64_t s = a + b;
  return s >= q ? s - q : s;
}
HE_HD uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t q) { return a >= b ? a - b : a + q - b; }
HE_HD uint64_t neg_mod(uint64_t a, uint64_t q) { return a == 0 ? 0 : q - a; }

// a * w mod q for any a < 2^64; result in [0, 2q).
HE_HD uint64_t mul_shoup_lazy(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
  uint64_t t = mulhi(a, wp);
  return a * w - t * q;
}
HE_HD uint64_t mul_shoup(uint64_t a, uint64_t w, uint64_t wp, uint64_t q) {
  uint64_t r = mul_shoup_lazy(a, w, wp, q);
  return r >= q ? r - q : r;
}

// Montgomery: REDC(T) = T * 2^-64 mod q for T < q 2^64, qinv = q^{-1} mod 2^64.
HE_HD uint64_t mont_redc(U128 t, uint64_t q, uint64_t qinv) {
  uint64_t m = t.lo * qinv;
  uint64_t h = mulhi(m, q);
  return t.hi >= h ? t.hi - h : t.hi + q - h;
}

// Barrett (HAC 14.42 in base 2): x < q^2 with q of k bits (2^(k-1) <= q < 2^k),
// mu = floor(2^(2k) / q) < 2^(k+1).  Two conditional subtractions.
HE_HD uint64_t barrett_reduce(U128 x, uint64_t q, uint64_t mu, int k) {
  uint64_t q1 = (x.hi << (65 - k)) | (x.lo >> (k - 1));
  uint64_t plo = q1 * mu, phi = mulhi(q1, mu);
  uint64_t q3 = (phi << (63 - k)) | (plo >> (k + 1));
  uint64_t r = x.lo - q3 * q;
  if (r >= q) r -= q;
  if (r >= q) r -= q;
  return r;
}

// FP64 product for primes q < 2^50 (residues kept below 4q < 2^52, exact in a
// double): with wq = fl(w/q), quot = floor(fl(a wq)) is within 1 of
// floor(a w / q) (|a (wq - w/q)| <= 2^52 2^-54 and the rounding of a wq adds
// at most 2^-2), so r = a w - quot q lies in [-q, 2q).  a w = hi + lo exactly
// (two-product with one FMA), hi - quot q is an integer below 2^53 in
// magnitude and therefore exact in one FMA, and r = (hi - quot q) + lo is
// exact as well.  Returns r in [0, 2q) (same range as mul_shoup_lazy).
HE_HD double mul_f64_lazy(double a, double w, double wq, double q) {
  const double quot = floor(a * wq);
  const double hi = a * w;
  const double lo = fma(a, w, -hi);
  const double r = fma(-quot, q, hi) + lo;
  return r < 0.0 ? r + q : r;
}

// Per-modulus constants (device resident).
struct ModInfo {
  uint64_t q;
  uint64_t qinv;      // q^{-1} mod 2^64 (Montgomery)
  uint64_t r2;        // 2^128 mod q   (to Montgomery form: REDC(x * r2))
  uint64_t mu;        // floor(2^(2k) / q) (Barrett)
  uint64_t ninv, ninv_p;   // N^{-1} mod q and Shoup companion
  int32_t k;          // bit length of q
  int32_t pad;
  double dninv, dninvq;  // N^{-1} and N^{-1}/q as doubles (FP64 NTT path, q < 2^50)
};

HE_HD uint64_t mul_mod(uint64_t a, uint64_t b, const ModInfo& m) {
  return barrett_reduce(mul_wide(a, b), m.q, m.mu, m.k);
}

}  // namespace he
