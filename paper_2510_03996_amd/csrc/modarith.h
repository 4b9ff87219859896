// Word-size modular arithmetic for primes q < 2^61 on gfx950.
//
// Every modular product runs on the vector ALUs: 32-bit integer multiplies
// for primes of 51 bits and more, centred FP64 FMA for primes below 2^50.
// The basis conversion, the one contraction of the key switch, is a short
// sum (at most ten inputs) per output residue and runs on the same ALUs
// (ConvDesc in elem_core.h).  Three integer reductions are used:
//   * Shoup multiplication by a constant w with companion w' = floor(w 2^64 / q)
//     (NTT twiddles, the inverse transform's finishing factors, q^{-1}, P^{-1});
//   * Montgomery reduction of a 128-bit accumulator (key inner product, the
//     basis conversion into primes of 51 bits and more) with constants stored
//     premultiplied by 2^64 mod q;
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

// Centred FP64 arithmetic for primes q < 2^50 (the NTT's FP64 path).
// Residues are integer-valued doubles of magnitude below 8q < 2^53, so every
// value is exact.  mul_f64_c(a, w, wq): with wq = fl(w/q) the estimate
// fl(a wq) is within |a| 2^-52 <= |a| / (4q) of a w / q, so the quotient
// quot = rint(fl(a wq)) leaves r = a w - quot q with |r| <= q (1/2 + |a| / (4q)).
// a w = hi + lo exactly (two-product with one FMA); hi - quot q is an integer
// below 2^53 in magnitude, hence exact in one FMA, and r = (hi - quot q) + lo
// is exact too.  No conditional corrections are needed: callers keep |a| <= 8q
// and re-centre with centre_f64 (|result| <= q/2 + 1) once per LDS round.
// The same argument holds for a centred |w| <= 3q/4 with wq = fl(w fl(1/q))
// (the NTT's factored twiddles): the estimate is then within
// 1.125 |a| 2^-52 of a w / q.
HE_HD double mul_f64_c(double a, double w, double wq, double q) {
  const double quot = rint(a * wq);
  const double hi = a * w;
  const double lo = fma(a, w, -hi);
  return fma(-quot, q, hi) + lo;
}
HE_HD double centre_f64(double x, double qinv, double q) { return fma(-rint(x * qinv), q, x); }
HE_HD double bits_to_f64(uint64_t b) {
  double d;
  __builtin_memcpy(&d, &b, 8);
  return d;
}
HE_HD uint64_t f64_to_bits(double d) {
  uint64_t b;
  __builtin_memcpy(&b, &d, 8);
  return b;
}
// Exact conversions of integers below 2^52: x is the low mantissa of 2^52 + x.
HE_HD double u52_to_f64(uint64_t x) { return bits_to_f64(x | 0x4330000000000000ull) - 4503599627370496.0; }
HE_HD uint64_t f64_to_u52(double v) { return f64_to_bits(v + 4503599627370496.0) & 0x000FFFFFFFFFFFFFull; }
// canonical representative in [0, q) of an integer-valued |x| < 2^53 (q > 4):
// fl(x fl(1/q)) is within 2^-51 |x| / q < 1 of x / q, so its floor is off by
// at most one, x - floor q (exact in one FMA) lies in [-q, 2q) and one
// correction either way ends it
HE_HD double canon_f64(double x, double qinv, double q) {
  double r = fma(-floor(x * qinv), q, x);
  r = r < 0.0 ? r + q : r;
  return r >= q ? r - q : r;
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
  double dqinv;          // 1/q as a double (FP64 NTT path)
  double drinv, drinvq;  // 2^-64 mod q and fl(that / q) (FP64 key inner product)
  double dpad;
};

HE_HD uint64_t mul_mod(uint64_t a, uint64_t b, const ModInfo& m) {
  return barrett_reduce(mul_wide(a, b), m.q, m.mu, m.k);
}

}  // namespace he
