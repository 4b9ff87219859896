// Host check of the fused kernel's FP64 key inner product for primes below
// 2^50: centred digit values (|v| up to 2.9q, including both extremes) times
// Montgomery-form key words, summed over one to four digits, then one
// centred product by 2^-64 mod q and canon_f64; compared with
// (sum_j v_j k_j) 2^-64 mod q computed with 128-bit integers and %.
#include <cstdio>
#include <random>

#include "../../paper_2510_03996_amd/csrc/modarith.h"
using namespace he;
typedef unsigned __int128 u128;
static uint64_t hmul(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }
static uint64_t hpow(uint64_t a, uint64_t e, uint64_t q) {
  uint64_t r = 1;
  while (e) { if (e & 1) r = hmul(r, a, q); a = hmul(a, a, q); e >>= 1; }
  return r;
}
int main() {
  std::mt19937_64 rng(3);
  long bad = 0, total = 0;
  for (uint64_t q : {1125899903827969ull, 1125899844714497ull, 1099511480321ull, 35184371138561ull, 1099511390209ull}) {
    const uint64_t r64 = (uint64_t)(((u128)1 << 64) % q), rinv = hpow(r64, q - 2, q);
    const double dq = (double)q, qi = 1.0 / dq, rv = (double)rinv, rvq = (double)rinv / dq;
    const long long lim = (long long)(2.9 * (double)q);
    for (int t = 0; t < 1000000; t++) {
      const int dn = 1 + t % 4;
      double acc = 0;
      uint64_t want = 0;
      for (int j = 0; j < dn; j++) {
        const long long v = (t % 7 == 0) ? (j & 1 ? lim : -lim) : (long long)(rng() % (2 * (uint64_t)lim + 1)) - lim;
        const uint64_t km = (t % 11 == 0) ? q - 1 : rng() % q;
        const double w = u52_to_f64(km);
        acc += mul_f64_c((double)v, w, w * qi, dq);
        const uint64_t vc = (uint64_t)(((v % (long long)q) + (long long)q) % (long long)q);
        want = (want + hmul(vc, km, q)) % q;
      }
      want = hmul(want, rinv, q);
      const uint64_t got = f64_to_u52(canon_f64(mul_f64_c(acc, rv, rvq, dq), qi, dq));
      total++;
      if (got != want) {
        if (bad < 5) printf("q %llu digits %d: got %llu want %llu\n", (unsigned long long)q, dn, (unsigned long long)got,
                            (unsigned long long)want);
        bad++;
      }
    }
  }
  printf("fp64 inner product: %ld mismatches of %ld\n", bad, total);
  printf(bad ? "FAIL\n" : "OK\n");
  return bad != 0;
}
