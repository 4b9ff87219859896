// Host check of the basis conversion's per-residue arithmetic as the fused
// conversion kernel runs it (elem_core.h): inputs split into parts
// (conv_part_ab / conv_part: one exact double below 2^50, or the low 32 bits
// and the rest of a wider residue), FP64 outputs as a sum of centred
// products mul_f64_c re-centred after every eighth part, integer outputs as
// 128-bit products with Montgomery constants (conv_mac_int) and one REDC.
// Constants are formed as the library forms them ([Qin/q_i]_p 2^shift,
// centred for FP64 outputs, times 2^64 for integer ones).  Reference:
// y_p = sum_i t_i [Qin/q_i]_p mod p with 128-bit integers and %.  Inputs
// include 0 and q_i - 1; the FP64 sums are also checked to stay integral and
// below 5.5 p in magnitude (the bound the column pass relies on).
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <vector>
#include <random>
#include "../../paper_2510_03996_amd/csrc/elem_core.h"
using namespace he;
typedef unsigned __int128 u128;
static uint64_t hmul(uint64_t a, uint64_t b, uint64_t q) { return (uint64_t)((u128)a * b % q); }
static uint64_t hpow(uint64_t a, uint64_t e, uint64_t q) { uint64_t r = 1 % q; while (e) { if (e & 1) r = hmul(r, a, q); a = hmul(a, a, q); e >>= 1; } return r; }
static bool isprime(uint64_t n) { if (n < 2) return false; for (uint64_t a : {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37}) { if (n % a == 0) return n == a; }
  uint64_t d = n - 1; int s = 0; while (!(d & 1)) { d >>= 1; s++; }
  for (uint64_t a : {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37}) { uint64_t x = hpow(a, d, n); if (x == 1 || x == n - 1) continue; bool ok = false;
    for (int r = 1; r < s; r++) { x = hmul(x, x, n); if (x == n - 1) { ok = true; break; } } if (!ok) return false; } return true; }
static std::vector<uint64_t> primes(int bits, int cnt, uint64_t two_n) {
  std::vector<uint64_t> v; uint64_t k = ((uint64_t)1 << bits) / two_n;
  while ((int)v.size() < cnt && k > 0) { uint64_t p = k * two_n + 1; if (p < ((uint64_t)1 << bits) && isprime(p)) v.push_back(p); k--; } return v; }
static int bits(uint64_t q) { return 64 - __builtin_clzll(q); }

int main() {
  std::mt19937_64 rng(7);
  int bad = 0, total = 0, nf64 = 0, nint = 0, nwide = 0;
  double worst = 0.0;  // largest |FP64 sum| / p
  // (input bits, inputs, output bits, outputs); the first input of some
  // cases is a wider prime (as q_0 of a digit)
  struct Case { int bin0, bin, nin, bout, nout; } cases[] = {
      {60, 50, 8, 50, 25}, {50, 50, 8, 60, 1}, {50, 50, 9, 50, 24}, {50, 50, 9, 60, 1}, {54, 40, 1, 40, 2},
      {55, 55, 1, 40, 3}, {60, 45, 2, 45, 6}, {60, 60, 2, 45, 8}, {60, 60, 2, 60, 1}, {50, 50, 10, 50, 33},
      {61, 61, 10, 50, 8}, {61, 61, 10, 61, 3}, {40, 40, 3, 54, 1}, {45, 45, 10, 41, 16}, {24, 24, 4, 24, 5}};
  for (auto cs : cases) {
    std::vector<uint64_t> qin = primes(cs.bin0, 1, 1 << 13);
    auto rest = primes(cs.bin, cs.nin + 1, 1 << 13);
    for (uint64_t q : rest) if ((int)qin.size() < cs.nin && q != qin[0]) qin.push_back(q);
    if ((int)qin.size() < cs.nin) { printf("not enough input primes\n"); return 1; }
    auto qout = primes(cs.bout, cs.nout + cs.nin + 1, 1 << 13);
    std::vector<uint64_t> qo;
    for (uint64_t q : qout) { bool used = false; for (uint64_t a : qin) used |= a == q; if (!used && (int)qo.size() < cs.nout) qo.push_back(q); }
    if ((int)qo.size() < cs.nout) { printf("not enough output primes\n"); return 1; }
    // parts
    std::vector<int> part_in, part_kind, part_sh;
    for (int i = 0; i < cs.nin; i++) {
      if (conv_in_narrow(bits(qin[i]))) { part_in.push_back(i); part_kind.push_back(0); part_sh.push_back(0); }
      else { nwide++; for (int h = 0; h < 2; h++) { part_in.push_back(i); part_kind.push_back(1 + h); part_sh.push_back(32 * h); } }
    }
    const int np = (int)part_in.size();
    for (int p = 0; p < cs.nout; p++) {
      const uint64_t po = qo[p];
      const bool f64 = conv_out_f64(bits(po));
      (f64 ? nf64 : nint)++;
      std::vector<uint64_t> cst(2 * np);
      std::vector<uint64_t> plain(cs.nin);  // [Qin/q_i]_p
      for (int i = 0; i < cs.nin; i++) { uint64_t v = 1 % po; for (int i2 = 0; i2 < cs.nin; i2++) if (i2 != i) v = hmul(v, qin[i2] % po, po); plain[i] = v; }
      for (int v = 0; v < np; v++) {
        const uint64_t w = hmul(plain[part_in[v]], (uint64_t)(((u128)1 << part_sh[v]) % po), po);
        if (f64) {
          const double wc = w > po / 2 ? -(double)(po - w) : (double)w, wq = wc / (double)po;
          cst[2 * v] = f64_to_bits(wc); cst[2 * v + 1] = f64_to_bits(wq);
        } else {
          cst[2 * v] = hmul(w, (uint64_t)(((u128)1 << 64) % po), po); cst[2 * v + 1] = 0;
        }
      }
      uint64_t pinv64 = 1; for (int it = 0; it < 7; it++) pinv64 *= 2 - po * pinv64;
      for (int trial = 0; trial < 400; trial++) {
        std::vector<uint64_t> t(cs.nin);
        for (int i = 0; i < cs.nin; i++) t[i] = trial < 2 ? (trial ? qin[i] - 1 : 0) : rng() % qin[i];
        double x[2 * MAX_BCONV_IN];
        for (int v = 0; v < np; v++) { double a, b; conv_part_ab(part_kind[v], a, b); x[v] = conv_part(t[part_in[v]], a, b); }
        uint64_t got;
        if (f64) {
          const double pd = (double)po, pi = 1.0 / pd;
          double acc = 0.0;
          for (int v = 0; v < np; v++) {
            acc += mul_f64_c(x[v], bits_to_f64(cst[2 * v]), bits_to_f64(cst[2 * v + 1]), pd);
            if ((v & 7) == 7) acc = centre_f64(acc, pi, pd);
            if (acc != std::floor(acc)) { bad++; printf("non-integral sum\n"); }
          }
          worst = std::max(worst, std::fabs(acc) / pd);
          got = f64_to_u52(canon_f64(acc, pi, pd));
        } else {
          U128 acc{0, 0};
          for (int v = 0; v < np; v++) conv_mac_int(acc, x[v], cst[2 * v], po);
          got = mont_redc(acc, po, pinv64);
        }
        u128 want = 0;
        for (int i = 0; i < cs.nin; i++) want += (u128)t[i] * plain[i];
        const uint64_t w = (uint64_t)(want % po);
        total++;
        if (got != w) { if (bad < 5) printf("case nin=%d bout=%d p=%d got %llu want %llu\n", cs.nin, cs.bout, p, (unsigned long long)got, (unsigned long long)w); bad++; }
      }
    }
  }
  printf("bconv emu: %d mismatches of %d outputs (%d FP64 and %d integer output moduli, %d wide inputs), max |FP64 sum| = %.3f p\n",
         bad, total, nf64, nint, nwide, worst);
  const bool ok = bad == 0 && nf64 > 0 && nint > 0 && nwide > 0 && worst < 5.5;
  printf(ok ? "OK\n" : "FAIL\n");
  return ok ? 0 : 1;
}
