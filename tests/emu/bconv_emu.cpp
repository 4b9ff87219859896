// Host check of the int8 matrix-core basis conversion: the constant tables
// and A-operand fragments built as the library builds them, the digit
// products summed in the lane/row layout of v_mfma_i32_32x32x16_i8, and the
// library's epilogues (bconv_out: Montgomery for outputs modulo primes above
// 2^50, FP64 below), against y_p = sum_i t_i [Qin/q_i]_p mod p computed with
// 128-bit integers and %.  Inputs include 0 and q_i - 1.
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
  while ((int)v.size() < cnt) { uint64_t p = k * two_n + 1; if (p < ((uint64_t)1 << bits) && isprime(p)) v.push_back(p); k--; } return v; }
int main() {
  std::mt19937_64 rng(7);
  int bad = 0, total = 0, nf64 = 0;
  struct Case { int bin, nin, bout, nout; } cases[] = {{50, 8, 60, 24}, {60, 8, 50, 24}, {40, 1, 55, 3}, {45, 2, 60, 7}, {50, 5, 40, 61}, {60, 3, 60, 1}, {50, 9, 50, 24}, {50, 8, 50, 25}, {60, 10, 60, 30}, {50, 10, 40, 9}, {40, 2, 40, 5}, {40, 3, 54, 1}, {50, 9, 50, 33}, {45, 10, 41, 16}};
  for (auto cs : cases) {
    auto qin = primes(cs.bin, cs.nin, 1 << 17);
    auto qout = primes(cs.bout, cs.nout + cs.nin, 1 << 17);
    qout.erase(qout.begin(), qout.begin() + cs.nin);  // distinct from the inputs when the sizes match
    int nsteps = (cs.nin + 1) / 2, ngroups = (cs.nout + 3) / 4;
    std::vector<uint64_t> cst(cs.nin * cs.nout), pre(cs.nin);
    for (int i = 0; i < cs.nin; i++) {
      uint64_t prod = 1;
      for (int i2 = 0; i2 < cs.nin; i2++) if (i2 != i) prod = hmul(prod, qin[i2] % qin[i], qin[i]);
      pre[i] = hpow(prod, qin[i] - 2, qin[i]);
      for (int p = 0; p < cs.nout; p++) { uint64_t v = 1; for (int i2 = 0; i2 < cs.nin; i2++) if (i2 != i) v = hmul(v, qin[i2] % qout[p], qout[p]); int kb = 64 - __builtin_clzll(qout[p]); cst[i * cs.nout + p] = bconv_out_f64(kb) ? v : hmul(v, (uint64_t)(((u128)1 << 64) % qout[p]), qout[p]); }
    }
    std::vector<uint64_t> frag(ngroups * nsteps * 64, 0);
    for (int g = 0; g < ngroups; g++) for (int st = 0; st < nsteps; st++) for (int l = 0; l < 64; l++) {
      int m, b; bconv_row(l % 32, m, b); int p = 4 * g + m, i = 2 * st + l / 32;
      if (p >= cs.nout || i >= cs.nin) continue;
      uint64_t word = 0, cp = cst[i * cs.nout + p];
      for (int a = 0; a < 8; a++) { word |= (uint64_t)(uint8_t)(int8_t)sdigit(cp, b) << (8 * a); cp = hmul(cp, 256 % qout[p], qout[p]); }
      frag[(g * nsteps + st) * 64 + l] = word;
    }
    std::vector<uint64_t> ep(cs.nout * BCONV_EPW);
    for (int p = 0; p < cs.nout; p++) { uint64_t po = qout[p]; uint64_t inv = 1; for (int it = 0; it < 7; it++) inv *= 2 - po * inv;
      bconv_ep_fill(po, 64 - __builtin_clzll(po), inv, &ep[BCONV_EPW * p]); nf64 += ep[BCONV_EPW * p + 4] != 0; }
    for (int trial = 0; trial < 64; trial++) {  // 32 coefficients per trial (one wave)
      uint64_t x[10][32], t[10][32];
      for (int i = 0; i < cs.nin; i++) for (int c = 0; c < 32; c++) {
        x[i][c] = trial < 2 ? (trial ? qin[i] - 1 : 0) : rng() % qin[i];
        t[i][c] = hmul(x[i][c], pre[i], qin[i]); }
      for (int g = 0; g < ngroups; g++) {
        int32_t acc[64][16] = {};
        for (int st = 0; st < nsteps; st++) for (int row = 0; row < 32; row++) for (int col = 0; col < 32; col++) {
          int32_t sum = 0;
          for (int kk = 0; kk < 16; kk++) {
            int la = row + 32 * (kk / 8), lb = col + 32 * (kk / 8);
            int i = 2 * st + lb / 32;
            uint64_t bw = i < cs.nin ? sdigits(t[i][col]) : 0;
            int8_t av = (int8_t)(frag[(g * nsteps + st) * 64 + la] >> (8 * (kk % 8)));
            int8_t bv = (int8_t)(bw >> (8 * (kk % 8)));
            sum += av * bv;
          }
          acc[col + 32 * ((row / 4) % 2)][(row % 4) + 4 * (row / 8)] += sum;
        }
        for (int l = 0; l < 64; l++) for (int mm = 0; mm < 2; mm++) {
          int p = 4 * g + 2 * (l / 32) + mm; if (p >= cs.nout) continue;
          int col = l % 32;
          uint64_t got = bconv_out(&acc[l][8 * mm], &ep[BCONV_EPW * p]);
          u128 want = 0; for (int i = 0; i < cs.nin; i++) { uint64_t pl = 1; for (int i2 = 0; i2 < cs.nin; i2++) if (i2 != i) pl = hmul(pl, qin[i2] % qout[p], qout[p]); want += (u128)t[i][col] * pl; }
          uint64_t w = (uint64_t)(want % qout[p]);
          total++; if (got != w) { if (bad < 5) printf("case %d/%d p=%d col=%d got %llu want %llu\n", cs.nin, cs.nout, p, col, (unsigned long long)got, (unsigned long long)w); bad++; }
        }
      }
    }
  }
  printf("bconv emu: %d mismatches of %d outputs (%d FP64 output moduli)\n", bad, total, nf64);
  const bool ok = bad == 0 && nf64 > 0;
  printf(ok ? "OK\n" : "FAIL\n");
  return ok ? 0 : 1;
}
