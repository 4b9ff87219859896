// Host check that the NTT-form automorphism phi_g maps every aligned block of
// 2^t positions onto one aligned block, for the tile sizes the fused
// inner-product kernel may use (2^9 .. 2^12): every Galois element at
// N = 2^12, an evenly spaced sample plus the rotation elements 5^r at 2^14 and
// 2^16.  The kernel stages one source tile per output tile on this property.
#include <cstdio>
#include <vector>

#include "../../paper_2510_03996_amd/csrc/elem_core.h"
using namespace he;
int main() {
  long bad = 0, checked = 0;
  for (int logn : {12, 14, 16}) {
    const uint32_t n = 1u << logn, two_n = 2 * n;
    std::vector<uint32_t> gs;
    const uint32_t step = logn == 12 ? 2 : logn == 14 ? 258 : 4098;
    for (uint32_t g = 1; g < two_n; g += step) gs.push_back(g);
    uint32_t g5 = 1;
    for (int r = 0; r < 64; r++) { gs.push_back(g5); g5 = (uint32_t)((5ull * g5) % two_n); }
    gs.push_back(two_n - 1);  // conjugation
    for (int lt = 9; lt <= 12; lt++) {
      const uint32_t T = (1u << lt) > n ? n : (1u << lt);
      for (uint32_t g : gs)
        for (uint32_t b = 0; b < n; b += T) {
          const uint32_t s0 = automorph_src(b, g, logn) & ~(T - 1);
          for (uint32_t e = 0; e < T; e++) {
            const uint32_t s = automorph_src(b + e, g, logn);
            checked++;
            if (s < s0 || s >= s0 + T) bad++;
          }
        }
    }
  }
  printf("automorphism blocks: %ld positions checked, %ld outside their block\n", checked, bad);
  printf(bad ? "FAIL\n" : "OK\n");
  return bad != 0;
}
