// Host run of the NTT kernels' own round code (ntt_core.h compiled for the
// CPU, one workgroup after another, thread after thread inside each LDS round)
// against the oracle's textbook transform, for every (tile, residues per
// thread) shape the library launches: integer arithmetic for a 60-bit prime,
// centred FP64 for primes below 2^50 with table and with factored pass-2
// twiddles.  It also records the largest |value| / q met at the start of a
// round or after a pass, the quantity the FP64 exactness bounds are about.
#include <cmath>
#include <cstdio>
#include <random>
#include <type_traits>
#include <vector>

#include "../../paper_2510_03996_amd/csrc/ntt_core.h"

extern "C" {
void or_ntt_fwd_limb(uint64_t* a, size_t n, uint64_t q, uint64_t psi);
uint64_t or_powmod(uint64_t a, uint64_t e, uint64_t q);
uint64_t or_invmod(uint64_t a, uint64_t q);
}
using namespace he;
typedef unsigned __int128 u128;

static int brv(int x, int logn) {
  int r = 0;
  for (int i = 0; i < logn; i++) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

static double g_max_ratio = 0;
static long g_non_integer = 0;
template <class T>
static void note_values(const T* v, int n, double q) {
  if constexpr (std::is_same<T, double>::value)
    for (int i = 0; i < n; i++) {
      const double x = v[i];
      if (x != x || std::fabs(x) / q > g_max_ratio) g_max_ratio = std::fabs(x) / q;
      if (std::floor(x) != x) g_non_integer++;
    }
}

// all LDS rounds of one workgroup, forward (rounds 0..NR-1) or inverse
template <class P, bool FACT, class T, class TW, class Q>
static void run_rounds(T* lds, int wg, const TW* tw, const TW* twq, Q q, bool inv) {
  auto one = [&](auto idx_c) {
    constexpr int IDX = decltype(idx_c)::value;
    if constexpr (IDX < P::NR) {
      note_values(lds, P::LDS_WORDS, (double)q);
      for (int t = 0; t < P::THREADS; t++) {
        if constexpr (std::is_same<T, double>::value)
          P::template round_f64<P::rbits(IDX), FACT>(lds, t, wg, P::rstart(IDX), tw, twq, q, 1.0 / q);
        else
          P::template round<P::rbits(IDX)>(lds, t, wg, P::rstart(IDX), tw, twq, q);
      }
    }
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  if (!inv) { one(I0{}); one(I1{}); one(I2{}); one(I3{}); }
  else { one(I3{}); one(I2{}); one(I1{}); one(I0{}); }
}

template <int LOGN, int PASS, bool INV, int E, int T>
static void pass_int(std::vector<uint64_t>& a, const std::vector<uint64_t>& tw, const std::vector<uint64_t>& twp,
                     uint64_t q, uint64_t ninv, uint64_t ninvp) {
  using P = NttPass<LOGN, PASS, INV, E, T>;
  std::vector<uint64_t> lds(P::LDS_WORDS);
  for (int wg = 0; wg < P::WG_PER_LIMB; wg++) {
    for (int e = 0; e < P::TILE; e++) { int g, k; P::tile_elem(e, g, k); lds[P::lidx(g, k)] = a[P::gidx(wg, g, k)]; }
    run_rounds<P, false>(lds.data(), wg, tw.data(), twp.data(), q, INV);
    for (int e = 0; e < P::TILE; e++) {
      int g, k;
      P::tile_elem(e, g, k);
      a[P::gidx(wg, g, k)] = P::finish(lds[P::lidx(g, k)], ninv, ninvp, q);
    }
  }
}

template <int LOGN, int PASS, bool INV, int E, int T, bool FACT>
static void pass_f64(std::vector<uint64_t>& a, const std::vector<double>& tw, const std::vector<double>& twq, double q,
                     double ninv, double ninvq) {
  using P = NttPass<LOGN, PASS, INV, E, T>;
  std::vector<double> lds(P::LDS_WORDS);
  for (int wg = 0; wg < P::WG_PER_LIMB; wg++) {
    for (int e = 0; e < P::TILE; e++) { int g, k; P::tile_elem(e, g, k); lds[P::lidx(g, k)] = P::load_f64(a[P::gidx(wg, g, k)]); }
    run_rounds<P, FACT>(lds.data(), wg, tw.data(), twq.data(), q, INV);
    note_values(lds.data(), P::LDS_WORDS, q);
    for (int e = 0; e < P::TILE; e++) {
      int g, k;
      P::tile_elem(e, g, k);
      a[P::gidx(wg, g, k)] = P::finish_f64(lds[P::lidx(g, k)], ninv, ninvq, q, 1.0 / q);
    }
  }
}

struct Tables {
  uint64_t q, psi, ninv, ninvp;
  std::vector<uint64_t> tw, twp, itw, itwp;
  std::vector<double> dtw, dtwq, ditw, ditwq;
};

static Tables make_tables(int logn, uint64_t q) {
  const int n = 1 << logn;
  Tables t;
  t.q = q;
  // minimum primitive 2N-th root of unity
  uint64_t c = 0;
  for (uint64_t x = 2;; x++) {
    c = or_powmod(x, (q - 1) / (2 * (uint64_t)n), q);
    if (or_powmod(c, n, q) == q - 1) break;
  }
  const uint64_t sq = (uint64_t)((u128)c * c % q);
  uint64_t cur = c, psi = c;
  for (int k = 1; k < n; k++) { cur = (uint64_t)((u128)cur * sq % q); if (cur < psi) psi = cur; }
  t.psi = psi;
  const uint64_t ipsi = or_invmod(psi, q);
  std::vector<uint64_t> pw(n), ipw(n);
  pw[0] = ipw[0] = 1;
  for (int k = 1; k < n; k++) { pw[k] = (uint64_t)((u128)pw[k - 1] * psi % q); ipw[k] = (uint64_t)((u128)ipw[k - 1] * ipsi % q); }
  t.tw.resize(n); t.twp.resize(n); t.itw.resize(n); t.itwp.resize(n);
  t.dtw.resize(n); t.dtwq.resize(n); t.ditw.resize(n); t.ditwq.resize(n);
  for (int k = 0; k < n; k++) {
    const int b = brv(k, logn);
    t.tw[k] = pw[b];
    t.itw[k] = ipw[b];
    t.twp[k] = (uint64_t)(((u128)t.tw[k] << 64) / q);
    t.itwp[k] = (uint64_t)(((u128)t.itw[k] << 64) / q);
    t.dtw[k] = (double)t.tw[k];
    t.dtwq[k] = (double)t.tw[k] / (double)q;
    t.ditw[k] = (double)t.itw[k];
    t.ditwq[k] = (double)t.itw[k] / (double)q;
  }
  t.ninv = or_invmod((uint64_t)n % q, q);
  t.ninvp = (uint64_t)(((u128)t.ninv << 64) / q);
  return t;
}

static int g_cases = 0, g_bad = 0;
static void report(const char* what, int logn, int e1, int t1, int e2, int t2, bool fact, uint64_t q, int bad) {
  g_cases++;
  if (bad) {
    g_bad++;
    printf("MISMATCH %s logn=%d pass1=(2^%d, 2^%d) pass2=(2^%d, 2^%d) fact=%d q=%llu: %d residues\n", what, logn, e1,
           t1, e2, t2, (int)fact, (unsigned long long)q, bad);
  }
}

// one forward + inverse transform with pass 1 shaped (E1, T1) and pass 2 (E2, T2)
template <int LOGN, int E1, int T1, int E2, int T2>
static void check(const Tables& t, std::mt19937_64& rng) {
  const int n = 1 << LOGN;
  std::vector<uint64_t> a(n);
  for (auto& x : a) x = rng() % t.q;
  a[0] = t.q - 1;  // the largest residue
  std::vector<uint64_t> want = a;
  or_ntt_fwd_limb(want.data(), n, t.q, t.psi);
  if (t.q >> 50 == 0) {
    const double dq = (double)t.q, dn = (double)t.ninv, dnq = (double)t.ninv / dq;
    auto run = [&](auto fact_c) {
      constexpr bool F = decltype(fact_c)::value;
      std::vector<uint64_t> b = a;
      pass_f64<LOGN, 1, false, E1, T1, false>(b, t.dtw, t.dtwq, dq, dn, dnq);
      pass_f64<LOGN, 2, false, E2, T2, F>(b, t.dtw, t.dtwq, dq, dn, dnq);
      int bad = 0;
      for (int k = 0; k < n; k++) bad += b[k] != want[k];
      report("fp64 forward", LOGN, E1, T1, E2, T2, F, t.q, bad);
      pass_f64<LOGN, 2, true, E2, T2, F>(b, t.ditw, t.ditwq, dq, dn, dnq);
      pass_f64<LOGN, 1, true, E1, T1, false>(b, t.ditw, t.ditwq, dq, dn, dnq);
      bad = 0;
      for (int k = 0; k < n; k++) bad += b[k] != a[k];
      report("fp64 round trip", LOGN, E1, T1, E2, T2, F, t.q, bad);
    };
    run(std::false_type{});
    run(std::true_type{});
  } else {
    std::vector<uint64_t> b = a;
    pass_int<LOGN, 1, false, E1, T1>(b, t.tw, t.twp, t.q, t.ninv, t.ninvp);
    pass_int<LOGN, 2, false, E2, T2>(b, t.tw, t.twp, t.q, t.ninv, t.ninvp);
    int bad = 0;
    for (int k = 0; k < n; k++) bad += b[k] != want[k];
    report("integer forward", LOGN, E1, T1, E2, T2, false, t.q, bad);
    pass_int<LOGN, 2, true, E2, T2>(b, t.itw, t.itwp, t.q, t.ninv, t.ninvp);
    pass_int<LOGN, 1, true, E1, T1>(b, t.itw, t.itwp, t.q, t.ninv, t.ninvp);
    bad = 0;
    for (int k = 0; k < n; k++) bad += b[k] != a[k];
    report("integer round trip", LOGN, E1, T1, E2, T2, false, t.q, bad);
  }
}

template <int LOGN>
static void all_shapes(uint64_t q) {
  const Tables t = make_tables(LOGN, q);
  std::mt19937_64 rng(q ^ LOGN);
  // the autotuned shapes (same shape for both passes)
  check<LOGN, 2, 12, 2, 12>(t, rng);
  check<LOGN, 3, 12, 3, 12>(t, rng);
  check<LOGN, 4, 12, 4, 12>(t, rng);
  check<LOGN, 2, 11, 2, 11>(t, rng);
  check<LOGN, 3, 11, 3, 11>(t, rng);
  // pass 2 on the fused inner-product kernel's 512-position tiles
  check<LOGN, 3, 11, 3, 9>(t, rng);
}

int main() {
  // 60-bit (integer path) and 40-50-bit (FP64 path) primes = 1 mod 2^17
  all_shapes<12>(18014398509309953ull);
  all_shapes<12>(1099511480321ull);
  all_shapes<12>(1099511390209ull);
  all_shapes<14>(1152921504606748673ull);
  all_shapes<14>(35184371138561ull);
  all_shapes<14>(35184368320513ull);
  all_shapes<16>(1152921504606584833ull);
  all_shapes<16>(1125899903827969ull);
  all_shapes<16>(1125899844714497ull);
  printf("ntt rounds: %d checks, %d with mismatches; FP64 max |value| / q = %.3f, non-integer values = %ld\n", g_cases,
         g_bad, g_max_ratio, g_non_integer);
  const bool ok = g_bad == 0 && g_non_integer == 0 && g_max_ratio <= 8.01;
  printf(ok ? "OK\n" : "FAIL\n");
  return ok ? 0 : 1;
}
