// Negacyclic NTT over Z_q[X]/(X^N+1), N = 2^LOGN, in two LDS passes.
//
// Convention (the library's data format): a limb in NTT form stores at index j
// the value a(psi^(2 brv(j) + 1)), psi the minimum primitive 2N-th root of
// unity mod q.  The forward transform is the merged-twist Cooley-Tukey
// recursion on natural-order input (stage s: 2^s blocks, butterfly distance
// N / 2^(s+1), twiddle Psi[2^s + block] with Psi[k] = psi^brv(k)); the inverse
// is the matching Gentleman-Sande recursion with Psi^{-1} and a final N^{-1}.
//
// MI355X mapping: one limb (up to 512 KiB) does not fit in LDS, so the
// LOGN stages are split as L1 + L2.  Pass 1 runs stages 0..L1-1: these only
// couple elements whose index differs by a multiple of N2 = 2^L2, i.e. the
// N2 "columns" {c + k N2} are independent size-2^L1 transforms sharing the
// twiddles Psi[2^s + block].  Pass 2 runs stages L1..LOGN-1 inside contiguous
// "chunks" of N2 elements, chunk b using Psi[2^(L1+s) + b 2^s + block].
// A workgroup stages TILE (2048 or 4096) elements (several columns / chunks) in LDS; each
// thread keeps a radix-2^r butterfly group (r <= 4 stages) in registers per
// LDS round, so a pass costs one HBM read + write and ceil(L/4) LDS rounds.
//
// Everything here is __host__ __device__ so a workgroup can be emulated on the
// CPU (round by round) with exactly the kernel's index arithmetic.
#pragma once
#include "modarith.h"

namespace he {

template <int LOGN, int PASS, bool INV, int LOG_EPT = 4, int LOG_TILE = 12>
struct NttPass {
  static constexpr int N = 1 << LOGN;
  static constexpr int PASS_NO = PASS;
  static constexpr int L1 = (LOGN + 1) / 2;
  static constexpr int L2 = LOGN - L1;
  static constexpr int N2 = 1 << L2;
  static constexpr int LM = PASS == 1 ? L1 : L2;  // stages in this pass
  static constexpr int M = 1 << LM;               // sub-transform size
  static constexpr int TILE = LOGN < LOG_TILE ? N : (1 << LOG_TILE);  // elements per workgroup
  static constexpr int G = TILE / M;              // sub-transforms per workgroup
  static constexpr int WG_PER_LIMB = N / TILE;
  // each thread keeps 2^LOG_EPT elements (one radix-2^LOG_EPT group) per round
  static constexpr int THREADS = TILE >> LOG_EPT;
  // pass-2 chunks get one pad word per 16 so that the stride-16 accesses of
  // the last round fall in different LDS banks
  static constexpr int CHUNK_WORDS = M + (M >> 4);
  static constexpr int LDS_WORDS = PASS == 1 ? TILE : G * CHUNK_WORDS;

  // global element index of (workgroup tile wg, sub-transform g, local index k)
  HE_HD static int gidx(int wg, int g, int k) {
    if (PASS == 1) return k * N2 + wg * G + g;
    return (wg * G + g) * M + k;
  }
  HE_HD static int lidx(int g, int k) {
    if (PASS == 1) return k * G + g;
    return g * CHUNK_WORDS + k + (k >> 4);
  }
  // tile element e <-> (g, k) for the coalesced HBM <-> LDS copy
  HE_HD static void tile_elem(int e, int& g, int& k) {
    if (PASS == 1) { g = e % G; k = e / G; }
    else { g = e / M; k = e % M; }
  }

  // One LDS round of R stages starting at local stage s0, for thread tid.
  // R is a compile-time constant so the butterfly group stays in registers.
  template <int R>
  HE_HD static void round(uint64_t* lds, int tid, int wg, int s0, const uint64_t* tw,
                          const uint64_t* twp, uint64_t q) {
    constexpr int GPS = M >> R;  // groups per sub-transform
    constexpr int TOTAL = G * GPS;
    const int dmin = M >> (s0 + R);
    const int span = M >> s0;
    for (int gid = tid; gid < TOTAL; gid += THREADS) {
      int g, gg;
      if (PASS == 1) { g = gid % G; gg = gid / G; }
      else { g = gid / GPS; gg = gid % GPS; }
      const int lo = gg % dmin, hi = gg / dmin;
      const int base = hi * span + lo;
      uint64_t x[1 << R];
#pragma unroll
      for (int u = 0; u < (1 << R); u++) x[u] = lds[lidx(g, base + u * dmin)];
      const int sub_off = PASS == 2 ? (wg * G + g) : 0;
      if (!INV) {
#pragma unroll
        for (int ss = 0; ss < R; ss++) {
          const int s = s0 + ss;
          const int sg = (PASS == 2 ? L1 : 0) + s;
          const int half = 1 << (R - 1 - ss);
#pragma unroll
          for (int u = 0; u < (1 << R); u++) {
            if (u & half) continue;
            const int iloc = (hi << ss) + (u >> (R - ss));
            const int ti = (1 << sg) + (sub_off << s) + iloc;
            // Harvey butterfly: inputs in [0, 4q), outputs in [0, 4q)
            const uint64_t y = mul_shoup_lazy(x[u + half], tw[ti], twp[ti], q);
            uint64_t a = x[u];
            a = a >= 2 * q ? a - 2 * q : a;
            x[u] = a + y;
            x[u + half] = a - y + 2 * q;
          }
        }
      } else {
#pragma unroll
        for (int ss = R - 1; ss >= 0; ss--) {
          const int s = s0 + ss;
          const int sg = (PASS == 2 ? L1 : 0) + s;
          const int half = 1 << (R - 1 - ss);
#pragma unroll
          for (int u = 0; u < (1 << R); u++) {
            if (u & half) continue;
            const int iloc = (hi << ss) + (u >> (R - ss));
            const int ti = (1 << sg) + (sub_off << s) + iloc;
            // Gentleman-Sande with lazy reduction: inputs and outputs in [0, 2q)
            const uint64_t a = x[u], b = x[u + half];
            const uint64_t sm = a + b;
            x[u] = sm >= 2 * q ? sm - 2 * q : sm;
            x[u + half] = mul_shoup_lazy(a - b + 2 * q, tw[ti], twp[ti], q);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < (1 << R); u++) lds[lidx(g, base + u * dmin)] = x[u];
    }
  }

  // FP64 round for q < 2^50: the same butterflies in centred arithmetic
  // (mul_f64_c, full-rate FP64 FMA instead of 32-bit integer multiplies).
  // Each round starts by re-centring its inputs to |x| <= q/2 + 1; over at
  // most four stages the forward butterflies (a + y, a - y) stay below 4.25q
  // and the inverse ones (a + b, (a - b) w) below 8q + 16, so everything is
  // exact.
  //
  // FACT (pass 2 only): the twiddle of chunk b, stage s, index i is built from
  // two entries of the same table instead of being read from its own slot.
  // The three parts of the table index 2^(L1+s) + b 2^s + i occupy disjoint
  // bits, so its bit reversal (the exponent of psi) is the sum of those of
  // 2^(L1+s) + i and b 2^s:  Psi[2^(L1+s) + b 2^s + i] =
  // Psi[2^(L1+s) + i] Psi[b 2^s] mod q.  The first factor lies in the 2^L2
  // entries shared by every chunk, the second is one entry per chunk and
  // stage, so a pass reads a few KiB of table per modulus instead of N
  // entries.  The product w = mul_f64_c(., .) has |w| <= 3q/4 and
  // wq = fl(w fl(1/q)) is within 2^-52 (relatively) of w / q; the quotient
  // estimate of a product by w is then off by at most 1.125 |a| 2^-52, which
  // is what the bounds above allow for.
  template <int R, bool FACT = false>
  HE_HD static void round_f64(double* lds, int tid, int wg, int s0, const double* tw, const double* twq, double q,
                              double qinv) {
    static_assert(R <= 4, "the centred bounds assume at most four stages per round");
    static_assert(!FACT || PASS == 2, "factored twiddles are for pass 2");
    constexpr int GPS = M >> R;
    constexpr int TOTAL = G * GPS;
    const int dmin = M >> (s0 + R);
    const int span = M >> s0;
    for (int gid = tid; gid < TOTAL; gid += THREADS) {
      int g, gg;
      if (PASS == 1) { g = gid % G; gg = gid / G; }
      else { g = gid / GPS; gg = gid % GPS; }
      const int lo = gg % dmin, hi = gg / dmin;
      const int base = hi * span + lo;
      double x[1 << R];
#pragma unroll
      for (int u = 0; u < (1 << R); u++) x[u] = centre_f64(lds[lidx(g, base + u * dmin)], qinv, q);
      const int sub_off = PASS == 2 ? (wg * G + g) : 0;
      if (!INV) {
#pragma unroll
        for (int ss = 0; ss < R; ss++) {
          const int s = s0 + ss;
          const int sg = (PASS == 2 ? L1 : 0) + s;
          const int half = 1 << (R - 1 - ss);
#pragma unroll
          for (int u = 0; u < (1 << R); u++) {
            if (u & half) continue;
            const int iloc = (hi << ss) + (u >> (R - ss));
            double w, wq;
            twiddle_f64<FACT>(tw, twq, sg, s, sub_off, iloc, q, qinv, w, wq);
            const double y = mul_f64_c(x[u + half], w, wq, q);
            const double a = x[u];
            x[u] = a + y;
            x[u + half] = a - y;
          }
        }
      } else {
#pragma unroll
        for (int ss = R - 1; ss >= 0; ss--) {
          const int s = s0 + ss;
          const int sg = (PASS == 2 ? L1 : 0) + s;
          const int half = 1 << (R - 1 - ss);
#pragma unroll
          for (int u = 0; u < (1 << R); u++) {
            if (u & half) continue;
            const int iloc = (hi << ss) + (u >> (R - ss));
            double w, wq;
            twiddle_f64<FACT>(tw, twq, sg, s, sub_off, iloc, q, qinv, w, wq);
            const double a = x[u], b = x[u + half];
            x[u] = a + b;
            x[u + half] = mul_f64_c(a - b, w, wq, q);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < (1 << R); u++) lds[lidx(g, base + u * dmin)] = x[u];
    }
  }

  // twiddle of global stage sg (local stage s), sub-transform sub_off, index
  // iloc: the table entry, or (FACT) the product of its two factors
  template <bool FACT>
  HE_HD static void twiddle_f64(const double* tw, const double* twq, int sg, int s, int sub_off, int iloc, double q,
                                double qinv, double& w, double& wq) {
    if constexpr (FACT) {
      const int fi = sub_off << s;
      w = mul_f64_c(tw[(1 << sg) + iloc], tw[fi], twq[fi], q);
      wq = w * qinv;
    } else {
      const int ti = (1 << sg) + (sub_off << s) + iloc;
      w = tw[ti];
      wq = twq[ti];
    }
  }

  // FP64 path between the passes: the intermediate (written by forward pass 1
  // and inverse pass 2, read only by the other pass of the same transform)
  // is kept as raw double bits; the transform's own input and output are
  // canonical residues (< 2^50), converted exactly through the mantissa.
  static constexpr bool IN_RAW = (!INV && PASS == 2) || (INV && PASS == 1);
  HE_HD static double load_f64(uint64_t w) { return IN_RAW ? bits_to_f64(w) : u52_to_f64(w); }
  // the forward transform canonicalises after pass 2, the inverse multiplies
  // by N^{-1} and canonicalises after pass 1
  HE_HD static uint64_t finish_f64(double v, double ninv, double ninvq, double q, double qinv) {
    if (!INV && PASS == 2) return f64_to_u52(canon_f64(v, qinv, q));
    if (INV && PASS == 1) return f64_to_u52(canon_f64(mul_f64_c(v, ninv, ninvq, q), qinv, q));
    return f64_to_bits(v);
  }

  // Value written back to HBM after the pass: the forward transform leaves
  // pass 1 lazily reduced ([0, 4q)) and canonicalises after pass 2; the
  // inverse multiplies by N^{-1} and canonicalises after pass 1.
  HE_HD static uint64_t finish(uint64_t v, uint64_t ninv, uint64_t ninvp, uint64_t q) {
    if (!INV && PASS == 2) {
      v = v >= 2 * q ? v - 2 * q : v;
      return v >= q ? v - q : v;
    }
    if (INV && PASS == 1) {
      v = mul_shoup_lazy(v, ninv, ninvp, q);
      return v >= q ? v - q : v;
    }
    return v;
  }

  // rounds of LOG_EPT stages (the last one may be shorter)
  static constexpr int NR = (LM + LOG_EPT - 1) / LOG_EPT;
  static constexpr int rbits(int idx) { return idx < NR - 1 ? LOG_EPT : LM - LOG_EPT * (NR - 1); }
  static constexpr int rstart(int idx) { return idx * LOG_EPT; }
  static_assert(NR <= 4, "at most four LDS rounds per pass");
};

}  // namespace he
