/*
 * CPU oracle for the RNS-CKKS hot path — TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously-correct integer routines used by tests, the smoke
 * check and the CPU-baseline leg of the benchmark to define what the GPU
 * library must compute bit-for-bit.  Nothing in the product path may load
 * this library.  It shares no code, header or table with the GPU library.
 *
 * The paper (FHEON, "Secure Neural Network Layers" and "Background: CKKS")
 * builds on RNS-CKKS over R = Z[X]/(X^N + 1) and does not spell out the ring
 * arithmetic; the definitions below are the standard RNS-CKKS ones, with the
 * conventions this project pins (documented per function).
 *
 * All modular products are computed with a 128-bit product and the C `%`
 * operator: no Barrett, Montgomery, Shoup or lazy reduction here.
 * Parallelism: OpenMP over independent limbs / coefficients only; the
 * arithmetic of every output element is the same as the serial loop.
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef unsigned __int128 u128;

/* ---------------------------------------------------------------- scalar */

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((u128)a * (u128)b) % q);
}
static uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) {
    return (uint64_t)(((u128)a + (u128)b) % q);
}
static uint64_t submod(uint64_t a, uint64_t b, uint64_t q) {
    /* a, b in [0, q) */
    return (uint64_t)(((u128)a + (u128)(q - b)) % q);
}

uint64_t or_powmod(uint64_t a, uint64_t e, uint64_t q) {
    uint64_t r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulmod(r, a, q);
        a = mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}

/* inverse modulo a prime q (Fermat) */
uint64_t or_invmod(uint64_t a, uint64_t q) { return or_powmod(a, q - 2, q); }

static size_t bitrev(size_t x, int logn) {
    size_t r = 0;
    for (int i = 0; i < logn; i++) { r = (r << 1) | (x & 1); x >>= 1; }
    return r;
}
static int ilog2(size_t n) { int l = 0; while (((size_t)1 << l) < n) l++; return l; }

/* ---------------------------------------------------------------- NTT
 * Negacyclic NTT convention (the boundary format):
 *   out[j] = sum_k a_k * psi^((2*brv(j)+1)*k)  mod q,
 * i.e. the evaluation of a(X) at the odd powers of psi, stored in
 * bit-reversed order; psi is a primitive 2N-th root of unity mod q.
 * The oracle computes it the textbook way:
 *   (1) twist b_k = a_k psi^k,
 *   (2) cyclic DFT B_t = sum_k b_k omega^(t k) with omega = psi^2, by the
 *       iterative radix-2 decimation-in-time algorithm (bit-reverse the
 *       input, then log2 N butterfly levels),
 *   (3) out[j] = B[brv(j)].
 * Because b(omega^t) = a(psi^(2t+1)), this equals the definition above.
 */
static void bitrev_permute(uint64_t* a, size_t n) {
    int logn = ilog2(n);
    for (size_t i = 0; i < n; i++) {
        size_t j = bitrev(i, logn);
        if (i < j) { uint64_t t = a[i]; a[i] = a[j]; a[j] = t; }
    }
}

static void cyclic_dft(uint64_t* a, size_t n, uint64_t omega, uint64_t q) {
    bitrev_permute(a, n);
    for (size_t len = 2; len <= n; len <<= 1) {
        uint64_t wlen = or_powmod(omega, n / len, q);
        for (size_t i = 0; i < n; i += len) {
            uint64_t w = 1;
            for (size_t j = 0; j < len / 2; j++) {
                uint64_t u = a[i + j];
                uint64_t v = mulmod(a[i + j + len / 2], w, q);
                a[i + j] = addmod(u, v, q);
                a[i + j + len / 2] = submod(u, v, q);
                w = mulmod(w, wlen, q);
            }
        }
    }
}

void or_ntt_fwd_limb(uint64_t* a, size_t n, uint64_t q, uint64_t psi) {
    uint64_t pk = 1;
    for (size_t k = 0; k < n; k++) { a[k] = mulmod(a[k] % q, pk, q); pk = mulmod(pk, psi, q); }
    cyclic_dft(a, n, mulmod(psi, psi, q), q);
    bitrev_permute(a, n);
}

/* Inverse of or_ntt_fwd_limb: undo (3), inverse DFT with omega^-1 and 1/N,
 * then untwist by psi^-k. */
void or_ntt_inv_limb(uint64_t* a, size_t n, uint64_t q, uint64_t psi) {
    bitrev_permute(a, n);
    uint64_t psi_inv = or_invmod(psi, q);
    cyclic_dft(a, n, mulmod(psi_inv, psi_inv, q), q);
    uint64_t n_inv = or_invmod((uint64_t)(n % q), q);
    uint64_t pk = 1;
    for (size_t k = 0; k < n; k++) {
        a[k] = mulmod(mulmod(a[k], n_inv, q), pk, q);
        pk = mulmod(pk, psi_inv, q);
    }
}

/* a: [nlimbs][n], limb i modulo qs[i] with root psis[i]. */
void or_ntt(uint64_t* a, int nlimbs, size_t n, const uint64_t* qs, const uint64_t* psis, int inverse) {
    #pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < nlimbs; i++) {
        if (inverse) or_ntt_inv_limb(a + (size_t)i * n, n, qs[i], psis[i]);
        else         or_ntt_fwd_limb(a + (size_t)i * n, n, qs[i], psis[i]);
    }
}

/* ---------------------------------------------------------------- pointwise
 * Elementwise ring operations on [nlimbs][n] arrays, limb i modulo qs[i].
 * Inputs must already be reduced into [0, q_i). */
void or_mul(const uint64_t* a, const uint64_t* b, uint64_t* out, int nlimbs, size_t n, const uint64_t* qs) {
    #pragma omp parallel for
    for (int i = 0; i < nlimbs; i++)
        for (size_t k = 0; k < n; k++)
            out[(size_t)i * n + k] = mulmod(a[(size_t)i * n + k], b[(size_t)i * n + k], qs[i]);
}
void or_add(const uint64_t* a, const uint64_t* b, uint64_t* out, int nlimbs, size_t n, const uint64_t* qs) {
    #pragma omp parallel for
    for (int i = 0; i < nlimbs; i++)
        for (size_t k = 0; k < n; k++)
            out[(size_t)i * n + k] = addmod(a[(size_t)i * n + k], b[(size_t)i * n + k], qs[i]);
}
void or_sub(const uint64_t* a, const uint64_t* b, uint64_t* out, int nlimbs, size_t n, const uint64_t* qs) {
    #pragma omp parallel for
    for (int i = 0; i < nlimbs; i++)
        for (size_t k = 0; k < n; k++)
            out[(size_t)i * n + k] = submod(a[(size_t)i * n + k], b[(size_t)i * n + k], qs[i]);
}
/* out = a * c_i (a scalar per limb) */
void or_mul_scalar(const uint64_t* a, const uint64_t* c, uint64_t* out, int nlimbs, size_t n, const uint64_t* qs) {
    #pragma omp parallel for
    for (int i = 0; i < nlimbs; i++)
        for (size_t k = 0; k < n; k++)
            out[(size_t)i * n + k] = mulmod(a[(size_t)i * n + k], c[i] % qs[i], qs[i]);
}
/* out[i][k] = a[k] mod q_i for an array of arbitrary u64 values a (one row) */
void or_reduce_row(const uint64_t* a, uint64_t* out, int nlimbs, size_t n, const uint64_t* qs) {
    #pragma omp parallel for
    for (int i = 0; i < nlimbs; i++)
        for (size_t k = 0; k < n; k++)
            out[(size_t)i * n + k] = a[k] % qs[i];
}
/* Signed small integers (secret, errors) into RNS: out[i][k] = s[k] mod q_i. */
void or_from_signed(const int64_t* s, uint64_t* out, int nlimbs, size_t n, const uint64_t* qs) {
    #pragma omp parallel for
    for (int i = 0; i < nlimbs; i++)
        for (size_t k = 0; k < n; k++) {
            int64_t v = s[k];
            uint64_t q = qs[i];
            uint64_t r = v >= 0 ? ((uint64_t)v) % q : (q - (((uint64_t)(-(v + 1)) + 1) % q)) % q;
            out[(size_t)i * n + k] = r;
        }
}

/* ---------------------------------------------------------------- basis conversion
 * Fast (floor-type, non-centred) basis conversion from a basis
 * {qin_0..qin_{a-1}} with product Qin to a basis {qout_0..}:
 *   t_i   = [x_i * (Qin/qin_i)^{-1}]_{qin_i}              in [0, qin_i)
 *   y_p   = sum_i t_i * [(Qin/qin_i)]_{qout_p}   mod qout_p
 * so that y = x + u*Qin with 0 <= u < a (as integers).
 * qhat_inv[i] = (Qin/qin_i)^{-1} mod qin_i;  qhat[i*nout + p] = (Qin/qin_i) mod qout_p.
 * x: [nin][n] (coefficient form), y: [nout][n].
 */
void or_bconv(const uint64_t* x, int nin, const uint64_t* qin, const uint64_t* qhat_inv,
              uint64_t* y, int nout, const uint64_t* qout, const uint64_t* qhat, size_t n) {
    #pragma omp parallel for
    for (long long kk = 0; kk < (long long)n; kk++) {
        size_t k = (size_t)kk;
        uint64_t t[64];
        for (int i = 0; i < nin; i++) t[i] = mulmod(x[(size_t)i * n + k], qhat_inv[i], qin[i]);
        for (int p = 0; p < nout; p++) {
            uint64_t acc = 0;
            for (int i = 0; i < nin; i++)
                acc = addmod(acc, mulmod(t[i] % qout[p], qhat[(size_t)i * nout + p], qout[p]), qout[p]);
            y[(size_t)p * n + k] = acc;
        }
    }
}

/* ---------------------------------------------------------------- automorphism
 * phi_g(a)(X) = a(X^g), g odd.  In coefficient form, coefficient k moves to
 * g*k mod 2N and is negated when that index is >= N (X^N = -1).
 */
void or_automorph_coeff(const uint64_t* in, uint64_t* out, int nlimbs, size_t n, const uint64_t* qs, uint64_t g) {
    #pragma omp parallel for
    for (int i = 0; i < nlimbs; i++) {
        for (size_t k = 0; k < n; k++) {
            uint64_t e = (uint64_t)(((u128)g * k) % (2 * n));
            uint64_t v = in[(size_t)i * n + k];
            if (e < n) out[(size_t)i * n + e] = v;
            else out[(size_t)i * n + (e - n)] = (v == 0) ? 0 : qs[i] - v;
        }
    }
}

/* In NTT form (bit-reversed evaluation order), phi_g is the index map
 *   out[j] = in[ brv( ((g * (2 brv(j) + 1)) mod 2N - 1) / 2 ) ],
 * because slot j holds a(psi^(2 brv(j)+1)) and phi_g(a) evaluated there is
 * a(psi^(g (2 brv(j)+1))).  perm[j] receives the source index. */
void or_automorph_perm(size_t n, uint64_t g, int64_t* perm) {
    int logn = ilog2(n);
    for (size_t j = 0; j < n; j++) {
        uint64_t e = (uint64_t)(((u128)g * (2 * bitrev(j, logn) + 1)) % (2 * n));
        perm[j] = (int64_t)bitrev((size_t)((e - 1) / 2), logn);
    }
}

/* ---------------------------------------------------------------- sampling
 * SplitMix64 (Steele, Lea, Flood 2014) seeds xoshiro256** (Blackman & Vigna
 * 2018).  One generator per (seed, stream) pair: state words are four
 * consecutive SplitMix64 outputs started from seed ^ stream.
 */
typedef struct { uint64_t s[4]; } xoshiro;

static uint64_t splitmix64(uint64_t* x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static void xo_seed(xoshiro* g, uint64_t seed, uint64_t stream) {
    uint64_t x = seed ^ stream;
    for (int i = 0; i < 4; i++) g->s[i] = splitmix64(&x);
}
static uint64_t xo_next(xoshiro* g) {
    uint64_t* s = g->s;
    uint64_t result = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl(s[3], 45);
    return result;
}
/* uniform in [0, q) by rejection of the top partial block */
static uint64_t xo_uniform(xoshiro* g, uint64_t q) {
    uint64_t lim = (UINT64_MAX / q) * q;
    for (;;) { uint64_t x = xo_next(g); if (x < lim) return x % q; }
}
uint64_t or_rng_first(uint64_t seed, uint64_t stream) { xoshiro g; xo_seed(&g, seed, stream); return xo_next(&g); }

/* out[i][k] uniform in [0, q_i); limb i uses sub-stream (stream, i). */
void or_sample_uniform(uint64_t seed, uint64_t stream, const uint64_t* qs, int nlimbs, size_t n, uint64_t* out) {
    #pragma omp parallel for
    for (int i = 0; i < nlimbs; i++) {
        xoshiro g;
        xo_seed(&g, seed, stream * 1000003ull + (uint64_t)i);
        for (size_t k = 0; k < n; k++) out[(size_t)i * n + k] = xo_uniform(&g, qs[i]);
    }
}
/* uniform ternary {-1, 0, 1}: x mod 3 - 1 with rejection of x >= 3 floor(2^64/3) */
void or_sample_ternary(uint64_t seed, uint64_t stream, size_t n, int64_t* out) {
    xoshiro g; xo_seed(&g, seed, stream);
    uint64_t lim = (UINT64_MAX / 3) * 3;
    for (size_t k = 0; k < n; k++) {
        uint64_t x;
        do { x = xo_next(&g); } while (x >= lim);
        out[k] = (int64_t)(x % 3) - 1;
    }
}
/* Rounded continuous Gaussian (Box-Muller, cosine branch), rejected if |e| > bound. */
void or_sample_gaussian(uint64_t seed, uint64_t stream, size_t n, double sigma, int64_t bound, int64_t* out) {
    xoshiro g; xo_seed(&g, seed, stream);
    const double two_pi = 6.283185307179586476925286766559;
    for (size_t k = 0; k < n; k++) {
        for (;;) {
            double u1 = ((double)(xo_next(&g) >> 11) + 1.0) * (1.0 / 9007199254740992.0); /* (0,1] */
            double u2 = (double)(xo_next(&g) >> 11) * (1.0 / 9007199254740992.0);        /* [0,1) */
            double z = sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
            int64_t e = llround(sigma * z);
            if (e <= bound && e >= -bound) { out[k] = e; break; }
        }
    }
}

/* ---------------------------------------------------------------- misc */
/* Deterministic Miller-Rabin for 64-bit n with the first 12 prime bases. */
int or_is_prime(uint64_t n) {
    if (n < 2) return 0;
    static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (int i = 0; i < 12; i++) { if (n == bases[i]) return 1; if (n % bases[i] == 0) return 0; }
    uint64_t d = n - 1; int s = 0;
    while ((d & 1) == 0) { d >>= 1; s++; }
    for (int i = 0; i < 12; i++) {
        uint64_t x = or_powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int comp = 1;
        for (int r = 1; r < s; r++) { x = mulmod(x, x, n); if (x == n - 1) { comp = 0; break; } }
        if (comp) return 0;
    }
    return 1;
}
