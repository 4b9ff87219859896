"""Pins for the oracle's ring arithmetic (CPU only).

Each test checks the oracle against something other than itself: the
definition evaluated by brute force with Python integers on tiny rings, the
convolution theorem, exact CRT/floor identities, or number-theoretic
invariants.  A dropped term, a wrong sign or a transposed index anywhere in
NTT / automorphism / basis conversion / rescale / ModDown fails one of them.
"""
import math
import random

import numpy as np
import pytest

from oracle import _lib as C
from oracle import ckks
from tests import t0_bigint as B

TINY = [
    # (log_n, q_bits, p_bits, alpha)
    (3, [28, 24, 24], [30], 1),
    (4, [30, 26, 26, 26], [31, 31], 2),
    (5, [30, 25, 25], [30], 1),
    (6, [31, 27, 27, 27], [31, 31], 2),
]


def tiny_params(i):
    log_n, qb, pb, alpha = TINY[i]
    return ckks.Params(log_n, qb, pb, alpha, 20)


def rand_poly(rng, n, q):
    return [rng.randrange(q) for _ in range(n)]


# ------------------------------------------------------------------ primes
@pytest.mark.parametrize("name", ["config0", "config1", "config2"])
def test_prime_rule_invariants(name):
    cfg = ckks.CONFIGS[name]
    pr = ckks.Params(**cfg)
    two_n = 2 * pr.n
    bits = cfg["q_bits"] + cfg["p_bits"]
    assert len(set(pr.moduli)) == len(pr.moduli)
    for q, b in zip(pr.moduli, bits):
        assert B.is_prime(q)
        assert q % two_n == 1
        assert q.bit_length() == b
    # each prime is the largest of its size not taken by an earlier allocation
    taken = set()
    for q, b in zip(pr.moduli, bits):
        cand = q + two_n
        while cand < (1 << b):
            assert cand in taken or not B.is_prime(cand), (q, cand)
            cand += two_n
        taken.add(q)


def test_config_prime_values():
    """The first primes of each configuration (regression of the rule)."""
    p0 = ckks.Params(**ckks.CONFIGS["config0"])
    assert p0.q[:2] == [18014398509309953, 1099511480321] and p0.p == [36028797018652673]
    p1 = ckks.Params(**ckks.CONFIGS["config1"])
    assert p1.q[:2] == [1152921504606748673, 35184371138561] and p1.p[0] == 1152921504606683137


@pytest.mark.parametrize("i", range(len(TINY)))
def test_min_root_is_minimum_primitive(i):
    pr = tiny_params(i)
    for q, psi in zip(pr.moduli, pr.psi):
        assert pow(psi, pr.n, q) == q - 1
        roots = [r for r in range(2, q) if pow(r, 2 * pr.n, q) == 1 and pow(r, pr.n, q) == q - 1] \
            if q < 5000 else None
        # brute force over the odd powers of psi (all primitive 2N-th roots)
        allroots = sorted(pow(psi, 2 * t + 1, q) for t in range(pr.n))
        assert allroots[0] == psi
        if roots is not None:
            assert min(roots) == psi


# ------------------------------------------------------------------ NTT
@pytest.mark.parametrize("i", range(len(TINY)))
def test_ntt_matches_definition(i):
    pr = tiny_params(i)
    rng = random.Random(100 + i)
    a = np.array([rand_poly(rng, pr.n, q) for q in pr.moduli], dtype=np.uint64)
    got = C.ntt(a, pr.moduli, pr.psi)
    for li, (q, psi) in enumerate(zip(pr.moduli, pr.psi)):
        want = B.ntt_definition([int(x) for x in a[li]], q, psi)
        assert [int(x) for x in got[li]] == want


@pytest.mark.parametrize("i", range(len(TINY)))
def test_ntt_convolution_theorem(i):
    pr = tiny_params(i)
    rng = random.Random(200 + i)
    for q, psi in zip(pr.moduli, pr.psi):
        a, b = rand_poly(rng, pr.n, q), rand_poly(rng, pr.n, q)
        c = B.negacyclic_mul(a, b, q)
        A = C.ntt(np.array([a], dtype=np.uint64), [q], [psi])
        Bn = C.ntt(np.array([b], dtype=np.uint64), [q], [psi])
        Cn = C.ntt(np.array([c], dtype=np.uint64), [q], [psi])
        assert np.array_equal(C.mul(A, Bn, [q]), Cn)


def test_ntt_convolution_theorem_real_prime():
    """Same identity with a 60-bit production prime at N = 256."""
    pr = ckks.Params(**ckks.CONFIGS["config1"])
    n = 256
    q = pr.q[0]
    psi = ckks.min_root(q, n)
    rng = random.Random(7)
    a, b = rand_poly(rng, n, q), rand_poly(rng, n, q)
    c = B.negacyclic_mul(a, b, q)
    A = C.ntt(np.array([a], dtype=np.uint64), [q], [psi])
    Bn = C.ntt(np.array([b], dtype=np.uint64), [q], [psi])
    assert [int(x) for x in C.mul(A, Bn, [q])[0]] == [int(x) for x in C.ntt(np.array([c], dtype=np.uint64), [q], [psi])[0]]


@pytest.mark.parametrize("name", ["config0", "config1", "config2"])
def test_ntt_roundtrip_production(name):
    pr = ckks.Params(**ckks.CONFIGS[name])
    rng = np.random.default_rng(5)
    nl = min(4, len(pr.moduli))
    mods = pr.moduli[-nl:]
    psis = pr.psi[-nl:]
    a = np.stack([rng.integers(0, q, pr.n, dtype=np.uint64) for q in mods])
    f = C.ntt(a, mods, psis)
    assert not np.array_equal(f, a)
    assert np.array_equal(C.ntt(f, mods, psis, inverse=True), a)


# ------------------------------------------------------------------ automorphism
@pytest.mark.parametrize("i", range(len(TINY)))
def test_automorphism_ntt_index_map(i):
    pr = tiny_params(i)
    ctx = ckks.Context(pr)
    rng = random.Random(300 + i)
    for r in [1, -1, 2, 3, pr.n // 2 - 1]:
        g = ctx.galois_element(r)
        for q, psi in zip(pr.moduli[:2], pr.psi[:2]):
            a = rand_poly(rng, pr.n, q)
            want = B.automorph(a, g, q)
            A = C.ntt(np.array([a], dtype=np.uint64), [q], [psi])
            got = C.ntt(A[:, ctx.perm(g)], [q], [psi], inverse=True)
            assert [int(x) for x in got[0]] == want
            # the coefficient-form routine agrees as well
            assert [int(x) for x in C.automorph_coeff(np.array([a], dtype=np.uint64), [q], g)[0]] == want


def test_galois_elements():
    pr = tiny_params(1)
    ctx = ckks.Context(pr)
    n = pr.n
    assert ctx.galois_element(0) == 1
    assert ctx.galois_element(1) == 5
    assert ctx.galois_element(-1) == pow(5, n // 2 - 1, 2 * n)
    assert ctx.galois_element(1) * ctx.galois_element(-1) % (2 * n) == 1


# ------------------------------------------------------------------ basis conversion
@pytest.mark.parametrize("name,level", [("config1", 8), ("config2", 24), ("config2", 13), ("config0", 3)])
def test_bconv_floor_identity(name, level):
    """y = x + u*Q_j with 0 <= u < alpha for every digit (exact big integers)."""
    pr = ckks.Params(**ckks.CONFIGS[name])
    ctx = ckks.Context(pr)
    rng = random.Random(11)
    n = 8
    for j in range(pr.dnum(level)):
        idx, outs, qin, qout, qhat_inv, qhat = ctx.modup_consts(j, level)
        x = np.array([[rng.randrange(q) for _ in range(n)] for q in qin], dtype=np.uint64)
        y = C.bconv(x, qin, qhat_inv, qout, qhat)
        Qj = math.prod(qin)
        for k in range(n):
            X, _ = B.crt([int(x[i, k]) for i in range(len(qin))], qin)
            us = set()
            for p, po in enumerate(qout):
                u = (int(y[p, k]) - X) * pow(Qj % po, -1, po) % po
                us.add(u)
            assert len(us) == 1
            assert us.pop() < len(qin)


# ------------------------------------------------------------------ rescale / moddown
def _coeff_ints(ctx, poly, moduli, psis):
    co = C.ntt(poly, moduli, psis, inverse=True)
    return [B.crt([int(co[i, k]) for i in range(len(moduli))], moduli)[0] for k in range(ctx.n)]


@pytest.mark.parametrize("i", [1, 3])
def test_rescale_is_floor(i):
    pr = tiny_params(i)
    ctx = ckks.Context(pr)
    rng = np.random.default_rng(i)
    level = pr.L
    data = np.stack([np.stack([rng.integers(0, q, pr.n, dtype=np.uint64) for q in pr.q]) for _ in range(2)])
    ct = ckks.Ciphertext(data, 2.0 ** 40)
    out = ctx.rescale(ct)
    qt = pr.q[level - 1]
    assert out.scale == 2.0 ** 40 / float(qt)
    for k in range(2):
        before = _coeff_ints(ctx, data[k], pr.q, pr.psi[:level])
        after = _coeff_ints(ctx, out.data[k], pr.q[:-1], pr.psi[: level - 1])
        assert after == [c // qt for c in before]


@pytest.mark.parametrize("i", [1, 3])
def test_moddown_is_floor_minus_small(i):
    """ModDown(U) = floor(U / P) - v with 0 <= v < K (mod Q), for U over Q u P."""
    pr = tiny_params(i)
    ctx = ckks.Context(pr)
    rng = np.random.default_rng(10 + i)
    level = pr.L
    mods = ctx.ext_moduli(level)
    psis = ctx.ext_psis(level)
    u = np.stack([rng.integers(0, q, pr.n, dtype=np.uint64) for q in mods])
    out = ctx.moddown(u, level)
    U = _coeff_ints(ctx, u, mods, psis)
    O = _coeff_ints(ctx, out, pr.q, pr.psi[:level])
    Q = math.prod(pr.q)
    for Uk, Ok in zip(U, O):
        v = (Uk // pr.P - Ok) % Q
        assert 0 <= v < pr.K


# ------------------------------------------------------------------ sampling
def test_samplers_statistics_and_determinism():
    s = C.sample_ternary(42, 1, 1 << 16)
    assert set(np.unique(s).tolist()) == {-1, 0, 1}
    counts = np.bincount(s + 1)
    assert np.all(np.abs(counts / s.size - 1 / 3) < 0.01)
    e = C.sample_gaussian(42, 3, 1 << 16)
    assert abs(e.std() - 3.2) < 0.05 and abs(e.mean()) < 0.05 and np.abs(e).max() <= 19
    assert np.array_equal(e, C.sample_gaussian(42, 3, 1 << 16))
    assert not np.array_equal(e, C.sample_gaussian(43, 3, 1 << 16))
    q = [1099511480321, 18014398509309953]
    u = C.sample_uniform(1, 2, q, 1 << 14)
    assert u[0].max() < q[0] and u[1].max() < q[1]
    assert abs(u[1].astype(np.float64).mean() / q[1] - 0.5) < 0.01


def test_xoshiro_reference_value():
    """xoshiro256** seeded by SplitMix64 from 0: first output of the published
    generators (SplitMix64 sequence from state 0 begins 0xE220A8397B1DCDAF)."""
    # state words are SplitMix64 outputs from x=0; reproduce with Python ints
    M = (1 << 64) - 1

    def sm(x):
        x = (x + 0x9E3779B97F4A7C15) & M
        z = x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        return x, z ^ (z >> 31)

    x, s0 = sm(0)
    assert s0 == 0xE220A8397B1DCDAF
    x, s1 = sm(x)
    rot = lambda v, k: ((v << k) | (v >> (64 - k))) & M
    want = (rot((s1 * 5) & M, 7) * 9) & M
    assert C.lib().or_rng_first(0, 0) == want
