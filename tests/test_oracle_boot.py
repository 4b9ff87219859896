"""Pins for the oracle's bootstrapping (CPU only).

ModRaise against Python big integers; the butterfly factors of the slot
decoding map against the decoding sums evaluated directly and against the
oracle's FFT decoder; the baby-step giant-step evaluation against dense
diagonal sums in a complex slot simulation; the conjugation and monomial
steps by decryption; the EvalMod interpolant against the sine; the whole
procedure by decryption at N = 2^12.
"""
import cmath
import functools
import math

import numpy as np
import pytest

from oracle import _lib as C
from oracle import boot as BT
from oracle import ckks
from oracle import layers as LY
from tests import t0_bigint as B

# bootstrapping ring used by the tests: N = 2^12, q_0 60 bits + 16 x 50 bits,
# 7 special primes of 50 bits, dnum = 3, base scale 2^50
BOOT_PARAMS = dict(log_n=12, q_bits=[60] + [50] * 16, p_bits=[50] * 7, alpha=6, log_scale=50)
BOOT_HAMMING = 32
BOOT_KMIN = 12.0
BOOT_DEGREE = 159
BOOT_LEVELS = 3
# the double-angle EvalMod: cosine of degree 39, three double angles
BOOT_DA = (39, 3)
# decrypted error bound of a refreshed ciphertext: the coefficient-to-slot
# output x = t / (2^e delta) carries about 2^-36 relative error (plaintext
# rounding at 45-bit integers over ~31 diagonals); EvalMod multiplies it by
# 2 pi K / (2 pi) = K ~ 16 against m / q_0 ~ 2^-16, i.e. ~2^-16 relative on
# the coefficients; slot values in [-1, 1] then carry ~1e-5.  Bound 2^-13.
BOOT_TOL = 2.0 ** -13


@functools.lru_cache(maxsize=None)
def boot_setup(double_angles=0):
    pr = ckks.Params(**BOOT_PARAMS)
    ctx = ckks.Context(pr)
    sk, pk = ctx.keygen(7, hamming=BOOT_HAMMING)
    degree = BOOT_DA[0] if double_angles else BOOT_DEGREE
    plan = BT.BootPlan(pr.log_n, BOOT_LEVELS, BOOT_KMIN, pr.scale, degree, double_angles)
    keys = {r: ctx.gen_rotation_key(sk, r, 7) for r in plan.rotations()}
    keys[ckks.CONJ] = ctx.gen_rotation_key(sk, ckks.CONJ, 7)
    rk = ctx.gen_relin_key(sk, 7)
    cts, stc = BT.boot_plaintexts(ctx, plan, pr.L)
    return ctx, sk, pk, plan, keys, rk, cts, stc


def bitrev_perm(n):
    b = n.bit_length() - 1
    return np.array([int(format(i, "0%db" % b)[::-1], 2) if b else 0 for i in range(n)])


def apply_diags(d, x):
    return sum(v * np.roll(x, -s) for s, v in d.items())


# ------------------------------------------------------------------ secret
def test_sparse_secret_weight_and_values():
    pr = ckks.Params(**BOOT_PARAMS)
    ctx = ckks.Context(pr)
    sk, _ = ctx.keygen(3, hamming=BOOT_HAMMING)
    assert np.count_nonzero(sk.s) == BOOT_HAMMING
    assert set(np.unique(sk.s)) <= {-1, 0, 1}
    sk2, _ = ctx.keygen(3, hamming=BOOT_HAMMING)
    assert np.array_equal(sk.s, sk2.s)


# ------------------------------------------------------------------ ModRaise
def test_mod_raise_is_the_centred_lift():
    """Every raised limb, back in coefficient form, holds the centred lift
    of limb 0's coefficient (Python integers)."""
    pr = ckks.Params(5, [40, 30, 30, 31], [41], 1, 20)
    ctx = ckks.Context(pr)
    q0 = pr.q[0]
    rng = np.random.default_rng(4)
    limb0 = np.stack([ctx.ntt(rng.integers(0, q0, (1, ctx.n), dtype=np.uint64), [q0], pr.psi[:1]) for _ in range(2)])
    # make sure both halves of [0, q0) and the boundary values occur
    co = ctx.intt(limb0[0], [q0], pr.psi[:1])[0]
    co[:4] = [0, q0 // 2, q0 // 2 + 1, q0 - 1]
    limb0[0] = ctx.ntt(co[None, :], [q0], pr.psi[:1])
    ct = ckks.Ciphertext(limb0, 3.0)
    out = BT.mod_raise(ctx, ct, pr.L)
    assert out.level == pr.L and out.scale == 3.0
    assert np.array_equal(out.data[:, 0], limb0[:, 0])
    for k in range(2):
        a = [int(v) for v in ctx.intt(limb0[k], [q0], pr.psi[:1])[0]]
        raised = ctx.intt(out.data[k], pr.q, pr.psi[: pr.L])
        for i, q in enumerate(pr.q):
            want = [(x if x <= (q0 - 1) // 2 else x - q0) % q for x in a]
            assert [int(v) for v in raised[i]] == want


def test_mod_raise_adds_a_small_multiple_of_q0():
    """Decrypted over every limb (exact CRT), the raised ciphertext holds
    t = m + q0 I with m the level-1 decryption and |I| <= (h + 1) / 2."""
    pr = ckks.Params(6, [40, 30, 30], [41], 1, 20)
    ctx = ckks.Context(pr)
    sk, pk = ctx.keygen(5, hamming=8)
    v = np.random.default_rng(2).uniform(-1, 1, ctx.n // 2)
    ct = ctx.encrypt(pk, ctx.encode(v, 2.0 ** 20, 1), 5)
    m = ctx.decrypt_coeffs(sk, ct)
    out = BT.mod_raise(ctx, ct, pr.L)
    qs = pr.q
    t = C.add(out.data[0], C.mul(out.data[1], sk.s_ntt[: pr.L], qs), qs)
    co = ctx.intt(t, qs, pr.psi[: pr.L])
    Q = math.prod(qs)
    q0 = pr.q[0]
    seen = 0
    for k in range(ctx.n):
        x, _ = B.crt([int(co[i, k]) for i in range(pr.L)], qs)
        x = x - Q if x > Q // 2 else x
        assert (x - int(m[k])) % q0 == 0
        I = (x - int(m[k])) // q0
        assert abs(I) <= (8 + 1) // 2 + 1
        seen = max(seen, abs(I))
    assert seen >= 1  # the lift does add multiples of q0


# ------------------------------------------------------------------ butterfly factors
def direct_decode(n_slots, log_n, w):
    """z_j = sum_k w_k zeta^(5^j k), exponents reduced mod 2N before the
    complex exponential."""
    two_n = 2 << log_n
    z = np.zeros(n_slots, dtype=np.complex128)
    for j in range(n_slots):
        e = pow(5, j, two_n)
        z[j] = sum(w[k] * cmath.exp(1j * math.pi * ((e * k) % two_n) / (two_n // 2)) for k in range(n_slots))
    return z


@pytest.mark.parametrize("log_n,levels", [(4, 1), (4, 3), (6, 2), (7, 3), (8, 4)])
def test_factors_equal_the_decoding_sums(log_n, levels):
    n = 1 << (log_n - 1)
    rng = np.random.default_rng(log_n * 10 + levels)
    w = rng.normal(size=n) + 1j * rng.normal(size=n)
    z = direct_decode(n, log_n, w)
    a = w[bitrev_perm(n)]
    plan = BT.BootPlan(log_n, levels, 12.0, 2.0 ** 40, 31)
    y = a.copy()
    for d in plan.stc_diags:
        y = apply_diags(d, y)
    assert np.max(np.abs(y - z)) < 1e-11 * n
    x = z.copy()
    for d in plan.cts_diags:
        x = apply_diags(d, x)
    assert np.max(np.abs(x - a)) < 1e-12 * n


def test_factors_match_the_fft_decoder_at_n4096():
    """At N = 2^12 the factors against the oracle's FFT decoder: for integer
    coefficients m, decode(m) = SlotToCoeff(bitrev(m_lo + i m_hi)) and
    CoeffToSlot(decode(m)) = bitrev(m_lo + i m_hi)."""
    pr = ckks.Params(12, [40], [41], 1, 20)
    ctx = ckks.Context(pr)
    n = ctx.n // 2
    m = np.random.default_rng(5).integers(-1000, 1000, ctx.n).astype(np.float64)
    z = ctx.decode_coeffs_complex(m, 1.0)
    w = (m[:n] + 1j * m[n:])[bitrev_perm(n)]
    plan = BT.BootPlan(12, 3, 12.0, 2.0 ** 40, 31)
    y = w.copy()
    for d in plan.stc_diags:
        y = apply_diags(d, y)
    assert np.max(np.abs(y - z)) < 1e-9 * np.max(np.abs(z))
    x = z.copy()
    for d in plan.cts_diags:
        x = apply_diags(d, x)
    assert np.max(np.abs(x - w)) < 1e-9 * np.max(np.abs(w))


def test_compose_equals_dense_product():
    n = 16
    a = BT.stage_diags(n, 4, False)
    b = BT.stage_diags(n, 2, True)
    def dense(d):
        M = np.zeros((n, n), dtype=np.complex128)
        for s, v in d.items():
            for p in range(n):
                M[p, (p + s) % n] += v[p]
        return M
    assert np.allclose(dense(BT.compose(a, b, n)), dense(a) @ dense(b), atol=1e-14)


def test_level_plans_at_n4096():
    """Diagonal counts and rotation keys of the three-level transforms at
    N = 2^12 (stages 4 + 4 + 3): 16 diagonals (shift unit 128, all residues
    of 2048 / 128), 31 (unit 8, k in [-15, 15]) and 15 (unit 1, k in
    [-7, 7]); 22 distinct rotations for both transforms."""
    plan = BT.BootPlan(12, 3, 12.0, 2.0 ** 50, 159)
    assert [p.count() for p in plan.cts_plans] == [16, 31, 15]
    assert [p.count() for p in plan.stc_plans] == [15, 31, 16]
    assert [p.B for p in plan.cts_plans] == [4, 8, 4]
    assert len(plan.rotations()) == 22
    for p in plan.cts_plans + plan.stc_plans:
        ks = [(j, i) for j, t in p.giants for i, _ in t]
        assert len(ks) == len(set(ks)) == p.count()


@pytest.mark.parametrize("which", ["cts", "stc"])
def test_bsgs_equals_the_diagonal_sum(which):
    """linear_transform in a plain complex slot simulation equals
    sum_d D_d (.) roll(x, -d) for every level."""
    plan = BT.BootPlan(12, 3, 12.0, 2.0 ** 50, 159)
    n = plan.n
    diags = plan.cts_diags if which == "cts" else plan.stc_diags
    plans = plan.cts_plans if which == "cts" else plan.stc_plans
    vals = plan.cts_values() if which == "cts" else plan.stc_values()
    rng = np.random.default_rng(11)
    for d, p, v in zip(diags, plans, vals):
        x = rng.normal(size=n) + 1j * rng.normal(size=n)
        ev = LY.SimEval(n)
        got = BT.linear_transform(ev, LY.SimCt(x, 5), p, v)
        assert got.level == 4
        assert np.allclose(got.v, apply_diags(d, x), atol=1e-12)
        assert ev.ks == len(p.babies) + sum(1 for j, _ in p.giants if j != 0)


# ------------------------------------------------------------------ EvalMod
@pytest.mark.parametrize("K,degree", [(8.0, 95), (16.0, 159)])
def test_mod_coeffs_interpolate_the_sine(K, degree):
    c = BT.mod_coeffs(K, degree)
    assert np.all(c[0::2] == 0.0)
    x = np.linspace(-1, 1, 20001)
    f = np.polynomial.chebyshev.chebval(x, np.concatenate([[c[0] / 2], c[1:]]))
    assert np.max(np.abs(f - np.sin(2 * np.pi * K * x) / (2 * np.pi))) < 1e-12


@pytest.mark.parametrize("K,degree,r", [(16.0, 39, 3), (16.0, 63, 2), (8.0, 31, 3)])
def test_mod_coeffs_double_angles_reach_the_sine(K, degree, r):
    """The cosine interpolant through r double angles c <- 2 c^2 - 1 equals
    sin(2 pi K x) (the identity cos(2 t) = 2 cos(t)^2 - 1 applied to
    t = 2 pi (K x - 1/4) / 2^r)."""
    c = BT.mod_coeffs(K, degree, r)
    x = np.linspace(-1, 1, 40001)
    y = np.polynomial.chebyshev.chebval(x, np.concatenate([[c[0] / 2], c[1:]]))
    for _ in range(r):
        y = 2 * y * y - 1
    assert np.max(np.abs(y - np.sin(2 * np.pi * K * x))) < 1e-11


def test_raise_scale_and_range():
    pr = ckks.Params(**BOOT_PARAMS)
    plan = BT.BootPlan(pr.log_n, 3, BOOT_KMIN, pr.scale, BOOT_DEGREE)
    q0 = pr.q[0]
    e = plan.raise_exp(q0)
    assert plan.raise_scale(q0) == 2.0 ** (50 + e)
    assert plan.K(q0) >= BOOT_KMIN and plan.K(q0) < 2 * BOOT_KMIN
    assert sum(plan.cts_exponents(q0)) == e
    assert sum(plan.stc_exponents(q0)) == 10
    plan_da = BT.BootPlan(pr.log_n, 3, BOOT_KMIN, pr.scale, 39, 3)
    assert sum(plan_da.stc_exponents(q0)) == 7  # 2^10 / (2 pi) ~ 2^7.35


# ------------------------------------------------------------------ conjugation and monomials
def test_conjugation_and_monomials_by_decryption():
    ctx, sk, pk, plan, keys, rk, _, _ = boot_setup()
    rng = np.random.default_rng(8)
    z = rng.uniform(-1, 1, ctx.n // 2) + 1j * rng.uniform(-1, 1, ctx.n // 2)
    ct = ctx.encrypt(pk, ctx.encode_complex(z, 2.0 ** 40, 4), 8)
    w = ctx.rotate(ct, ckks.CONJ, keys)
    assert np.max(np.abs(ctx.decrypt_complex(sk, w) - np.conj(z))) < 1e-6
    iz = ctx.mul_plain(ct, BT.monomial_pt(ctx, ctx.n // 2, 4))
    assert np.max(np.abs(ctx.decrypt_complex(sk, iz) - 1j * z)) < 1e-6
    miz = ctx.mul_plain(ct, BT.monomial_pt(ctx, 3 * ctx.n // 2, 4))
    assert np.max(np.abs(ctx.decrypt_complex(sk, miz) + 1j * z)) < 1e-6


# ------------------------------------------------------------------ the whole procedure
@pytest.mark.parametrize("double_angles", [0, BOOT_DA[1]])
def test_bootstrap_refreshes_within_bound(double_angles):
    ctx, sk, pk, plan, keys, rk, cts, stc = boot_setup(double_angles)
    pr = ctx.pr
    v = np.random.default_rng(3).uniform(-1, 1, ctx.n // 2)
    ct = ctx.encrypt(pk, ctx.encode(v, pr.scale, 1), 9)
    # the multiple of q_0 ModRaise adds stays inside EvalMod's range
    m = ctx.decrypt_coeffs(sk, ct)
    x = BT.mod_raise(ctx, ct, pr.L)
    t = C.add(x.data[0], C.mul(x.data[1], sk.s_ntt[: pr.L], pr.q), pr.q)
    co = ctx.intt(t, pr.q, pr.psi[: pr.L])
    q0 = pr.q[0]
    Q = math.prod(pr.q)
    imax = 0
    for k in range(0, ctx.n, 7):
        tv, _ = B.crt([int(co[i, k]) for i in range(pr.L)], pr.q)
        tv = tv - Q if tv > Q // 2 else tv
        imax = max(imax, abs((tv - int(m[k])) // q0))
    assert imax + 0.5 < plan.K(q0)
    out, ks = BT.bootstrap(ctx, ct, plan, keys, rk, cts, stc)
    lv, relins = LY.cheb_plan(plan.mod_coeffs(q0), False)
    assert out.level == pr.L - 2 * plan.levels - lv - double_angles
    n_rot = sum(len(p.babies) + sum(1 for j, _ in p.giants if j != 0) for p in plan.cts_plans + plan.stc_plans)
    assert ks == n_rot + 1 + 2 * (relins + double_angles)
    assert abs(math.log2(out.scale) - 50) < 0.5
    got = ctx.decrypt(sk, out)
    assert np.max(np.abs(got - v)) < BOOT_TOL
