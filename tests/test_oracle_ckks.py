"""Pins for the oracle's CKKS layer: encoding, keys, encryption, rotations,
relinearization (CPU only).

Checks use exact big-integer decryption over every Q limb (tiny rings), the
encoding definition evaluated directly, and decrypted results against the
plaintext computation at the real ring sizes.
"""
import cmath
import math

import numpy as np
import pytest

from oracle import _lib as C
from oracle import ckks
from tests import t0_bigint as B


def tiny():
    # N = 16, alpha = 2, K = 2: several digits, a short last digit at odd levels
    return ckks.Params(4, [31, 26, 26, 26, 26], [31, 31], 2, 20)


def full_decrypt(ctx, sk, ct):
    """Exact c0 + c1 s over all active limbs, CRT-combined and centred."""
    pr = ctx.pr
    lv = ct.level
    qs = pr.q[:lv]
    m = C.add(ct.data[0], C.mul(ct.data[1], sk.s_ntt[:lv], qs), qs)
    co = C.ntt(m, qs, pr.psi[:lv], inverse=True)
    Q = math.prod(qs)
    out = []
    for k in range(ctx.n):
        x, _ = B.crt([int(co[i, k]) for i in range(lv)], qs)
        out.append(x - Q if x > Q // 2 else x)
    return out, Q


# ------------------------------------------------------------------ encoding
@pytest.mark.parametrize("log_n", [4, 6])
def test_encode_matches_direct_formula(log_n):
    pr = ckks.Params(log_n, [30], [31], 1, 20)
    ctx = ckks.Context(pr)
    n = pr.n
    rng = np.random.default_rng(log_n)
    v = rng.uniform(-1, 1, n // 2)
    scale = 2.0 ** 30
    got = ctx.encode_coeffs(v, scale)
    for k in range(n):
        mk = (2.0 / n) * sum(v[j] * math.cos(math.pi * pow(5, j, 2 * n) * k / n) for j in range(n // 2))
        assert abs(got[k] - mk * scale) <= 0.5 + 1e-6 * scale


@pytest.mark.parametrize("log_n", [4, 6])
def test_encoding_evaluates_to_slots(log_n):
    """m(zeta^(5^j)) = scale * v_j up to rounding, by Horner in complex doubles."""
    pr = ckks.Params(log_n, [30], [31], 1, 20)
    ctx = ckks.Context(pr)
    n = pr.n
    v = np.random.default_rng(9).uniform(-1, 1, n // 2)
    scale = 2.0 ** 30
    m = ctx.encode_coeffs(v, scale)
    for j in range(n // 2):
        z = cmath.exp(1j * math.pi * pow(5, j, 2 * n) / n)
        acc = 0j
        for k in reversed(range(n)):
            acc = acc * z + float(m[k])
        assert abs(acc.real / scale - v[j]) < 1e-6 and abs(acc.imag / scale) < 1e-6
    dec = ctx.decode_coeffs(m.astype(np.float64), scale)
    assert np.max(np.abs(dec - v)) < 1e-6


def test_encode_const_is_constant_polynomial():
    pr = ckks.Params(**ckks.CONFIGS["config0"])
    ctx = ckks.Context(pr)
    pt = ctx.encode_const(-0.3, 2.0 ** 40, 3)
    co = C.ntt(pt.data, pr.q[:3], pr.psi[:3], inverse=True)
    r = -int(math.floor(0.3 * 2.0 ** 40 + 0.5))
    for i, q in enumerate(pr.q[:3]):
        assert int(co[i, 0]) == r % q and not co[i, 1:].any()


# ------------------------------------------------------------------ encryption
def test_encrypt_decrypt_exact_noise_tiny():
    pr = tiny()
    ctx = ckks.Context(pr)
    sk, pk = ctx.keygen(7)
    v = np.linspace(-1, 1, pr.n // 2)
    pt = ctx.encode(v, 2.0 ** 20, pr.L)
    ct = ctx.encrypt(pk, pt, 7)
    got, _ = full_decrypt(ctx, sk, ct)
    want = ctx.encode_coeffs(v, 2.0 ** 20)
    noise = max(abs(int(a) - int(b)) for a, b in zip(got, want))
    assert noise < 2 ** 12


@pytest.mark.parametrize("name", ["config0", "config1"])
def test_encrypt_decrypt_roundtrip(name):
    pr = ckks.Params(**ckks.CONFIGS[name])
    ctx = ckks.Context(pr)
    sk, pk = ctx.keygen(3)
    v = np.random.default_rng(1).uniform(-1, 1, pr.n // 2)
    ct = ctx.encrypt(pk, ctx.encode(v, pr.scale, pr.L), 3)
    assert np.max(np.abs(ctx.decrypt(sk, ct) - v)) < 1e-6


# ------------------------------------------------------------------ key switching
@pytest.mark.parametrize("level", [5, 4, 3])
def test_rotation_decryption_identity_tiny(level):
    """c0' + c1' s = phi_g(c0 + c1 s) + small, exactly over every Q limb."""
    pr = tiny()
    ctx = ckks.Context(pr)
    sk, pk = ctx.keygen(11)
    rs = [1, -1, 3]
    keys = {r: ctx.gen_rotation_key(sk, r, 11) for r in rs}
    rng = np.random.default_rng(level)
    v = rng.uniform(-1, 1, pr.n // 2)
    ct = ctx.encrypt(pk, ctx.encode(v, 2.0 ** 20, pr.L), 11)
    ct = ctx.drop_level(ct, level)
    before, Q = full_decrypt(ctx, sk, ct)
    outs = ctx.rotate_hoisted(ct, rs, keys)
    for r, o in zip(rs, outs):
        g = ctx.galois_element(r)
        want = B.automorph([x % Q for x in before], g, Q)
        want = [w - Q if w > Q // 2 else w for w in want]
        got, _ = full_decrypt(ctx, sk, o)
        err = max(abs(a - b) for a, b in zip(got, want))
        assert err < 2 ** 12, (r, err)


def test_keyswitch_gadget_identity_tiny():
    """sum_j [c]_{Q_j} * gadget_j == P * c mod PQ (exact big integers), where the
    gadget is what b_j - (-a_j s + e_j) carries: [P]_{q_i} s' on digit j."""
    pr = tiny()
    P = pr.P
    Q = math.prod(pr.q)
    rng = np.random.default_rng(3)
    for _ in range(20):
        c = int(rng.integers(0, 2 ** 62)) * int(rng.integers(0, 2 ** 62)) % Q
        acc = 0
        for j in range(pr.dnum(pr.L)):
            idx = pr.digit(j, pr.L)
            Qj = math.prod(pr.q[i] for i in idx)
            # gadget_j as the CRT element: P mod q_i on digit j, 0 elsewhere (incl. P)
            res = [(P % q) if i in idx else 0 for i, q in enumerate(pr.q)] + [0] * pr.K
            g, _ = B.crt(res, pr.q + pr.p)
            acc += (c % Qj) * g
        assert acc % (P * Q) == (P * c) % (P * Q)


@pytest.mark.parametrize("name", ["config0", "config1"])
def test_rotation_semantics(name):
    """Rot_r moves slot i + r to slot i (decrypted, full packing)."""
    pr = ckks.Params(**ckks.CONFIGS[name])
    ctx = ckks.Context(pr)
    sk, pk = ctx.keygen(5)
    rs = [1, -1, 7, -(pr.n // 8)]
    keys = {r: ctx.gen_rotation_key(sk, r, 5) for r in rs}
    v = np.random.default_rng(2).uniform(-1, 1, pr.n // 2)
    ct = ctx.encrypt(pk, ctx.encode(v, pr.scale, pr.L), 5)
    for r, o in zip(rs, ctx.rotate_hoisted(ct, rs, keys)):
        assert np.max(np.abs(ctx.decrypt(sk, o) - np.roll(v, -r))) < 1e-5
    # one formula for all: a single rotation equals the hoisted one bit for bit
    one = ctx.rotate(ct, rs[2], keys)
    assert np.array_equal(one.data, ctx.rotate_hoisted(ct, rs, keys)[2].data)


def test_mul_plain_rescale_relin_config1():
    pr = ckks.Params(**ckks.CONFIGS["config1"])
    ctx = ckks.Context(pr)
    sk, pk = ctx.keygen(9)
    rk = ctx.gen_relin_key(sk, 9)
    rng = np.random.default_rng(4)
    a = rng.uniform(-1, 1, pr.n // 2)
    b = rng.uniform(-1, 1, pr.n // 2)
    w = rng.uniform(-1, 1, pr.n // 2)
    ca = ctx.encrypt(pk, ctx.encode(a, pr.scale, pr.L), 9, 0)
    cb = ctx.encrypt(pk, ctx.encode(b, pr.scale, pr.L), 9, 1)
    m = ctx.rescale(ctx.mul_plain(ca, ctx.encode(w, pr.scale, pr.L)))
    assert m.level == pr.L - 1
    assert np.max(np.abs(ctx.decrypt(sk, m) - a * w)) < 1e-4
    r = ctx.rescale(ctx.mul_relin(ca, cb, rk))
    assert np.max(np.abs(ctx.decrypt(sk, r) - a * b)) < 1e-4
    s = ctx.add(ca, cb)
    assert np.max(np.abs(ctx.decrypt(sk, s) - (a + b))) < 1e-5
    with pytest.raises(ValueError):
        ctx.add(ca, m)


def test_relin_decryption_identity_tiny():
    """(d0 + u0) + (d1 + u1) s = d0 + d1 s + d2 s^2 + small, exactly."""
    pr = tiny()
    ctx = ckks.Context(pr)
    sk, pk = ctx.keygen(21)
    rk = ctx.gen_relin_key(sk, 21)
    rng = np.random.default_rng(0)
    ca = ctx.encrypt(pk, ctx.encode(rng.uniform(-1, 1, 8), 2.0 ** 20, pr.L), 21, 0)
    cb = ctx.encrypt(pk, ctx.encode(rng.uniform(-1, 1, 8), 2.0 ** 20, pr.L), 21, 1)
    d, sc = ctx.tensor(ca, cb)
    qs = pr.q
    s = sk.s_ntt[: pr.L]
    m3 = C.add(C.add(d[0], C.mul(d[1], s, qs), qs), C.mul(d[2], C.mul(s, s, qs), qs), qs)
    co = C.ntt(m3, qs, pr.psi[: pr.L], inverse=True)
    Q = math.prod(qs)
    want = []
    for k in range(ctx.n):
        x, _ = B.crt([int(co[i, k]) for i in range(pr.L)], qs)
        want.append(x - Q if x > Q // 2 else x)
    got, _ = full_decrypt(ctx, sk, ctx.relin(d, sc, rk))
    assert max(abs(a - b) for a, b in zip(got, want)) < 2 ** 12


def test_hoisted_differs_from_naive_order_but_decrypts_equal():
    """The other valid order (automorph c1 first, then ModUp) gives different
    bits but the same message: documents why the order is pinned."""
    pr = ckks.Params(**ckks.CONFIGS["config0"])
    ctx = ckks.Context(pr)
    sk, pk = ctx.keygen(1)
    keys = {1: ctx.gen_rotation_key(sk, 1, 1)}
    v = np.random.default_rng(0).uniform(-1, 1, pr.n // 2)
    ct = ctx.encrypt(pk, ctx.encode(v, pr.scale, pr.L), 1)
    pinned = ctx.rotate(ct, 1, keys)
    g = ctx.galois_element(1)
    lv = ct.level
    ext = ctx.modup(ctx.automorph(ct.data[1], g), lv)
    u0, u1 = ctx.keyswitch_ext(ext, keys[1], 1, lv)
    c0 = C.add(ctx.automorph(ct.data[0], g), u0, pr.q[:lv])
    other = ckks.Ciphertext(np.stack([c0, u1]), ct.scale)
    assert not np.array_equal(pinned.data, other.data)
    assert np.max(np.abs(ctx.decrypt(sk, pinned) - ctx.decrypt(sk, other))) < 1e-6
