"""Bootstrapping at the full N = 2^16, L = 24 ring against the oracle (needs
MI355X).  The oracle's part (40 keys, 316 encoded diagonals, 111 key
switches) takes about 25 s of CPU time on 16 threads; the test prints each
phase as it ends."""
import time

import numpy as np
import pytest

from oracle import boot as BT
from oracle import ckks
from tests import helpers as H
from tests import test_gpu_boot as GB


pytestmark = pytest.mark.gpu


def test_bootstrap_n16_bit_exact():
    """Cosine of degree 39 with three double angles, three-level transforms,
    a secret of Hamming weight 32: every limb of the refreshed ciphertext
    equal to the oracle's, and its decryption within 2^-11 of the message
    (3.0e-4 measured: a coefficient's error reaches a slot with a factor
    growing as sqrt(N), so the N = 2^12 rings' 1e-5 becomes a few 1e-4
    here with the same 50-bit primes)."""
    from paper_2510_03996_amd import he

    t0 = time.time()
    pr = ckks.Params(**ckks.CONFIGS["config2"])
    ctx = ckks.Context(pr)
    sk, pk = ctx.keygen(11, hamming=32)
    plan = BT.BootPlan(pr.log_n, 3, 12.0, pr.scale, 39, 3)
    keys = {r: ctx.gen_rotation_key(sk, r, 11) for r in plan.rotations()}
    keys[ckks.CONJ] = ctx.gen_rotation_key(sk, ckks.CONJ, 11)
    rk = ctx.gen_relin_key(sk, 11)
    print("keys %.1f s" % (time.time() - t0), flush=True)
    cts, stc = BT.boot_plaintexts(ctx, plan, pr.L)
    print("plaintexts %.1f s" % (time.time() - t0), flush=True)
    v = np.random.default_rng(12).uniform(-1, 1, ctx.n // 2)
    ct = ctx.encrypt(pk, ctx.encode(v, pr.scale, 1), 12)
    want, ks = BT.bootstrap(ctx, ct, plan, keys, rk, cts, stc)
    print("oracle bootstrap %.1f s, %d key switches" % (time.time() - t0, ks), flush=True)
    g = H.gpu_ctx("config2")
    try:
        assert [int(x) for x in g.moduli] == pr.q + pr.p
        GB.upload_boot_keys(g, keys, rk)
        desc = he.boot_desc(3, 39, 12.0, pr.scale, double_angles=3)
        gct = g.ct_from_numpy(ct.data, ct.scale)
        gcts = [g.pt_from_numpy(p.data, p.scale) for lv in cts for p in lv]
        gstc = [g.pt_from_numpy(p.data, p.scale) for lv in stc for p in lv]
        coeffs = list(plan.mod_coeffs(pr.q[0]))
        got = g.bootstrap(gct, desc, gcts, gstc, coeffs)
        assert got.level == want.level == pr.L - 15 and got.scale == want.scale
        H.assert_limbs_equal(got.numpy(), want.data, "bootstrap at N=2^16")
        err = np.max(np.abs(ctx.decrypt(sk, ckks.Ciphertext(got.numpy(), got.scale)) - v))
        print("GPU bootstrap bit-exact, max decryption error %.3g, %.1f s" % (err, time.time() - t0), flush=True)
        assert err < 2.0 ** -11
        # one stream (no helpers), and four (giant steps over four streams,
        # the EvalMod parts on the caller and its second helper)
        for n in (1, 4):
            g.layer_streams(n)
            got = g.bootstrap(gct, desc, gcts, gstc, coeffs)
            H.assert_limbs_equal(got.numpy(), want.data, "bootstrap at N=2^16 on %d layer stream(s)" % n)
            print("bit-exact on %d layer stream(s)" % n, flush=True)
    finally:
        g.close()
