"""GPU vs oracle parity for the Chebyshev secure ReLU (needs MI355X)."""
import numpy as np
import pytest

from oracle import ckks
from oracle import layers as LY
from tests import helpers as H

pytestmark = pytest.mark.gpu


def run(name, beta, n, seed):
    from paper_2510_03996_amd import he

    octx, sk, _ = H.oracle_ctx(name)
    slots = octx.n // 2
    g = H.gpu_ctx(name)
    try:
        g.key_upload(he.KEY_RELIN, H.oracle_key(name, "relin"))
        x = np.zeros(slots)
        x[:n] = np.linspace(-beta, beta, n) if seed is None else np.random.default_rng(seed).uniform(-beta, beta, n)
        _, ct = H.encrypt_slots(name, 90, values=x)
        c = LY.cheb_relu_coeffs(beta)
        mask = octx.encode(LY.cheb_scale_mask(beta, n, slots), octx.pr.scale, ct.level) if beta > 1 else None
        ev = LY.HEEval(octx, {}, H.oracle_key(name, "relin"))
        want = LY.cheb_eval(ev, ct, c, mask, octx.pr.scale)
        levels, relins = he.cheb_plan(list(c), mask is not None)
        assert ev.ks == relins == 14 and ct.level - want.level == levels
        gct = g.ct_from_numpy(ct.data, ct.scale)
        gmask = g.pt_from_numpy(mask.data, mask.scale) if mask is not None else None
        for n_streams in (1, 2):  # terms and the division tree over one or two streams (N=2^16)
            g.layer_streams(n_streams)
            got = g.cheb(gct, list(c), octx.pr.scale, scale_mask=gmask)
            H.assert_limbs_equal(got.numpy(), want.data, "Chebyshev ReLU on %d stream(s)" % n_streams)
            assert got.level == want.level and got.scale == want.scale
        dec = octx.decrypt(sk, ckks.Ciphertext(got.numpy(), got.scale))
        assert np.max(np.abs(dec[:n] - LY.cheb_relu_ref(x[:n], beta))) < 1e-3  # the per-layer tolerance
        assert np.max(np.abs(dec[:n] - np.maximum(0.0, x[:n]))) < 0.012 * beta
    finally:
        g.close()


def test_config2_beta4_masked():
    """N=2^16, level 24 -> 17, beta = 4 with the 1/beta mask on 1024 slots."""
    run("config2", 4.0, 1024, 91)


def test_config1_beta1():
    """N=2^14, level 8 -> 2 (six levels), beta = 1 without a mask."""
    run("config1", 1.0, 4096, None)


def test_errors():
    from paper_2510_03996_amd import he

    name = "config1"
    g = H.gpu_ctx(name)
    try:
        _, ct = H.encrypt_slots(name, 92)
        c = list(LY.cheb_relu_coeffs(1.0))
        gct = g.ct_from_numpy(ct.data, ct.scale)
        with pytest.raises(he.HEError) as e:
            g.cheb(gct, c, 2.0 ** 45, out=g.new_ct())
        assert e.value.name == "HE_ENOKEY"
        g.key_upload(he.KEY_RELIN, H.oracle_key(name, "relin"))
        low = g.drop_level(gct, 6)  # the degree-59 evaluation needs more than six levels
        with pytest.raises(he.HEError) as e:
            g.cheb(low, c, 2.0 ** 45, out=g.new_ct())
        assert e.value.name == "HE_ELEVEL"
    finally:
        g.close()
