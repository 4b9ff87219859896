"""Pins for the Chebyshev secure ReLU (CPU only).

The oracle's coefficients, term selection and evaluation schedule are checked
against things that do not share its code: numpy's own Chebyshev
interpolation at first-kind points, exact interpolation at the nodes, the
known approximation quality for |z|, a float slot simulation of the schedule
against direct Clenshaw evaluation, the closed-form plan for D = 59, and the
CKKS evaluation decrypting to the FP64 polynomial.
"""
import numpy as np
import pytest

import synth
from oracle import ckks
from oracle import layers as LY
from tests import helpers as H


@pytest.mark.parametrize("beta", [1.0, 4.0])
@pytest.mark.parametrize("degree", [7, 27, 59])
def test_coefficients_match_numpy_interpolation(beta, degree):
    ours = LY.cheb_relu_coeffs(beta, degree)
    ref = np.polynomial.chebyshev.chebinterpolate(lambda z: beta * np.maximum(0.0, z), degree)
    want = ref.copy()
    want[0] *= 2.0  # our series is c_0/2 + sum c_j T_j
    assert np.max(np.abs(ours - want)) < 1e-13 * beta
    assert all(ours[j] == 0.0 for j in range(3, degree + 1, 2)) and ours[1] == beta / 2


@pytest.mark.parametrize("degree", [7, 59])
def test_interpolates_at_the_nodes(degree):
    beta = 2.5
    c = LY.cheb_relu_coeffs(beta, degree).copy()
    c[0] /= 2
    n = degree + 1
    z = np.cos(np.pi * (np.arange(n) + 0.5) / n)
    assert np.max(np.abs(np.polynomial.chebyshev.chebval(z, c) - beta * np.maximum(0.0, z))) < 1e-12 * beta


def test_degree59_approximates_relu():
    # |z| interpolated at 60 Chebyshev nodes: error of order 1/(pi D), largest near 0
    for beta in (1.0, 4.0):
        x = np.linspace(-beta, beta, 20001)
        err = np.abs(LY.cheb_relu_ref(x, beta) - np.maximum(0.0, x))
        assert err.max() < 0.012 * beta
        assert err[np.abs(x) > 0.2 * beta].max() < 1e-3 * beta


def test_terms_and_plan_closed_form():
    c = LY.cheb_relu_coeffs(1.0)
    # leaves use T_1, T_2, T_4, T_6 (odd coefficients vanish); giant steps T_8, T_16, T_32; T_3 is a factor of T_6
    assert LY.cheb_terms(c) == [1, 2, 3, 4, 6, 8, 16, 32]
    assert LY.cheb_plan(c, True) == (7, 14) and LY.cheb_plan(c, False) == (6, 14)
    assert [LY.cheb_depth(j) for j in (1, 2, 3, 4, 5, 8, 9, 16, 17, 32, 33, 58)] == [0, 1, 2, 2, 3, 3, 4, 4, 5, 5, 6, 6]
    # only T_1 and even T_j carry coefficients
    assert [j for j in range(60) if c[j] != 0.0] == [0, 1] + list(range(2, 59, 2))


@pytest.mark.parametrize("degree", [40, 59, 100])
def test_split_tree_reconstructs_the_series(degree):
    """The recursive division by giant steps is an identity of polynomials
    (checked by evaluating both sides at many points with numpy)."""
    rng = np.random.default_rng(degree)
    a = rng.normal(size=degree + 1)
    x = np.linspace(-1, 1, 257)

    def val(t):
        if t[0] == "leaf":
            return np.polynomial.chebyshev.chebval(x, t[1])
        return val(t[2]) * np.polynomial.chebyshev.chebval(x, np.eye(t[1] + 1)[t[1]]) + val(t[3])

    tree = LY.cheb_tree(a)
    assert np.max(np.abs(val(tree) - np.polynomial.chebyshev.chebval(x, a))) < 1e-10 * np.abs(a).sum()


@pytest.mark.parametrize("beta", [1.0, 4.0])
def test_sim_schedule_equals_clenshaw(beta):
    slots, n = 1024, 600
    x = np.zeros(slots)
    x[:n] = synth.uniform_slots(70, n, -beta, beta)
    c = LY.cheb_relu_coeffs(beta)
    ev = LY.SimEval(slots)
    mask = LY.cheb_scale_mask(beta, n, slots) if beta > 1 else None
    y = LY.cheb_eval(ev, LY.SimCt(x, 24, 2.0 ** 50), c, mask, 2.0 ** 50)
    assert ev.ks == 0  # the slot simulation counts rotations only
    assert y.level == 24 - LY.cheb_plan(c, mask is not None)[0]
    assert np.max(np.abs(y.v[:n] - LY.cheb_relu_ref(x[:n], beta))) < 1e-9 * beta
    if mask is not None:  # slots beyond n are masked to zero input: p(0) there
        assert np.max(np.abs(y.v[n:] - LY.cheb_relu_ref(0.0, beta))) < 1e-12


@pytest.mark.slow
def test_he_config1_cheb_relu_decrypts():
    """N=2^14, 8 limbs, beta = 1 (no mask): six levels, level 8 -> 2."""
    name = "config1"
    octx, sk, _ = H.oracle_ctx(name)
    c = LY.cheb_relu_coeffs(1.0)
    v, ct = H.encrypt_slots(name, 71)
    ev = LY.HEEval(octx, {}, H.oracle_key(name, "relin"))
    y = LY.cheb_eval(ev, ct, c, None, octx.pr.scale)
    assert y.level == 2 and ev.ks == 14
    dec = octx.decrypt(sk, ckks.Ciphertext(y.data, y.scale))
    assert np.max(np.abs(dec - LY.cheb_relu_ref(v, 1.0))) < 1e-3
