"""Host-side bootstrapping recipes of the C ABI against the oracle (CPU only):
the transform plan (rotation keys, plaintext counts), the plaintext slot
vectors in consumption order, the EvalMod coefficients."""
import numpy as np
import pytest

from oracle import boot as BT
from paper_2510_03996_amd import he

CASES = [(4, 1), (4, 3), (6, 2), (8, 3), (12, 3), (12, 2), (13, 4), (16, 3)]


@pytest.mark.parametrize("log_n,levels", CASES)
def test_boot_plan_matches_oracle(log_n, levels):
    plan = BT.BootPlan(log_n, levels, 12.0, 2.0 ** 50, 31)
    rots, counts, ks = he.boot_plan(log_n, levels, key_switches=True)
    assert rots == plan.rotations()
    assert counts == [p.count() for p in plan.cts_plans] + [p.count() for p in plan.stc_plans]
    assert ks == sum(len(p.babies) + sum(1 for j, _ in p.giants if j != 0) for p in plan.cts_plans + plan.stc_plans)


@pytest.mark.parametrize("log_n,levels", [(4, 3), (6, 2), (8, 3), (12, 3)])
@pytest.mark.parametrize("inverse", [True, False])
def test_boot_diagonals_match_oracle(log_n, levels, inverse):
    plan = BT.BootPlan(log_n, levels, 12.0, 2.0 ** 50, 31)
    want = [v for lv in (plan.cts_values() if inverse else plan.stc_values()) for v in lv]
    got = he.boot_diagonals(log_n, levels, inverse)
    assert len(got) == len(want)
    for g, w in zip(got, want):
        assert np.array_equal(g == 0, w == 0)
        assert np.max(np.abs(g - w)) < 1e-12


@pytest.mark.parametrize("K,degree,r", [(8.0, 95, 0), (16.000000001, 159, 0), (3.0, 31, 0), (16.0, 39, 3),
                                         (12.5, 63, 2)])
def test_boot_mod_coeffs_match_oracle(K, degree, r):
    got = np.array(he.boot_mod_coeffs(K, degree, r))
    assert np.max(np.abs(got - BT.mod_coeffs(K, degree, r))) < 1e-14


def test_boot_recipe_errors():
    with pytest.raises(he.HEError):
        he.boot_plan(12, 0)
    with pytest.raises(he.HEError):
        he.boot_plan(12, 12)
    with pytest.raises(he.HEError):
        he.boot_mod_coeffs(0.0, 31)
    with pytest.raises(he.HEError):
        he.boot_mod_coeffs(8.0, 0)
    with pytest.raises(he.HEError):
        he.boot_mod_coeffs(8.0, 31, 9)


@pytest.mark.parametrize("log_n", [3, 5, 9, 13, 14])
def test_boot_plan_every_level_count(log_n):
    """Every level count from 1 to log2(N/2): rotation keys, plaintext counts
    and key switches of the C plan equal the oracle's, and the transforms'
    diagonals at the small rings equal the oracle's values."""
    for levels in range(1, log_n):
        plan = BT.BootPlan(log_n, levels, 12.0, 2.0 ** 50, 31)
        rots, counts, ks = he.boot_plan(log_n, levels, key_switches=True)
        assert rots == plan.rotations(), (log_n, levels)
        assert counts == [p.count() for p in plan.cts_plans] + [p.count() for p in plan.stc_plans]
        assert ks == sum(len(p.babies) + sum(1 for j, _ in p.giants if j != 0)
                         for p in plan.cts_plans + plan.stc_plans)
        if log_n <= 9:
            for inverse in (True, False):
                want = [v for lv in (plan.cts_values() if inverse else plan.stc_values()) for v in lv]
                got = he.boot_diagonals(log_n, levels, inverse)
                assert len(got) == len(want)
                assert max(np.max(np.abs(g - w)) for g, w in zip(got, want)) < 1e-12
