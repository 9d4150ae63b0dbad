"""Pins of the oracle's PSC weighting functions (Sec. 2.3, Eqs. 8, 9, 13)."""
import numpy as np
import pytest

import oracle
from conftest import read_golden


@pytest.mark.parametrize("row", read_golden("worked_example_weights.txt"))
def test_worked_example(row):
    tau, e1, e2, printed_orig, modified = row
    b_orig, _ = oracle.weights([e1, e2], tau, mode=1)
    b_mod, bs_mod = oracle.weights([e1, e2], tau, mode=0)
    # the printed totals are given to two decimals
    assert round(b_orig, 2) == pytest.approx(printed_orig, abs=1e-12)
    assert b_mod == pytest.approx(modified, abs=1e-15)
    assert bs_mod.sum() == pytest.approx(modified, abs=1e-15)


@pytest.mark.parametrize("tau", [0.51, 0.6, 0.8, 1.0, 2.0])
def test_single_particle_endpoints_and_identity(tau):
    # B = 0 at eps = 0, B = 1 at eps = 1 (text after Eq. 9)
    assert oracle.weights([0.0], tau, 0)[0] == 0.0
    assert oracle.weights([1.0], tau, 0)[0] == pytest.approx(1.0, abs=1e-15)
    # Eq. 13 reduces to Eq. 9 for a single particle (text after Eq. 13)
    for e in np.linspace(0.01, 0.99, 23):
        bm, bsm = oracle.weights([e], tau, 0)
        bo, bso = oracle.weights([e], tau, 1)
        assert bm == pytest.approx(bo, rel=1e-14)
        assert bsm[0] == pytest.approx(bso[0], rel=1e-14)
    # monotone increasing in eps
    vals = [oracle.weights([e], tau, 0)[0] for e in np.linspace(0, 1, 50)]
    assert np.all(np.diff(vals) > 0)


@pytest.mark.parametrize("tau", [0.6, 0.8, 1.0])
def test_modified_weights_sum_linearly(tau):
    # Eq. 13: sum_s B_{n,s}(eps_{n,s}) = B(sum_s eps_{n,s}) for any split.
    rng = np.random.default_rng(11)
    for _ in range(50):
        k = rng.integers(1, 4)
        eps = rng.dirichlet(np.ones(k)) * rng.uniform(0.05, 1.0)
        b_total, b_slot = oracle.weights(eps, tau, 0)
        b_single, _ = oracle.weights([eps.sum()], tau, 0)
        assert b_slot.sum() == pytest.approx(b_single, rel=1e-13)
        assert b_total == pytest.approx(b_single, rel=1e-13)
        # each particle's share is proportional to its solid fraction
        assert np.allclose(b_slot / eps, b_slot[0] / eps[0], rtol=1e-13)


def test_original_underestimates():
    # Fig. 3(b) discussion: the original total weight always underestimates
    # the weight of the summed solid fraction when two particles share a cell.
    for tau in (0.6, 0.8, 1.0):
        for en in (0.6, 0.8, 1.0):
            for e1 in np.linspace(0.05, en - 0.05, 9):
                bo, _ = oracle.weights([e1, en - e1], tau, 1)
                bm, _ = oracle.weights([e1, en - e1], tau, 0)
                assert bo < bm


def test_overfull_cell_shares():
    # Table 1 clamps the cell total to one; the shares still add to B_n = 1.
    b_total, b_slot = oracle.weights([0.7, 0.6], 0.8, 0)
    assert b_total == pytest.approx(1.0, abs=1e-15)
    assert b_slot.sum() == pytest.approx(1.0, abs=1e-15)
    assert b_slot[0] / b_slot[1] == pytest.approx(0.7 / 0.6, rel=1e-14)
