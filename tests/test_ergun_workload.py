"""The packed bed of Sec. 3.4 as a synthetic workload (CPU): the dimensionless
numbers of Eqs. 35-36 against Eq. 34 written out, and the geometry of the
8-sphere lattice packing as the oracle rasterises it."""
import numpy as np
import pytest

import oracle
import workloads as W


@pytest.mark.parametrize("dp,U", [(10, 1e-3), (20, 7e-4), (40, 3e-4)])
def test_dimensionless_form_is_eq34(dp, U):
    # Eq. 34 gives the pressure gradient of a bed at superficial velocity U;
    # Eq. 36 of that gradient must land on Eq. 35 at the same Re_p*
    eps, tau = W.ERGUN_POROSITY, 0.65
    mu = (tau - 0.5) / 3.0  # rho = 1
    G = 150 * mu * U * (1 - eps) ** 2 / (dp ** 2 * eps ** 3) + 1.75 * U ** 2 * (1 - eps) / (dp * eps ** 3)
    re, dps = W.ergun_numbers(G, U, dp, tau)
    assert re == pytest.approx(dp * U / (mu * (1 - eps)), rel=1e-14)
    assert dps == pytest.approx(W.ergun_dp_star(re), rel=1e-12)


@pytest.mark.parametrize("re", [0.1, 1.0, 10.0])
def test_workload_force_is_eq35_at_target(re):
    # the body force of the workload, with the superficial velocity that the
    # target Re_p* defines, returns that Re_p* and Eq. 35's dP*
    w = W.ergun(20, re)
    U = re * (w.lattice.tau - 0.5) / 3.0 * (1 - W.ERGUN_POROSITY) / 20
    r, dps = W.ergun_numbers(w.lattice.force[0], U, 20, w.lattice.tau)
    assert r == pytest.approx(re, rel=1e-13)
    assert dps == pytest.approx(150.0 / re + 1.75, rel=1e-12)


@pytest.mark.parametrize("dp", [10, 20])
def test_packing_geometry(dp):
    w = W.ergun(dp)
    lat, p = w.lattice, w.particles
    assert (lat.nx, lat.ny, lat.nz) == (2 * dp,) * 3 and p.n == 8
    assert np.all(p.r == dp / 2)
    # simple cubic: every sphere touches its six periodic neighbours
    L = 2 * dp
    d = p.x[:, None, :] - p.x[None, :, :]
    d -= L * np.round(d / L)
    dist = np.sqrt((d ** 2).sum(-1)) + np.eye(8) * 1e9
    assert dist.min() == pytest.approx(dp, abs=1e-12)
    # solid volume of the rasterised spheres (Eqs. 15-19) and the porosity
    nslot, ids, eps, _ = oracle.rasterize(lat, p.x, p.r)
    vol = 8 * 4.0 / 3.0 * np.pi * (dp / 2) ** 3
    assert abs(eps.sum() - vol) / vol < 2e-3
    assert abs(1 - np.minimum(eps.sum(axis=1), 1).sum() / L ** 3 - W.ERGUN_POROSITY) < 2e-3
    # the contact cells are shared by the two touching spheres
    assert nslot.max() == 2
