"""Sec. 3.1 on the GPU: the 10 x 51 x 51 D3Q19 duct (walls on the two
cross-stream axes, periodic along the flow, tau = 0.65), driven from rest by
a constant body force to steady state, against the series solution of
Eq. 30 with the printed 0.5 % bound, in the FP64 and FP32 forms; and FP64
parity with the oracle over the first steps from rest."""
import numpy as np
import pytest

import oracle
import workloads as W
from conftest import read_golden
from helpers import gpu_lattice, relerr
from test_oracle_lbm import _duct_series

pytestmark = pytest.mark.gpu


def _duct(ny, nz, tau, g):
    return W.LatticeSpec(q=19, nx=10, ny=ny, nz=nz, tau=tau, force=(g, 0.0, 0.0),
                         faces=(W.PERIODIC, W.PERIODIC, W.BOUNCE_BACK, W.BOUNCE_BACK,
                                W.BOUNCE_BACK, W.BOUNCE_BACK))


@pytest.mark.parametrize("form", ["fp64", "fp32"])
@pytest.mark.parametrize("row", read_golden("duct_flow.txt"))
def test_duct_from_rest_reaches_the_series(row, form):
    ny, nz, tau, g, tol = int(row[0]), int(row[1]), row[2], row[3], row[4]
    print(f"case: duct {ny}x{nz} g={g} {form}", flush=True)
    lat = _duct(ny, nz, tau, g)
    nu = (tau - 0.5) / 3
    ref = _duct_series(ny, nz, g, nu)
    G = gpu_lattice(lat, None, precision=form)
    G.rasterize(None)
    # slowest mode decays as exp(-nu pi^2 (1/ny^2 + 1/nz^2) t): 14 e-folds
    steps = int(14 / (nu * np.pi ** 2 * (1 / ny ** 2 + 1 / nz ** 2)))
    G.step(steps)
    _, u = G.macros()
    G.sync()
    ux = u.cpu().numpy().reshape(nz, ny, 10, 3)[..., 0]
    err = np.abs(ux - ref.T[:, :, None]).max() / ref.max()
    print(f"steps {steps}, max relative error {err:.2e}", flush=True)
    assert err < tol
    # the flow is uniform along the duct
    assert np.abs(ux - ux[:, :, :1]).max() < 1e-6 * ref.max()


def test_duct_parity_from_rest():
    lat = _duct(51, 51, 0.65, 6.4e-5)
    L = oracle.Lattice(lat)
    for _ in range(300):
        L.step()
    G = gpu_lattice(lat, None)
    G.rasterize(None)
    G.step(300)
    G.sync()
    assert relerr(G.get_f().cpu().numpy(), L.f) < 1e-12
