"""GPU parity at the parameters of the Sec. 3.5 random-packing runs (the
100 x 50 x 50 D3Q19 box at tau = 2, JKR or Hertz with sliding, twisting and
rolling friction, four DEM sub-steps) against the oracle: 30 coupled steps
from a seeded, jittered lattice of 48 spheres whose neighbours and bottom
row overlap by 0.02, so every contact kind is loaded from the first step.
Tolerances as for the other DEM tests."""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import gpu_lattice, relerr

pytestmark = pytest.mark.gpu


def _start(adhesive, seed=36):
    w = W.random_packing(adhesive)
    rng = np.random.default_rng(seed)
    s = 5.98
    pts = [[2.48 + i * s, 10.0 + j * s, 10.0 + k * s]
           for i in range(3) for j in range(4) for k in range(4)]
    n = len(pts)
    x = np.array(pts) + rng.normal(0.0, 0.005, (n, 3))
    u = rng.normal(0.0, 1e-3, (n, 3))
    om = rng.normal(0.0, 2e-4, (n, 3))
    return w.lattice, W.Particles(x, u, om, np.full(n, 3.0)), w.dem


@pytest.mark.parametrize("adhesive", [True, False])
def test_packing_parameters_parity(adhesive):
    import paper_1901_09745_amd.psclbm as P
    print(f"case: packing {'JKR' if adhesive else 'Hertz'}", flush=True)
    lat, p, dem = _start(adhesive)
    ref = oracle.Lattice(lat)
    D = oracle.Dem(lat, dem, p.n)
    pr = p.copy()
    for _ in range(30):
        F, T = ref.step(pr)
        D.step(pr, F, T)
    assert sum(len(c) for c in D.contacts()) > 150
    G = gpu_lattice(lat, p)
    dp = P.DeviceParticles.from_host(p)
    G.coupled_step(P.make_dem_params(dem), dp, 30)
    G.sync()
    assert relerr(G.get_f().cpu().numpy(), ref.f) < 1e-12
    assert np.abs(dp.x.cpu().numpy() - pr.x).max() < 1e-9
    assert np.abs(dp.u.cpu().numpy() - pr.u).max() < 1e-11
    assert np.abs(dp.omega.cpu().numpy() - pr.omega).max() < 1e-11
