"""The Sec. 3.5 random-packing workload and the packing statistics that
bench.py reports for it: phi and Z of regular lattices (simple cubic:
pi/6 and 6; body-centred cubic: pi sqrt(3)/8 and 8), and the generator's
placement, box and materials."""
import math

import numpy as np
import pytest

import bench
import workloads as W


def _stats(x, r, L):
    return bench.packing_stats(x, np.full(len(x), r), L, (False, True, True), 1e-9)


def test_simple_cubic_lattice():
    r, d = 3.0, 6.0
    x = np.array([[r - 0.5 + i * d, j * d, k * d]
                  for i in range(12) for j in range(8) for k in range(8)])
    st = _stats(x, r, (100.0, 48.0, 48.0))
    assert st["phi"] == pytest.approx(math.pi / 6, rel=1e-12)
    assert st["Z"] == 6.0


def test_body_centred_cubic_lattice():
    r = 3.0
    a = 4 * r / math.sqrt(3)          # spheres touch along the body diagonal
    n = 7
    pts = []
    for i in range(10):
        for j in range(n):
            for k in range(n):
                pts.append([r - 0.5 + i * a, j * a, k * a])
                pts.append([r - 0.5 + (i + 0.5) * a, (j + 0.5) * a, (k + 0.5) * a])
    x = np.array(pts)
    st = _stats(x, r, (100.0, n * a, n * a))
    assert st["phi"] == pytest.approx(math.pi * math.sqrt(3) / 8, rel=2e-2)   # slab cuts cells
    assert st["Z"] == 8.0


@pytest.mark.parametrize("adhesive", [True, False])
def test_random_packing_workload(adhesive):
    w = W.random_packing(adhesive)
    p, lat, dem = w.particles, w.lattice, w.dem
    assert (lat.q, lat.nx, lat.ny, lat.nz, lat.tau) == (19, 100, 50, 50, 2.0)
    assert lat.faces[:2] == (W.BOUNCE_BACK, W.BOUNCE_BACK)
    assert p.n == 500 and np.all(p.r == 3.0)
    assert np.all(p.x[:, 0] - 3.0 >= -0.5 + 0.5 - 1e-9)
    assert np.all(p.x[:, 0] + 3.0 <= 99.5 - 0.5 + 1e-9)
    dv = p.x[None] - p.x[:, None]
    for ax, L in ((1, 50.0), (2, 50.0)):
        dv[:, :, ax] -= L * np.round(dv[:, :, ax] / L)
    dist = np.sqrt((dv ** 2).sum(-1)) + np.eye(p.n) * 1e9
    assert dist.min() >= 6.5 - 1e-9                       # gap 0.5
    assert (dem.gamma > 0) == adhesive
    assert dem.mu_f > 0 and dem.theta_r > 0 and dem.n_sub == 4
    assert dem.g[0] < 0 and dem.g[1] == dem.g[2] == 0.0
