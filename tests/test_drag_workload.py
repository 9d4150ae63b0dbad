"""The fixed-sphere drag case of Sec. 3.2 as a synthetic workload (CPU):
Eq. 32 and Eq. 33 against each other in the Stokes limit, and the box."""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("re", [1e-3, 1e-2])
def test_eq32_of_stokes_drag_is_eq33_limit(re):
    # Stokes drag 3 pi mu d U through Eq. 32 is 24 / Re_p, the Re_p -> 0 limit
    # of Eq. 33 (whose correction 0.15 Re^0.687 then vanishes)
    dp, u0 = 10.0, 0.01
    nu = u0 * dp / re
    cd = W.drag_coefficient(3 * np.pi * nu * dp * u0, u0, dp)
    assert cd == pytest.approx(24.0 / re, rel=1e-13)
    assert W.schiller_naumann(re) / cd - 1 == pytest.approx(0.15 * re ** 0.687, rel=1e-12)


def test_box_and_viscosity():
    w = W.sphere_drag(10, 50.0, u0=0.05)
    lat, p = w.lattice, w.particles
    assert (lat.nx, lat.ny, lat.nz) == (200, 100, 100)
    assert p.n == 1 and p.r[0] == 5.0
    assert np.allclose(p.x[0], [99.5, 49.5, 49.5])
    nu = (lat.tau - 0.5) / 3.0
    assert 0.05 * 10 / nu == pytest.approx(50.0, rel=1e-13)
    assert lat.faces == (W.INLET_EQ,) + (W.OUTLET_EQ,) * 5
    assert lat.face_u[0] == (0.05, 0.0, 0.0)
