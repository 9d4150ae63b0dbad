"""Drag on a fixed sphere (Sec. 3.2) on the GPU: an equilibrium inlet and five
constant-pressure outlets (the open side faces), so outlet faces on every
axis, their edges and corners.  Parity with the oracle on a small box, then
the steady drag coefficient against Schiller-Naumann (Eq. 33) at Re_p = 10."""
import numpy as np
import pytest

import workloads as W
from helpers import _print_case, force_scale, gpu_lattice, gpu_run, oracle_run, relerr

pytestmark = pytest.mark.gpu


def test_drag_box_parity():
    w = W.sphere_drag(4, 10.0)
    lat, p = w.lattice, w.particles
    _print_case(test="drag box parity", shape=(lat.nx, lat.ny, lat.nz))
    f0 = W.random_state(lat, 31, amp=1e-3)
    for steps in (1, 3):
        ref, F_ref, _ = oracle_run(lat, f0, p, steps)
        _, f, F, _ = gpu_run(lat, f0, p, steps)
        assert relerr(f, ref.f) < 1e-12
        prev, _, _ = oracle_run(lat, f0, p, steps - 1)
        scale = force_scale(lat, prev.f, p)
        assert np.all(np.abs(F - F_ref).max(axis=1) <= 1e-12 * scale + 1e-300)


def test_drag_coefficient_re10():
    import paper_1901_09745_amd.psclbm as P
    dp, re, u0 = 10, 10.0, 0.05
    w = W.sphere_drag(dp, re, u0)
    G = gpu_lattice(w.lattice, w.particles)
    G.rasterize(P.DeviceParticles.from_host(w.particles))
    steps, prev = 0, None
    min_steps = int(5 * w.lattice.nx / u0)   # five flow-through times
    while steps < 100000:
        G.step(1000)
        steps += 1000
        F, _ = G.forces()
        fx = float(F[0, 0])
        if steps >= min_steps and prev is not None and abs(fx - prev) < 1e-5 * abs(fx):
            break
        prev = fx
    cd = W.drag_coefficient(fx, u0, dp)
    err = cd / W.schiller_naumann(re) - 1
    print(f"C_d = {cd:.4f} after {steps} steps, Eq. 33 {W.schiller_naumann(re):.4f}, "
          f"error {err:+.4f}", flush=True)
    assert steps < 100000
    assert abs(err) < 0.05
