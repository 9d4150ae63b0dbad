"""Error paths of the C ABI on the GPU, each forced from the host so that
every kernel still exits normally: capacity overflows, invalid radii, calls
out of order, and a non-finite state."""
import numpy as np
import pytest

import workloads as W
from helpers import gpu_lattice

pytestmark = pytest.mark.gpu


def _P():
    import paper_1901_09745_amd.psclbm as P
    return P


def test_step_before_rasterize_is_a_state_error():
    P = _P()
    G = P.Lattice(W.LatticeSpec(q=9, nx=64, ny=16), "fp64")
    with pytest.raises(P.PsclbmError) as e:
        G.step(1)
    assert e.value.code == P.ESTATE


def test_cell_slot_overflow():
    # five spheres on nearly one spot: cells covered by more than four
    P = _P()
    lat = W.LatticeSpec(q=19, nx=32, ny=32, nz=32)
    x = np.array([[16.0 + 0.1 * k, 16.0, 16.0] for k in range(5)])
    p = W.Particles(x, np.zeros((5, 3)), np.zeros((5, 3)), np.full(5, 3.0))
    G = gpu_lattice(lat, p)
    G.rasterize(P.DeviceParticles.from_host(p))
    G.step(1)
    with pytest.raises(P.PsclbmError) as e:
        G.sync()
    assert e.value.code == P.ESLOTS
    G.sync()  # the flag is cleared once reported


def test_tile_list_overflow():
    P = _P()
    lat = W.LatticeSpec(q=9, nx=128, ny=64)
    x = np.array([[20.0, 30.0, 0], [40.0, 30.0, 0], [60.0, 30.0, 0]])
    p = W.Particles(x, np.zeros((3, 3)), np.zeros((3, 3)), np.full(3, 6.0))
    G = gpu_lattice(lat, p, cap=2)
    G.rasterize(P.DeviceParticles.from_host(p))
    with pytest.raises(P.PsclbmError) as e:
        G.sync()
    assert e.value.code == P.ESLOTS


def test_invalid_radius_is_sticky_einval():
    P = _P()
    lat = W.LatticeSpec(q=19, nx=32, ny=32, nz=32)
    p = W.Particles(np.array([[10.0, 10.0, 10.0]]), np.zeros((1, 3)), np.zeros((1, 3)),
                    np.array([0.5]))   # r^2 = 1/4 <= 1/2: outside the domain of Eq. 17
    G = gpu_lattice(lat, p, rmax=1.0)
    G.rasterize(P.DeviceParticles.from_host(p))
    with pytest.raises(P.PsclbmError) as e:
        G.sync()
    assert e.value.code == P.EINVAL


@pytest.mark.parametrize("kind", ["jkr", "friction", "hertz"])
def test_contact_overflow(kind):
    # particle 0 touches two others with room for one contact: the contact
    # kernel (in each instantiation) keeps the first and raises ECONTACTS
    P = _P()
    print(f"case: contact overflow, {kind}", flush=True)
    lat = W.LatticeSpec(q=9, nx=64, ny=64)
    x = np.array([[20.0, 20.0, 0], [27.9, 20.0, 0], [12.1, 20.0, 0]])
    p = W.Particles(x, np.zeros((3, 3)), np.zeros((3, 3)), np.full(3, 4.0))
    G = P.Lattice(lat, "fp64", max_particles=3, max_radius=4.0, max_contacts=1)
    dp = P.DeviceParticles.from_host(p)
    dem = {"jkr": W.DemSpec(), "hertz": W.DemSpec(gamma=0.0),
           "friction": W.DemSpec(mu_f=0.3, k_t=1e-3, eta_t=0.02, theta_r=0.01)}[kind]
    G.dem_step(P.make_dem_params(dem), dp, dp.u * 0, dp.u * 0)
    with pytest.raises(P.PsclbmError) as e:
        G.sync()
    assert e.value.code == P.ECONTACTS


def test_nonfinite_mass():
    import torch
    P = _P()
    lat = W.LatticeSpec(q=9, nx=64, ny=8)
    G = P.Lattice(lat, "fp32")
    f = torch.from_numpy(W.random_state(lat, 3)).cuda()
    f[2, 0, 3, 5] = float("nan")
    G.set_f(f)
    with pytest.raises(P.PsclbmError) as e:
        G.mass()
    assert e.value.code == P.ENONFINITE


def test_argument_errors():
    P = _P()
    lat = W.LatticeSpec(q=9, nx=64, ny=8)
    G = P.Lattice(lat, "fp64", max_particles=2, max_radius=3.0)
    with pytest.raises(P.PsclbmError) as e:
        G.step(0)
    assert e.value.code == P.EINVAL
    x = np.zeros((3, 3))
    p = W.Particles(x, x, x, np.ones(3) * 2)
    with pytest.raises(P.PsclbmError) as e:   # more particles than max_particles
        G.rasterize(P.DeviceParticles.from_host(p))
    assert e.value.code == P.EINVAL


def test_coupled_step_argument_errors():
    P = _P()
    lat = W.LatticeSpec(q=9, nx=64, ny=32)
    G = P.Lattice(lat, "fp64", max_particles=2, max_radius=3.0)
    x = np.array([[20.0, 10.0, 0.0], [40.0, 20.0, 0.0]])
    p = W.Particles(x, np.zeros((2, 3)), np.zeros((2, 3)), np.array([3.0, 2.5]))
    dp = P.DeviceParticles.from_host(p)
    prm = P.make_dem_params(W.DemSpec())
    for nsteps in (0, -1):
        with pytest.raises(P.PsclbmError) as e:
            G.coupled_step(prm, dp, nsteps)
        assert e.value.code == P.EINVAL
    bad = P.make_dem_params(W.DemSpec(n_sub=0))
    with pytest.raises(P.PsclbmError) as e:
        G.coupled_step(bad, dp, 1)
    assert e.value.code == P.EINVAL
    bad = P.make_dem_params(W.DemSpec(poisson=0.5))
    with pytest.raises(P.PsclbmError) as e:
        G.coupled_step(bad, dp, 1)
    assert e.value.code == P.EINVAL
    three = W.Particles(np.zeros((3, 3)), np.zeros((3, 3)), np.zeros((3, 3)), np.ones(3) * 2)
    with pytest.raises(P.PsclbmError) as e:   # more particles than max_particles
        G.coupled_step(prm, P.DeviceParticles.from_host(three), 1)
    assert e.value.code == P.EINVAL
    import ctypes
    rc = P.load().coupled_step(G.ctx, ctypes.byref(prm), None, None, None, None, 2, 1)
    assert rc == P.EINVAL   # null particle arrays
    # a valid call still works after the rejected ones, and the state moved
    G.coupled_step(prm, dp, 3)
    assert P.lbm_step_count(G.ctx) == 3
    G.sync()
