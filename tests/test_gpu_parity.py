"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (FP64 form): distributions within 1e-12 of max|f|; per-particle
forces within 1e-12 of the L1 size of their Eq. 14 summands (the GPU sums them
in a different order with FP64 atomics).
"""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import (CASES, _particles, _print_case, case_particles, force_floor, force_scale,
                     gpu_lattice, gpu_run, oracle_run, relerr)

pytestmark = pytest.mark.gpu

@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("steps", [1, 2, 5])
def test_fluid_steps_parity(name, steps):
    lat = CASES[name]
    _print_case(test="fluid", name=name, steps=steps)
    f0 = W.random_state(lat, 11)
    ref, _, _ = oracle_run(lat, f0, None, steps)
    _, f, _, _ = gpu_run(lat, f0, None, steps)
    assert relerr(f, ref.f) < 1e-12


@pytest.mark.parametrize("name", sorted(CASES))
def test_psc_steps_parity(name):
    lat = CASES[name]
    _print_case(test="psc", name=name)
    if lat.q == 9:
        p = _particles(lat, 6, 4.0, 9.0, seed=3, overlap=True)
    else:
        p = _particles(lat, 5, 3.0, 5.0, seed=4, overlap=True)
    f0 = W.random_state(lat, 12)
    for steps in (1, 3):
        ref, F_ref, T_ref = oracle_run(lat, f0, p, steps)
        _, f, F, T = gpu_run(lat, f0, p, steps)
        assert relerr(f, ref.f) < 1e-12
        # the last step's forces start from the state after steps-1 steps
        prev, _, _ = oracle_run(lat, f0, p, steps - 1)
        scale = force_scale(lat, prev.f, p)
        assert np.all(np.abs(F - F_ref).max(axis=1) <= 1e-12 * scale + 1e-300)
        assert np.all(np.abs(T - T_ref).max(axis=1) <= 1e-12 * scale * 30 + 1e-300)


@pytest.mark.parametrize("name", ["d2q9_periodic", "d2q9_walls", "d3q19_periodic",
                                  "d3q19_walls"])
def test_original_weighting_parity(name):
    # Eqs. 7-9, 11: each particle weighted by its own fraction, B_n their sum
    # (above one where the shells of the overlapping particles cross), the
    # force weighted by B_n
    lat = CASES[name]
    _print_case(test="original weighting", name=name)
    p = case_particles(lat)
    f0 = W.random_state(lat, 12)
    for steps in (1, 3):
        ref, F_ref, T_ref = oracle_run(lat, f0, p, steps, mode=1)
        _, f, F, T = gpu_run(lat, f0, p, steps, weighting="original")
        assert relerr(f, ref.f) < 1e-12
        prev, _, _ = oracle_run(lat, f0, p, steps - 1, mode=1)
        scale = 2 * force_scale(lat, prev.f, p)   # B_n <= 2 with two covering particles
        assert np.all(np.abs(F - F_ref).max(axis=1) <= 1e-12 * scale + 1e-300)
        # where cells are shared by two particles the weighting matters
        if oracle.rasterize(lat, p.x, p.r)[0].max() > 1:
            ref0, _, _ = oracle_run(lat, f0, p, steps, mode=0)
            assert relerr(ref0.f, ref.f) > 1e-8


def test_original_weighting_has_no_adjoint():
    import torch
    import paper_1901_09745_amd.psclbm as P
    lat = CASES["d2q9_periodic"]
    p = case_particles(lat)
    G = gpu_lattice(lat, p, weighting="original")
    G.rasterize(P.DeviceParticles.from_host(p))
    q, N = lat.q, lat.ncells
    f = G.get_f().reshape(q, N)
    lam = torch.zeros_like(f)
    with pytest.raises(P.PsclbmError):
        P.lbm_step_adjoint(G.ctx, f, lam, torch.empty_like(lam))


@pytest.mark.parametrize("q", [9, 19])
def test_rasterize_parity(q):
    if q == 9:
        lat = W.LatticeSpec(q=9, nx=140, ny=90)
        p = _particles(lat, 12, 3.0, 10.0, seed=5, overlap=True)
    else:
        lat = W.LatticeSpec(q=19, nx=70, ny=40, nz=36)
        p = _particles(lat, 10, 2.5, 6.0, seed=6, overlap=True)
    _print_case(test="rasterize", q=q)
    nslot, ids, eps, ssum = oracle.rasterize(lat, p.x, p.r)
    assert nslot.max() <= 4
    G = gpu_lattice(lat, p)
    import paper_1901_09745_amd.psclbm as P
    G.rasterize(P.DeviceParticles.from_host(p))
    e, gid, geps = G.solid_fraction(4)
    G.sync()
    e = e.cpu().numpy().reshape(-1)
    gid = gid.cpu().numpy().reshape(-1, 4)
    geps = geps.cpu().numpy().reshape(-1, 4)
    assert np.allclose(e, np.minimum(ssum, 1.0), rtol=0, atol=1e-14)
    for k in range(4):
        ref_ids = np.where(nslot > k, ids[:, k], -1)
        assert np.array_equal(gid[:, k], ref_ids)
        ref_eps = np.where(nslot > k, eps[:, k], 0.0)
        assert np.allclose(geps[:, k], ref_eps, rtol=0, atol=1e-14)


def test_c1_full_run():
    # D2Q9 tau=0.8 200x100 channel, body force 1e-6, fixed disk r=10 at
    # (60,50), 2000 steps: full-run FP64 parity.
    w = W.c1()
    _print_case(test="c1", steps=w.steps)
    ref, F_ref, T_ref = oracle_run(w.lattice, None, w.particles, w.steps)
    _, f, F, T = gpu_run(w.lattice, None, w.particles, w.steps)
    df = float(np.abs(f - ref.f).max())
    assert df < 1e-12 * np.abs(ref.f).max()
    rho_r, u_r = ref.macros()
    Lg = oracle.Lattice(w.lattice, f)
    rho_g, u_g = Lg.macros()
    # Eq. 5 carries a state difference df into the velocity as at most
    # sum_i |df_i| (1 + |u|) / rho <= Q df (1 + |u|max) / rho_min per cell
    q = w.lattice.q
    umax = float(np.abs(u_r).max())
    du_bound = q * df * (1.0 + umax) / float(rho_r.min())
    print(f"f err {df:.3e}, u err {np.abs(u_g - u_r).max():.3e} (bound {du_bound:.3e})")
    assert np.abs(u_g - u_r).max() <= du_bound
    # the drag (Eq. 14) of the last step: the order-dependent rounding of its
    # sum (1e-12 of the L1 size of the summands, and the rounding floor of
    # u), plus the state difference carried by each covered cell's exchange
    # B rho (u_s - u) + F, at most B (|d rho| |u| + rho |du|) per cell
    nslot, _, _, _ = oracle.rasterize(w.lattice, w.particles.x, w.particles.r)
    ncov = int((nslot > 0).sum())
    F_bound = (1e-12 * force_scale(w.lattice, ref.f, w.particles)[0]
               + force_floor(w.lattice, ref.f, w.particles)[0]
               + ncov * (q * df * umax + float(rho_r.max()) * du_bound))
    print(f"drag err {np.abs(F[0, :2] - F_ref[0, :2]).max():.3e} (bound {F_bound:.3e}, "
          f"drag {F_ref[0, 0]:.3e})")
    assert np.abs(F[0, :2] - F_ref[0, :2]).max() <= F_bound


def test_mass_and_roundtrip():
    lat = CASES["d3q19_walls"]
    f0 = W.random_state(lat, 13)
    G, f, _, _ = gpu_run(lat, f0, None, 0 + 1)
    ref, _, _ = oracle_run(lat, f0, None, 1)
    m = G.mass()
    assert m == pytest.approx(ref.mass(), rel=1e-14)
    import torch
    G.set_f(torch.from_numpy(f0).cuda())
    assert np.array_equal(G.get_f().cpu().numpy(), f0)
    assert G.mass() == pytest.approx(oracle.Lattice(lat, f0).mass(), rel=1e-14)
