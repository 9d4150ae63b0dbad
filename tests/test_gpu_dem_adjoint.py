"""GPU dem_step_adjoint against torch autograd of the differentiable DEM
statement (oracle/torch_dem.py, itself pinned to central differences of the
C oracle): after the cases of tests/test_oracle_dem_adjoint.py have settled
into contacts (GPU and oracle in lockstep, so their contact histories
agree), the GPU takes one step from the oracle's state and its adjoint is
compared with the vector-Jacobian product over the oracle's contact set."""
import numpy as np
import pytest
import torch

import oracle
from helpers import gpu_lattice
from oracle import torch_dem
from test_oracle_dem_adjoint import CASES, SETTLE, _c_step, _start, _t

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", CASES)
def test_dem_step_adjoint_matches_autograd(name):
    import paper_1901_09745_amd.psclbm as P
    print(f"case: dem adjoint {name}", flush=True)
    lat, dem, p, F, T = _start(name)
    D = oracle.Dem(lat, dem, p.n)
    pr = p.copy()
    G = gpu_lattice(lat, p)
    dp = P.DeviceParticles.from_host(p)
    Fg = torch.from_numpy(F).cuda()
    Tg = torch.from_numpy(T).cuda()
    prm = P.make_dem_params(dem)
    for _ in range(SETTLE):
        D.step(pr, F, T)
        G.dem_step(prm, dp, Fg, Tg)
    G.sync()
    assert np.abs(dp.x.cpu().numpy() - pr.x).max() < 1e-9
    # one step from the oracle's state exactly
    for t, a in ((dp.x, pr.x), (dp.u, pr.u), (dp.omega, pr.omega)):
        t.copy_(torch.from_numpy(a))
    before = P.DeviceParticles.from_host(pr)
    G.dem_step(prm, dp, Fg, Tg)
    q, contacts = _c_step(lat, dem, D, pr, F, T)
    assert sum(len(c) for c in contacts) > 4
    G.sync()
    assert np.abs(dp.x.cpu().numpy() - q.x).max() < 1e-12
    rng = np.random.default_rng(9)
    a, b, c = (rng.normal(size=(p.n, 3)) for _ in range(3))
    if lat.q == 9:
        a[:, 2] = b[:, 2] = 0.0
        c[:, :2] = 0.0
    outs = G.dem_step_adjoint(prm, before, *(torch.from_numpy(m).cuda() for m in (a, b, c)))
    G.sync()
    ins = [_t(pr.x), _t(pr.u), _t(pr.omega), _t(F), _t(T)]
    X, U, Wt = torch_dem.dem_step(lat, dem, *ins[:3], list(pr.r), ins[3], ins[4], contacts)
    J = sum((torch.from_numpy(m) * v).sum() for m, v in ((a, X), (b, U), (c, Wt)))
    ref = torch.autograd.grad(J, ins)
    for k, (got, want) in enumerate(zip(outs, ref)):
        got, want = got.cpu().numpy(), want.numpy()
        scale = max(np.abs(want).max(), 1e-300)
        assert np.abs(got - want).max() <= 1e-10 * scale, (k, np.abs(got - want).max(), scale)


def test_adjoint_of_the_last_coupled_step():
    # coupled_step gathers the contacts in the step kernel; the adjoint of
    # its last DEM step reads those lists, with that step's fluid force
    import paper_1901_09745_amd.psclbm as P
    import workloads as W
    print("case: dem adjoint after coupled_step, 3d lattice block", flush=True)
    # a jittered block of spheres whose neighbours and bottom row overlap by
    # 0.02, so contacts are loaded from the first step
    lat = W.LatticeSpec(q=19, nx=32, ny=24, nz=24,
                        faces=(W.BOUNCE_BACK, W.BOUNCE_BACK) + (W.PERIODIC,) * 4)
    rng = np.random.default_rng(12)
    pts = [[2.48 + i * 5.98, 6.0 + j * 5.98, 6.0 + m * 5.98]
           for i in range(2) for j in range(3) for m in range(3)]
    n = len(pts)
    p = W.Particles(np.array(pts) + rng.normal(0.0, 0.005, (n, 3)),
                    rng.normal(0.0, 1e-3, (n, 3)), rng.normal(0.0, 2e-4, (n, 3)), np.full(n, 3.0))
    dem = W.DemSpec(g=(-2e-4, 0.0, 0.0), E_p=1e-3, gamma=1e-5, eta_n=0.05)
    ref = oracle.Lattice(lat)
    D = oracle.Dem(lat, dem, p.n)
    pr = p.copy()
    k = 20
    for t in range(k):
        if t == k - 1:
            before_h = pr.copy()
        F_ref, T_ref = ref.step(pr)
        D.step(pr, F_ref, T_ref)
    contacts = D.contacts()
    assert sum(len(c) for c in contacts) > 4
    G = gpu_lattice(lat, p)
    dp = P.DeviceParticles.from_host(p)
    prm = P.make_dem_params(dem)
    G.coupled_step(prm, dp, k - 1)
    before = P.DeviceParticles(dp.x.clone(), dp.u.clone(), dp.omega.clone(), dp.r)
    G.coupled_step(prm, dp, 1)
    G.sync()
    assert np.abs(dp.x.cpu().numpy() - pr.x).max() < 1e-9
    rng = np.random.default_rng(11)
    a, b, c = (rng.normal(size=(p.n, 3)) for _ in range(3))
    outs = G.dem_step_adjoint(prm, before, *(torch.from_numpy(m).cuda() for m in (a, b, c)))
    G.sync()
    ins = [_t(before_h.x), _t(before_h.u), _t(before_h.omega), _t(F_ref), _t(T_ref)]
    X, U, Wt = torch_dem.dem_step(lat, dem, *ins[:3], list(before_h.r), ins[3], ins[4], contacts)
    J = sum((torch.from_numpy(m) * v).sum() for m, v in ((a, X), (b, U), (c, Wt)))
    ref_g = torch.autograd.grad(J, ins)
    for kk, (got, want) in enumerate(zip(outs, ref_g)):
        got, want = got.cpu().numpy(), want.numpy()
        scale = max(np.abs(want).max(), 1e-300)
        # the GPU's pre-step state differs from the oracle's by the rounding of
        # the 39 coupled steps before it
        assert np.abs(got - want).max() <= 1e-7 * scale, (kk, np.abs(got - want).max(), scale)


def test_dem_step_adjoint_rejects_what_it_does_not_cover():
    import dataclasses
    import paper_1901_09745_amd.psclbm as P
    lat, dem, p, F, T = _start("2d_jkr")
    G = gpu_lattice(lat, p)
    dp = P.DeviceParticles.from_host(p)
    z = torch.zeros((p.n, 3), dtype=torch.float64, device="cuda")
    for bad in (dataclasses.replace(dem, n_sub=2), dataclasses.replace(dem, mu_f=0.3, k_t=1e-3),
                dataclasses.replace(dem, theta_r=0.01), dataclasses.replace(dem, kinematic=True)):
        with pytest.raises(P.PsclbmError) as e:
            G.dem_step_adjoint(P.make_dem_params(bad), dp, z, z, z)
        assert e.value.code == P.EINVAL
    G.sync()
