"""GPU adjoint (lbm_step_adjoint, psc_rasterize_adjoint) against the oracle
adjoint (autograd of the plain-PyTorch FP64 statement of the step, pinned in
tests/test_oracle_adjoint.py) and against central differences of the C
oracle.  FP64: agreement within 1e-11 relative."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from helpers import CASES, case_particles, gpu_lattice
from oracle import torch_step as TS

pytestmark = pytest.mark.gpu


def _oracle_vjp(lat, f0, p, lam, gF, gT):
    geo = TS.Geometry(lat)
    f = torch.tensor(f0.reshape(lat.q, -1), requires_grad=True)
    X = torch.tensor(p.x, requires_grad=True)
    U = torch.tensor(p.u, requires_grad=True)
    Wt = torch.tensor(p.omega, requires_grad=True)
    fu = torch.tensor(np.asarray(lat.face_u, dtype=np.float64), requires_grad=True)
    g, F, T = TS.step(geo, f, X, U, Wt, p.r, fu)
    J = (torch.from_numpy(lam) * g).sum() + (torch.from_numpy(gF) * F).sum() + \
        (torch.from_numpy(gT) * T).sum()
    ins = [f, X, U, Wt, fu]
    gr = torch.autograd.grad(J, ins, allow_unused=True)
    return [np.zeros(a.shape) if t is None else t.numpy() for a, t in zip(ins, gr)]


def _gpu_vjp(lat, f0, p, lam, gF, gT):
    import paper_1901_09745_amd.psclbm as P
    G = gpu_lattice(lat, p)
    dp = P.DeviceParticles.from_host(p)
    G.rasterize(dp)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    f = d(f0.reshape(lat.q, -1))
    lam_in = d(lam)
    lam_out = torch.empty_like(lam_in)
    gX = torch.zeros((p.n, 3), dtype=torch.float64, device="cuda")
    gU, gW = torch.zeros_like(gX), torch.zeros_like(gX)
    gface = torch.zeros((6, 3), dtype=torch.float64, device="cuda")
    P.lbm_step_adjoint(G.ctx, f, lam_in, lam_out, d(gF), d(gT), gX, gU, gW, gface)
    G.sync()
    return [t.cpu().numpy() for t in (lam_out, gX, gU, gW, gface)]


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("name", sorted(CASES))
def test_one_step_adjoint_matches_oracle_vjp(name):
    lat = CASES[name]
    print(f"case: {name}", flush=True)
    p = case_particles(lat)
    f0 = W.random_state(lat, 12)
    rng = np.random.default_rng(41)
    lam = rng.normal(size=(lat.q, lat.ncells))
    gF = rng.normal(size=(p.n, 3))
    gT = rng.normal(size=(p.n, 3))
    if lat.q == 9:
        gF[:, 2] = 0
        gT[:, :2] = 0
    ref = _oracle_vjp(lat, f0, p, lam, gF, gT)
    got = _gpu_vjp(lat, f0, p, lam, gF, gT)
    names = ["dJ/df", "dJ/dX", "dJ/dU", "dJ/dOmega", "dJ/dface_u"]
    for nm, a, b in zip(names, got, ref):
        b = b.reshape(a.shape)
        if np.abs(b).max() == 0:
            assert np.abs(a).max() < 1e-12, nm
        else:
            assert _rel(a, b) < 1e-11, (nm, _rel(a, b))


@pytest.mark.parametrize("q", [9, 19])
def test_rasterize_adjoint_matches_central_differences(q):
    import paper_1901_09745_amd.psclbm as P
    lat = CASES["d2q9_periodic"] if q == 9 else CASES["d3q19_periodic"]
    p = case_particles(lat)
    rng = np.random.default_rng(43)
    g = rng.normal(size=(lat.ncells, 4))

    def J(x):
        nslot, ids, eps, _ = oracle.rasterize(lat, x, p.r)
        e = np.where(np.arange(oracle.KMAX)[None, :] < nslot[:, None], eps, 0.0)[:, :4]
        return float((g * e).sum())

    G = gpu_lattice(lat, p)
    G.rasterize(P.DeviceParticles.from_host(p))
    gX = torch.zeros((p.n, 3), dtype=torch.float64, device="cuda")
    P.psc_rasterize_adjoint(G.ctx, torch.from_numpy(g).cuda(), 4, gX)
    G.sync()
    gX = gX.cpu().numpy()
    for _ in range(3):
        v = rng.normal(size=(p.n, 3))
        if q == 9:
            v[:, 2] = 0
        h = 1e-7
        d = (J(p.x + h * v) - J(p.x - h * v)) / (2 * h)
        assert d == pytest.approx((gX * v).sum(), rel=1e-5, abs=1e-8)
