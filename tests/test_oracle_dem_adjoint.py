"""Pins of the differentiable DEM statement (oracle/torch_dem.py), the
reference for the GPU adjoint of a DEM step: its forward equals the C
oracle's step with the contact set that step formed, and its vector-Jacobian
products equal central differences of the C oracle's step, for JKR (with
bonded pairs past zero overlap) and Hertz contacts, pairs and walls, 2D and
3D."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from oracle import torch_dem


def _start(name):
    """The seeded initial state of a case: lat, dem, particles, F, T."""
    if name.startswith("2d"):
        lat = W.LatticeSpec(q=9, nx=64, ny=48, faces=(W.PERIODIC, W.PERIODIC, W.BOUNCE_BACK,
                                                       W.BOUNCE_BACK, W.PERIODIC, W.PERIODIC))
        rng = np.random.default_rng(41)
        r = np.sort(rng.uniform(4.0, 6.0, 14))[::-1].copy()
        x = W.rsa(rng, r, (64.0, 48.0), (True, False), gap=0.05)
        u = rng.normal(0.0, 2e-3, (14, 3))
        u[:, 2] = 0.0
        g = (0.0, -2e-4, 0.0)
    else:
        lat = W.LatticeSpec(q=19, nx=32, ny=24, nz=24,
                            faces=(W.BOUNCE_BACK, W.BOUNCE_BACK) + (W.PERIODIC,) * 4)
        rng = np.random.default_rng(42)
        r = np.sort(rng.uniform(3.0, 5.0, 16))[::-1].copy()
        x = W.rsa(rng, r, (32.0, 24.0, 24.0), (False, True, True), gap=0.05)
        u = rng.normal(0.0, 2e-3, (16, 3))
        g = (-2e-4, 0.0, 0.0)
    gamma = 0.0 if name.endswith("hertz") else 1e-5
    dem = W.DemSpec(g=g, E_p=1e-3, gamma=gamma, eta_n=0.05)
    p = W.Particles(x, u, rng.normal(0.0, 1e-4, (len(r), 3)), r)
    F = rng.normal(0.0, 1e-4, (len(r), 3))
    T = rng.normal(0.0, 1e-4, (len(r), 3))
    return lat, dem, p, F, T


SETTLE = 300                                # steps into contacts, walls and pairs


def _case(name):
    lat, dem, p, F, T = _start(name)
    D = oracle.Dem(lat, dem, p.n)
    for _ in range(SETTLE):
        D.step(p, F, T)
    return lat, dem, p, F, T, D


def _c_step(lat, dem, D, p, F, T):
    """The C oracle's step from D's contact state, leaving D untouched."""
    E = oracle.Dem(lat, dem, p.n)
    E.ncontact[:] = D.ncontact
    E.ids[:] = D.ids
    E.hist[:] = D.hist
    q = p.copy()
    E.step(q, F, T)
    return q, E.contacts()


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, requires_grad=True)


CASES = ["2d_jkr", "3d_jkr", "3d_hertz"]


@pytest.mark.parametrize("name", CASES)
def test_forward_equals_c_oracle(name):
    lat, dem, p, F, T, D = _case(name)
    q, contacts = _c_step(lat, dem, D, p, F, T)
    assert sum(len(c) for c in contacts) > 4
    X, U, Wt = torch_dem.dem_step(lat, dem, _t(p.x), _t(p.u), _t(p.omega), list(p.r), _t(F),
                                  _t(T), contacts)
    assert np.abs(X.detach().numpy() - q.x).max() < 1e-12
    assert np.abs(U.detach().numpy() - q.u).max() < 1e-15
    assert np.abs(Wt.detach().numpy() - q.omega).max() < 1e-15


@pytest.mark.parametrize("name", CASES)
def test_vjp_matches_central_differences_of_c_oracle(name):
    lat, dem, p, F, T, D = _case(name)
    _, contacts = _c_step(lat, dem, D, p, F, T)
    rng = np.random.default_rng(7)
    a, b, c = (rng.normal(size=(p.n, 3)) for _ in range(3))
    if lat.q == 9:
        for m in (a, b):
            m[:, 2] = 0.0
        c[:, :2] = 0.0

    def J(q):
        return float((a * q.x).sum() + 1e3 * (b * q.u).sum() + 1e3 * (c * q.omega).sum())

    ins = [_t(p.x), _t(p.u), _t(p.omega), _t(F), _t(T)]
    X, U, Wt = torch_dem.dem_step(lat, dem, ins[0], ins[1], ins[2], list(p.r), ins[3], ins[4],
                                  contacts)
    Jt = (torch.from_numpy(a) * X).sum() + 1e3 * (torch.from_numpy(b) * U).sum() + \
        1e3 * (torch.from_numpy(c) * Wt).sum()
    grads = torch.autograd.grad(Jt, ins)
    # the particles in contact, where the contact terms act
    touching = [i for i in range(p.n) if contacts[i]]
    checked = 0
    for k, h in ((0, 1e-6), (1, 1e-7), (2, 1e-7), (3, 1e-6), (4, 1e-6)):
        for i in touching[:6]:
            for ax in range(3 if lat.q == 19 else 2):
                if k == 2 and lat.q == 9:
                    ax = 2
                if k == 4 and lat.q == 9:
                    ax = 2
                vals = []
                for sgn in (1.0, -1.0):
                    pp, Fp, Tp = p.copy(), F.copy(), T.copy()
                    arr = [pp.x, pp.u, pp.omega, Fp, Tp][k]
                    arr[i, ax] += sgn * h
                    q, cs = _c_step(lat, dem, D, pp, Fp, Tp)
                    assert cs == contacts                       # the contact set held
                    vals.append(J(q))
                fd = (vals[0] - vals[1]) / (2 * h)
                ad = float(grads[k][i, ax])
                assert ad == pytest.approx(fd, rel=1e-5, abs=1e-7 * max(1.0, abs(fd))), (k, i, ax)
                checked += 1
    assert checked > 20
