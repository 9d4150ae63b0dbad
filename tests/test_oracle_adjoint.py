"""Pins of the oracle adjoint: a plain-PyTorch CPU FP64 statement of the step
(oracle/torch_step.py) whose autograd vector-Jacobian products are the
reference for the GPU adjoint.  Its forward must equal the C oracle, and its
derivatives must equal central differences of the C oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from helpers import CASES, case_particles
from oracle import torch_step as TS


def _c_J(lat, f0, p, lam, gF, gT, steps=1):
    L = oracle.Lattice(lat, f0)
    for _ in range(steps):
        F, T = L.step(p)
    return float((lam * L.f.reshape(lat.q, -1)).sum() + (gF * F).sum() + (gT * T).sum())


def _torch_J(lat, f0, p, lam, gF, gT, steps=1):
    geo = TS.Geometry(lat)
    f = torch.tensor(f0.reshape(lat.q, -1), requires_grad=True)
    X = torch.tensor(p.x, requires_grad=True)
    U = torch.tensor(p.u, requires_grad=True)
    Wt = torch.tensor(p.omega, requires_grad=True)
    fu = torch.tensor(np.asarray(lat.face_u, dtype=np.float64), requires_grad=True)
    g = f
    for _ in range(steps):
        g, F, T = TS.step(geo, g, X, U, Wt, p.r, fu)
    J = (torch.from_numpy(lam) * g).sum() + (torch.from_numpy(gF) * F).sum() + \
        (torch.from_numpy(gT) * T).sum()
    ins = [f, X, U, Wt, fu]
    grads = torch.autograd.grad(J, ins, allow_unused=True)
    grads = [torch.zeros_like(a) if gr is None else gr for a, gr in zip(ins, grads)]
    return float(J), g.detach().numpy(), [t.numpy() for t in grads]


@pytest.mark.parametrize("name", sorted(CASES))
def test_torch_statement_equals_c_oracle(name):
    lat = CASES[name]
    p = case_particles(lat)
    f0 = W.random_state(lat, 12)
    ref = oracle.Lattice(lat, f0)
    Fr, Tr = ref.step(p)
    geo = TS.Geometry(lat)
    fn, F, T = TS.step(geo, torch.from_numpy(f0.reshape(lat.q, -1)), torch.from_numpy(p.x),
                       torch.from_numpy(p.u), torch.from_numpy(p.omega), p.r,
                       torch.tensor(np.asarray(lat.face_u, dtype=np.float64)))
    assert np.abs(fn.numpy() - ref.f.reshape(lat.q, -1)).max() < 1e-14
    assert np.abs(F.numpy() - Fr).max() <= 1e-13 * np.abs(Fr).max()
    assert np.abs(T.numpy() - Tr).max() <= 1e-13 * max(np.abs(Tr).max(), 1e-30)


@pytest.mark.parametrize("name,steps", [(n, 1) for n in sorted(CASES)] + [("d2q9_open", 4)])
def test_vjp_matches_central_differences_of_c_oracle(name, steps):
    lat = CASES[name]
    p = case_particles(lat)
    f0 = W.random_state(lat, 12)
    rng = np.random.default_rng(31)
    lam = rng.normal(size=(lat.q, lat.ncells))
    gF = rng.normal(size=(p.n, 3))
    gT = rng.normal(size=(p.n, 3))
    if lat.q == 9:
        gF[:, 2] = 0
        gT[:, :2] = 0
    J, _, (gf, gX, gU, gW, gfu) = _torch_J(lat, f0, p, lam, gF, gT, steps)
    assert J == pytest.approx(_c_J(lat, f0, p, lam, gF, gT, steps), rel=1e-12)

    def fd(perturb, h):
        # perturb(h) -> (f0, particles, lattice spec) for the C oracle
        fa, pa, la = perturb(h)
        fb, pb, lb = perturb(-h)
        return (_c_J(la, fa, pa, lam, gF, gT, steps) - _c_J(lb, fb, pb, lam, gF, gT, steps)) / (2 * h)

    # f: J is quadratic-ish in f, central differences are accurate
    df = rng.normal(size=f0.shape) * 1e-2
    d = fd(lambda h: (f0 + h * df, p, lat), 1e-4)
    assert d == pytest.approx((gf * df.reshape(lat.q, -1)).sum(), rel=1e-7, abs=1e-9)
    # particle position, velocity, angular velocity
    for arr, grad, h in (("x", gX, 1e-6), ("u", gU, 1e-5), ("omega", gW, 1e-5)):
        v = rng.normal(size=(p.n, 3))
        if lat.q == 9:
            if arr == "omega":
                v[:, :2] = 0
            else:
                v[:, 2] = 0

        def pert(hh, arr=arr, v=v):
            q2 = p.copy()
            setattr(q2, arr, getattr(q2, arr) + hh * v)
            return f0, q2, lat
        d = fd(pert, h)
        assert d == pytest.approx((grad * v).sum(), rel=2e-5, abs=1e-9), arr
    # face velocities (inlet / moving walls)
    if any(k in ("inlet_eq", "moving_wall") for k in lat.faces):
        v = rng.normal(size=(6, 3))
        if lat.q == 9:
            v[:, 2] = 0

        def pertf(hh):
            fu = tuple(tuple(np.asarray(lat.face_u[k]) + hh * v[k]) for k in range(6))
            return f0, p, lat.replace(face_u=fu)
        # one step: J is at most quadratic in the face velocities (exact at any h)
        d = fd(pertf, 1e-3 if steps == 1 else 1e-5)
        assert d == pytest.approx((gfu * v).sum(), rel=1e-6, abs=1e-9)
