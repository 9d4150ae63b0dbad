"""Differentiable FP64 statement of one frictionless DEM step -- TEST
INFRASTRUCTURE ONLY.

The same sub-step as ``or_dem_step`` in ``psc_oracle.c`` (Sec. 2.5, Eq. 21
with the JKR normal force of Eqs. 25-27, or Hertz's without adhesion, the
normal damping of Eq. 26, gravity and the frozen hydrodynamic force and
torque), written in plain PyTorch CPU ops so that ``torch.autograd`` supplies
exact vector-Jacobian products: the reference for the GPU adjoint of a DEM
step.  The contact set is an input (the one the C oracle's step formed), so
the statement is the step with its contact decisions held fixed; the
derivative of the jump-on / pull-off switches is taken as zero, as for the
clamps of Table 1.  The JKR branch is solved by Newton's method in torch, so
that the derivative of the contact radius comes from differentiating the
converged iteration (the implicit function), not from a hand-written
formula.  The forward is pinned to the C oracle, and the derivatives to
central differences of the C oracle, by ``tests/test_oracle_dem_adjoint.py``.
"""
from __future__ import annotations

import math

import torch


def normal_force(R: float, E: float, gamma: float, delta: torch.Tensor) -> torch.Tensor:
    """Elastic normal force (repulsive positive) at overlap delta: JKR on its
    stable branch (Eqs. 26-27, F/F_C = 4 (x^3 - x^{3/2}) with
    delta/delta_C = 6^{1/3} (2 x^2 - 4/3 x^{1/2})), or Hertz for gamma = 0."""
    if gamma == 0.0:
        d = torch.clamp(delta, min=0.0)
        return 4.0 / 3.0 * E * math.sqrt(R) * d * torch.sqrt(d)
    FC = 3.0 * math.pi * gamma * R
    a0 = (9.0 * math.pi * gamma * R * R / E) ** (1.0 / 3.0)
    dC = a0 * a0 / (2.0 * 6.0 ** (1.0 / 3.0) * R)
    target = delta / dC / 6.0 ** (1.0 / 3.0)          # 2 s^4 - 4/3 s, s = x^{1/2}
    sC = 6.0 ** (-1.0 / 3.0)
    gC = 2.0 * sC ** 4 - 4.0 / 3.0 * sC
    s = torch.clamp((1.5 * torch.clamp(target, min=0.0).detach()) ** 0.25, min=1.0)
    for _ in range(80):
        s = s - (2.0 * s ** 4 - 4.0 / 3.0 * s - target) / (8.0 * s ** 3 - 4.0 / 3.0)
    s = torch.where(target <= gC, torch.full_like(s, sC), s)
    x = s * s
    return 4.0 * FC * (x ** 3 - x * s)


def dem_step(lat, dem, X, U, W, R, Ff, Tf, contacts):
    """One DEM step (n_sub = 1) of n particles: X, U, W (n, 3) tensors, R a
    sequence of radii, Ff, Tf (n, 3) tensors, contacts[i] the partners of i
    (particle ids, walls -1-face).  Returns X', U', W'."""
    two_d = lat.q == 9
    L = (lat.nx, lat.ny, lat.nz)
    periodic = [lat.faces[2 * a] == "periodic" for a in range(3)]
    E = 1.0 / (2.0 * (1.0 - dem.poisson ** 2) / dem.E_p)      # Eq. 25, identical bodies
    dt = dem.dt
    n = X.shape[0]
    D = 2 if two_d else 3
    fc = [torch.zeros(3, dtype=torch.float64) for _ in range(n)]
    for i in range(n):
        for c in contacts[i]:
            if c < 0:
                face = -1 - c
                a = face // 2
                sgn = -1.0 if face % 2 == 0 else 1.0               # normal towards the wall
                dist = X[i, a] + 0.5 if face % 2 == 0 else (L[a] - 0.5) - X[i, a]
                delta = R[i] - dist
                vrn = -U[i, a] * sgn
                g = (-normal_force(R[i], E, dem.gamma, delta) + dem.eta_n * vrn) * sgn
                e = torch.zeros(3, dtype=torch.float64)
                e[a] = 1.0
                fc[i] = fc[i] + g * e
            else:
                j = c
                parts = []
                for a in range(3):
                    if a == 2 and two_d:
                        parts.append(torch.zeros((), dtype=torch.float64))
                        continue
                    d = X[j, a] - X[i, a]
                    if periodic[a]:
                        d = d - L[a] * torch.round(d.detach() / L[a])
                    parts.append(d)
                dv = torch.stack(parts)
                dist = torch.sqrt((dv * dv).sum())
                nrm = dv / dist
                delta = R[i] + R[j] - dist
                Reff = 1.0 / (1.0 / R[i] + 1.0 / R[j])
                vrn = ((U[j] - U[i]) * nrm).sum()
                fc[i] = fc[i] + (-normal_force(Reff, E, dem.gamma, delta) + dem.eta_n * vrn) * nrm
    Xn, Un, Wn = [], [], []
    for i in range(n):
        r = R[i]
        V = math.pi * r * r if two_d else 4.0 / 3.0 * math.pi * r ** 3
        m = dem.rho_p * V
        I = 0.5 * m * r * r if two_d else 0.4 * m * r * r
        ux, xx, wx = [], [], []
        for a in range(3):
            if a < D:
                G = (dem.rho_p - dem.rho_f) * V * dem.g[a]
                ua = U[i, a] + dt * (Ff[i, a] + fc[i][a] + G) / m
                xa = X[i, a] + dt * ua
                if periodic[a]:
                    xa = xa - L[a] * torch.floor(xa.detach() / L[a])
            else:
                ua, xa = U[i, a], X[i, a]
            ux.append(ua)
            xx.append(xa)
            if two_d and a < 2:
                wx.append(W[i, a])
            else:
                wx.append(W[i, a] + dt * Tf[i, a] / I)
        Xn.append(torch.stack(xx))
        Un.append(torch.stack(ux))
        Wn.append(torch.stack(wx))
    return torch.stack(Xn), torch.stack(Un), torch.stack(Wn)
