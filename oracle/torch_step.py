"""Differentiable FP64 statement of one oracle step -- TEST INFRASTRUCTURE ONLY.

The same per-step algorithm as ``psc_oracle.c`` (Secs. 2.1-2.4, Eqs. 1-6,
10, 12-14 and Table 1, with the readings listed there), written in plain
PyTorch CPU ops so that ``torch.autograd`` supplies exact vector-Jacobian
products.  These serve as the reference adjoint for the hand-written GPU
adjoint.  The forward is pinned to the C oracle, and the derivatives to central
differences of the C oracle, by ``tests/test_oracle_adjoint.py``.

All tensors are float64 on the CPU.  f has shape (Q, N) in the canonical
velocity order and cell order n = x + nx (y + ny z).
"""
from __future__ import annotations

import math

import numpy as np
import torch

_E9 = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
       (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)]
_W9 = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
_E19 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
        (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
        (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
_W19 = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12
_KIND = {"periodic": 0, "bounce_back": 1, "moving_wall": 2, "inlet_eq": 3, "outlet_eq": 4}


def _lattice(q):
    e = np.array(_E9 if q == 9 else _E19, dtype=np.int64)
    w = np.array(_W9 if q == 9 else _W19)
    opp = np.array([int(np.nonzero((e == -e[i]).all(axis=1))[0][0]) for i in range(q)])
    return e, w, opp


class Geometry:
    """Index maps of a lattice (no arithmetic of the method)."""

    def __init__(self, lat):
        self.lat = lat
        self.q = lat.q
        self.e, self.w, self.opp = _lattice(lat.q)
        self.dims = (lat.nx, lat.ny, lat.nz)
        self.N = lat.ncells
        self.periodic = [lat.periodic(a) for a in range(3)]
        nx, ny, nz = self.dims
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        self.coords = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
        # streaming: destination of f*_i(n); out-of-domain links reflect
        self.dest = np.zeros((self.q, self.N), dtype=np.int64)
        self.inside = np.zeros((self.q, self.N), dtype=bool)
        self.cross = np.zeros((self.q, self.N, 6))  # moving-wall faces a link leaves through
        for i in range(self.q):
            p = self.coords + self.e[i]
            ok = np.ones(self.N, dtype=bool)
            for a in range(3):
                L = self.dims[a]
                low, high = p[:, a] < 0, p[:, a] >= L
                if self.periodic[a]:
                    p[:, a] = np.mod(p[:, a], L)
                else:
                    ok &= ~(low | high)
                    for face, m in ((2 * a, low), (2 * a + 1, high)):
                        if lat.faces[face] == "moving_wall":
                            self.cross[i, m, face] = 1.0
            self.inside[i] = ok
            self.dest[i] = np.where(ok, p[:, 0] + nx * (p[:, 1] + ny * p[:, 2]),
                                    np.arange(self.N))


def feq(e_t, w_t, rho, u):
    """Eq. 3 for rho (M,) and u (M, 3): returns (Q, M)."""
    eu = e_t @ u.T
    uu = (u * u).sum(dim=1)
    return w_t[:, None] * rho[None, :] * (1 + 3 * eu + 4.5 * eu * eu - 1.5 * uu[None, :])


def step(geo: Geometry, f: torch.Tensor, X: torch.Tensor, U: torch.Tensor, W: torch.Tensor,
         R: np.ndarray, face_u: torch.Tensor):
    """One step.  Returns (f_new (Q, N), F (n, 3), T (n, 3)).  face_u (6, 3)
    carries the inlet / wall velocities (differentiable)."""
    lat = geo.lat
    q, N = geo.q, geo.N
    e_t = torch.as_tensor(geo.e, dtype=torch.float64)
    w_t = torch.as_tensor(geo.w, dtype=torch.float64)
    tau = lat.tau
    Fb = torch.tensor(list(lat.force), dtype=torch.float64)
    two_d = q == 9

    # --- inlet / outlet layers: every outlet takes its neighbour's velocity
    # from the state entering the step (before any reset), the later face
    # winning on a cell of two outlet faces; then the inlets ---
    f_in = f
    f = f.clone()
    resets = []
    for face in range(6):
        if lat.faces[face] != "outlet_eq":
            continue
        a = face // 2
        L = geo.dims[a]
        layer = 0 if face % 2 == 0 else L - 1
        cells = np.nonzero(geo.coords[:, a] == layer)[0]
        step_in = 1 if face % 2 == 0 else -1
        nbr = cells + step_in * (1 if a == 0 else (lat.nx if a == 1 else lat.nx * lat.ny))
        fn = f_in[:, nbr]
        rho_n = fn.sum(dim=0)
        resets.append((cells, ((e_t.T @ fn).T + 0.5 * Fb) / rho_n[:, None]))
    for face in range(6):
        if lat.faces[face] != "inlet_eq":
            continue
        a = face // 2
        layer = 0 if face % 2 == 0 else geo.dims[a] - 1
        cells = np.nonzero(geo.coords[:, a] == layer)[0]
        resets.append((cells, face_u[face].expand(len(cells), 3)))
    for cells, ub in resets:
        fe = feq(e_t, w_t, torch.full((len(cells),), lat.rho0, dtype=torch.float64), ub)
        f = f.index_copy(1, torch.as_tensor(cells), fe)

    # --- moments (Eq. 5), equilibrium (Eq. 3), Guo forcing (Eq. 4) ---
    rho = f.sum(dim=0)
    u = ((e_t.T @ f).T + 0.5 * Fb) / rho[:, None]
    fe = feq(e_t, w_t, rho, u)
    eu = e_t @ u.T
    eF = e_t @ Fb
    uF = (u * Fb).sum(dim=1)
    Fi = (1 - 1 / (2 * tau)) * w_t[:, None] * (3 * (eF[:, None] - uF[None, :]) + 9 * eu * eF[:, None])

    # --- Table 1 solid fractions, as (cell, particle) pairs ---
    h = lat.h
    pc, pp, peps, parm = [], [], [], []
    n = R.shape[0]
    for s in range(n):
        r = float(R[s])
        if two_d:
            va = 0.5 * math.sqrt(r * r - 0.25) + r * r * math.atan(0.5 / math.sqrt(r * r - 0.25))
        else:
            r2, sq = r * r, math.sqrt(r * r - 0.5)
            va = ((1 / 12 - r2) * math.atan(0.5 * sq / (0.5 - r2)) + sq / 3
                  + (r2 - 1 / 12) * math.atan(0.5 / sq) - 4 / 3 * r2 * r * math.atan(0.25 / (r * sq)))
        cs = va + 0.5
        xs = X[s].detach().numpy()
        rng = []
        for a in range(3):
            if a == 2 and two_d:
                rng.append(np.array([0]))
                continue
            lo, hi = math.ceil(xs[a] - (r + h)), math.floor(xs[a] + (r + h))
            k = np.arange(lo, hi + 1)
            L = geo.dims[a]
            if geo.periodic[a]:
                k = np.mod(k, L)
            else:
                k = k[(k >= 0) & (k < L)]
            rng.append(k)
        kz, ky, kx = np.meshgrid(rng[2], rng[1], rng[0], indexing="ij")
        cells = (kx + lat.nx * (ky + lat.ny * kz)).ravel()
        cc = torch.as_tensor(np.stack([kx.ravel(), ky.ravel(), kz.ravel()], axis=1),
                             dtype=torch.float64)
        d = cc - X[s]
        for a in range(3):
            if geo.periodic[a] and not (a == 2 and two_d):
                L = float(geo.dims[a])
                d[:, a] = torch.where(d[:, a] > 0.5 * L, d[:, a] - L,
                                      torch.where(d[:, a] < -0.5 * L, d[:, a] + L, d[:, a]))
        if two_d:
            d = torch.cat([d[:, :2], torch.zeros(len(cells), 1, dtype=torch.float64)], dim=1)
        dist = torch.sqrt((d * d).sum(dim=1))
        eps = torch.where(dist >= r + h, torch.zeros_like(dist),
                          torch.where(dist <= r - h, torch.ones_like(dist),
                                      torch.clamp(cs - dist, 0.0, 1.0)))
        keep = (eps > 0).detach().numpy()
        pc.append(cells[keep])
        pp.append(np.full(int(keep.sum()), s))
        peps.append(eps[torch.as_tensor(keep)])
        parm.append(d[torch.as_tensor(keep)])
    f_star = f - (f - fe) / tau + Fi  # pure-fluid update (B_n = 0)
    F = torch.zeros(max(n, 1), 3, dtype=torch.float64)
    T = torch.zeros(max(n, 1), 3, dtype=torch.float64)
    if n > 0 and sum(len(c) for c in pc) > 0:
        cells = torch.as_tensor(np.concatenate(pc))
        part = torch.as_tensor(np.concatenate(pp))
        eps = torch.cat(peps)
        arm = torch.cat(parm)
        S = torch.zeros(N, dtype=torch.float64).index_add(0, cells, eps)
        tm = tau - 0.5
        en = torch.clamp(S, max=1.0)
        Bn = en * tm / ((1 - en) + tm)
        Sp = S[cells]
        Bs = torch.where(Sp <= 1.0, eps * tm / ((1 - en[cells]) + tm), eps / Sp)
        # rigid-body velocity at the cell centre
        us = U[part] + torch.cross(W[part], arm, dim=1)
        rp = rho[cells]
        fs_pair = feq(e_t, w_t, rp, us)
        fp = f[:, cells]
        fe_pair = fe[:, cells]
        om = fp[geo.opp] - fe_pair[geo.opp] + fs_pair - fp          # Eq. 10
        # Eq. 12: (1 - B_n) on BGK and forcing, plus sum_s B_s Omega^s
        f_star = f - (1 - Bn)[None, :] * (f - fe) / tau + (1 - Bn)[None, :] * Fi
        f_star = f_star.index_add(1, cells, Bs[None, :] * om)
        # Eq. 14
        mom = Bs[:, None] * (om.T @ e_t)
        F = F.index_add(0, part, -mom)
        T = T.index_add(0, part, -torch.cross(arm, mom, dim=1))
    # --- streaming with bounce-back and the moving-wall term ---
    f_new = torch.zeros_like(f)
    for i in range(q):
        ins = torch.as_tensor(geo.inside[i])
        dest = torch.as_tensor(np.where(geo.inside[i], geo.dest[i], -1))
        src = f_star[i]
        # inside links move to the neighbour, slot i
        f_new[i] = f_new[i].index_add(0, dest[ins], src[ins])
        if (~geo.inside[i]).any():
            out = torch.as_tensor(np.nonzero(~geo.inside[i])[0])
            uwt = torch.as_tensor(geo.cross[i][~geo.inside[i]]) @ face_u   # wall velocity
            corr = 6 * geo.w[i] * rho[out] * (uwt @ e_t[i])
            f_new[geo.opp[i]] = f_new[geo.opp[i]].index_add(0, out, src[out] - corr)
    return f_new, F[:n], T[:n]


def run(lat, f0, X, U, W, R, face_u, steps, seed_F=None, seed_T=None):
    """J = sum over the last step of seed . F + seed . T, after `steps` steps
    with the particles held fixed.  Returns (J, f_final, F, T); the inputs
    may require grad."""
    geo = Geometry(lat)
    f = f0
    F = T = None
    for _ in range(steps):
        f, F, T = step(geo, f, X, U, W, R, face_u)
    J = torch.zeros((), dtype=torch.float64)
    if seed_F is not None:
        J = J + (seed_F * F).sum()
    if seed_T is not None:
        J = J + (seed_T * T).sum()
    return J, f, F, T
