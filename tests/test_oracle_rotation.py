"""Pins of the oracle's rotating-particle terms against closed forms.

Eq. 10 takes the solid velocity at a covered node as the particle's rigid-body
velocity there, u_s = U_s + Omega_s x (x_n - X_s), and Eq. 14 gives the torque
on the particle as minus the sum of (x_n - X_s) x m_{n,s}, with the momentum
exchange m_{n,s} = B_{n,s} sum_i Omega^s_i e_i.  Eq. 11 (the original scheme)
weighs each particle's exchange by the cell's total B_n instead.  The checks
below fix the sign and the arm of both terms, and the weight of Eq. 11 in
cells that two particles share, through special cases whose outcome follows
from the definitions alone:

* a rigid rotation of the fluid about a particle that spins with it is in
  equilibrium with the particle: the solid operator vanishes in every covered
  cell, so the force and torque are zero;
* in fluid at rest (f = f^eq(rho, 0), no body force), the first moment of
  Eq. 3 gives sum_i Omega^s_i e_i = rho u_s exactly, so F_s and T_s are sums
  of closed-form terms over the covered cells, with the fractions taken from
  the rasteriser (pinned on its own in test_oracle_solid_fraction.py) and the
  weights from Eqs. 9 and 13 (pinned in test_oracle_weights.py).

The arms and cross products here are numpy's, written independently of the
oracle.
"""
import numpy as np
import pytest

import oracle
import workloads as W


def _arms(lat, X):
    """x_n - X for every cell centre (nearest image on periodic axes), (N, 3)."""
    z, y, x = np.meshgrid(np.arange(lat.nz), np.arange(lat.ny), np.arange(lat.nx), indexing="ij")
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.float64)
    r = pts - np.asarray(X, dtype=np.float64)[None, :]
    for a, L in enumerate((lat.nx, lat.ny, lat.nz)):
        if a == 2 and lat.q == 9:
            r[:, 2] = 0.0
            continue
        if lat.periodic(a):
            r[:, a] -= L * np.round(r[:, a] / L)
    return r


def _box(q):
    if q == 9:
        return W.LatticeSpec(q=9, nx=28, ny=26, tau=0.75)
    return W.LatticeSpec(q=19, nx=22, ny=20, nz=18, tau=0.7)


def _spin(q, rng, scale):
    w = rng.uniform(-scale, scale, 3)
    if q == 9:
        w[:2] = 0.0
    return w


@pytest.mark.parametrize("q", [9, 19])
def test_rigid_rotation_with_the_particle_exerts_nothing(q):
    # f = f^eq(1, U + Omega x (x_n - X)) with the particle translating at U and
    # spinning at Omega: u = u_s in every covered cell, Omega^s = 0, F = T = 0.
    lat = _box(q)
    rng = np.random.default_rng(11 + q)
    X = np.array([13.37, 12.61, 8.83 if q == 19 else 0.0])
    U = np.array([2e-3, -1e-3, 1.5e-3 if q == 19 else 0.0])
    Om = _spin(q, rng, 1.5e-3)
    r = 5.3
    arms = _arms(lat, X)
    u = U[None, :] + np.cross(Om[None, :], arms)
    L = oracle.Lattice(lat)
    L.set_equilibrium(u=u)
    p = W.Particles(X[None, :].copy(), U[None, :].copy(), Om[None, :].copy(), np.array([r]))
    F, T = L.step(p)
    # the torque a mistaken arm or sign would give is of the order of the
    # moment of inertia of the covered cells times |Omega|
    nslot, ids, eps, _ = oracle.rasterize(lat, p.x, p.r)
    covered = nslot > 0
    inertia = (arms[covered] ** 2).sum() * np.abs(Om).max()
    assert covered.sum() > 50
    assert np.abs(F).max() < 1e-13 * inertia
    assert np.abs(T).max() < 1e-13 * inertia * r
    # and the fixed point is not vacuous: a particle spinning the other way
    # meets a torque of that order
    p.omega[:] = -Om
    L = oracle.Lattice(lat)
    L.set_equilibrium(u=u)
    F, T = L.step(p)
    assert np.abs(T).max() > 1e-2 * inertia


def _touching_pair(q):
    """Three particles whose shells overlap, so that some cells are covered
    by two of them."""
    if q == 9:
        X = np.array([[9.3, 10.6, 0.0], [16.0, 11.4, 0.0], [12.6, 16.9, 0.0]])
        R = np.array([4.2, 3.9, 3.6])
    else:
        X = np.array([[7.4, 8.3, 8.9], [13.6, 9.1, 9.4], [10.2, 13.7, 7.6]])
        R = np.array([3.4, 3.1, 2.9])
    return X, R


def _rest_fluid_exchange(lat, p, mode):
    """Per covered (cell, particle): the weight of Eq. 14 (mode 0: B_{n,s},
    Eq. 13 with the clamped total) or of Eq. 11 (mode 1: the cell's B_n,
    Eq. 8's sum of the Eq. 9 weights), and rho u_s in fluid at rest."""
    nslot, ids, eps, _ = oracle.rasterize(lat, p.x, p.r)
    F = np.zeros((p.n, 3))
    T = np.zeros((p.n, 3))
    scale = np.zeros(p.n)
    arms = [_arms(lat, p.x[s]) for s in range(p.n)]
    shared = 0
    for n in np.nonzero(nslot)[0]:
        k = nslot[n]
        Bn, Bs = oracle.weights(eps[n, :k], lat.tau, mode)
        shared += k > 1
        for j in range(k):
            s = ids[n, j]
            rn = arms[s][n]
            us = p.u[s] + np.cross(p.omega[s], rn)
            B = Bs[j] if mode == 0 else Bn
            m = B * lat.rho0 * us
            F[s] -= m
            T[s] -= np.cross(rn, m)
            scale[s] += np.abs(m).sum() * (1.0 + np.abs(rn).sum())
    return F, T, scale, shared


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("q", [9, 19])
def test_force_and_torque_in_fluid_at_rest(q, mode):
    # F_s = -sum_n B rho (U_s + Omega_s x r_n), T_s = -sum_n r_n x [B rho
    # (U_s + Omega_s x r_n)], B = B_{n,s} (Eq. 14) or B_n (Eq. 11).
    lat = _box(q)
    rng = np.random.default_rng(5 + q + 10 * mode)
    X, R = _touching_pair(q)
    n = X.shape[0]
    U = rng.uniform(-2e-3, 2e-3, (n, 3))
    Om = np.stack([_spin(q, rng, 1e-3) for _ in range(n)])
    if q == 9:
        U[:, 2] = 0.0
    p = W.Particles(X, U, Om, R)
    Fx, Tx, scale, shared = _rest_fluid_exchange(lat, p, mode)
    assert shared > 10  # cells covered by two particles take part
    L = oracle.Lattice(lat)
    F, T = L.step(p, mode)
    for s in range(n):
        assert np.abs(F[s] - Fx[s]).max() <= 1e-13 * scale[s]
        assert np.abs(T[s] - Tx[s]).max() <= 1e-13 * scale[s]
        # each particle's torque is far above that bound: the pin has teeth
        assert np.abs(Tx[s]).max() > 1e4 * 1e-13 * scale[s]


@pytest.mark.parametrize("q", [9, 19])
def test_spin_alone_gives_the_rotational_torque(q):
    # U = 0: T_s = -sum_n B_{n,s} rho (|r_n|^2 Omega - r_n (r_n . Omega)), the
    # double cross product written out, for a particle alone in fluid at rest.
    lat = _box(q)
    X = np.array([[12.4, 11.7, 9.2 if q == 19 else 0.0]])
    Om = np.array([[3e-4, -5e-4, 7e-4]]) if q == 19 else np.array([[0.0, 0.0, 7e-4]])
    p = W.Particles(X, np.zeros((1, 3)), Om, np.array([4.6]))
    nslot, ids, eps, _ = oracle.rasterize(lat, p.x, p.r)
    arms = _arms(lat, X[0])
    T = np.zeros(3)
    for n in np.nonzero(nslot)[0]:
        _, Bs = oracle.weights(eps[n, :nslot[n]], lat.tau, 0)
        rn = arms[n]
        T -= Bs[0] * lat.rho0 * (rn @ rn * Om[0] - rn * (rn @ Om[0]))
    L = oracle.Lattice(lat)
    F, Tg = L.step(p)
    assert np.allclose(Tg[0], T, rtol=1e-12, atol=1e-15 * np.abs(T).max())
    # the torque opposes the spin
    assert T @ Om[0] < 0


def test_original_weighting_uses_the_cell_total_for_each_particle():
    # In a cell covered by two particles Eq. 11 weighs each particle's exchange
    # by B_n, Eq. 14 by B_{n,s}: the two schemes' forces differ there by the
    # ratio of the weights, which the rest-fluid closed form fixes.
    lat = _box(9)
    X, R = _touching_pair(9)
    U = np.array([[1e-3, 0, 0], [-1e-3, 5e-4, 0], [0, -1e-3, 0]])
    p = W.Particles(X, U, np.zeros((3, 3)), R)
    F0, _ = oracle.Lattice(lat).step(p, 0)
    F1, _ = oracle.Lattice(lat).step(p, 1)
    Fx0, _, _, _ = _rest_fluid_exchange(lat, p, 0)
    Fx1, _, _, _ = _rest_fluid_exchange(lat, p, 1)
    assert np.allclose(F0, Fx0, rtol=1e-12, atol=1e-18)
    assert np.allclose(F1, Fx1, rtol=1e-12, atol=1e-18)
    # the shared cells make the two schemes differ visibly
    assert np.abs(F1 - F0).max() > 1e-3 * np.abs(F0).max()
