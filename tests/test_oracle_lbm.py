"""Pins of the oracle's lattice Boltzmann step (Secs. 2.1-2.3, Eqs. 1-14)
against moment identities, closed-form flows, conservation laws, fixed points
and symmetries."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from conftest import read_golden

WALLS_Y = (W.PERIODIC, W.PERIODIC, W.BOUNCE_BACK, W.BOUNCE_BACK, W.PERIODIC, W.PERIODIC)


def _evecs(q):
    """Lattice velocities recovered from the oracle's equilibrium: the first
    moment of f^eq(1, u) along unit u directions is u, so e_i is read off
    feq(1, t e_a) with the known weights of Eq. 3 (w_i = f^eq_i(1, 0))."""
    w = oracle.feq(q, 1.0, [0, 0, 0])
    e = np.zeros((q, 3))
    t = 1e-3
    for a in range(3 if q == 19 else 2):
        u = np.zeros(3)
        u[a] = t
        fp, fm = oracle.feq(q, 1.0, u), oracle.feq(q, 1.0, -u)
        e[:, a] = np.round((fp - fm) / (6.0 * t * w))
    return w, e


@pytest.mark.parametrize("q", [9, 19])
def test_velocity_set(q):
    w, e = _evecs(q)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    if q == 19:
        # D3Q19 weights printed below Eq. 3
        assert np.allclose(sorted(set(np.round(w, 15))), [1 / 36, 1 / 18, 1 / 3])
    # isotropy of the lattice tensors up to 4th order
    assert np.allclose(w @ e, 0)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, e, e)[:2, :2], np.eye(2) / 3)
    s4 = np.einsum("i,ia,ib,ic,id->abcd", w, e, e, e, e)
    assert s4[0, 0, 1, 1] == pytest.approx(1 / 9)
    assert s4[0, 0, 0, 0] == pytest.approx(1 / 3)
    # the canonical order puts v and -v at the documented positions
    if q == 9:
        assert e[1].tolist() == [1, 0, 0] and e[3].tolist() == [-1, 0, 0]
        assert e[5].tolist() == [1, 1, 0] and e[7].tolist() == [-1, -1, 0]
    else:
        for i in range(1, 19, 2):
            assert (e[i] == -e[i + 1]).all()


@pytest.mark.parametrize("q", [9, 19])
def test_equilibrium_moments(q):
    # Eq. 3 reproduces rho, rho u and rho c_s^2 I + rho u u exactly.
    w, e = _evecs(q)
    rho, u = 1.07, np.array([0.03, -0.02, 0.01 if q == 19 else 0.0])
    fe = oracle.feq(q, rho, u)
    assert fe.sum() == pytest.approx(rho, rel=1e-14)
    assert np.allclose(fe @ e, rho * u, atol=1e-15)
    pi = np.einsum("i,ia,ib->ab", fe, e, e)
    d = 3 if q == 19 else 2
    assert np.allclose(pi[:d, :d], rho / 3 * np.eye(d) + rho * np.outer(u, u)[:d, :d], atol=1e-15)


@pytest.mark.parametrize("q", [9, 19])
@pytest.mark.parametrize("tau", [0.6, 0.8])
def test_guo_forcing_moments(q, tau):
    # Eq. 4 (Guo et al.): zeroth moment 0, first moment (1-1/(2tau)) F,
    # second moment (1-1/(2tau)) (uF + Fu).
    w, e = _evecs(q)
    u = np.array([0.02, 0.01, -0.015 if q == 19 else 0.0])
    F = np.array([1e-3, -2e-3, 5e-4 if q == 19 else 0.0])
    Fi = oracle.guo(q, tau, u, F)
    k = 1 - 1 / (2 * tau)
    assert abs(Fi.sum()) < 1e-18
    assert np.allclose(Fi @ e, k * F, atol=1e-18)
    d = 3 if q == 19 else 2
    m2 = np.einsum("i,ia,ib->ab", Fi, e, e)[:d, :d]
    assert np.allclose(m2, k * (np.outer(u, F) + np.outer(F, u))[:d, :d], atol=1e-18)


@pytest.mark.parametrize("q", [9, 19])
def test_solid_operator_identities(q):
    # Eq. 10: sum_i Omega^s_i = 0 and, with u from Eq. 5,
    # sum_i Omega^s_i e_i = rho (u_s - u) + F.  With u_s = u and f = f^eq the
    # operator vanishes; it is antisymmetric in its non-equilibrium part.
    w, e = _evecs(q)
    rng = np.random.default_rng(3)
    F = np.array([1e-4, 2e-4, -1e-4 if q == 19 else 0.0])
    f = w * (1 + 0.05 * rng.uniform(-1, 1, q))
    rho, u = oracle.moments(q, f, F)
    us = np.array([0.01, -0.02, 0.005 if q == 19 else 0.0])
    om = oracle.omega_s(q, f, rho, u, us)
    assert abs(om.sum()) < 1e-15
    assert np.allclose(om @ e, rho * (us - u) + F, atol=1e-15)
    fe = oracle.feq(q, rho, u)
    assert np.allclose(oracle.omega_s(q, fe, rho, u, u), 0, atol=1e-16)


def _channel(q, H, tau, g=1e-6, nx=2):
    return W.LatticeSpec(q=q, nx=nx, ny=H, nz=1 if q == 9 else 2, tau=tau, force=(g, 0, 0),
                         faces=WALLS_Y)


@pytest.mark.parametrize("q,tau", [(9, 0.8), (9, 0.6), (9, 0.5 + math.sqrt(3) / 4), (19, 0.65)])
def test_poiseuille_exact_discrete(q, tau):
    # BGK with Guo forcing and halfway bounce-back walls at y=-1/2, H-1/2: the
    # steady channel profile is the continuum parabola plus a uniform slip
    # g (16 Lambda - 3) / (24 nu), Lambda = (tau-1/2)^2; at tau = 1/2+sqrt(3)/4
    # the slip vanishes and the parabola is exact.
    H, g = 8, 1e-6
    lat = _channel(q, H, tau, g)
    L = oracle.Lattice(lat)
    nu = (tau - 0.5) / 3
    nsteps = int(60 * H * H / (math.pi ** 2 * nu))
    for _ in range(nsteps):
        L.step()
    _, u = L.macros()
    y = np.arange(H)
    lam = (tau - 0.5) ** 2
    parab = g / (2 * nu) * (y + 0.5) * (H - 0.5 - y)
    exact = parab + g * (16 * lam - 3) / (24 * nu)
    got = u[0, :, 0, 0]
    assert np.abs(got - exact).max() / exact.max() < 1e-10
    assert np.abs(u[..., 1:]).max() < 1e-14


@pytest.mark.parametrize("q,tau", [(9, 0.8), (19, 0.65)])
def test_couette_exact(q, tau):
    # Moving wall (Sec. 2.2; Ladd's momentum term): linear profile
    # u = u_w (y + 1/2) / H between a resting wall at -1/2 and the moving wall.
    H, uw = 8, 0.01
    fu = [(0.0, 0.0, 0.0)] * 6
    fu[3] = (uw, 0.0, 0.0)
    lat = W.LatticeSpec(q=q, nx=2, ny=H, nz=1 if q == 9 else 2, tau=tau,
                        faces=(W.PERIODIC, W.PERIODIC, W.BOUNCE_BACK, W.MOVING_WALL,
                               W.PERIODIC, W.PERIODIC), face_u=tuple(fu))
    L = oracle.Lattice(lat)
    nu = (tau - 0.5) / 3
    for _ in range(int(60 * H * H / (math.pi ** 2 * nu))):
        L.step()
    _, u = L.macros()
    y = np.arange(H)
    assert np.abs(u[0, :, 0, 0] - uw * (y + 0.5) / H).max() < 1e-14


def _duct_series(ny, nz, G, mu, terms=200):
    # Eq. 30 with the walls at -1/2 and n-1/2 on both cross-stream axes.
    lh, lw = float(ny), float(nz)
    y = np.arange(ny)[:, None] + 0.5
    z = np.arange(nz)[None, :] + 0.5
    U = G / (2 * mu) * y * (lh - y)
    for m in range(1, terms + 1):
        b = (2 * m - 1) * math.pi / lh
        ratio = (np.exp(b * (z - lw)) - np.exp(-b * (z + lw)) + np.exp(-b * z) - np.exp(b * (z - 2 * lw))) \
            / (1 - np.exp(-2 * b * lw))
        U = U - 4 * G * lh ** 2 / (mu * math.pi ** 3) / (2 * m - 1) ** 3 * ratio * np.sin(b * y)
    return U


@pytest.mark.parametrize("row", read_golden("duct_flow.txt"))
def test_duct_flow_series(row):
    # Sec. 3.1: 3D duct with walls on y and z; the profile matches the series
    # of Eq. 30 within the printed 0.5 % (max relative to the centre speed).
    ny, nz, tau, g, tol = int(row[0]), int(row[1]), row[2], row[3], row[4]
    lat = W.LatticeSpec(q=19, nx=1, ny=ny, nz=nz, tau=tau, force=(g, 0, 0),
                        faces=(W.PERIODIC, W.PERIODIC, W.BOUNCE_BACK, W.BOUNCE_BACK,
                               W.BOUNCE_BACK, W.BOUNCE_BACK))
    nu = (tau - 0.5) / 3
    ref = _duct_series(ny, nz, g, nu)
    L = oracle.Lattice(lat)
    u0 = np.zeros((nz, ny, 1, 3))
    u0[..., 0] = ref.T[:, :, None]
    L.set_equilibrium(u=u0.reshape(-1, 3))
    for _ in range(1500):
        L.step()
    _, u = L.macros()
    err = np.abs(u[:, :, 0, 0].T - ref).max() / ref.max()
    assert err < tol
    # and the series itself satisfies the no-slip limit at the walls
    assert np.abs(_duct_series(ny, nz, g, nu)[0]).max() < 0.05 * ref.max()


def _random_particles(lat, n, rmin, rmax, seed, umax=0.0, wmax=0.0):
    rng = np.random.default_rng(seed)
    box = [lat.nx, lat.ny] + ([lat.nz] if lat.q == 19 else [])
    periodic = tuple(lat.periodic(a) for a in range(len(box)))
    r = np.sort(rng.uniform(rmin, rmax, n))[::-1]
    x = W.rsa(rng, r, tuple(float(b) for b in box), periodic, gap=-0.8 * rmin)  # allow overlaps
    u = rng.uniform(-umax, umax, (n, 3))
    w = rng.uniform(-wmax, wmax, (n, 3))
    if lat.q == 9:
        u[:, 2] = 0
        w[:, :2] = 0
    return W.Particles(x, u, w, r)


@pytest.mark.parametrize("q", [9, 19])
def test_mass_conservation_with_particles(q):
    # BGK, Omega^s and F_i each conserve the cell mass and streaming with
    # bounce-back permutes populations: the total mass is invariant up to
    # rounding.
    lat = W.LatticeSpec(q=q, nx=24, ny=20, nz=1 if q == 9 else 12, tau=0.7, force=(1e-5, 0, 0),
                        faces=WALLS_Y)
    p = _random_particles(lat, 6, 2.5, 4.0, seed=q, umax=0.01, wmax=0.002)
    L = oracle.Lattice(lat, W.random_state(lat, 1))
    m0 = L.mass()
    for _ in range(40):
        L.step(p)
    eps = np.finfo(float).eps
    assert abs(L.mass() - m0) <= 40 * lat.ncells * q * eps * 4


@pytest.mark.parametrize("q", [9, 19])
def test_momentum_balance_periodic(q):
    # With no body force in a periodic box, the fluid momentum changes by
    # minus the total hydrodynamic force of Eq. 14 (Newton's third law).
    lat = W.LatticeSpec(q=q, nx=24, ny=24, nz=1 if q == 9 else 16, tau=0.8)
    p = _random_particles(lat, 5, 3.0, 4.5, seed=7, umax=0.02, wmax=0.003)
    L = oracle.Lattice(lat, W.random_state(lat, 2))
    _, e = _evecs(q)
    for _ in range(3):
        P0 = L.f.reshape(q, -1).sum(axis=1) @ e
        F, T = L.step(p)
        P1 = L.f.reshape(q, -1).sum(axis=1) @ e
        scale = np.abs(F).sum() + 1e-30
        assert np.allclose(P1 - P0, -F.sum(axis=0), atol=1e-13 * max(scale, 1.0))


@pytest.mark.parametrize("q", [9, 19])
def test_momentum_gain_from_body_force(q):
    # Without particles the fluid gains exactly N F per step (Guo first moment
    # plus the half-force shift of Eq. 5).
    F = np.array([2e-5, -1e-5, 3e-6 if q == 19 else 0.0])
    lat = W.LatticeSpec(q=q, nx=12, ny=10, nz=1 if q == 9 else 8, tau=0.75, force=tuple(F))
    L = oracle.Lattice(lat, W.random_state(lat, 3))
    _, e = _evecs(q)
    P0 = L.f.reshape(q, -1).sum(axis=1) @ e
    L.step()
    P1 = L.f.reshape(q, -1).sum(axis=1) @ e
    assert np.allclose(P1 - P0, lat.ncells * F, atol=1e-14)


@pytest.mark.parametrize("q", [9, 19])
def test_rest_and_comoving_fixed_points(q):
    lat = W.LatticeSpec(q=q, nx=20, ny=20, nz=1 if q == 9 else 16, tau=0.9)
    p = _random_particles(lat, 4, 3.0, 4.0, seed=4)
    # (i) fluid at rest, particles at rest: nothing moves, no force
    L = oracle.Lattice(lat)
    f0 = L.f.copy()
    F, T = L.step(p)
    assert np.abs(L.f - f0).max() < 4e-16  # a few ulp of 4/9
    assert np.abs(F).max() < 1e-16 and np.abs(T).max() < 1e-15
    # (ii) uniform flow with particles translating at the same velocity
    u0 = np.array([0.03, -0.01, 0.02 if q == 19 else 0.0])
    p.u[:] = u0
    L = oracle.Lattice(lat)
    L.set_equilibrium(u=np.tile(u0, (lat.ncells, 1)))
    f0 = L.f.copy()
    F, T = L.step(p)
    assert np.abs(L.f - f0).max() < 4e-16  # a few ulp of 4/9
    assert np.abs(F).max() < 1e-13 and np.abs(T).max() < 1e-12  # rounding of ~10^2 terms


def test_centreline_disk_symmetry():
    # A disk on the channel's mid-plane (y = 49.5 for walls at -1/2, 99.5) feels
    # no lift and no torque under a symmetric body-force flow.
    w = W.c1()
    p = w.particles.copy()
    p.x[0, 1] = 49.5
    L = oracle.Lattice(w.lattice)
    for _ in range(30):
        F, T = L.step(p)
    # mirrored cells sum their populations in a different order, so the
    # symmetry holds to accumulated rounding, far below the drag itself
    assert abs(F[0, 1]) < 1e-11 * abs(F[0, 0])
    assert abs(T[0, 2]) < 1e-11 * abs(F[0, 0]) * p.r[0]
    assert F[0, 0] > 0


@pytest.mark.parametrize("q", [9, 19])
def test_translation_invariance(q):
    # Shifting the state and the particles by whole cells on a periodic box
    # shifts every output exactly (positions are dyadic so differences are exact).
    lat = W.LatticeSpec(q=q, nx=20, ny=18, nz=1 if q == 9 else 14, tau=0.7, force=(1e-5, 2e-6, 0))
    f0 = W.random_state(lat, 5)
    X = np.array([[6.25, 7.5, 5.0], [13.75, 9.0, 8.5]])
    if q == 9:
        X[:, 2] = 0
    p = W.Particles(X, np.array([[0.01, 0.0, 0.0], [0.0, -0.01, 0.0]]), np.zeros((2, 3)),
                    np.array([3.5, 3.0]))
    A = oracle.Lattice(lat, f0)
    FA, TA = A.step(p)
    sh = np.array([3, 5, 2 if q == 19 else 0])
    p2 = p.copy()
    p2.x = np.mod(p2.x + sh, [lat.nx, lat.ny, lat.nz])
    B = oracle.Lattice(lat, np.roll(f0, shift=(sh[2], sh[1], sh[0]), axis=(1, 2, 3)))
    FB, TB = B.step(p2)
    assert np.array_equal(np.roll(A.f, shift=(sh[2], sh[1], sh[0]), axis=(1, 2, 3)), B.f)
    assert np.allclose(FA, FB, rtol=1e-13, atol=1e-18)
    assert np.allclose(TA, TB, rtol=1e-12, atol=1e-17)


def test_open_layers_keep_uniform_flow():
    # Equilibrium inlet (u_in) and local-velocity outlet keep the uniform
    # stream f^eq(rho0, u_in) unchanged in a y-periodic box.
    uin = 0.02
    fu = [(uin, 0.0, 0.0)] + [(0.0, 0.0, 0.0)] * 5
    lat = W.LatticeSpec(q=9, nx=16, ny=6, tau=0.8, faces=(W.INLET_EQ, W.OUTLET_EQ, W.PERIODIC,
                                                         W.PERIODIC, W.PERIODIC, W.PERIODIC),
                        face_u=tuple(fu))
    L = oracle.Lattice(lat)
    L.set_equilibrium(u=np.tile([uin, 0, 0], (lat.ncells, 1)))
    f0 = L.f.copy()
    for _ in range(20):
        L.step()
    # the two boundary layers hold the populations streamed in this step
    # (reset before the next collision); the interior is unchanged
    assert np.abs(L.f[:, :, :, 1:-1] - f0[:, :, :, 1:-1]).max() < 1e-15


def test_original_mode_matches_modified_for_single_cover():
    # With no shared cells Eqs. 7/9/11 and Eqs. 12/13/14 coincide.
    w = W.c1()
    A = oracle.Lattice(w.lattice)
    B = oracle.Lattice(w.lattice)
    for _ in range(5):
        FA, TA = A.step(w.particles, mode=0)
        FB, TB = B.step(w.particles, mode=1)
    assert np.allclose(A.f, B.f, rtol=0, atol=1e-16)
    assert np.allclose(FA, FB, rtol=1e-14)
