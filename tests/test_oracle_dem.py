"""Pins of the oracle's adhesive DEM (Sec. 2.5, Eqs. 21, 23, 25-27)."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads as W
from conftest import read_golden

R, E, GAMMA = 4.0, 5.49e-4, 1e-5
FC = 3 * math.pi * GAMMA * R                      # Eq. 27 text


def test_jump_on_and_pull_off_points():
    F0, dC = oracle.jkr_force(R, E, GAMMA, 0.0)
    # JKR: at zero approach the force is -8/9 of the load-controlled pull-off
    # force F_C (the jump-on point A of Fig. 6)
    assert F0 == pytest.approx(-8.0 / 9.0 * FC, rel=1e-12)
    # fixed-grip separation (point C) at delta = -delta_C with F = -5/9 F_C
    Fc, _ = oracle.jkr_force(R, E, GAMMA, -dC)
    assert Fc == pytest.approx(-5.0 / 9.0 * FC, rel=1e-9)
    # the force minimum along the stable branch is -F_C
    res = [oracle.jkr_force(R, E, GAMMA, d)[0] for d in np.linspace(-dC, 0.5 * dC, 4001)]
    assert min(res) == pytest.approx(-FC, rel=1e-6)
    # fixed-grip pull-off happens at contact radius a0 / 36^(1/3)
    assert oracle.jkr_x(-1.0) == pytest.approx(36.0 ** (-1.0 / 3.0), rel=1e-13)


@pytest.mark.parametrize("row", read_golden("jkr_adhesion_energy.txt"))
def test_eq23_adhesion_energy(row):
    const, tol = row
    for (r, e, g) in [(R, E, GAMMA), (3.0, 1e-3, 2e-5), (6.0, 2e-4, 5e-6)]:
        _, dC = oracle.jkr_force(r, e, g, 0.0)
        energy = integrate.quad(lambda d: oracle.jkr_force(r, e, g, d)[0], -dC, 0.0,
                                epsabs=0, epsrel=1e-12, limit=200)[0]
        scale = (g ** 5 * r ** 4 / e ** 2) ** (1 / 3)
        assert abs(energy) / scale == pytest.approx(const, rel=tol)


def test_hertz_limit():
    # Without adhesion JKR reduces to Hertz: F = 4/3 E sqrt(R) delta^{3/2}.
    g = 1e-14
    for d in (0.05, 0.2, 0.5):
        F, _ = oracle.jkr_force(R, E, g, d)
        assert F == pytest.approx(4.0 / 3.0 * E * math.sqrt(R) * d ** 1.5, rel=2e-3)


def _box(q=19, n=40, walls=False):
    faces = (W.BOUNCE_BACK, W.BOUNCE_BACK) + (W.PERIODIC,) * 4 if walls else (W.PERIODIC,) * 6
    return W.LatticeSpec(q=q, nx=n, ny=n, nz=n if q == 19 else 1, faces=faces)


def test_free_flight_and_constant_force():
    lat = _box()
    dem = W.DemSpec(g=(0.0, -1e-5, 0.0), rho_p=3.0, rho_f=1.0)
    x0 = np.array([[10.0, 20.0, 20.0], [30.0, 20.0, 20.0]])
    u0 = np.array([[1e-3, 0.0, 0.0], [0.0, 2e-3, 0.0]])
    p = W.Particles(x0.copy(), u0.copy(), np.zeros((2, 3)), np.array([3.0, 4.0]))
    D = oracle.Dem(lat, dem, 2)
    zeros = np.zeros((2, 3))
    n = 50
    for _ in range(n):
        D.step(p, zeros, zeros)
    a = (dem.rho_p - dem.rho_f) / dem.rho_p * dem.g[1]   # (rho_p-rho_f) V g / (rho_p V)
    # semi-implicit Euler: U_n = U_0 + n a, X_n = X_0 + n U_0 + a n (n+1) / 2
    assert np.allclose(p.u[:, 1], u0[:, 1] + n * a, rtol=0, atol=1e-16)
    assert np.allclose(p.x[:, 1], x0[:, 1] + n * u0[:, 1] + a * n * (n + 1) / 2, rtol=0, atol=1e-12)
    assert np.allclose(p.x[:, 0], x0[:, 0] + n * u0[:, 0], atol=1e-12)


def test_hydrodynamic_force_and_torque_integration():
    lat = _box(q=9, n=40)
    dem = W.DemSpec()
    p = W.Particles(np.array([[10.0, 10.0, 0.0]]), np.zeros((1, 3)), np.zeros((1, 3)),
                    np.array([5.0]))
    D = oracle.Dem(lat, dem, 1)
    F = np.array([[2e-3, -1e-3, 0.0]])
    T = np.array([[0.0, 0.0, 4e-3]])
    D.step(p, F, T)
    m = dem.rho_p * math.pi * 25.0
    I = 0.5 * m * 25.0
    assert p.u[0, 0] == pytest.approx(2e-3 / m, rel=1e-14)
    assert p.u[0, 1] == pytest.approx(-1e-3 / m, rel=1e-14)
    assert p.omega[0, 2] == pytest.approx(4e-3 / I, rel=1e-14)


def test_head_on_contact_conserves_momentum_and_hysteresis():
    lat = _box()
    dem = W.DemSpec(E_p=1e-3, poisson=0.3, gamma=1e-5, rho_p=3.0)
    Estar = 1.0 / (2 * (1 - 0.3 ** 2) / 1e-3)
    p = W.Particles(np.array([[18.0, 20.0, 20.0], [26.5, 20.0, 20.0]]),
                    np.array([[2e-3, 0.0, 0.0], [-2e-3, 0.0, 0.0]]), np.zeros((2, 3)),
                    np.array([4.0, 4.0]))
    D = oracle.Dem(lat, dem, 2)
    zeros = np.zeros((2, 3))
    m = dem.rho_p * 4 / 3 * math.pi * 64
    P0 = (m * p.u).sum(axis=0)
    _, dC = oracle.jkr_force(2.0, Estar, 1e-5, 0.0)
    seen_contact = False
    for _ in range(400):
        gap_before = np.linalg.norm(p.x[1] - p.x[0]) - 8.0
        D.step(p, zeros, zeros)
        c = D.contacts()
        if c[0]:
            seen_contact = True
            assert c[0] == [1] and c[1] == [0]
            if gap_before > 0:            # still bonded at negative overlap
                assert gap_before < dC
        else:
            # an approach does not bond before the surfaces touch
            if not seen_contact:
                assert gap_before > 0
        assert np.allclose((m * p.u).sum(axis=0), P0, atol=1e-15)
    assert seen_contact


def test_wall_contact_stops_settling():
    # A heavy sphere settling onto the wall at x = -1/2 comes to rest where the
    # JKR wall force (flat of infinite radius, Eq. 25 with 1/R = 1/r) carries
    # its buoyant weight.
    lat = _box(walls=True)
    dem = W.DemSpec(g=(-1e-5, 0.0, 0.0), gamma=1e-7, E_p=1e-2, eta_n=5.0)
    p = W.Particles(np.array([[5.0, 20.0, 20.0]]), np.zeros((1, 3)), np.zeros((1, 3)),
                    np.array([4.0]))
    D = oracle.Dem(lat, dem, 1)
    zeros = np.zeros((1, 3))
    for _ in range(6000):
        D.step(p, zeros, zeros)
    weight = (dem.rho_p - dem.rho_f) * 4 / 3 * math.pi * 64 * 1e-5
    Estar = 1.0 / (2 * (1 - dem.poisson ** 2) / dem.E_p)
    overlap = 4.0 - (p.x[0, 0] + 0.5)
    F, _ = oracle.jkr_force(4.0, Estar, dem.gamma, overlap)
    assert overlap > 0
    assert F == pytest.approx(weight, rel=1e-3)
    assert D.contacts()[0] == [-1]
    assert abs(p.u[0, 0]) < 1e-6


def test_kinematic_mode_and_wrap():
    lat = _box(q=19, n=16)
    dem = W.DemSpec(kinematic=True)
    p = W.Particles(np.array([[15.9, 0.05, 8.0]]), np.array([[0.2, -0.1, 0.0]]), np.zeros((1, 3)),
                    np.array([3.0]))
    D = oracle.Dem(lat, dem, 1)
    D.step(p, np.zeros((1, 3)), np.zeros((1, 3)))
    assert p.x[0, 0] == pytest.approx(0.1, abs=1e-13)
    assert p.x[0, 1] == pytest.approx(15.95, abs=1e-13)
