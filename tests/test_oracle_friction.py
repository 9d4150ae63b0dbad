"""Pins of the oracle's sliding and twisting friction (Sec. 2.5, Eqs. 22, 28,
29): a sphere (or disk) resting on a wall under its buoyant weight W, pushed
or twisted, against the closed forms of rigid-body mechanics with a Coulomb
cap mu_f (W + 2 F_C):

* below the cap it rolls without slipping, a = F / (m + I / r^2);
* far above it it slides, a = (F - F_crit) / m, spin-up r F_crit / I;
* twisted above the cap M_crit = 3 pi a F_crit / 16 it spins up at
  (T - M_crit) / I, with the contact radius a from the JKR relation
  4 F_C (x^3 - x^{3/2}) = W solved in closed form for x = a / a0;
* twisted below it, it stops at the twist angle T / (k_T a^2 / 2).

Also pair invariants: momentum is conserved with friction, and a central
impact without spin sees no tangential force at all."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads as W

R0, G0 = 4.0, 1e-5
GAMMA, EP, POISSON = 1e-5, 1e-2, 0.3
ESTAR = 1.0 / (2 * (1 - POISSON ** 2) / EP)          # Eq. 25, identical bodies
FC = 3 * math.pi * GAMMA * R0                         # Eq. 27 text, wall: R = r


def _wall_lattice(q):
    faces = (W.BOUNCE_BACK, W.BOUNCE_BACK) + (W.PERIODIC,) * 4
    return W.LatticeSpec(q=q, nx=40, ny=40, nz=40 if q == 19 else 1, faces=faces)


def _mass(q, rho=3.0):
    V = math.pi * R0 ** 2 if q == 9 else 4.0 / 3.0 * math.pi * R0 ** 3
    m = rho * V
    I = 0.5 * m * R0 ** 2 if q == 9 else 0.4 * m * R0 ** 2
    return V, m, I


def _settled(q, gamma=GAMMA, **fric):
    """A sphere (disk) at rest on the wall x = -1/2 under gravity -x, settled
    without friction; returns the particle, the DEM state and the load W."""
    lat = _wall_lattice(q)
    eta_n = 2.0 if q == 9 else 5.0                    # near-critical normal damping
    base = W.DemSpec(g=(-G0, 0.0, 0.0), gamma=gamma, E_p=EP, poisson=POISSON, eta_n=eta_n)
    p = W.Particles(np.array([[R0 - 0.5, 20.0, 20.0 if q == 19 else 0.0]]), np.zeros((1, 3)),
                    np.zeros((1, 3)), np.array([R0]))
    D = oracle.Dem(lat, base, 1)
    z = np.zeros((1, 3))
    for _ in range(8000):
        D.step(p, z, z)
    assert D.contacts()[0] == [-1] and abs(p.u[0, 0]) < 1e-12
    fr = W.DemSpec(g=(-G0, 0.0, 0.0), gamma=gamma, E_p=EP, poisson=POISSON, eta_n=eta_n, **fric)
    D.params = oracle.make_dem(fr)
    V, _, _ = _mass(q)
    return lat, p, D, (3.0 - 1.0) * V * G0


def _run(D, p, F, T, steps):
    Fa = np.array([F], dtype=np.float64)
    Ta = np.array([T], dtype=np.float64)
    hist = []
    for _ in range(steps):
        D.step(p, Fa, Ta)
        hist.append((p.u[0].copy(), p.omega[0].copy()))
    return hist


@pytest.mark.parametrize("q", [9, 19])
def test_rolls_without_slipping_below_the_cap(q):
    _, p, D, Wl = _settled(q, k_t=5e-3, eta_t=2.0, mu_f=1.0)
    _, m, I = _mass(q)
    F = 2e-4
    assert F * I / (m * R0 ** 2 + I) < 1.0 * (Wl + 2 * FC)   # static friction suffices
    h = _run(D, p, (0.0, F, 0.0), (0.0, 0.0, 0.0), 5000)
    a = (h[-1][0][1] - h[2999][0][1]) / 2000.0
    assert a == pytest.approx(F / (m + I / R0 ** 2), rel=1e-5)
    # no slip: the contact point (at -r x) is at rest, u_y = r omega_z
    u, w = h[-1]
    assert abs(u[1] - R0 * w[2]) < 1e-5 * abs(u[1])
    # the spring carries the friction force the rolling needs
    xi, theta, _ = D.springs(0)[-1]
    assert 5e-3 * xi[1] == pytest.approx(-F * I / (m * R0 ** 2 + I), rel=1e-4)
    assert theta == 0.0


@pytest.mark.parametrize("q", [9, 19])
def test_slides_at_the_adhesive_coulomb_cap(q):
    mu = 0.05
    _, p, D, Wl = _settled(q, k_t=5e-3, eta_t=2.0, mu_f=mu)
    _, m, I = _mass(q)
    Fcrit = mu * (Wl + 2 * FC)                        # Eq. 29, F_ne = W at rest
    F = 2e-3
    assert F > Fcrit * (1 + m * R0 ** 2 / I)          # the contact keeps slipping
    h = _run(D, p, (0.0, F, 0.0), (0.0, 0.0, 0.0), 1500)
    a = (h[-1][0][1] - h[499][0][1]) / 1000.0
    alpha = (h[-1][1][2] - h[499][1][2]) / 1000.0
    assert a == pytest.approx((F - Fcrit) / m, rel=1e-7)
    assert alpha == pytest.approx(R0 * Fcrit / I, rel=1e-7)
    # the slider: while capped, spring plus dashpot give exactly F_crit, so
    # the spring's stretch stays bounded instead of growing with the slip
    u, w = h[-2]                          # state at the start of the last step
    vt = -(u[1] - R0 * w[2])              # the wall's velocity relative to the contact point
    xi, _, _ = D.springs(0)[-1]
    assert 5e-3 * xi[1] + 2.0 * vt == pytest.approx(-Fcrit, rel=1e-12)


def _contact_radius(Wl):
    # 4 F_C (x^3 - x^{3/2}) = W with s^3 = x^{3/2}: s^3 = (1 + sqrt(1 + W/F_C)) / 2
    s3 = 0.5 * (1.0 + math.sqrt(1.0 + Wl / FC))
    a0 = (9 * math.pi * GAMMA * R0 ** 2 / ESTAR) ** (1.0 / 3.0)   # Eq. 27
    return s3 ** (2.0 / 3.0) * a0


def test_twist_slips_above_its_cap():
    mu = 0.05
    _, p, D, Wl = _settled(19, k_t=5e-3, eta_t=2.0, mu_f=mu)
    _, _, I = _mass(19)
    a = _contact_radius(Wl)
    Mcrit = 3 * math.pi * a * mu * (Wl + 2 * FC) / 16          # Eq. 29
    T = 1e-3
    assert T > Mcrit
    h = _run(D, p, (0.0, 0.0, 0.0), (T, 0.0, 0.0), 1500)
    alpha = (h[-1][1][0] - h[499][1][0]) / 1000.0
    assert alpha == pytest.approx((T - Mcrit) / I, rel=1e-7)
    # the twist slider holds spring plus dashpot at the cap
    Om = h[-2][1][0]                      # relative twist rate about n = -x
    _, theta, _ = D.springs(0)[-1]
    assert 5e-3 * a * a / 2 * theta + 2.0 * a * a / 2 * Om == pytest.approx(Mcrit, rel=1e-9)
    # twisting about the normal moves nothing else
    assert np.abs(h[-1][0]).max() < 1e-15 and np.abs(h[-1][1][1:]).max() < 1e-15


def test_twist_sticks_below_its_cap():
    mu, kt = 0.05, 5e-3
    _, p, D, Wl = _settled(19, k_t=kt, eta_t=8.0, mu_f=mu)
    a = _contact_radius(Wl)
    T = 1e-4
    assert T < 3 * math.pi * a * mu * (Wl + 2 * FC) / 16
    h = _run(D, p, (0.0, 0.0, 0.0), (T, 0.0, 0.0), 12000)
    angle = sum(w[0] for _, w in h)                            # dt = 1
    assert abs(h[-1][1][0]) < 1e-9
    assert angle == pytest.approx(T / (kt * a * a / 2), rel=1e-3)


def _pair(q, spin):
    lat = W.LatticeSpec(q=q, nx=40, ny=40, nz=40 if q == 19 else 1)
    x = np.array([[16.0, 20.0, 20.0], [24.5, 21.0 if spin else 20.0, 20.0]])
    if q == 9:
        x[:, 2] = 0.0
    u = np.array([[2e-3, 0.0, 0.0], [-2e-3, 0.0, 0.0]])
    w = np.zeros((2, 3))
    if spin:
        w[:, 2] = [3e-3, -1e-3]
        if q == 19:
            w[:, 0] = [1e-3, 2e-3]
            u[:, 2] = [5e-4, -5e-4]
    return lat, W.Particles(x, u, w, np.array([4.0, 4.5]))


@pytest.mark.parametrize("q", [9, 19])
def test_pair_with_friction_conserves_momentum(q):
    lat, p = _pair(q, spin=True)
    dem = W.DemSpec(E_p=1e-3, gamma=1e-5, eta_n=0.05, k_t=2e-3, eta_t=0.05, mu_f=0.3)
    D = oracle.Dem(lat, dem, 2)
    V = math.pi * p.r ** 2 if q == 9 else 4.0 / 3.0 * math.pi * p.r ** 3
    m = (dem.rho_p * V)[:, None]
    P0 = (m * p.u).sum(axis=0)
    z = np.zeros((2, 3))
    w0 = p.omega.copy()
    touched = False
    tangent_checked = 0
    for _ in range(800):
        x0 = p.x.copy()
        D.step(p, z, z)
        touched |= bool(D.contacts()[0])
        assert np.allclose((m * p.u).sum(axis=0), P0, rtol=0, atol=1e-14 * np.abs(m * p.u).sum())
        # the tangential spring lies in the tangent plane of the contact's
        # current normal (Eq. 28 integrates the displacement along t_s)
        for i, j in ((0, 1), (1, 0)):
            sp = D.springs(i)
            if j in sp:
                n = (x0[j] - x0[i]) / np.linalg.norm(x0[j] - x0[i])
                xi = sp[j][0]
                assert abs(xi @ n) <= 1e-12 * np.linalg.norm(xi)
                tangent_checked += np.linalg.norm(xi) > 0
    assert touched and tangent_checked > 100
    assert np.abs(p.omega - w0).max() > 1e-5                      # friction torqued them


@pytest.mark.parametrize("q", [9, 19])
def test_central_impact_without_spin_feels_no_friction(q):
    lat, p0 = _pair(q, spin=False)
    runs = []
    for fric in ({}, dict(k_t=2e-3, eta_t=0.05, mu_f=0.3)):
        p = p0.copy()
        D = oracle.Dem(lat, W.DemSpec(E_p=1e-3, gamma=1e-5, eta_n=0.05, **fric), 2)
        z = np.zeros((2, 3))
        for _ in range(600):
            D.step(p, z, z)
        runs.append(p)
    assert np.array_equal(runs[0].x, runs[1].x) and np.array_equal(runs[0].u, runs[1].u)
    assert np.abs(runs[1].omega).max() == 0.0


# Rolling resistance (Eq. 28 third line, Eq. 29 third line): stiffness
# k_r = 4 F_C (a/a0)^{3/2} per unit rolling displacement, capped at the
# displacement theta_crit R.  On the wall R = r and (a/a0)^{3/2} = s^3 of
# the JKR load relation above.

def _rolling_stiffness(Wl):
    return 4 * FC * 0.5 * (1.0 + math.sqrt(1.0 + Wl / FC))


@pytest.mark.parametrize("q", [9, 19])
def test_rolling_resistance_holds_a_torque_below_its_cap(q):
    # a torque below the cap winds the rolling spring: the sphere (disk), which
    # rolls without slipping on the sticking contact, oscillates undamped
    # about phi = T / (k_r r) between 0 and twice that
    theta = 0.05
    _, p, D, Wl = _settled(q, k_t=5e-2, eta_t=5.0, mu_f=1.0, theta_r=theta)
    kr = _rolling_stiffness(Wl)
    T = 0.5 * kr * theta * R0
    h = _run(D, p, (0.0, 0.0, 0.0), (0.0, 0.0, T), 12000)
    phi = np.cumsum([w[2] for _, w in h])                       # dt = 1
    phi_eq = T / (kr * R0)
    assert phi.max() == pytest.approx(2 * phi_eq, rel=1e-2)
    assert phi.min() > -1e-3 * phi_eq
    _, _, xr = D.springs(0)[-1]
    assert np.linalg.norm(xr) <= theta * R0 * (1 + 1e-12)


@pytest.mark.parametrize("q", [9, 19])
def test_rolling_resistance_caps_at_theta_crit(q):
    # above the cap k_r theta_crit r the sphere rolls on, without slipping,
    # at (T - M_r,crit) / (I + m r^2)
    theta = 0.02
    _, p, D, Wl = _settled(q, k_t=5e-2, eta_t=5.0, mu_f=1.0, theta_r=theta)
    _, m, I = _mass(q)
    kr = _rolling_stiffness(Wl)
    Mcrit = kr * theta * R0
    T = 3 * Mcrit
    h = _run(D, p, (0.0, 0.0, 0.0), (0.0, 0.0, T), 4000)
    alpha = (h[-1][1][2] - h[1999][1][2]) / 2000.0
    assert alpha == pytest.approx((T - Mcrit) / (I + m * R0 ** 2), rel=1e-5)
    _, _, xr = D.springs(0)[-1]
    assert np.linalg.norm(xr) == pytest.approx(theta * R0, rel=1e-12)


@pytest.mark.parametrize("q", [9, 19])
def test_rolling_couples_conserve_angular_momentum(q):
    # normal forces are central and the rolling moments act on the two
    # bodies as equal and opposite couples, so the total angular momentum
    # sum(m x cross u + I omega) is conserved (semi-implicit Euler keeps it
    # exactly for central forces)
    lat, p = _pair(q, spin=True)
    dem = W.DemSpec(E_p=1e-3, gamma=1e-5, eta_n=0.05, theta_r=0.01)
    D = oracle.Dem(lat, dem, 2)
    V = math.pi * p.r ** 2 if q == 9 else 4.0 / 3.0 * math.pi * p.r ** 3
    m = dem.rho_p * V
    I = (0.5 if q == 9 else 0.4) * m * p.r ** 2

    def L():
        return (m[:, None] * np.cross(p.x, p.u)).sum(axis=0) + (I[:, None] * p.omega).sum(axis=0)

    L0 = L()
    z = np.zeros((2, 3))
    w0 = p.omega.copy()
    tangent_checked = 0
    for _ in range(800):
        x0 = p.x.copy()
        D.step(p, z, z)
        assert np.allclose(L(), L0, rtol=0, atol=1e-13 * np.abs(L0).max())
        # the rolling spring lies in the tangent plane of the current normal
        sp = D.springs(0)
        if 1 in sp:
            n = (x0[1] - x0[0]) / np.linalg.norm(x0[1] - x0[0])
            xr = sp[1][2]
            assert abs(xr @ n) <= 1e-12 * np.linalg.norm(xr)
            tangent_checked += np.linalg.norm(xr) > 0
    assert np.abs(p.omega - w0).max() > 1e-6                      # the couples acted
    assert tangent_checked > 50


# Without adhesion (gamma = 0) the contact is Hertz's.

def test_hertz_collision_time_and_restitution():
    lat = W.LatticeSpec(q=19, nx=40, ny=40, nz=40)
    v0, r = 4e-4, 4.0
    p = W.Particles(np.array([[15.9, 20.0, 20.0], [24.1, 20.0, 20.0]]),
                    np.array([[v0 / 2, 0.0, 0.0], [-v0 / 2, 0.0, 0.0]]), np.zeros((2, 3)),
                    np.array([r, r]))
    dem = W.DemSpec(E_p=1e-3, poisson=0.3, gamma=0.0)
    D = oracle.Dem(lat, dem, 2)
    Estar = 1.0 / (2 * (1 - 0.3 ** 2) / 1e-3)
    m = dem.rho_p * 4.0 / 3.0 * math.pi * r ** 3
    K = 4.0 / 3.0 * Estar * math.sqrt(r / 2)                    # F = K delta^{3/2}, R = r/2
    dmax = (5 * (m / 2) * v0 ** 2 / (4 * K)) ** 0.4
    shape = integrate.quad(lambda s: 1 / math.sqrt(1 - s ** 2.5), 0, 1)[0]
    t_contact = 2 * dmax / v0 * shape
    z = np.zeros((2, 3))
    steps_in_contact = 0
    for _ in range(int(1.5 * t_contact) + 200):
        D.step(p, z, z)
        steps_in_contact += bool(D.contacts()[0])
    assert steps_in_contact == pytest.approx(t_contact, rel=2e-3)
    assert p.u[1, 0] - p.u[0, 0] == pytest.approx(v0, rel=1e-4)   # elastic: e = 1


def test_hertz_wall_rest_overlap():
    lat = _wall_lattice(19)
    dem = W.DemSpec(g=(-G0, 0.0, 0.0), E_p=EP, poisson=POISSON, gamma=0.0, eta_n=5.0)
    p = W.Particles(np.array([[R0 - 0.5, 20.0, 20.0]]), np.zeros((1, 3)), np.zeros((1, 3)),
                    np.array([R0]))
    D = oracle.Dem(lat, dem, 1)
    z = np.zeros((1, 3))
    for _ in range(8000):
        D.step(p, z, z)
    V, _, _ = _mass(19)
    Wl = 2.0 * V * G0
    overlap = R0 - (p.x[0, 0] + 0.5)
    assert overlap == pytest.approx((Wl / (4.0 / 3.0 * ESTAR * math.sqrt(R0))) ** (2 / 3),
                                    rel=1e-9)


@pytest.mark.parametrize("q", [9, 19])
def test_hertz_slides_at_the_coulomb_cap(q):
    # without adhesion the cap of Eq. 29 is mu_f F_ne = mu_f W: Amontons
    mu = 0.05
    _, p, D, Wl = _settled(q, gamma=0.0, k_t=5e-3, eta_t=2.0, mu_f=mu)
    _, m, I = _mass(q)
    F = 2e-3
    assert F > mu * Wl * (1 + m * R0 ** 2 / I)
    h = _run(D, p, (0.0, F, 0.0), (0.0, 0.0, 0.0), 1500)
    a = (h[-1][0][1] - h[499][0][1]) / 1000.0
    assert a == pytest.approx((F - mu * Wl) / m, rel=1e-7)


def test_hertz_has_no_rolling_resistance():
    # rolling resistance scales with F_C, which is zero without adhesion: a
    # torque rolls the sphere (its contact sticking) at T / (I + m r^2)
    _, p, D, Wl = _settled(19, gamma=0.0, k_t=5e-2, eta_t=5.0, mu_f=1.0, theta_r=0.05)
    _, m, I = _mass(19)
    T = 1e-3
    h = _run(D, p, (0.0, 0.0, 0.0), (0.0, 0.0, T), 4000)
    alpha = (h[-1][1][2] - h[1999][1][2]) / 2000.0
    assert alpha == pytest.approx(T / (I + m * R0 ** 2), rel=1e-5)
    _, _, xr = D.springs(0)[-1]
    assert np.abs(xr).max() == 0.0
