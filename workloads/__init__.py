"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the method: it only describes lattices
(sizes, relaxation time, boundary kinds), draws particle sets by seeded random
sequential addition (RSA, largest radius first, rejecting overlaps) and returns
plain numpy arrays.  Both the FP64 CPU oracle and the HIP library consume these
descriptors through their own code.

The five workloads mirror the configurations used to exercise the
partially-saturated-cell LBM of Liu & Wu (arXiv 1901.09745):

* ``c1`` D2Q9 tau=0.8 200x100 channel, bounce-back walls in y, body force
  1e-6 along x, one fixed disk r=10 at (60, 50)  (``c1b``: no disk).
* ``c2`` D2Q9 tau=0.7 1024^2 periodic, 2000 disks r~U(6,12), gap 0.5, JKR DEM,
  gravity 1e-6 on the particles.
* ``c3`` D3Q19 tau=0.6 256^3 periodic, 8000 spheres r~U(4,6), prescribed
  velocities ~N(0, 1e-3^2).
* ``c4`` D2Q9 tau=0.8 512x256 channel, equilibrium inlet u=0.02 / outlet,
  64 fixed disks r=8.
* ``c5`` D3Q19 tau=0.65 384x192x192, walls on x (vertical), 20000 adhesive
  spheres r~U(3,5) settling under gravity 1e-6.

Every generator takes ``scale`` (linear factor on the box, particle count
scaled with the area/volume so the packing fraction is kept) so the same recipe
yields the small cases that the oracle finishes in seconds.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Face boundary kinds, by name (each implementation maps them to its own enum).
PERIODIC = "periodic"
BOUNCE_BACK = "bounce_back"
MOVING_WALL = "moving_wall"
INLET_EQ = "inlet_eq"
OUTLET_EQ = "outlet_eq"
FACE_KINDS = (PERIODIC, BOUNCE_BACK, MOVING_WALL, INLET_EQ, OUTLET_EQ)


@dataclass
class LatticeSpec:
    """Lattice, fluid and boundary description (lattice units)."""

    q: int                      # 9 (D2Q9) or 19 (D3Q19)
    nx: int
    ny: int
    nz: int = 1
    tau: float = 0.8
    force: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    faces: Tuple[str, ...] = (PERIODIC,) * 6       # x-, x+, y-, y+, z-, z+
    face_u: Tuple[Tuple[float, float, float], ...] = ((0.0, 0.0, 0.0),) * 6
    rho0: float = 1.0
    h: float = 1.0              # half-width of the solid-fraction shell

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    def periodic(self, axis: int) -> bool:
        if axis == 2 and self.q == 9:
            return True
        return self.faces[2 * axis] == PERIODIC and self.faces[2 * axis + 1] == PERIODIC

    def replace(self, **kw) -> "LatticeSpec":
        return dataclasses.replace(self, **kw)


@dataclass
class Particles:
    """Particle state as FP64 SoA arrays: x, u, omega of shape (n, 3), r (n,)."""

    x: np.ndarray
    u: np.ndarray
    omega: np.ndarray
    r: np.ndarray

    @property
    def n(self) -> int:
        return int(self.r.shape[0])

    def copy(self) -> "Particles":
        return Particles(self.x.copy(), self.u.copy(), self.omega.copy(), self.r.copy())

    @staticmethod
    def empty() -> "Particles":
        z = np.zeros((0, 3))
        return Particles(z.copy(), z.copy(), z.copy(), np.zeros(0))


@dataclass
class DemSpec:
    """DEM material and time-stepping parameters (lattice units)."""

    rho_p: float = 3.0
    rho_f: float = 1.0
    E_p: float = 1e-3
    poisson: float = 0.3
    gamma: float = 1e-5
    eta_n: float = 0.0
    g: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    dt: float = 1.0
    n_sub: int = 1
    kinematic: bool = False
    max_contacts: int = 16
    k_t: float = 0.0       # tangential stiffness k_T (Eq. 28)
    eta_t: float = 0.0     # tangential dissipation coefficient eta_T (Eq. 28)
    mu_f: float = 0.0      # friction coefficient (Eq. 29); 0: no friction
    theta_r: float = 0.0   # critical rolling angle theta_crit (Eq. 29); 0: no rolling resistance


@dataclass
class Workload:
    name: str
    lattice: LatticeSpec
    particles: Particles
    steps: int
    dem: Optional[DemSpec] = None        # None: particles held fixed
    description: str = ""


# --------------------------------------------------------------------------
# Random sequential addition
# --------------------------------------------------------------------------

def _min_image(d: np.ndarray, L: float, periodic: bool) -> np.ndarray:
    if not periodic:
        return d
    return d - L * np.round(d / L)


def rsa(rng: np.random.Generator, radii: Sequence[float], box: Tuple[float, ...],
        periodic: Tuple[bool, ...], gap: float = 0.0, clearance: float = 0.0,
        xrange: Optional[Tuple[float, float]] = None, max_trials: int = 200_000_000,
        multi: bool = False) -> np.ndarray:
    """Place disks/spheres of the given radii (in the given order) uniformly at
    random without overlap: a candidate is accepted when its distance to every
    placed particle is at least r_i + r_j + gap (nearest image on periodic
    axes).  On a walled axis the centre keeps ``clearance`` + r from the walls at
    -1/2 and L-1/2.  ``xrange`` optionally narrows the x placement window.
    Candidates are drawn in batches, the first acceptable one in a batch wins.
    With ``multi`` (radii in descending order, for packings near the RSA
    jamming limit) every candidate of a batch that clears the placed particles
    at the current radius -- an upper bound of the radii still to come -- is
    taken in draw order if it also clears those taken before it in the batch,
    each with the next radius.
    Returns positions of shape (n, 3) (z = 0 in 2D).
    """
    dim = len(box)
    radii = np.asarray(radii, dtype=np.float64)
    n = radii.shape[0]
    rmax = float(radii.max()) if n else 1.0
    cell = 2.0 * rmax + gap + 1e-9
    nb = [max(1, int(np.floor(box[a] / cell))) for a in range(dim)]
    bsz = [box[a] / nb[a] for a in range(dim)]
    cap = 4
    bins = -np.ones(tuple(nb) + (cap,), dtype=np.int64)
    counts = np.zeros(tuple(nb), dtype=np.int64)
    pos = np.zeros((n, 3))
    offs = np.array(np.meshgrid(*[[-1, 0, 1]] * dim, indexing="ij")).reshape(dim, -1).T
    batch = 4
    trials = 0
    if multi and n > 1 and np.any(np.diff(radii) > 0):
        raise ValueError("rsa(multi=True) needs radii in descending order")

    def insert(k, p):
        nonlocal bins, cap
        bb = tuple(int(v) for v in np.minimum(
            np.floor(np.mod(p, np.asarray(box)) / np.asarray(bsz)).astype(np.int64),
            np.asarray(nb) - 1))
        if counts[bb] >= cap:
            cap *= 2
            nbins = -np.ones(tuple(nb) + (cap,), dtype=np.int64)
            nbins[..., : cap // 2] = bins
            bins = nbins
        bins[bb + (int(counts[bb]),)] = k
        counts[bb] += 1

    k = 0
    while k < n:
        r = radii[k]
        lo = np.zeros(dim)
        hi = np.zeros(dim)
        for a in range(dim):
            if periodic[a]:
                lo[a], hi[a] = 0.0, box[a]
            else:
                lo[a], hi[a] = -0.5 + r + clearance, box[a] - 0.5 - r - clearance
        if xrange is not None:
            lo[0], hi[0] = max(lo[0], xrange[0]), min(hi[0], xrange[1])
        while True:
            if trials > max_trials:
                raise RuntimeError(f"RSA: gave up after {trials} trials at particle {k}")
            P = rng.uniform(lo, hi, size=(batch, dim))
            trials += batch
            b = np.floor(np.mod(P, np.asarray(box)) / np.asarray(bsz)).astype(np.int64)
            b = np.minimum(b, np.asarray(nb) - 1)
            nbr = b[:, None, :] + offs[None, :, :]            # (B, 3^dim, dim)
            for a in range(dim):
                if periodic[a]:
                    nbr[..., a] %= nb[a]
            valid = np.ones(nbr.shape[:2], dtype=bool)
            for a in range(dim):
                if not periodic[a]:
                    valid &= (nbr[..., a] >= 0) & (nbr[..., a] < nb[a])
                    nbr[..., a] = np.clip(nbr[..., a], 0, nb[a] - 1)
            ids = bins[tuple(nbr[..., a] for a in range(dim))]  # (B, 3^dim, cap)
            ids = np.where(valid[..., None], ids, -1).reshape(batch, -1)
            safe = np.where(ids >= 0, ids, 0)
            d2 = np.zeros(ids.shape)
            for a in range(dim):
                d = _min_image(pos[safe, a] - P[:, a:a + 1], box[a], periodic[a])
                d2 += d * d
            need = (radii[safe] + r + gap) ** 2
            clash = ((d2 < need) & (ids >= 0)).any(axis=1)
            ok = np.nonzero(~clash)[0]
            if ok.size and multi:
                taken = []
                for j in ok:
                    if k + len(taken) >= n:
                        break
                    rj = radii[k + len(taken)]
                    fine = True
                    for (t, pt) in taken:
                        d2t = 0.0
                        for a in range(dim):
                            da = float(_min_image(np.array([P[j, a] - pt[a]]), box[a],
                                                  periodic[a])[0])
                            d2t += da * da
                        if d2t < (radii[t] + rj + gap) ** 2:
                            fine = False
                            break
                    if fine:
                        taken.append((k + len(taken), P[j]))
                for (t, pt) in taken:
                    pos[t, :dim] = pt
                    insert(t, pt)
                k += len(taken)
                if ok[0] == 0 and batch > 4:
                    batch //= 2
                break
            if ok.size:
                p = P[ok[0]]
                pos[k, :dim] = p
                insert(k, p)
                k += 1
                if ok[0] == 0 and batch > 4:
                    batch //= 2
                break
            batch = min(batch * 4, 16384)
    return pos


def _particles(x: np.ndarray, u: Optional[np.ndarray] = None, r: Optional[np.ndarray] = None
               ) -> Particles:
    n = x.shape[0]
    return Particles(np.ascontiguousarray(x, dtype=np.float64),
                     np.zeros((n, 3)) if u is None else np.ascontiguousarray(u, dtype=np.float64),
                     np.zeros((n, 3)),
                     np.ascontiguousarray(r, dtype=np.float64))


def _scaled_count(n: int, scale: float, dim: int) -> int:
    return max(1, int(round(n * scale ** dim)))


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

def c1(with_disk: bool = True) -> Workload:
    lat = LatticeSpec(q=9, nx=200, ny=100, tau=0.8, force=(1e-6, 0.0, 0.0),
                      faces=(PERIODIC, PERIODIC, BOUNCE_BACK, BOUNCE_BACK, PERIODIC, PERIODIC))
    if with_disk:
        p = _particles(np.array([[60.0, 50.0, 0.0]]), r=np.array([10.0]))
    else:
        p = Particles.empty()
    return Workload("c1" if with_disk else "c1b", lat, p, steps=2000,
                    description="D2Q9 tau=0.8 200x100 channel, body force 1e-6, "
                    + ("one fixed disk r=10 at (60,50)" if with_disk else "no disk"))


def c2(scale: float = 1.0, seed: int = 2) -> Workload:
    L = int(round(1024 * scale))
    n = _scaled_count(2000, scale, 2)
    rng = np.random.default_rng(seed)
    radii = np.sort(rng.uniform(6.0, 12.0, size=n))[::-1]
    x = rsa(rng, radii, (float(L), float(L)), (True, True), gap=0.5)
    lat = LatticeSpec(q=9, nx=L, ny=L, tau=0.7)
    dem = DemSpec(g=(0.0, -1e-6, 0.0))
    return Workload("c2", lat, _particles(x, r=radii), steps=10_000, dem=dem,
                    description=f"D2Q9 tau=0.7 {L}^2 periodic, {n} disks r~U(6,12) seed {seed}, "
                    "gap 0.5, JKR E=1e-3 nu=0.3 gamma=1e-5, gravity 1e-6 on particles")


def c3(scale: float = 1.0, seed: int = 3) -> Workload:
    L = int(round(256 * scale))
    n = _scaled_count(8000, scale, 3)
    ss = np.random.SeedSequence(seed)
    rng_pos, rng_vel = [np.random.default_rng(s) for s in ss.spawn(2)]
    radii = np.sort(rng_pos.uniform(4.0, 6.0, size=n))[::-1]
    x = rsa(rng_pos, radii, (float(L),) * 3, (True, True, True))
    u = rng_vel.normal(0.0, 1e-3, size=(n, 3))
    lat = LatticeSpec(q=19, nx=L, ny=L, nz=L, tau=0.6)
    dem = DemSpec(kinematic=True)
    return Workload("c3", lat, _particles(x, u=u, r=radii), steps=1000, dem=dem,
                    description=f"D3Q19 tau=0.6 {L}^3 periodic, {n} spheres r~U(4,6) seed {seed}, "
                    "prescribed velocities N(0,1e-3^2), particles advected kinematically")


def c4(scale: float = 1.0, seed: int = 4, u_in: float = 0.02) -> Workload:
    nx, ny = int(round(512 * scale)), int(round(256 * scale))
    n = _scaled_count(64, scale, 2)
    rng = np.random.default_rng(seed)
    radii = np.full(n, 8.0)
    x = rsa(rng, radii, (float(nx), float(ny)), (False, False), gap=0.5, clearance=1.0,
            xrange=(40.0 * scale, nx - 40.0 * scale))
    lat = LatticeSpec(q=9, nx=nx, ny=ny, tau=0.8,
                      faces=(INLET_EQ, OUTLET_EQ, BOUNCE_BACK, BOUNCE_BACK, PERIODIC, PERIODIC),
                      face_u=((u_in, 0.0, 0.0),) + ((0.0, 0.0, 0.0),) * 5)
    return Workload("c4", lat, _particles(x, r=radii), steps=4000,
                    description=f"D2Q9 tau=0.8 {nx}x{ny} channel, equilibrium inlet u={u_in}, "
                    f"outlet rho=1, {n} fixed disks r=8 seed {seed}")


def c5(scale: float = 1.0, seed: int = 5) -> Workload:
    nx, ny, nz = int(round(384 * scale)), int(round(192 * scale)), int(round(192 * scale))
    n = _scaled_count(20000, scale, 3)
    rng = np.random.default_rng(seed)
    radii = np.sort(rng.uniform(3.0, 5.0, size=n))[::-1]
    x = rsa(rng, radii, (float(nx), float(ny), float(nz)), (False, True, True), multi=True)
    lat = LatticeSpec(q=19, nx=nx, ny=ny, nz=nz, tau=0.65,
                      faces=(BOUNCE_BACK, BOUNCE_BACK, PERIODIC, PERIODIC, PERIODIC, PERIODIC))
    dem = DemSpec(g=(-1e-6, 0.0, 0.0))
    return Workload("c5", lat, _particles(x, r=radii), steps=20_000, dem=dem,
                    description=f"D3Q19 tau=0.65 {nx}x{ny}x{nz}, walls at x=-1/2 and {nx}-1/2, "
                    f"{n} adhesive spheres r~U(3,5) seed {seed}, gravity 1e-6 along -x")


# --------------------------------------------------------------------------
# Packed bed of Sec. 3.4 (Ergun, Eqs. 34-36)
# --------------------------------------------------------------------------

# porosity of the simple-cubic lattice packing of touching spheres
ERGUN_POROSITY = 1.0 - np.pi / 6.0


def ergun_dp_star(re: float) -> float:
    """Eq. 35: dimensionless pressure loss 150 / Re_p* + 1.75."""
    return 150.0 / re + 1.75


def ergun_numbers(force: float, U: float, dp: float, tau: float, rho: float = 1.0,
                  porosity: float = ERGUN_POROSITY) -> Tuple[float, float]:
    """Eq. 36 for a bed driven by a body force (pressure gradient dP/h = force)
    with superficial velocity U: (Re_p*, dP*), lattice units, nu = (tau - 1/2)/3.
    dP* carries eps^3 / (1 - eps): with that factor Eq. 35 is Eq. 34 divided
    through; the printed (1 - eps)^2 would leave a stray factor 1 - eps."""
    nu = (tau - 0.5) / 3.0
    re = dp * U / (nu * (1.0 - porosity))
    dps = force * dp / (rho * U * U) * porosity ** 3 / (1.0 - porosity)
    return re, dps


def ergun(dp: int, re: float = 1.0, tau: float = 0.65) -> Workload:
    """Sec. 3.4: the lattice packing of 8 fixed spheres of diameter dp in a
    periodic 2dp cube (neighbouring spheres touch, so the cells at the
    contacts are shared), D3Q19, driven along x by the body force for which
    Eq. 35 gives the modified Reynolds number `re`.  Centres at
    ((i + 1/2) dp, ...): every contact point is a cell centre, a cell the
    two touching spheres share (the paper leaves the alignment open)."""
    L = 2 * dp
    c = [(i + 0.5) * dp for i in range(2)]
    x = np.array([[cx, cy, cz] for cz in c for cy in c for cx in c])
    eps = ERGUN_POROSITY
    nu = (tau - 0.5) / 3.0
    U = re * nu * (1.0 - eps) / dp
    force = ergun_dp_star(re) * U * U * (1.0 - eps) / (dp * eps ** 3)
    lat = LatticeSpec(q=19, nx=L, ny=L, nz=L, tau=tau, force=(force, 0.0, 0.0))
    return Workload(f"ergun{dp}", lat, _particles(x, r=np.full(8, dp / 2.0)), steps=0,
                    description=f"D3Q19 tau={tau} {L}^3 periodic, 8 fixed spheres d_p={dp} in "
                    f"simple-cubic contact, body force {force:.3e} (Eq. 35 at Re_p*={re})")


# --------------------------------------------------------------------------
# Drag on a fixed sphere, Sec. 3.2 (Eqs. 32-33)
# --------------------------------------------------------------------------

def drag_coefficient(force: float, u0: float, dp: float, rho: float = 1.0) -> float:
    """Eq. 32: C_d = 8 F_d / (rho U0^2 pi d_p^2)."""
    return 8.0 * force / (rho * u0 * u0 * np.pi * dp * dp)


def schiller_naumann(re: float) -> float:
    """Eq. 33: C_d = 24 / Re_p (1 + 0.15 Re_p^0.687)."""
    return 24.0 / re * (1.0 + 0.15 * re ** 0.687)


def sphere_drag(dp: int, re: float, u0: float = 0.05) -> Workload:
    """Sec. 3.2: a fixed sphere of diameter dp at the centre of a
    20dp x 10dp x 10dp box, D3Q19; equilibrium inlet u0 along x on x = 0, a
    constant-pressure outlet on x = nx - 1, and the four side faces open
    (constant-pressure outlets: zero normal gradient of the velocity, rho0);
    tau from Re_p = u0 dp / nu."""
    nx, ny, nz = 20 * dp, 10 * dp, 10 * dp
    nu = u0 * dp / re
    lat = LatticeSpec(q=19, nx=nx, ny=ny, nz=nz, tau=3.0 * nu + 0.5,
                      faces=(INLET_EQ, OUTLET_EQ, OUTLET_EQ, OUTLET_EQ, OUTLET_EQ, OUTLET_EQ),
                      face_u=((u0, 0.0, 0.0),) + ((0.0, 0.0, 0.0),) * 5)
    x = np.array([[(nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0]])
    return Workload(f"drag{dp}_re{re:g}", lat, _particles(x, r=np.array([dp / 2.0])), steps=0,
                    description=f"D3Q19 {nx}x{ny}x{nz}, tau={3.0 * nu + 0.5:.4f}, inlet u0={u0} "
                    f"on x, outlets elsewhere, fixed sphere d_p={dp} at the centre (Re_p={re:g})")


# --------------------------------------------------------------------------
# Random packing of Sec. 3.5 (adhesive and non-adhesive microspheres)
# --------------------------------------------------------------------------

# Lattice-unit material of the packing runs (the paper takes its values from
# the literature and prints none): with gravity 8e-4 the hindered settling
# forms the bed in about 20,000 steps, F_C = 3 pi gamma R is about ten times
# a sphere's buoyant weight, E* = E_p / (2 (1 - nu^2)) = 20 keeps delta_C
# near 0.1, and four sub-steps resolve the contact oscillation.
PACKING_DEM = dict(rho_p=3.0, rho_f=1.0, E_p=36.4, poisson=0.3, eta_n=50.0, n_sub=4,
                   k_t=15.0, eta_t=25.0, mu_f=0.3, theta_r=0.01, max_contacts=16)
PACKING_GAMMA = 0.128


def random_packing(adhesive: bool = True, n: int = 500, d: float = 6.0, g: float = 8e-4,
                   seed: int = 35) -> Workload:
    """Sec. 3.5: n spheres of diameter d placed at random in a 100 x 50 x 50
    box (walls at the ends of the 100-long x axis, periodic y and z), D3Q19
    tau = 2, settling under gravity g along -x onto the wall at x = -1/2;
    adhesive (JKR, gamma = PACKING_GAMMA) or not (Hertz, gamma = 0), with
    sliding, twisting and rolling friction."""
    lat = LatticeSpec(q=19, nx=100, ny=50, nz=50, tau=2.0,
                      faces=(BOUNCE_BACK, BOUNCE_BACK, PERIODIC, PERIODIC, PERIODIC, PERIODIC))
    rng = np.random.default_rng(seed)
    r = np.full(n, d / 2.0)
    x = rsa(rng, r, (100.0, 50.0, 50.0), (False, True, True), gap=0.5, clearance=0.5)
    dem = DemSpec(g=(-g, 0.0, 0.0), gamma=PACKING_GAMMA if adhesive else 0.0, **PACKING_DEM)
    kind = "adhesive (JKR)" if adhesive else "non-adhesive (Hertz)"
    return Workload(f"packing_{'adh' if adhesive else 'hertz'}", lat, _particles(x, r=r),
                    steps=60_000, dem=dem,
                    description=f"D3Q19 tau=2 100x50x50, walls on x, {n} {kind} spheres d={d} "
                    f"seed {seed}, gravity {g} along -x, sliding/twisting/rolling friction")


WORKLOADS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5}


def random_state(lat: LatticeSpec, seed: int, amp: float = 1e-2) -> np.ndarray:
    """A seeded non-equilibrium distribution field f[Q, nz, ny, nx] around
    w_i * rho0 built from uniform noise: f_i = rho0 / Q * (1 + amp * xi) with
    xi ~ U(-1, 1) -- a generic positive state for one-step parity checks."""
    rng = np.random.default_rng(seed)
    f = lat.rho0 / lat.q * (1.0 + amp * rng.uniform(-1.0, 1.0, size=(lat.q,) + lat.shape))
    return np.ascontiguousarray(f)
