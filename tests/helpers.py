"""Shared helpers of the GPU parity tests: run the same seeded case through
the FP64 oracle and through the HIP library (via its C ABI)."""
import numpy as np

import oracle
import workloads as W


def relerr(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def oracle_run(lat, f0, p, steps, mode=0):
    L = oracle.Lattice(lat, f0)
    F = T = None
    for _ in range(steps):
        F, T = L.step(p, mode)
    return L, F, T


def gpu_lattice(lat, p, precision="fp64", cap=64, rmax=None, weighting="modified"):
    import paper_1901_09745_amd.psclbm as P
    n = 0 if p is None else p.n
    rm = rmax if rmax is not None else (float(p.r.max()) if n else 1.0)
    return P.Lattice(lat, precision, max_particles=max(n, 1), max_radius=rm,
                     max_tile_particles=cap, weighting=weighting)


def gpu_run(lat, f0, p, steps, precision="fp64", cap=64, weighting="modified"):
    import torch
    import paper_1901_09745_amd.psclbm as P
    G = gpu_lattice(lat, p, precision, cap, weighting=weighting)
    if f0 is not None:
        G.set_f(torch.from_numpy(np.ascontiguousarray(f0)).cuda())
    dp = None if p is None or p.n == 0 else P.DeviceParticles.from_host(p)
    G.rasterize(dp)
    G.step(steps)
    F, T = G.forces()
    G.sync()
    return G, G.get_f().cpu().numpy(), F.cpu().numpy(), T.cpu().numpy()


def force_scale(lat, f, p):
    """L1 size of the summands of Eq. 14 for each particle, B_s*|rho(u_s-u)+F|
    bounded by |rho(u_s-u)| + |F| over the covered cells (a conservative
    scale for the order-dependent FP64 rounding of the force sums)."""
    nslot, ids, eps, _ = oracle.rasterize(lat, p.x, p.r)
    L = oracle.Lattice(lat, f)
    rho, u = L.macros()
    rho = rho.reshape(-1)
    absu = np.abs(u.reshape(-1, 3)).sum(axis=1)
    absU = np.abs(p.u).sum(axis=1)
    absW = np.abs(p.omega).sum(axis=1) * 20
    absF = float(np.abs(np.asarray(lat.force)).sum())
    scale = np.zeros(p.n)
    covered = np.nonzero(nslot)[0]
    for k in range(ids.shape[1]):
        sel = covered[nslot[covered] > k]
        if sel.size == 0:
            break
        s = ids[sel, k]
        np.add.at(scale, s, rho[sel] * (absu[sel] + absU[s] + absW[s]) + absF)
    return scale


def force_floor(lat, f, p):
    """Absolute rounding floor of each particle's Eq. 14 sum: u = (sum_i e_i
    f_i + F/2)/rho carries up to (Q-1) eps of error from the direction sum
    (|f_i| summing to rho), so each covered cell's summand B_s rho (u_s - u)
    may differ by rho (Q-1) eps between two FP64 evaluations, on both sides:
    2 (Q-1) eps sum_n rho_n over the particle's cells (B_s <= 1)."""
    nslot, ids, eps, _ = oracle.rasterize(lat, p.x, p.r)
    rho, _ = oracle.Lattice(lat, f).macros()
    rho = rho.reshape(-1)
    floor = np.zeros(p.n)
    covered = np.nonzero(nslot)[0]
    for k in range(ids.shape[1]):
        sel = covered[nslot[covered] > k]
        np.add.at(floor, ids[sel, k], rho[sel])
    return 2 * (lat.q - 1) * np.finfo(np.float64).eps * floor


WALLS_Y = (W.PERIODIC, W.PERIODIC, W.BOUNCE_BACK, W.BOUNCE_BACK, W.PERIODIC, W.PERIODIC)


def _print_case(**kw):
    print("case:", ", ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _particles(lat, n, rmin, rmax, seed, umax=0.01, wmax=0.002, overlap=False):
    rng = np.random.default_rng(seed)
    dim = 2 if lat.q == 9 else 3
    box = (lat.nx, lat.ny, lat.nz)[:dim]
    periodic = tuple(lat.periodic(a) for a in range(dim))
    r = np.sort(rng.uniform(rmin, rmax, n))[::-1]
    gap = -0.6 * rmin if overlap else 0.3
    x = W.rsa(rng, r, tuple(float(b) for b in box), periodic, gap=gap, clearance=0.5)
    u = rng.uniform(-umax, umax, (n, 3))
    w = rng.uniform(-wmax, wmax, (n, 3))
    if dim == 2:
        u[:, 2] = 0
        w[:, :2] = 0
        x[:, 2] = 0
    return W.Particles(x, u, w, r)


CASES = {
    "d2q9_periodic": W.LatticeSpec(q=9, nx=150, ny=70, tau=0.7, force=(1e-5, -3e-6, 0)),
    "d2q9_walls": W.LatticeSpec(q=9, nx=130, ny=37, tau=0.8, force=(2e-5, 0, 0), faces=WALLS_Y),
    "d2q9_couette": W.LatticeSpec(q=9, nx=67, ny=29, tau=0.9, faces=(
        W.PERIODIC, W.PERIODIC, W.MOVING_WALL, W.MOVING_WALL, W.PERIODIC, W.PERIODIC),
        face_u=((0, 0, 0), (0, 0, 0), (-0.01, 0, 0), (0.02, 0.001, 0), (0, 0, 0), (0, 0, 0))),
    "d2q9_open": W.LatticeSpec(q=9, nx=100, ny=45, tau=0.8, faces=(
        W.INLET_EQ, W.OUTLET_EQ, W.BOUNCE_BACK, W.BOUNCE_BACK, W.PERIODIC, W.PERIODIC),
        face_u=((0.02, 0.0, 0),) + ((0, 0, 0),) * 5),
    # x = nx - 1 = 128 starts a 64-cell row segment: its outlet velocity comes
    # from the separate pre-pass, not from the neighbour lane
    "d2q9_open_seam": W.LatticeSpec(q=9, nx=129, ny=40, tau=0.75, force=(1e-6, 0, 0), faces=(
        W.INLET_EQ, W.OUTLET_EQ, W.BOUNCE_BACK, W.BOUNCE_BACK, W.PERIODIC, W.PERIODIC),
        face_u=((0.015, 0.002, 0),) + ((0, 0, 0),) * 5),
    "d3q19_periodic": W.LatticeSpec(q=19, nx=70, ny=21, nz=18, tau=0.6, force=(1e-5, 0, 2e-6)),
    # outlets on x = 0 (neighbour lane) and y = 0 (pre-pass), an inlet on
    # x = nx - 1; the corners take the later outlet and then the inlet
    "d3q19_open": W.LatticeSpec(q=19, nx=40, ny=30, nz=20, tau=0.7, faces=(
        W.OUTLET_EQ, W.INLET_EQ, W.OUTLET_EQ, W.BOUNCE_BACK, W.PERIODIC, W.PERIODIC),
        face_u=((0, 0, 0), (-0.02, 0.0, 0.003), (0, 0, 0), (0, 0, 0), (0, 0, 0), (0, 0, 0))),
    "d3q19_walls": W.LatticeSpec(q=19, nx=33, ny=26, nz=22, tau=0.65, force=(-1e-5, 0, 0), faces=(
        W.BOUNCE_BACK, W.MOVING_WALL, W.PERIODIC, W.PERIODIC, W.BOUNCE_BACK, W.BOUNCE_BACK),
        face_u=((0, 0, 0), (0, 0.01, -0.005), (0, 0, 0), (0, 0, 0), (0, 0, 0), (0, 0, 0))),
}




def case_particles(lat, seed=3):
    """The overlapping particle sets used with CASES."""
    if lat.q == 9:
        return _particles(lat, 6, 4.0, 9.0, seed=seed, overlap=True)
    return _particles(lat, 5, 3.0, 5.0, seed=seed + 1, overlap=True)
