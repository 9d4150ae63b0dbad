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


def gpu_lattice(lat, p, precision="fp64", cap=64, rmax=None):
    import paper_1901_09745_amd.psclbm as P
    n = 0 if p is None else p.n
    rm = rmax if rmax is not None else (float(p.r.max()) if n else 1.0)
    return P.Lattice(lat, precision, max_particles=max(n, 1), max_radius=rm,
                     max_tile_particles=cap)


def gpu_run(lat, f0, p, steps, precision="fp64", cap=64):
    import torch
    import paper_1901_09745_amd.psclbm as P
    G = gpu_lattice(lat, p, precision, cap)
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
    u = u.reshape(-1, 3)
    scale = np.zeros(p.n)
    F = np.asarray(lat.force)
    for n in np.nonzero(nslot)[0]:
        for k in range(nslot[n]):
            s = ids[n, k]
            scale[s] += rho[n] * (np.abs(u[n]).sum() + np.abs(p.u[s]).sum() +
                                  np.abs(p.omega[s]).sum() * 20) + np.abs(F).sum()
    return scale
