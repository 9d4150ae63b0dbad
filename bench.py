"""Benchmark of the MI355X PSC-LBM hot path.

One "step" is one time step of the whole hot path on the 3D workload (D3Q19
tau=0.6, 256^3 periodic, 8000 spheres r~U(4,6) with prescribed velocities
~N(0, 1e-3^2)), in the FP32-compute / FP32-shifted-storage form:
rasterisation of the spheres at their current positions -> the fused PSC
collide-stream with the Eq. 14 force/torque reduction and the FP64 mass
partials -> the particle update (advection by the prescribed velocity, with
the next step's rasterisation fused into it), run by coupled_step.  Its
distributions (1.27 GB in FP32) live in HBM, far beyond the 256 MB last-level
cache.  Inputs are resident in HBM before the timed region; the timed region
is the median of five repetitions of max(--steps, 200) steps.

The JSON line reports:
  value          MLUPS (lattice cell updates per second / 1e6) of that step;
  roofline       its dominant kernel, the fused collide-stream k_step<19,fp32>:
                 algorithmic bytes 2*Q*s per cell per launch over its average
                 launch duration (HIP events around each launch on the
                 library's stream), against the 8 TB/s HBM peak;
  ceiling        the same volume moved by the library's own copy kernel and by
                 the even step's data movement without arithmetic, GB/s;
  forms_3d       the 3D workload in the FP64 and FP16-storage forms, with each
                 form's velocity / drag / mass-drift error against FP64;
  packing_3d     the 3D packing workload (D3Q19 tau=0.65 384x192x192, walls on
                 x, 20000 JKR spheres settling under gravity, FP16 storage),
                 coupled steps with DEM contacts, and its forms' errors;
  cache_resident the 2D workload (D2Q9 tau=0.7 1024^2 periodic, 2000 JKR
                 disks), whose distributions fit in the last-level cache, and
                 its forms' errors;
  adjoint        differentiable runs of the drag through torch.autograd
                 (forward with checkpoints, backward by ring recompute + the
                 hand-written FP64 adjoint): the time of the backward over
                 that of the forward, on the 2D inlet/outlet channel (D2Q9
                 tau=0.8 512x256, 64 fixed disks r=8, 4000 steps, checkpoint
                 every 100, J = drag of disk 0 at the last step) and on the
                 last 500 steps of a 20000-step settling run of the 3D
                 packing (checkpoint every 50, J = drag of the 100 lowest
                 spheres summed over the 500 steps), the window with FP64 and
                 with FP16-storage forwards;
  cpu_baseline   the FP64 oracle timed on the host, at all cores and at one
                 thread, on bounded samples of the 3D workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-3d]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
STORE_BYTES = {"fp64": 8, "fp32": 4, "fp16": 2}
DTYPE = {"fp64": "f64", "fp32": "f32", "fp16": "f32 (f16 storage)"}
METRIC = "PSC-LBM MLUPS & % HBM peak (FP64/FP32/FP16-store); adjoint/forward time ratio"


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def run_form(w, form, steps, warmup, coupled=True, observe=False, reps=1, ksteps=100,
             cap=64):
    """Time `steps` coupled steps of workload w in precision form `form`
    (coupled_step: rasterize -> fused collide-stream with forces -> DEM or
    advection, the next step's rasterisation fused into the DEM kernel), `reps`
    times, then `ksteps` step-kernel launches between event pairs.  Returns
    (median ms per coupled step, mean step-kernel ms, observation or None,
    details: every repetition's ms per step and the even / odd step-kernel
    means)."""
    import torch
    import paper_1901_09745_amd.psclbm as P

    lat = w.lattice
    rmax = float(w.particles.r.max())
    G = P.Lattice(lat, form, max_particles=w.particles.n, max_radius=rmax,
                  max_tile_particles=cap, max_contacts=16)
    p = P.DeviceParticles.from_host(w.particles)
    n = p.n
    prm = P.make_dem_params(w.dem)
    ctx = G.ctx

    def one(k_ev=None):
        # the three calls of a coupled step, with an event pair around the
        # step kernel's launch
        P.psc_rasterize(ctx, p.x, p.u, p.omega, p.r)
        if k_ev is not None:
            k_ev[0].record()
        P.lbm_step(ctx, 1)
        if k_ev is not None:
            k_ev[1].record()
        if coupled:
            # the DEM reads the step's FP64 force/torque accumulators in place
            P.dem_step(ctx, prm, p.x, p.u, p.omega, p.r, None, None)

    def run(nsteps):
        # nsteps coupled steps in one call (rasterize -> step -> DEM each)
        P.coupled_step(ctx, prm, p.x, p.u, p.omega, p.r, nsteps)

    mass0 = G.mass()
    run(warmup)
    torch.cuda.synchronize()
    G.sync()
    # timed regions: the coupled steps alone
    per = []
    for _ in range(reps):
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        run(steps)
        end.record()
        torch.cuda.synchronize()
        per.append(start.elapsed_time(end) / steps)
    G.sync()
    # the same workload continued as separate calls, with an event pair around
    # each step-kernel launch (on the library's stream, torch's current
    # stream); launches alternate between the even and the odd step
    par0 = P.lbm_step_count(ctx) % 2
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(ksteps)]
    for k in range(ksteps):
        one(evs[k])
    torch.cuda.synchronize()
    kt = [a.elapsed_time(b) for a, b in evs]
    kern_ms = float(np.mean(kt))
    even = [t for k, t in enumerate(kt) if (par0 + k) % 2 == 0]
    odd = [t for k, t in enumerate(kt) if (par0 + k) % 2 == 1]
    G.sync()
    mass = G.mass()
    if not np.isfinite(mass):
        raise RuntimeError("non-finite mass")
    obs = None
    if observe:
        Fo = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
        P.particle_forces(ctx, Fo, None)
        _, uo = G.macros()
        obs = {"F": Fo.clone(), "u": uo, "mass0": mass0, "mass1": mass}
    del G
    torch.cuda.empty_cache()
    det = {"ms_per_step_reps": per,
           "step_kernel_ms_even": float(np.mean(even)) if even else None,
           "step_kernel_ms_odd": float(np.mean(odd)) if odd else None}
    return float(np.median(per)), kern_ms, obs, det


def form_errors(obs, ref):
    """Velocity, drag and mass-drift error of each form's observation against
    the FP64 form's on the same trajectory (the FP64 form matches the oracle
    within 1e-12 per step)."""
    out = {}
    for form, ob in obs.items():
        du = float((ob["u"] - ref["u"]).abs().max() / ref["u"].abs().max())
        dF = float((ob["F"] - ref["F"]).abs().max() / max(float(ref["F"].abs().max()), 1e-300))
        out[form] = {"velocity_max_rel_err": du, "drag_max_rel_err": dF,
                     "mass_drift_rel": (ob["mass1"] - ob["mass0"]) / ob["mass0"],
                     "mass_vs_fp64_rel": (ob["mass1"] - ref["mass1"]) / ref["mass1"]}
    return out


def ceilings(n_cells, q=19, reps=20):
    """The library's bandwidth-ceiling kernels on the volume of one lattice of
    n_cells cells and q FP32 distributions: a streaming copy of that many
    bytes, and the even step's data movement without arithmetic (read and
    write in place).  Median GB/s over `reps` launches each."""
    import torch
    import paper_1901_09745_amd.psclbm as P

    # non-zero data: zero-filled lines can move less than their size
    a = torch.ones((q, n_cells), dtype=torch.float32, device="cuda")
    b = torch.ones_like(a)
    out = {}
    for name, fn in (("copy", lambda: P.psclbm_stream_copy(a, b)),
                     ("swap", lambda: P.psclbm_stream_swap(a, q))):
        for _ in range(3):
            fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        out[name] = {"GBs": 2 * 4 * q * n_cells / (ms * 1e-3) / 1e9, "ms": ms}
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_moved": 2 * 4 * q * n_cells,
            "copy_GBs": out["copy"]["GBs"], "swap_GBs": out["swap"]["GBs"],
            "attainable_GBs": max(out["copy"]["GBs"], out["swap"]["GBs"]),
            "note": "psclbm_stream_copy (16-byte non-temporal loads and stores per thread) and "
                    "psclbm_stream_swap (the even step's in-place exchange of the 19 FP32 "
                    "arrays, no arithmetic), each the median of 20 launches"}


def run_adjoint(lat, p, steps, every, label, select, precision="fp64", f0=None, window=1):
    """Forward and backward wall time of a differentiable run from state f0
    (None: rest): J = the x drag (Eq. 14) summed over the last `window` of
    `steps` steps and over the particles `select`, with its gradient w.r.t.
    all particle
    positions, velocities, spins and the face velocities (checkpoint every
    `every` steps).  The run is made twice and the second one is timed."""
    import torch
    from paper_1901_09745_amd.autograd import psc_drag

    dev = "cuda"
    r = torch.tensor(p.r, device=dev)
    sel = torch.as_tensor(select, device=dev)

    def once():
        x = torch.tensor(p.x, device=dev, requires_grad=True)
        u = torch.tensor(p.u, device=dev, requires_grad=True)
        om = torch.tensor(p.omega, device=dev, requires_grad=True)
        fu = torch.tensor(np.asarray(lat.face_u, dtype=np.float64), device=dev,
                          requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F, _ = psc_drag(x, u, om, fu, lat, r, steps, checkpoint_every=every, window=window,
                        precision=precision, f0=f0)
        J = F[sel, 0].sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        J.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        gx = float(x.grad.abs().max())
        if not (np.isfinite(gx) and torch.isfinite(fu.grad).all()):
            raise RuntimeError("non-finite adjoint")
        return (t1 - t0) * 1e3, (t2 - t1) * 1e3, float(J.detach()), gx

    once()                             # warm-up (allocator and code paths)
    fwd, bwd, J, gx = once()
    torch.cuda.empty_cache()
    return {"workload": label, "cells": lat.ncells, "particles": p.n,
            "forward_precision": precision, "adjoint_precision": "fp64", "steps": steps,
            "checkpoint_every": every, "window": window, "J": J, "max_abs_dJ_dX": gx, "forward_ms": fwd,
            "backward_ms": bwd, "ratio": bwd / fwd, "forward_ms_per_step": fwd / steps,
            "backward_ms_per_step": bwd / steps}


def run_coupled_gradient(w, steps, every=10):
    """Gradient of a coupled run with moving particles (autograd.coupled_run:
    forward with a checkpoint every `every` steps, backward replaying each
    segment and walking it back through dem_step_adjoint and
    lbm_step_adjoint), FP64, J = the mean x of the particles at the end:
    wall-clock forward and backward, each measured on a second call."""
    import torch
    import paper_1901_09745_amd.psclbm as P
    from paper_1901_09745_amd.autograd import coupled_run

    p = w.particles
    G = P.Lattice(w.lattice, "fp64", max_particles=p.n, max_radius=float(p.r.max()))
    f0 = G.get_f()                              # the equilibrium at rest
    del G
    r = torch.from_numpy(np.ascontiguousarray(p.r)).cuda()
    res = None
    for _ in range(2):
        xs = [torch.tensor(np.ascontiguousarray(m), dtype=torch.float64, device="cuda",
                           requires_grad=True) for m in (p.x, p.u, p.omega)]
        fin = f0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, _, _, _ = coupled_run(*xs, fin, w.lattice, r, w.dem, steps, checkpoint_every=every)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        grads = torch.autograd.grad(X[:, 0].mean(), xs + [fin])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res = {"steps": steps, "checkpoint_every": every,
               "forward_ms": (t1 - t0) * 1e3, "backward_ms": (t2 - t1) * 1e3,
               "ratio": (t2 - t1) / (t1 - t0),
               "dJ_dx_norm": float(grads[0].norm()), "dJ_df0_norm": float(grads[3].norm())}
        del X, grads
    torch.cuda.empty_cache()
    return res


def settle_packing(w, nsteps):
    """The 3D packing after nsteps coupled steps from rest (FP16 storage, JKR
    DEM, gravity): its canonical FP64 state and particle state."""
    import torch
    import paper_1901_09745_amd.psclbm as P
    import workloads as W

    p = w.particles
    G = P.Lattice(w.lattice, "fp16", max_particles=p.n, max_radius=float(p.r.max()),
                  max_tile_particles=64, max_contacts=16)
    dp = P.DeviceParticles.from_host(p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G.coupled_step(P.make_dem_params(w.dem), dp, nsteps)
    G.sync()
    ms = (time.perf_counter() - t0) * 1e3 / nsteps
    f0 = G.get_f()
    G.sync()
    ps = W.Particles(dp.x.cpu().numpy(), dp.u.cpu().numpy(), dp.omega.cpu().numpy(),
                     dp.r.cpu().numpy())
    del G
    torch.cuda.empty_cache()
    info = {"steps": nsteps, "form": "fp16", "ms_per_step": ms,
            "mlups": w.lattice.ncells / (ms * 1e-3) / 1e6,
            "note": "coupled steps (rasterize + PSC collide-stream + JKR DEM) in one call, "
                    "wall clock"}
    return f0, ps, info


FRICTION = {"k_t": 1e-3, "eta_t": 0.02, "mu_f": 0.3, "theta_r": 0.02}


def run_friction(w, f0, ps, steps, warmup=5, ksteps=20):
    """The settled 3D packing (canonical state f0, particles ps) continued in
    the FP16 form without and with sliding, twisting and rolling friction
    (Eqs. 22, 28, 29): ms per coupled step (contacts gathered by the step
    kernel without friction, by the DEM kernel with it), and the DEM step
    alone (binning and the contact kernel) between event pairs on the
    library's stream."""
    import dataclasses
    import torch
    import paper_1901_09745_amd.psclbm as P

    out = {}
    cases = (("frictionless", w.dem), ("friction", dataclasses.replace(w.dem, **FRICTION)))
    for label, dem in cases:
        G = P.Lattice(w.lattice, "fp16", max_particles=ps.n, max_radius=float(ps.r.max()),
                      max_tile_particles=64, max_contacts=16)
        G.set_f(f0)
        dp = P.DeviceParticles.from_host(ps)
        prm = P.make_dem_params(dem)
        G.coupled_step(prm, dp, warmup)
        G.sync()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        G.coupled_step(prm, dp, steps)
        end.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(end) / steps
        G.sync()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(ksteps)]
        for a, b in evs:
            a.record()
            P.dem_step(G.ctx, prm, dp.x, dp.u, dp.omega, dp.r, None, None)
            b.record()
        torch.cuda.synchronize()
        G.sync()
        out[label] = {"ms_per_step": ms, "mlups": w.lattice.ncells / (ms * 1e-3) / 1e6,
                      "dem_step_ms": float(np.mean([a.elapsed_time(b) for a, b in evs]))}
        if label == "frictionless":
            # the adjoint of one DEM step (its contact set held), event-timed
            before = P.DeviceParticles(dp.x.clone(), dp.u.clone(), dp.omega.clone(), dp.r)
            P.dem_step(G.ctx, prm, dp.x, dp.u, dp.omega, dp.r, None, None)
            g = [torch.randn_like(dp.x) for _ in range(3)]
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(ksteps)]
            for a, b in evs:
                a.record()
                G.dem_step_adjoint(prm, before, *g)
                b.record()
            torch.cuda.synchronize()
            G.sync()
            out[label]["dem_step_adjoint_ms"] = float(np.mean([a.elapsed_time(b) for a, b in evs]))
        del G
        torch.cuda.empty_cache()
    out["params"] = dict(FRICTION)
    out["steps"] = steps
    return out


def packing_stats(x, r, L, periodic, reach=0.0):
    """Packing fraction and coordination number of a bed settled along -x
    onto the wall at x = -1/2: phi is the solid fraction of the slab from 2d
    above the wall to 2d below the bed's top (the highest sphere surface),
    Z the mean number of sphere-sphere contacts (centres closer than
    r_i + r_j + reach, nearest image on periodic axes) of the spheres whose
    centres lie in that slab."""
    x = np.asarray(x, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    d = 2.0 * float(r.max())
    lo = -0.5 + 2.0 * d
    hi = float((x[:, 0] + r).max()) - 2.0 * d
    if hi <= lo:
        return {"phi": None, "Z": None, "slab": [lo, hi]}
    # volume of each sphere between the planes x = lo and x = hi
    a = np.clip(lo - x[:, 0], -r, r)
    b = np.clip(hi - x[:, 0], -r, r)
    vol = np.pi * ((r ** 2) * (b - a) - (b ** 3 - a ** 3) / 3.0)
    phi = float(vol.sum() / ((hi - lo) * L[1] * L[2]))
    dv = x[None, :, :] - x[:, None, :]
    for ax in (1, 2):
        if periodic[ax]:
            dv[:, :, ax] -= L[ax] * np.round(dv[:, :, ax] / L[ax])
    dist = np.sqrt((dv ** 2).sum(axis=2))
    touch = dist < (r[:, None] + r[None, :] + reach)
    np.fill_diagonal(touch, False)
    inside = (x[:, 0] > lo) & (x[:, 0] < hi)
    Z = float(touch[inside].sum(axis=1).mean()) if inside.any() else None
    return {"phi": phi, "Z": Z, "slab": [lo, hi], "spheres_in_slab": int(inside.sum())}


def run_packing(steps, chunk=10000, precision="fp32"):
    """Sec. 3.5: the 500-sphere random packing settled from a random
    placement, adhesive (JKR) and non-adhesive (Hertz), both with sliding,
    twisting and rolling friction; phi and Z every chunk steps."""
    import torch
    import paper_1901_09745_amd.psclbm as P
    import workloads as W

    out = {}
    for adhesive in (True, False):
        w = W.random_packing(adhesive)
        lat, p, dem = w.lattice, w.particles, w.dem
        G = P.Lattice(lat, precision, max_particles=p.n, max_radius=float(p.r.max()),
                      max_tile_particles=64, max_contacts=dem.max_contacts)
        dp = P.DeviceParticles.from_host(p)
        prm = P.make_dem_params(dem)
        # bonded pairs reach down to -delta_C (Eq. 27 with R = r/2)
        R = float(p.r[0]) / 2.0
        Es = dem.E_p / (2.0 * (1.0 - dem.poisson ** 2))
        a0 = (9.0 * np.pi * dem.gamma * R * R / Es) ** (1.0 / 3.0)
        reach = a0 * a0 / (2.0 * 6.0 ** (1.0 / 3.0) * R)
        hist = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            k = min(chunk, steps - done)
            G.coupled_step(prm, dp, k)
            done += k
            G.sync()
            st = packing_stats(dp.x.cpu().numpy(), p.r, (lat.nx, lat.ny, lat.nz),
                               (False, True, True), reach)
            umax = float(dp.u.abs().max())
            umean = float(dp.u.norm(dim=1).mean())
            hist.append({"step": done, "phi": st["phi"], "Z": st["Z"], "u_max": umax,
                         "u_mean": umean})
            _log(f"bench: packing {'adhesive' if adhesive else 'Hertz'} step {done}: "
                 f"phi={st['phi']}, Z={st['Z']}, u_max={umax:.2e}, u_mean={umean:.2e}")
        ms = (time.perf_counter() - t0) * 1e3 / steps
        out["adhesive" if adhesive else "non_adhesive"] = {
            "phi": hist[-1]["phi"], "Z": hist[-1]["Z"], "history": hist,
            "ms_per_step": ms, "contact_reach": reach}
        del G
        torch.cuda.empty_cache()
    out["paper"] = {"adhesive": {"phi": 0.495, "Z": 5.08},
                    "non_adhesive": {"phi": 0.557, "Z": 5.50}}
    return out


def run_ergun(dps, res, weightings, chunk=500, tol=1e-6, max_steps=200_000):
    """Sec. 3.4 packed bed (8 fixed spheres in simple-cubic contact, periodic
    2 d_p cube, body force): each case run to steady state in the FP64 form
    (relative change of the superficial velocity below `tol` per `chunk`
    steps), then Eq. 36's Re_p* and dP* against Eq. 35."""
    import time
    import torch
    import paper_1901_09745_amd.psclbm as P
    import workloads as W

    out = []
    for dp in dps:
        for re in res:
            w = W.ergun(dp, re)
            lat = w.lattice
            for wt in weightings:
                G = P.Lattice(lat, "fp64", max_particles=8, max_radius=dp / 2.0,
                              max_tile_particles=64, weighting=wt)
                G.rasterize(P.DeviceParticles.from_host(w.particles))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                steps, U_prev, U = 0, None, 0.0
                while steps < max_steps:
                    G.step(chunk)
                    steps += chunk
                    rho, u = G.macros()
                    # superficial velocity: flux through the plane x = 0 over its area
                    U = float((rho[:, :, 0] * u[:, :, 0, 0]).mean()) / lat.rho0
                    if not np.isfinite(U):   # unstable (lattice too coarse for the velocity)
                        break
                    if U_prev is not None and abs(U - U_prev) < tol * abs(U):
                        break
                    U_prev = U
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                stable = bool(np.isfinite(U))
                rec = {"d_p": dp, "Re_target": re, "weighting": wt, "cells": lat.ncells,
                       "steps": steps, "stable": stable,
                       "converged": stable and steps < max_steps,
                       "seconds": dt, "mlups": lat.ncells * steps / dt / 1e6,
                       "U": None, "Re_p*": None, "dP*": None, "dP*_Eq35": None,
                       "rel_err": None}
                if stable:
                    re_m, dps_m = W.ergun_numbers(lat.force[0], U, dp, lat.tau)
                    ref = W.ergun_dp_star(re_m)
                    rec.update({"U": U, "Re_p*": re_m, "dP*": dps_m, "dP*_Eq35": ref,
                                "rel_err": dps_m / ref - 1.0})
                    _log(f"bench: ergun d_p={dp} Re*={re_m:.3f} {wt}: dP*={dps_m:.2f} vs "
                         f"{ref:.2f} ({dps_m / ref - 1.0:+.4f}), {steps} steps")
                else:
                    _log(f"bench: ergun d_p={dp} target Re*={re} {wt}: unstable after "
                         f"{steps} steps")
                out.append(rec)
                del G
    return out


def run_drag(cases, precision="fp32", chunk=1000, tol=1e-5, max_steps=150_000):
    """Sec. 3.2 fixed sphere in a 20d x 10d x 10d box (equilibrium inlet u0,
    constant-pressure outlet and open sides): each case (d_p, Re_p, u0) run
    until, after five flow-through times, the drag changes by less than `tol`
    per `chunk` steps; the drag coefficient (Eq. 32) against Eq. 33."""
    import time
    import torch
    import paper_1901_09745_amd.psclbm as P
    import workloads as W

    out = []
    for dp, re, u0 in cases:
        w = W.sphere_drag(dp, re, u0)
        lat = w.lattice
        G = P.Lattice(lat, precision, max_particles=1, max_radius=dp / 2.0,
                      max_tile_particles=64)
        G.rasterize(P.DeviceParticles.from_host(w.particles))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps, prev, fx = 0, None, float("nan")
        min_steps = int(5 * lat.nx / u0)
        while steps < max_steps:
            G.step(chunk)
            steps += chunk
            F, _ = G.forces()
            fx = float(F[0, 0])
            if not np.isfinite(fx):
                break
            if steps >= min_steps and prev is not None and abs(fx - prev) < tol * abs(fx):
                break
            prev = fx
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        stable = bool(np.isfinite(fx))
        cd = W.drag_coefficient(fx, u0, dp) if stable else None
        ref = W.schiller_naumann(re)
        out.append({"d_p": dp, "Re_p": re, "u0": u0, "tau": lat.tau, "cells": lat.ncells,
                    "precision": precision, "steps": steps, "stable": stable,
                    "converged": stable and steps < max_steps, "seconds": dt,
                    "mlups": lat.ncells * steps / dt / 1e6, "C_d": cd, "C_d_Eq33": ref,
                    "rel_err": (cd / ref - 1.0) if stable else None})
        _log(f"bench: drag d_p={dp} Re_p={re} u0={u0}: C_d="
             + (f"{cd:.4f} vs {ref:.4f} ({cd / ref - 1.0:+.4f})" if stable else "unstable")
             + f", {steps} steps")
        del G
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(w, budget_s, threads):
    """The FP64 oracle's coupled steps of workload w (Table 1 + the PSC step +
    the particle update), timed for about budget_s seconds at `threads`
    OpenMP threads: (MLUPS, steps, seconds)."""
    import oracle

    oracle.set_num_threads(threads)
    L = oracle.Lattice(w.lattice)
    D = oracle.Dem(w.lattice, w.dem, w.particles.n)
    p = w.particles.copy()
    steps, t0 = 0, time.perf_counter()
    while True:
        F, T = L.step(p)
        D.step(p, F, T)
        steps += 1
        dt = time.perf_counter() - t0
        if dt >= budget_s or dt / steps * (steps + 1) > 1.5 * budget_s:
            break
    return w.lattice.ncells * steps / dt / 1e6, steps, dt


def cpu_baseline(budget_s=15.0):
    """The FP64 oracle on the host on bounded samples of the 3D workload: at
    every core the benchmark's own 256^3 workload, at one thread the same
    recipe at half the linear size (128^3, 1000 spheres: the rate per cell is
    that of the full box, whose single-thread step alone would take close to
    a minute)."""
    import oracle
    import workloads as W

    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    full = W.c3()
    v_all, n_all, t_all = _oracle_rate(full, budget_s, cores)
    half = W.c3(scale=0.5)
    v_one, n_one, t_one = _oracle_rate(half, budget_s, 1)
    oracle.set_num_threads(cores)
    return {"value": v_all, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": f"{n_all} coupled FP64 steps of the 256^3 / 8000-sphere workload in "
                      f"{t_all:.1f} s, OpenMP cell loop on {cores} threads",
            "one_thread": {"value": v_one, "unit": "MLUPS", "cores": 1,
                           "sample": f"{n_one} coupled FP64 steps of the same recipe at "
                                     f"128^3 / {half.particles.n} spheres in {t_one:.1f} s"},
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count()}


# the sources the step kernel is compiled from
KERNEL_SOURCES = ("lbm.hip", "common.hpp", "tiles.hpp", "dem.hpp", "dem.hip")


def kernel_digest():
    """sha256 prefix over the step kernel's sources (the staleness key of the
    committed counter summary)."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1901_09745_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def _traffic(kernel_key):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    digest = kernel_digest()
    data = json.load(open(path))
    ent = data.get(kernel_key)
    if not ent or ent.get("source_sha256_16") != digest:
        return None
    return ent.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--reps", type=int, default=5, help="timed repetitions (median reported)")
    ap.add_argument("--forms", default="fp32,fp64,fp16")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-3d", action="store_true", help="skip the 3D packing and adjoint legs")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--adjoint-steps", type=int, default=4000,
                    help="steps of the differentiable channel run (0: skip)")
    ap.add_argument("--adjoint-3d-steps", type=int, default=500,
                    help="steps of the differentiable 3D packing window (0: skip)")
    ap.add_argument("--settle-steps", type=int, default=19500,
                    help="coupled steps that settle the 3D packing before its window")
    ap.add_argument("--friction-steps", type=int, default=100,
                    help="coupled steps of the settled 3D packing timed without and with "
                         "friction (needs the 3D adjoint leg's packing; 0 skips)")
    ap.add_argument("--packing-steps", type=int, default=60000,
                    help="coupled steps of the Sec. 3.5 random packings (0 skips)")
    ap.add_argument("--ergun-dps", default="10,20,40,80",
                    help="sphere diameters of the packed-bed (Sec. 3.4) runs ('' to skip)")
    ap.add_argument("--no-drag", action="store_true",
                    help="skip the fixed-sphere drag runs (Sec. 3.2)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the 3D workload's forms, the ceilings and the 3D packing in FP16 "
                         "(for profiler runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 1 GiB three times with the library's streaming copy (the "
                         "reference dispatch that scales the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: one GPU is measured; --gpus {args.gpus} is not supported (the "
              "multi-GPU domain decomposition is designed, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        import paper_1901_09745_amd.psclbm as P
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            P.psclbm_stream_copy(a, b)
        torch.cuda.synchronize()
        del a, b
    steps = max(args.steps, 200)
    reps = max(args.reps, 1)
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    head = "fp32" if "fp32" in forms else forms[0]

    # ---- the headline: the 3D workload, every form, FP32 first ----
    _log("bench: generating the 3D workload")
    w3 = W.c3()
    N3 = w3.lattice.ncells
    res3, obs3 = {}, {}
    for form in [head] + [f for f in forms if f != head]:
        _log(f"bench: 3D coupled step, form {form}")
        ms, kms, ob, det = run_form(w3, form, steps, args.warmup, observe=True, reps=reps)
        obs3[form] = ob
        b = 2 * 19 * STORE_BYTES[form] * N3
        res3[form] = {"mlups": N3 / (ms * 1e-3) / 1e6, "ms_per_step": ms,
                      "step_kernel_ms": kms, "step_kernel_GBs": b / (kms * 1e-3) / 1e9,
                      "frac_of_hbm_peak": b / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "bytes_per_launch": b, **det}
    if "fp64" in obs3:
        for form, e in form_errors(obs3, obs3["fp64"]).items():
            res3[form]["vs_fp64"] = e
    obs3.clear()
    torch.cuda.empty_cache()
    _log("bench: bandwidth ceilings")
    ceil = ceilings(N3, 19)
    hr = res3[head]
    ach = hr["step_kernel_GBs"]
    roof = {"kernel": f"k_step<19,{head}> (fused PSC collide-stream, 3D workload)",
            "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": _traffic(f"k_step_d3q19_{head}_c3"),
            "algorithmic_bytes_per_launch": hr["bytes_per_launch"],
            "frac_of_attainable": ach / ceil["attainable_GBs"]}

    # ---- the 3D packing: walled box, JKR contacts, its own FP16 form ----
    pack = None
    if not args.no_3d:
        _log("bench: generating the 3D packing workload")
        w5 = W.c5()
        N5 = w5.lattice.ncells
        pack, obs5 = {}, {}
        pforms = ["fp16"] if args.headline_only else ["fp16"] + [f for f in forms if f != "fp16"]
        for form in pforms:
            _log(f"bench: 3D packing coupled step, form {form}")
            ms, kms, ob, det = run_form(w5, form, steps, args.warmup, observe=True, reps=reps)
            obs5[form] = ob
            b = 2 * 19 * STORE_BYTES[form] * N5
            pack[form] = {"mlups": N5 / (ms * 1e-3) / 1e6, "ms_per_step": ms,
                          "step_kernel_ms": kms, "step_kernel_GBs": b / (kms * 1e-3) / 1e9,
                          "frac_of_hbm_peak": b / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "bytes_per_launch": b, **det}
        if "fp64" in obs5:
            for form, e in form_errors(obs5, obs5["fp64"]).items():
                pack[form]["vs_fp64"] = e
        obs5.clear()
        torch.cuda.empty_cache()

    if args.headline_only:
        print(json.dumps({"metric": METRIC, "value": hr["mlups"], "unit": "MLUPS", "n_gpus": 1,
                          "steps": steps, "repetitions": reps, "ms_per_step": hr["ms_per_step"],
                          "roofline": roof, "ceiling": ceil, "forms_3d": res3,
                          "packing_3d": pack}), flush=True)
        return

    # ---- the 2D workload (cache-resident) ----
    _log("bench: generating the 2D workload")
    w2 = W.c2()
    N2 = w2.lattice.ncells
    res2, obs2 = {}, {}
    for form in forms:
        _log(f"bench: 2D coupled step, form {form}")
        ms, kms, ob, det = run_form(w2, form, steps, args.warmup, observe=True, reps=reps)
        obs2[form] = ob
        b = 2 * 9 * STORE_BYTES[form] * N2
        res2[form] = {"mlups": N2 / (ms * 1e-3) / 1e6, "ms_per_step": ms,
                      "step_kernel_ms": kms, "step_kernel_GBs": b / (kms * 1e-3) / 1e9,
                      **det}
    if "fp64" in obs2:
        for form, e in form_errors(obs2, obs2["fp64"]).items():
            res2[form]["vs_fp64"] = e
    obs2.clear()
    torch.cuda.empty_cache()
    fric2d = None
    if args.friction_steps > 0 and head in res2:
        import dataclasses
        _log(f"bench: 2D coupled step with friction, form {head}")
        w2f = dataclasses.replace(w2, dem=dataclasses.replace(w2.dem, **FRICTION))
        ms, kms, _, _ = run_form(w2f, head, steps, args.warmup, reps=reps)
        fric2d = {"workload": "the 2D workload with sliding, twisting and rolling "
                              "friction (contacts gathered by the DEM kernel)",
                  "form": head, "ms_per_step": ms, "mlups": N2 / (ms * 1e-3) / 1e6,
                  "frictionless_ms_per_step": res2[head]["ms_per_step"],
                  "params": dict(FRICTION)}

    out = {
        "metric": METRIC,
        "value": hr["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "repetitions": reps,
        "steps_requested": args.steps,
        "ms_per_step": hr["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[head],
        "data": "synthetic (seeded RSA particle placement, seeded velocities)",
        "config": {"workload": "D3Q19 tau=0.6 256^3 periodic, 8000 spheres r~U(4,6) seed 3, "
                               "prescribed velocities N(0,1e-3^2); step: rasterize + PSC "
                               "collide-stream + Eq. 14 forces + FP64 mass partials + "
                               "advection",
                   "cells": N3, "particles": w3.particles.n, "precision_form": head},
        "roofline": roof,
        "ceiling": ceil,
        "frac_fp64": res3.get("fp64", {}).get("frac_of_hbm_peak"),
        "frac_fp16": res3.get("fp16", {}).get("frac_of_hbm_peak"),
        "frac_packing_fp16": (pack or {}).get("fp16", {}).get("frac_of_hbm_peak"),
        "forms_3d": res3,
        "packing_3d": ({"workload": "D3Q19 tau=0.65 384x192x192, walls at x=-1/2 and 383.5, "
                                    "20000 JKR spheres r~U(3,5) seed 5 from rest, gravity 1e-6 "
                                    "along -x; coupled step with DEM contacts", **pack}
                       if pack else None),
        "cache_resident": {"workload": "D2Q9 tau=0.7 1024^2 periodic, 2000 disks r~U(6,12) "
                                       "seed 2, JKR DEM; its distributions (38-75 MB) fit in "
                                       "the 256 MB last-level cache", **res2},
    }
    if fric2d is not None:
        out["friction"] = {"disks_2d": fric2d}
    if args.adjoint_steps > 0:
        _log("bench: adjoint of the 2D channel run")
        w4 = W.c4()
        _log("bench: gradient of a 2D coupled run with moving particles")
        adj_run = run_coupled_gradient(w2, 100)
        adj = {"channel_2d": run_adjoint(
            w4.lattice, w4.particles, args.adjoint_steps, 100,
            "D2Q9 tau=0.8 512x256 channel from rest, equilibrium inlet u=0.02, outlet rho=1, "
            "64 fixed disks r=8; J = x drag of disk 0 at the last step", [0])}
        if args.adjoint_3d_steps > 0 and not args.no_3d:
            _log(f"bench: settling the 3D packing for {args.settle_steps} coupled steps")
            f0, p5, settle = settle_packing(w5, args.settle_steps)
            adj["packing_3d_settle"] = settle
            if args.friction_steps > 0:
                _log("bench: the settled 3D packing without and with friction")
                out.setdefault("friction", {})["packing_3d"] = {
                    "workload": "the settled 3D packing (384x192x192, 20000 spheres, FP16 "
                                "storage) continued without and with sliding, twisting and "
                                "rolling friction",
                    **run_friction(w5, f0, p5, args.friction_steps)}
            lowest = np.argsort(p5.x[:, 0])[:100].tolist()
            win = args.adjoint_3d_steps
            label = (f"D3Q19 tau=0.65 384x192x192, walls on x, 20000 spheres r~U(3,5) after "
                     f"{args.settle_steps} coupled steps from rest (FP16 storage, JKR DEM, "
                     "gravity 1e-6 along -x), held fixed over the window; J = x drag (along "
                     f"gravity) of the 100 lowest spheres summed over the {win} steps")
            for prec in ("fp64", "fp16"):
                _log(f"bench: adjoint of a 3D packing window, {prec} forward")
                adj[f"packing_3d_{prec}"] = run_adjoint(
                    w5.lattice, p5, win, 50, label, lowest, precision=prec, f0=f0, window=win)
            del f0
        adj["coupled_run_2d"] = {
            "workload": "the 2D workload (1024x1024, 2000 JKR disks), 100 coupled "
                        "steps with moving particles, FP64, J = mean final x",
            **adj_run}
        adj["ratio"] = adj["channel_2d"]["ratio"]
        out["adjoint"] = adj
    dps = [int(v) for v in args.ergun_dps.split(",") if v.strip()]
    if dps:
        out["ergun"] = {
            "workload": "Sec. 3.4 packed bed: 8 fixed spheres of diameter d_p in simple-cubic "
                        "contact, periodic 2d_p cube, D3Q19 tau=0.65, body force from Eq. 35 "
                        "at the target Re_p*, FP64, run to steady state",
            "runs": run_ergun(dps, (1.0, 10.0), ("modified", "original"))}
    if args.packing_steps > 0:
        out["packing"] = {
            "workload": "Sec. 3.5 random packing: 500 spheres d=6 settling in a 100x50x50 box "
                        "(walls on x, periodic y and z), D3Q19 tau=2, gravity 8e-4 along -x, "
                        "JKR (gamma=0.128) or Hertz, sliding/twisting/rolling friction, FP32",
            **run_packing(args.packing_steps)}
    if not args.no_drag:
        out["drag"] = {
            "workload": "Sec. 3.2 fixed sphere at the centre of a 20d x 10d x 10d box, D3Q19, "
                        "equilibrium inlet u0 on x, constant-pressure outlets on the other "
                        "five faces, tau from Re_p = u0 d_p / nu, FP32 form, run to steady drag",
            "runs": run_drag([(10, 10.0, 0.05), (10, 50.0, 0.05), (10, 100.0, 0.05),
                              (20, 10.0, 0.05), (20, 100.0, 0.05),
                              (10, 10.0, 0.02), (10, 1.0, 0.05)])}
    if not args.no_cpu:
        _log("bench: CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
