"""torch.autograd.Function over a PSC-LBM run, backed by the hand-written
adjoint of the C ABI (lbm_step_adjoint) with checkpoint-and-recompute.

``psc_drag(x, u, omega, face_velocity, spec, radius, steps, ...)`` runs
``steps`` lattice steps from the equilibrium at rest (or a given state) with
the particles held at (x, u, omega), and returns the hydrodynamic force and
torque of Eq. 14 summed over the last ``window`` steps, each (n, 3).  Its
backward gives dJ/dx, dJ/du, dJ/domega and dJ/d(face velocity) (inlet and
moving-wall faces): the path-wise sensitivities of a run in which the
particle state is a fixed parameter.

Memory: one canonical FP64 state per ``checkpoint_every`` steps is kept from
the forward; the backward recomputes each segment (lbm_recompute, FP64, each
step reading one ring slot and writing the next) into a ring of
``checkpoint_every - 1`` states, then walks it backwards.  Every step and
every adjoint step runs in the HIP kernels; torch holds the buffers.  The
forward may run in any precision form; its checkpoints are the canonical FP64
images of its state, and the recompute and adjoint are FP64.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import torch

from . import psclbm as P


def _spec_with_faces(spec, face_velocity: torch.Tensor):
    fu = tuple(tuple(float(v) for v in row) for row in face_velocity.detach().cpu().tolist())
    return dataclasses.replace(spec, face_u=fu)


class PscDrag(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, u, omega, face_velocity, spec, radius, steps: int, checkpoint_every: int,
                window: int, precision: str, f0: Optional[torch.Tensor], max_tile_particles: int):
        dev = x.device
        n = radius.numel()
        sp = _spec_with_faces(spec, face_velocity)
        G = P.Lattice(sp, precision, max_particles=max(n, 1),
                      max_radius=float(radius.max()) if n else 1.0,
                      max_tile_particles=max_tile_particles)
        if f0 is not None:
            G.set_f(f0.detach().to(dev, torch.float64).contiguous())
        xs, us, ws, rs = (t.detach().to(dev, torch.float64).contiguous() for t in (x, u, omega, radius))
        P.psc_rasterize(G.ctx, xs, us, ws, rs)
        k = max(1, min(checkpoint_every, steps))
        checkpoints = []
        Fsum = torch.zeros((n, 3), dtype=torch.float64, device=dev)
        Tsum = torch.zeros_like(Fsum)
        Ft, Tt = torch.zeros_like(Fsum), torch.zeros_like(Fsum)
        for t in range(steps):
            if t % k == 0:
                checkpoints.append(G.get_f())
            G.step(1)
            if t >= steps - window and n > 0:
                P.particle_forces(G.ctx, Ft, Tt)
                Fsum += Ft
                Tsum += Tt
        G.sync()
        ctx.G = G
        ctx.checkpoints = checkpoints
        ctx.meta = (steps, k, window, n)
        ctx.particles = (xs, us, ws, rs)
        return Fsum, Tsum

    @staticmethod
    def backward(ctx, gF, gT):
        G = ctx.G
        steps, k, window, n = ctx.meta
        dev = gF.device
        q, N = G.q, G.N
        gF = gF.to(torch.float64).contiguous()
        gT = gT.to(torch.float64).contiguous()
        gX = torch.zeros((n, 3), dtype=torch.float64, device=dev)
        gU, gW = torch.zeros_like(gX), torch.zeros_like(gX)
        gface = torch.zeros((6, 3), dtype=torch.float64, device=dev)
        lam = torch.zeros((q, N), dtype=torch.float64, device=dev)
        lam2 = torch.empty_like(lam)
        nseg = len(ctx.checkpoints)
        ring = torch.empty((max(k - 1, 1), q, N), dtype=torch.float64, device=dev)
        for j in reversed(range(nseg)):
            t0 = j * k
            t1 = min(steps, t0 + k)
            ck = ctx.checkpoints[j].reshape(q, N)
            # recompute the segment's states straight into the ring
            if t1 - t0 > 1:
                P.lbm_recompute(G.ctx, ck, t1 - t0 - 1, ring)
            for t in reversed(range(t0, t1)):
                seeded = t >= steps - window
                state = ck if t == t0 else ring[t - t0 - 1]
                P.lbm_step_adjoint(G.ctx, state, lam, lam2,
                                   gF if seeded else None, gT if seeded else None,
                                   gX, gU, gW, gface)
                lam, lam2 = lam2, lam
        G.sync()
        ctx.G = None
        ctx.checkpoints = None
        return gX, gU, gW, gface, None, None, None, None, None, None, None, None


def psc_drag(x, u, omega, face_velocity, spec, radius, steps: int, checkpoint_every: int = 100,
             window: int = 1, precision: str = "fp64", f0: Optional[torch.Tensor] = None,
             max_tile_particles: int = 64):
    """Force and torque (Eq. 14) per particle summed over the last `window` of
    `steps` steps, differentiable in x, u, omega and the face velocities."""
    return PscDrag.apply(x, u, omega, face_velocity, spec, radius, steps, checkpoint_every,
                         window, precision, f0, max_tile_particles)


def coupled_step_vjp(G, dem_params, f_t: torch.Tensor, before, lam_f: torch.Tensor,
                     g_x: torch.Tensor, g_u: torch.Tensor, g_omega: torch.Tensor):
    """Vector-Jacobian product of the coupled step just taken on the lattice
    ``G`` (rasterise, lbm_step, dem_step driven by that step's force and
    torque; coupled_step(1) or the three calls, frictionless with n_sub = 1)
    from the canonical FP64 state ``f_t`` and the particle state ``before``
    (a DeviceParticles copy kept from before the step).  Given
    dJ/d(f', x', u', omega') of the step's result, returns
    dJ/d(f, x, u, omega) of its input, with the moving particles: the DEM
    step's adjoint (contacts held) gives the sensitivities of the force and
    torque, which seed lbm_step_adjoint, whose particle sensitivities
    (through the solid fractions, the rigid-body velocities and the torque
    arms) add to the DEM's."""
    ax, au, aw, aF, aT = G.dem_step_adjoint(dem_params, before, g_x, g_u, g_omega)
    lam_t = torch.empty_like(lam_f)
    P.lbm_step_adjoint(G.ctx, f_t.contiguous(), lam_f.contiguous(), lam_t, aF, aT, ax, au, aw,
                       None)
    return lam_t, ax, au, aw


class CoupledRun(torch.autograd.Function):
    """``steps`` coupled steps with moving particles (rasterise, lbm_step,
    frictionless dem_step with n_sub = 1, in FP64) from the fluid state
    ``f0`` (canonical FP64) and the particle state (x, u, omega); returns the
    final particle state and fluid state.  The forward keeps, every
    ``checkpoint_every`` steps, the FP64 state, the particle state and the
    contact lists in force before that step (dem_get_contacts).  The
    backward replays each segment from its checkpoint (dem_set_contacts puts
    its lists back), keeping the state, particles and formed contact lists
    of every step of the segment, and walks them in reverse with
    coupled_step_vjp.  Memory: steps / checkpoint_every + checkpoint_every
    canonical FP64 states."""

    @staticmethod
    def forward(ctx, x, u, omega, f0, spec, radius, dem_spec, steps: int,
                checkpoint_every: int = 32):
        if (dem_spec.mu_f or dem_spec.theta_r or dem_spec.n_sub != 1 or dem_spec.kinematic
                or steps < 1):
            raise ValueError("coupled_run differentiates frictionless DEM steps with n_sub = 1 "
                             "and at least one step")
        n = x.shape[0]
        G = P.Lattice(spec, "fp64", max_particles=n, max_radius=float(radius.max()),
                      max_tile_particles=64, max_contacts=dem_spec.max_contacts)
        G.set_f(f0.detach().contiguous())
        dp = P.DeviceParticles(x.detach().clone(), u.detach().clone(), omega.detach().clone(),
                               radius)
        prm = P.make_dem_params(dem_spec)
        k = max(1, int(checkpoint_every))
        segs = []
        for t in range(steps):
            if t % k == 0:
                segs.append((t, G.get_f(), _copy(dp)) + G.get_contacts())
            G.coupled_step(prm, dp, 1)
        f_end = G.get_f()
        G.sync()
        ctx.G, ctx.prm, ctx.segs, ctx.steps, ctx.k = G, prm, segs, steps, k
        return dp.x.clone(), dp.u.clone(), dp.omega.clone(), f_end

    @staticmethod
    def backward(ctx, gx, gu, gw, gf):
        G, prm = ctx.G, ctx.prm
        _, f_first, p_first, _, _ = ctx.segs[0]
        z = lambda t, like: (t if t is not None else torch.zeros_like(like)).contiguous()
        lam_x, lam_u, lam_w = z(gx, p_first.x), z(gu, p_first.u), z(gw, p_first.omega)
        lam_f = z(gf, f_first)
        for t0, f_c, p_c, cnt_c, ids_c in reversed(ctx.segs):
            # replay the segment, keeping what each of its steps needs
            G.set_f(f_c)
            dq = _copy(p_c)
            G.set_contacts(cnt_c, ids_c)
            ring = []
            for _ in range(t0, min(ctx.steps, t0 + ctx.k)):
                f_t = G.get_f()
                before = _copy(dq)
                G.coupled_step(prm, dq, 1)
                ring.append((f_t, before) + G.get_contacts())
            for f_t, before, cnt, ids in reversed(ring):
                G.set_contacts(cnt, ids)
                G.rasterize(before)
                lam_f, lam_x, lam_u, lam_w = coupled_step_vjp(G, prm, f_t, before, lam_f,
                                                              lam_x, lam_u, lam_w)
        G.sync()
        ctx.G = ctx.segs = None
        return lam_x, lam_u, lam_w, lam_f, None, None, None, None, None


def _copy(p):
    return P.DeviceParticles(p.x.clone(), p.u.clone(), p.omega.clone(), p.r)


def coupled_run(x, u, omega, f0, spec, radius, dem_spec, steps: int, checkpoint_every: int = 32):
    """Final (x, u, omega, f) after `steps` coupled steps with moving
    particles, differentiable in x, u, omega and f0."""
    return CoupledRun.apply(x, u, omega, f0, spec, radius, dem_spec, steps, checkpoint_every)
