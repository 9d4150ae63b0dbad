"""ctypes binding of ``libpsclbm.so`` (the gfx950 C ABI declared in include/psclbm.h).

Argument marshalling only: every step of the PSC-LBM path runs in the HIP
kernels of the library.  PyTorch provides device memory and the stream.  The
functions keep the C names (``lbm_init``, ``psc_rasterize``, ``lbm_step``,
``particle_forces``, ``dem_step`` ...); ``Lattice`` bundles a context with its
workspace tensor for convenience.

There is no fallback: if the library is missing or cannot be loaded the
import of the binding raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsclbm.so")

OK, EINVAL, ENOMEM, EHIP, ESLOTS, ECONTACTS, ENONFINITE, ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
PERIODIC, BOUNCE_BACK, MOVING_WALL, INLET_EQ, OUTLET_EQ = 0, 1, 2, 3, 4
FP64, FP32, FP32_FP16STORE = 0, 1, 2
_FACE = {"periodic": PERIODIC, "bounce_back": BOUNCE_BACK, "moving_wall": MOVING_WALL,
         "inlet_eq": INLET_EQ, "outlet_eq": OUTLET_EQ}
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16": FP32_FP16STORE}


class PsclbmError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


class Config(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("nz", ctypes.c_int), ("tau", ctypes.c_double),
                ("body_force", ctypes.c_double * 3), ("face_bc", ctypes.c_int * 6),
                ("face_velocity", (ctypes.c_double * 3) * 6), ("rho0", ctypes.c_double),
                ("shell_h", ctypes.c_double), ("precision", ctypes.c_int),
                ("max_particles", ctypes.c_int), ("max_radius", ctypes.c_double),
                ("max_tile_particles", ctypes.c_int), ("max_contacts", ctypes.c_int),
                ("weighting", ctypes.c_int)]


class ParticlesC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("x", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("omega", ctypes.c_void_p), ("radius", ctypes.c_void_p)]


class DemParams(ctypes.Structure):
    _fields_ = [("rho_p", ctypes.c_double), ("rho_f", ctypes.c_double),
                ("E_p", ctypes.c_double), ("poisson", ctypes.c_double),
                ("gamma", ctypes.c_double), ("eta_n", ctypes.c_double),
                ("g", ctypes.c_double * 3), ("dt", ctypes.c_double),
                ("n_sub", ctypes.c_int), ("kinematic", ctypes.c_int),
                ("k_t", ctypes.c_double), ("eta_t", ctypes.c_double),
                ("mu_f", ctypes.c_double), ("theta_r", ctypes.c_double)]


# Every symbol the header declares, with its ctypes signature.
_VP, _I, _D, _SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
SIGNATURES = {
    "psclbm_workspace_bytes": (_SZ, [ctypes.POINTER(Config)]),
    "lbm_init": (_I, [ctypes.POINTER(Config), _VP, _SZ, _VP, ctypes.POINTER(_VP)]),
    "lbm_free": (None, [_VP]),
    "psclbm_set_stream": (_I, [_VP, _VP]),
    "lbm_set_f": (_I, [_VP, _VP]),
    "lbm_get_f": (_I, [_VP, _VP]),
    "lbm_set_equilibrium": (_I, [_VP, _VP, _VP]),
    "lbm_get_macros": (_I, [_VP, _VP, _VP]),
    "psc_rasterize": (_I, [_VP, ctypes.POINTER(ParticlesC)]),
    "psc_get_solid_fraction": (_I, [_VP, _VP, _VP, _VP, _I]),
    "lbm_step": (_I, [_VP, _I]),
    "particle_forces": (_I, [_VP, _VP, _VP]),
    "dem_step": (_I, [_VP, ctypes.POINTER(DemParams), _VP, _VP, _VP, _VP, _I, _VP, _VP]),
    "dem_reset_contacts": (_I, [_VP]),
    "dem_get_contacts": (_I, [_VP, _VP, _VP]),
    "dem_set_contacts": (_I, [_VP, _VP, _VP]),
    "dem_step_adjoint": (_I, [_VP, ctypes.POINTER(DemParams), _VP, _VP, _VP, _VP, _I, _VP, _VP,
                              _VP, _VP, _VP, _VP, _VP, _VP]),
    "lbm_mass": (_I, [_VP, ctypes.POINTER(_D)]),
    "psclbm_sync": (_I, [_VP]),
    "psclbm_strerror": (ctypes.c_char_p, [_I]),
    "lbm_step_count": (ctypes.c_longlong, [_VP]),
    "lbm_step_adjoint": (_I, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "coupled_step": (_I, [_VP, ctypes.POINTER(DemParams), _VP, _VP, _VP, _VP, _I, _I]),
    "lbm_recompute": (_I, [_VP, _VP, _I, _VP]),
    "psc_rasterize_adjoint": (_I, [_VP, _VP, _I, _VP]),
    "psc_solid_fraction_noalloc": (_I, [ctypes.POINTER(Config), ctypes.POINTER(ParticlesC), _VP,
                                        _VP, _VP, _I, _VP]),
    # bandwidth ceilings (include/psclbm_probe.h)
    "psclbm_stream_copy": (_I, [_VP, _VP, _SZ, _VP]),
    "psclbm_stream_swap": (_I, [_VP, ctypes.c_longlong, _I, _VP]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (torch is imported first so the library binds to
    torch's HIP runtime).  Raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built; run __graft_entry__.build() "
                              "or python -m paper_1901_09745_amd.build")
        L = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return load().psclbm_strerror(code).decode()


def _check(rc: int, where: str) -> None:
    if rc != OK:
        raise PsclbmError(rc, where)


def _ptr(t: Optional[torch.Tensor], dtype=torch.float64) -> Optional[int]:
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"expected a contiguous CUDA {dtype} tensor")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


# ---------------------------------------------------------------------------
# The C functions under their own names
# ---------------------------------------------------------------------------

def psclbm_stream_copy(src: torch.Tensor, dst: torch.Tensor) -> None:
    """Copy src to dst (same byte size, a multiple of 16) with the library's
    streaming copy kernel, on torch's current stream."""
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("expected contiguous CUDA tensors")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("size mismatch")
    _check(load().psclbm_stream_copy(src.data_ptr(), dst.data_ptr(), nbytes, _stream()),
           "psclbm_stream_copy")


def psclbm_stream_swap(a: torch.Tensor, q: int) -> None:
    """The data movement of an even lattice step over the q FP32 arrays of a
    (shape [q, n]), on torch's current stream."""
    if not (a.is_cuda and a.dtype == torch.float32 and a.is_contiguous() and a.dim() == 2
            and a.shape[0] == q):
        raise ValueError("expected a contiguous CUDA float32 tensor of shape [q, n]")
    _check(load().psclbm_stream_swap(a.data_ptr(), a.shape[1], q, _stream()),
           "psclbm_stream_swap")


def psclbm_workspace_bytes(cfg: Config) -> int:
    return int(load().psclbm_workspace_bytes(ctypes.byref(cfg)))


def lbm_init(cfg: Config, workspace: torch.Tensor, stream: Optional[int] = None) -> int:
    ctx = ctypes.c_void_p()
    _check(load().lbm_init(ctypes.byref(cfg), workspace.data_ptr(), workspace.numel(),
                           _stream() if stream is None else stream, ctypes.byref(ctx)),
           "lbm_init")
    return ctx.value


def lbm_free(ctx: int) -> None:
    load().lbm_free(ctx)


def lbm_set_f(ctx: int, f: torch.Tensor) -> None:
    _check(load().lbm_set_f(ctx, _ptr(f)), "lbm_set_f")


def lbm_get_f(ctx: int, f: torch.Tensor) -> None:
    _check(load().lbm_get_f(ctx, _ptr(f)), "lbm_get_f")


def lbm_set_equilibrium(ctx: int, rho: Optional[torch.Tensor], u: Optional[torch.Tensor]) -> None:
    _check(load().lbm_set_equilibrium(ctx, _ptr(rho), _ptr(u)), "lbm_set_equilibrium")


def lbm_get_macros(ctx: int, rho: Optional[torch.Tensor], u: Optional[torch.Tensor]) -> None:
    _check(load().lbm_get_macros(ctx, _ptr(rho), _ptr(u)), "lbm_get_macros")


def psc_rasterize(ctx: int, x: torch.Tensor, u: torch.Tensor, omega: torch.Tensor,
                  radius: torch.Tensor) -> None:
    n = radius.numel()
    p = ParticlesC(n, _ptr(x), _ptr(u), _ptr(omega), _ptr(radius))
    _check(load().psc_rasterize(ctx, ctypes.byref(p)), "psc_rasterize")


def psc_get_solid_fraction(ctx: int, eps_total: Optional[torch.Tensor],
                           slot_id: Optional[torch.Tensor], slot_eps: Optional[torch.Tensor],
                           kslots: int) -> None:
    _check(load().psc_get_solid_fraction(ctx, _ptr(eps_total), _ptr(slot_id, torch.int32),
                                         _ptr(slot_eps), kslots), "psc_get_solid_fraction")


def psc_solid_fraction_noalloc(cfg: Config, x: torch.Tensor, u: torch.Tensor,
                               omega: torch.Tensor, radius: torch.Tensor,
                               eps_total: torch.Tensor, slot_id: Optional[torch.Tensor],
                               slot_eps: Optional[torch.Tensor], kslots: int) -> int:
    """The context-free solid fractions (no allocation); returns the C code
    (the caller decides how to treat errors)."""
    n = radius.numel()
    p = ParticlesC(n, _ptr(x), _ptr(u), _ptr(omega), _ptr(radius))
    return int(load().psc_solid_fraction_noalloc(
        ctypes.byref(cfg), ctypes.byref(p), _ptr(eps_total), _ptr(slot_id, torch.int32),
        _ptr(slot_eps), kslots, _stream()))


def lbm_step(ctx: int, nsteps: int = 1) -> None:
    _check(load().lbm_step(ctx, nsteps), "lbm_step")


def particle_forces(ctx: int, force: Optional[torch.Tensor], torque: Optional[torch.Tensor]) -> None:
    _check(load().particle_forces(ctx, _ptr(force), _ptr(torque)), "particle_forces")


def dem_step(ctx: int, prm: DemParams, x: torch.Tensor, u: torch.Tensor, omega: torch.Tensor,
             radius: torch.Tensor, force: Optional[torch.Tensor],
             torque: Optional[torch.Tensor]) -> None:
    _check(load().dem_step(ctx, ctypes.byref(prm), _ptr(x), _ptr(u), _ptr(omega), _ptr(radius),
                           radius.numel(), _ptr(force), _ptr(torque)), "dem_step")


def dem_step_adjoint(ctx: int, prm: DemParams, x: torch.Tensor, u: torch.Tensor,
                     omega: torch.Tensor, radius: torch.Tensor, gx: torch.Tensor,
                     gu: torch.Tensor, gw: torch.Tensor, ax: torch.Tensor, au: torch.Tensor,
                     aw: torch.Tensor, aF: torch.Tensor, aT: torch.Tensor) -> None:
    _check(load().dem_step_adjoint(ctx, ctypes.byref(prm), _ptr(x), _ptr(u), _ptr(omega),
                                   _ptr(radius), radius.numel(), _ptr(gx), _ptr(gu), _ptr(gw),
                                   _ptr(ax), _ptr(au), _ptr(aw), _ptr(aF), _ptr(aT)),
           "dem_step_adjoint")


def coupled_step(ctx: int, prm: DemParams, x: torch.Tensor, u: torch.Tensor, omega: torch.Tensor,
                 radius: torch.Tensor, nsteps: int = 1) -> None:
    _check(load().coupled_step(ctx, ctypes.byref(prm), _ptr(x), _ptr(u), _ptr(omega),
                               _ptr(radius), int(radius.numel()), nsteps), "coupled_step")


def dem_reset_contacts(ctx: int) -> None:
    _check(load().dem_reset_contacts(ctx), "dem_reset_contacts")


def lbm_mass(ctx: int) -> float:
    m = ctypes.c_double()
    _check(load().lbm_mass(ctx, ctypes.byref(m)), "lbm_mass")
    return m.value


def psclbm_sync(ctx: int) -> None:
    _check(load().psclbm_sync(ctx), "psclbm_sync")


def lbm_step_count(ctx: int) -> int:
    return int(load().lbm_step_count(ctx))


def lbm_step_adjoint(ctx: int, f: torch.Tensor, lam_in: torch.Tensor, lam_out: torch.Tensor,
                     dJ_dF: Optional[torch.Tensor] = None, dJ_dT: Optional[torch.Tensor] = None,
                     g_x: Optional[torch.Tensor] = None, g_u: Optional[torch.Tensor] = None,
                     g_omega: Optional[torch.Tensor] = None,
                     g_face: Optional[torch.Tensor] = None) -> None:
    _check(load().lbm_step_adjoint(ctx, _ptr(f), _ptr(lam_in), _ptr(lam_out), _ptr(dJ_dF),
                                   _ptr(dJ_dT), _ptr(g_x), _ptr(g_u), _ptr(g_omega),
                                   _ptr(g_face)), "lbm_step_adjoint")


def lbm_recompute(ctx: int, f0: torch.Tensor, nsteps: int, ring: torch.Tensor) -> None:
    _check(load().lbm_recompute(ctx, _ptr(f0), nsteps, _ptr(ring)), "lbm_recompute")


def psc_rasterize_adjoint(ctx: int, g_slot_eps: torch.Tensor, kslots: int,
                          g_x: torch.Tensor) -> None:
    _check(load().psc_rasterize_adjoint(ctx, _ptr(g_slot_eps), kslots, _ptr(g_x)),
           "psc_rasterize_adjoint")


# ---------------------------------------------------------------------------
# Marshalling helpers
# ---------------------------------------------------------------------------

WEIGHTINGS = {"modified": 0, "original": 1}


def make_config(spec, precision: str = "fp64", max_particles: int = 0, max_radius: float = 0.0,
                max_tile_particles: int = 128, max_contacts: int = 16,
                weighting: str = "modified") -> Config:
    """Config from a ``workloads.LatticeSpec``."""
    c = Config()
    c.lattice, c.nx, c.ny, c.nz = spec.q, spec.nx, spec.ny, spec.nz
    c.tau = spec.tau
    for a in range(3):
        c.body_force[a] = spec.force[a]
    for f in range(6):
        c.face_bc[f] = _FACE[spec.faces[f]]
        for a in range(3):
            c.face_velocity[f][a] = spec.face_u[f][a]
    c.rho0 = spec.rho0
    c.shell_h = spec.h
    c.precision = PRECISIONS[precision]
    c.max_particles = max_particles
    c.max_radius = max_radius
    c.max_tile_particles = max_tile_particles
    c.max_contacts = max_contacts
    c.weighting = WEIGHTINGS[weighting]
    return c


def make_dem_params(d) -> DemParams:
    """DemParams from a ``workloads.DemSpec``."""
    p = DemParams()
    p.rho_p, p.rho_f, p.E_p, p.poisson = d.rho_p, d.rho_f, d.E_p, d.poisson
    p.gamma, p.eta_n = d.gamma, d.eta_n
    for a in range(3):
        p.g[a] = d.g[a]
    p.dt, p.n_sub, p.kinematic = d.dt, d.n_sub, int(d.kinematic)
    p.k_t, p.eta_t, p.mu_f, p.theta_r = d.k_t, d.eta_t, d.mu_f, d.theta_r
    return p


class DeviceParticles:
    """FP64 particle SoA on the device: x, u, omega (n, 3), r (n,)."""

    def __init__(self, x, u, omega, r, device="cuda"):
        def t(a):
            if not isinstance(a, torch.Tensor):
                import numpy as np
                a = np.ascontiguousarray(a, dtype=np.float64)
            return torch.as_tensor(a, dtype=torch.float64).to(device).contiguous()
        self.x, self.u, self.omega, self.r = t(x).reshape(-1, 3), t(u).reshape(-1, 3), \
            t(omega).reshape(-1, 3), t(r).reshape(-1)

    @staticmethod
    def from_host(p, device="cuda") -> "DeviceParticles":
        return DeviceParticles(p.x, p.u, p.omega, p.r, device)

    @property
    def n(self) -> int:
        return self.r.numel()


class Lattice:
    """A context plus its caller-owned workspace tensor."""

    def __init__(self, spec, precision: str = "fp64", max_particles: int = 0,
                 max_radius: float = 0.0, max_tile_particles: int = 128, max_contacts: int = 16,
                 device: str = "cuda", weighting: str = "modified"):
        # held for __del__, which may run after the module's globals are gone
        self._lib = load()
        self.spec = spec
        self.cfg = make_config(spec, precision, max_particles, max_radius, max_tile_particles,
                               max_contacts, weighting)
        nbytes = psclbm_workspace_bytes(self.cfg)
        if nbytes == 0:
            raise PsclbmError(EINVAL, "psclbm_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.ctx = lbm_init(self.cfg, self.workspace)
        self.q = spec.q
        self.N = spec.ncells
        self.n_particles = 0

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        lib = getattr(self, "_lib", None)
        if ctx and lib is not None:
            lib.lbm_free(ctx)
            self.ctx = None

    # state I/O -------------------------------------------------------------
    def set_f(self, f: torch.Tensor) -> None:
        lbm_set_f(self.ctx, f.to(torch.float64).contiguous())

    def get_f(self) -> torch.Tensor:
        out = torch.empty((self.q,) + self.spec.shape, dtype=torch.float64, device="cuda")
        lbm_get_f(self.ctx, out)
        return out

    def set_equilibrium(self, rho=None, u=None) -> None:
        lbm_set_equilibrium(self.ctx, None if rho is None else rho.contiguous(),
                            None if u is None else u.contiguous())

    def macros(self) -> Tuple[torch.Tensor, torch.Tensor]:
        rho = torch.empty(self.spec.shape, dtype=torch.float64, device="cuda")
        u = torch.empty(self.spec.shape + (3,), dtype=torch.float64, device="cuda")
        lbm_get_macros(self.ctx, rho, u)
        return rho, u

    # particles -------------------------------------------------------------
    def rasterize(self, p: Optional[DeviceParticles]) -> None:
        if p is None or p.n == 0:
            z = torch.zeros(3, dtype=torch.float64, device="cuda")
            psc_rasterize(self.ctx, z, z, z, torch.zeros(0, dtype=torch.float64, device="cuda"))
            self.n_particles = 0
        else:
            psc_rasterize(self.ctx, p.x, p.u, p.omega, p.r)
            self.n_particles = p.n

    def solid_fraction(self, kslots: int = 4):
        eps = torch.empty(self.spec.shape, dtype=torch.float64, device="cuda")
        ids = torch.empty(self.spec.shape + (kslots,), dtype=torch.int32, device="cuda")
        seps = torch.empty(self.spec.shape + (kslots,), dtype=torch.float64, device="cuda")
        psc_get_solid_fraction(self.ctx, eps, ids, seps, kslots)
        return eps, ids, seps

    def step(self, nsteps: int = 1) -> None:
        lbm_step(self.ctx, nsteps)

    def forces(self) -> Tuple[torch.Tensor, torch.Tensor]:
        n = max(self.n_particles, 1)
        F = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
        T = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
        particle_forces(self.ctx, F, T)
        return F[: self.n_particles], T[: self.n_particles]

    def dem_step(self, dem_params: DemParams, p: DeviceParticles, F=None, T=None) -> None:
        dem_step(self.ctx, dem_params, p.x, p.u, p.omega, p.r, F, T)

    def get_contacts(self):
        """The current DEM contact lists: (counts (max_particles,), ids
        (max_particles, max_contacts)) int32 device tensors."""
        n, mc = max(self.cfg.max_particles, 1), self.cfg.max_contacts
        cnt = torch.empty(n, dtype=torch.int32, device="cuda")
        ids = torch.empty((n, mc), dtype=torch.int32, device="cuda")
        _check(load().dem_get_contacts(self.ctx, _ptr(cnt, torch.int32), _ptr(ids, torch.int32)),
               "dem_get_contacts")
        return cnt, ids

    def set_contacts(self, cnt: torch.Tensor, ids: torch.Tensor) -> None:
        _check(load().dem_set_contacts(self.ctx, _ptr(cnt, torch.int32), _ptr(ids, torch.int32)),
               "dem_set_contacts")

    def dem_step_adjoint(self, dem_params: DemParams, before: DeviceParticles, gx, gu, gw):
        """Adjoint of the DEM step just taken from the state ``before``: given
        dJ/d(x', u', omega'), returns dJ/d(x, u, omega, force, torque)."""
        outs = [torch.empty_like(gx) for _ in range(5)]
        dem_step_adjoint(self.ctx, dem_params, before.x, before.u, before.omega, before.r,
                         gx.contiguous(), gu.contiguous(), gw.contiguous(), *outs)
        return tuple(outs)

    def coupled_step(self, dem_params: DemParams, p: DeviceParticles, nsteps: int = 1) -> None:
        coupled_step(self.ctx, dem_params, p.x, p.u, p.omega, p.r, nsteps)
        self.n_particles = p.n

    def mass(self) -> float:
        return lbm_mass(self.ctx)

    def sync(self) -> None:
        psclbm_sync(self.ctx)
