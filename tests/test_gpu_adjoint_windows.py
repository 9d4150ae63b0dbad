"""Gradients of drag functionals through lattice runs, at the configurations
the benchmark differentiates.

* The 2D inlet channel (512 x 256, 64 disks r = 8, 4000 steps, checkpoint
  every 100, J = x drag of disk 0 at the last step): the gradient with an FP32
  forward against the one with an FP64 forward, on every component of
  dJ/dX and dJ/dU (64 x 2 each) and on dJ/d(inlet velocity).  Both are the
  FP64 adjoint; they differ by the FP32 trajectory's distance from the FP64
  one, which the FP32 form keeps within 1e-5 of the flow; the bound is 1e-4
  of the largest component.
* A window of the 3D packing at a quarter of its linear size (96 x 48 x 48,
  walls on x, 312 JKR spheres, after 100 coupled steps from rest), the
  particles held fixed over a 20-step window with a checkpoint every 5 steps,
  J = the x drag of the 10 lowest spheres summed over the window (the
  functional of the benchmark's 3D window): dJ/dX and dJ/dU against central
  differences of the C oracle over the same window (h = 1e-5; the difference
  error is O(h^2), about 1e-9 relative here, and the FP64 roundoff of J about
  1e-11 over h).
"""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def _drag_grad(lat, p, steps, every, precision, select, window=1, f0=None):
    from paper_1901_09745_amd.autograd import psc_drag
    dev = "cuda"
    x = torch.tensor(p.x, device=dev, requires_grad=True)
    u = torch.tensor(p.u, device=dev, requires_grad=True)
    om = torch.tensor(p.omega, device=dev, requires_grad=True)
    fu = torch.tensor(np.asarray(lat.face_u, dtype=np.float64), device=dev, requires_grad=True)
    F, _ = psc_drag(x, u, om, fu, lat, torch.tensor(p.r, device=dev), steps,
                    checkpoint_every=every, window=window, precision=precision, f0=f0)
    J = F[torch.as_tensor(select, device=dev), 0].sum()
    J.backward()
    return (float(J.detach()), x.grad.cpu().numpy(), u.grad.cpu().numpy(),
            fu.grad.cpu().numpy())


def test_channel_fp32_gradient_matches_fp64_on_every_component():
    w = W.c4()
    lat, p = w.lattice, w.particles
    print("case: c4 full size, fp32 against fp64 forward", flush=True)
    J64, gx64, gu64, gf64 = _drag_grad(lat, p, 4000, 100, "fp64", [0])
    J32, gx32, gu32, gf32 = _drag_grad(lat, p, 4000, 100, "fp32", [0])
    ex = np.abs(gx32[:, :2] - gx64[:, :2]).max() / np.abs(gx64[:, :2]).max()
    eu = np.abs(gu32[:, :2] - gu64[:, :2]).max() / np.abs(gu64[:, :2]).max()
    ef = abs(gf32[0, 0] - gf64[0, 0]) / abs(gf64[0, 0])
    print(f"J rel {abs(J32 - J64) / abs(J64):.3e}; dJ/dX {ex:.3e}, dJ/dU {eu:.3e}, "
          f"dJ/du_in {ef:.3e}")
    assert np.count_nonzero(gx64[:, :2]) > 64  # the drag of disk 0 reaches the other disks
    assert ex < 1e-4
    assert eu < 1e-4
    assert ef < 1e-4


def _settled_packing():
    import paper_1901_09745_amd.psclbm as P
    w = W.c5(scale=0.25)
    p = w.particles
    G = P.Lattice(w.lattice, "fp64", max_particles=p.n, max_radius=float(p.r.max()),
                  max_tile_particles=64, max_contacts=16)
    dp = P.DeviceParticles.from_host(p)
    G.coupled_step(P.make_dem_params(w.dem), dp, 100)
    f0 = G.get_f().clone()
    G.sync()
    ps = W.Particles(dp.x.cpu().numpy(), dp.u.cpu().numpy(), dp.omega.cpu().numpy(),
                     dp.r.cpu().numpy())
    return w.lattice, ps, f0


def _oracle_window_J(lat, f0, p, steps, select):
    L = oracle.Lattice(lat, f0)
    J = 0.0
    for _ in range(steps):
        F, _ = L.step(p)
        J += F[select, 0].sum()
    return J


def test_packing_window_gradient_vs_oracle_differences():
    lat, p, f0 = _settled_packing()
    steps, every, h = 20, 5, 1e-5
    sel = np.argsort(p.x[:, 0])[:10]
    print(f"case: packing window 96x48x48, {p.n} spheres, {steps} steps", flush=True)
    J, gx, gu, _ = _drag_grad(lat, p, steps, every, "fp64", sel.tolist(), window=steps, f0=f0)
    f0h = f0.cpu().numpy()
    J_ref = _oracle_window_J(lat, f0h, p, steps, sel)
    assert abs(J - J_ref) <= 1e-12 * abs(J_ref) * steps
    checks = [("x", sel[0], 0), ("x", sel[1], 1), ("x", sel[2], 2), ("u", sel[0], 0),
              ("u", sel[3], 1)]
    for kind, s, a in checks:
        pp, pm = p.copy(), p.copy()
        arr_p, arr_m = (pp.x, pm.x) if kind == "x" else (pp.u, pm.u)
        arr_p[s, a] += h
        arr_m[s, a] -= h
        fd = (_oracle_window_J(lat, f0h, pp, steps, sel) -
              _oracle_window_J(lat, f0h, pm, steps, sel)) / (2 * h)
        g = (gx if kind == "x" else gu)[s, a]
        err = abs(g - fd) / max(abs(fd), 1e-300)
        print(f"dJ/d{kind}[{s},{a}]: adjoint {g:.10e} differences {fd:.10e} rel {err:.2e}",
              flush=True)
        assert err < 1e-5
