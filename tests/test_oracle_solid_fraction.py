"""Pins of the oracle's linear solid-fraction approximation (Sec. 2.4,
Eqs. 15-20, Table 1) against quadrature, brute-force sub-sampling, closed
asymptotes and exact-area invariants."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads as W

RADII = [0.75, 1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 10.0, 50.0]


def _va2d_quad(r):
    return integrate.quad(lambda x: math.sqrt(r * r - x * x), -0.5, 0.5, epsabs=1e-14,
                          epsrel=1e-14)[0]


def _va3d_quad(r):
    return integrate.dblquad(lambda y, x: math.sqrt(r * r - x * x - y * y), -0.5, 0.5,
                             -0.5, 0.5, epsabs=1e-14, epsrel=1e-14)[0]


@pytest.mark.parametrize("r", RADII)
def test_va_closed_forms_match_quadrature(r):
    # Eq. 19 and Eq. 17 are closed forms of the integrals of the square-root
    # integrands over the unit segment / unit square.
    assert oracle.va2d(r) == pytest.approx(_va2d_quad(r), abs=2e-14)
    assert oracle.va3d(r) == pytest.approx(_va3d_quad(r), abs=2e-13)


@pytest.mark.parametrize("r", [20.0, 50.0, 200.0])
def test_va_asymptotes(r):
    # sqrt(r^2 - s) ~ r - s / (2r): V_a -> r - 1/(24 r) in 2D, r - 1/(12 r) in 3D
    assert oracle.va2d(r) == pytest.approx(r - 1.0 / (24 * r), abs=5.0 / r ** 3)
    assert oracle.va3d(r) == pytest.approx(r - 1.0 / (12 * r), abs=5.0 / r ** 3)


def _lat2(n=40):
    return W.LatticeSpec(q=9, nx=n, ny=n)


def _lat3(n=24):
    return W.LatticeSpec(q=19, nx=n, ny=n, nz=n)


def _exact_overlap_2d(cx, cy, r, x, y):
    """Exact area of the disk (cx, cy, r) inside the unit cell centred at (x, y)."""
    def chord(t):
        dx = t - cx
        if abs(dx) >= r:
            return 0.0
        s = math.sqrt(r * r - dx * dx)
        lo, hi = max(cy - s, y - 0.5), min(cy + s, y + 0.5)
        return max(0.0, hi - lo)
    pts = [p for p in (cx - r, cx + r) if x - 0.5 < p < x + 0.5]
    return integrate.quad(chord, x - 0.5, x + 0.5, points=pts or None, epsabs=1e-13,
                          limit=200)[0]


@pytest.mark.parametrize("r", [6.0, 8.0, 10.0])
def test_on_axis_cells_are_exact_2d(r):
    # Under assumptions (i)-(iii) of Sec. 2.4 (cell centre on an axis through
    # the particle centre, the arc crossing only the two side faces), the
    # linear formula is the exact overlap (Eq. 16): y_c in [r-1/2, sqrt(r^2-1/4)+1/2].
    top = math.sqrt(r * r - 0.25) + 0.5
    for yc in np.linspace(r - 0.5, top, 6):
        X = np.array([[20.0, 30.0 - yc, 0.0]])
        nslot, ids, eps, ssum = oracle.rasterize(_lat2(), X, np.array([r]))
        n = 20 + 40 * 30
        exact = _exact_overlap_2d(20.0, 30.0 - yc, r, 20.0, 30.0)
        got = eps[n, 0] if nslot[n] else 0.0
        assert got == pytest.approx(exact, abs=1e-12)


@pytest.mark.parametrize("r", [4.0, 6.0])
def test_on_axis_cells_are_exact_3d(r):
    top = math.sqrt(r * r - 0.5) + 0.5
    for yc in np.linspace(r - 0.5, top, 4):
        X = np.array([[12.0, 18.0 - yc, 12.0]])
        nslot, ids, eps, ssum = oracle.rasterize(_lat3(), X, np.array([r]))
        n = 12 + 24 * (18 + 24 * 12)
        exact = integrate.dblquad(
            lambda z, x: min(1.0, max(0.0, math.sqrt(max(r * r - x * x - z * z, 0.0)) - (yc - 0.5))),
            -0.5, 0.5, -0.5, 0.5, epsabs=1e-12)[0]
        got = eps[n, 0] if nslot[n] else 0.0
        assert got == pytest.approx(exact, abs=1e-10)


def _subsample_2d(cx, cy, r, x, y, m=1024):
    """Deterministic m x m midpoint sampling of the disk inside a unit cell
    (the sampling estimate of Sec. 2.4 with a regular grid)."""
    t = (np.arange(m) + 0.5) / m - 0.5
    px, py = np.meshgrid(x + t - cx, y + t - cy, indexing="ij")
    return float(np.count_nonzero(px * px + py * py < r * r)) / (m * m)


@pytest.mark.parametrize("r", [3.0, 6.0, 10.0])
def test_general_cells_within_linear_bound(r):
    # Not exact off-axis: per cell |eps_linear - eps_true| stays below 0.045
    # (largest near 45-degree corner cells); checked against both exact
    # quadrature and brute-force sub-sampling on a ring of boundary cells.
    rng = np.random.default_rng(int(r * 10))
    for _ in range(2):
        cx, cy = 20.0 + rng.uniform(-0.5, 0.5), 20.0 + rng.uniform(-0.5, 0.5)
        nslot, ids, eps, ssum = oracle.rasterize(_lat2(), np.array([[cx, cy, 0.0]]), np.array([r]))
        worst = 0.0
        checked = 0
        for n in range(40 * 40):
            x, y = n % 40, n // 40
            d = math.hypot(x - cx, y - cy)
            if abs(d - r) > 1.0:
                continue
            exact = _exact_overlap_2d(cx, cy, r, x, y)
            got = eps[n, 0] if nslot[n] else 0.0
            worst = max(worst, abs(got - exact))
            if checked < 6:
                assert _subsample_2d(cx, cy, r, x, y) == pytest.approx(exact, abs=5e-5)
            checked += 1
        assert checked > 10
        assert worst < 0.045


@pytest.mark.parametrize("r,bound", [(3.0, 3e-3), (6.0, 3e-3), (8.0, 1e-3), (12.0, 1e-3)])
def test_total_area_invariant_2d(r, bound):
    # sum_n eps_{n,s} approximates the disk area; over these random sub-cell
    # offsets the relative error measures 2.6e-3 (r = 3), 2.5e-3 (6), 9.3e-4
    # (8) and 7.9e-4 (12), shrinking as the partial band's share of the area
    # does.  A dropped 1/2 in the offset of Eq. 18 would give an error near
    # 1/r.
    rng = np.random.default_rng(5)
    for _ in range(3):
        c = np.array([[20.0 + rng.uniform(-0.5, 0.5), 20.0 + rng.uniform(-0.5, 0.5), 0.0]])
        nslot, ids, eps, ssum = oracle.rasterize(_lat2(), c, np.array([r]))
        area = eps[nslot > 0, 0].sum()
        assert abs(area - math.pi * r * r) / (math.pi * r * r) < bound


@pytest.mark.parametrize("d", [10, 20])
def test_eq20_sphere_volume_error(d):
    # Eq. 20 setup: a sphere of diameter d centred in a (d+5)^3 box; the
    # relative volume error of the linear method is 0.076 % (d = 10) and
    # 0.098 % (d = 20), under 0.1 %.
    n = d + 5
    lat = W.LatticeSpec(q=19, nx=n, ny=n, nz=n)
    c = float(n // 2)
    nslot, ids, eps, ssum = oracle.rasterize(lat, np.array([[c, c, c]]), np.array([d / 2.0]))
    vol = eps[nslot > 0, 0].sum()
    err = abs(vol - math.pi * d ** 3 / 6.0) / (math.pi * d ** 3 / 6.0)
    assert err < 1e-3


def test_table1_step3_inside_outside_and_clamp():
    # Sec. 2.4: cells fully inside (d <= r-h) are solid, fully outside
    # (d >= r+h) are fluid; every fraction lies in [0, 1].
    r, h = 7.3, 1.0
    c = np.array([[20.25, 19.6, 0.0]])
    nslot, ids, eps, ssum = oracle.rasterize(_lat2(), c, np.array([r]))
    for n in range(1600):
        x, y = n % 40, n // 40
        d = math.hypot(x - c[0, 0], y - c[0, 1])
        e = eps[n, 0] if nslot[n] else 0.0
        assert 0.0 <= e <= 1.0
        if d <= r - h:
            assert e == 1.0
        if d >= r + h:
            assert e == 0.0


def test_small_shell_is_literal():
    # With a shell thinner than the clamp band, Table 1 cuts the linear ramp:
    # cells just outside r+h get 0 even where the ramp would be positive.
    lat = W.LatticeSpec(q=9, nx=40, ny=40, h=0.25)
    r = 6.0
    c = np.array([[20.0, 20.0, 0.0]])
    nslot, ids, eps, _ = oracle.rasterize(lat, c, np.array([r]))
    cs = oracle.va2d(r) + 0.5
    for n in range(1600):
        x, y = n % 40, n // 40
        d = math.hypot(x - 20.0, y - 20.0)
        e = eps[n, 0] if nslot[n] else 0.0
        if d >= r + 0.25:
            assert e == 0.0
        elif d <= r - 0.25:
            assert e == 1.0
        else:
            assert e == pytest.approx(min(1.0, max(0.0, cs - d)), abs=0)


def test_shared_cells_sum_and_order():
    # the cell total is the sum of the recorded fractions, recorded
    # in ascending particle order; periodic images wrap.
    lat = _lat2()
    X = np.array([[10.0, 20.0, 0.0], [22.4, 20.0, 0.0], [39.0, 5.0, 0.0]])
    R = np.array([6.0, 6.0, 4.0])
    nslot, ids, eps, ssum = oracle.rasterize(lat, X, R)
    shared = np.nonzero(nslot == 2)[0]
    assert shared.size > 0
    for n in shared:
        assert ids[n, 0] < ids[n, 1]
        assert ssum[n] == eps[n, 0] + eps[n, 1]
    # particle 2 at x=39 wraps onto x=0..3
    wrapped = [n for n in range(1600) if nslot[n] and 2 in ids[n, :nslot[n]] and n % 40 < 5]
    assert wrapped
