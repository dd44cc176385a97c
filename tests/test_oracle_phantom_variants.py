"""Pins of the oracle's phantom variants (Sec. II-A) on the CPU: the weighted-area pixel
rule and turned ellipses.

  * weighted area: the RSP-weighted area sum tends to pi a b RSP as the midpoints per
    axis S grow; a pixel cut by the boundary holds RSP x its exact area fraction
    (scipy quadrature of the clipped chord) within the midpoint rule's error; pixels
    wholly inside or outside hold the exact RSP; 3D volume sums tend to 4/3 pi a b c;
  * turned ellipses: the chord through the center of a turned ellipse has the closed
    form 2 a b / sqrt(b^2 cos^2 + a^2 sin^2) of the angle between the line and the major
    axis; a quarter turn equals swapped semi-axes; a circle is unchanged by any turn.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import oracle as O
from paper_2108_12369_amd import workloads as W


def _single(a, b, rsp=1.3, angle=0.0, n=(64, 48), h=(4.0, 4.0), samples=8, voxelize="area_avg", center=(0, 0)):
    regs = [W._e(center, (a, b), rsp, angle_deg=angle)]
    return W.phantom(2, n, h, regs, voxelize=voxelize, area_samples=samples)


@pytest.mark.parametrize("angle", [0.0, 33.0])
def test_area_rule_converges_to_ellipse_area(angle):
    errs = []
    for S in (2, 4, 8, 16):
        ph = _single(70.0, 45.0, angle=angle, samples=S)
        x = O.phantom_build(ph)
        total = float(x.astype(np.float64).sum()) * 16.0
        errs.append(abs(total - 1.3 * math.pi * 70.0 * 45.0) / (1.3 * math.pi * 70.0 * 45.0))
    assert errs[-1] < 2e-4, errs
    assert errs[-1] < errs[0]


def _exact_fraction(a, b, x0, x1, y0, y1):
    """Area of {(x/a)^2 + (y/b)^2 <= 1} inside [x0,x1] x [y0,y1], by quadrature."""
    def chord(x):
        if abs(x) >= a:
            return 0.0
        yh = b * math.sqrt(1.0 - (x / a) ** 2)
        return max(0.0, min(yh, y1) - max(-yh, y0))
    lo, hi = max(x0, -a), min(x1, a)
    if lo >= hi:
        return 0.0
    v, _ = integrate.quad(chord, lo, hi, limit=200, epsabs=1e-12)
    return v / ((x1 - x0) * (y1 - y0))


def test_boundary_pixels_hold_their_area_fraction():
    a, b, S = 70.0, 45.0, 16
    ph = _single(a, b, rsp=1.0, samples=S)
    x = O.phantom_build(ph).reshape(48, 64)
    o = (-128.0, -96.0)
    cut = 0
    for iy in range(48):
        for ix in range(64):
            x0, y0 = o[0] + 4.0 * ix, o[1] + 4.0 * iy
            f = _exact_fraction(a, b, x0, x0 + 4.0, y0, y0 + 4.0)
            if 0.0 < f < 1.0:
                cut += 1
                assert abs(float(x[iy, ix]) - f) <= 2.0 / S, (ix, iy, float(x[iy, ix]), f)
            else:
                assert float(x[iy, ix]) == f   # wholly inside (1) or outside (0): exact
    assert cut > 50


def test_area_rule_painter_order_and_bounds():
    ph = W.phantom(2, (100, 80), (2.0, 2.0), W.neo1_regions(), voxelize="area_avg", area_samples=8)
    x = O.phantom_build(ph)
    assert x.min() >= 0.0 and x.max() <= 1.6
    xc = O.phantom_build(dict(ph, voxelize="center"))
    # interior pixels agree with the center rule; only boundary pixels differ
    assert (x == xc).mean() > 0.8


def test_area_rule_3d_volume():
    regs = [W._e((0, 0, 0), (60.0, 45.0, 50.0), 1.0, "ellipsoid")]
    ph = W.phantom(3, (40, 32, 36), (4.0, 4.0, 4.0), regs, voxelize="area_avg", area_samples=6)
    x = O.phantom_build(ph)
    vol = float(x.astype(np.float64).sum()) * 64.0
    want = 4.0 / 3.0 * math.pi * 60 * 45 * 50
    assert abs(vol - want) / want < 2e-3


@pytest.mark.parametrize("theta,phi", [(0.0, 0.0), (30.0, 0.0), (30.0, 75.0), (-50.0, 10.0), (90.0, 45.0)])
def test_turned_outer_boundary_chord(theta, phi):
    a, b = 90.0, 70.0
    ph = W.phantom(2, (10, 10), (1.0, 1.0), [W._e((5.0, -3.0), (a, b), 1.0, angle_deg=theta)])
    p = math.radians(phi)
    d = [math.cos(p), math.sin(p), 0.0]
    hit, l1, l2, _ = O.boundary_hit(ph, [5.0, -3.0, 0.0], d)
    assert hit
    rel = math.radians(phi - theta)
    want = 2 * a * b / math.sqrt((b * math.cos(rel)) ** 2 + (a * math.sin(rel)) ** 2)
    assert l2 - l1 == pytest.approx(want, rel=1e-13)
    assert l1 == pytest.approx(-want / 2, rel=1e-13)


def test_quarter_turn_swaps_semi_axes():
    for vox in ("center", "area_avg"):
        turned = O.phantom_build(_single(50.0, 30.0, angle=90.0, voxelize=vox, n=(40, 40), h=(3.0, 3.0)))
        swapped = O.phantom_build(_single(30.0, 50.0, angle=0.0, voxelize=vox, n=(40, 40), h=(3.0, 3.0)))
        # cos(90 deg) is not exactly 0: only points within rounding of the boundary may flip
        assert (turned != swapped).mean() < 0.01
        assert abs(float(turned.sum()) - float(swapped.sum())) / float(swapped.sum()) < 0.01
    # a turned circle is the circle
    c0 = O.phantom_build(_single(40.0, 40.0, angle=0.0, voxelize="area_avg", n=(40, 40), h=(3.0, 3.0)))
    c1 = O.phantom_build(_single(40.0, 40.0, angle=27.0, voxelize="area_avg", n=(40, 40), h=(3.0, 3.0)))
    assert np.abs(c0 - c1).max() <= 1.0 / 64 + 1e-7


def test_turned_point_membership():
    ph = {"dim": 2, "n": [1, 1, 1], "h": [1.0, 1.0, 1.0], "origin": None, "voxelize": "center",
          "regions": [W._e((10.0, 5.0), (20.0, 5.0), 1.0, angle_deg=30.0)]}
    t = math.radians(30.0)
    u = (math.cos(t), math.sin(t))
    v = (-math.sin(t), math.cos(t))
    # along the turned major axis: inside up to 20, outside beyond; along the minor: 5
    assert O.rsp_at(ph, [10 + 19.9 * u[0], 5 + 19.9 * u[1]]) == 1.0
    assert O.rsp_at(ph, [10 + 20.1 * u[0], 5 + 20.1 * u[1]]) == 0.0
    assert O.rsp_at(ph, [10 + 4.9 * v[0], 5 + 4.9 * v[1]]) == 1.0
    assert O.rsp_at(ph, [10 + 5.1 * v[0], 5 + 5.1 * v[1]]) == 0.0
