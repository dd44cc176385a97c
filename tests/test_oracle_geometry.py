"""Pins of the oracle's geometry: boundary solves, the Hermite path and the phantom.

Closed forms used:
  * chord of a centred axis-aligned ellipse (semi-axes a, b) cut by the line at signed
    distance t from the centre with direction (cos phi, sin phi):
        2 a b sqrt(R^2 - t^2) / R^2,   R^2 = a^2 sin^2 phi + b^2 cos^2 phi;
  * axis-parallel chords of an ellipsoid: 2 a sqrt(1 - (y/b)^2 - (z/c)^2);
  * a tilted line against an elliptic cylinder: the 2D chord of its x-y projection,
    scaled by |d| / |d_xy|;
  * cubic Hermite end points and end tangents.
"""
import math

import numpy as np
import pytest


def _ellipse_phantom(W, a=90.0, b=70.0, dim=2, shape="ellipse", c=80.0, n=(200, 200, 160), h=1.0):
    semi = (a, b) if dim == 2 else (a, b, c)
    center = (0.0, 0.0) if dim == 2 else (0.0, 0.0, 0.0)
    regs = [{"shape": shape, "center": list(center), "semi": list(semi), "rsp": 1.0}]
    return W.phantom(dim, n[:dim], (h,) * dim, regs)


def _q(p, center, semi):
    return sum(((p[i] - center[i]) / semi[i]) ** 2 for i in range(len(semi)))


@pytest.mark.parametrize("a,b", [(90.0, 70.0), (70.0, 90.0), (50.0, 50.0), (12.0, 6.0)])
def test_ellipse_chord_closed_form(oracle, W, a, b):
    ph = _ellipse_phantom(W, a, b)
    rng = np.random.default_rng(1)
    for _ in range(300):
        phi = rng.uniform(0, 2 * math.pi)
        c, s = math.cos(phi), math.sin(phi)
        R2 = a * a * s * s + b * b * c * c
        t = rng.uniform(-1.2, 1.2) * math.sqrt(R2)
        hit, l1, l2, hc = oracle.boundary_hit(ph, (-t * s, t * c, 0.0), (c, s, 0.0))
        if t * t >= R2:
            assert not hit
            continue
        assert hit and l1 < l2
        chord = 2.0 * a * b * math.sqrt(R2 - t * t) / R2
        assert abs((l2 - l1) - chord) <= 1e-12 * max(chord, 1e-3) + 1e-12
        assert abs(hc - chord / 2) <= 1e-9 * max(chord, 1.0)
        for lam in (l1, l2):
            p = (-t * s + lam * c, t * c + lam * s)
            assert abs(_q(p, (0, 0), (a, b)) - 1.0) < 1e-12


def test_ellipse_chord_axes(oracle, W):
    ph = _ellipse_phantom(W, 90.0, 70.0)
    # phi = 0: horizontal line at y = t -> 2 a sqrt(1 - t^2/b^2)
    for t in (0.0, 10.0, -35.0, 69.0):
        hit, l1, l2, _ = oracle.boundary_hit(ph, (0.0, t, 0.0), (1.0, 0.0, 0.0))
        assert hit and abs((l2 - l1) - 2 * 90.0 * math.sqrt(1 - t * t / 4900.0)) < 1e-12
    # phi = 90: vertical line at x = -t -> 2 b sqrt(1 - t^2/a^2)
    for t in (0.0, 10.0, -35.0, 89.0):
        hit, l1, l2, _ = oracle.boundary_hit(ph, (-t, 0.0, 0.0), (0.0, 1.0, 0.0))
        assert hit and abs((l2 - l1) - 2 * 70.0 * math.sqrt(1 - t * t / 8100.0)) < 1e-12
    hit, *_ = oracle.boundary_hit(ph, (0.0, 70.5, 0.0), (1.0, 0.0, 0.0))
    assert not hit


def test_ellipsoid_chords(oracle, W):
    a, b, c = 90.0, 70.0, 80.0
    ph = _ellipse_phantom(W, a, b, dim=3, shape="ellipsoid", c=c)
    rng = np.random.default_rng(2)
    for _ in range(200):
        y, z = rng.uniform(-70, 70), rng.uniform(-80, 80)
        inside = 1 - (y / b) ** 2 - (z / c) ** 2
        hit, l1, l2, _ = oracle.boundary_hit(ph, (0.0, y, z), (1.0, 0.0, 0.0))
        assert hit == (inside > 0)
        if hit:
            assert abs((l2 - l1) - 2 * a * math.sqrt(inside)) < 1e-11
    # general lines: both roots lie on the surface and between them the line is inside
    for _ in range(300):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        Q = rng.uniform(-60, 60, 3)
        hit, l1, l2, _ = oracle.boundary_hit(ph, tuple(Q), tuple(d))
        qmid = _q(Q + 0.5 * (l1 + l2) * d, (0, 0, 0), (a, b, c)) if hit else None
        if hit:
            for lam in (l1, l2):
                assert abs(_q(Q + lam * d, (0, 0, 0), (a, b, c)) - 1.0) < 1e-11
            assert qmid < 1.0


def test_cylinder_tilted_line(oracle, W):
    """In 3D an 'ellipse' region is an elliptic cylinder along z."""
    a, b = 90.0, 70.0
    ph = _ellipse_phantom(W, a, b, dim=3, shape="ellipse")
    rng = np.random.default_rng(4)
    for _ in range(200):
        phi = rng.uniform(0, 2 * math.pi)
        tilt = rng.uniform(-0.3, 0.3)
        c, s = math.cos(phi), math.sin(phi)
        d = np.array([c, s, math.tan(tilt)])
        R2 = a * a * s * s + b * b * c * c
        t = rng.uniform(-0.9, 0.9) * math.sqrt(R2)
        hit, l1, l2, _ = oracle.boundary_hit(ph, (-t * s, t * c, rng.uniform(-50, 50)), tuple(d))
        assert hit
        chord_xy = 2.0 * a * b * math.sqrt(R2 - t * t) / R2
        assert abs((l2 - l1) * np.linalg.norm(d) - chord_xy * np.linalg.norm(d)) < 1e-10


def test_hermite_identities(oracle):
    rng = np.random.default_rng(5)
    for _ in range(50):
        P0, P1 = rng.uniform(-80, 80, 3), rng.uniform(-80, 80, 3)
        d0, d1 = rng.normal(size=3), rng.normal(size=3)
        d0 /= np.linalg.norm(d0)
        d1 /= np.linalg.norm(d1)
        L = float(np.linalg.norm(P1 - P0))
        H = lambda s: np.array(oracle.hermite(P0, d0, P1, d1, L, s))
        assert np.array_equal(H(0.0), P0)
        assert np.allclose(H(1.0), P1, atol=1e-12, rtol=0)
        eps = 1e-6
        # one-sided second-order differences for the end tangents
        dH0 = (-3 * H(0.0) + 4 * H(eps) - H(2 * eps)) / (2 * eps)
        dH1 = (3 * H(1.0) - 4 * H(1 - eps) + H(1 - 2 * eps)) / (2 * eps)
        assert np.allclose(dH0, L * d0, atol=1e-5 * max(L, 1))
        assert np.allclose(dH1, L * d1, atol=1e-5 * max(L, 1))
    # with both tangents along the chord the curve is the straight segment
    P0, P1 = np.array([-50.0, 3.0, 1.0]), np.array([60.0, -7.0, 2.0])
    L = float(np.linalg.norm(P1 - P0))
    d = (P1 - P0) / L
    for s in np.linspace(0, 1, 17):
        assert np.allclose(oracle.hermite(P0, d, P1, d, L, s), P0 + s * (P1 - P0), atol=1e-12)


def test_phantom_painters_order(oracle, W):
    ph = W.phantom(2, (200, 200), (1.0, 1.0), W.neo1_regions())
    assert oracle.rsp_at(ph, (0.0, 0.0)) == pytest.approx(1.04, abs=1e-7)
    assert oracle.rsp_at(ph, (10.0, 5.0)) == pytest.approx(0.9, abs=1e-7)
    assert oracle.rsp_at(ph, (-10.0, 5.0)) == pytest.approx(0.9, abs=1e-7)
    assert oracle.rsp_at(ph, (0.0, 55.0)) == 0.0
    assert oracle.rsp_at(ph, (88.0, 0.0)) == pytest.approx(1.6, abs=1e-7)
    assert oracle.rsp_at(ph, (95.0, 0.0)) == 0.0
    assert oracle.rsp_at(ph, (90.0, 0.0)) == pytest.approx(1.6, abs=1e-7)  # closed boundary


def _area_weighted_total(regions, dim):
    """Sum of RSP x area of each region's visible part, by fine numerical integration
    (independent of the voxel rules)."""
    xs = np.linspace(-100, 100, 4001)[:-1] + 0.025
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    val = np.zeros_like(X)
    for r in regions:
        q = ((X - r["center"][0]) / r["semi"][0]) ** 2 + ((Y - r["center"][1]) / r["semi"][1]) ** 2
        val = np.where(q <= 1.0, r["rsp"], val)
    return val.sum() * 0.05 * 0.05


def test_phantom_corner_average_values(oracle, W):
    ph = W.phantom(2, (200, 200), (1.0, 1.0), W.neo1_regions())
    x = oracle.phantom_build(ph)
    rsps = sorted({float(np.float32(r["rsp"])) for r in ph["regions"]} | {0.0})
    allowed = set()
    for i in rsps:
        for j in rsps:
            for k in rsps:
                for m in rsps:
                    allowed.add(float(np.float32((i + j + k + m) / 4.0)))
    assert set(np.unique(x).tolist()) <= allowed
    assert x.min() >= 0.0 and x.max() <= 1.6 + 1e-6


@pytest.mark.parametrize("voxelize", ["corner_avg", "center"])
def test_phantom_mass_converges(oracle, W, voxelize):
    regs = W.neo1_regions()
    ref = _area_weighted_total(regs, 2)
    errs = []
    for h in (2.0, 1.0, 0.5):
        n = int(round(200 / h))
        x = oracle.phantom_build(W.phantom(2, (n, n), (h, h), regs, voxelize))
        errs.append(abs(float(x.astype(np.float64).sum()) * h * h - ref))
    assert errs[-1] < 0.01 * ref
    assert errs[2] < errs[0]


def test_phantom_3d_cylinder_is_stacked_2d(oracle, W):
    regs2 = W.neo1_regions()
    x2 = oracle.phantom_build(W.phantom(2, (40, 30), (5.0, 5.0), regs2))
    x3 = oracle.phantom_build(W.phantom(3, (40, 30, 6), (5.0, 5.0, 2.0), regs2))
    assert np.array_equal(x3.reshape(6, 30 * 40), np.tile(x2, (6, 1)))


def test_ellipsoid_phantom_volume(oracle, W):
    """Homogeneous ellipsoid: sum x h^3 -> 4/3 pi a b c."""
    regs = [{"shape": "ellipsoid", "center": [0, 0, 0], "semi": [30.0, 20.0, 25.0], "rsp": 1.0}]
    vols = []
    for h in (4.0, 2.0, 1.0):
        n = int(round(80 / h))
        x = oracle.phantom_build(W.phantom(3, (n, n, n), (h, h, h), regs))
        vols.append(float(x.astype(np.float64).sum()) * h ** 3)
    exact = 4.0 / 3.0 * math.pi * 30 * 20 * 25
    errs = [abs(v - exact) / exact for v in vols]
    assert errs[-1] < 0.01 and errs[-1] < errs[0]
