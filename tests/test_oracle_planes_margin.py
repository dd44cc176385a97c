"""Pins of the oracle's scattering planes and of its per-row margin (CPU only).

Scattering planes (Sec. II-B: in 3D the exit pair is drawn in the ut-plane and in the
uv-plane separately).  From the path the oracle records (entry P0 and direction d0, exit
P1 and direction d1, offsets t and v) the test recovers, with geometry of its own:

  * the entry angles per plane, tan(theta) = (d0 . t) / (d0 . u) and (d0 . v) / (d0 . u);
  * the lateral exit offsets per plane, from P1 - (t t + v v) = lat_t n_t + lat_v n_v + m d0
    (n_t, n_v: the unit components of t and v normal to d0; they need not be orthogonal,
    so a 2 x 2 system is solved);
  * the exit angles per plane, from d1 / (d1 . d0) = d0 + tan_t n_t + tan_v n_v.

They must equal the widths times the Gaussian pairs of the stated Philox streams (1: entry,
2: ut-plane exit pair, 3: uv-plane exit pair) to rounding, and over many protons have the
widths, the correlation rho inside each plane and no correlation across the planes.  A
displaced exit line that misses the outer boundary (checked with the test's own quadratic)
leaves the undisplaced exit.

Margin (the reading of "within 1e-6 mm of a voxel face"): the smallest distance of any
integer decision of the traversal from flipping, in mm:
  * the along-path gap between the next crossing and the next crossing of another axis;
  * the distance of a clipped segment end (or a spline sample) to the nearest interior face;
  * an axis-parallel segment's distance to the box faces it runs along;
  * the clipped length of a segment (grazing the box);
  * a boundary solve with half-chord below 1e-4 mm, or L / step within 1e-9 mm of an
    integer, makes the margin 0.
It is recomputed here in exact rational arithmetic from the same float inputs (straight
segments on tiny grids) and from the recorded path of curved rows, and planted
near-degenerate lines must come out below 1e-6 mm.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest


# ------------------------------------------------------------------ planes

def _frame(oracle, bm, g):
    k = oracle.angle_of(int(g), bm["n_protons"], bm["n_angles"])
    c, s = oracle.angle(bm.get("angle0_deg", 0.0), bm["dangle_deg"], k)
    return np.array([c, s, 0.0]), np.array([-s, c, 0.0]), np.array([0.0, 0.0, 1.0])


def _quadratic(reg, dim, Q, d):
    """Coefficients A l^2 + 2 B l + C of Q + l d against region 0 (ellipse or elliptic
    cylinder in x-y, or ellipsoid; not turned), in the region's scaled coordinates."""
    na = 3 if (dim == 3 and reg["shape"] == "ellipsoid") else 2
    c = np.array(list(reg["center"]) + [0.0] * (3 - len(reg["center"])))
    s = np.array(list(reg["semi"]) + [1.0] * (3 - len(reg["semi"])))
    q = (Q - c)[:na] / s[:na]
    e = d[:na] / s[:na]
    return e @ e, q @ e, q @ q - 1.0


def _ellipsoid_hit(reg, dim, Q, d):
    """Far root of Q + l d against region 0, or None when the line misses it."""
    A, B, C = _quadratic(reg, dim, Q, d)
    disc = B * B - A * C
    if disc <= 0:
        return None
    return (-B + math.sqrt(disc)) / A


def _half_chord(reg, dim, Q, d):
    """Half the chord of the line (d a unit vector); for a miss, the same expression of
    |discriminant|: how far the line is from touching the boundary."""
    A, B, C = _quadratic(reg, dim, Q, d)
    return math.sqrt(abs(B * B - A * C)) / A


def _recover(oracle, cfg, r):
    """Per curved row: (g, entry angles, exit offsets, exit angles, fallback flag)."""
    bm, ph = cfg["beam"], cfg["phantom"]
    dim = ph["dim"]
    out = []
    for i, g in enumerate(r["rows"]):
        p = r["paths"][i]
        if p.kind != oracle.KIND_CURVED:
            continue
        u, t, v = _frame(oracle, bm, g)
        d0, d1 = np.array(p.d0), np.array(p.d1)
        P1 = np.array(p.P1)
        th_t = math.atan((d0 @ t) / (d0 @ u))
        th_v = math.atan((d0 @ v) / (d0 @ u)) if dim == 3 else 0.0
        nt = t - (t @ d0) * d0
        nt /= np.linalg.norm(nt)
        if dim == 3:
            nv = v - (v @ d0) * d0
            nv /= np.linalg.norm(nv)
        else:
            nv = np.zeros(3)
        cc = nt @ nv
        G = np.array([[1.0, cc], [cc, 1.0]])
        Q = p.t * t + p.v * v
        rel = P1 - Q
        if dim == 3:
            lat = np.linalg.solve(G, [rel @ nt, rel @ nv])
        else:
            lat = np.array([rel @ nt, 0.0])
        w = d1 / (d1 @ d0)
        if dim == 3:
            tn = np.linalg.solve(G, [w @ nt, w @ nv])
        else:
            tn = np.array([w @ nt, 0.0])
        ang = np.arctan(tn)
        out.append(dict(i=i, g=int(g), th=(th_t, th_v), lat=lat, ang=ang, nt=nt, nv=nv, Q=Q, d0=d0, P1=P1))
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_exit_pairs_follow_their_streams(oracle, W, dim):
    """Every recovered angle and offset is the width times the draw of its own stream and
    plane (stream 1: entry t, v; stream 2: ut-plane exit pair; stream 3: uv-plane pair)."""
    sig_in, sig_out, sig_lat, rho = 0.05, 0.03, 1.5, 0.5
    if dim == 2:
        cfg = W.scaled(W.c1(), n_protons=360 * 8, sigma_in=sig_in, sigma_out=sig_out, sigma_lat=sig_lat, rho=rho)
    else:
        cfg = W.scaled(W.c2(), n_protons=90 * 40, sigma_in=sig_in, sigma_out=sig_out, sigma_lat=sig_lat, rho=rho)
    seed = cfg["beam"]["seed"]
    reg0 = cfg["phantom"]["regions"][0]
    r = oracle.run(cfg, with_paths=True)
    rec = _recover(oracle, cfg, r)
    assert len(rec) > 0.4 * len(r["rows"])
    crho = math.sqrt(1.0 - rho * rho)
    n_fallback = 0
    for q in rec:
        g = q["g"]
        zt, zv, _ = oracle.normal_pair(seed, 1, g)
        assert abs(q["th"][0] - sig_in * zt) < 1e-12
        if dim == 3:
            assert abs(q["th"][1] - sig_in * zv) < 1e-12
        z1, z2, _ = oracle.normal_pair(seed, 2, g)
        lat_t, ang_t = sig_lat * z1, sig_out * (rho * z1 + crho * z2)
        lat_v = ang_v = 0.0
        if dim == 3:
            z1, z2, _ = oracle.normal_pair(seed, 3, g)
            lat_v, ang_v = sig_lat * z1, sig_out * (rho * z1 + crho * z2)
        assert abs(q["ang"][0] - ang_t) < 1e-12, (g, q["ang"], ang_t)
        assert abs(q["ang"][1] - ang_v) < 1e-12, (g, q["ang"], ang_v)
        # the displaced line through Q + lat_t n_t + lat_v n_v along d0 exits the outer
        # boundary at P1; if it misses, P1 is the undisplaced exit (offsets 0)
        Qd = q["Q"] + lat_t * q["nt"] + lat_v * q["nv"]
        far = _ellipsoid_hit(reg0, dim, Qd, q["d0"])
        if far is None:
            n_fallback += 1
            assert np.all(np.abs(q["lat"]) < 1e-9), (g, q["lat"])
        else:
            assert abs(q["lat"][0] - lat_t) < 1e-9, (g, q["lat"], lat_t)
            assert abs(q["lat"][1] - lat_v) < 1e-9, (g, q["lat"], lat_v)
            assert np.allclose(q["P1"], Qd + far * q["d0"], atol=1e-9, rtol=0)
    assert n_fallback < 0.05 * len(rec)


def _corr(a, b):
    a, b = a - a.mean(), b - b.mean()
    return float((a @ b) / math.sqrt((a @ a) * (b @ b)))


def test_scattering_planes_statistics_3d(oracle, W):
    """Entry angles, exit offsets and exit angles in both planes: Gaussian widths, the
    correlation rho between offset and angle inside a plane, and independence across the
    planes (within 5 standard errors), and the mean square 3D lateral displacement
    2 sigma_lat^2."""
    sig_in, sig_out, sig_lat, rho = 0.05, 0.03, 1.5, 0.5
    cfg = W.scaled(W.c2(), n_protons=90 * 240, sigma_in=sig_in, sigma_out=sig_out, sigma_lat=sig_lat, rho=rho,
                   noise_rel=0.0)
    reg0 = cfg["phantom"]["regions"][0]
    r = oracle.run(cfg, rows=np.arange(0, 90 * 240, 2), with_paths=True)
    rec = _recover(oracle, cfg, r)
    # offsets only where the displaced line meets the boundary (else they are 0 by design)
    keep = []
    for q in rec:
        keep.append(bool(np.any(np.abs(q["lat"]) > 1e-12)))
    keep = np.array(keep)
    th_t = np.array([q["th"][0] for q in rec])
    th_v = np.array([q["th"][1] for q in rec])
    ang_t = np.array([q["ang"][0] for q in rec])
    ang_v = np.array([q["ang"][1] for q in rec])
    lat_t = np.array([q["lat"][0] for q in rec])[keep]
    lat_v = np.array([q["lat"][1] for q in rec])[keep]
    n, nl = len(rec), int(keep.sum())
    assert n > 4000 and nl > 0.95 * n

    def std_ok(x, sig, m):
        assert abs(x.std() - sig) < 5 * sig / math.sqrt(2 * m), (x.std(), sig)
        assert abs(x.mean()) < 5 * sig / math.sqrt(m)

    std_ok(th_t, sig_in, n)
    std_ok(th_v, sig_in, n)
    std_ok(ang_t, sig_out, n)
    std_ok(ang_v, sig_out, n)
    std_ok(lat_t, sig_lat, nl)
    std_ok(lat_v, sig_lat, nl)
    # inside a plane: correlation rho (standard error (1 - rho^2) / sqrt(m))
    se = (1 - rho * rho) / math.sqrt(nl)
    at, av = ang_t[keep], ang_v[keep]
    assert abs(_corr(lat_t, at) - rho) < 5 * se
    assert abs(_corr(lat_v, av) - rho) < 5 * se
    # across the planes: no correlation (standard error 1 / sqrt(m))
    for a, b in ((th_t, th_v), (ang_t, ang_v)):
        assert abs(_corr(a, b)) < 5 / math.sqrt(n)
    for a, b in ((lat_t, lat_v), (lat_t, av), (lat_v, at)):
        assert abs(_corr(a, b)) < 5 / math.sqrt(nl)
    # 3D lateral displacement |lat_t n_t + lat_v n_v|^2 has mean 2 sigma_lat^2
    d2 = []
    for q, k in zip(rec, keep):
        if k:
            dv = q["lat"][0] * q["nt"] + q["lat"][1] * q["nv"]
            d2.append(dv @ dv)
    d2 = np.array(d2)
    assert abs(d2.mean() - 2 * sig_lat ** 2) < 5 * d2.std() / math.sqrt(nl)
    # the exit point lies on the outer ellipsoid
    s = np.array(reg0["semi"])
    for q in rec[:500]:
        assert abs(float(np.sum((q["P1"] / s) ** 2)) - 1.0) < 1e-12


def test_scattering_planes_statistics_2d(oracle, W):
    sig_in, sig_out, sig_lat, rho = 0.02, 0.03, 1.5, 0.5
    cfg = W.scaled(W.c1(), n_protons=360 * 24, sigma_in=sig_in, sigma_out=sig_out, sigma_lat=sig_lat, rho=rho,
                   noise_rel=0.0)
    r = oracle.run(cfg, with_paths=True)
    rec = [q for q in _recover(oracle, cfg, r) if abs(q["lat"][0]) > 1e-12]
    n = len(rec)
    assert n > 6000
    lat = np.array([q["lat"][0] for q in rec])
    ang = np.array([q["ang"][0] for q in rec])
    th = np.array([q["th"][0] for q in rec])
    for x, sig in ((th, sig_in), (ang, sig_out), (lat, sig_lat)):
        assert abs(x.std() - sig) < 5 * sig / math.sqrt(2 * n)
    assert abs(_corr(lat, ang) - rho) < 5 * (1 - rho * rho) / math.sqrt(n)
    assert abs(_corr(th, ang)) < 5 / math.sqrt(n)


# ------------------------------------------------------------------ margin

def _F(v):
    return Fr(float(v))


def _point_margin(ph, p):
    """Distance (mm) of a point to the nearest interior face, per axis, minimised."""
    m = None
    o = _origin(ph)
    for d in range(ph["dim"]):
        n = ph["n"][d]
        if n < 2:
            continue
        f = (p[d] - _F(o[d])) / _F(ph["h"][d])
        j = math.floor(f + Fr(1, 2))
        j = min(max(j, 1), n - 1)
        v = abs(f - j) * _F(ph["h"][d])
        m = v if m is None else min(m, v)
    return m


def _origin(ph):
    if ph.get("origin") is not None:
        return list(ph["origin"])
    return [-(ph["n"][d] * ph["h"][d]) / 2.0 for d in range(3)]


def _floor_idx(ph, d, p):
    o = _origin(ph)
    f = math.floor((p - _F(o[d])) / _F(ph["h"][d]))
    return min(max(f, 0), ph["n"][d] - 1)


def _exact_segment_margin(ph, A, D, lo, hi, B=None):
    """Margin of one segment A + l D, l in [lo, hi] (floats; +-inf allowed), computed in
    exact rational arithmetic from the definition; None when nothing constrains it."""
    dim = ph["dim"]
    o = _origin(ph)
    cands = []
    Af = [_F(a) for a in A]
    Df = [_F(x) for x in D]
    lo_f = None if math.isinf(lo) else _F(lo)
    hi_f = None if math.isinf(hi) else _F(hi)
    hi_unclipped = True
    for d in range(dim):
        blo = _F(o[d])
        bhi = _F(o[d] + ph["n"][d] * ph["h"][d])
        if Df[d] != 0:
            t1, t2 = (blo - Af[d]) / Df[d], (bhi - Af[d]) / Df[d]
            a, b = min(t1, t2), max(t1, t2)
            lo_f = a if lo_f is None else max(lo_f, a)
            if hi_f is None or b < hi_f:
                hi_f = b
                hi_unclipped = False
        else:
            cands.append(min(abs(Af[d] - blo), abs(Af[d] - bhi)))
            if Af[d] < blo or Af[d] > bhi:
                return min(cands) if cands else None
    Dn = math.sqrt(float(sum(x * x for x in Df[:dim])))
    if lo_f is None or hi_f is None:
        return min(cands) if cands else None
    cands.append(abs(hi_f - lo_f) * _F(Dn))
    if not lo_f < hi_f:
        return min(cands)
    P = [Af[d] + lo_f * Df[d] for d in range(3)]
    if B is not None and hi_unclipped and not math.isinf(hi):
        E = [_F(b) for b in B]
    else:
        E = [Af[d] + hi_f * Df[d] for d in range(3)]
    for q in (P, E):
        pm = _point_margin(ph, q)
        if pm is not None:
            cands.append(pm)
    # crossings of the faces between the end voxels, merged in order
    xs = []
    for d in range(dim):
        i0, i1 = _floor_idx(ph, d, P[d]), _floor_idx(ph, d, E[d])
        if i1 > i0:
            faces = range(i0 + 1, i1 + 1)
        else:
            faces = range(i1 + 1, i0 + 1)
        for k in faces:
            plane = _F(o[d]) + k * _F(ph["h"][d])
            xs.append(((plane - Af[d]) / Df[d], d))
    xs.sort()
    for j, (la, a) in enumerate(xs):
        for lb, b in xs[j + 1:]:
            if b != a:
                cands.append((lb - la) * _F(Dn))
                break
    return min(cands)


def _tiny(W, dim):
    if dim == 2:
        return W.phantom(2, (8, 8), (1.0, 1.0), [{"shape": "ellipse", "center": [0, 0], "semi": [1e6, 1e6],
                                                   "rsp": 1.0}])
    return W.phantom(3, (6, 5, 4), (1.0, 1.0, 1.0), [{"shape": "ellipse", "center": [0, 0, 0],
                                                       "semi": [1e6, 1e6, 1e6], "rsp": 1.0}])


@pytest.mark.parametrize("dim", [2, 3])
def test_margin_equals_exact_definition(oracle, W, dim):
    """Random lines and segments on tiny grids: the oracle's margin equals the margin of
    the definition computed in rational arithmetic from the same inputs."""
    ph = _tiny(W, dim)
    rng = np.random.default_rng(200 + dim)
    half = np.array([ph["n"][d] * ph["h"][d] / 2 for d in range(3)])
    checked = 0
    for trial in range(160):
        A = np.zeros(3)
        B = np.zeros(3)
        A[:dim] = rng.uniform(-1.3, 1.3, dim) * half[:dim]
        B[:dim] = rng.uniform(-1.3, 1.3, dim) * half[:dim]
        if trial % 7 == 0:
            B[1:dim] = A[1:dim]           # axis-parallel
        D = B - A
        lo, hi = [(0.0, 1.0), (-math.inf, math.inf), (-0.5, 1.5), (-math.inf, 0.0)][trial % 4]
        got = oracle.trace_segments(ph, [A], [D], [lo], [hi])
        ref = _exact_segment_margin(ph, A, D, lo, hi)
        if ref is None:
            assert math.isinf(got["margin"])
            continue
        checked += 1
        assert abs(got["margin"] - float(ref)) <= 1e-12 * max(1.0, float(ref)), (trial, got["margin"], float(ref))
    assert checked > 120


@pytest.mark.parametrize("dim", [2, 3])
def test_margin_flags_planted_near_degenerate_lines(oracle, W, dim):
    """A line through a voxel edge (corner in 2D) shifted by 1e-8 mm, an end point 1e-8 mm
    from a face, an axis-parallel line 1e-8 mm from the box, and a segment 1e-8 mm long
    inside the box all report margins below 1e-6 mm; the same lines moved 0.3 mm away
    report margins above it."""
    ph = _tiny(W, dim)
    eps = 1e-8
    rng = np.random.default_rng(300 + dim)
    for trial in range(40):
        # through grid point (1, 2[, 1]) in voxel units of the centred grid
        corner = np.array([1.0, 2.0, 1.0 if dim == 3 else 0.0]) - np.array(
            [ph["n"][d] / 2.0 if d < dim else 0.0 for d in range(3)])
        ang = rng.uniform(0.2, 1.3)
        D = np.array([math.cos(ang), math.sin(ang), 0.0])
        if dim == 3:
            D[2] = rng.uniform(-0.5, 0.5)
            D /= np.linalg.norm(D)
        n = np.array([-D[1], D[0], 0.0])
        n /= np.linalg.norm(n)
        for off, small in ((eps, True), (0.3, False)):
            A = corner + off * n
            got = oracle.trace_segments(ph, [A], [D], [-math.inf], [math.inf])
            ref = float(_exact_segment_margin(ph, A, D, -math.inf, math.inf))
            assert abs(got["margin"] - ref) <= 1e-12 * max(1.0, ref)
            if small:
                assert got["margin"] < 1e-6
            elif dim == 2:
                # nothing else in this line comes within 1e-6 mm (2D: only corners matter)
                assert got["margin"] > 1e-6 or ref < 1e-6
    # end point near a face
    A = np.array([1.0 + eps, 0.25, 0.3 if dim == 3 else 0.0])   # faces lie at integers
    got = oracle.trace_segments(ph, [A], [np.array([-1.7, 0.9, 0.2 if dim == 3 else 0.0])], [0.0], [1.0])
    assert got["margin"] < 1e-6
    A[0] = 1.0 + 0.3
    got = oracle.trace_segments(ph, [A], [np.array([-1.7, 0.9, 0.2 if dim == 3 else 0.0])], [0.0], [1.0])
    assert got["margin"] > 1e-6 or float(_exact_segment_margin(ph, A, [-1.7, 0.9, 0.2 if dim == 3 else 0.0],
                                                                 0.0, 1.0)) < 1e-6
    # axis-parallel line close to the box face
    top = ph["n"][1] * ph["h"][1] / 2.0
    A = np.array([-9.0, top - eps, 0.1 if dim == 3 else 0.0])
    got = oracle.trace_segments(ph, [A], [np.array([1.0, 0.0, 0.0])], [-math.inf], [math.inf])
    assert got["margin"] < 1e-6
    # a tiny segment
    A = np.array([0.3, 0.3, 0.3 if dim == 3 else 0.0])
    got = oracle.trace_segments(ph, [A], [np.array([eps, 0.0, 0.0])], [0.0], [1.0])
    assert got["margin"] < 1e-6


def _hermite(P0, d0, P1, d1, L, s):
    h00 = 2 * s ** 3 - 3 * s ** 2 + 1
    h10 = s ** 3 - 2 * s ** 2 + s
    h01 = -2 * s ** 3 + 3 * s ** 2
    h11 = s ** 3 - s ** 2
    return h00 * P0 + h10 * L * d0 + h01 * P1 + h11 * L * d1


@pytest.mark.parametrize("which", ["c1", "c2"])
def test_margin_of_curved_rows_from_their_paths(oracle, W, which):
    """Curved rows: the margin is the minimum of the segment margins of the polyline
    (entry ray, the chords between the samples, exit ray), rebuilt from the recorded path,
    or 0 when either boundary solve (the entry line, the displaced exit line) has a
    half-chord below 1e-4 mm or L / step is within 1e-9 mm of an integer."""
    if which == "c1":
        cfg = W.scaled(W.c1(), n_protons=360 * 4)
    else:
        cfg = W.scaled(W.c2(), n_protons=90 * 4)
    ph, bm = cfg["phantom"], cfg["beam"]
    dim = ph["dim"]
    reg0 = ph["regions"][0]
    rows = np.arange(0, bm["n_protons"], 3)
    r = oracle.run(cfg, rows=rows, with_paths=True)
    seed = bm["seed"]
    checked = zeros = 0
    for q in _recover(oracle, cfg, r):
        i = q["i"]
        p = r["paths"][i]
        P0, P1, d0, d1 = (np.array(v) for v in (p.P0, p.P1, p.d0, p.d1))
        N = p.n_samples
        steps = p.L / bm["step"]
        # the displaced exit line from the exit-pair draws (streams 2 and 3)
        z1, _, _ = oracle.normal_pair(seed, 2, q["g"])
        lat_v = oracle.normal_pair(seed, 3, q["g"])[0] * bm["sigma_lat"] if dim == 3 else 0.0
        Qd = q["Q"] + bm["sigma_lat"] * z1 * q["nt"] + lat_v * q["nv"]
        fragile = (abs(steps - math.floor(steps + 0.5)) * bm["step"] < 1e-9 or p.thickness / 2 < 1e-4
                   or _half_chord(reg0, dim, Qd, d0) < 1e-4)
        if fragile:
            assert r["margin"][i] == 0.0
            zeros += 1
            continue
        ms = [_exact_segment_margin(ph, P0, d0, -math.inf, 0.0)]
        S = [P0] + [_hermite(P0, d0, P1, d1, p.L, j / N) for j in range(1, N)] + [P1]
        for j in range(N):
            ms.append(_exact_segment_margin(ph, S[j], S[j + 1] - S[j], 0.0, 1.0, B=S[j + 1]))
        ms.append(_exact_segment_margin(ph, P1, d1, 0.0, math.inf))
        ref = float(min(m for m in ms if m is not None))
        assert abs(r["margin"][i] - ref) <= 1e-9, (i, r["margin"][i], ref)
        checked += 1
    assert checked > len(rows) // 3 and zeros < checked // 20


def test_margin_zero_for_fragile_solves(oracle, W):
    """Planted curved rows (one projection angle, no scattering, every proton at one
    offset t): a line tangent to the outer ellipse to 1e-13 relative, and the line whose
    chord is 179.75 mm = 719 samples of 0.25 mm (to rounding), report margin 0; a line at
    t = 30.1 mm (no face, no tangency, a non-integer sample count) does not."""
    base = W.scaled(W.c1(), n_protons=4, n_angles=1, dangle_deg=1.0, sigma_in=0.0, sigma_out=0.0,
                    sigma_lat=0.0, noise_rel=0.0)
    a, b = base["phantom"]["regions"][0]["semi"][:2]
    t719 = b * math.sqrt(1.0 - (179.75 / (2.0 * a)) ** 2)   # chord 2 a sqrt(1 - t^2 / b^2)
    for t0, fragile in ((b * (1.0 - 1e-13), True), (t719, True), (30.1, False)):
        cfg = W.scaled(base, t_range=(t0, t0))
        r = oracle.run(cfg, with_paths=True)
        assert all(r["paths"][i].kind == oracle.KIND_CURVED for i in range(4))
        if fragile:
            assert np.all(r["margin"] == 0.0), (t0, r["margin"])
        else:
            assert np.all(r["margin"] > 1e-3), (t0, r["margin"])
