"""Pins of the oracle's voxel traversal, rows and WEPL (CPU only).

  * brute force: on tiny grids every segment is sampled every 1e-5 mm (midpoint rule)
    and the samples are binned by voxel; lengths agree within 2e-5 mm;
  * the chord of a straight row inside the grid box, computed by intersecting the line
    with the four (six) box faces as bounded facets, equals the sum of the row;
  * nnz of a straight row is 1 + sum_d |i_d(exit) - i_d(entry)|;
  * a curved row sums to the grid-clipped length of its polyline;
  * with zero scattering the curved row is the straight row;
  * reversing a line reverses its row;
  * 3D rows through an elliptic-cylinder phantom are 2D rows shifted by the slice;
  * WEPL of a homogeneous grid is rsp x chord; of a homogeneous ellipse it is within
    rsp x (length in boundary voxels) of rsp x the closed-form ellipse chord;
  * noise has relative standard deviation r.
"""
import math

import numpy as np
import pytest


def _grid(W, n, h, dim, regs=None):
    if regs is None:
        c = [0.0] * dim
        regs = [{"shape": "ellipse", "center": c, "semi": [1e6] * dim, "rsp": 1.0}]
    return W.phantom(dim, n, h, regs)


def _origin(ph):
    return [-(ph["n"][d] * ph["h"][d]) / 2.0 for d in range(3)]


def _brute_row(ph, A, D, lo, hi, ds=1e-5):
    """Bin midpoint samples of A + l D, l in [lo, hi], by voxel (only inside the box)."""
    dim = ph["dim"]
    o = _origin(ph)
    n, h = ph["n"], ph["h"]
    A, D = np.asarray(A, float), np.asarray(D, float)
    Dn = float(np.linalg.norm(D[:dim]))
    L = (hi - lo) * Dn
    m = max(1, int(math.ceil(L / ds)))
    lam = lo + (np.arange(m) + 0.5) * (hi - lo) / m
    P = A[None, :] + lam[:, None] * D[None, :]
    idx = [np.floor((P[:, d] - o[d]) / h[d]).astype(np.int64) for d in range(dim)]
    inside = np.ones(m, bool)
    for d in range(dim):
        inside &= (idx[d] >= 0) & (idx[d] < n[d])
    col = idx[0] + n[0] * idx[1]
    if dim == 3:
        col = col + n[0] * n[1] * idx[2]
    col = col[inside]
    w = L / m
    out = {}
    for c, k in zip(*np.unique(col, return_counts=True)):
        out[int(c)] = k * w
    return out


def _agg(cols, vals):
    out = {}
    for c, v in zip(cols.tolist(), vals.tolist()):
        out[c] = out.get(c, 0.0) + v
    return out


def _compare_brute(got, ref, tol=2e-5):
    for c in set(got) | set(ref):
        g, r = got.get(c, 0.0), ref.get(c, 0.0)
        assert abs(g - r) <= tol, (c, g, r)
        if r > 1e-4:
            assert c in got
        if g > 1e-4:
            assert c in ref


@pytest.mark.parametrize("dim", [2, 3])
def test_bruteforce_tiny_grids(oracle, W, dim):
    if dim == 2:
        ph = _grid(W, (8, 8), (1.0, 1.0), 2)
    else:
        ph = _grid(W, (6, 5, 4), (1.0, 1.0, 1.0), 3)
    rng = np.random.default_rng(10 + dim)
    half = np.array([ph["n"][d] * ph["h"][d] / 2 for d in range(3)])
    for trial in range(25):
        A = np.zeros(3)
        B = np.zeros(3)
        A[:dim] = rng.uniform(-1.3, 1.3, dim) * half[:dim]
        B[:dim] = rng.uniform(-1.3, 1.3, dim) * half[:dim]
        if trial % 5 == 0:  # axis-parallel segment
            B[1:dim] = A[1:dim]
        D = B - A
        lo, hi = (0.0, 1.0) if trial % 3 else (-0.5, 1.5)
        got = oracle.trace_segments(ph, [A], [D], [lo], [hi])
        ref = _brute_row(ph, A, D, lo, hi)
        _compare_brute(_agg(got["cols"], got["vals"]), ref)
        # consecutive entries are face neighbours (one index changes by one)
        n = ph["n"]
        ids = [np.unravel_index(c, (n[2], n[1], n[0]) if dim == 3 else (n[1], n[0])) for c in got["cols"]]
        for p, q in zip(ids, ids[1:]):
            assert sum(abs(int(a) - int(b)) for a, b in zip(p, q)) == 1


def test_bruteforce_polyline_merges_joints(oracle, W):
    ph = _grid(W, (8, 8), (1.0, 1.0), 2)
    rng = np.random.default_rng(21)
    pts = np.zeros((12, 3))
    pts[0, :2] = (-3.7, -2.2)
    for k in range(1, 12):
        pts[k, :2] = pts[k - 1, :2] + rng.uniform(-0.4, 0.9, 2)
    A = pts[:-1]
    D = pts[1:] - pts[:-1]
    got = oracle.trace_segments(ph, A, D, np.zeros(len(A)), np.ones(len(A)))
    ref = {}
    for a, d in zip(A, D):
        for c, v in _brute_row(ph, a, d, 0.0, 1.0).items():
            ref[c] = ref.get(c, 0.0) + v
    _compare_brute(_agg(got["cols"], got["vals"]), ref, tol=4e-5)
    # a merged joint never leaves two consecutive entries with the same column
    assert np.all(got["cols"][1:] != got["cols"][:-1])


def _box_chord(o, hi_, Q, d, dim):
    """Grid-box chord by intersecting the line with each face as a bounded facet."""
    pts = []
    for a in range(dim):
        if d[a] == 0.0:
            continue
        for plane in (o[a], hi_[a]):
            lam = (plane - Q[a]) / d[a]
            p = Q + lam * d
            ok = all(o[b] - 1e-9 <= p[b] <= hi_[b] + 1e-9 for b in range(dim) if b != a)
            if ok:
                pts.append(lam)
    if len(pts) < 2:
        return 0.0, None, None
    return (max(pts) - min(pts)) * float(np.linalg.norm(d[:dim])), min(pts), max(pts)


def test_straight_rows_chord_and_count(oracle, W):
    cfg = W.c0()
    ph = cfg["phantom"]
    o = np.array(_origin(ph))
    top = o + np.array(ph["n"]) * np.array(ph["h"])
    rows = np.arange(0, cfg["beam"]["n_protons"], 37)
    r = oracle.run(cfg, rows=rows, with_paths=True)
    for i, g in enumerate(rows):
        p = r["paths"][i]
        k = oracle.angle_of(int(g), cfg["beam"]["n_protons"], cfg["beam"]["n_angles"])
        c, s = oracle.angle(0.0, cfg["beam"]["dangle_deg"], k)
        Q = np.array([-p.t * s, p.t * c, 0.0])
        d = np.array([c, s, 0.0])
        chord, l_in, l_out = _box_chord(o, top, Q, d, 2)
        a, b = r["row_ptr"][i], r["row_ptr"][i + 1]
        assert abs(r["vals"][a:b].sum() - chord) <= 1e-12 * 300
        if chord > 0:
            pin, pout = Q + l_in * d, Q + l_out * d
            ii = [min(max(int(math.floor(pin[q] - o[q])), 0), 199) for q in range(2)]
            ee = [min(max(int(math.floor(pout[q] - o[q])), 0), 199) for q in range(2)]
            if r["margin"][i] > 1e-6:
                assert b - a == 1 + abs(ee[0] - ii[0]) + abs(ee[1] - ii[1])


@pytest.mark.parametrize("which", ["c1", "c2"])
def test_curved_rows_polyline_length(oracle, W, which):
    if which == "c1":
        cfg = W.scaled(W.c1(), n_protons=360 * 16)
    else:
        cfg = W.scaled(W.c2(), n_protons=90 * 40)
    ph = cfg["phantom"]
    dim = ph["dim"]
    o = np.array(_origin(ph))
    top = o + np.array(ph["n"]) * np.array(ph["h"])
    rows = np.arange(0, cfg["beam"]["n_protons"], 11)
    r = oracle.run(cfg, rows=rows, with_paths=True)
    n_curved = 0
    for i in range(len(rows)):
        p = r["paths"][i]
        a, b = r["row_ptr"][i], r["row_ptr"][i + 1]
        total = r["vals"][a:b].sum()
        if p.kind != oracle.KIND_CURVED:
            continue
        n_curved += 1
        P0, P1 = np.array(p.P0), np.array(p.P1)
        d0, d1 = np.array(p.d0), np.array(p.d1)
        _, l_in, _ = _box_chord(o, top, P0, d0, dim)
        _, _, l_out = _box_chord(o, top, P1, d1, dim)
        length = -l_in + l_out  # rays from the box to P0 and from P1 to the box
        S = [P0] + [np.array(oracle.hermite(P0, d0, P1, d1, p.L, j / p.n_samples))
                    for j in range(1, p.n_samples)] + [P1]
        length += sum(float(np.linalg.norm(S[j + 1] - S[j])) for j in range(len(S) - 1))
        assert abs(total - length) < 1e-9 * 300
    assert n_curved > len(rows) // 2


def test_scattering_distributions(oracle, W):
    """Entry angle, exit angle and lateral exit displacement have the Gaussian widths
    the beam asks for, in the ut plane (2D) and in both planes (3D)."""
    for cfg in (W.scaled(W.c1(), n_protons=360 * 40, sigma_in=0.02, sigma_out=0.03, sigma_lat=1.5),
                W.scaled(W.c2(), n_protons=90 * 160, sigma_in=0.02, sigma_out=0.03, sigma_lat=1.5)):
        bm = cfg["beam"]
        dim = cfg["phantom"]["dim"]
        r = oracle.run(cfg, with_paths=True)
        th_in, th_out, lat = [], [], []
        for i, g in enumerate(r["rows"]):
            p = r["paths"][i]
            if p.kind != oracle.KIND_CURVED:
                continue
            k = oracle.angle_of(int(g), bm["n_protons"], bm["n_angles"])
            c, s_ = oracle.angle(0.0, bm["dangle_deg"], k)
            u, t = np.array([c, s_, 0.0]), np.array([-s_, c, 0.0])
            d0, d1 = np.array(p.d0), np.array(p.d1)
            th_in.append(math.atan2(d0 @ t, d0 @ u))
            nt = t - (t @ d0) * d0
            nt /= np.linalg.norm(nt)
            th_out.append(math.atan2(d1 @ nt, d1 @ d0))
            Q = p.t * t + np.array([0.0, 0.0, p.v])
            # the exit lies on the displaced line Q + lat n_t (+ lat_v n_v) + l d0
            lat.append((np.array(p.P1) - Q) @ nt)
        th_in, th_out, lat = map(np.array, (th_in, th_out, lat))
        n = len(th_in)
        tol = lambda sig: 5 * sig / math.sqrt(2 * n)
        assert abs(th_in.std() - 0.02) < tol(0.02)
        assert abs(th_out.std() - 0.03) < tol(0.03) + 2e-4 * (dim == 3)
        if dim == 2:
            assert abs(lat.std() - 1.5) < tol(1.5)
            # the entry point is on the line t t_hat + l d0, the exit on the displaced one
        assert abs(th_in.mean()) < 5 * 0.02 / math.sqrt(n)


def test_zero_scatter_curved_equals_straight(oracle, W):
    base = W.scaled(W.c0(), n_protons=90 * 8)
    straight = oracle.run(base)
    cur = W.scaled(base, path="hermite", sigma_in=0.0, sigma_out=0.0, sigma_lat=0.0, step=0.25)
    curved = oracle.run(cur, with_paths=True)
    compared = 0
    for i in range(len(straight["rows"])):
        if straight["margin"][i] < 1e-6 or curved["margin"][i] < 1e-6:
            continue
        a, b = straight["row_ptr"][i], straight["row_ptr"][i + 1]
        c, d = curved["row_ptr"][i], curved["row_ptr"][i + 1]
        assert np.array_equal(straight["cols"][a:b], curved["cols"][c:d])
        assert np.allclose(straight["vals"][a:b], curved["vals"][c:d], atol=1e-9, rtol=0)
        assert abs(straight["b"][i] - curved["b"][i]) < 1e-9
        compared += 1
    assert compared > 0.9 * len(straight["rows"])


def test_reversed_line_reverses_row(oracle, W):
    ph = W.c0()["phantom"]
    rng = np.random.default_rng(8)
    for _ in range(40):
        phi = rng.uniform(0, 2 * math.pi)
        t = rng.uniform(-100, 100)
        c, s = math.cos(phi), math.sin(phi)
        Q = [-t * s, t * c, 0.0]
        f = oracle.trace_segments(ph, [Q], [[c, s, 0.0]], [-np.inf], [np.inf])
        r = oracle.trace_segments(ph, [Q], [[-c, -s, 0.0]], [-np.inf], [np.inf])
        if f["margin"] < 1e-6:
            continue
        assert np.array_equal(f["cols"], r["cols"][::-1])
        assert np.allclose(f["vals"], r["vals"][::-1], atol=1e-11, rtol=0)


def test_3d_cylinder_rows_are_2d_rows(oracle, W):
    regs = W.neo1_regions()
    b2 = W.beam(555, 12, 30.0, 12 * 40, (-100, 100))
    b3 = W.beam(555, 12, 30.0, 12 * 40, (-100, 100), (-20.0, 20.0))
    c2 = W.workload("2d", W.phantom(2, (100, 100), (2.0, 2.0), regs), b2)
    c3 = W.workload("3d", W.phantom(3, (100, 100, 20), (2.0, 2.0, 2.0), regs), b3)
    r2 = oracle.run(c2, with_paths=True)
    r3 = oracle.run(c3, with_paths=True)
    for i in range(len(r2["rows"])):
        assert r2["paths"][i].t == r3["paths"][i].t
        if r3["margin"][i] < 1e-6 or r2["margin"][i] < 1e-6:
            continue
        iz = int(math.floor((r3["paths"][i].v + 20.0) / 2.0))
        a, b = r2["row_ptr"][i], r2["row_ptr"][i + 1]
        c, d = r3["row_ptr"][i], r3["row_ptr"][i + 1]
        assert np.array_equal(r2["cols"][a:b] + iz * 100 * 100, r3["cols"][c:d])
        assert np.array_equal(r2["vals"][a:b], r3["vals"][c:d])
        assert abs(r2["b"][i] - r3["b"][i]) <= 1e-12 * max(1.0, r2["b"][i])


def test_wepl_homogeneous_grid(oracle, W):
    """Every voxel holds r, so b = r x chord of the line in the grid box."""
    r_val = 1.04
    regs = [{"shape": "ellipse", "center": [0.0, 0.0], "semi": [1e5, 1e5], "rsp": r_val}]
    cfg = W.workload("homog", W.phantom(2, (200, 200), (1.0, 1.0), regs),
                     W.beam(77, 90, 4.0, 90 * 32, (-140.0, 140.0)))
    r = oracle.run(cfg, with_paths=True)
    x = r["x"]
    assert np.all(x == np.float32(r_val))
    o = np.array([-100.0, -100.0, 0.0])
    top = np.array([100.0, 100.0, 0.0])
    for i, g in enumerate(r["rows"]):
        k = oracle.angle_of(int(g), 90 * 32, 90)
        c, s = oracle.angle(0.0, 4.0, k)
        t = r["paths"][i].t
        chord, *_ = _box_chord(o, top, np.array([-t * s, t * c, 0.0]), np.array([c, s, 0.0]), 2)
        assert abs(r["b"][i] - float(np.float32(r_val)) * chord) <= 1e-10 * max(chord, 1.0)
        if chord == 0.0:
            assert r["row_ptr"][i + 1] == r["row_ptr"][i]


def test_wepl_homogeneous_ellipse_bound(oracle, W):
    a_, b_, rv = 90.0, 70.0, 1.0
    regs = [{"shape": "ellipse", "center": [0.0, 0.0], "semi": [a_, b_], "rsp": rv}]
    cfg = W.workload("ell", W.phantom(2, (200, 200), (1.0, 1.0), regs),
                     W.beam(78, 90, 4.0, 90 * 32, (-100.0, 100.0)))
    r = oracle.run(cfg, with_paths=True)
    # voxels that can meet the boundary: centre within h sqrt(2)/2 of it
    n = 200
    cx = -100.0 + np.arange(n) + 0.5
    X, Y = np.meshgrid(cx, cx, indexing="xy")
    sq = np.sqrt((X / a_) ** 2 + (Y / b_) ** 2).reshape(-1)
    boundary = np.abs(sq - 1.0) <= (math.sqrt(2) / 2) / min(a_, b_) * 1.0001
    for i, g in enumerate(r["rows"]):
        k = oracle.angle_of(int(g), 90 * 32, 90)
        c, s = oracle.angle(0.0, 4.0, k)
        t = r["paths"][i].t
        R2 = a_ * a_ * s * s + b_ * b_ * c * c
        chord = 2 * a_ * b_ * math.sqrt(max(R2 - t * t, 0.0)) / R2
        lo, hi = r["row_ptr"][i], r["row_ptr"][i + 1]
        cols, vals = r["cols"][lo:hi], r["vals"][lo:hi]
        slack = rv * vals[boundary[cols]].sum()
        assert abs(r["b"][i] - rv * chord) <= slack + 1e-9


def test_noise_relative_sigma(oracle, W):
    cfg = W.scaled(W.c0(), n_protons=90 * 200, noise_rel=0.02)
    r = oracle.run(cfg)
    ok = r["b_clean"] > 1.0
    rel = r["b"][ok] / r["b_clean"][ok] - 1.0
    n = ok.sum()
    assert abs(rel.std() - 0.02) < 4 * 0.02 / math.sqrt(2 * n)
    assert abs(rel.mean()) < 4 * 0.02 / math.sqrt(n)
    assert np.all(r["b"][~(r["b_clean"] > 0)] == 0.0)


def test_grid_miss_rows_are_empty(oracle, W):
    cfg = W.scaled(W.c0(), n_protons=90 * 4, t_range=[150.0, 160.0])
    r = oracle.run(cfg, with_paths=True)
    # offsets of 150 mm miss the 200 mm box at 0 and 90 degrees, hit it near 45 degrees
    for i, g in enumerate(r["rows"]):
        k = oracle.angle_of(int(g), 90 * 4, 90)
        phi = math.radians(4.0 * k)
        reach = 100.0 * (abs(math.cos(phi)) + abs(math.sin(phi)))
        if abs(r["paths"][i].t) > reach + 1e-9:
            assert r["row_ptr"][i + 1] == r["row_ptr"][i]
            assert r["b"][i] == 0.0
            assert r["kind"][i] == oracle.KIND_MISS_GRID


def test_sizes_match_paper(oracle, W):
    """Printed sizes (tests/golden/paper_sizes.json): 32,000 pixels for the 2D example,
    6.4M voxels for the 3D volume, and roughly 100 GB of CSR for 64M histories on it."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_sizes.json")) as f:
        gold = json.load(f)
    assert oracle.n_voxels(W.c_paper()["phantom"]) == gold["pixels_2d_example"]["value"]
    assert oracle.n_voxels(W.c2()["phantom"]) == gold["voxels_3d_example"]["value"]
    # mean nnz of straight 3D rows on the 200x200x160 volume, sampled
    regs = W.neo_ellipsoid_regions()
    cfg = W.workload("s3", W.phantom(3, (200, 200, 160), (1, 1, 1), regs),
                     W.beam(9, 180, 2.0, 64_000_000, (-125.0, 125.0), (-80.0, 80.0)))
    r = oracle.run(cfg, rows=np.arange(0, 64_000_000, 64_000_000 // 2000))
    mean_nnz = len(r["cols"]) / len(r["rows"])
    rows = gold["csr_bytes_64M"]["rows"]
    est = rows * mean_nnz * (4 + 4) + 8 * (rows + 1)
    assert 0.5 * gold["csr_bytes_64M"]["value"] < est < 2.0 * gold["csr_bytes_64M"]["value"]
