"""3D grids, and 2D grids with straight paths, on both sides of the limits of the bricked
copy of x (8 x 8 x 1 voxels per brick; x < 1024, y and z < 2048 voxels), and grids whose
sizes are not multiples of 8, against the oracle row by row: the staged packed
coordinates must give the columns, and the gathers from the copy the b, of the plain
layout.  The copy is refilled from x on every call.
"""
import numpy as np
import pytest
import torch

from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_2108_12369_amd import pct
    pct.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pct


# (grid, voxel sizes in mm): at and past each limit, and ragged in x and y
GRIDS = [((1024, 6, 5), (0.5, 4.0, 4.0)), ((1025, 6, 5), (0.5, 4.0, 4.0)),
         ((9, 2048, 4), (30.0, 0.25, 5.0)), ((9, 2049, 4), (30.0, 0.25, 5.0)),
         ((7, 6, 2048), (40.0, 40.0, 0.05)), ((7, 6, 2049), (40.0, 40.0, 0.05)),
         ((13, 11, 7), (9.0, 11.0, 6.0))]


def _cfg(W, n, h, seed):
    ext = [n[d] * h[d] for d in range(3)]
    regs = [W._e((0, 0, 0), (0.4 * ext[0], 0.4 * ext[1], 0.4 * ext[2]), 1.0, "ellipsoid"),
            W._e((0.1 * ext[0], 0, 0), (0.15 * ext[0], 0.2 * ext[1], 0.2 * ext[2]), 1.6, "ellipsoid")]
    ph = W.phantom(3, n, h, regs)
    span = min(ext[0], ext[1])
    bm = W.beam(seed, 12, 15.0, 600, (-0.45 * span, 0.45 * span), (-0.4 * ext[2], 0.4 * ext[2]),
                path="hermite", sigma_in=0.01, sigma_out=0.01, sigma_lat=0.2, step=0.5, noise_rel=0.01)
    return W.workload(f"bricks-{n[0]}x{n[1]}x{n[2]}", ph, bm, "f16")


@pytest.mark.parametrize("grid", GRIDS, ids=[f"{g[0][0]}x{g[0][1]}x{g[0][2]}" for g in GRIDS])
def test_bricked_gathers_match_the_oracle(P, oracle, W, grid):
    n, h = grid
    cfg = _cfg(W, n, h, 7000 + sum(n))
    rows = np.arange(cfg["beam"]["n_protons"], dtype=np.int64)
    print(cfg["name"], flush=True)
    out = P.simulate(cfg)
    torch.cuda.synchronize()
    g = parity.gather_rows(out["row_ptr"], out["cols"], out["vals"], out["b"], rows)
    o = oracle.run(cfg, rows=rows)
    st = parity.compare(g, o, min(h), "f16")
    print({k: v for k, v in st.items() if k != "failures"}, st["failures"][:3], flush=True)
    assert st["n_failures"] == 0, st["failures"]
    assert st["nnz"] > 10 * len(rows)
    assert st["excluded"] <= 0.02 * st["rows"] + 3


# 2D grids with straight paths (voxel sizes in mm): at and past each limit, and ragged
GRIDS_2D = [((1024, 7), (0.2, 30.0)), ((1025, 7), (0.2, 30.0)), ((9, 2048), (25.0, 0.1)),
            ((9, 2049), (25.0, 0.1)), ((13, 11), (16.0, 17.0)), ((300, 201), (0.7, 1.0))]


def _cfg2(W, n, h, seed, path="straight"):
    ext = [n[0] * h[0], n[1] * h[1]]
    regs = [W._e((0, 0), (0.4 * ext[0], 0.4 * ext[1]), 1.0),
            W._e((0.1 * ext[0], 0), (0.15 * ext[0], 0.2 * ext[1]), 1.6)]
    ph = W.phantom(2, n, h, regs)
    span = min(ext[0], ext[1])
    extra = dict(path="hermite", sigma_in=0.01, sigma_out=0.01, sigma_lat=0.2, step=0.5) if path != "straight" else {}
    bm = W.beam(seed, 12, 15.0, 600, (-0.45 * span, 0.45 * span), noise_rel=0.01, **extra)
    return W.workload(f"bricks2d-{n[0]}x{n[1]}-{path}", ph, bm, "f16")


@pytest.mark.parametrize("grid", GRIDS_2D, ids=[f"{g[0][0]}x{g[0][1]}" for g in GRIDS_2D])
def test_bricked_gathers_2d_straight_match_the_oracle(P, oracle, W, grid):
    n, h = grid
    cfg = _cfg2(W, n, h, 7100 + sum(n))
    rows = np.arange(cfg["beam"]["n_protons"], dtype=np.int64)
    print(cfg["name"], flush=True)
    out = P.simulate(cfg)
    torch.cuda.synchronize()
    g = parity.gather_rows(out["row_ptr"], out["cols"], out["vals"], out["b"], rows)
    o = oracle.run(cfg, rows=rows)
    st = parity.compare(g, o, min(h), "f16")
    print({k: v for k, v in st.items() if k != "failures"}, st["failures"][:3], flush=True)
    assert st["n_failures"] == 0, st["failures"]
    assert st["nnz"] > 5 * len(rows)
    assert st["excluded"] <= 0.02 * st["rows"] + 3


def test_bricked_and_plain_2d_jobs_in_one_call(P, oracle, W):
    """A straight 2D job (bricked) and a curved one (plain x) in one call: each against
    the oracle."""
    cfgs = [_cfg2(W, (70, 60), (2.5, 3.0), 7201), _cfg2(W, (70, 60), (2.5, 3.0), 7202, path="hermite")]
    xs = [P.phantom_build(c["phantom"]) for c in cfgs]
    rps = [torch.empty(c["beam"]["n_protons"] + 1, dtype=torch.int64, device="cuda") for c in cfgs]
    js = P.JobSet()
    for c, x, rp in zip(cfgs, xs, rps):
        js.add(c["phantom"], c["beam"], x, row_ptr=rp, val_dtype="f16")
    ws = torch.empty(P.workspace_bytes(js), dtype=torch.uint8, device="cuda")
    nnz = torch.empty(len(cfgs), dtype=torch.int64, device="cuda")
    P.count_rows(js, ws, nnz)
    caps = [int(v) for v in nnz.cpu()]
    outs = []
    js2 = P.JobSet()
    for c, x, rp, cap in zip(cfgs, xs, rps, caps):
        cols = torch.empty(cap, dtype=torch.int32, device="cuda")
        vals = torch.empty(cap, dtype=torch.float16, device="cuda")
        b = torch.empty(c["beam"]["n_protons"], dtype=torch.float32, device="cuda")
        js2.add(c["phantom"], c["beam"], x, row_ptr=rp, cols=cols, vals=vals, b=b, nnz_capacity=cap, val_dtype="f16")
        outs.append((rp, cols, vals, b))
    P.emit_csr(js2, ws)
    torch.cuda.synchronize()
    assert P.device_status(ws) == P.PCT_OK
    for c, (rp, cols, vals, b) in zip(cfgs, outs):
        rows = np.arange(c["beam"]["n_protons"], dtype=np.int64)
        g = parity.gather_rows(rp, cols, vals, b, rows)
        st = parity.compare(g, oracle.run(c, rows=rows), 2.5, "f16")
        assert st["n_failures"] == 0, (c["name"], st["failures"][:3])
        assert st["nnz"] > 5 * len(rows)


def test_bricked_copy_is_refilled_on_every_call(P, W):
    """The same workspace and jobs, x doubled in place between two emit calls: b doubles
    exactly (a factor of 2 scales every product and sum exactly), for a bricked 3D job."""
    cfg = _cfg(W, (13, 11, 7), (9.0, 11.0, 6.0), 7031)
    ph, bm = cfg["phantom"], cfg["beam"]
    x = P.phantom_build(ph)
    rp = torch.empty(bm["n_protons"] + 1, dtype=torch.int64, device="cuda")
    js = P.JobSet()
    js.add(ph, bm, x, row_ptr=rp, val_dtype="f16")
    ws = torch.empty(P.workspace_bytes(js), dtype=torch.uint8, device="cuda")
    nnz = torch.empty(1, dtype=torch.int64, device="cuda")
    P.count_rows(js, ws, nnz)
    cap = int(nnz.item())
    cols = torch.empty(cap, dtype=torch.int32, device="cuda")
    vals = torch.empty(cap, dtype=torch.float16, device="cuda")
    b1 = torch.empty(bm["n_protons"], dtype=torch.float32, device="cuda")
    b2 = torch.empty_like(b1)
    for b in (b1, b2):
        js2 = P.JobSet()
        js2.add(ph, bm, x, row_ptr=rp, cols=cols, vals=vals, b=b, nnz_capacity=cap, val_dtype="f16")
        P.emit_csr(js2, ws)
        x.mul_(2.0)
    torch.cuda.synchronize()
    assert P.device_status(ws) == P.PCT_OK
    assert float(b1.abs().max()) > 0
    assert torch.equal(b2, 2.0 * b1)
