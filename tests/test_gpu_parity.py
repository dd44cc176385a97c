"""Parity of the HIP path (through the C ABI) with the CPU oracle, on the GPU.

Full-size workloads are run in the same launch configuration as the benchmark and
compared on seeded row samples; the small workload is compared in full.  See
tests/parity.py for the bar.
"""
import math

import numpy as np
import pytest
import torch

from tests import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_2108_12369_amd import pct
    pct.lib()  # raises if libpct.so is missing: no silent fallback
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pct


def _h_min(cfg):
    ph = cfg["phantom"]
    return min(ph["h"][: ph["dim"]])


def _sample(n, k, seed):
    rng = np.random.default_rng(seed)
    if n <= k:
        return np.arange(n, dtype=np.int64)
    s = rng.choice(n, size=k, replace=False)
    s = np.union1d(s, [0, n - 1])
    return np.sort(s).astype(np.int64)


def _check(stats, max_excluded_frac=0.01):
    print({k: v for k, v in stats.items() if k != "failures"}, stats["failures"][:3], flush=True)
    assert stats["n_failures"] == 0, stats["failures"]
    assert stats["excluded"] <= max_excluded_frac * stats["rows"] + 2


def _run_compare(P, oracle, cfg, sample, precision="mixed", row_begin=0, row_count=None, max_excl=0.01):
    out = P.simulate(cfg, precision=precision, row_begin=row_begin, row_count=row_count)
    torch.cuda.synchronize()
    g = parity.gather_rows(out["row_ptr"], out["cols"], out["vals"], out["b"], sample)
    o = oracle.run(cfg, rows=sample + row_begin)
    st = parity.compare(g, o, _h_min(cfg), cfg["val_dtype"])
    _check(st, max_excl)
    return out, st


def test_phantom_build_bit_exact(P, oracle, W):
    for cfg in (W.c0(), W.c1(), W.c2(), W.c4(), W.c_paper()):
        x = P.phantom_build(cfg["phantom"]).cpu().numpy()
        xo = oracle.phantom_build(cfg["phantom"])
        assert x.shape == xo.shape
        assert np.array_equal(x, xo), (cfg["name"], int((x != xo).sum()))
    ph = W.phantom(2, (64, 48), (3.0, 3.5), W.neo1_regions(), voxelize="center")
    assert np.array_equal(P.phantom_build(ph).cpu().numpy(), oracle.phantom_build(ph))


def test_c0_full(P, oracle, W):
    cfg = W.c0()
    n = cfg["beam"]["n_protons"]
    out, st = _run_compare(P, oracle, cfg, np.arange(n, dtype=np.int64))
    assert out["nnz"] == st["nnz"] or st["excluded"] > 0


def test_c1_sampled(P, oracle, W):
    cfg = W.c1()
    _run_compare(P, oracle, cfg, _sample(cfg["beam"]["n_protons"], 100_000, 1))


def test_c2_sampled(P, oracle, W):
    cfg = W.c2()
    _run_compare(P, oracle, cfg, _sample(cfg["beam"]["n_protons"], 100_000, 2))


def test_c4_first_chunk_and_chunk_invariance(P, oracle, W):
    cfg = W.c4()
    chunk = cfg["chunk_rows"]
    out0, _ = _run_compare(P, oracle, cfg, _sample(chunk, 100_000, 4), row_count=chunk)
    rows0 = np.arange(chunk - 300, chunk, dtype=np.int64)
    a = parity.gather_rows(out0["row_ptr"], out0["cols"], out0["vals"], out0["b"], rows0)
    del out0
    # the same rows computed inside a chunk that starts elsewhere are bit-identical
    out1 = P.simulate(cfg, row_begin=chunk - 1000, row_count=1300)
    b = parity.gather_rows(out1["row_ptr"], out1["cols"], out1["vals"], out1["b"], rows0 - (chunk - 1000))
    for k in ("row_ptr", "cols", "vals", "b"):
        assert np.array_equal(a[k], b[k]), k


def test_ragged_and_offset_chunks(P, oracle, W):
    cfg = W.scaled(W.c1(), n_protons=360 * 40)
    for rb, rc in ((0, 1), (777, 1000), (360 * 40 - 300, 300), (5, 257)):
        _run_compare(P, oracle, cfg, np.arange(rc, dtype=np.int64), row_begin=rb, row_count=rc)


def test_edge_cases(P, oracle, W):
    # all rows miss the grid (offsets beyond the box diagonal)
    cfg = W.scaled(W.c0(), n_protons=90 * 4, t_range=[150.0, 160.0])
    out, st = _run_compare(P, oracle, cfg, np.arange(360, dtype=np.int64))
    # fewer protons than angles: most angles hold no proton
    cfg = W.scaled(W.c1(), n_protons=7)
    _run_compare(P, oracle, cfg, np.arange(7, dtype=np.int64))
    # tiny grids, 2D and 3D cylinder, center voxelisation, odd voxel sizes
    regs = W.neo1_regions()
    cfg = W.workload("tiny2d", W.phantom(2, (4, 3), (50.0, 70.0), regs, "center"),
                     W.beam(3, 7, 13.0, 700, (-120.0, 120.0), path="hermite", sigma_in=0.05,
                            sigma_out=0.05, sigma_lat=3.0, step=0.7, noise_rel=0.03))
    _run_compare(P, oracle, cfg, np.arange(700, dtype=np.int64))
    cfg = W.workload("cyl3d", W.phantom(3, (50, 40, 8), (4.0, 4.0, 5.0), regs),
                     W.beam(4, 30, 12.0, 3000, (-100.0, 100.0), (-25.0, 25.0), path="hermite",
                            sigma_in=0.01, sigma_out=0.02, sigma_lat=1.0, rho=0.5, noise_rel=0.01),
                     "f16")
    _run_compare(P, oracle, cfg, np.arange(3000, dtype=np.int64))
    # axis-aligned beams (0 and 90 degrees): paths parallel to voxel faces
    cfg = W.workload("axis", W.phantom(2, (100, 100), (2.0, 2.0), regs),
                     W.beam(5, 4, 90.0, 400, (-100.0, 100.0)))
    _run_compare(P, oracle, cfg, np.arange(400, dtype=np.int64), max_excl=0.05)


def test_empty_job(P, W):
    cfg = W.c0()
    x = P.phantom_build(cfg["phantom"])
    row_ptr = torch.full((1,), -7, dtype=torch.int64, device="cuda")
    js = P.JobSet()
    js.add(cfg["phantom"], cfg["beam"], x, row_ptr=row_ptr, row_begin=100, row_count=0)
    ws = torch.empty(P.workspace_bytes(js), dtype=torch.uint8, device="cuda")
    nnz = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    P.count_rows(js, ws, nnz)
    P.emit_csr(js, ws)
    assert int(nnz.item()) == 0 and int(row_ptr.item()) == 0
    assert P.device_status(ws) == P.PCT_OK


def test_wepl_matches_emit(P, W):
    cfg = W.scaled(W.c1(), n_protons=360 * 64)
    out = P.simulate(cfg)
    b2 = torch.empty_like(out["b"])
    js = P.JobSet()
    js.add(cfg["phantom"], cfg["beam"], out["x"], b=b2, val_dtype="f16")
    ws = torch.empty(P.workspace_bytes(js), dtype=torch.uint8, device="cuda")
    P.wepl(js, ws)
    assert torch.equal(out["b"], b2)


def test_wepl_matches_emit_2d_and_3d_batch(P, W):
    """pct_wepl on one batch of a 2D and a 3D job (both instances of the count kernel,
    counts not stored) gives the b that the emit of each job writes."""
    cfgs = [W.scaled(W.c1(), n_protons=360 * 16), W.scaled(W.c2(), n_protons=90 * 64)]
    outs = [P.simulate(c) for c in cfgs]
    js = P.JobSet()
    bs = []
    for c, o in zip(cfgs, outs):
        b2 = torch.full_like(o["b"], -1.0)
        bs.append(b2)
        js.add(c["phantom"], c["beam"], o["x"], b=b2, val_dtype=c["val_dtype"])
    ws = torch.empty(P.workspace_bytes(js), dtype=torch.uint8, device="cuda")
    P.wepl(js, ws)
    torch.cuda.synchronize()
    assert P.device_status(ws) == P.PCT_OK
    for o, b2 in zip(outs, bs):
        assert torch.equal(o["b"], b2)


@pytest.mark.parametrize("name", ["c1", "c2"])
def test_emit_without_b_writes_the_same_rows(P, W, name):
    """pct_emit_csr with b_dev NULL (the copy-out without the WEPL gathers) writes the same
    row_ptr, cols and vals, bit for bit, in 2D and in 3D."""
    cfg = W.scaled(W.by_name(name), n_protons=(360 if name == "c1" else 90) * 32)
    out = P.simulate(cfg)
    n, nnz_total = cfg["beam"]["n_protons"], out["nnz"]
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    cols = torch.full((nnz_total,), -7, dtype=torch.int32, device="cuda")
    vals = torch.zeros(nnz_total, dtype=out["vals"].dtype, device="cuda")
    js = P.JobSet()
    js.add(cfg["phantom"], cfg["beam"], out["x"], row_ptr=row_ptr, val_dtype=cfg["val_dtype"])
    ws = torch.empty(P.workspace_bytes(js), dtype=torch.uint8, device="cuda")
    nnz = torch.empty(1, dtype=torch.int64, device="cuda")
    P.count_rows(js, ws, nnz)
    js2 = P.JobSet()
    js2.add(cfg["phantom"], cfg["beam"], out["x"], row_ptr=row_ptr, cols=cols, vals=vals,
            nnz_capacity=nnz_total, val_dtype=cfg["val_dtype"])
    P.emit_csr(js2, ws)
    assert P.device_status(ws) == P.PCT_OK
    assert torch.equal(row_ptr, out["row_ptr"])
    assert torch.equal(cols, out["cols"])
    assert torch.equal(vals.view(torch.int16) if vals.dtype == torch.float16 else vals.view(torch.int32),
                       out["vals"].view(torch.int16) if vals.dtype == torch.float16 else out["vals"].view(torch.int32))


def test_capacity_overflow_is_reported_without_writes(P, W):
    cfg = W.scaled(W.c0(), n_protons=90 * 8)
    x = P.phantom_build(cfg["phantom"])
    n = cfg["beam"]["n_protons"]
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device="cuda")
    js = P.JobSet()
    js.add(cfg["phantom"], cfg["beam"], x, row_ptr=row_ptr)
    ws = torch.empty(P.workspace_bytes(js), dtype=torch.uint8, device="cuda")
    nnz = torch.empty(1, dtype=torch.int64, device="cuda")
    P.count_rows(js, ws, nnz)
    total = int(nnz.item())
    cap = total // 2
    guard = 4096
    cols = torch.full((cap + guard,), -5, dtype=torch.int32, device="cuda")
    vals = torch.full((cap + guard,), -5.0, dtype=torch.float32, device="cuda")
    b = torch.empty(n, dtype=torch.float32, device="cuda")
    js2 = P.JobSet()
    js2.add(cfg["phantom"], cfg["beam"], x, row_ptr=row_ptr, cols=cols, vals=vals, b=b, nnz_capacity=cap)
    P.emit_csr(js2, ws)
    assert P.device_status(ws) == P.PCT_ECAPACITY
    assert torch.all(cols[cap:] == -5) and torch.all(vals[cap:] == -5.0)
    # rows that fit are complete
    rp = row_ptr.cpu().numpy()
    last_ok = int(np.searchsorted(rp, cap, side="right")) - 1
    assert last_ok > 0 and torch.all(cols[: rp[last_ok]] >= 0)


def test_batched_jobs_match_single_and_oracle(P, oracle, W):
    jobs = W.c3_jobs()[:12]
    xs, rps, outs = [], [], []
    js = P.JobSet()
    for cfg in jobs:
        x = P.phantom_build(cfg["phantom"])
        n = cfg["beam"]["n_protons"]
        rp = torch.empty(n + 1, dtype=torch.int64, device="cuda")
        xs.append(x)
        rps.append(rp)
        js.add(cfg["phantom"], cfg["beam"], x, row_ptr=rp, val_dtype="f16")
    ws = torch.empty(P.workspace_bytes(js), dtype=torch.uint8, device="cuda")
    nnz = torch.empty(len(jobs), dtype=torch.int64, device="cuda")
    P.count_rows(js, ws, nnz)
    nnz_h = nnz.cpu().numpy()
    js2 = P.JobSet()
    for cfg, x, rp, nz in zip(jobs, xs, rps, nnz_h):
        n = cfg["beam"]["n_protons"]
        cols = torch.empty(max(int(nz), 1), dtype=torch.int32, device="cuda")
        vals = torch.empty(max(int(nz), 1), dtype=torch.float16, device="cuda")
        b = torch.empty(n, dtype=torch.float32, device="cuda")
        outs.append((cols, vals, b))
        js2.add(cfg["phantom"], cfg["beam"], x, row_ptr=rp, cols=cols, vals=vals, b=b,
                nnz_capacity=int(nz), val_dtype="f16")
    P.emit_csr(js2, ws)
    assert P.device_status(ws) == P.PCT_OK
    for j, cfg in enumerate(jobs):
        n = cfg["beam"]["n_protons"]
        sample = _sample(n, 400, 100 + j)
        cols, vals, b = outs[j]
        g = parity.gather_rows(rps[j], cols, vals, b, sample)
        o = oracle.run(cfg, rows=sample)
        _check(parity.compare(g, o, _h_min(cfg), "f16"))
        if j < 3:
            alone = P.simulate(cfg)
            assert torch.equal(alone["row_ptr"], rps[j])
            assert torch.equal(alone["cols"], cols[: alone["nnz"]])
            assert torch.equal(alone["vals"], vals[: alone["nnz"]])
            assert torch.equal(alone["b"], b)


def test_plain_f32_form_reported(P, oracle, W):
    """The plain FP32 form is a comparison baseline: its index mismatches are reported,
    not gated; its lengths and b stay close to the oracle."""
    cfg = W.scaled(W.c1(), n_protons=360 * 32)
    cfg["val_dtype"] = "f32"
    out = P.simulate(cfg, precision="plain_f32")
    sample = np.arange(cfg["beam"]["n_protons"], dtype=np.int64)
    g = parity.gather_rows(out["row_ptr"], out["cols"], out["vals"], out["b"], sample)
    o = oracle.run(cfg, rows=sample)
    st = parity.compare(g, o, _h_min(cfg), "f32")
    frac = st["n_failures"] / st["rows"]
    print("plain FP32: rows", st["rows"], "mismatching rows", st["n_failures"], f"({100 * frac:.2f}%)", flush=True)
    rel = np.abs(g["b"] - o["b"]) / np.maximum(o["b"], 1.0)
    assert np.median(rel) < 1e-4
