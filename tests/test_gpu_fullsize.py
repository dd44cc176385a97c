"""Parity at the benchmark's full sizes, on the GPU (see tests/parity.py for the bar).

  * c1 compared in full: every one of its 2,949,120 rows against the oracle;
  * the batched workload exactly as the benchmark times it -- the 64 uneven jobs captured
    with their phantom builds in one HIP graph and replayed -- on seeded rows spread over
    every job, each job's first and last rows included;
  * rows longer than the LDS slice of a wavefront (more than 1023 entries), which the
    count pass hands to the per-lane walk, and rows of 979 to 1023 entries, which reach
    into the slots that hold the wave's copy of the next row's description: straight and
    curved, FP32 and FP16, alone and inside a batch with a job whose rows are short.

The oracle runs on a thread pool: each call is one C call that releases the GIL.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

from tests import parity

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def P():
    from paper_2108_12369_amd import pct
    pct.lib()  # raises if libpct.so is missing: no silent fallback
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pct.set_launch_config()
    yield pct
    pct.set_launch_config()


def _h_min(cfg):
    ph = cfg["phantom"]
    return min(ph["h"][: ph["dim"]])


def _oracle_rows(oracle, cfg, rows, x, parts):
    """The oracle on `rows`, split over the thread pool; results merged in order."""
    chunks = [c for c in np.array_split(rows, parts) if len(c)]
    with ThreadPoolExecutor(THREADS) as ex:
        res = list(ex.map(lambda c: oracle.run(cfg, rows=c, x=x), chunks))
    out = {"rows": rows, "margin": np.concatenate([r["margin"] for r in res]),
           "b": np.concatenate([r["b"] for r in res]),
           "cols": np.concatenate([r["cols"] for r in res]), "vals": np.concatenate([r["vals"] for r in res])}
    rp = [np.zeros(1, np.int64)]
    base = 0
    for r in res:
        rp.append(r["row_ptr"][1:] + base)
        base += int(r["row_ptr"][-1])
    out["row_ptr"] = np.concatenate(rp)
    return out


def _check(st, max_excl=0.01):
    print({k: v for k, v in st.items() if k != "failures"}, st["failures"][:3], flush=True)
    assert st["n_failures"] == 0, st["failures"]
    assert st["excluded"] <= max_excl * st["rows"] + 2


def test_c1_every_row(P, oracle, W):
    cfg = W.c1()
    n = cfg["beam"]["n_protons"]
    out = P.simulate(cfg)
    torch.cuda.synchronize()
    x = oracle.phantom_build(cfg["phantom"])
    tot = {"rows": 0, "excluded": 0, "nnz": 0}
    step = 245_760   # 30 angles of 8192 rows
    for r0 in range(0, n, step):
        rows = np.arange(r0, min(n, r0 + step), dtype=np.int64)
        g = parity.gather_rows(out["row_ptr"], out["cols"], out["vals"], out["b"], rows)
        o = _oracle_rows(oracle, cfg, rows, x, 4 * THREADS)
        st = parity.compare(g, o, _h_min(cfg), "f16")
        assert st["n_failures"] == 0, (r0, st["failures"])
        for k in tot:
            tot[k] += st[k]
    print("c1 in full:", tot, flush=True)
    assert tot["rows"] == n
    assert tot["excluded"] <= 0.01 * n


def test_c3_graph_as_benchmarked(P, oracle, W):
    """The 64-job batch in one graph (phantom builds, count, scan, emit), replayed twice:
    both replays write the same CSR, and >= 100,000 seeded rows over all jobs (each job's
    first and last rows among them) match the oracle."""
    jobs = W.c3_jobs()
    xs = [torch.empty(P.n_voxels(c["phantom"]), dtype=torch.float32, device="cuda") for c in jobs]
    rps = [torch.empty(c["beam"]["n_protons"] + 1, dtype=torch.int64, device="cuda") for c in jobs]
    for c, x in zip(jobs, xs):
        P.phantom_build(c["phantom"], x)
    js = P.JobSet()
    for c, x, rp in zip(jobs, xs, rps):
        js.add(c["phantom"], c["beam"], x, row_ptr=rp, val_dtype="f16")
    ws = torch.empty(P.workspace_bytes(js), dtype=torch.uint8, device="cuda")
    nnz = torch.empty(len(jobs), dtype=torch.int64, device="cuda")
    P.count_rows(js, ws, nnz)
    caps = [int(v) for v in nnz.cpu().numpy()]
    cols = [torch.empty(max(v, 1), dtype=torch.int32, device="cuda") for v in caps]
    vals = [torch.empty(max(v, 1), dtype=torch.float16, device="cuda") for v in caps]
    bs = [torch.empty(c["beam"]["n_protons"], dtype=torch.float32, device="cuda") for c in jobs]
    js2 = P.JobSet()
    for j, c in enumerate(jobs):
        js2.add(c["phantom"], c["beam"], xs[j], row_ptr=rps[j], cols=cols[j], vals=vals[j], b=bs[j],
                nnz_capacity=caps[j], val_dtype="f16")
    for x in xs:
        x.zero_()   # the graph's own phantom builds must write x
    graph = P.Graph(js2, ws, nnz, build_x=True)
    graph.launch()
    torch.cuda.synchronize()
    assert P.device_status(ws) == P.PCT_OK
    sums = [int(c.sum(dtype=torch.int64).item()) for c in cols]
    vsum = [float(v.float().sum().item()) for v in vals]
    graph.launch()
    torch.cuda.synchronize()
    assert P.device_status(ws) == P.PCT_OK
    assert sums == [int(c.sum(dtype=torch.int64).item()) for c in cols]
    assert vsum == [float(v.float().sum().item()) for v in vals]
    graph.close()
    total = sum(c["beam"]["n_protons"] for c in jobs)
    rng = np.random.default_rng(12372)
    n_rows = 0
    for j, c in enumerate(jobs):
        n = c["beam"]["n_protons"]
        k = max(400, int(round(100_000 * n / total)))
        rows = np.union1d(rng.choice(n, size=min(k, n), replace=False), [0, n - 1]).astype(np.int64)
        g = parity.gather_rows(rps[j], cols[j], vals[j], bs[j], rows)
        o = _oracle_rows(oracle, c, rows, oracle.phantom_build(c["phantom"]), THREADS)
        st = parity.compare(g, o, _h_min(c), "f16")
        print(c["name"], c["phantom"]["dim"], c["beam"]["path"], {k2: v for k2, v in st.items() if k2 != "failures"},
              flush=True)
        assert st["n_failures"] == 0, (c["name"], st["failures"])
        assert st["excluded"] <= 0.01 * st["rows"] + 2
        n_rows += len(rows)
    assert n_rows >= 100_000


def _long_rows_cfg(W, path, val_dtype):
    """768 x 768 pixels of 0.25 mm (192 mm field), the NEO 1 phantom, beams at 45 and 135
    degrees through the middle: the rows cross about 1,500 faces."""
    ph = W.phantom(2, (768, 768), (0.25, 0.25), W.neo1_regions())
    extra = dict(path="hermite", sigma_in=0.01, sigma_out=0.01, sigma_lat=1.0, step=0.25) if path == "hermite" else {}
    bm = W.beam(777, 2, 90.0, 2000, (-30.0, 30.0), angle0_deg=45.0, noise_rel=0.01, **extra)
    return W.workload(f"long-rows-{path}-{val_dtype}", ph, bm, val_dtype)


@pytest.mark.parametrize("path", ["straight", "hermite"])
@pytest.mark.parametrize("val_dtype", ["f32", "f16"])
def test_rows_longer_than_the_lds_slice(P, oracle, W, path, val_dtype):
    cfg = _long_rows_cfg(W, path, val_dtype)
    out = P.simulate(cfg)
    rows = np.arange(cfg["beam"]["n_protons"], dtype=np.int64)
    g = parity.gather_rows(out["row_ptr"], out["cols"], out["vals"], out["b"], rows)
    o = _oracle_rows(oracle, cfg, rows, oracle.phantom_build(cfg["phantom"]), THREADS)
    lens = np.diff(o["row_ptr"])
    long_rows = int((lens > 1023).sum())
    print("rows over 1023 entries:", long_rows, "rows of 979-1023:", int(((lens > 978) & (lens <= 1023)).sum()), "longest", int(np.diff(o["row_ptr"]).max()), flush=True)
    assert long_rows > 1000
    _check(parity.compare(g, o, _h_min(cfg), val_dtype))


def _mid_rows_cfg(W, path, val_dtype):
    """512 x 512 pixels of 0.375 mm (192 mm field), beams at 45 and 135 degrees with random
    offsets in [-30, 30) mm: rows of about 800 to 1023 entries in random order, a fifth of
    them over 978, whose entries overwrite the slots of the wave's copy of the next row's
    description."""
    ph = W.phantom(2, (512, 512), (0.375, 0.375), W.neo1_regions())
    extra = dict(path="hermite", sigma_in=0.01, sigma_out=0.01, sigma_lat=1.0, step=0.375) if path == "hermite" else {}
    bm = W.beam(778, 2, 90.0, 2000, (-30.0, 30.0), angle0_deg=45.0, noise_rel=0.01, **extra)
    return W.workload(f"mid-rows-{path}-{val_dtype}", ph, bm, val_dtype)


@pytest.mark.parametrize("path,val_dtype", [("straight", "f16"), ("hermite", "f16"), ("straight", "f32")])
def test_rows_reaching_into_the_description_copy(P, oracle, W, path, val_dtype):
    cfg = _mid_rows_cfg(W, path, val_dtype)
    out = P.simulate(cfg)
    rows = np.arange(cfg["beam"]["n_protons"], dtype=np.int64)
    g = parity.gather_rows(out["row_ptr"], out["cols"], out["vals"], out["b"], rows)
    o = _oracle_rows(oracle, cfg, rows, oracle.phantom_build(cfg["phantom"]), THREADS)
    lens = np.diff(o["row_ptr"])
    mid = int(((lens > 978) & (lens <= 1023)).sum())
    print("rows of 979-1023 entries:", mid, "longest", int(lens.max()), flush=True)
    assert mid > 200 and int((lens <= 978).sum()) > 1000 and int(lens.max()) <= 1023
    _check(parity.compare(g, o, _h_min(cfg), val_dtype))


def test_long_rows_inside_a_batch(P, oracle, W):
    """The long-row job between two jobs of short rows in one batch: every job's rows as
    when it runs alone, and as the oracle gives them."""
    cfgs = [W.scaled(W.c3_jobs()[1], n_protons=3000), _long_rows_cfg(W, "hermite", "f16"),
            W.scaled(W.c1(), n_protons=360 * 8)]
    xs = [P.phantom_build(c["phantom"]) for c in cfgs]
    rps = [torch.empty(c["beam"]["n_protons"] + 1, dtype=torch.int64, device="cuda") for c in cfgs]
    js = P.JobSet()
    for c, x, rp in zip(cfgs, xs, rps):
        js.add(c["phantom"], c["beam"], x, row_ptr=rp, val_dtype="f16")
    ws = torch.empty(P.workspace_bytes(js), dtype=torch.uint8, device="cuda")
    nnz = torch.empty(len(cfgs), dtype=torch.int64, device="cuda")
    P.count_rows(js, ws, nnz)
    caps = [int(v) for v in nnz.cpu().numpy()]
    outs = []
    js2 = P.JobSet()
    for j, c in enumerate(cfgs):
        o = (torch.empty(max(caps[j], 1), dtype=torch.int32, device="cuda"),
             torch.empty(max(caps[j], 1), dtype=torch.float16, device="cuda"),
             torch.empty(c["beam"]["n_protons"], dtype=torch.float32, device="cuda"))
        outs.append(o)
        js2.add(c["phantom"], c["beam"], xs[j], row_ptr=rps[j], cols=o[0], vals=o[1], b=o[2],
                nnz_capacity=caps[j], val_dtype="f16")
    P.emit_csr(js2, ws)
    assert P.device_status(ws) == P.PCT_OK
    for j, c in enumerate(cfgs):
        alone = P.simulate(c)
        assert torch.equal(alone["row_ptr"], rps[j])
        assert torch.equal(alone["cols"], outs[j][0][: alone["nnz"]])
        assert torch.equal(alone["vals"].view(torch.int16), outs[j][1][: alone["nnz"]].view(torch.int16))
        assert torch.equal(alone["b"], outs[j][2])
        rows = np.arange(c["beam"]["n_protons"], dtype=np.int64)
        g = parity.gather_rows(rps[j], outs[j][0], outs[j][1], outs[j][2], rows)
        o = _oracle_rows(oracle, c, rows, oracle.phantom_build(c["phantom"]), THREADS)
        _check(parity.compare(g, o, _h_min(c), "f16"))
