"""Batched launches on the GPU: launch configurations, the autotuner and graph replay.

Every row is computed the same way whatever the order or grouping of the rows, so all
launch configurations must give bit-identical outputs; a replayed graph must write what
the eager calls write.
"""
import time

import numpy as np
import pytest
import torch

from tests import parity

pytestmark = pytest.mark.gpu

# every configuration the autotuner tries: rows per wave x order x (0: a grid over the
# tiles, 4: a persistent grid of 4 blocks per CU taking tiles from a queue)
CONFIGS = [(rpw, order, bpc) for bpc in (0, 4) for order in ("given", "lpt") for rpw in (16, 32, 64)]


@pytest.fixture(scope="module")
def P():
    from paper_2108_12369_amd import pct
    pct.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    pct.set_launch_config()
    yield pct
    pct.set_launch_config()


def _jobs(W, k, rows):
    """k jobs of the uneven batched workload, each cut to at most `rows` protons."""
    out = []
    for cfg in W.c3_jobs()[:k]:
        n = min(cfg["beam"]["n_protons"], rows)
        out.append(W.scaled(cfg, n_protons=n))
    return out


class Batch:
    """Device buffers of a job set, sized by a first count."""

    def __init__(self, P, cfgs):
        self.P, self.cfgs = P, cfgs
        self.xs = [P.phantom_build(c["phantom"]) for c in cfgs]
        self.rps = [torch.empty(c["beam"]["n_protons"] + 1, dtype=torch.int64, device="cuda") for c in cfgs]
        js = P.JobSet()
        for c, x, rp in zip(cfgs, self.xs, self.rps):
            js.add(c["phantom"], c["beam"], x, row_ptr=rp, val_dtype="f16")
        self.ws = torch.empty(P.workspace_bytes(js), dtype=torch.uint8, device="cuda")
        self.nnz = torch.empty(len(cfgs), dtype=torch.int64, device="cuda")
        P.count_rows(js, self.ws, self.nnz)
        nz = self.nnz.cpu().numpy()
        self.cols = [torch.empty(max(int(v), 1), dtype=torch.int32, device="cuda") for v in nz]
        self.vals = [torch.empty(max(int(v), 1), dtype=torch.float16, device="cuda") for v in nz]
        self.bs = [torch.empty(max(c["beam"]["n_protons"], 1), dtype=torch.float32, device="cuda") for c in cfgs]
        self.cap = [int(v) for v in nz]
        self.js = P.JobSet()
        for j, c in enumerate(cfgs):
            self.js.add(c["phantom"], c["beam"], self.xs[j], row_ptr=self.rps[j], cols=self.cols[j],
                        vals=self.vals[j], b=self.bs[j], nnz_capacity=self.cap[j], val_dtype="f16")

    def run(self):
        self.P.count_rows(self.js, self.ws, self.nnz)
        self.P.emit_csr(self.js, self.ws)
        assert self.P.device_status(self.ws) == self.P.PCT_OK

    def clear(self):
        for t in self.rps + self.cols + self.bs + self.xs:
            t.fill_(-1)
        for t in self.vals:
            t.fill_(-1.0)
        self.nnz.fill_(-1)

    def snapshot(self):
        torch.cuda.synchronize()
        return {"nnz": self.nnz.clone(), "x": [t.clone() for t in self.xs], "rp": [t.clone() for t in self.rps],
                "cols": [c[:n].clone() for c, n in zip(self.cols, self.cap)],
                "vals": [v[:n].clone() for v, n in zip(self.vals, self.cap)], "b": [t.clone() for t in self.bs]}


def _equal(a, b):
    assert torch.equal(a["nnz"], b["nnz"])
    for k in ("x", "rp", "cols", "vals", "b"):
        for u, v in zip(a[k], b[k]):
            assert torch.equal(u, v), k


def test_launch_configs_give_identical_outputs(P, oracle, W):
    cfgs = _jobs(W, 10, 6000)
    B = Batch(P, cfgs)
    ref = None
    for rpw, order, bpc in CONFIGS + [(64, "lpt", 1), (32, "given", 2), (16, "lpt", 8)]:
        P.set_launch_config(rpw, order, bpc)
        assert P.get_launch_config() == {"rows_per_wave": rpw, "order": order, "blocks_per_cu": bpc}
        B.clear()
        for c, x in zip(cfgs, B.xs):
            P.phantom_build(c["phantom"], x)
        B.run()
        snap = B.snapshot()
        if ref is None:
            ref = snap
        else:
            _equal(ref, snap)
    P.set_launch_config()
    # per-job totals are reported in the order of the job array
    for j in range(len(cfgs)):
        assert int(ref["nnz"][j]) == int(ref["rp"][j][-1])
    for j, c in enumerate(cfgs[:4]):
        n = c["beam"]["n_protons"]
        rows = np.unique(np.linspace(0, n - 1, 200).astype(np.int64))
        g = parity.gather_rows(B.rps[j], B.cols[j], B.vals[j], B.bs[j], rows)
        o = oracle.run(c, rows=rows)
        st = parity.compare(g, o, min(c["phantom"]["h"][: c["phantom"]["dim"]]), "f16")
        assert st["n_failures"] == 0, st["failures"]


def test_bad_launch_config_rejected(P):
    from paper_2108_12369_amd.pct import PctError
    with pytest.raises(PctError):
        P.set_launch_config(48, "lpt")
    assert P.get_launch_config()["rows_per_wave"] in (16, 32, 64)


@pytest.mark.parametrize("bpc", [0, 4])
def test_graph_replays_match_eager(P, W, bpc):
    """Replays of a captured batch match the eager calls, with the grid over the tiles and
    with the persistent grid (whose tile counters a kernel of the graph resets)."""
    P.set_launch_config(64, "lpt", bpc)
    cfgs = _jobs(W, 6, 4000)
    B = Batch(P, cfgs)
    B.run()
    eager = B.snapshot()
    G = P.Graph(B.js, B.ws, B.nnz, build_x=True)
    other = Batch(P, _jobs(W, 2, 1000)[::-1])
    for rep in range(3):
        B.clear()
        # eager work of the program between replays
        a = torch.randn(256, 256, device="cuda")
        (a @ a).sum().item()
        other.run()
        G.launch()
        torch.cuda.synchronize()
        assert P.device_status(B.ws) == P.PCT_OK
        _equal(eager, B.snapshot())
    G.close()
    P.set_launch_config()


def test_autotune_sets_a_valid_config_and_keeps_outputs(P, W):
    cfgs = _jobs(W, 8, 5000)
    B = Batch(P, cfgs)
    B.run()
    eager = B.snapshot()
    B.clear()
    for c, x in zip(cfgs, B.xs):
        P.phantom_build(c["phantom"], x)
    best = P.autotune(B.js, B.ws, B.nnz)
    assert (best["rows_per_wave"], best["order"], best["blocks_per_cu"]) in CONFIGS
    assert P.get_launch_config() == best
    assert P.device_status(B.ws) == P.PCT_OK
    _equal(eager, B.snapshot())
    P.set_launch_config()


def _chunked(P, W, n_chunks=4, rows=20_000):
    """A 3D curved workload (the head-scale geometry) cut into row chunks, each chunk a
    job set of one job with outputs of its own, sized by a first count."""
    cfg = W.scaled(W.c4(), n_protons=n_chunks * rows)
    x = P.phantom_build(cfg["phantom"])
    sets, outs = [], []
    probe = P.JobSet()
    rps = [torch.empty(rows + 1, dtype=torch.int64, device="cuda") for _ in range(n_chunks)]
    for k in range(n_chunks):
        probe.add(cfg["phantom"], cfg["beam"], x, row_ptr=rps[k], val_dtype="f16", row_begin=k * rows,
                  row_count=rows)
    ws = torch.empty(P.workspace_bytes(probe), dtype=torch.uint8, device="cuda")
    nnz = torch.empty(n_chunks, dtype=torch.int64, device="cuda")
    P.count_rows(probe, ws, nnz)
    caps = [int(v) for v in nnz.cpu().numpy()]
    for k in range(n_chunks):
        o = (torch.empty(caps[k], dtype=torch.int32, device="cuda"),
             torch.empty(caps[k], dtype=torch.float16, device="cuda"),
             torch.empty(rows, dtype=torch.float32, device="cuda"))
        outs.append(o)
        js = P.JobSet()
        js.add(cfg["phantom"], cfg["beam"], x, row_ptr=rps[k], cols=o[0], vals=o[1], b=o[2], nnz_capacity=caps[k],
               val_dtype="f16", row_begin=k * rows, row_count=rows)
        sets.append(js)
    return cfg, x, sets, rps, outs, caps, ws


def test_graph_of_chunk_sets_matches_eager(P, W):
    """One graph for a chunk loop (count then emit per chunk, the phantom built once):
    every chunk's outputs and count equal the eager calls', on every replay."""
    cfg, x, sets, rps, outs, caps, ws = _chunked(P, W)
    nnz1 = torch.empty(1, dtype=torch.int64, device="cuda")
    for js in sets:
        P.count_rows(js, ws, nnz1)
        P.emit_csr(js, ws)
    assert P.device_status(ws) == P.PCT_OK
    eager = [[t.clone() for t in (rp,) + o] for rp, o in zip(rps, outs)]
    nnz = torch.empty(len(sets), dtype=torch.int64, device="cuda")
    G = P.Graph(sets, ws, nnz, build_x=True)
    for rep in range(3):
        for rp, o in zip(rps, outs):
            for t in (rp,) + o:
                t.fill_(-1)
        x.zero_()   # the graph's phantom build must write x
        G.launch()
        torch.cuda.synchronize()
        assert P.device_status(ws) == P.PCT_OK
        assert [int(v) for v in nnz.cpu().numpy()] == caps
        for e, rp, o in zip(eager, rps, outs):
            for a, b in zip(e, (rp,) + o):
                assert torch.equal(a.view(torch.int16) if a.dtype == torch.float16 else a,
                                   b.view(torch.int16) if b.dtype == torch.float16 else b)
    G.close()


def test_graph_of_sets_keeps_an_early_capacity_error(P, W):
    """A chunk whose capacity is too small sets PCT_ECAPACITY, and the later chunks' count
    passes do not clear it."""
    cfg, x, sets, rps, outs, caps, ws = _chunked(P, W, n_chunks=3, rows=5000)
    rows = 5000
    small = P.JobSet()
    small.add(cfg["phantom"], cfg["beam"], x, row_ptr=rps[0], cols=outs[0][0], vals=outs[0][1], b=outs[0][2],
              nnz_capacity=caps[0] // 2, val_dtype="f16", row_begin=0, row_count=rows)
    nnz = torch.empty(3, dtype=torch.int64, device="cuda")
    G = P.Graph([small] + sets[1:], ws, nnz, build_x=False)
    G.launch()
    assert P.device_status(ws) == P.PCT_ECAPACITY
    G.close()


def test_autotune_cache(P, W):
    """The autotuner's result is cached per shape of batch: a second call takes it without
    timing, with the same outputs; another shape is not found; clearing forgets it."""
    P.autotune_cache_clear()
    cfgs = _jobs(W, 6, 3000)
    B = Batch(P, cfgs)
    B.run()
    eager = B.snapshot()
    assert P.autotune_cached(B.js) is None
    best = P.autotune(B.js, B.ws, B.nnz)
    assert P.autotune_cached(B.js) == best
    P.set_launch_config()
    B.clear()
    for c, x in zip(cfgs, B.xs):
        P.phantom_build(c["phantom"], x)
    t0 = time.perf_counter()
    again = P.autotune(B.js, B.ws, B.nnz)
    dt = time.perf_counter() - t0
    assert again == best and P.get_launch_config() == best
    assert P.device_status(B.ws) == P.PCT_OK
    _equal(eager, B.snapshot())
    print("cached autotune call:", dt, "s", flush=True)
    other = Batch(P, _jobs(W, 3, 3000))
    assert P.autotune_cached(other.js) is None
    P.autotune_cache_clear()
    assert P.autotune_cached(B.js) is None
    P.set_launch_config()


@pytest.mark.parametrize("seed", list(range(24)))
def test_random_batch_matches_jobs_alone(P, W, seed):
    """A batch of 2-6 random small jobs (2D and 3D, straight or curved, fixed or Highland
    widths, any pixel rule, exact or constant chord), in a random launch configuration,
    writes for every job what the job writes alone, bit for bit."""
    from tests.test_gpu_random import _case
    rng = np.random.default_rng(5300 + seed)
    cfgs = [_case(W, int(rng.integers(0, 10**6))) for _ in range(int(rng.integers(2, 7)))]
    for c in cfgs:
        c["val_dtype"] = "f16"
    rpw, order, bpc = CONFIGS[int(rng.integers(0, len(CONFIGS)))]
    P.set_launch_config(rows_per_wave=rpw, order=order, blocks_per_cu=bpc)
    try:
        alone = [P.simulate(c) for c in cfgs]
        js = P.JobSet()
        xs, rps = [], []
        for c in cfgs:
            xs.append(P.phantom_build(c["phantom"]))
            rps.append(torch.empty(c["beam"]["n_protons"] + 1, dtype=torch.int64, device="cuda"))
            js.add(c["phantom"], c["beam"], xs[-1], row_ptr=rps[-1], val_dtype="f16")
        ws = torch.empty(P.workspace_bytes(js), dtype=torch.uint8, device="cuda")
        nnz = torch.empty(len(cfgs), dtype=torch.int64, device="cuda")
        P.count_rows(js, ws, nnz)
        js2 = P.JobSet()
        outs = []
        for c, x, rp, nz in zip(cfgs, xs, rps, nnz.cpu().numpy()):
            cols = torch.empty(max(int(nz), 1), dtype=torch.int32, device="cuda")
            vals = torch.empty(max(int(nz), 1), dtype=torch.float16, device="cuda")
            b = torch.empty(max(c["beam"]["n_protons"], 1), dtype=torch.float32, device="cuda")
            outs.append((cols, vals, b))
            js2.add(c["phantom"], c["beam"], x, row_ptr=rp, cols=cols, vals=vals, b=b, nnz_capacity=int(nz),
                    val_dtype="f16", chord_mm=c.get("chord_mm") or 0.0)
        P.emit_csr(js2, ws)
        assert P.device_status(ws) == P.PCT_OK
        for a, rp, (cols, vals, b), c in zip(alone, rps, outs, cfgs):
            n = c["beam"]["n_protons"]
            assert torch.equal(a["row_ptr"], rp)
            assert torch.equal(a["cols"], cols[: a["nnz"]])
            assert torch.equal(a["vals"].view(torch.int16), vals[: a["nnz"]].view(torch.int16))
            assert torch.equal(a["b"], b[:n])
    finally:
        P.set_launch_config()
