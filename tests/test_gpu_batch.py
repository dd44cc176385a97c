"""Batched launches on the GPU: launch configurations, the autotuner and graph replay.

Every row is computed the same way whatever the order or grouping of the rows, so all
launch configurations must give bit-identical outputs; a replayed graph must write what
the eager calls write.
"""
import numpy as np
import pytest
import torch

from tests import parity

pytestmark = pytest.mark.gpu

CONFIGS = [(rpw, order) for order in ("given", "lpt") for rpw in (16, 32, 64)]


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
    for rpw, order in CONFIGS:
        P.set_launch_config(rpw, order)
        assert P.get_launch_config() == {"rows_per_wave": rpw, "order": order}
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


def test_graph_replays_match_eager(P, W):
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


def test_autotune_sets_a_valid_config_and_keeps_outputs(P, W):
    cfgs = _jobs(W, 8, 5000)
    B = Batch(P, cfgs)
    B.run()
    eager = B.snapshot()
    B.clear()
    for c, x in zip(cfgs, B.xs):
        P.phantom_build(c["phantom"], x)
    best = P.autotune(B.js, B.ws, B.nnz)
    assert (best["rows_per_wave"], best["order"]) in CONFIGS
    assert P.get_launch_config() == best
    assert P.device_status(B.ws) == P.PCT_OK
    _equal(eager, B.snapshot())
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
    rpw, order = CONFIGS[int(rng.integers(0, len(CONFIGS)))]
    P.set_launch_config(rows_per_wave=rpw, order=order)
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
