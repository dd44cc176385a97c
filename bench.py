"""Benchmark of the proton-CT hot path on one MI355X.

One step = the whole path over one batch: phantom voxelisation (x), count pass, scan
(row_ptr), emit pass (cols, vals and the WEPL b).  Outputs are allocated once before
the timed region; nothing is read back inside it.

The headline is the batched workload: 64 uneven jobs (2D and 3D phantoms, straight and
curved paths) in mixed precision with FP16 stored lengths, captured as one HIP graph and
replayed per step, against the plain FP32 single-phantom form (the same jobs one after
another).  Prints one JSON line: throughput in protons/s (whole job), nnz/s, the emit
pass's algorithmic HBM bandwidth against the 8 TB/s peak (HIP events on the launch
stream), the other workloads as legs, and the CPU oracle timed on a bounded seeded
sample of the same jobs.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3",
                    help="headline: c3 (the batched graph; default) | c0 | c1 | c2 | c4 | paper")
    ap.add_argument("--no-legs", action="store_true", help="skip the c1, c2 and c4 legs")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 comparison form")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched (64 uneven jobs, one graph) vs plain single-phantom comparison")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch configuration")
    ap.add_argument("--launch", default="",
                    help="ROWS_PER_WAVE,ORDER[,BLOCKS_PER_CU]: this launch configuration for the headline workload instead of "
                         "the autotuner's pick (profiling runs, where the tuner's candidate launches would "
                         "mix into the per-kernel figures)")
    ap.add_argument("--no-sap", action="store_true", help="skip the SAP reconstruction leg")
    ap.add_argument("--no-options", action="store_true",
                    help="skip the Highland-width and constant-chord variants of the path")
    ap.add_argument("--sap-only", action="store_true", help="only the SAP reconstruction leg")
    ap.add_argument("--no-io", action="store_true", help="skip the CSR file output leg")
    ap.add_argument("--cpu-rows", type=int, default=0, help="oracle sample size (0: auto)")
    ap.add_argument("--no-probe", action="store_true", help="skip the streaming-store reference (8 GiB fill)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


class Pipeline:
    """Pre-allocated buffers for a list of jobs (optionally split in row chunks)."""

    def __init__(self, P, cfgs, precision="mixed", chunk_rows=None, val_dtype=None, per_job=False):
        import torch
        self.P, self.torch = P, torch
        self.cfgs = cfgs
        self.precision = precision
        self.val_dtype = [val_dtype or c.get("val_dtype", "f32") for c in cfgs]
        self.xs = [P.phantom_build(c["phantom"]) for c in cfgs]
        self.graph = None
        # chunks: list of lists of (job index, row_begin, row_count); one call set per chunk
        if chunk_rows:
            assert len(cfgs) == 1
            n = cfgs[0]["beam"]["n_protons"]
            self.chunks = [[(0, rb, min(chunk_rows, n - rb))] for rb in range(0, n, chunk_rows)]
        elif per_job:
            self.chunks = [[(j, 0, c["beam"]["n_protons"])] for j, c in enumerate(cfgs)]
        else:
            self.chunks = [[(j, 0, c["beam"]["n_protons"]) for j, c in enumerate(cfgs)]]
        max_rows = {}
        for ch in self.chunks:
            for j, rb, rc in ch:
                max_rows[j] = max(max_rows.get(j, 0), rc)
        dev = "cuda"
        self.row_ptr = {j: torch.empty(r + 1, dtype=torch.int64, device=dev) for j, r in max_rows.items()}
        self.b = {j: torch.empty(max(r, 1), dtype=torch.float32, device=dev) for j, r in max_rows.items()}
        ws_bytes = 0
        for ch in self.chunks:
            ws_bytes = max(ws_bytes, P.workspace_bytes(self._jobset(ch, count_only=True)))
        self.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        self.nnz = torch.empty(len(cfgs), dtype=torch.int64, device=dev)
        # size the outputs from a first count of every chunk
        self.chunk_nnz = []
        cap = {}
        for ch in self.chunks:
            P.count_rows(self._jobset(ch, count_only=True), self.ws, self.nnz)
            nz = self.nnz.cpu().numpy()
            self.chunk_nnz.append([int(nz[k]) for k in range(len(ch))])
            for k, (j, rb, rc) in enumerate(ch):
                cap[j] = max(cap.get(j, 0), int(nz[k]))
        self.cols = {j: torch.empty(max(c, 1), dtype=torch.int32, device=dev) for j, c in cap.items()}
        self.vals = {j: torch.empty(max(c, 1), dtype=torch.float16 if self.val_dtype[j] == "f16" else torch.float32,
                                    device=dev) for j, c in cap.items()}
        self.cap = cap
        self.count_sets = [self._jobset(ch, count_only=True) for ch in self.chunks]
        self.emit_sets = [self._jobset(ch, count_only=False) for ch in self.chunks]
        self.total_rows = sum(rc for ch in self.chunks for _, _, rc in ch)
        self.total_nnz = sum(sum(v) for v in self.chunk_nnz)

    def _jobset(self, ch, count_only):
        js = self.P.JobSet()
        for j, rb, rc in ch:
            c = self.cfgs[j]
            if count_only:
                js.add(c["phantom"], c["beam"], self.xs[j], row_ptr=self.row_ptr[j], val_dtype=self.val_dtype[j],
                       precision=self.precision, row_begin=rb, row_count=rc)
            else:
                js.add(c["phantom"], c["beam"], self.xs[j], row_ptr=self.row_ptr[j], cols=self.cols[j],
                       vals=self.vals[j], b=self.b[j], nnz_capacity=self.cap[j], val_dtype=self.val_dtype[j],
                       precision=self.precision, row_begin=rb, row_count=rc)
        js.array()
        return js

    def autotune(self):
        """Pick the launch configuration on this workload (the first chunk)."""
        return self.P.autotune(self.emit_sets[0], self.ws, self.nnz)

    def capture(self):
        """Record the whole step (phantoms, count, emit) in one HIP graph: one job set, or
        the chunk loop (every chunk's count and emit, one after another, into the same
        outputs, whose capacity is the largest chunk's)."""
        if len(self.chunks) == 1:
            self.graph = self.P.Graph(self.emit_sets[0], self.ws, self.nnz, build_x=True)
        else:
            self.nnz_sets = self.torch.empty(sum(len(ch) for ch in self.chunks), dtype=self.torch.int64,
                                             device="cuda")
            self.graph = self.P.Graph(self.emit_sets, self.ws, self.nnz_sets, build_x=True)

    def emit_only(self, reps=3):
        """Average emit duration (ms) per chunk: eager count and emit calls, HIP events
        around each emit call on the stream it is launched on (torch's current stream,
        which the binding passes to the library)."""
        torch = self.torch
        st = torch.cuda.current_stream()
        ts = []
        for _ in range(reps):
            for k in range(len(self.chunks)):
                self.P.count_rows(self.count_sets[k], self.ws, self.nnz)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(st)
                self.P.emit_csr(self.emit_sets[k], self.ws)
                e1.record(st)
                e1.synchronize()
                ts.append(e0.elapsed_time(e1))
        st_ = self.P.device_status(self.ws)
        if st_ != self.P.PCT_OK:
            raise RuntimeError(f"device status {self.P.status_string(st_)}")
        return float(np.mean(ts))

    def step(self, emit_events=None):
        P = self.P
        if self.graph is not None:
            self.graph.launch()
            return
        for j, c in enumerate(self.cfgs):
            P.phantom_build(c["phantom"], self.xs[j])
        for k in range(len(self.chunks)):
            P.count_rows(self.count_sets[k], self.ws, self.nnz)
            if emit_events is not None:
                e0, e1 = self.torch.cuda.Event(enable_timing=True), self.torch.cuda.Event(enable_timing=True)
                e0.record()
                P.emit_csr(self.emit_sets[k], self.ws)
                e1.record()
                emit_events.append((e0, e1))
            else:
                P.emit_csr(self.emit_sets[k], self.ws)

    def bytes_emit(self):
        """Algorithmic HBM bytes of all emit launches of one step: cols (4 B) and
        vals (2 or 4 B) per nnz written, b (4 B) per row written, row_ptr (8 B) per row read."""
        tot = 0
        for ch, nzs in zip(self.chunks, self.chunk_nnz):
            for (j, rb, rc), nz in zip(ch, nzs):
                vb = 2 if self.val_dtype[j] == "f16" else 4
                tot += nz * (4 + vb) + rc * (4 + 8) + 8
        return tot

    def bytes_step(self):
        """Algorithmic bytes of a whole step: emit bytes + x written + counts written and
        read twice + row_ptr written."""
        nvox = sum(self.P.n_voxels(c["phantom"]) for c in self.cfgs)
        return self.bytes_emit() + 4 * nvox + self.total_rows * (4 * 3 + 8)


def stored_traffic(kernel, workload_name, key="traffic_bytes_per_launch"):
    """HBM bytes per launch of `kernel` on this workload from the committed profile
    summaries (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration), or None when
    no summary exists or the kernels have changed since it was taken.  key
    "valu_issue_frac": the emit kernels' VALU wave instructions per second over the
    chip's issue rate (one per CU per clock), from the same summary's counters."""
    from paper_2108_12369_amd import build as B
    digest = B.source_digest()
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    for fn in sorted(os.listdir(pdir)):
        if not fn.endswith(".md"):
            continue
        kv = {}
        with open(os.path.join(pdir, fn)) as fh:
            for line in fh:
                if line.startswith("- ") and ":" in line:
                    k, v = line[2:].split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel") == kernel and kv.get("workload") == workload_name \
                and kv.get("source_digest") == digest and key in kv:
            return float(kv[key])
    return None


C3_NAME = "c3-64-uneven-jobs-graph"


def workload(name, W):
    if name == "c3":
        return W.c3_jobs(), None
    cfg = W.by_name(name)
    return [cfg], cfg.get("chunk_rows")


def time_pipeline(pl, steps, warmup):
    torch = pl.torch
    for _ in range(warmup):
        pl.step()
    torch.cuda.synchronize()
    events = []
    t0 = time.perf_counter()
    for _ in range(steps):
        pl.step(events)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    emit_ms = [a.elapsed_time(b) for a, b in events]
    st = pl.P.device_status(pl.ws)
    if st != pl.P.PCT_OK:
        raise RuntimeError(f"device status {pl.P.status_string(st)}")
    return dt, emit_ms


def cpu_baseline(cfgs, n_rows_target):
    """The oracle, single-threaded, on evenly spaced rows of the same workload."""
    from oracle import oracle as O
    O.build(force=False)
    total = sum(c["beam"]["n_protons"] for c in cfgs)
    per = [max(1, int(round(n_rows_target * c["beam"]["n_protons"] / total))) for c in cfgs]
    rows_done, nnz_done, secs = 0, 0, 0.0
    for c, k in zip(cfgs, per):
        n = c["beam"]["n_protons"]
        rows = np.unique(np.linspace(0, n - 1, min(k, n)).astype(np.int64))
        x = O.phantom_build(c["phantom"])
        t0 = time.perf_counter()
        r = O.run(c, rows=rows, x=x)
        secs += time.perf_counter() - t0
        rows_done += len(rows)
        nnz_done += len(r["cols"])
    return rows_done, nnz_done, secs


_PAR = {}   # (cfgs, x per job) for the forked oracle workers


def _par_rows(task):
    j, rows = task
    from oracle import oracle as O
    cfgs, xs = _PAR["cfgs"], _PAR["xs"]
    r = O.run(cfgs[j], rows=rows, x=xs[j])
    return len(rows), len(r["cols"])


def sample_target(cfgs, seconds=12.0):
    """Rows of the oracle sample: about `seconds` of single-threaded oracle time."""
    n0, _, s0 = cpu_baseline(cfgs, 1000)
    return max(1000, int(seconds * n0 / max(s0, 1e-3)))


def cpu_parallel(cfgs, n_rows_target, workers):
    """The same oracle sample spread over `workers` forked processes (rows are
    independent).  Run before anything touches the GPU, so forking is safe."""
    import multiprocessing as mp
    from oracle import oracle as O
    O.build(force=False)
    total = sum(c["beam"]["n_protons"] for c in cfgs)
    tasks = []
    for j, c in enumerate(cfgs):
        n = c["beam"]["n_protons"]
        k = max(1, int(round(n_rows_target * n / total)))
        rows = np.unique(np.linspace(0, n - 1, min(k, n)).astype(np.int64))
        tasks += [(j, part) for part in np.array_split(rows, 4 * workers) if len(part)]
    _PAR["cfgs"] = cfgs
    _PAR["xs"] = [O.phantom_build(c["phantom"]) for c in cfgs]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        out = pool.map(_par_rows, tasks, chunksize=1)
    secs = time.perf_counter() - t0
    _PAR.clear()
    return sum(a for a, _ in out), sum(b for _, b in out), secs


def launch_config(P, pl, tune, launch):
    """The launch configuration for a pipeline: `launch` ("rows_per_wave,order") if given,
    else the autotuner's pick on it (or the default without tuning)."""
    if launch:
        parts = launch.split(",")
        P.set_launch_config(int(parts[0]), parts[1].strip(), int(parts[2]) if len(parts) > 2 else 0)
        return P.get_launch_config()
    return pl.autotune() if tune else P.get_launch_config()


def batched_vs_single(P, W, steps, warmup, tune, launch="", plain=True):
    """The 64 uneven jobs of the batched workload: mixed precision in one launch set
    captured as a HIP graph (autotuned), against plain FP32 with one call set per job.
    The emit pass is timed apart, with eager calls and HIP events around them."""
    import torch
    jobs = W.c3_jobs()
    out = {}
    pb = Pipeline(P, jobs, "mixed")
    cfg = launch_config(P, pb, tune, launch)
    pb.capture()
    dt, _ = time_pipeline(pb, steps, warmup)
    ms = 1e3 * dt / steps
    emit_ms = pb.emit_only(max(3, steps))
    emit_bytes = pb.bytes_emit()
    out["batched"] = {"workload": C3_NAME, "rows": pb.total_rows, "nnz": pb.total_nnz,
                      "protons_per_s": pb.total_rows / (ms * 1e-3), "nnz_per_s": pb.total_nnz / (ms * 1e-3),
                      "ms_per_step": ms, "emit_ms_per_launch": emit_ms, "algorithmic_bytes_per_launch": emit_bytes,
                      "step_algorithmic_GBps": pb.bytes_step() / (ms * 1e-3) / 1e9, "launch": cfg,
                      "precision": "mixed, FP16 stored lengths"}
    del pb
    torch.cuda.empty_cache()
    P.set_launch_config()
    if not plain:
        return out
    ps = Pipeline(P, jobs, "plain_f32", val_dtype="f32", per_job=True)
    dt, _ = time_pipeline(ps, steps, warmup)
    ms = 1e3 * dt / steps
    out["plain_single"] = {"workload": f"c3-{len(jobs)}-uneven-jobs-one-by-one", "rows": ps.total_rows,
                           "nnz": ps.total_nnz, "protons_per_s": ps.total_rows / (ms * 1e-3),
                           "nnz_per_s": ps.total_nnz / (ms * 1e-3), "ms_per_step": ms,
                           "precision": "plain FP32, FP32 stored lengths"}
    out["batched_mixed_over_plain_single"] = out["batched"]["protons_per_s"] / out["plain_single"]["protons_per_s"]
    del ps
    torch.cuda.empty_cache()
    return out


def workload_leg(P, W, name, steps, warmup, tune, plain=True):
    """One workload (chunked when it has row chunks) in mixed precision, eager calls,
    with the emit launches timed by HIP events, and the plain FP32 form beside it."""
    import torch
    cfgs, chunk = workload(name, W)
    pl = Pipeline(P, cfgs, "mixed", chunk)
    cfg = pl.autotune() if tune else P.get_launch_config()
    dt, emit_ms = time_pipeline(pl, steps, warmup)
    ms = 1e3 * dt / steps
    e_ms = float(np.mean(emit_ms))
    eb = pl.bytes_emit() / len(pl.chunks)
    out = {"workload": cfgs[0]["name"], "rows": pl.total_rows, "nnz": pl.total_nnz, "chunks": len(pl.chunks),
           "protons_per_s": pl.total_rows / (ms * 1e-3), "nnz_per_s": pl.total_nnz / (ms * 1e-3),
           "ms_per_step": ms, "emit_ms_per_launch": e_ms, "algorithmic_bytes_per_launch": eb,
           "emit_GBps": eb / (e_ms * 1e-3) / 1e9, "emit_frac": eb / (e_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "launch": cfg, "val_dtype": pl.val_dtype[0]}
    if len(pl.chunks) > 1:
        out["per_chunk"] = {"rows": pl.total_rows // len(pl.chunks), "ms": ms / len(pl.chunks),
                            "protons_per_s": pl.total_rows / (ms * 1e-3)}
        out["end_to_end"] = {"ms": ms, "protons_per_s": pl.total_rows / (ms * 1e-3)}
        # the same chunk loop captured in one HIP graph (phantom once, then each chunk's
        # count and emit), replayed per step
        pl.capture()
        dtg, _ = time_pipeline(pl, steps, warmup)
        msg = 1e3 * dtg / steps
        out["graph"] = {"ms_per_step": msg, "per_chunk_ms": msg / len(pl.chunks),
                        "protons_per_s": pl.total_rows / (msg * 1e-3)}
        pl.graph.close()
        pl.graph = None
    del pl
    torch.cuda.empty_cache()
    P.set_launch_config()
    if plain:
        pf = Pipeline(P, cfgs, "plain_f32", chunk, val_dtype="f32")
        dtp, emit_p = time_pipeline(pf, steps, warmup)
        msp = 1e3 * dtp / steps
        out["plain_f32"] = {"protons_per_s": pf.total_rows / (msp * 1e-3), "ms_per_step": msp,
                            "emit_ms_per_launch": float(np.mean(emit_p))}
        out["mixed_over_plain"] = out["protons_per_s"] / out["plain_f32"]["protons_per_s"]
        del pf
        torch.cuda.empty_cache()
    return out


def sap_leg(P, W, iters=20, n_strings=100, relax=0.1):
    """SAP (Sec. II-D) on systems emitted on the GPU: the paper's example (m = 20n,
    200 x 160 pixels: string iterates in LDS) and c1 (400 x 400: iterates in HBM).
    Timed with HIP events on the stream the kernels run on."""
    import torch
    out = {}
    for name, cfg, k in (("paper", W.c_paper(), iters), ("c1", W.c1(), 2)):
        o = P.simulate(cfg)
        n = o["x"].numel()
        S = P.Sap(o["row_ptr"], o["cols"], o["vals"], o["b"], n, n_strings=n_strings, relax=relax)
        x = torch.zeros_like(o["x"])
        S.iterate(x, 1)   # warm-up
        x.zero_()
        torch.cuda.synchronize()
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        S.iterate(x, k)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / k
        if S.status() != P.PCT_OK:
            raise RuntimeError("SAP device status " + P.status_string(S.status()))
        m, nnz = o["row_ptr"].numel() - 1, o["nnz"]
        vb = o["vals"].element_size()
        # per iteration: A once (cols, vals, row_ptr, b, coefficient), x read by every
        # string, string iterates written and read back by the average, x written
        byt = nnz * (4 + vb) + m * (8 + 4 + 4) + 3 * n_strings * n * 4 + n * 4
        xt = o["x"].double()
        err = float(torch.linalg.norm(x.double() - xt) / torch.linalg.norm(xt))
        lds = (n + 64) * 4 <= 160 * 1024
        out[name] = {"workload": cfg["name"], "rows": m, "nnz": nnz, "cols": n, "strings": n_strings,
                     "relax": relax, "iterations": k, "ms_per_iteration": ms,
                     "row_actions_per_s": m / (ms * 1e-3), "nnz_per_s": nnz / (ms * 1e-3),
                     "GBps": byt / (ms * 1e-3) / 1e9, "frac_hbm": byt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "iterate": "LDS" if lds else "HBM", "rel_error_vs_x": err}
        del S, o, x
        torch.cuda.empty_cache()
    return out


def io_leg(P, W):
    """pct_csr_write of the paper's example system (A, b and x) to a temporary file."""
    import tempfile
    import torch
    cfg = W.c_paper()
    o = P.simulate(cfg)
    torch.cuda.synchronize()
    d = tempfile.mkdtemp(prefix="pctcsr-")
    path = os.path.join(d, "paper.pctcsr")
    try:
        t0 = time.perf_counter()
        P.csr_write(path, o["row_ptr"], o["cols"], o["vals"], o["b"], o["x"])
        dt = time.perf_counter() - t0
        size = os.path.getsize(path)
    finally:
        if os.path.exists(path):
            os.remove(path)
        os.rmdir(d)
    return {"workload": cfg["name"], "bytes": size, "seconds": dt, "GBps": size / dt / 1e9,
            "target": "a new file in " + tempfile.gettempdir()}


def options_leg(P, W, steps, warmup):
    """The path with Highland widths per proton (c1) and with the constant chord length
    of the paper's example, against their default forms."""
    import torch
    out = {}
    for name, cfg in (("c1_highland", W.c1_highland()), ("paper_const_chord", W.c_paper_const()),
                      ("paper_exact", W.c_paper())):
        pl = Pipeline(P, [cfg], "mixed")
        dt, _ = time_pipeline(pl, steps, warmup)
        ms = 1e3 * dt / steps
        out[name] = {"workload": cfg["name"], "protons_per_s": pl.total_rows / (ms * 1e-3), "ms_per_step": ms,
                     "nnz_per_s": pl.total_nnz / (ms * 1e-3)}
        del pl
        torch.cuda.empty_cache()
    return out


def store_probe(torch, gib=8, reps=5):
    """Streaming-store reference for the roofline: the best of `reps` fills of a `gib` GiB
    buffer by torch (vectorised stores, nothing read), HIP events on the current stream."""
    n = (gib << 30) // 4
    buf = torch.empty(n, dtype=torch.float32, device="cuda")
    buf.fill_(1.0)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    best = None
    for i in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        buf.fill_(float(i))
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del buf
    torch.cuda.empty_cache()
    return 4 * n / (best * 1e-3) / 1e9


def cpu_sample_label(cfgs, nrow, nnz, secs, cores):
    what = (f"{nrow} rows spread over the {len(cfgs)} jobs in proportion to their sizes (evenly spaced in each)"
            if len(cfgs) > 1 else f"{nrow} evenly spaced rows")
    return (f"{what} of the same workload ({nnz} nnz), FP64 oracle on {cores} host "
            f"{'core' if cores == 1 else 'processes'}, {secs:.2f} s; the rate is the sample's, "
            f"extrapolated to the whole workload as a rate")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "gpus_requested": args.gpus}))
        sys.exit(2)
    # the oracle on all host cores first, while no process has touched the GPU
    cpu_target, par = 0, None
    if not (args.no_cpu or args.sap_only or args.copy_calibration):
        from paper_2108_12369_amd import workloads as W0
        cfgs0, _ = workload(args.workload, W0)
        cpu_target = args.cpu_rows or sample_target(cfgs0)
        workers = max(1, min(16, os.cpu_count() or 1))
        par = (workers,) + cpu_parallel(cfgs0, cpu_target, workers)
    import torch

    from paper_2108_12369_amd import build as B
    from paper_2108_12369_amd import pct as P
    from paper_2108_12369_amd import workloads as W

    P.lib()
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)

    if args.copy_calibration:
        n = 1 << 28  # 1 GiB of float32
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n}))
        return

    if args.sap_only:
        print(json.dumps({"sap": sap_leg(P, W), "sap_source_digest": B.source_digest("sap")}))
        return

    cfgs, chunk = workload(args.workload, W)
    precision = ("mixed: FP64 geometry and face ordering, FP32 lengths, FP32 partial WEPL sums folded "
                 "in FP64, FP16 stored lengths")
    if args.workload == "c3":
        bt = batched_vs_single(P, W, args.steps, args.warmup, not args.no_tune, args.launch, not args.no_plain)
        head = bt["batched"]
        ms_step, rows, nnz = head["ms_per_step"], head["rows"], head["nnz"]
        emit_launch_ms, emit_bytes_launch = head["emit_ms_per_launch"], head["algorithmic_bytes_per_launch"]
        wname = C3_NAME
        config = {"workload": wname, "jobs": len(cfgs), "rows": rows, "nnz": nnz, "chunks": 1,
                  "val_dtype": "f16", "graph": True, "launch": head["launch"]}
        step_gbps = head["step_algorithmic_GBps"]
    else:
        pl = Pipeline(P, cfgs, "mixed", chunk)
        tuned = launch_config(P, pl, not args.no_tune, args.launch)
        dt, emit_ms = time_pipeline(pl, args.steps, args.warmup)
        ms_step = 1e3 * dt / args.steps
        rows, nnz = pl.total_rows, pl.total_nnz
        emit_launch_ms = float(np.mean(emit_ms))   # one event pair per emit launch
        emit_bytes_launch = pl.bytes_emit() / len(pl.chunks)
        wname = cfgs[0]["name"]
        config = {"workload": wname, "jobs": len(cfgs), "rows": rows, "nnz": nnz, "chunks": len(pl.chunks),
                  "val_dtype": pl.val_dtype[0], "graph": False, "launch": tuned}
        step_gbps = pl.bytes_step() / (ms_step * 1e-3) / 1e9
        if pl.val_dtype[0] != "f16":
            precision = precision.replace("FP16 stored lengths", "FP32 stored lengths")
        del pl
        torch.cuda.empty_cache()
    achieved = emit_bytes_launch / (emit_launch_ms * 1e-3) / 1e9
    res = {
        "metric": "protons/s and CSR nnz/s (HBM GB/s % peak), batched mixed vs plain FP32",
        "value": rows / (ms_step * 1e-3),
        "unit": "protons/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32 (mixed), f16 stored",
        "precision": precision,
        "data": "synthetic",
        "config": config,
        "nnz_per_s": nnz / (ms_step * 1e-3),
        "step_algorithmic_GBps": step_gbps,
        "source_digest": B.source_digest(),
        "roofline": {"bound": "hbm", "kernel": "k_emit_wave",
                     "kernels_timed": "pct_emit_csr: k_emit_wave (2D and 3D instances) and k_emit_lane",
                     "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": stored_traffic("k_emit_wave", wname),
                     "valu_issue_frac": stored_traffic("k_emit_wave", wname, "valu_issue_frac"),
                     "emit_ms_per_launch": emit_launch_ms, "algorithmic_bytes_per_launch": emit_bytes_launch},
    }
    if args.workload == "c3" and "plain_single" in bt:
        res["plain_single"] = bt["plain_single"]
        res["batched_mixed_over_plain_single"] = bt["batched_mixed_over_plain_single"]

    if not args.no_probe:
        probe = store_probe(torch)
        res["roofline"]["store_probe_GBps"] = probe
        res["roofline"]["frac_of_store_probe"] = achieved / probe

    if args.workload != "c3" and not args.no_plain:
        plf = Pipeline(P, cfgs, "plain_f32", chunk, val_dtype="f32")
        dtp, emit_p = time_pipeline(plf, args.steps, args.warmup)
        msp = 1e3 * dtp / args.steps
        res["plain_f32"] = {"protons_per_s": plf.total_rows / (msp * 1e-3), "ms_per_step": msp,
                            "nnz_per_s": plf.total_nnz / (msp * 1e-3),
                            "emit_ms_per_launch": float(np.mean(emit_p)),
                            "emit_GBps": plf.bytes_emit() / len(plf.chunks) / (float(np.mean(emit_p)) * 1e-3) / 1e9}
        res["mixed_over_plain"] = res["value"] / res["plain_f32"]["protons_per_s"]
        del plf
        torch.cuda.empty_cache()

    if args.workload == "c3" and not args.no_legs:
        legs = {}
        for name, k, w in (("c1", args.steps, args.warmup), ("c2", min(args.steps, 5), 1),
                           ("c4", min(args.steps, 2), 1)):
            legs[name] = workload_leg(P, W, name, k, w, not args.no_tune, plain=not args.no_plain)
            legs[name]["roofline_traffic"] = stored_traffic("k_emit_wave", legs[name]["workload"])
            legs[name]["valu_issue_frac"] = stored_traffic("k_emit_wave", legs[name]["workload"], "valu_issue_frac")
        res["legs"] = legs

    if not args.no_options:
        res["options"] = options_leg(P, W, max(3, args.steps // 2), 1)

    if not args.no_sap:
        res["sap"] = sap_leg(P, W)
        res["sap"]["source_digest"] = B.source_digest("sap")

    if not args.no_io:
        res["csr_write"] = io_leg(P, W)

    if not args.no_cpu:
        # the sample is sized for about 12 s of single-threaded oracle time
        nrow, nnz1, secs = cpu_baseline(cfgs, cpu_target)
        res["cpu_baseline"] = {"value": nrow / secs, "unit": "protons/s", "cores": 1, "kind": "oracle",
                               "sample": cpu_sample_label(cfgs, nrow, nnz1, secs, 1),
                               "nnz_per_s": nnz1 / secs, "host_cpus": os.cpu_count()}
        if par is not None:
            w, prow, pnnz, psecs = par
            res["cpu_baseline"]["all_cores"] = {
                "value": prow / psecs, "unit": "protons/s", "cores": w, "nnz_per_s": pnnz / psecs,
                "sample": cpu_sample_label(cfgs, prow, pnnz, psecs, w)}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
