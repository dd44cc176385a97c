"""Row-by-row comparison of the HIP path with the oracle (used by the GPU tests).

Bar, per row of the sample:
  * rows whose oracle margin is below 1e-6 mm (a traversal decision within 1e-6 mm of a
    voxel face, or a near-tangent / grazing case) are excluded from the column check
    and counted;
  * every other row: identical entry count and column sequence (bit-exact);
  * FP32 lengths: |gpu - oracle| <= 1e-5 * max(oracle, h_min);
  * FP16 lengths: within one binary16 ulp of the oracle length rounded to binary32
    then binary16 (round to nearest even), or within the FP32 bar plus half a binary16
    ulp (the storage rounding) -- the second form matters only for tiny pieces;
  * b (every non-excluded row): |gpu - oracle| <= 1e-5 * |oracle| + 1e-6 mm.
"""
from __future__ import annotations

import numpy as np
import torch

MARGIN_MM = 1e-6
LEN_REL = 1e-5
B_REL = 1e-5
B_ABS = 1e-6


def gather_rows(row_ptr: torch.Tensor, cols: torch.Tensor, vals: torch.Tensor, b: torch.Tensor | None,
                rows: np.ndarray) -> dict:
    """Pull the CSR entries of the given local rows to the host."""
    dev = row_ptr.device
    r = torch.as_tensor(rows, dtype=torch.int64, device=dev)
    start = row_ptr[r]
    cnt = row_ptr[r + 1] - start
    total = int(cnt.sum().item())
    if total > 0:
        rep = torch.repeat_interleave(torch.arange(len(rows), device=dev), cnt)
        first = torch.cumsum(cnt, 0) - cnt
        pos = start[rep] + (torch.arange(total, device=dev) - first[rep])
        c = cols[pos].cpu().numpy()
        v = vals[pos].cpu().numpy()
    else:
        c = np.zeros(0, np.int32)
        v = np.zeros(0, np.float32)
    rp = np.zeros(len(rows) + 1, np.int64)
    rp[1:] = np.cumsum(cnt.cpu().numpy())
    out = {"row_ptr": rp, "cols": c, "vals": v}
    if b is not None:
        out["b"] = b[r].cpu().numpy()
    return out


def compare(g: dict, o: dict, h_min: float, val_dtype: str, check_b: bool = True) -> dict:
    """g: gathered GPU rows; o: oracle result on the same rows (same order)."""
    n = len(o["rows"])
    assert len(g["row_ptr"]) == n + 1
    excl = o["margin"] < MARGIN_MM
    stats = {"rows": n, "excluded": int(excl.sum()), "excluded_mismatch": 0, "max_len_err": 0.0,
             "max_b_rel": 0.0, "nnz": int(o["row_ptr"][-1])}
    bad = []
    for i in range(n):
        ga, gb = g["row_ptr"][i], g["row_ptr"][i + 1]
        oa, ob = o["row_ptr"][i], o["row_ptr"][i + 1]
        same = (gb - ga == ob - oa) and np.array_equal(g["cols"][ga:gb], o["cols"][oa:ob])
        if excl[i]:
            stats["excluded_mismatch"] += int(not same)
            continue
        if not same:
            bad.append((i, int(o["rows"][i]), gb - ga, ob - oa))
            continue
        ol = o["vals"][oa:ob]
        gl = g["vals"][ga:gb]
        if val_dtype == "f16":
            # within one binary16 ulp of the rounded oracle length, or within the FP32
            # tolerance plus the binary16 storage rounding (matters for tiny pieces)
            ref = ol.astype(np.float32).astype(np.float16).view(np.uint16).astype(np.int32)
            got16 = gl.astype(np.float16)
            got = got16.view(np.uint16).astype(np.int32)
            d = np.abs(ref - got)
            half_ulp = np.abs(np.spacing(got16).astype(np.float64)) / 2
            err = np.abs(got16.astype(np.float64) - ol)
            okv = (d <= 1) | (err <= LEN_REL * np.maximum(ol, h_min) + half_ulp)
            if len(d):
                stats["max_f16_ulp"] = max(stats.get("max_f16_ulp", 0), int(d.max()))
            if not np.all(okv):
                bad.append((i, int(o["rows"][i]), "f16", int(d.max()), float(err.max())))
        else:
            err = np.abs(gl.astype(np.float64) - ol)
            lim = LEN_REL * np.maximum(ol, h_min)
            if len(err):
                stats["max_len_err"] = max(stats["max_len_err"], float((err / np.maximum(ol, h_min)).max()))
                if np.any(err > lim):
                    bad.append((i, int(o["rows"][i]), "len", float(err.max())))
        if check_b:
            bo = o["b"][i]
            db = abs(float(g["b"][i]) - bo)
            if bo != 0:
                stats["max_b_rel"] = max(stats["max_b_rel"], db / abs(bo))
            if db > B_REL * abs(bo) + B_ABS:
                bad.append((i, int(o["rows"][i]), "b", float(g["b"][i]), bo))
    stats["failures"] = bad[:10]
    stats["n_failures"] = len(bad)
    return stats
