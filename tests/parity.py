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
  * b on every row, excluded ones too (a crossing decided the other way near an edge moves
    at most a piece shorter than the margin between voxels, which b feels only within its
    bar): |gpu - oracle| <= 1e-5 * |oracle| + 1e-6 mm, and exactly 0 where the oracle's b
    is 0 (every entry in air, or a miss).  The one exception: rows whose margin is below
    1e-12 mm -- a near-tangent boundary solve, a sample count L / step at an integer, or
    a path lying on a face to rounding -- can take materially different voxels, so their
    b is counted apart ("b_excluded") and not compared.
"""
from __future__ import annotations

import numpy as np
import torch

MARGIN_MM = 1e-6
B_MARGIN_MM = 1e-12
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
    """g: gathered GPU rows; o: oracle result on the same rows (same order).  Vectorised
    over the entries, so that whole workloads of millions of rows can be compared."""
    n = len(o["rows"])
    assert len(g["row_ptr"]) == n + 1
    grp, orp = np.asarray(g["row_ptr"], np.int64), np.asarray(o["row_ptr"], np.int64)
    gcnt, ocnt = np.diff(grp), np.diff(orp)
    excl = o["margin"] < MARGIN_MM
    b_excl = o["margin"] < B_MARGIN_MM
    stats = {"rows": n, "excluded": int(excl.sum()), "excluded_mismatch": 0, "max_len_err": 0.0,
             "max_b_rel": 0.0, "nnz": int(orp[-1]), "b_excluded": int(b_excl.sum()) if check_b else n,
             "b_zero_rows": 0}
    bad = []
    # rows of equal length: entry-wise comparison of the columns
    eq = gcnt == ocnt
    rows_e = np.nonzero(eq)[0]
    cnt_e = ocnt[rows_e]
    tot = int(cnt_e.sum())
    rep = np.repeat(np.arange(len(rows_e)), cnt_e)
    off = np.arange(tot, dtype=np.int64) - np.repeat(np.cumsum(cnt_e) - cnt_e, cnt_e)
    gi = grp[rows_e][rep] + off
    oi = orp[rows_e][rep] + off
    gcols, ocols = np.asarray(g["cols"]), np.asarray(o["cols"])
    col_bad = gcols[gi] != ocols[oi] if tot else np.zeros(0, bool)
    row_colbad = np.zeros(n, bool)
    if tot:
        row_colbad[rows_e[rep[col_bad]]] = True
    same = eq & ~row_colbad
    stats["excluded_mismatch"] = int((excl & ~same).sum())
    for i in np.nonzero(~excl & ~same)[0][:10]:
        bad.append((int(i), int(o["rows"][i]), int(gcnt[i]), int(ocnt[i])))
    n_bad = int((~excl & ~same).sum())
    # lengths of the rows compared (same columns, not excluded)
    keep_row = same & ~excl
    ke = keep_row[rows_e][rep] if tot else np.zeros(0, bool)
    ol = np.asarray(o["vals"], np.float64)[oi[ke]]
    gl = np.asarray(g["vals"])[gi[ke]]
    erow = rows_e[rep[ke]] if tot else np.zeros(0, np.int64)
    if len(ol):
        if val_dtype == "f16":
            # within one binary16 ulp of the rounded oracle length, or within the FP32
            # tolerance plus the binary16 storage rounding (matters for tiny pieces)
            ref = ol.astype(np.float32).astype(np.float16).view(np.uint16).astype(np.int32)
            got16 = gl.astype(np.float16)
            d = np.abs(ref - got16.view(np.uint16).astype(np.int32))
            half_ulp = np.abs(np.spacing(got16).astype(np.float64)) / 2
            err = np.abs(got16.astype(np.float64) - ol)
            okv = (d <= 1) | (err <= LEN_REL * np.maximum(ol, h_min) + half_ulp)
            stats["max_f16_ulp"] = int(d.max())
            for e in np.nonzero(~okv)[0][:10]:
                bad.append((int(erow[e]), int(o["rows"][erow[e]]), "f16", int(d[e]), float(err[e])))
            n_bad += len(np.unique(erow[~okv]))
        else:
            err = np.abs(gl.astype(np.float64) - ol)
            lim = LEN_REL * np.maximum(ol, h_min)
            stats["max_len_err"] = float((err / np.maximum(ol, h_min)).max())
            over = err > lim
            for e in np.nonzero(over)[0][:10]:
                bad.append((int(erow[e]), int(o["rows"][erow[e]]), "len", float(err[e])))
            n_bad += len(np.unique(erow[over]))
    if check_b:
        bo = np.asarray(o["b"], np.float64)
        gb = np.asarray(g["b"], np.float64)
        chk = ~b_excl
        zero = chk & (bo == 0.0)
        stats["b_zero_rows"] = int(zero.sum())
        z_bad = zero & (gb != 0.0)
        nz = chk & (bo != 0.0)
        db = np.abs(gb - bo)
        if nz.any():
            stats["max_b_rel"] = float((db[nz] / np.abs(bo[nz])).max())
        b_bad = nz & (db > B_REL * np.abs(bo) + B_ABS)
        for i in np.nonzero(z_bad | b_bad)[0][:10]:
            bad.append((int(i), int(o["rows"][i]), "b0" if z_bad[i] else "b", float(gb[i]), float(bo[i])))
        n_bad += int((z_bad | b_bad).sum())
    stats["failures"] = bad[:10]
    stats["n_failures"] = n_bad
    return stats
