"""SAP reconstruction (Sec. II-D) on the GPU through the C ABI, against the oracle.

Inputs: systems built by the oracle's own traversal (binary64 lengths and WEPL rounded
once to binary32, or to binary16 for the values), handed unchanged to both sides.

Bar: the GPU keeps y in binary32 and sums in binary64; one row update rounds y[c] once
(relative 2^-24) and a voxel takes a few updates per row block, so after K iterations
the deviation from the binary64 oracle stays near K * 1e-7 of the largest RSP.  The
tests allow 1e-5 (K <= 2) and 1e-4 (K = 20) of max|x|, plus 1e-6 absolute.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_2108_12369_amd import pct
    pct.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return pct


def _system(oracle, W, ph, bm, val_dtype="f32"):
    o = oracle.run(W.workload("sap-input", ph, bm))
    vt = np.float16 if val_dtype == "f16" else np.float32
    vals = o["vals"].astype(np.float32).astype(vt)
    b = o["b"].astype(np.float32)
    return dict(row_ptr=o["row_ptr"], cols=o["cols"], vals=vals, b=b, x_true=o["x"], n=len(o["x"]))


def _to_dev(sysd):
    dev = "cuda"
    return (torch.as_tensor(sysd["row_ptr"], device=dev), torch.as_tensor(sysd["cols"], device=dev),
            torch.as_tensor(sysd["vals"], device=dev), torch.as_tensor(sysd["b"], device=dev))


def _gpu_sap(P, sysd, x0, n_iter, **kw):
    rp, c, v, b = _to_dev(sysd)
    order = kw.pop("order", None)
    if order is not None:
        order = torch.as_tensor(order, dtype=torch.int64, device="cuda")
    S = P.Sap(rp, c, v, b, sysd["n"], order=order, **kw)
    x = torch.as_tensor(np.asarray(x0, dtype=np.float32), device="cuda").clone()
    S.iterate(x, n_iter)
    torch.cuda.synchronize()
    return x.cpu().numpy(), S.status()


def _oracle_sap(oracle, sysd, x0, n_iter, **kw):
    return oracle.sap(sysd["row_ptr"], sysd["cols"], sysd["vals"].astype(np.float64),
                      sysd["b"].astype(np.float64), sysd["n"], np.asarray(x0, dtype=np.float64),
                      n_iter=n_iter, **kw)


def _close(got, want, rel):
    scale = max(float(np.abs(want).max()), 1e-30)
    err = float(np.abs(got.astype(np.float64) - want).max())
    print("max err", err, "scale", scale, flush=True)
    assert err <= rel * scale + 1e-6, (err, scale)


def _paper_sys(oracle, W, m_mult=5, val_dtype="f32"):
    cfg = W.c_paper()
    bm = dict(cfg["beam"], n_protons=32000 * m_mult)
    return _system(oracle, W, cfg["phantom"], bm, val_dtype)


def test_sap_lds_path_paper_grid(P, oracle, W):
    """200 x 160 pixels (the iterate fits in LDS), m = 5n, M = 100, lambda = 0.1."""
    s = _paper_sys(oracle, W, 5)
    x0 = np.zeros(s["n"])
    for K in (1, 2):
        got, st = _gpu_sap(P, s, x0, K, n_strings=100, relax=0.1)
        assert st == 0
        _close(got, _oracle_sap(oracle, s, x0, K, n_strings=100, relax=0.1), 1e-5)


def test_sap_paper_system_full_size(P, oracle, W):
    """The benchmark's SAP workload at its full size: the paper's 200 x 160 system with
    m = 20n = 640,000 straight rows (104M entries, traced by the oracle, binary32 values),
    M = 100 strings, lambda = 0.1, two iterations from x = 0, y in LDS."""
    s = _paper_sys(oracle, W, m_mult=20)
    assert len(s["row_ptr"]) - 1 == 640_000
    x0 = np.zeros(s["n"])
    got, st = _gpu_sap(P, s, x0, 2, n_strings=100, relax=0.1)
    assert st == 0
    _close(got, _oracle_sap(oracle, s, x0, 2, n_strings=100, relax=0.1), 1e-5)


def test_sap_c1_grid_workspace(P, oracle, W):
    """The benchmark's c1 SAP setting on an eighth of its protons: the 400 x 400 grid of
    0.5 mm (the iterate in the workspace), 368,640 curved rows traced by the oracle,
    binary16 values, M = 100 strings, lambda = 0.1, two iterations from x = 0."""
    cfg = W.c1()
    bm = dict(cfg["beam"], n_protons=cfg["beam"]["n_protons"] // 8)
    s = _system(oracle, W, cfg["phantom"], bm, "f16")
    assert len(s["row_ptr"]) - 1 == 368_640 and s["n"] * 4 > 160 * 1024
    x0 = np.zeros(s["n"])
    got, st = _gpu_sap(P, s, x0, 2, n_strings=100, relax=0.1)
    assert st == 0
    _close(got, _oracle_sap(oracle, s, x0, 2, n_strings=100, relax=0.1), 1e-5)


def test_sap_fp16_values(P, oracle, W):
    s = _paper_sys(oracle, W, 2, "f16")
    x0 = np.full(s["n"], 0.5)
    got, st = _gpu_sap(P, s, x0, 2, n_strings=100, relax=0.2)
    assert st == 0
    _close(got, _oracle_sap(oracle, s, x0, 2, n_strings=100, relax=0.2), 1e-5)


def test_sap_workspace_path_large_grid(P, oracle, W):
    """256 x 256 pixels: more than one workgroup's LDS, the iterate lives in HBM."""
    ph = W.phantom(2, (256, 256), (0.8, 0.8), W.neo1_regions())
    bm = W.beam(555, 60, 3.0, 12000, (-102.4, 102.4), path="hermite", sigma_in=0.01, sigma_out=0.01,
                sigma_lat=1.0, step=0.4)
    s = _system(oracle, W, ph, bm)
    assert s["n"] * 4 > 160 * 1024
    x0 = np.zeros(s["n"])
    got, st = _gpu_sap(P, s, x0, 2, n_strings=50, relax=0.3)
    assert st == 0
    _close(got, _oracle_sap(oracle, s, x0, 2, n_strings=50, relax=0.3), 1e-5)


@pytest.mark.parametrize("val_dtype", ["f16", "f32"])
def test_sap_workspace_long_rows(P, oracle, W, val_dtype):
    """760 x 600 pixels of 0.25 mm (the iterate lives in HBM), binary16 or binary32 values,
    curved rows longer than the 768 entries the iterate stages per row (the rest read
    directly), one string, ragged weighted strings in a permuted order, and more strings
    than rows."""
    ph = W.phantom(2, (760, 600), (0.25, 0.25), W.neo1_regions())
    bm = W.beam(559, 12, 15.0, 1200, (-80.0, 80.0), path="hermite", sigma_in=0.01, sigma_out=0.01,
                sigma_lat=1.0, step=0.5)
    s = _system(oracle, W, ph, bm, val_dtype)
    lens = np.diff(s["row_ptr"])
    assert s["n"] * 4 > 160 * 1024
    assert (lens > 768).sum() > 50, lens.max()
    x0 = np.zeros(s["n"])
    got, st = _gpu_sap(P, s, x0, 2, n_strings=1, relax=0.4)
    assert st == 0
    _close(got, _oracle_sap(oracle, s, x0, 2, n_strings=1, relax=0.4), 1e-5)
    rng = np.random.default_rng(4)
    order = rng.permutation(1200)
    w = rng.uniform(0.1, 1.0, 7)
    w /= w.sum()
    x1 = rng.uniform(0, 1.5, s["n"])
    got, st = _gpu_sap(P, s, x1, 2, n_strings=7, relax=1.1, weights=list(w), order=order)
    assert st == 0
    _close(got, _oracle_sap(oracle, s, x1, 2, n_strings=7, relax=1.1, weights=w, order=order), 1e-5)
    # the first 100 rows, 130 strings: 30 strings are empty and return x_k
    m = 100
    sub = dict(s, row_ptr=s["row_ptr"][: m + 1].copy(), cols=s["cols"][: s["row_ptr"][m]].copy(),
               vals=s["vals"][: s["row_ptr"][m]].copy(), b=s["b"][:m].copy())
    got, st = _gpu_sap(P, sub, x1, 2, n_strings=130, relax=0.9)
    assert st == 0
    _close(got, _oracle_sap(oracle, sub, x1, 2, n_strings=130, relax=0.9), 1e-5)


@pytest.mark.parametrize("val_dtype", ["f16", "f32"])
def test_sap_lds_rows_of_every_length(P, oracle, val_dtype):
    """A synthetic system with y in LDS (n = 20,000) whose rows hold 1 to 900 entries in
    random distinct columns: every row body of the LDS iterate (1 to 6 chunks of 64, the
    lengths on both sides of each chunk boundary) and rows past the six prefetched
    chunks; some rows repeat a column; natural and permuted order, ragged strings."""
    rng = np.random.default_rng(77)
    n, m = 20000, 1500
    lens = rng.integers(1, 901, m)
    lens[:14] = [1, 63, 64, 65, 127, 128, 129, 255, 256, 383, 384, 385, 767, 900]
    rp = np.zeros(m + 1, np.int64)
    rp[1:] = np.cumsum(lens)
    cols = np.concatenate([rng.choice(n, int(k), replace=False) for k in lens]).astype(np.int32)
    for r in rng.choice(np.nonzero(lens >= 2)[0], 100, replace=False):
        cols[rp[r + 1] - 1] = cols[rp[r]]
    vt = np.float16 if val_dtype == "f16" else np.float32
    vals = rng.uniform(0.05, 2.0, int(rp[-1])).astype(np.float32).astype(vt)
    x_true = rng.uniform(0.0, 1.5, n)
    b = np.add.reduceat(vals.astype(np.float64) * x_true[cols], rp[:-1]).astype(np.float32)
    sd = dict(row_ptr=rp, cols=cols, vals=vals, b=b, n=n)
    assert (n + 64) * 4 <= 160 * 1024
    x0 = rng.uniform(0.0, 1.5, n)
    got, st = _gpu_sap(P, sd, x0, 2, n_strings=7, relax=0.8)
    assert st == 0
    _close(got, _oracle_sap(oracle, sd, x0, 2, n_strings=7, relax=0.8), 1e-5)
    order = rng.permutation(m)
    got, st = _gpu_sap(P, sd, x0, 1, n_strings=33, relax=1.3, order=order)
    assert st == 0
    _close(got, _oracle_sap(oracle, sd, x0, 1, n_strings=33, relax=1.3, order=order), 1e-5)


def _chain_system(seed, n, m, vdt):
    """Synthetic rows whose columns lie in a window that drifts by less than a row's
    length, so most consecutive rows share hundreds of columns: lengths 0 to 3,000
    (around the 768 entries the workspace iterate stages and the 2,048 above which a row
    waits for its own stores), some rows empty, some repeating a column."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(size=m)
    lens = np.where(u < 0.6, rng.integers(1, 769, m),
                    np.where(u < 0.85, rng.integers(769, 2049, m), rng.integers(2049, 3001, m)))
    lens[rng.uniform(size=m) < 0.08] = 0
    lens[:10] = [1, 767, 768, 769, 0, 2047, 2048, 2049, 3000, 5]
    cols, center = [], n // 2
    for L in (int(v) for v in lens):
        if L == 0:
            continue
        w = max(L, int(L * rng.uniform(1.0, 2.0)))
        start = min(max(center - w // 2, 0), n - w)
        cols.append(start + rng.choice(w, L, replace=False))
        center = int(min(max(center + rng.integers(-(L // 4) - 1, L // 4 + 2), 0), n - 1))
    rp = np.zeros(m + 1, np.int64)
    rp[1:] = np.cumsum(lens)
    cols = np.concatenate(cols).astype(np.int32)
    rep = rng.choice(np.nonzero(lens >= 2)[0], m // 12, replace=False)
    cols[rp[rep + 1] - 1] = cols[rp[rep]]   # the last entry repeats the first column
    vals = rng.uniform(0.05, 2.0, int(rp[-1])).astype(np.float32).astype(vdt)
    rows = np.repeat(np.arange(m), lens)
    b = np.bincount(rows, vals.astype(np.float64) * rng.uniform(0.0, 1.5, n)[cols], minlength=m)
    b[lens == 0] = 1.0
    return dict(row_ptr=rp, cols=cols, vals=vals, b=b.astype(np.float32), n=n), rng.uniform(0.0, 1.5, n)


@pytest.mark.parametrize("val_dtype", ["f16", "f32"])
def test_sap_workspace_consecutive_rows_share_columns(P, oracle, val_dtype):
    """y in the workspace (n = 50,000) and consecutive rows that share columns: a row's
    gathers are issued while the previous row's stores to the same columns may still be
    in flight, and must see those stores' values.  Rows that repeat a column, rows too
    long for the table of writes in flight and empty rows sit between them.  A row that
    missed the previous row's writes would move the result by a few percent; the FP32
    iterate stays within 1e-6 of max|x| of the binary64 oracle here."""
    sd, x0 = _chain_system(81 if val_dtype == "f16" else 82, 50000, 600,
                           np.float16 if val_dtype == "f16" else np.float32)
    assert sd["n"] * 4 > 160 * 1024
    lens = np.diff(sd["row_ptr"])
    assert (lens > 2048).sum() > 20 and (lens == 0).sum() > 20
    for M, relax, it in ((1, 0.8, 2), (4, 1.3, 1)):
        got, st = _gpu_sap(P, sd, x0, it, n_strings=M, relax=relax)
        assert st == 0
        _close(got, _oracle_sap(oracle, sd, x0, it, n_strings=M, relax=relax), 1e-5)


@pytest.mark.parametrize("n", [40896, 40897])
def test_sap_at_the_lds_limit(P, oracle, n):
    """n on both sides of the LDS limit: 4 (n + 64) bytes = 160 KiB at n = 40,896 (the
    iterate in LDS), one more column and it lives in the workspace.  Synthetic rows of 1
    to 500 entries whose columns include the last ones."""
    rng = np.random.default_rng(n)
    m = 600
    lens = rng.integers(1, 501, m)
    rp = np.zeros(m + 1, np.int64)
    rp[1:] = np.cumsum(lens)
    cols = np.concatenate([rng.choice(n, int(k), replace=False) for k in lens]).astype(np.int32)
    cols[rp[:-1][:50]] = n - 1   # the last column in the first entry of 50 rows
    vals = rng.uniform(0.05, 2.0, int(rp[-1])).astype(np.float32)
    b = np.add.reduceat(vals.astype(np.float64) * rng.uniform(0.0, 1.5, n)[cols], rp[:-1]).astype(np.float32)
    sd = dict(row_ptr=rp, cols=cols, vals=vals, b=b, n=n)
    x0 = rng.uniform(0.0, 1.5, n)
    got, st = _gpu_sap(P, sd, x0, 2, n_strings=5, relax=0.9)
    assert st == 0
    _close(got, _oracle_sap(oracle, sd, x0, 2, n_strings=5, relax=0.9), 1e-5)


@pytest.mark.parametrize("grid", [(64, 48, 3.0), (300, 260, 0.7), (460, 400, 0.45)])
def test_sap_repeated_columns(P, oracle, W, grid):
    """Rows that hold a column twice (as a path that re-enters a voxel would): every entry
    counts in the dot product, the norm and the update, with y in LDS (64 x 48) and in the
    workspace (300 x 260 and 460 x 400, where such rows take atomic adds and the others
    plain stores).  The prepare pass finds the repeats with a column bitmap up to 163,840
    columns and with a hash table above (460 x 400 = 184,000)."""
    nx, ny, h = grid
    ph = W.phantom(2, (nx, ny), (h, h), W.neo1_regions())
    bm = W.beam(560, 20, 9.0, 2000, (-90.0, 90.0), path="hermite", sigma_in=0.01, sigma_out=0.01,
                sigma_lat=1.0, step=0.5)
    s = _system(oracle, W, ph, bm)
    rp, cols = s["row_ptr"], s["cols"].copy()
    rows = np.nonzero(np.diff(rp) >= 3)[0][::3]
    assert len(rows) > 100
    cols[rp[rows + 1] - 1] = cols[rp[rows]]   # the last entry repeats the first column
    sd = dict(s, cols=cols)
    x0 = np.random.default_rng(5).uniform(0, 1.5, s["n"])
    got, st = _gpu_sap(P, sd, x0, 2, n_strings=9, relax=0.7)
    assert st == 0
    _close(got, _oracle_sap(oracle, sd, x0, 2, n_strings=9, relax=0.7), 1e-5)


@pytest.mark.parametrize("n", [1000, 60000])
def test_sap_no_entries(P, n):
    """A system whose rows are all empty (nnz = 0, no column or value array) leaves x as it
    is, with y in LDS (n = 1000) and in the workspace (n = 60000)."""
    m = 10
    dev = "cuda"
    rp = torch.zeros(m + 1, dtype=torch.int64, device=dev)
    cols = torch.empty(0, dtype=torch.int32, device=dev)
    vals = torch.empty(0, dtype=torch.float32, device=dev)
    b = torch.ones(m, dtype=torch.float32, device=dev)
    x0 = torch.linspace(0, 2, n, dtype=torch.float32, device=dev)
    for M in (1, 3, 40):
        S = P.Sap(rp, cols, vals, b, n, n_strings=M, relax=0.5)
        x = x0.clone()
        S.iterate(x, 2)
        torch.cuda.synchronize()
        assert S.status() == 0
        assert torch.equal(x, x0)


def test_sap_order_weights_and_ragged_strings(P, oracle, W):
    ph = W.phantom(2, (64, 48), (3.0, 3.0), W.neo1_regions())
    bm = W.beam(556, 30, 6.0, 3001, (-100.0, 100.0))
    s = _system(oracle, W, ph, bm)
    rng = np.random.default_rng(3)
    order = rng.permutation(3001)
    w = rng.uniform(0.1, 1.0, 7)
    w /= w.sum()
    x0 = rng.uniform(0, 1, s["n"])
    got, st = _gpu_sap(P, s, x0, 3, n_strings=7, relax=1.3, weights=list(w), order=order)
    assert st == 0
    _close(got, _oracle_sap(oracle, s, x0, 3, n_strings=7, relax=1.3, weights=w, order=order), 1e-5)


def test_sap_edge_cases(P, oracle, W):
    ph = W.phantom(2, (32, 32), (6.0, 6.0), W.neo1_regions())
    # offsets beyond the grid: many empty rows (zero norm, skipped)
    bm = W.beam(557, 10, 36.0, 300, (-200.0, 200.0))
    s = _system(oracle, W, ph, bm)
    assert (np.diff(s["row_ptr"]) == 0).any()
    x0 = np.linspace(0, 1, s["n"])
    for M in (1, 300, 1000):   # one chain, one row per string, more strings than rows
        got, st = _gpu_sap(P, s, x0, 2, n_strings=M, relax=0.9)
        assert st == 0
        _close(got, _oracle_sap(oracle, s, x0, 2, n_strings=M, relax=0.9), 1e-5)
    got, st = _gpu_sap(P, s, x0, 0, n_strings=5, relax=0.9)
    assert np.array_equal(got, x0.astype(np.float32))


def test_sap_bad_order_entry_is_reported_and_skipped(P, oracle, W):
    """Order entries outside [0, m) set PCT_EINVAL; their positions project nothing, as an
    empty row in their place would (the strings keep their positions)."""
    ph = W.phantom(2, (32, 32), (6.0, 6.0), W.neo1_regions())
    bm = W.beam(557, 10, 36.0, 300, (-200.0, 200.0))
    s = _system(oracle, W, ph, bm)
    empty = np.nonzero(np.diff(s["row_ptr"]) == 0)[0]
    assert len(empty) > 0
    order = np.random.default_rng(6).permutation(300)
    bad = order.copy()
    bad[17], bad[40] = 300, -1
    x0 = np.linspace(0, 1, s["n"])
    got, st = _gpu_sap(P, s, x0, 2, n_strings=5, relax=0.7, order=bad)
    assert st == P.PCT_EINVAL
    ref = order.copy()
    ref[17] = ref[40] = empty[0]
    _close(got, _oracle_sap(oracle, s, x0, 2, n_strings=5, relax=0.7, order=ref), 1e-5)


def test_sap_bad_column_is_reported_and_skipped(P, oracle, W):
    ph = W.phantom(2, (32, 32), (6.0, 6.0), W.neo1_regions())
    bm = W.beam(558, 10, 36.0, 200, (-90.0, 90.0))
    s = _system(oracle, W, ph, bm)
    bad_row = int(np.argmax(np.diff(s["row_ptr"])))
    s_bad = dict(s, cols=s["cols"].copy())
    s_bad["cols"][s["row_ptr"][bad_row]] = s["n"] + 5
    x0 = np.zeros(s["n"])
    got, st = _gpu_sap(P, s_bad, x0, 1, n_strings=4, relax=0.5)
    assert st == P.PCT_EINVAL
    keep = np.array([i for i in range(200) if i != bad_row])
    # the flagged row is skipped: same as the system without it, in a string of its own
    # position (strings keep their row ranges)
    want = _oracle_sap(oracle, dict(s, b=np.where(np.arange(200) == bad_row, 0.0, s["b"]).astype(np.float32),
                                    vals=np.where(np.repeat(np.arange(200), np.diff(s["row_ptr"])) == bad_row, 0.0,
                                                  s["vals"]).astype(np.float32)), x0, 1, n_strings=4, relax=0.5)
    _close(got, want, 1e-5)
    assert len(keep) == 199


def test_sap_reconstructs_emitted_system(P, oracle, W):
    """GPU emit -> GPU SAP, 20 iterations, on the paper's example (m = 20n, straight,
    lambda = 0.1, M = 100): close to the oracle's own pipeline, and approaching x."""
    cfg = W.c_paper()
    out = P.simulate(cfg)
    S = P.Sap(out["row_ptr"], out["cols"], out["vals"], out["b"], out["x"].numel(), n_strings=100, relax=0.1)
    x = torch.zeros_like(out["x"])
    errs = []
    xt = out["x"].double()
    for _ in range(4):
        S.iterate(x, 5)
        errs.append(float(torch.linalg.norm(x.double() - xt) / torch.linalg.norm(xt)))
    assert S.status() == 0
    print("relative error after 5/10/15/20 iterations", errs, flush=True)
    assert all(errs[i + 1] < errs[i] for i in range(3))
    o = oracle.run(cfg)
    want = oracle.sap(o["row_ptr"], o["cols"], o["vals"].astype(np.float32).astype(np.float64),
                      o["b"].astype(np.float32).astype(np.float64), len(o["x"]), np.zeros(len(o["x"])),
                      n_strings=100, relax=0.1, n_iter=20)
    _close(x.cpu().numpy(), want, 1e-4)
