"""Seeded random SAP systems (Sec. II-D) on the GPU through the C ABI, against the oracle.

Each case draws a 2D grid (small, with y in LDS, or above the LDS limit, with y in the
workspace), a straight or curved beam, binary16 or binary32 values, sometimes rows that
repeat a column, a number of strings from 1 to more than the rows, a relaxation in
(0, 2), a row order or none, weights or none, one or two iterations, and a random x_0.
The bar is that of tests/test_gpu_sap.py for one or two iterations: the GPU keeps y in
binary32 and sums in binary64, so it stays within 1e-5 of max|x| (plus 1e-6) of the
binary64 oracle.
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


def _case(oracle, W, seed):
    rng = np.random.default_rng(seed)
    big = rng.uniform() < 0.4
    nx = int(rng.integers(210, 320)) if big else int(rng.integers(8, 120))
    ny = int(rng.integers(210, 300)) if big else int(rng.integers(8, 120))
    h = float(rng.uniform(0.6, 1.2)) if big else float(rng.uniform(1.0, 6.0))
    sc = min(nx, ny) * h / 200.0
    ph = W.phantom(2, (nx, ny), (h, h), W.neo1_regions(sc, sc))
    kw = {}
    if rng.uniform() < 0.5:
        kw = dict(path="hermite", sigma_in=0.01, sigma_out=0.01, sigma_lat=1.0, step=float(rng.uniform(0.3, 1.0)))
    K = int(rng.integers(1, 30))
    m = int(rng.integers(K, 1500 if big else 800))
    span = min(nx, ny) * h * float(rng.uniform(0.5, 1.3))
    bm = W.beam(int(rng.integers(1, 2**31)), K, 360.0 / K, m, (-span / 2, span / 2), **kw)
    o = oracle.run(W.workload("sap-random", ph, bm))
    rp, cols = o["row_ptr"], o["cols"].copy()
    if rng.uniform() < 0.3 and len(cols) > 0:
        rows = np.nonzero(np.diff(rp) >= 3)[0][:: int(rng.integers(2, 6))]
        cols[rp[rows + 1] - 1] = cols[rp[rows]]   # the last entry repeats the first column
    vdt = np.float16 if rng.uniform() < 0.5 else np.float32
    sysd = dict(row_ptr=rp, cols=cols, vals=o["vals"].astype(np.float32).astype(vdt),
                b=o["b"].astype(np.float32), n=len(o["x"]))
    M = int(rng.integers(1, m + 12))
    w = None
    if rng.uniform() < 0.4:
        w = rng.uniform(0.1, 1.0, M)
        w /= w.sum()
    params = dict(n_strings=M, relax=float(rng.uniform(0.05, 1.9)), weights=w,
                  order=rng.permutation(m) if rng.uniform() < 0.5 else None)
    x0 = rng.uniform(0, 1.5, sysd["n"]).astype(np.float32)
    return sysd, params, int(rng.integers(1, 3)), x0, big


@pytest.mark.parametrize("seed", list(range(40)))
def test_sap_random_case(P, oracle, W, seed):
    sysd, prm, n_iter, x0, big = _case(oracle, W, 7100 + seed)
    dev = "cuda"
    order = None if prm["order"] is None else torch.as_tensor(prm["order"], dtype=torch.int64, device=dev)
    S = P.Sap(torch.as_tensor(sysd["row_ptr"], device=dev), torch.as_tensor(sysd["cols"], device=dev),
              torch.as_tensor(sysd["vals"], device=dev), torch.as_tensor(sysd["b"], device=dev), sysd["n"],
              n_strings=prm["n_strings"], relax=prm["relax"],
              weights=None if prm["weights"] is None else list(prm["weights"]), order=order)
    x = torch.as_tensor(x0, device=dev).clone()
    S.iterate(x, n_iter)
    torch.cuda.synchronize()
    assert S.status() == 0
    want = oracle.sap(sysd["row_ptr"], sysd["cols"], sysd["vals"].astype(np.float64), sysd["b"].astype(np.float64),
                      sysd["n"], x0.astype(np.float64), n_iter=n_iter, n_strings=prm["n_strings"],
                      relax=prm["relax"], weights=prm["weights"], order=prm["order"])
    got = x.cpu().numpy().astype(np.float64)
    scale = max(float(np.abs(want).max()), 1e-30)
    err = float(np.abs(got - want).max())
    print("seed", seed, "n", sysd["n"], "workspace iterate" if big else "LDS iterate", "err", err, flush=True)
    assert err <= 1e-5 * scale + 1e-6, (err, scale)
