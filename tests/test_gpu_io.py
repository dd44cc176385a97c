"""Binary CSR files written from device memory (through the C ABI), read back."""
import os

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


def test_csr_file_round_trip_multi_chunk(P, oracle, W, tmp_path):
    cfg = W.c0()   # 22M entries: cols span two 64 MiB staging chunks
    out = P.simulate(cfg)
    f = str(tmp_path / "c0.pctcsr")
    P.csr_write(f, out["row_ptr"], out["cols"], out["vals"], out["b"], out["x"])
    r = P.read_csr(f)
    assert r["nnz"] == out["nnz"] and r["n_rows"] == cfg["beam"]["n_protons"]
    assert r["n_cols"] == out["x"].numel() and r["val_dtype"] == "f32"
    assert np.array_equal(r["row_ptr"], out["row_ptr"].cpu().numpy())
    assert np.array_equal(r["cols"], out["cols"].cpu().numpy())
    assert np.array_equal(r["vals"], out["vals"].cpu().numpy())
    assert np.array_equal(r["b"], out["b"].cpu().numpy())
    assert np.array_equal(r["x"], out["x"].cpu().numpy())
    # the file's rows against the oracle
    rows = np.sort(np.random.default_rng(5).choice(len(r["b"]), 500, replace=False)).astype(np.int64)
    rp = torch.from_numpy(np.array(r["row_ptr"]))
    g = parity.gather_rows(rp, torch.from_numpy(np.array(r["cols"])), torch.from_numpy(np.array(r["vals"])),
                           torch.from_numpy(np.array(r["b"])), rows)
    st = parity.compare(g, oracle.run(cfg, rows=rows), 1.0, "f32")
    assert st["n_failures"] == 0, st["failures"]
    assert os.path.getsize(f) >= 128 + 8 * (len(r["b"]) + 1) + 8 * r["nnz"]


def test_csr_file_fp16_without_b_and_x(P, W, tmp_path):
    cfg = W.scaled(W.c1(), n_protons=36000)
    out = P.simulate(cfg)
    f = str(tmp_path / "c1.pctcsr")
    P.csr_write(f, out["row_ptr"], out["cols"], out["vals"], None, None, n_cols=out["x"].numel())
    r = P.read_csr(f, mmap=False)
    assert r["val_dtype"] == "f16" and r["b"] is None and r["x"] is None
    assert np.array_equal(r["vals"].view(np.uint16), out["vals"].cpu().numpy().view(np.uint16))
    assert np.array_equal(r["cols"], out["cols"].cpu().numpy())


def test_csr_file_errors(P, W, tmp_path):
    cfg = W.scaled(W.c0(), n_protons=1000)
    out = P.simulate(cfg)
    with pytest.raises(P.PctError) as e:
        P.csr_write(str(tmp_path / "missing-dir" / "a.pctcsr"), out["row_ptr"], out["cols"], out["vals"],
                    out["b"], out["x"])
    assert e.value.status == P.PCT_EIO
    # capacity smaller than row_ptr[m]: refused, nothing read beyond the arrays
    with pytest.raises(P.PctError) as e:
        P.csr_write(str(tmp_path / "b.pctcsr"), out["row_ptr"], out["cols"][: out["nnz"] // 2],
                    out["vals"][: out["nnz"] // 2], out["b"], out["x"])
    assert e.value.status == P.PCT_EINVAL
