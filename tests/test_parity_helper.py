"""The row comparison used by the GPU tests catches what it must (CPU only): oracle rows
compared with a copy of themselves pass, and a copy with one planted change fails."""
import numpy as np

from tests import parity


def _copy(o, val_dtype):
    vals = o["vals"].astype(np.float32)
    return {"row_ptr": o["row_ptr"].copy(), "cols": o["cols"].copy(),
            "vals": vals.astype(np.float16) if val_dtype == "f16" else vals, "b": o["b"].astype(np.float32)}


def test_compare_passes_and_catches_planted_changes(oracle, W):
    cfg = W.scaled(W.c1(), n_protons=360 * 3)
    o = oracle.run(cfg)
    for vd in ("f32", "f16"):
        st = parity.compare(_copy(o, vd), o, 0.5, vd)
        assert st["n_failures"] == 0 and st["rows"] == len(o["rows"])
    ok = np.nonzero(o["margin"] >= parity.MARGIN_MM)[0]
    i = int(ok[len(ok) // 2])
    a, b = int(o["row_ptr"][i]), int(o["row_ptr"][i + 1])
    g = _copy(o, "f32")
    g["cols"][a + 1] += 1                       # a wrong column
    assert parity.compare(g, o, 0.5, "f32")["n_failures"] == 1
    g = _copy(o, "f32")
    g["vals"][a] *= 1.0 + 3e-5                  # a length beyond 1e-5 relative
    assert parity.compare(g, o, 0.5, "f32")["n_failures"] == 1
    g = _copy(o, "f16")
    g["vals"][a] = np.float16(float(g["vals"][a]) * 1.01)   # more than one binary16 ulp
    assert parity.compare(g, o, 0.5, "f16")["n_failures"] == 1
    g = _copy(o, "f32")
    g["b"][i] *= 1.0 + 3e-5                     # b beyond 1e-5 relative
    assert parity.compare(g, o, 0.5, "f32")["n_failures"] == 1
    z = np.nonzero((o["b"] == 0.0) & (o["margin"] >= parity.B_MARGIN_MM))[0]
    assert len(z) > 0
    g = _copy(o, "f32")
    g["b"][z[0]] = 1e-12                        # b of an all-air row must be exactly 0
    assert parity.compare(g, o, 0.5, "f32")["n_failures"] == 1
    # a row excluded by its margin: a different column is counted, not failed; its b is still checked
    ex = np.nonzero((o["margin"] < parity.MARGIN_MM) & (o["margin"] >= parity.B_MARGIN_MM)
                    & (np.diff(o["row_ptr"]) > 1))[0]
    if len(ex):
        j = int(ex[0])
        g = _copy(o, "f32")
        g["cols"][int(o["row_ptr"][j])] += 1
        st = parity.compare(g, o, 0.5, "f32")
        assert st["n_failures"] == 0 and st["excluded_mismatch"] == 1
        g["b"][j] *= 1.0 + 3e-5
        assert parity.compare(g, o, 0.5, "f32")["n_failures"] == 1
    # a missing entry (shorter row) fails
    g = _copy(o, "f32")
    g["row_ptr"][i + 1:] -= 1
    g["cols"] = np.delete(g["cols"], a)
    g["vals"] = np.delete(g["vals"], a)
    assert parity.compare(g, o, 0.5, "f32")["n_failures"] >= 1
