"""Seeded random small configurations, every option of the path, against the oracle.

Each case draws a grid (2D or 3D, uneven sizes and voxel shapes, offset origins), a
phantom (ellipses or ellipsoids, some turned, one of the three pixel rules), a beam
(any angles, straight or Hermite, fixed or Highland widths, noise) and the output form
(FP32 or FP16, exact or constant chord lengths), and compares every row with the oracle
to the bar of tests/parity.py.
"""
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


def _case(W, seed):
    rng = np.random.default_rng(seed)
    dim = 2 if rng.uniform() < 0.6 else 3
    n = [int(rng.integers(3, 70)), int(rng.integers(3, 70)), int(rng.integers(3, 30))]
    h = [float(rng.uniform(0.5, 4.0)) for _ in range(3)]
    if rng.uniform() < 0.5:
        h[1] = h[0]
    origin = [float(-n[d] * h[d] / 2 + rng.uniform(-5, 5)) for d in range(3)]
    ext = min(n[d] * h[d] for d in range(dim))
    regs = []
    shape = "ellipsoid" if (dim == 3 and rng.uniform() < 0.6) else "ellipse"
    a = ext * rng.uniform(0.2, 0.7)
    b = ext * rng.uniform(0.2, 0.7)
    c = (n[2] * h[2] if dim == 3 else 10.0) * rng.uniform(0.2, 0.7)
    regs.append(W._e((0, 0, 0), (a, b, c), float(rng.choice([1.0, 1.6])), shape,
                     angle_deg=float(rng.choice([0.0, rng.uniform(-90, 90)]))))
    for _ in range(int(rng.integers(0, 4))):
        regs.append(W._e((rng.uniform(-a, a) / 2, rng.uniform(-b, b) / 2, 0), (a * rng.uniform(0.1, 0.5),
                         b * rng.uniform(0.1, 0.5), c * rng.uniform(0.2, 0.6)), float(rng.choice([0.0, 0.9, 1.04])),
                         shape, angle_deg=float(rng.uniform(-60, 60))))
    vox = str(rng.choice(["corner_avg", "center", "area_avg"]))
    ph = W.phantom(dim, n[:dim], h[:dim], regs, voxelize=vox, origin=origin[:dim],
                   area_samples=int(rng.integers(2, 7)))
    K = int(rng.integers(1, 40))
    Pn = int(rng.integers(K, 2500))
    curved = rng.uniform() < 0.6
    kw = {}
    if curved:
        kw = dict(path="hermite", sigma_in=float(rng.uniform(0, 0.05)), sigma_out=float(rng.uniform(0, 0.05)),
                  sigma_lat=float(rng.uniform(0, 3.0)), rho=float(rng.uniform(-0.9, 0.9)),
                  step=float(rng.uniform(0.1, 2.0)))
        if rng.uniform() < 0.4:
            kw.update(scatter="highland", energy_mev=float(rng.uniform(80, 250)))
    span = ext * rng.uniform(0.6, 1.4)
    vr = (-n[2] * h[2] * 0.6, n[2] * h[2] * 0.6) if dim == 3 else (0.0, 0.0)
    bm = W.beam(int(rng.integers(1, 2**40)), K, float(rng.uniform(0.5, 360.0 / K)), Pn, (-span / 2, span / 2), vr,
                noise_rel=float(rng.choice([0.0, 0.01])), angle0_deg=float(rng.uniform(0, 360)), **kw)
    vt = str(rng.choice(["f32", "f16"]))
    chord = float(rng.uniform(0.5, 2.0)) if rng.uniform() < 0.2 else None
    return W.workload(f"random-{seed}", ph, bm, vt, chord_mm=chord)


@pytest.mark.parametrize("seed", list(range(64)))
def test_random_case(P, oracle, W, seed):
    cfg = _case(W, 9000 + seed)
    x = P.phantom_build(cfg["phantom"]).cpu().numpy()
    assert np.array_equal(x, oracle.phantom_build(cfg["phantom"]))
    n = cfg["beam"]["n_protons"]
    for precision in ("mixed",):
        out = P.simulate(cfg, precision=precision)
        torch.cuda.synchronize()
        rows = np.arange(n, dtype=np.int64)
        g = parity.gather_rows(out["row_ptr"], out["cols"], out["vals"], out["b"], rows)
        o = oracle.run(cfg, rows=rows)
        ph = cfg["phantom"]
        st = parity.compare(g, o, min(ph["h"][: ph["dim"]]), cfg["val_dtype"])
        print(cfg["name"], {k: v for k, v in st.items() if k != "failures"}, st["failures"][:3], flush=True)
        assert st["n_failures"] == 0, st["failures"]
        assert st["excluded"] <= 0.02 * st["rows"] + 3
