"""Options of the hot path on the GPU (through the C ABI), against the oracle:
Highland exit-pair widths per proton, and the constant chord length of the paper's
examples.  The bar is the one of tests/parity.py."""
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


def _sample(n, k, seed):
    rng = np.random.default_rng(seed)
    s = rng.choice(n, size=min(k, n), replace=False)
    return np.sort(np.union1d(s, [0, n - 1])).astype(np.int64)


def _compare(P, oracle, cfg, sample, precision="mixed"):
    out = P.simulate(cfg, precision=precision)
    torch.cuda.synchronize()
    g = parity.gather_rows(out["row_ptr"], out["cols"], out["vals"], out["b"], sample)
    o = oracle.run(cfg, rows=sample)
    ph = cfg["phantom"]
    st = parity.compare(g, o, min(ph["h"][: ph["dim"]]), cfg["val_dtype"])
    print({k: v for k, v in st.items() if k != "failures"}, st["failures"][:3], flush=True)
    assert st["n_failures"] == 0, st["failures"]
    assert st["excluded"] <= 0.01 * st["rows"] + 2
    return out


def test_highland_full_size_sampled(P, oracle, W):
    cfg = W.c1_highland()
    _compare(P, oracle, cfg, _sample(cfg["beam"]["n_protons"], 3000, 11))


def test_highland_small_3d_full(P, oracle, W):
    ph = W.phantom(3, (40, 40, 32), (5.0, 5.0, 5.0), W.neo_ellipsoid_regions())
    bm = W.beam(4242, 9, 40.0, 4000, (-100.0, 100.0), (-80.0, 80.0), path="hermite",
                sigma_in=0.01, step=1.0, noise_rel=0.01, scatter="highland", energy_mev=150.0)
    cfg = W.workload("highland-3d-small", ph, bm, "f32")
    _compare(P, oracle, cfg, np.arange(4000, dtype=np.int64))


def test_highland_differs_from_fixed(P, W):
    cfg = W.scaled(W.c1(), n_protons=20000)
    a = P.simulate(cfg)
    hcfg = W.scaled(W.c1_highland(), n_protons=20000)
    b = P.simulate(hcfg)
    # same entry lines, different exit pairs: the rows must not all agree
    assert a["nnz"] != b["nnz"] or not torch.equal(a["cols"], b["cols"])


@pytest.mark.parametrize("val_dtype", ["f32", "f16"])
def test_constant_chord(P, oracle, W, val_dtype):
    cfg = W.c_paper_const()
    cfg["val_dtype"] = val_dtype
    n = cfg["beam"]["n_protons"]
    out = _compare(P, oracle, cfg, _sample(n, 3000, 12))
    assert bool(torch.all(out["vals"] == 1.0))
    exact = dict(cfg, chord_mm=None)
    e = P.simulate(exact)
    assert e["nnz"] == out["nnz"]
    assert torch.equal(e["cols"], out["cols"])
    assert torch.equal(e["b"], out["b"])       # b keeps the true path lengths
    assert not torch.equal(e["vals"], out["vals"])


def test_constant_chord_curved_lane_walk(P, oracle, W):
    # curved rows whose spline leaves the grid box take the per-lane walk
    ph = W.phantom(2, (60, 60), (2.0, 2.0), W.neo1_regions())
    bm = W.beam(99, 8, 45.0, 3000, (-100.0, 100.0), path="hermite", sigma_in=0.02,
                sigma_out=0.02, sigma_lat=3.0, step=0.5)
    cfg = W.workload("const-chord-curved", ph, bm, "f32", chord_mm=2.0)
    out = _compare(P, oracle, cfg, np.arange(3000, dtype=np.int64))
    assert bool(torch.all(out["vals"] == 2.0))


def _phantoms_f3(W):
    out = [W.c_paper_area()["phantom"]]
    out.append(W.phantom(2, (120, 90), (2.0, 2.0), W.neo_turned_regions(25.0, -12.0), voxelize="area_avg",
                         area_samples=13))
    out.append(W.phantom(2, (120, 90), (2.0, 2.0), W.neo_turned_regions(25.0, -12.0), voxelize="corner_avg"))
    out.append(W.phantom(2, (120, 90), (2.0, 2.0), W.neo_turned_regions(25.0, 40.0), voxelize="center"))
    regs3 = W.neo_ellipsoid_regions()
    regs3[2]["angle_deg"] = 30.0
    regs3[3]["angle_deg"] = -30.0
    regs3.append(W._e((0, -40, 0), (15, 5), 1.2, "ellipse", angle_deg=60.0))   # turned cylinder
    out.append(W.phantom(3, (50, 50, 40), (4.0, 4.0, 4.0), regs3, voxelize="area_avg", area_samples=4))
    return out


def test_phantom_area_rule_and_turned_regions_bit_exact(P, oracle, W):
    for ph in _phantoms_f3(W):
        x = P.phantom_build(ph).cpu().numpy()
        xo = oracle.phantom_build(ph)
        assert np.array_equal(x, xo), (ph["voxelize"], int((x != xo).sum()))


def test_corner_rule_runs_bit_exact(P, oracle, W):
    """The corner rule takes its voxels in runs of four along the last axis, sharing the
    scaled coordinates of the grid lines between them: grids whose last axis is not a
    multiple of four (runs of 1 to 3 at the end), a last axis of one voxel, turned and
    unturned regions, a cylinder among ellipsoids, and c3 jobs of both dimensions, against
    the oracle bit for bit."""
    regs2 = W.neo1_regions()
    regs2[2]["angle_deg"] = 35.0
    regs3 = W.neo_ellipsoid_regions()
    regs3.append(W._e((10, -20, 0), (25, 8), 1.2, "ellipse"))   # a cylinder along z
    regs3.append(W._e((-30, 15, 5), (12, 20, 9), 0.9, "ellipsoid", angle_deg=-50.0))
    phs = [W.phantom(2, (37, 53), (5.1, 3.7), regs2), W.phantom(2, (29, 1), (6.0, 9.0), regs2),
           W.phantom(2, (64, 6), (3.0, 30.0), regs2)]
    for n in ((21, 19, 23), (9, 6, 5), (17, 13, 1), (12, 10, 2), (8, 8, 7)):
        phs.append(W.phantom(3, n, (200.0 / n[0], 180.0 / n[1], 160.0 / n[2]), regs3))
    phs += [c["phantom"] for c in W.c3_jobs()[:4]]
    for ph in phs:
        x = P.phantom_build(ph).cpu().numpy()
        xo = oracle.phantom_build(ph)
        assert np.array_equal(x, xo), (ph["n"], int((x != xo).sum()))


def test_turned_outer_boundary_parity(P, oracle, W):
    cfg = W.c_paper_area()
    _compare(P, oracle, cfg, _sample(cfg["beam"]["n_protons"], 3000, 13))
    ph = W.phantom(2, (90, 80), (2.2, 2.2), W.neo_turned_regions(15.0, 35.0), voxelize="area_avg")
    bm = W.beam(808, 16, 22.5, 4000, (-99.0, 99.0), path="hermite", sigma_in=0.01, sigma_out=0.01,
                sigma_lat=1.0, step=0.5, noise_rel=0.01)
    _compare(P, oracle, W.workload("turned-curved", ph, bm, "f16"), np.arange(4000, dtype=np.int64))
    ph3 = W.phantom(3, (40, 40, 32), (5.0, 5.0, 5.0), W.neo_ellipsoid_regions())
    ph3["regions"][0]["angle_deg"] = 25.0
    bm3 = W.beam(809, 9, 40.0, 3000, (-100.0, 100.0), (-80.0, 80.0), path="hermite", sigma_in=0.01,
                 sigma_out=0.01, sigma_lat=1.0, step=1.0)
    _compare(P, oracle, W.workload("turned-3d", ph3, bm3, "f32"), np.arange(3000, dtype=np.int64))


def test_short_rays_inside_one_voxel_both_directions(P, oracle, W):
    """Rays that cut a grid corner stay inside one voxel of their dominant axis; moving
    down or up along it, their end points (and so the single entry's length) must hold."""
    ph = W.phantom(2, (16, 16), (1.0, 1.0), [W._e((0, 0), (5.0, 4.0), 1.3)])
    bm = W.beam(4711, 8, 45.0, 8 * 2000, (-11.4, 11.4))
    cfg = W.workload("corner-rays", ph, bm, "f32")
    out = _compare(P, oracle, cfg, np.arange(16000, dtype=np.int64))
    rp = out["row_ptr"].cpu().numpy()
    assert int(((rp[1:] - rp[:-1]) == 1).sum()) > 100   # many one-entry rows
    bm2 = W.beam(4712, 8, 45.0, 8 * 2000, (-11.4, 11.4), path="hermite", sigma_in=0.05, sigma_out=0.05,
                 sigma_lat=1.0, step=0.25)
    _compare(P, oracle, W.workload("corner-rays-curved", ph, bm2, "f16"), np.arange(16000, dtype=np.int64))
