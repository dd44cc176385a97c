"""Seeded synthetic workloads (phantom tables, grids and beam parameters).

This module only lays out input descriptions as plain dictionaries; it holds none of
the simulator's arithmetic.  Both the GPU path and the CPU oracle consume the same
dictionaries.

Phantoms follow the non-homogeneous ellipse objects of the paper (Sec. II-A): an outer
ellipse with axes 180 mm x 140 mm and inner regions for skull bone (RSP 1.6), brain
(1.04), cerebro-spinal fluid in the ventricles (0.9) and an air-filled frontal sinus
(0.0); the second variant adds a skin layer.  The inner-region geometry is not printed
in the paper (its figure is an image); the layout below is the one this project uses.
"""
from __future__ import annotations

import copy
import math

import numpy as np

RSP_SET = (0.0, 0.9, 1.0, 1.04, 1.6)


def _e(center, semi, rsp, shape="ellipse", angle_deg=0.0):
    return {"shape": shape, "center": list(center), "semi": list(semi), "rsp": float(rsp),
            "angle_deg": float(angle_deg)}


def neo1_regions(scale_x=1.0, scale_y=1.0):
    """Outer skull ellipse 90x70 (semi-axes), brain 85x65, ventricles, sinus."""
    sx, sy = scale_x, scale_y
    return [
        _e((0, 0), (90 * sx, 70 * sy), 1.6),
        _e((0, 0), (85 * sx, 65 * sy), 1.04),
        _e((10 * sx, 5 * sy), (12 * sx, 6 * sy), 0.9),
        _e((-10 * sx, 5 * sy), (12 * sx, 6 * sy), 0.9),
        _e((0, 55 * sy), (10 * sx, 6 * sy), 0.0),
    ]


def neo2_regions():
    """NEO 1 with a 2 mm skin layer (RSP 1.0) inside the same 90x70 outer boundary."""
    return [
        _e((0, 0), (90, 70), 1.0),
        _e((0, 0), (88, 68), 1.6),
        _e((0, 0), (83, 63), 1.04),
        _e((10, 5), (12, 6), 0.9),
        _e((-10, 5), (12, 6), 0.9),
        _e((0, 55), (10, 6), 0.0),
    ]


def neo_turned_regions(tilt=20.0, outer_deg=0.0):
    """NEO 1 with turned inner ellipses: ventricles tilted by +-tilt degrees, the sinus
    by tilt / 2, and the whole outer boundary (skull and brain) by outer_deg."""
    return [
        _e((0, 0), (90, 70), 1.6, angle_deg=outer_deg),
        _e((0, 0), (85, 65), 1.04, angle_deg=outer_deg),
        _e((10, 5), (12, 6), 0.9, angle_deg=tilt),
        _e((-10, 5), (12, 6), 0.9, angle_deg=-tilt),
        _e((0, 55), (10, 6), 0.0, angle_deg=tilt / 2),
    ]


def neo_ellipsoid_regions(scale=1.0, a=90.0, b=70.0, c=80.0):
    """3D NEO: the 2D layout as ellipsoids; inner z semi-axes equal their y semi-axes."""
    sx, sy, sz = scale * a / 90.0, scale * b / 70.0, scale * c / 80.0
    return [
        _e((0, 0, 0), (90 * sx, 70 * sy, 80 * sz), 1.6, "ellipsoid"),
        _e((0, 0, 0), (85 * sx, 65 * sy, 75 * sz), 1.04, "ellipsoid"),
        _e((10 * sx, 5 * sy, 0), (12 * sx, 6 * sy, 6 * sz), 0.9, "ellipsoid"),
        _e((-10 * sx, 5 * sy, 0), (12 * sx, 6 * sy, 6 * sz), 0.9, "ellipsoid"),
        _e((0, 55 * sy, 0), (10 * sx, 6 * sy, 6 * sz), 0.0, "ellipsoid"),
    ]


def phantom(dim, n, h, regions, voxelize="corner_avg", origin=None, area_samples=8):
    """voxelize: "corner_avg" (the paper's examples), "center" or "area_avg" (weighted-area
    average over area_samples^dim midpoints per voxel)."""
    n = list(n) + [1] * (3 - len(n))
    h = list(h) + [1.0] * (3 - len(h))
    return {"dim": int(dim), "n": [int(v) for v in n], "h": [float(v) for v in h],
            "origin": origin, "regions": regions, "voxelize": voxelize, "area_samples": int(area_samples)}


def beam(seed, n_angles, dangle_deg, n_protons, t_range, v_range=(0.0, 0.0), path="straight",
         sigma_in=0.0, sigma_out=0.0, sigma_lat=0.0, rho=0.0, step=0.25, noise_rel=0.0,
         angle0_deg=0.0, scatter="fixed", energy_mev=200.0, x0_mm=360.8):
    """scatter="highland": exit-pair widths per proton from Highland's formula for a
    proton of kinetic energy energy_mev in a medium of radiation length x0_mm (water)."""
    return {"seed": int(seed), "n_angles": int(n_angles), "angle0_deg": float(angle0_deg),
            "dangle_deg": float(dangle_deg), "n_protons": int(n_protons),
            "t_range": [float(t_range[0]), float(t_range[1])],
            "v_range": [float(v_range[0]), float(v_range[1])], "path": path,
            "sigma_in": float(sigma_in), "sigma_out": float(sigma_out),
            "sigma_lat": float(sigma_lat), "rho": float(rho), "step": float(step),
            "noise_rel": float(noise_rel), "scatter": scatter, "energy_mev": float(energy_mev),
            "x0_mm": float(x0_mm)}


def workload(name, ph, bm, val_dtype="f32", chunk_rows=None, chord_mm=None):
    return {"name": name, "phantom": ph, "beam": bm, "val_dtype": val_dtype, "chord_mm": chord_mm,
            "chunk_rows": chunk_rows}


CURVED = dict(path="hermite", sigma_in=0.010, sigma_out=0.010, sigma_lat=1.0, rho=0.0, step=0.25)


def c0():
    """2D NEO 1, 200x200 pixels of 1 mm, 90 angles x 4 deg, 1024 protons per angle,
    offsets U[-100,100) mm, straight paths, no noise, FP32 lengths."""
    return workload("c0-2d-neo1-200sq-straight",
                    phantom(2, (200, 200), (1.0, 1.0), neo1_regions()),
                    beam(12369, 90, 4.0, 90 * 1024, (-100.0, 100.0)), "f32")


def c1():
    """2D NEO 2 (skin), 400x400 pixels of 0.5 mm, 360 angles x 8192 protons, cubic
    Hermite paths (sigma 10 mrad in/out, 1 mm lateral, 0.25 mm samples), 1% WEPL noise,
    FP16 stored lengths."""
    return workload("c1-2d-neo2-400sq-hermite",
                    phantom(2, (400, 400), (0.5, 0.5), neo2_regions()),
                    beam(12370, 360, 1.0, 360 * 8192, (-100.0, 100.0), noise_rel=0.01, **CURVED),
                    "f16")


def c2():
    """3D NEO ellipsoid 90x70x80, 200x200x160 voxels of 1 mm, 90 angles x 4 deg,
    10M protons over 200x160 mm, curved paths, 1% noise, FP16 lengths."""
    return workload("c2-3d-ellipsoid-200sq160-hermite",
                    phantom(3, (200, 200, 160), (1.0, 1.0, 1.0), neo_ellipsoid_regions()),
                    beam(12371, 90, 4.0, 10_000_000, (-100.0, 100.0), (-80.0, 80.0),
                         noise_rel=0.01, **CURVED), "f16")


def c4():
    """Head-scale 3D: 256x256x160 voxels of 0.8 mm, the 3D phantom scaled by 0.8,
    100M curved protons over 180 angles x 2 deg, 1% noise, FP16, 5M-row chunks."""
    return workload("c4-3d-ellipsoid-256sq160-hermite-chunked",
                    phantom(3, (256, 256, 160), (0.8, 0.8, 0.8), neo_ellipsoid_regions(scale=0.8)),
                    beam(12374, 180, 2.0, 100_000_000, (-102.4, 102.4), (-64.0, 64.0),
                         noise_rel=0.01, **CURVED), "f16", chunk_rows=5_000_000)


def c_paper():
    """The paper's own example shape: 200 mm x 160 mm at 1 mm (32,000 pixels), 180
    angles x 2 deg, offsets U[-125,125) mm, m = 20 n = 640,000 straight protons."""
    return workload("paper-2d-neo1-200x160-straight",
                    phantom(2, (200, 160), (1.0, 1.0), neo1_regions()),
                    beam(12375, 180, 2.0, 640_000, (-125.0, 125.0)), "f32")


def c_paper_const():
    """The paper's example with its constant chord length: every entry of A is the
    pixel size (1 mm) while b is the WEPL of the true path lengths."""
    cfg = c_paper()
    cfg["name"] = "paper-2d-neo1-200x160-straight-const-chord"
    cfg["chord_mm"] = 1.0
    return cfg


def c_paper_area():
    """The paper's example grid with the weighted-area pixel rule (8 x 8 midpoints per
    pixel) and turned inner ellipses, outer boundary turned by 15 degrees."""
    cfg = c_paper()
    cfg["name"] = "paper-2d-neo1t-200x160-straight-area"
    cfg["phantom"] = phantom(2, (200, 160), (1.0, 1.0), neo_turned_regions(20.0, 15.0), voxelize="area_avg",
                             area_samples=8)
    return cfg


def c1_highland():
    """c1 with the exit-pair widths of every proton from Highland's formula (200 MeV in
    water, X0 = 360.8 mm) instead of fixed widths."""
    cfg = c1()
    cfg["name"] = "c1h-2d-neo2-400sq-hermite-highland"
    cfg["beam"].update(scatter="highland", energy_mev=200.0, x0_mm=360.8)
    return cfg


def c3_jobs(seed=12372, n_jobs=64):
    """64 uneven jobs drawn with numpy's PCG64: even ids 2D (N in 64..512 step 64), odd
    ids 3D (N in 64, 96, 128, 160), field of view 200 mm, outer semi-axes U[60,90],
    region RSPs from {0, 0.9, 1.0, 1.04, 1.6}, 30-180 angles over 360 degrees,
    log-uniform 1e4..2e6 protons, straight or Hermite paths, 0-2% noise, FP16."""
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs = []
    for j in range(n_jobs):
        dim = 2 if j % 2 == 0 else 3
        if dim == 2:
            N = int(rng.choice(np.arange(64, 513, 64)))
        else:
            N = int(rng.choice(np.array([64, 96, 128, 160])))
        h = 200.0 / N
        a = float(rng.uniform(60.0, 90.0))
        b = float(rng.uniform(60.0, 90.0))
        c = float(rng.uniform(60.0, 90.0)) if dim == 3 else 0.0
        rsps = [float(rng.choice(RSP_SET)) for _ in range(5)]
        K = int(rng.integers(30, 181))
        P = int(round(math.exp(rng.uniform(math.log(1e4), math.log(2e6)))))
        curved = bool(rng.uniform() < 0.5)
        noise = float(rng.uniform(0.0, 0.02))
        if dim == 2:
            regs = neo1_regions(a / 90.0, b / 70.0)
            ph = phantom(2, (N, N), (h, h), regs)
            vr = (0.0, 0.0)
        else:
            regs = neo_ellipsoid_regions(1.0, a, b, c)
            ph = phantom(3, (N, N, N), (h, h, h), regs)
            vr = (-100.0, 100.0)
        for r, v in zip(regs, rsps):
            r["rsp"] = v
        extra = CURVED if curved else {}
        bm = beam(seed * 1000 + j, K, 360.0 / K, P, (-100.0, 100.0), vr, noise_rel=noise, **extra)
        jobs.append(workload(f"c3-job{j:02d}", ph, bm, "f16"))
    return jobs


def by_name(name: str):
    table = {"c0": c0, "c1": c1, "c2": c2, "c4": c4, "paper": c_paper,
             "paper_const": c_paper_const, "c1_highland": c1_highland, "paper_area": c_paper_area}
    return table[name]()


def scaled(cfg: dict, n_protons: int | None = None, **beam_overrides) -> dict:
    """A copy of a workload with fewer protons or other beam parameters (tests)."""
    out = copy.deepcopy(cfg)
    if n_protons is not None:
        out["beam"]["n_protons"] = int(n_protons)
    out["beam"].update(beam_overrides)
    return out
