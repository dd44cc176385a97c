"""Python wrapper of the CPU oracle (``pct_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU
baseline leg of the benchmark.  It never imports the GPU package and the GPU package
never imports it.  Inputs are plain workload dictionaries (see the workload generator
of the package); marshalling into the oracle's own C structs happens here.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pct_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SHAPES = {"ellipse": 0, "ellipsoid": 1}
VOXELIZE = {"corner_avg": 0, "center": 1, "area_avg": 2}
PATHS = {"straight": 0, "hermite": 1}
KIND_MISS_GRID, KIND_STRAIGHT, KIND_CURVED, KIND_STRAIGHT_FALLBACK = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (binary64, no fused multiply-add)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"])
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Region(C.Structure):
    _fields_ = [("shape", C.c_int32), ("center", C.c_double * 3), ("semi", C.c_double * 3),
                ("rsp", C.c_float), ("angle_deg", C.c_double)]


class Phantom(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("h", C.c_double * 3),
                ("origin", C.c_double * 3), ("n_regions", C.c_int32),
                ("regions", C.POINTER(Region)), ("voxelize", C.c_int32), ("area_samples", C.c_int32)]


class Beam(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("n_angles", C.c_int32), ("angle0_deg", C.c_double),
                ("dangle_deg", C.c_double), ("n_protons", C.c_int64),
                ("t_range", C.c_double * 2), ("v_range", C.c_double * 2), ("path", C.c_int32),
                ("sigma_in", C.c_double), ("sigma_out", C.c_double), ("sigma_lat", C.c_double),
                ("rho", C.c_double), ("step", C.c_double), ("noise_rel", C.c_double),
                ("scatter", C.c_int32), ("energy_mev", C.c_double), ("x0_mm", C.c_double)]


class Path(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_samples", C.c_int32), ("t", C.c_double),
                ("v", C.c_double), ("P0", C.c_double * 3), ("P1", C.c_double * 3),
                ("d0", C.c_double * 3), ("d1", C.c_double * 3), ("L", C.c_double),
                ("thickness", C.c_double), ("sigma_out", C.c_double), ("sigma_lat", C.c_double),
                ("rho", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        L.or_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.or_draw64.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32, C.POINTER(C.c_uint64)]
        L.or_uniform53.argtypes = [C.c_uint64]
        L.or_uniform53.restype = C.c_double
        L.or_normal_pair.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]
        L.or_normal_pair.restype = C.c_int
        L.or_angle.argtypes = [C.c_double, C.c_double, C.c_int32, C.POINTER(C.c_double),
                               C.POINTER(C.c_double)]
        L.or_angle_of.argtypes = [C.c_int64, C.c_int64, C.c_int32]
        L.or_angle_of.restype = C.c_int32
        L.or_boundary_hit.argtypes = [C.POINTER(Phantom), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.or_boundary_hit.restype = C.c_int
        L.or_hermite.argtypes = [C.POINTER(C.c_double)] * 4 + [C.c_double, C.c_double, C.POINTER(C.c_double)]
        L.or_highland.argtypes = [C.c_double, C.c_double, C.c_double]
        L.or_highland.restype = C.c_double
        L.or_sap.argtypes = [C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_int32, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32]
        L.or_rsp_at.argtypes = [C.POINTER(Phantom), C.POINTER(C.c_double)]
        L.or_rsp_at.restype = C.c_double
        L.or_phantom_build.argtypes = [C.POINTER(Phantom), C.c_void_p]
        L.or_run.argtypes = [C.POINTER(Phantom), C.POINTER(Beam), C.c_void_p, C.c_void_p, C.c_int64]
        L.or_run.restype = C.c_void_p
        L.or_trace_segments.argtypes = [C.POINTER(Phantom), C.c_int32, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p]
        L.or_trace_segments.restype = C.c_void_p
        L.or_result_nnz.argtypes = [C.c_void_p]
        L.or_result_nnz.restype = C.c_int64
        L.or_result_copy.argtypes = [C.c_void_p] + [C.c_void_p] * 7
        L.or_result_free.argtypes = [C.c_void_p]
        for name in ("or_sizeof_path", "or_sizeof_region", "or_sizeof_phantom", "or_sizeof_beam"):
            getattr(L, name).restype = C.c_int32
        assert L.or_sizeof_path() == C.sizeof(Path)
        assert L.or_sizeof_region() == C.sizeof(Region)
        assert L.or_sizeof_phantom() == C.sizeof(Phantom)
        assert L.or_sizeof_beam() == C.sizeof(Beam)
        _lib = L
    return _lib


# ------------------------------------------------------------------ marshalling

def make_phantom(ph: dict):
    """Returns (Phantom struct, keep-alive region array)."""
    regs = ph["regions"]
    arr = (Region * max(1, len(regs)))()
    for i, r in enumerate(regs):
        arr[i].shape = SHAPES[r["shape"]]
        c = list(r["center"]) + [0.0] * (3 - len(r["center"]))
        s = list(r["semi"]) + [1.0] * (3 - len(r["semi"]))
        arr[i].center[:] = [float(v) for v in c]
        arr[i].semi[:] = [float(v) for v in s]
        arr[i].rsp = float(r["rsp"])
        arr[i].angle_deg = float(r.get("angle_deg", 0.0))
    p = Phantom()
    dim = int(ph["dim"])
    n = list(ph["n"]) + [1] * (3 - len(ph["n"]))
    h = list(ph["h"]) + [1.0] * (3 - len(ph["h"]))
    p.dim = dim
    p.n[:] = [int(v) for v in n]
    p.h[:] = [float(v) for v in h]
    if ph.get("origin") is not None:
        o = list(ph["origin"]) + [0.0] * (3 - len(ph["origin"]))
    else:
        o = [-(n[d] * h[d]) / 2.0 if d < dim else 0.0 for d in range(3)]
    p.origin[:] = [float(v) for v in o]
    p.n_regions = len(regs)
    p.regions = C.cast(arr, C.POINTER(Region))
    p.voxelize = VOXELIZE[ph.get("voxelize", "corner_avg")]
    p.area_samples = int(ph.get("area_samples") or 8)
    return p, arr


def make_beam(bm: dict) -> Beam:
    b = Beam()
    b.seed = int(bm["seed"])
    b.n_angles = int(bm["n_angles"])
    b.angle0_deg = float(bm.get("angle0_deg", 0.0))
    b.dangle_deg = float(bm["dangle_deg"])
    b.n_protons = int(bm["n_protons"])
    b.t_range[:] = [float(v) for v in bm["t_range"]]
    b.v_range[:] = [float(v) for v in bm.get("v_range", (0.0, 0.0))]
    b.path = PATHS[bm.get("path", "straight")]
    b.sigma_in = float(bm.get("sigma_in", 0.0))
    b.sigma_out = float(bm.get("sigma_out", 0.0))
    b.sigma_lat = float(bm.get("sigma_lat", 0.0))
    b.rho = float(bm.get("rho", 0.0))
    b.step = float(bm.get("step", 0.25))
    b.noise_rel = float(bm.get("noise_rel", 0.0))
    b.scatter = {"fixed": 0, "highland": 1}[bm.get("scatter", "fixed")]
    b.energy_mev = float(bm.get("energy_mev", 200.0))
    b.x0_mm = float(bm.get("x0_mm", 360.8))
    return b


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ------------------------------------------------------------------ entry points

def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def draw64(seed, stream, g, draw):
    w = (C.c_uint64 * 2)()
    lib().or_draw64(seed, stream, g, draw, w)
    return int(w[0]), int(w[1])


def uniform53(w):
    return lib().or_uniform53(w)


def normal_pair(seed, stream, g):
    z1, z2 = C.c_double(), C.c_double()
    att = lib().or_normal_pair(seed, stream, g, C.byref(z1), C.byref(z2))
    return z1.value, z2.value, att


def angle(angle0_deg, dangle_deg, k):
    c, s = C.c_double(), C.c_double()
    lib().or_angle(angle0_deg, dangle_deg, k, C.byref(c), C.byref(s))
    return c.value, s.value


def angle_of(g, P, K):
    return lib().or_angle_of(g, P, K)


def boundary_hit(ph: dict, Q, d):
    p, keep = make_phantom(ph)
    q = (C.c_double * 3)(*Q)
    dd = (C.c_double * 3)(*d)
    l1, l2, hc = C.c_double(), C.c_double(), C.c_double()
    hit = lib().or_boundary_hit(C.byref(p), q, dd, C.byref(l1), C.byref(l2), C.byref(hc))
    return bool(hit), l1.value, l2.value, hc.value


def hermite(P0, d0, P1, d1, L, s):
    arrs = [(C.c_double * 3)(*v) for v in (P0, d0, P1, d1)]
    out = (C.c_double * 3)()
    lib().or_hermite(*arrs, L, s, out)
    return list(out)


def highland(energy_mev, x0_mm, x_mm):
    """Highland's projected multiple-scattering width (rad) for a proton."""
    return lib().or_highland(float(energy_mev), float(x0_mm), float(x_mm))


def rsp_at(ph: dict, p):
    pp, keep = make_phantom(ph)
    q = (C.c_double * 3)(*(list(p) + [0.0] * (3 - len(p))))
    return lib().or_rsp_at(C.byref(pp), q)


def n_voxels(ph: dict) -> int:
    n = list(ph["n"]) + [1] * (3 - len(ph["n"]))
    return int(n[0]) * int(n[1]) * (int(n[2]) if int(ph["dim"]) == 3 else 1)


def phantom_build(ph: dict) -> np.ndarray:
    p, keep = make_phantom(ph)
    x = np.zeros(n_voxels(ph), dtype=np.float32)
    lib().or_phantom_build(C.byref(p), _ptr(x))
    return x


def _collect(res, nrows, with_paths):
    L = lib()
    nnz = L.or_result_nnz(res)
    row_ptr = np.zeros(nrows + 1, dtype=np.int64)
    cols = np.zeros(max(nnz, 1), dtype=np.int32)
    vals = np.zeros(max(nnz, 1), dtype=np.float64)
    b = np.zeros(nrows, dtype=np.float64)
    bc = np.zeros(nrows, dtype=np.float64)
    margin = np.zeros(nrows, dtype=np.float64)
    paths = (Path * max(nrows, 1))() if with_paths else None
    L.or_result_copy(res, _ptr(row_ptr), _ptr(cols), _ptr(vals), _ptr(b), _ptr(bc), _ptr(margin),
                     C.cast(paths, C.c_void_p) if paths is not None else None)
    L.or_result_free(res)
    out = dict(row_ptr=row_ptr, cols=cols[:nnz], vals=vals[:nnz], b=b, b_clean=bc, margin=margin)
    if with_paths:
        out["paths"] = paths
        out["kind"] = np.array([paths[i].kind for i in range(nrows)], dtype=np.int32)
    return out


def run(cfg: dict, rows=None, x: np.ndarray | None = None, with_paths: bool = False) -> dict:
    """Trace the given global proton ids (default: all) of a workload.

    Returns CSR (int64 row_ptr, int32 cols, float64 lengths), b (with noise), b_clean,
    margin (mm) and, on request, the per-row path records."""
    ph, bm = cfg["phantom"], cfg["beam"]
    if x is None:
        x = phantom_build(ph)
    if rows is None:
        rows = np.arange(int(bm["n_protons"]), dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    p, keep = make_phantom(ph)
    b = make_beam(bm)
    x = np.ascontiguousarray(x, dtype=np.float32)
    res = lib().or_run(C.byref(p), C.byref(b), _ptr(x), _ptr(rows), len(rows))
    out = _collect(res, len(rows), with_paths)
    chord = cfg.get("chord_mm") or 0.0
    if chord > 0.0:
        # constant chord length: every entry of A holds the constant; b keeps the WEPL
        # of the true lengths (Sec. II-C, Sec. III)
        out["true_vals"] = out["vals"]
        out["vals"] = np.full_like(out["vals"], float(chord))
    out["x"] = x
    out["rows"] = rows
    return out


def trace_segments(ph: dict, A, D, lo, hi) -> dict:
    """Traverse a list of segments A + l D, l in [lo, hi], as a single row."""
    p, keep = make_phantom(ph)
    A = np.ascontiguousarray(A, dtype=np.float64).reshape(-1, 3)
    D = np.ascontiguousarray(D, dtype=np.float64).reshape(-1, 3)
    lo = np.ascontiguousarray(lo, dtype=np.float64).reshape(-1)
    hi = np.ascontiguousarray(hi, dtype=np.float64).reshape(-1)
    res = lib().or_trace_segments(C.byref(p), len(A), _ptr(A), _ptr(D), _ptr(lo), _ptr(hi))
    out = _collect(res, 1, False)
    return dict(cols=out["cols"], vals=out["vals"], margin=float(out["margin"][0]))


def sap(row_ptr, cols, vals, b, n_cols, x0, n_strings=100, relax=0.1, n_iter=1, weights=None,
        order=None) -> np.ndarray:
    """String-averaging projections (Sec. II-D) in binary64: n_iter iterations from x0.

    vals and b are taken as given (converted to binary64 exactly); strings are the
    contiguous blocks floor(t m / M) of the row order."""
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    m = len(row_ptr) - 1
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    o = None if order is None else np.ascontiguousarray(order, dtype=np.int64)
    lib().or_sap(m, int(n_cols), _ptr(row_ptr), _ptr(cols), _ptr(vals), _ptr(b), int(n_strings),
                 float(relax), _ptr(w) if w is not None else None, _ptr(o) if o is not None else None,
                 _ptr(x), int(n_iter))
    return x
