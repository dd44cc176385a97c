"""Thin ctypes binding of libpct.so (the C ABI declared in include/pct.h).

Argument marshalling only: every step of the simulation runs in the HIP kernels of the
library.  torch provides device memory and the stream.  If the library is missing the
binding raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpct.so")

PCT_OK, PCT_EINVAL, PCT_ERANGE, PCT_ECAPACITY, PCT_EWORKSPACE, PCT_EHIP, PCT_EINTERNAL = 0, -1, -2, -3, -4, -5, -6
PCT_EIO, PCT_ESCRATCH = -7, -8
PCT_ELLIPSE, PCT_ELLIPSOID = 0, 1
PCT_CORNER_AVG, PCT_CENTER, PCT_AREA_AVG = 0, 1, 2
PCT_STRAIGHT, PCT_HERMITE = 0, 1
PCT_F32, PCT_F16 = 0, 1
PCT_MIXED, PCT_PLAIN_F32 = 0, 1
PCT_MAX_REGIONS = 16
PCT_ORDER_GIVEN, PCT_ORDER_LPT = 0, 1
PCT_SCATTER_FIXED, PCT_SCATTER_HIGHLAND = 0, 1

SHAPES = {"ellipse": PCT_ELLIPSE, "ellipsoid": PCT_ELLIPSOID}
VOXELIZE = {"corner_avg": PCT_CORNER_AVG, "center": PCT_CENTER, "area_avg": PCT_AREA_AVG}
PATHS = {"straight": PCT_STRAIGHT, "hermite": PCT_HERMITE}
VAL_DTYPES = {"f32": PCT_F32, "f16": PCT_F16}
PRECISIONS = {"mixed": PCT_MIXED, "plain_f32": PCT_PLAIN_F32}
SCATTER = {"fixed": PCT_SCATTER_FIXED, "highland": PCT_SCATTER_HIGHLAND}

SYMBOLS = ("pct_status_string", "pct_version", "pct_phantom_build", "pct_workspace_bytes",
           "pct_count_rows", "pct_emit_csr", "pct_wepl", "pct_device_status", "pct_set_launch_config",
           "pct_get_launch_config", "pct_autotune", "pct_graph_create", "pct_graph_launch", "pct_graph_destroy",
           "pct_sap_workspace_bytes", "pct_sap_prepare", "pct_sap_iterate", "pct_csr_write", "pct_wepl_static",
           "pct_autotune_cached", "pct_autotune_cache_clear", "pct_graph_create_sets")


class PctError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {status_string(status)} ({status})")
        self.status = status


class Region(C.Structure):
    _fields_ = [("shape", C.c_int32), ("rsp", C.c_float), ("center", C.c_double * 3),
                ("semi", C.c_double * 3), ("angle_deg", C.c_double)]


class Phantom(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("h", C.c_double * 3),
                ("origin", C.c_double * 3), ("n_regions", C.c_int32), ("voxelize", C.c_int32),
                ("regions", C.POINTER(Region)), ("area_samples", C.c_int32)]


class Beam(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("n_angles", C.c_int32), ("path", C.c_int32),
                ("angle0_deg", C.c_double), ("dangle_deg", C.c_double), ("n_protons", C.c_int64),
                ("row_begin", C.c_int64), ("row_count", C.c_int64), ("t_range", C.c_double * 2),
                ("v_range", C.c_double * 2), ("sigma_in_rad", C.c_double),
                ("sigma_out_rad", C.c_double), ("sigma_lat_mm", C.c_double), ("rho", C.c_double),
                ("step_mm", C.c_double), ("noise_rel", C.c_double), ("scatter", C.c_int32),
                ("energy_mev", C.c_double), ("x0_mm", C.c_double)]


class Job(C.Structure):
    _fields_ = [("phantom", C.POINTER(Phantom)), ("beam", C.POINTER(Beam)), ("x_dev", C.c_void_p),
                ("row_ptr_dev", C.c_void_p), ("cols_dev", C.c_void_p), ("vals_dev", C.c_void_p),
                ("nnz_capacity", C.c_int64), ("b_dev", C.c_void_p), ("val_dtype", C.c_int32),
                ("precision", C.c_int32), ("chord_mm", C.c_double)]


class Csr(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("n_cols", C.c_int32), ("val_dtype", C.c_int32), ("nnz", C.c_int64),
                ("row_ptr_dev", C.c_void_p), ("cols_dev", C.c_void_p), ("vals_dev", C.c_void_p),
                ("b_dev", C.c_void_p)]


class SapParams(C.Structure):
    _fields_ = [("n_strings", C.c_int32), ("relax", C.c_float), ("weights", C.POINTER(C.c_double)),
                ("order_dev", C.c_void_p)]


class LaunchConfig(C.Structure):
    _fields_ = [("rows_per_wave", C.c_int32), ("order", C.c_int32), ("blocks_per_cu", C.c_int32)]


_lib = None


def lib():
    """Load libpct.so; raise if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2108_12369_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        L.pct_status_string.argtypes = [C.c_int32]
        L.pct_status_string.restype = C.c_char_p
        L.pct_version.restype = C.c_int32
        L.pct_phantom_build.argtypes = [C.POINTER(Phantom), C.c_void_p, C.c_void_p]
        L.pct_phantom_build.restype = C.c_int32
        L.pct_workspace_bytes.argtypes = [C.c_int32, C.POINTER(Job)]
        L.pct_workspace_bytes.restype = C.c_size_t
        for name in ("pct_emit_csr", "pct_wepl"):
            getattr(L, name).argtypes = [C.c_int32, C.POINTER(Job), C.c_void_p, C.c_size_t, C.c_void_p]
            getattr(L, name).restype = C.c_int32
        L.pct_wepl_static.argtypes = [C.c_int32, C.POINTER(Job), C.c_void_p, C.c_void_p]
        L.pct_wepl_static.restype = C.c_int32
        L.pct_count_rows.argtypes = [C.c_int32, C.POINTER(Job), C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]
        L.pct_count_rows.restype = C.c_int32
        L.pct_device_status.argtypes = [C.c_void_p, C.c_void_p]
        L.pct_device_status.restype = C.c_int32
        L.pct_set_launch_config.argtypes = [C.POINTER(LaunchConfig)]
        L.pct_set_launch_config.restype = C.c_int32
        L.pct_get_launch_config.argtypes = [C.POINTER(LaunchConfig)]
        L.pct_get_launch_config.restype = C.c_int32
        L.pct_autotune.argtypes = [C.c_int32, C.POINTER(Job), C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                                   C.POINTER(LaunchConfig)]
        L.pct_autotune.restype = C.c_int32
        L.pct_autotune_cached.argtypes = [C.c_int32, C.POINTER(Job), C.POINTER(LaunchConfig), C.POINTER(C.c_int32)]
        L.pct_autotune_cached.restype = C.c_int32
        L.pct_autotune_cache_clear.argtypes = []
        L.pct_autotune_cache_clear.restype = C.c_int32
        L.pct_graph_create.argtypes = [C.c_int32, C.POINTER(Job), C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                       C.POINTER(C.c_void_p)]
        L.pct_graph_create.restype = C.c_int32
        L.pct_graph_create_sets.argtypes = [C.c_int32, C.POINTER(C.c_int32), C.POINTER(Job), C.c_int32, C.c_void_p,
                                            C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]
        L.pct_graph_create_sets.restype = C.c_int32
        L.pct_graph_launch.argtypes = [C.c_void_p, C.c_void_p]
        L.pct_graph_launch.restype = C.c_int32
        L.pct_graph_destroy.argtypes = [C.c_void_p]
        L.pct_graph_destroy.restype = C.c_int32
        L.pct_sap_workspace_bytes.argtypes = [C.POINTER(Csr), C.POINTER(SapParams)]
        L.pct_sap_workspace_bytes.restype = C.c_size_t
        L.pct_sap_prepare.argtypes = [C.POINTER(Csr), C.POINTER(SapParams), C.c_void_p, C.c_size_t, C.c_void_p]
        L.pct_sap_prepare.restype = C.c_int32
        L.pct_sap_iterate.argtypes = [C.POINTER(Csr), C.POINTER(SapParams), C.c_void_p, C.c_int32, C.c_void_p,
                                      C.c_size_t, C.c_void_p]
        L.pct_sap_iterate.restype = C.c_int32
        L.pct_csr_write.argtypes = [C.c_char_p, C.POINTER(Csr), C.c_void_p, C.c_void_p]
        L.pct_csr_write.restype = C.c_int32
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().pct_status_string(int(s)).decode()


def _check(s: int, what: str):
    if s != PCT_OK:
        raise PctError(s, what)


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


# ------------------------------------------------------------------ descriptors

def make_phantom(ph: dict):
    regs = ph["regions"]
    arr = (Region * max(1, len(regs)))()
    for i, r in enumerate(regs):
        arr[i].shape = SHAPES[r["shape"]]
        arr[i].rsp = float(r["rsp"])
        arr[i].angle_deg = float(r.get("angle_deg", 0.0))
        arr[i].center[:] = [float(v) for v in list(r["center"]) + [0.0] * (3 - len(r["center"]))]
        arr[i].semi[:] = [float(v) for v in list(r["semi"]) + [1.0] * (3 - len(r["semi"]))]
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
    p.voxelize = VOXELIZE[ph.get("voxelize", "corner_avg")]
    p.regions = C.cast(arr, C.POINTER(Region))
    p.area_samples = int(ph.get("area_samples") or 0)
    return p, arr


def make_beam(bm: dict, row_begin: int = 0, row_count: int | None = None) -> Beam:
    b = Beam()
    b.seed = int(bm["seed"])
    b.n_angles = int(bm["n_angles"])
    b.path = PATHS[bm.get("path", "straight")]
    b.angle0_deg = float(bm.get("angle0_deg", 0.0))
    b.dangle_deg = float(bm["dangle_deg"])
    b.n_protons = int(bm["n_protons"])
    b.row_begin = int(row_begin)
    b.row_count = int(bm["n_protons"]) - int(row_begin) if row_count is None else int(row_count)
    b.t_range[:] = [float(v) for v in bm["t_range"]]
    b.v_range[:] = [float(v) for v in bm.get("v_range", (0.0, 0.0))]
    b.sigma_in_rad = float(bm.get("sigma_in", 0.0))
    b.sigma_out_rad = float(bm.get("sigma_out", 0.0))
    b.sigma_lat_mm = float(bm.get("sigma_lat", 0.0))
    b.rho = float(bm.get("rho", 0.0))
    b.step_mm = float(bm.get("step", 0.25))
    b.noise_rel = float(bm.get("noise_rel", 0.0))
    b.scatter = SCATTER[bm.get("scatter", "fixed")]
    b.energy_mev = float(bm.get("energy_mev", 200.0))
    b.x0_mm = float(bm.get("x0_mm", 360.8))
    return b


def n_voxels(ph: dict) -> int:
    n = list(ph["n"]) + [1] * (3 - len(ph["n"]))
    return int(n[0]) * int(n[1]) * (int(n[2]) if int(ph["dim"]) == 3 else 1)


# ------------------------------------------------------------------ entry points

def phantom_build(ph: dict, x: torch.Tensor | None = None, stream=None, device="cuda") -> torch.Tensor:
    """pct_phantom_build: voxelised true RSP vector x (float32, device)."""
    if x is None:
        x = torch.empty(n_voxels(ph), dtype=torch.float32, device=device)
    p, keep = make_phantom(ph)
    _check(lib().pct_phantom_build(C.byref(p), _ptr(x), _stream_ptr(stream)), "pct_phantom_build")
    return x


class JobSet:
    """The job descriptors of one call, with the ctypes objects kept alive."""

    def __init__(self):
        self._keep = []
        self.entries = []

    def add(self, ph: dict, bm: dict, x, row_ptr=None, cols=None, vals=None, b=None,
            nnz_capacity=0, val_dtype="f32", precision="mixed", row_begin=0, row_count=None,
            chord_mm=0.0):
        p, arr = make_phantom(ph)
        be = make_beam(bm, row_begin, row_count)
        self._keep += [p, arr, be]
        j = Job()
        j.phantom = C.pointer(p)
        j.beam = C.pointer(be)
        j.x_dev = _ptr(x)
        j.row_ptr_dev = _ptr(row_ptr)
        j.cols_dev = _ptr(cols)
        j.vals_dev = _ptr(vals)
        j.nnz_capacity = int(nnz_capacity)
        j.b_dev = _ptr(b)
        j.val_dtype = VAL_DTYPES[val_dtype]
        j.precision = PRECISIONS[precision]
        j.chord_mm = float(chord_mm or 0.0)
        self.entries.append(j)
        return len(self.entries) - 1

    def array(self):
        arr = (Job * max(1, len(self.entries)))(*self.entries)
        self._keep.append(arr)
        return len(self.entries), arr


def workspace_bytes(jobs: JobSet) -> int:
    n, arr = jobs.array()
    return int(lib().pct_workspace_bytes(n, arr))


def count_rows(jobs: JobSet, ws: torch.Tensor, nnz_total: torch.Tensor, stream=None):
    n, arr = jobs.array()
    _check(lib().pct_count_rows(n, arr, _ptr(ws), ws.numel(), _ptr(nnz_total), _stream_ptr(stream)),
           "pct_count_rows")


def emit_csr(jobs: JobSet, ws: torch.Tensor, stream=None):
    n, arr = jobs.array()
    _check(lib().pct_emit_csr(n, arr, _ptr(ws), ws.numel(), _stream_ptr(stream)), "pct_emit_csr")


def wepl(jobs: JobSet, ws: torch.Tensor, stream=None):
    n, arr = jobs.array()
    _check(lib().pct_wepl(n, arr, _ptr(ws), ws.numel(), _stream_ptr(stream)), "pct_wepl")


def wepl_static(jobs: JobSet, status: torch.Tensor | None = None, stream=None):
    """pct_wepl_static: b of every job without a workspace (the library's static device
    scratch); status: optional device int32 tensor that receives the device status word."""
    n, arr = jobs.array()
    _check(lib().pct_wepl_static(n, arr, _ptr(status) if status is not None else None, _stream_ptr(stream)),
           "pct_wepl_static")


def device_status(ws: torch.Tensor, stream=None) -> int:
    return int(lib().pct_device_status(_ptr(ws), _stream_ptr(stream)))


ORDERS = {"given": PCT_ORDER_GIVEN, "lpt": PCT_ORDER_LPT}


def set_launch_config(rows_per_wave: int | None = None, order: str | None = None, blocks_per_cu: int | None = None):
    """pct_set_launch_config; no arguments resets the default.  blocks_per_cu: 0 for a
    grid over the emit tiles, 1-8 for a persistent grid taking them from a queue."""
    if rows_per_wave is None and order is None and blocks_per_cu is None:
        _check(lib().pct_set_launch_config(None), "pct_set_launch_config")
        return
    cur = get_launch_config()
    c = LaunchConfig(int(rows_per_wave if rows_per_wave is not None else cur["rows_per_wave"]),
                     ORDERS[order] if order is not None else ORDERS[cur["order"]],
                     int(blocks_per_cu if blocks_per_cu is not None else cur["blocks_per_cu"]))
    _check(lib().pct_set_launch_config(C.byref(c)), "pct_set_launch_config")


def _cfg_dict(c: LaunchConfig) -> dict:
    inv = {v: k for k, v in ORDERS.items()}
    return {"rows_per_wave": int(c.rows_per_wave), "order": inv[int(c.order)], "blocks_per_cu": int(c.blocks_per_cu)}


def get_launch_config() -> dict:
    c = LaunchConfig()
    _check(lib().pct_get_launch_config(C.byref(c)), "pct_get_launch_config")
    return _cfg_dict(c)


def autotune(jobs: JobSet, ws: torch.Tensor, nnz_total: torch.Tensor, stream=None) -> dict:
    """pct_autotune: picks (and sets) the fastest launch configuration for these jobs, or
    the cached one for their shape."""
    n, arr = jobs.array()
    c = LaunchConfig()
    _check(lib().pct_autotune(n, arr, _ptr(ws), ws.numel(), _ptr(nnz_total), _stream_ptr(stream), C.byref(c)),
           "pct_autotune")
    return _cfg_dict(c)


def autotune_cached(jobs: JobSet) -> dict | None:
    """pct_autotune_cached: the cached configuration for these jobs' shape, or None."""
    n, arr = jobs.array()
    c = LaunchConfig()
    found = C.c_int32(0)
    _check(lib().pct_autotune_cached(n, arr, C.byref(c), C.byref(found)), "pct_autotune_cached")
    return _cfg_dict(c) if found.value else None


def autotune_cache_clear():
    _check(lib().pct_autotune_cache_clear(), "pct_autotune_cache_clear")


class Graph:
    """pct_graph_create / pct_graph_launch / pct_graph_destroy for one job set, or
    pct_graph_create_sets for a list of job sets run one after another (nnz_total then
    holds every set's jobs back to back)."""

    def __init__(self, jobs, ws: torch.Tensor, nnz_total: torch.Tensor, build_x: bool = True):
        self._jobs, self._ws, self._nnz = jobs, ws, nnz_total   # the graph refers to their memory
        h = C.c_void_p()
        if isinstance(jobs, JobSet):
            n, arr = jobs.array()
            _check(lib().pct_graph_create(n, arr, 1 if build_x else 0, _ptr(ws), ws.numel(), _ptr(nnz_total),
                                          C.byref(h)), "pct_graph_create")
        else:
            arrays = [js.array() for js in jobs]
            sizes = (C.c_int32 * len(arrays))(*[n for n, _ in arrays])
            total = sum(n for n, _ in arrays)
            assert nnz_total.numel() >= total
            flat = (Job * max(total, 1))()
            k = 0
            for n, arr in arrays:
                for i in range(n):
                    flat[k] = arr[i]
                    k += 1
            self._flat = flat
            _check(lib().pct_graph_create_sets(len(arrays), sizes, flat, 1 if build_x else 0, _ptr(ws), ws.numel(),
                                               _ptr(nnz_total), C.byref(h)), "pct_graph_create_sets")
        self._h = h

    def launch(self, stream=None):
        _check(lib().pct_graph_launch(self._h, _stream_ptr(stream)), "pct_graph_launch")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().pct_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ convenience

def simulate(cfg: dict, row_begin: int = 0, row_count: int | None = None, precision: str = "mixed",
             val_dtype: str | None = None, x: torch.Tensor | None = None, stream=None,
             device="cuda") -> dict:
    """Phantom build, count, scan and emit for one workload (or one chunk of its rows).

    Returns device tensors x, row_ptr (int64), cols (int32), vals (float32/float16), b."""
    ph, bm = cfg["phantom"], cfg["beam"]
    val_dtype = val_dtype or cfg.get("val_dtype", "f32")
    chord = cfg.get("chord_mm") or 0.0
    if row_count is None:
        row_count = int(bm["n_protons"]) - row_begin
    if x is None:
        x = phantom_build(ph, stream=stream, device=device)
    row_ptr = torch.empty(row_count + 1, dtype=torch.int64, device=device)
    js = JobSet()
    js.add(ph, bm, x, row_ptr=row_ptr, val_dtype=val_dtype, precision=precision,
           row_begin=row_begin, row_count=row_count)
    ws = torch.empty(max(workspace_bytes(js), 256), dtype=torch.uint8, device=device)
    nnz_t = torch.empty(1, dtype=torch.int64, device=device)
    count_rows(js, ws, nnz_t, stream)
    nnz = int(nnz_t.item())
    cols = torch.empty(max(nnz, 1), dtype=torch.int32, device=device)
    vals = torch.empty(max(nnz, 1), dtype=torch.float16 if val_dtype == "f16" else torch.float32, device=device)
    b = torch.empty(max(row_count, 1), dtype=torch.float32, device=device)
    js2 = JobSet()
    js2.add(ph, bm, x, row_ptr=row_ptr, cols=cols, vals=vals, b=b, nnz_capacity=nnz,
            val_dtype=val_dtype, precision=precision, row_begin=row_begin, row_count=row_count,
            chord_mm=chord)
    emit_csr(js2, ws, stream)
    st = device_status(ws, stream)
    _check(st, "device status after pct_emit_csr")
    return {"x": x, "row_ptr": row_ptr, "cols": cols[:nnz], "vals": vals[:nnz], "b": b[:row_count],
            "nnz": nnz}


# ------------------------------------------------------------------ SAP reconstruction

class Sap:
    """pct_sap_prepare / pct_sap_iterate on one CSR system (device tensors).

    row_ptr int64 (m + 1), cols int32, vals float32 or float16, b float32 (m); strings
    are consecutive blocks of the row order (order: int64 device tensor or None)."""

    def __init__(self, row_ptr, cols, vals, b, n_cols: int, n_strings: int = 100, relax: float = 0.1,
                 weights=None, order=None, stream=None):
        self._keep = [row_ptr, cols, vals, b, order]
        A = Csr()
        A.n_rows = int(row_ptr.numel()) - 1
        A.n_cols = int(n_cols)
        A.val_dtype = PCT_F16 if vals.dtype == torch.float16 else PCT_F32
        A.nnz = int(cols.numel())
        A.row_ptr_dev = _ptr(row_ptr)
        A.cols_dev = _ptr(cols)
        A.vals_dev = _ptr(vals)
        A.b_dev = _ptr(b)
        p = SapParams()
        p.n_strings = int(n_strings)
        p.relax = float(relax)
        self._w = None
        if weights is not None:
            self._w = (C.c_double * len(weights))(*[float(v) for v in weights])
            p.weights = C.cast(self._w, C.POINTER(C.c_double))
        p.order_dev = _ptr(order)
        self.A, self.p = A, p
        nb = int(lib().pct_sap_workspace_bytes(C.byref(A), C.byref(p)))
        if nb == 0:
            raise PctError(PCT_EINVAL, "pct_sap_workspace_bytes")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=row_ptr.device)
        self.prepare(stream)

    def prepare(self, stream=None):
        _check(lib().pct_sap_prepare(C.byref(self.A), C.byref(self.p), _ptr(self.ws), self.ws.numel(),
                                     _stream_ptr(stream)), "pct_sap_prepare")

    def iterate(self, x: torch.Tensor, n_iter: int = 1, stream=None) -> torch.Tensor:
        """n_iter iterations in place on x (float32 device tensor of n_cols)."""
        assert x.dtype == torch.float32 and x.numel() == self.A.n_cols and x.is_contiguous()
        _check(lib().pct_sap_iterate(C.byref(self.A), C.byref(self.p), _ptr(x), int(n_iter), _ptr(self.ws),
                                     self.ws.numel(), _stream_ptr(stream)), "pct_sap_iterate")
        return x

    def status(self, stream=None) -> int:
        return device_status(self.ws, stream)


# ------------------------------------------------------------------ CSR files

def make_csr(row_ptr, cols, vals, b, n_cols: int) -> Csr:
    A = Csr()
    A.n_rows = int(row_ptr.numel()) - 1
    A.n_cols = int(n_cols)
    A.val_dtype = PCT_F16 if vals.dtype == torch.float16 else PCT_F32
    A.nnz = int(cols.numel())
    A.row_ptr_dev = _ptr(row_ptr)
    A.cols_dev = _ptr(cols)
    A.vals_dev = _ptr(vals)
    A.b_dev = _ptr(b)
    return A


def csr_write(path: str, row_ptr, cols, vals, b=None, x=None, n_cols: int | None = None, stream=None):
    """pct_csr_write: the system to a binary CSR file (returns when it is complete)."""
    n = int(n_cols if n_cols is not None else x.numel())
    A = make_csr(row_ptr, cols, vals, b, n)
    _check(lib().pct_csr_write(os.fsencode(path), C.byref(A), _ptr(x), _stream_ptr(stream)), "pct_csr_write")


def read_csr(path: str, mmap: bool = True) -> dict:
    """Read a file of pct_csr_write into numpy arrays (memory-mapped by default)."""
    hdr = np.fromfile(path, dtype=np.uint8, count=128)
    if bytes(hdr[:8]) != b"PCTCSR01":
        raise ValueError(f"{path}: not a PCTCSR01 file")
    m, n, nnz = (int(v) for v in hdr[8:32].view("<i8"))
    val_dtype, version = (int(v) for v in hdr[32:40].view("<i4"))
    o_rp, o_c, o_v, o_b, o_x = (int(v) for v in hdr[40:80].view("<i8"))
    vt = np.float16 if val_dtype == PCT_F16 else np.float32

    def arr(off, dt, count):
        if mmap:
            return np.memmap(path, dtype=dt, mode="r", offset=off, shape=(count,))
        with open(path, "rb") as f:
            f.seek(off)
            return np.fromfile(f, dtype=dt, count=count)
    out = {"n_rows": m, "n_cols": n, "nnz": nnz, "val_dtype": "f16" if val_dtype == PCT_F16 else "f32",
           "version": version, "row_ptr": arr(o_rp, "<i8", m + 1), "cols": arr(o_c, "<i4", nnz),
           "vals": arr(o_v, vt, nnz)}
    out["b"] = arr(o_b, "<f4", m) if o_b else None
    out["x"] = arr(o_x, "<f4", n) if o_x else None
    return out
