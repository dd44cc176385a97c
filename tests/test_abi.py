"""The C ABI library on the host (no GPU work): it loads, exports every entry point the
public header declares, its structs have the layout the binding assumes, and host-side
validation rejects bad descriptors before anything would be enqueued."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pct.h")


@pytest.fixture(scope="module")
def P():
    from paper_2108_12369_amd import pct
    return pct


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pct_[a-z_]+)\s*\(", text)))


def test_header_functions_exported(P):
    names = _declared_functions()
    assert set(names) == set(P.SYMBOLS)
    lib = P.lib()
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(P):
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        s = P.status_string(code)
        assert s.startswith("PCT_")
    assert P.lib().pct_version() >= 100


def test_struct_layout_matches_header(P, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "pct.h"
#define F(T, m) printf(#T "." #m " %zu\n", offsetof(T, m));
int main(void) {
  printf("pct_region %zu\npct_phantom %zu\npct_beam %zu\npct_job %zu\n",
         sizeof(pct_region), sizeof(pct_phantom), sizeof(pct_beam), sizeof(pct_job));
  F(pct_region, rsp) F(pct_region, center) F(pct_region, semi)
  F(pct_phantom, n) F(pct_phantom, h) F(pct_phantom, origin) F(pct_phantom, n_regions)
  F(pct_phantom, voxelize) F(pct_phantom, regions)
  F(pct_beam, n_angles) F(pct_beam, path) F(pct_beam, angle0_deg) F(pct_beam, n_protons)
  F(pct_beam, row_begin) F(pct_beam, row_count) F(pct_beam, t_range) F(pct_beam, v_range)
  F(pct_beam, sigma_in_rad) F(pct_beam, rho) F(pct_beam, step_mm) F(pct_beam, noise_rel)
  F(pct_beam, scatter) F(pct_beam, energy_mev) F(pct_beam, x0_mm)
  F(pct_job, x_dev) F(pct_job, row_ptr_dev) F(pct_job, cols_dev) F(pct_job, vals_dev)
  F(pct_job, nnz_capacity) F(pct_job, b_dev) F(pct_job, val_dtype) F(pct_job, precision)
  F(pct_job, chord_mm)
  printf("pct_csr %zu\npct_sap %zu\n", sizeof(pct_csr), sizeof(pct_sap));
  F(pct_csr, n_cols) F(pct_csr, val_dtype) F(pct_csr, nnz) F(pct_csr, row_ptr_dev) F(pct_csr, cols_dev)
  F(pct_csr, vals_dev) F(pct_csr, b_dev)
  F(pct_sap, relax) F(pct_sap, weights) F(pct_sap, order_dev)
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(line.split() for line in out if line.strip())
    types = {"pct_region": P.Region, "pct_phantom": P.Phantom, "pct_beam": P.Beam, "pct_job": P.Job,
             "pct_csr": P.Csr, "pct_sap": P.SapParams}
    for k, v in got.items():
        if "." in k:
            t, m = k.split(".")
            assert getattr(types[t], m).offset == int(v), k
        else:
            assert C.sizeof(types[k]) == int(v), k


def test_workspace_bytes_scales_with_rows(P, W):
    js = P.JobSet()
    cfg = W.c0()
    js.add(cfg["phantom"], cfg["beam"], None)
    small = P.workspace_bytes(js)
    js2 = P.JobSet()
    js2.add(cfg["phantom"], cfg["beam"], None)
    js2.add(cfg["phantom"], cfg["beam"], None)
    assert small > 92160 * 4
    assert P.workspace_bytes(js2) > small
    assert P.workspace_bytes(P.JobSet()) > 0  # header only


@pytest.mark.parametrize("field,value,code", [
    ("dim", 4, -1), ("voxelize", 7, -1), ("n_regions", 0, -1), ("n_regions", 17, -1),
    ("h0", 0.0, -1), ("h0", float("nan"), -1), ("n0", 0, -1), ("nvox", None, -2),
    ("semi", -1.0, -1), ("rsp", -0.5, -1)])
def test_phantom_validation(P, W, field, value, code):
    ph = W.c0()["phantom"]
    import copy
    ph = copy.deepcopy(ph)
    if field == "dim":
        ph["dim"] = value
    elif field == "voxelize":
        ph["voxelize"] = "center"
    elif field == "n_regions":
        ph["regions"] = [] if value == 0 else ph["regions"] * 4
    elif field == "h0":
        ph["h"][0] = value
    elif field == "n0":
        ph["n"][0] = value
    elif field == "nvox":
        ph["dim"] = 3
        ph["n"] = [2048, 2048, 1024]
        ph["h"] = [0.1, 0.1, 0.1]
    elif field == "semi":
        ph["regions"][1]["semi"][0] = value
    elif field == "rsp":
        ph["regions"][2]["rsp"] = value
    p, keep = P.make_phantom(ph)
    if field == "voxelize":
        p.voxelize = value
    if field == "dim":
        p.dim = value
    assert P.lib().pct_phantom_build(C.byref(p), C.c_void_p(0), C.c_void_p(0)) == code
    js = P.JobSet()
    js.add(ph, W.c0()["beam"], None)
    n, arr = js.array()
    if field in ("voxelize", "dim"):
        arr[0].phantom.contents.voxelize = p.voxelize
        arr[0].phantom.contents.dim = p.dim
    assert P.lib().pct_workspace_bytes(n, arr) == 0


@pytest.mark.parametrize("field,value", [
    ("n_angles", 0), ("n_protons", -1), ("row_count", 10**9), ("row_begin", -5),
    ("t_range", [1.0, -1.0]), ("sigma_in", -0.1), ("rho", 1.5), ("noise_rel", -0.01),
    ("step", 0.0), ("path", "spiral"), ("sigma_out", float("inf")), ("scatter", 7),
    ("energy_mev", 0.5), ("energy_mev", 2e4), ("x0_mm", 0.0), ("x0_mm", float("nan"))])
def test_beam_validation(P, W, field, value):
    import copy
    cfg = W.c1()
    bm = copy.deepcopy(cfg["beam"])
    row_begin, row_count = 0, None
    if field == "row_count":
        row_count = value
    elif field == "row_begin":
        row_begin = value
    elif field in ("path", "scatter"):
        bm["path"] = "straight"
    else:
        bm[field] = value
        if field in ("energy_mev", "x0_mm"):
            bm["scatter"] = "highland"
    js = P.JobSet()
    js.add(cfg["phantom"], bm, None, row_begin=row_begin, row_count=row_count)
    n, arr = js.array()
    if field == "path":
        arr[0].beam.contents.path = 9
    if field == "scatter":
        arr[0].beam.contents.scatter = value
    assert P.lib().pct_workspace_bytes(n, arr) == 0
    # the entry points reject it on the host, before anything is enqueued
    assert P.lib().pct_count_rows(n, arr, None, 1 << 30, None, None) == -1


def test_job_validation(P, W):
    cfg = W.c0()
    js = P.JobSet()
    js.add(cfg["phantom"], cfg["beam"], None)
    n, arr = js.array()
    arr[0].val_dtype = 5
    assert P.lib().pct_workspace_bytes(n, arr) == 0
    arr[0].val_dtype = 0
    arr[0].precision = 3
    assert P.lib().pct_workspace_bytes(n, arr) == 0
    arr[0].precision = 0
    arr[0].nnz_capacity = -1
    assert P.lib().pct_workspace_bytes(n, arr) == 0
    arr[0].nnz_capacity = 0
    for bad in (-1.0, float("nan"), float("inf")):
        arr[0].chord_mm = bad
        assert P.lib().pct_workspace_bytes(n, arr) == 0
    arr[0].chord_mm = 1.0
    assert P.lib().pct_workspace_bytes(n, arr) > 0
    arr[0].chord_mm = 0.0
    # emit needs row_ptr; wepl needs b (and x)
    assert P.lib().pct_emit_csr(n, arr, None, 1 << 30, None) == -1
    assert P.lib().pct_wepl(n, arr, None, 1 << 30, None) == -1
    # precision must agree across the jobs of one call
    js2 = P.JobSet()
    js2.add(cfg["phantom"], cfg["beam"], None)
    js2.add(cfg["phantom"], cfg["beam"], None, precision="plain_f32")
    n2, arr2 = js2.array()
    assert P.lib().pct_workspace_bytes(n2, arr2) == 0
    # a workspace that is missing or too small is refused before any launch
    import torch
    on_gpu = torch.cuda.is_available()
    dev = (lambda nbytes: torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")) if on_gpu else None
    keep = []

    def ptr(nbytes):
        if dev is None:
            return C.c_void_p(1 << 20)  # never dereferenced: no device in this process
        t = dev(nbytes)
        keep.append(t)
        return C.c_void_p(t.data_ptr())

    js3 = P.JobSet()
    js3.add(cfg["phantom"], cfg["beam"], None)
    n3, arr3 = js3.array()
    arr3[0].row_ptr_dev = ptr(8 * 92161).value
    need = P.lib().pct_workspace_bytes(n3, arr3)
    nnz = ptr(8)
    assert P.lib().pct_count_rows(n3, arr3, ptr(need - 1), need - 1, nnz, None) == -4
    assert P.lib().pct_count_rows(n3, arr3, None, need, nnz, None) == -4


def test_wepl_static_limits_on_host(P, W):
    """pct_wepl_static refuses, before touching the device: jobs without b or x
    (PCT_EINVAL), more than 64 jobs or more rows than its 64 MiB scratch holds
    (PCT_ESCRATCH)."""
    fake = 1 << 20   # never dereferenced: every case below is refused on the host
    cfg = W.c1()     # 2,949,120 rows: about 1.1 GB of workspace
    js = P.JobSet()
    js.add(cfg["phantom"], cfg["beam"], None)
    n, arr = js.array()
    assert P.lib().pct_wepl_static(n, arr, None, None) == P.PCT_EINVAL   # no b, no x
    arr[0].x_dev = fake
    arr[0].b_dev = fake
    assert P.lib().pct_workspace_bytes(n, arr) > (64 << 20)
    assert P.lib().pct_wepl_static(n, arr, None, None) == P.PCT_ESCRATCH
    small = W.scaled(W.c0(), n_protons=90)
    js2 = P.JobSet()
    for _ in range(65):
        js2.add(small["phantom"], small["beam"], None)
    n2, arr2 = js2.array()
    for k in range(n2):
        arr2[k].x_dev = fake
        arr2[k].b_dev = fake
    assert P.lib().pct_wepl_static(n2, arr2, None, None) == P.PCT_ESCRATCH


def test_launch_config_host_side(P):
    """pct_set/get_launch_config are host-only: valid values round-trip, others are refused
    and leave the configuration unchanged; NULL restores the default."""
    lib = P.lib()
    cfg = P.LaunchConfig()
    assert lib.pct_get_launch_config(C.byref(cfg)) == 0
    assert lib.pct_get_launch_config(None) == -1
    for rpw in (16, 32, 64):
        for order in (P.PCT_ORDER_GIVEN, P.PCT_ORDER_LPT):
            for bpc in (0, 1, 4, 8):
                assert lib.pct_set_launch_config(C.byref(P.LaunchConfig(rpw, order, bpc))) == 0
                got = P.LaunchConfig()
                lib.pct_get_launch_config(C.byref(got))
                assert (got.rows_per_wave, got.order, got.blocks_per_cu) == (rpw, order, bpc)
    before = P.LaunchConfig()
    lib.pct_get_launch_config(C.byref(before))
    for bad in ((0, 1, 0), (48, 1, 0), (128, 0, 0), (64, 2, 0), (64, -1, 0), (64, 1, -1), (64, 1, 9)):
        assert lib.pct_set_launch_config(C.byref(P.LaunchConfig(*bad))) == -1
        now = P.LaunchConfig()
        lib.pct_get_launch_config(C.byref(now))
        assert (now.rows_per_wave, now.order, now.blocks_per_cu) == \
            (before.rows_per_wave, before.order, before.blocks_per_cu)
    assert lib.pct_set_launch_config(None) == 0
    lib.pct_get_launch_config(C.byref(cfg))
    assert (cfg.rows_per_wave, cfg.order, cfg.blocks_per_cu) == (64, P.PCT_ORDER_LPT, 0)


def test_graph_and_autotune_validate_on_host(P, W):
    """Both refuse bad arguments before any HIP call (no GPU needed)."""
    lib = P.lib()
    cfg = W.c0()
    js = P.JobSet()
    js.add(cfg["phantom"], cfg["beam"], None)
    n, arr = js.array()
    h = C.c_void_p()
    # no row_ptr: the count pass cannot run
    assert lib.pct_graph_create(n, arr, 0, None, 1 << 30, None, C.byref(h)) == -1
    assert h.value is None
    assert lib.pct_graph_create(n, arr, 0, None, 1 << 30, None, None) == -1
    best = P.LaunchConfig()
    assert lib.pct_autotune(n, arr, None, 1 << 30, None, None, C.byref(best)) == -1
    assert lib.pct_autotune(n, arr, None, 1 << 30, None, None, None) == -1
    # a bad descriptor is refused the same way
    arr[0].val_dtype = 7
    arr[0].row_ptr_dev = 1 << 20
    assert lib.pct_graph_create(n, arr, 0, None, 1 << 30, C.c_void_p(1 << 20), C.byref(h)) == -1
    assert lib.pct_graph_launch(None, None) == -1
    assert lib.pct_graph_destroy(None) == 0


def test_sap_validation_on_host(P):
    """Descriptor checks of the SAP entry points happen before any launch."""
    A = P.Csr(n_rows=10, n_cols=5, val_dtype=0, nnz=30, row_ptr_dev=1 << 20, cols_dev=1 << 21,
              vals_dev=1 << 22, b_dev=1 << 23)
    p = P.SapParams(n_strings=3, relax=0.5)
    L = P.lib()
    need = L.pct_sap_workspace_bytes(C.byref(A), C.byref(p))
    # header + 10 coefficients + 3 weights + 3 x 5 string iterates, 256-byte aligned parts
    assert need == 256 + 256 + 256 + 3 * 5 * 4
    for field, bad in (("n_cols", 0), ("n_cols", 1 << 29), ("n_rows", -1), ("val_dtype", 7), ("nnz", -1)):
        B = P.Csr.from_buffer_copy(A)
        setattr(B, field, bad)
        assert L.pct_sap_workspace_bytes(C.byref(B), C.byref(p)) == 0, field
    for relax in (0.0, 2.0, -1.0, float("nan")):
        q = P.SapParams(n_strings=3, relax=relax)
        assert L.pct_sap_workspace_bytes(C.byref(A), C.byref(q)) == 0
    assert L.pct_sap_workspace_bytes(C.byref(A), C.byref(P.SapParams(n_strings=0, relax=0.5))) == 0
    for w in ([0.5, 0.5, 0.5], [1.0, 0.5, -0.5], [float("nan"), 0.5, 0.5]):
        arr = (C.c_double * 3)(*w)
        q = P.SapParams(n_strings=3, relax=0.5, weights=C.cast(arr, C.POINTER(C.c_double)))
        assert L.pct_sap_workspace_bytes(C.byref(A), C.byref(q)) == 0
    arr = (C.c_double * 3)(0.2, 0.3, 0.5)
    q = P.SapParams(n_strings=3, relax=0.5, weights=C.cast(arr, C.POINTER(C.c_double)))
    assert L.pct_sap_workspace_bytes(C.byref(A), C.byref(q)) == need
    # missing or short workspace, bad iteration count: refused on the host
    assert L.pct_sap_prepare(C.byref(A), C.byref(p), None, need, None) == -4
    assert L.pct_sap_prepare(C.byref(A), C.byref(p), C.c_void_p(1 << 20), need - 1, None) == -4
    assert L.pct_sap_iterate(C.byref(A), C.byref(p), C.c_void_p(1 << 24), -1, C.c_void_p(1 << 20), need,
                             None) == -1
    assert L.pct_sap_iterate(C.byref(A), C.byref(p), None, 1, C.c_void_p(1 << 20), need, None) == -1
    B = P.Csr.from_buffer_copy(A)
    B.b_dev = None
    assert L.pct_sap_prepare(C.byref(B), C.byref(p), C.c_void_p(1 << 20), need, None) == -1


def test_csr_file_reader_follows_layout(P, tmp_path):
    """A file laid out by hand as the header documents reads back through read_csr."""
    rng = np.random.default_rng(1)
    m, n = 7, 11
    counts = rng.integers(0, 5, m)
    rp = np.concatenate([[0], np.cumsum(counts)]).astype("<i8")
    nnz = int(rp[-1])
    cols = rng.integers(0, n, nnz).astype("<i4")
    vals = rng.uniform(0, 2, nnz).astype(np.float16)
    b = rng.uniform(0, 100, m).astype("<f4")
    al = lambda v: (v + 63) // 64 * 64
    o_rp = 128
    o_c = al(o_rp + 8 * (m + 1))
    o_v = al(o_c + 4 * nnz)
    o_b = al(o_v + 2 * nnz)
    end = o_b + 4 * m
    buf = bytearray(end)
    buf[0:8] = b"PCTCSR01"
    buf[8:32] = np.array([m, n, nnz], "<i8").tobytes()
    buf[32:40] = np.array([1, 1], "<i4").tobytes()
    buf[40:80] = np.array([o_rp, o_c, o_v, o_b, 0], "<i8").tobytes()
    buf[o_rp:o_rp + 8 * (m + 1)] = rp.tobytes()
    buf[o_c:o_c + 4 * nnz] = cols.tobytes()
    buf[o_v:o_v + 2 * nnz] = vals.tobytes()
    buf[o_b:o_b + 4 * m] = b.tobytes()
    f = tmp_path / "sys.pctcsr"
    f.write_bytes(bytes(buf))
    for mm in (True, False):
        r = P.read_csr(str(f), mmap=mm)
        assert (r["n_rows"], r["n_cols"], r["nnz"], r["val_dtype"], r["version"]) == (m, n, nnz, "f16", 1)
        assert np.array_equal(r["row_ptr"], rp) and np.array_equal(r["cols"], cols)
        assert np.array_equal(r["vals"], vals) and np.array_equal(r["b"], b) and r["x"] is None
    (tmp_path / "bad").write_bytes(b"NOTACSR!" + bytes(120))
    with pytest.raises(ValueError):
        P.read_csr(str(tmp_path / "bad"))


def test_csr_write_validation_on_host(P):
    A = P.Csr(n_rows=3, n_cols=4, val_dtype=0, nnz=5, row_ptr_dev=1 << 20, cols_dev=1 << 21, vals_dev=1 << 22)
    L = P.lib()
    assert L.pct_csr_write(None, C.byref(A), None, None) == -1
    for field, bad in (("n_cols", 0), ("n_rows", -1), ("val_dtype", 3), ("nnz", -2), ("row_ptr_dev", None)):
        B = P.Csr.from_buffer_copy(A)
        setattr(B, field, bad)
        assert L.pct_csr_write(b"/nonexistent/x", C.byref(B), None, None) == -1, field
