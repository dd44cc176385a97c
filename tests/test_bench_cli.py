"""The benchmark's host-side contract (CPU): more than one GPU is refused with a message,
and the HBM traffic it reports comes from the committed profile summary only while the
kernels' source digest matches the one recorded there."""
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"] and msg["gpus_requested"] == 2


def _profiles():
    out = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "profiles"))):
        if not fn.endswith(".md"):
            continue
        kv = {}
        for line in open(os.path.join(ROOT, "profiles", fn)):
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                kv[k.strip()] = v.strip()
        if "kernel" in kv:
            out.append(kv)
    return out


def _profile(kernel, workload):
    for kv in _profiles():
        if kv.get("kernel") == kernel and kv.get("workload") == workload:
            return kv
    return None


def test_every_stored_traffic_is_the_scaled_counters():
    """Each profile summary's traffic is FETCH_SIZE and WRITE_SIZE (KiB per dispatch,
    summed over the emit call's kernels) times the copy calibration factors."""
    kvs = _profiles()
    assert {kv["workload"] for kv in kvs} >= {"c3-64-uneven-jobs-graph", "c1-2d-neo2-400sq-hermite"}
    for kv in kvs:
        kib = float(kv["fetch_kib_per_dispatch"]) * float(kv["copy_fetch_factor"]) + \
            float(kv["write_kib_per_dispatch"]) * float(kv["copy_write_factor"])
        got = float(kv["traffic_bytes_per_launch"])
        assert abs(kib * 1024 - got) <= 1e-6 * got + 2048, kv["workload"]
        assert 1.9 < float(kv["copy_fetch_factor"]) < 2.1 and 0.9 < float(kv["copy_write_factor"]) < 1.1


def test_traffic_follows_the_source_digest(monkeypatch):
    import bench
    from paper_2108_12369_amd import build as B
    kv = _profile("k_emit_wave", "c1-2d-neo2-400sq-hermite")
    assert kv is not None and "traffic_bytes_per_launch" in kv
    got = bench.stored_traffic("k_emit_wave", "c1-2d-neo2-400sq-hermite")
    if kv["source_digest"] == B.source_digest():
        assert got == float(kv["traffic_bytes_per_launch"])
        # the figure is the two counters scaled by the copy calibration
        kib = float(kv["fetch_kib_per_dispatch"]) * float(kv["copy_fetch_factor"]) + \
            float(kv["write_kib_per_dispatch"]) * float(kv["copy_write_factor"])
        assert abs(kib * 1024 - got) <= 1e-6 * got + 2048
    else:
        assert got is None
    monkeypatch.setattr(B, "source_digest", lambda: "0000000000000000")
    assert bench.stored_traffic("k_emit_wave", "c1-2d-neo2-400sq-hermite") is None
    assert bench.stored_traffic("k_emit_wave", "no-such-workload") is None
