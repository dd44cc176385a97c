"""Build the HIP library (libpct.so) in-tree for gfx950 with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpct.so")
SOURCES = [os.path.join(CSRC, "pct.hip"), os.path.join(CSRC, "sap.hip"), os.path.join(CSRC, "csr_io.hip")]
HEADERS = [os.path.join(CSRC, "pct_device.h"), os.path.join(CSRC, "pct_wave.h"),
           os.path.join(ROOT, "include", "pct.h")]

ARCH = os.environ.get("PCT_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # every multiply-add is written explicitly (fma); nothing is fused implicitly, so the
    # count and emit passes round identically
    "-ffp-contract=off",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return exe


def source_digest(part: str = "sim") -> str:
    """Short SHA-256 over device sources, the public header and the compiler flags:
    identifies the kernels a stored profile was taken from.  part "sim": the simulator
    (every header and .hip file but the reconstruction and the file writer); "sap": the
    reconstruction (sap.hip and the headers it includes)."""
    import hashlib
    if part == "sap":
        names = ["sap.hip", "pct_device.h", "pct_wave.h"]
    else:
        names = [f for f in os.listdir(CSRC) if f.endswith((".hip", ".h")) and f not in ("sap.hip", "csr_io.hip")]
    files = sorted(os.path.join(CSRC, f) for f in names)
    files += [os.path.join(ROOT, "include", "pct.h")]
    h = hashlib.sha256(" ".join(FLAGS).encode())
    for f in files:
        h.update(os.path.relpath(f, ROOT).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=HERE)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
