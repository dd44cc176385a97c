"""MI355X-native hot path of the proton-CT data simulator (arXiv 2108.12369).

`pct` is the ctypes binding of the HIP library libpct.so (C ABI in include/pct.h);
`workloads` lays out the seeded synthetic inputs; `build` compiles the library.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "pct", "build"]
