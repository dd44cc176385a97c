"""The oracle and the GPU path share nothing, and the product has no CPU fallback (CPU).

- Importing the product package (binding, workloads, build) loads no module of the
  oracle; importing the oracle loads nothing of the product package.
- No source of either side includes or names a file of the other.
- With the HIP library absent, the binding raises instead of computing anything.
"""
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _modules_after(imports):
    code = ("import sys; sys.path.insert(0, %r)\n%s\n"
            "print('\\n'.join(sorted(m for m in sys.modules)))" % (ROOT, imports))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    return set(r.stdout.split())


def test_product_package_does_not_load_the_oracle():
    mods = _modules_after("from paper_2108_12369_amd import pct, workloads, build")
    assert not any(m == "oracle" or m.startswith("oracle.") for m in mods)


def test_oracle_does_not_load_the_product_package():
    mods = _modules_after("from oracle import oracle")
    assert not any(m.startswith("paper_2108_12369_amd") for m in mods)


def _sources(top, exts):
    for dp, _, fns in os.walk(os.path.join(ROOT, top)):
        if "__pycache__" in dp:
            continue
        for fn in fns:
            if fn.endswith(exts):
                yield os.path.join(dp, fn)


def test_no_source_names_the_other_side():
    for f in _sources("paper_2108_12369_amd", (".hip", ".h", ".py")):
        text = open(f).read()
        assert not re.search(r"^\s*(from|import)\s+oracle\b", text, re.M), f
        assert "pct_oracle" not in text and "liboracle" not in text, f
    for f in _sources("oracle", (".c", ".h", ".py")):
        text = open(f).read()
        assert "paper_2108_12369_amd" not in text and "pct.h" not in text and "libpct" not in text, f
        assert not re.search(r'#include\s+"', text), f   # system headers only


def test_binding_raises_without_the_library(tmp_path):
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2108_12369_amd import pct as P\n"
            "P.LIB_PATH = %r\n"
            "try:\n    P.lib()\nexcept RuntimeError as e:\n    print('raised', e)\n" % (ROOT, str(tmp_path / "libpct.so")))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.startswith("raised") and "missing" in r.stdout
