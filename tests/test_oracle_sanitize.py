"""The oracle under the address and undefined-behaviour sanitizers (CPU).

tests/oracle_sanitize_main.c drives every oracle entry point (phantom build with the
three pixel rules, straight, curved and Highland rows in 2D and 3D, a 1 x 1 grid, rows
that miss the grid, arbitrary segments, SAP with orders, weights and more strings than
rows); built with gcc and both sanitizers, it must run to the end with no report
(leaks included).
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fno-sanitize-recover=all",
             "-fsanitize=address", "-fsanitize=undefined"]
    subprocess.run(["gcc", *flags, "-I", os.path.join(ROOT, "oracle"), os.path.join(HERE, "oracle_sanitize_main.c"),
                    "-o", exe, "-lm"], check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "entries" in r.stdout
