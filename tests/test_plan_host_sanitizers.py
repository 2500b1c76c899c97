"""The host-side plan builder (basis enumeration, ranking codes and tables,
tile lists, serving maps) under AddressSanitizer and UndefinedBehaviorSanitizer.

Compiles plan.cpp host-only with tests/host/plan_checks.cpp (hipcc, the
sanitizers on the host pass only) and runs it: no memory or UB report, and
every doubled basis monomial ranks inside the coefficient range.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2410_19844_amd", "csrc")


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def test_plan_builder_under_sanitizers(tmp_path):
    cc = _hipcc()
    if cc is None:
        pytest.skip("hipcc not found")
    exe = str(tmp_path / "plan_checks")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    cmd = [cc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, *san,
           os.path.join(HERE, "host", "plan_checks.cpp"), os.path.join(CSRC, "plan.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0, (run.stdout + run.stderr)[-3000:]
    assert "bad ranks 0 bad tiles 0" in run.stdout
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr
