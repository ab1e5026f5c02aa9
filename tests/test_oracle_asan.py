"""The oracle's small-grid pins, run against an AddressSanitizer + UndefinedBehaviorSanitizer
build of the oracle (host code only; an out-of-bounds access, a use after free or undefined
behaviour aborts the run).

The sanitized library is built into a temporary folder and loaded by a child pytest process
(ORACLE_LIB names it; the ASan runtime is preloaded ahead of whatever the parent already
preloads, because ASan must come first).  The long relaxation pins (T13, the safety-factor
reject run) are left out: they repeat the same code paths for minutes.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    if shutil.which("gcc") is None:
        return None
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_small_pins_under_asan_and_ubsan(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("gcc's ASan runtime is not available")
    from oracle import build as oracle_build

    lib = oracle_build.build(sanitize=True, out=str(tmp_path / "liboracle_asan.so"))
    env = dict(os.environ)
    env["ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = rt + ((":" + os.environ["LD_PRELOAD"]) if os.environ.get("LD_PRELOAD") else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = env.get("OMP_NUM_THREADS", "4")
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-q", "-x",
           "-p", "no:cacheprovider", "-k", "not T13 and not T10_safety"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (r.stdout[-3000:] + r.stderr[-3000:])
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
