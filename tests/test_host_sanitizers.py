"""The library's host C++ (argument validation, the fusion planner and its JSON description,
plan choice, layouts, error paths) under AddressSanitizer and UndefinedBehaviorSanitizer.

The library is rebuilt with the host compilation instrumented (the kernels as usual) and the
CPU-side suites that call through the C ABI without a GPU -- the ABI checks, the plan
emulation, the plan choice and the density-matrix circuit builder -- run against it in a child process that preloads the ASan runtime.  Any report
aborts the child, so the test fails with the sanitizer's stack trace in its output.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_abi_and_planner_under_host_sanitizers(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_1412_2293_amd import build
    lib = build.build(sanitize=True)
    env = dict(os.environ)
    # the ASan runtime must come first; whatever the environment already preloads stays after it
    preload = build.asan_runtime()
    if env.get("LD_PRELOAD"):
        preload += ":" + env["LD_PRELOAD"]
    env.update({
        "LD_PRELOAD": preload,
        "ASAN_OPTIONS": "detect_leaks=0:verify_asan_link_order=0:abort_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
        "QSIM_TEST_LIB": lib,
        "PYTHONDONTWRITEBYTECODE": "1",
    })
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
           os.path.join(ROOT, "tests", "test_abi.py"), os.path.join(ROOT, "tests", "test_plan_emulation.py"),
           os.path.join(ROOT, "tests", "test_autotune.py"), os.path.join(ROOT, "tests", "test_dm_superop.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-6000:] + r.stderr[-6000:]
    assert r.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out
