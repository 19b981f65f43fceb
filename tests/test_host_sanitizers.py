"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
the parameter planner (every kernel, periodicity, window, pollution rule and
a spread of tolerances, boxes and sizes down to one source) and the oracle's
C routines (every kernel and periodicity on a small input with a coincident
pair), each built with -fsanitize=address,undefined and run to completion.
Device code is not built here."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
CSRC = os.path.join(ROOT, "paper_2210_01255_amd", "csrc")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


def _build_and_run(tmp_path, compiler, args, name):
    if shutil.which(compiler) is None:
        pytest.skip("%s not available" % compiler)
    exe = str(tmp_path / name)
    r = subprocess.run([compiler] + SAN + args + ["-o", exe], capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr + r.stdout).lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = run.stdout + run.stderr
    print(out[-1500:])
    assert run.returncode == 0, out[-3000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out and "LeakSanitizer" not in out
    return out


def test_planner_under_sanitizers(tmp_path):
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    out = _build_and_run(tmp_path, "g++", ["-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(rocm, "include"),
                                           "-I" + CSRC, os.path.join(HOST, "planner_check.cpp"),
                                           os.path.join(CSRC, "se_params.cpp")], "planner_check")
    assert "0 failures" in out


def test_oracle_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "gcc", ["-std=c11", "-Wno-unknown-pragmas", os.path.join(HOST, "oracle_check.c"),
                                           os.path.join(ROOT, "oracle", "ewald_oracle.c"),
                                           os.path.join(ROOT, "oracle", "reduced_oracle.c"), "-lm"], "oracle_check")
    assert "0 failures" in out
