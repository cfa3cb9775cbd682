"""CPU checks under AddressSanitizer and UndefinedBehaviorSanitizer: the FP64
oracle (built with GCC's sanitizers) runs its entry points on small inputs,
and the host-side paths of the HIP library that need no device (built with
the sanitizers on its host pass only) run parameter validation, workspace
sizes and the saved-state checker on random and corrupted inputs.  Each runs
in its own process with its sanitizer runtime preloaded; any report fails."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
ENV_OPTS = "detect_leaks=0:alloc_dealloc_mismatch=0:abort_on_error=1"


def _run(script, lib, runtime):
    env = dict(os.environ)
    env["LD_PRELOAD"] = runtime
    env["ASAN_OPTIONS"] = ENV_OPTS
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "2"
    r = subprocess.run([sys.executable, os.path.join(HERE, script), lib], env=env,
                       capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_sanitizers():
    from oracle import build as ob
    lib = ob.build(sanitize=True)
    runtime = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True,
                             text=True, check=True).stdout.strip()
    assert os.path.exists(runtime)
    assert "oracle scenarios clean" in _run("oracle_scenarios.py", lib, runtime)


def _clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm*/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_host_paths_under_sanitizers():
    runtime = _clang_asan_runtime()
    if runtime is None:
        pytest.skip("no clang AddressSanitizer runtime in this ROCm install")
    from paper_2504_12858_amd import build as hb
    lib = hb.build(sanitize=True)
    assert "host paths clean" in _run("host_paths.py", lib, runtime)
