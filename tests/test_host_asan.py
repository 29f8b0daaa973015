"""The host side of the library (planning, the level scheduler's host work,
the request loop against its simulated device, the autotuner's table, the
C ABI's argument checks) under AddressSanitizer: the *.cpp sources built
instrumented into libffp_asan.so, and the host test modules run against it
in a child process with the sanitizer runtime preloaded.  Any sanitizer
report fails the run."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_TESTS = ["tests/test_plan_sim.py", "tests/test_host_lib.py", "tests/test_serve_sim.py",
              "tests/test_tune_host.py", "tests/test_complex_plan.py", "tests/test_schedule_levels.py"]


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm*/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_host_code_under_address_sanitizer():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime in this ROCm install")
    from paper_2001_04109_amd import build
    lib = build.build_host_asan()
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_report_load" in syms, "the host sources were not instrumented"
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, LD_LIBRARY_PATH=os.path.dirname(rt) + ":" + env.get("LD_LIBRARY_PATH", ""),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1", FFP_LIBRARY=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", *HOST_TESTS, "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu"], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
