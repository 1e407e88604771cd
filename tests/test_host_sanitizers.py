"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the C
oracle (tests/oracle_sanitize_driver.c: every entry point on 200 random
small graphs), the graph generators (tests/graphgen_sanitize_driver.cpp:
each generator at small and degenerate sizes, then weights and sources)
and the OpenMP CPU baseline (tests/cpubase_sanitize_driver.c: transpose,
pull PageRank and BFS on 100 random small graphs).
Any out-of-bounds access, leak, undefined operation or malformed result
ends the run with an error."""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
FLAGS = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"]


def _env():
    env = dict(os.environ)
    # another library may be preloaded into every process; the check does
    # not need the sanitizer's runtime to come first
    env["ASAN_OPTIONS"] = "verify_asan_link_order=0:detect_leaks=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "4"
    return env


def _build_and_run(compiler, std, sources, exe, extra=()):
    cc = shutil.which(compiler)
    if cc is None:
        pytest.skip(f"{compiler} not found")
    build = subprocess.run([cc, *FLAGS, f"-std={std}", *extra, *map(str, sources), "-o", str(exe), "-lm"],
                           capture_output=True, text=True, timeout=180)
    if build.returncode != 0:
        pytest.skip(f"no sanitizer runtime for {compiler}: {build.stderr[-300:]}")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=_env())
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert "fails 0" in run.stdout


def test_oracle_is_clean_under_sanitizers(tmp_path):
    _build_and_run("gcc", "c11", [ROOT / "tests" / "oracle_sanitize_driver.c", ROOT / "oracle" / "oracle.c"],
                   tmp_path / "oracle_drv")


def test_generators_are_clean_under_sanitizers(tmp_path):
    _build_and_run("g++", "c++17", [ROOT / "tests" / "graphgen_sanitize_driver.cpp", ROOT / "graphgen" / "gen.cpp"],
                   tmp_path / "graphgen_drv", extra=("-fopenmp",))


def test_cpu_baseline_is_clean_under_sanitizers(tmp_path):
    _build_and_run("gcc", "gnu11", [ROOT / "tests" / "cpubase_sanitize_driver.c", ROOT / "cpubase" / "cpubase.c"],
                   tmp_path / "cpubase_drv", extra=("-fopenmp",))
