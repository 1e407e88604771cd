"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the C
oracle (tests/oracle_sanitize_driver.c: every entry point on 200 random
small graphs), the graph generators (tests/graphgen_sanitize_driver.cpp:
each generator at small and degenerate sizes, then weights and sources)
the OpenMP CPU baseline (tests/cpubase_sanitize_driver.c: transpose, pull
PageRank and BFS on 100 random small graphs) and the library's C ABI
argument checks (tests/abi_sanitize_driver.cpp, linked with the library's
sources built with host-only sanitizers; no GPU needed).
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



def test_abi_argument_checks_are_clean_under_sanitizers(tmp_path):
    hipcc = shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)
    if hipcc is None:
        pytest.skip("hipcc not found")
    import concurrent.futures
    csrc = ROOT / "paper_1904_02241_amd" / "csrc"
    # sanitizers on the host side only (each flag behind -Xarch_host)
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer"]
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
              "-packed-fp32-ops", "-I", str(ROOT / "include"), "-I", str(csrc), *host_san]
    sources = sorted(csrc.glob("*.hip")) + [ROOT / "tests" / "abi_sanitize_driver.cpp"]

    def compile_one(src):
        obj = tmp_path / (src.name + ".o")
        r = subprocess.run([hipcc, *common, "-c", str(src), "-o", str(obj)], capture_output=True, text=True,
                           timeout=600)
        return obj, r

    with concurrent.futures.ThreadPoolExecutor(max_workers=8) as ex:
        built = list(ex.map(compile_one, sources))
    for obj, r in built:
        if r.returncode != 0:
            pytest.skip(f"hipcc could not build {obj.name} with host sanitizers: {r.stderr[-300:]}")
    exe = tmp_path / "abi_drv"
    link = subprocess.run([hipcc, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                           "-fsanitize=undefined", *[str(o) for o, _ in built], "-o", str(exe)],
                          capture_output=True, text=True, timeout=300)
    if link.returncode != 0:
        pytest.skip(f"no host sanitizer runtime for hipcc: {link.stderr[-300:]}")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, env=_env())
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert "fails 0" in run.stdout
