"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): tests/oracle_sanitize_driver.c runs every oracle entry point on
200 random small graphs; any out-of-bounds access, leak, overflow or failed
call ends the run with an error."""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def test_oracle_is_clean_under_sanitizers(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not found")
    exe = tmp_path / "drv"
    build = subprocess.run([cc, "-O1", "-g", "-std=c11", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                            str(ROOT / "tests" / "oracle_sanitize_driver.c"), str(ROOT / "oracle" / "oracle.c"),
                            "-o", str(exe), "-lm"], capture_output=True, text=True, timeout=120)
    if build.returncode != 0:
        pytest.skip(f"no sanitizer runtime for gcc: {build.stderr[-300:]}")
    env = dict(os.environ)
    # another library may be preloaded into every process; the check does
    # not need the sanitizer's runtime to come first
    env["ASAN_OPTIONS"] = "verify_asan_link_order=0:detect_leaks=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert "fails 0" in run.stdout
