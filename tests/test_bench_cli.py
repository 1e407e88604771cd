"""bench.py's command line on the CPU: it measures one GPU and says so,
before it touches torch or the library, when asked for more (by --gpus or
by a launcher's WORLD_SIZE)."""
import os
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def _run(args, env_extra=None):
    env = dict(os.environ)
    env.update(env_extra or {})
    return subprocess.run([sys.executable, str(ROOT / "bench.py"), *args], cwd=ROOT, env=env,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    assert "measures one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def test_launcher_world_size_is_refused():
    r = _run([], {"WORLD_SIZE": "4"})
    assert r.returncode == 2
    assert "measures one GPU" in r.stderr


def test_help_lists_the_suites():
    r = _run(["--help"])
    assert r.returncode == 0
    for suite in ("pagerank", "traversal", "batched", "learned", "ladder", "spmv", "bc"):
        assert suite in r.stdout
