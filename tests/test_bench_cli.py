"""Command-line contract of bench.py that needs no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    for extra in ((), ("--speedup",), ("--serve", "10")):
        r = _run("--gpus", "2", *extra)
        assert r.returncode == 2, (extra, r.stdout, r.stderr)
        assert "one GPU" in r.stderr
        assert r.stdout == ""


def test_help_lists_the_modes():
    r = _run("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--workload", "--speedup", "--serve", "--no-cpu-baseline"):
        assert flag in r.stdout
