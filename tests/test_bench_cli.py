"""Host-side checks of the benchmark's command line (no GPU needed): one
GPU is the only configuration it measures, and it says so for any other."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*argv):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv],
                          capture_output=True, text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_the_workloads():
    r = _run("--help")
    assert r.returncode == 0
    for w in ("grid", "tex2d", "shade", "neural", "serving", "dct", "gauss", "ewa"):
        assert w in r.stdout
    assert "--cpu-seconds" in r.stdout
