"""CPU: bench.py's command line (no GPU is touched: the checks run before torch is imported)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_help_lists_every_workload_mode():
    r = run("--help")
    assert r.returncode == 0
    for mode in ("--uneven", "--csim", "--interp", "--nonstat", "--mixture", "--universal", "--exact", "--accuracy",
                 "--convergence"):
        assert mode in r.stdout, mode
