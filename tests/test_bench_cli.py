"""Host-side behaviour of the benchmark and trace command lines (no GPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, *args], cwd=ROOT, capture_output=True, text=True, timeout=300)


def test_bench_refuses_more_than_one_gpu():
    r = _run("bench.py", "--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_bench_and_trace_cli_parse():
    r = _run("bench.py", "--help")
    assert r.returncode == 0 and "--second-config" in r.stdout and "--serve-rate" in r.stdout
    r = _run("-m", "paper_1810_03063_amd.serve_trace", "--help")
    assert r.returncode == 0 and "--mode" in r.stdout
