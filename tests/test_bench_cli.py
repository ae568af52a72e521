"""The benchmark's command line on the CPU: it measures one GPU only and says so for more."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""  # no JSON line for a run that did not happen


def test_help_lists_the_workloads_and_the_serving_child():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True, text=True,
                       timeout=60)
    assert p.returncode == 0
    for w in ("g2000", "d3_2000", "g2000_fp8s", "sk8192", "--serving-child"):
        assert w in p.stdout
