"""The benchmark on the CPU: it measures one GPU only and says so for more; its energy-distribution
comparison equals the textbook two-sample statistics."""
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


def test_energy_deviation_matches_the_textbook_two_sample_statistics():
    """The KS statistic of the bench's energy comparison equals scipy's two-sample KS statistic;
    the mean difference is in units of its standard error."""
    import numpy as np
    from scipy import stats

    import bench

    rng = np.random.default_rng(3)
    for a, b in [(rng.normal(0, 1, 500), rng.normal(0.1, 1.2, 700)),
                 (rng.integers(-40, 0, 300).astype(float), rng.integers(-42, 2, 256).astype(float))]:
        d = bench.energy_deviation(a, b)
        assert abs(d["ks"] - stats.ks_2samp(a, b).statistic) < 1e-12
        se = np.sqrt(a.var(ddof=1) / a.size + b.var(ddof=1) / b.size)
        assert abs(d["mean_diff_se_units"] - (a.mean() - b.mean()) / se) < 1e-9
