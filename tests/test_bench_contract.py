"""The benchmark script's command-line contract, on the host: one GPU only,
every workload is offered, and the measurement helpers that need no GPU
(roofline object, CPU oracle samples, kernel fingerprint) are well formed."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    p = _bench("--gpus", "2")
    assert p.returncode != 0
    assert "one GPU" in json.loads(p.stdout.strip().splitlines()[-1])["error"]


def test_every_workload_is_offered():
    p = _bench("--help")
    assert p.returncode == 0
    for w in ("c8", "uneven", "search", "search-reverse", "surrogate", "tau", "lao", "overlap"):
        assert w in p.stdout


def test_roofline_object_and_fingerprint():
    sys.path.insert(0, ROOT)
    import bench
    r = bench.pt_roofline(attempts=10**12, kernel_ms=500.0, launches=2, kernel="k", wall_s=1.0)
    assert r["bound"] == "alu" and r["unit"].startswith("Tops/s")
    assert r["achieved"] == pytest.approx(1e12 * bench.A_OPS / 0.5 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"])
    assert r["kernel_ms_avg"] == 250.0 and r["chip_frac_over_wall"] == pytest.approx(1e12 * bench.A_OPS / bench.PEAK_INT32_OPS)
    fp = bench.kernel_fingerprint()
    assert isinstance(fp, str) and len(fp) == 16


def test_products_count_of_the_autocorrelation_sums():
    sys.path.insert(0, ROOT)
    import bench
    # sum over d = 0..M of (T - d), and lags beyond the run are empty
    assert bench._products(10, 3) == 10 + 9 + 8 + 7
    assert bench._products(4, 100) == 4 + 3 + 2 + 1
