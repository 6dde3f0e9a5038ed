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


def test_hardware_queue_count_is_bounded():
    """The search workloads set GPU_MAX_HW_QUEUES for their process; a count
    outside 1..32 is refused before anything touches the GPU."""
    for n in ("0", "33"):
        p = _bench("--workload", "search", "--hw-queues", n)
        assert p.returncode == 2
        assert "1..32" in json.loads(p.stdout.strip().splitlines()[-1])["error"]


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


def test_roofline_uses_the_committed_reference_op_count():
    """frac is reported at the reference op count fixed before tuning (22
    int32 lane operations per attempt, whose parts add up), with the
    implemented formulation's count (15.5) beside it, against the peak
    derived from the published fp32 vector figure."""
    sys.path.insert(0, ROOT)
    import bench
    with open(os.path.join(ROOT, "roofline_opcount.json")) as f:
        oc = json.load(f)
    for part in ("reference", "implemented"):
        assert sum(v["ops"] for v in oc[part]["parts"].values()) == oc[part]["ops_per_attempt"]
    assert bench.A_OPS == 22 and bench.A_OPS_IMPL == 15.5
    assert bench.PEAK_INT32_OPS == pytest.approx(157.3e12 / 2, rel=1e-3)
    r = bench.alu_roofline(1.46e12 * 0.5, 0.5)
    assert r["frac"] == pytest.approx(1.46e12 * 22 / bench.PEAK_INT32_OPS)
    assert r["frac_implemented_ops"] == pytest.approx(1.46e12 * 15.5 / bench.PEAK_INT32_OPS)


def test_cpu_baseline_records_the_host():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.host_info()
    assert h["host_nproc"] >= 1 and h["thread_cap"] == 16 and "16" in h["thread_cap_reason"]
