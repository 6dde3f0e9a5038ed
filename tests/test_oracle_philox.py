"""Pins for the oracle's Philox4x32-10: published known-answer vectors and an
independent third-party implementation (rocRAND's host engine)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat_rows():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,want", _kat_rows())
def test_known_answer_vectors(ctr, key, want):
    assert oracle.philox(ctr, key).tolist() == want


def _rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("rocRAND headers / hipcc not available")
    src = os.path.join(HERE, "support", "rocrand_philox_ref.cpp")
    out_dir = os.path.join(HERE, "support", "_build")
    os.makedirs(out_dir, exist_ok=True)
    exe = os.path.join(out_dir, "rocrand_philox_ref")
    if not os.path.exists(exe) or os.path.getmtime(exe) < os.path.getmtime(src):
        subprocess.run([hipcc, "-O1", "-o", exe, src], check=True, capture_output=True)
    return exe


def test_matches_rocrand_on_random_inputs():
    exe = _rocrand_ref()
    rng = np.random.default_rng(11)
    vals = rng.integers(0, 2 ** 32, size=(2000, 6), dtype=np.uint64)
    # include the counter patterns the method uses (small sweep / site / slot words)
    vals[:500, 0] = np.arange(500)
    vals[:500, 1] = rng.integers(0, 300, 500)
    vals[:500, 2] = rng.integers(0, 1 << 14, 500)
    vals[:500, 3] = rng.integers(0, 8, 500)
    text = "\n".join(" ".join(f"{int(x):08x}" for x in row) for row in vals)
    res = subprocess.run([exe], input=text, capture_output=True, text=True, check=True)
    ref = [[int(x, 16) for x in line.split()] for line in res.stdout.strip().splitlines()]
    for row, want in zip(vals, ref):
        got = oracle.philox(row[:4].astype(np.uint32), row[4:6].astype(np.uint32)).tolist()
        assert got == want
    assert len(ref) == len(vals)


def test_output_bits_uniform():
    """Sanity: over 2^16 counters each output bit is set about half the time."""
    n = 1 << 14
    outs = np.array([oracle.philox([i, 3, 5, 0], [1605, 42]) for i in range(n)], np.uint64)
    bits = (outs[:, :, None] >> np.arange(32, dtype=np.uint64)) & np.uint64(1)
    freq = bits.mean(axis=0)
    assert np.all(np.abs(freq - 0.5) < 5 * 0.5 / np.sqrt(n))
