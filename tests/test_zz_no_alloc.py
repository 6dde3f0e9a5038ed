"""hardness_eval_static (the entry point with a static device scratch, for
callers that cannot allocate) against hardness_eval with a caller buffer:
identical ln TTS, ground-state energies, confirmation, censored counts and
per-restart sweeps, on two calls in a row (the second with fewer and smaller
candidates, so it runs on what the first left in the scratch); a batch
larger than the static scratch is refused before any work."""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1605_03607_amd as hs
    hs.lib()
    return hs


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cands(n, L, seed):
    return [dict(L=L, J=workloads.couplings(L, "pm7", seed, i), live=workloads.missing_mask(L, 0.04, seed, i),
                 instance_id=300 + i) for i in range(n)]


def _same(a, b, what):
    ln_a, det_a = a
    ln_b, det_b = b
    assert np.array_equal(ln_a, ln_b), what
    for x, y in zip(det_a, det_b):
        for k in ("e_gs", "confirmed", "n_censored", "sweeps_total"):
            assert x[k] == y[k], (what, k)
        assert np.array_equal(x["restart_sweeps"], y["restart_sweeps"]), what


def test_static_scratch_matches_caller_buffer_twice():
    hs = _gpu()
    beta = workloads.geometric_betas(0.1, 5.0, 8)
    for call, (n, L, restarts) in enumerate([(6, 4, 8), (3, 2, 5)]):
        cands = _cands(n, L, 41 + call)
        _say(f"no-alloc hardness: call {call}, {n} C{L} candidates x {restarts} restarts")
        want = hs.hardness_eval(cands, restarts, 8, 2, beta, 1, 3000, 77)
        got = hs.hardness_eval_static(cands, restarts, 8, 2, beta, 1, 3000, 77)
        _same(got, want, f"call {call}")
        assert all(np.isfinite(got[0]))


def test_static_scratch_refuses_a_batch_beyond_its_size():
    hs = _gpu()
    beta = workloads.geometric_betas(0.1, 5.0, 32)
    cands = _cands(96, 12, 5)
    hi = hs._HostInstances([dict(c, K=32, R=2, beta=beta) for c in cands])
    p = hs.hs_hardness_params(32, 32, 2, np.ascontiguousarray(beta).ctypes.data, 1, 10, 77, 0, None)
    nb = C.c_size_t(0)
    assert hs.lib().hardness_workspace_bytes(hi.arr, len(cands), C.byref(p), C.byref(nb)) == 0
    assert nb.value > hs.HS_STATIC_SCRATCH_BYTES
    with pytest.raises(hs.HardspinError) as e:
        hs.hardness_eval_static(cands, 32, 32, 2, beta, 1, 10, 77)
    assert e.value.code == -2
