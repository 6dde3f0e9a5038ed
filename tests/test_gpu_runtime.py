"""Batch runtime on the GPU: HIP-graph replay of a sweep launch and the
workgroup-shape autotuner, both checked to leave the chains bit-identical
(to eager launches and to the CPU oracle)."""
import numpy as np
import pytest

from test_gpu_parity import SEED, _assert_same, _gpu, _oracle_run, _say, _uneven_instances

pytestmark = pytest.mark.gpu


def _state_all(b):
    return [b.state(n) for n in range(b.n)]


def test_graph_replay_matches_eager_launches():
    """Three replays of a captured 40-sweep launch, with eager work and a
    synchronisation between replays, equal three eager pt_sweep(40) calls
    after every replay; the final state equals the oracle's."""
    import torch
    hs = _gpu()
    insts = _uneven_instances()[:8]
    a = hs.PTBatch(insts, SEED, swap_interval=2)
    b = hs.PTBatch(insts, SEED, swap_interval=2)
    g = b.graph(40)
    for rep in range(3):
        _say(f"graph replay {rep}")
        a.sweep(40)
        g.launch()
        torch.cuda.synchronize()
        # eager work on the same stream between replays
        _ = (b.energy.float() * 2).sum().item()
        sa, sb = _state_all(a), _state_all(b)
        for n, (x, y) in enumerate(zip(sa, sb)):
            for k in x:
                assert np.array_equal(np.asarray(x[k]), np.asarray(y[k])), f"replay {rep}, instance {n}, {k}"
    assert b.measure() == 0
    for n in (0, 3, 7):
        o = _oracle_run(insts[n], SEED, 2, 120)
        _assert_same(b.state(n), o, f"instance {n} after graph replays")
    g.close()
    a.close()
    b.close()


def test_empty_graph():
    hs = _gpu()
    b = hs.PTBatch([], SEED, swap_interval=1)
    g = b.graph(10)
    g.launch()
    g.close()
    b.close()


def test_autotuner_picks_a_candidate_and_results_are_unchanged():
    """pt_autotune returns one of its candidate shapes; a batch run with that
    shape matches the oracle (tuning runs on scratch buffers only)."""
    hs = _gpu()
    insts = _uneven_instances()[:10]
    bw, us = hs.autotune(insts, SEED, swap_interval=1, trial_sweeps=40)
    _say(f"autotune: block_waves={bw}, {us:.1f} us/sweep")
    assert bw in (2, 4, 8, 16)
    assert us > 0
    b = hs.PTBatch(insts, SEED, swap_interval=1, block_waves=bw)
    b.sweep(60)
    assert b.measure() == 0
    for n in range(len(insts)):
        _assert_same(b.state(n), _oracle_run(insts[n], SEED, 1, 60), f"instance {n}")
    b.close()
