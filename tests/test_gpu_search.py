"""The instance search driver (Algorithm 1) on the GPU engine: every
acceptance decision of the forward and the reversed search (Sec. II.B) is
the oracle's test on +-ln TTS, and the chain state follows the decisions;
the surrogate-screened arm runs end to end (screen, PT scoring, training)."""
import math

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1605_03607_amd as hs
    hs.lib()
    return hs


def _run(mode, direction, steps=3, chains=4):
    hs = _gpu()
    from paper_1605_03607_amd import search as S
    cfg = S.SearchConfig(mode=mode, chains=chains, L=2, restarts=4, K=8, R=2, s_max=3000, proposals=6,
                         top=2, train_steps=2, train_batch=4, direction=direction)
    seeds = [workloads.couplings(2, "pm1", 31, c) for c in range(chains)]
    params = workloads.gnn_params(hs.lib().gnn_param_count(), hs.gnn_fan_ins())
    run = S.Search(cfg, seeds, surrogate_params=params if mode == "surrogate" else None)
    start = run.ln.copy()
    for _ in range(steps):
        run.run_step(bars=(math.log(1.5),))
    return cfg, run, start


@pytest.mark.parametrize("mode,direction", [("plain", 1), ("plain", -1), ("surrogate", 1), ("random", -1)])
def test_decisions_follow_the_acceptance_rule(mode, direction):
    cfg, run, start = _run(mode, direction)
    assert len(run.decisions) == 3 * cfg.chains
    cur = {ch: start[ch] for ch in range(cfg.chains)}
    for step, ch, ln_cur, ln_new, w, ok in run.decisions:
        assert ln_cur == cur[ch]
        assert ok == oracle.rao_accept(direction * ln_cur, direction * ln_new, cfg.t_s, w)
        if ok:
            cur[ch] = ln_new
    assert all(run.ln[ch] == cur[ch] for ch in range(cfg.chains))
    # counted states are accepted ones on the right side of the bar
    kept = [d for d in run.decisions if d[5] and direction * (d[3] - run.h0) >= math.log(1.5)]
    assert len(run.hard.get(math.log(1.5), set())) <= len(kept)
    if kept:
        assert len(run.hard[math.log(1.5)]) >= 1
