"""Planted-solution instances on the GPU engine (Sec. IV): parallel
tempering's ground-state energy (minimum over restarts) equals the planted
one, which pins hardness_eval's E_gs without brute force; and Loop Adaptive
Optimization's decisions follow the acceptance rule."""
import numpy as np
import pytest

import oracle
import oracle.lao as P
import workloads

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1605_03607_amd as hs
    hs.lib()
    return hs


@pytest.mark.parametrize("L,M", [(2, 14), (3, 40), (4, 70)])
def test_pt_finds_the_planted_ground_state(L, M):
    hs = _gpu()
    insts = [hs.lao_init(L, M, ch, 5) for ch in range(6)]
    beta = workloads.geometric_betas(0.1, 5.0, 16)
    cands = [dict(L=L, J=i["J"], live=None, instance_id=ch) for ch, i in enumerate(insts)]
    ln, det = hs.hardness_eval(cands, 8, 16, 2, beta, 1, 20_000, 3)
    for ch, (i, d) in enumerate(zip(insts, det)):
        assert oracle.energy(L, None, i["J"], i["bits"]) == i["e_gs"]
        assert d["e_gs"] == i["e_gs"], (ch, d["e_gs"], i["e_gs"])
        assert np.isfinite(ln[ch])


def test_lao_search_decisions_follow_the_rule():
    hs = _gpu()
    from paper_1605_03607_amd import search as S
    cfg = S.SearchConfig(mode="plain", chains=4, L=2, restarts=4, K=8, R=2, s_max=3000)
    run = S.LaoSearch(cfg, n_loops=14)
    start = run.ln.copy()
    for _ in range(3):
        run.run_step()
    cur = {ch: start[ch] for ch in range(4)}
    for step, ch, a, b, w, ok in run.decisions:
        assert a == cur[ch]
        assert ok == oracle.rao_accept(a, b, cfg.t_s, w)
        if ok:
            cur[ch] = b
    for ch in range(4):
        i = run.inst[ch]
        J, e = P.couplings(2, [tuple(r) for r in i["loops"].tolist()], P.cycles(2), i["bits"])
        assert np.array_equal(J.astype(np.int8), i["J"]) and e == i["e_gs"]
    assert run.scored == 4 + len(run.decisions) and run.voids == 12 - len(run.decisions)
    assert run.gs_found == run.scored


def test_grouped_lao_takes_the_same_decisions():
    hs = _gpu()
    from paper_1605_03607_amd import search as S
    cfg = S.SearchConfig(mode="plain", chains=5, L=2, restarts=4, K=8, R=2, s_max=3000)
    one = S.LaoSearch(cfg, n_loops=14)
    for _ in range(3):
        one.run_step()
    many = S.GroupedLao(cfg, n_loops=14, groups=2)
    many.run(3)
    assert many.decisions == sorted(one.decisions)
    assert np.array_equal(many.ln0, one.ln0) and np.array_equal(many.ln, one.ln)
    assert all(np.array_equal(a["J"], b["J"]) for a, b in zip(many.inst, one.inst))
    assert (many.scored, many.voids, many.accepted, many.gs_found) == (one.scored, one.voids, one.accepted,
                                                                        one.gs_found)


def test_lao_search_replays_on_the_oracle():
    """Algorithm 2 end to end on C3: the oracle's planted instances, loop
    moves, PT hardness and acceptance reproduce the GPU search's ln TTS,
    decisions, loops and planted energies over 4 steps."""
    hs = _gpu()
    from paper_1605_03607_amd import search as S
    L, chains, steps, n_loops = 3, 3, 4, 30
    cfg = S.SearchConfig(mode="plain", chains=chains, L=L, restarts=4, K=8, R=2, s_max=3000)
    run = S.LaoSearch(cfg, n_loops=n_loops)
    for _ in range(steps):
        run.run_step()
    cyc = P.cycles(L)

    def hard(J, ch):
        return oracle.hardness_eval(L, None, J, ch, cfg.seed, cfg.restarts, cfg.K, cfg.R, cfg.beta,
                                    cfg.swap_interval, cfg.s_max)
    want = []
    for ch in range(chains):
        print(f"LAO replay on the oracle: chain {ch}", flush=True)
        inst = P.init(L, n_loops, ch, cfg.seed, cyc=cyc)
        h = hard(inst["J"], ch)
        assert h["e_gs"] == inst["e_gs"] and h["ln_tts"] == run.ln0[ch]
        ln = h["ln_tts"]
        for k in range(steps):
            slot, lp, w, J2, e2 = P.move(L, inst, ch, cfg.seed, k, 0, cyc=cyc)
            if slot < 0:
                continue
            h2 = hard(J2, ch)
            assert h2["e_gs"] == e2
            ok = oracle.rao_accept(ln, h2["ln_tts"], cfg.t_s, w)
            want.append((k, ch, ln, h2["ln_tts"], w, ok))
            if ok:
                loops = list(inst["loops"])
                loops[slot] = lp
                inst = dict(loops=loops, bits=inst["bits"], J=J2, e_gs=e2)
                ln = h2["ln_tts"]
        assert np.array_equal(run.inst[ch]["J"], inst["J"]) and run.inst[ch]["e_gs"] == inst["e_gs"]
        assert [tuple(r) for r in run.inst[ch]["loops"].tolist()] == [tuple(x) for x in inst["loops"]]
        assert run.ln[ch] == ln
    assert sorted(want) == sorted(run.decisions)
