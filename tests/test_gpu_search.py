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


@pytest.mark.parametrize("mode", ["plain", "random"])
def test_grouped_search_takes_the_same_decisions(mode):
    """Chain groups on concurrent streams score each candidate exactly as
    one launch of all chains does (PT draws are keyed per chain and restart),
    so the grouped search repeats the single-group search decision for
    decision."""
    hs = _gpu()
    from paper_1605_03607_amd import search as S
    chains = 6
    cfg = S.SearchConfig(mode=mode, chains=chains, L=3, restarts=4, K=8, R=2, s_max=4000, proposals=5, top=2)
    seeds = [workloads.couplings(3, "pm1", 37, c) for c in range(chains)]
    one = S.Search(cfg, seeds)
    for _ in range(3):
        one.run_step(bars=(math.log(1.5),))
    many = S.GroupedSearch(cfg, seeds, groups=3)
    many.run(3, bars=(math.log(1.5),))
    assert many.h0 == one.h0
    assert many.decisions == sorted(one.decisions)
    assert np.array_equal(many.ln, one.ln)
    assert many.hard == one.hard


def test_grouped_surrogate_search_runs():
    hs = _gpu()
    from paper_1605_03607_amd import search as S
    chains = 6
    cfg = S.SearchConfig(mode="surrogate", chains=chains, L=2, restarts=4, K=8, R=2, s_max=3000, proposals=6,
                         top=2, train_steps=4, train_batch=4)
    seeds = [workloads.couplings(2, "pm1", 39, c) for c in range(chains)]
    params = workloads.gnn_params(hs.lib().gnn_param_count(), hs.gnn_fan_ins())
    many = S.GroupedSearch(cfg, seeds, groups=3, surrogate_params=params)
    start = many.ln.copy()
    many.run(3, bars=(math.log(1.5),))
    assert len(many.decisions) == 3 * chains
    cur = {ch: start[ch] for ch in range(chains)}
    for step, ch, ln_cur, ln_new, w, ok in many.decisions:
        assert ln_cur == cur[ch]
        assert ok == oracle.rao_accept(ln_cur, ln_new, cfg.t_s, w)
        if ok:
            cur[ch] = ln_new
    assert all(many.ln[ch] == cur[ch] for ch in range(chains))
    assert many.pool.sur.step == 3 * sum(g.train_steps for g in many.groups)
    assert np.isfinite(many.pool.sur.params.cpu().numpy()).all()


def test_surrogate_search_checkpoint_restores_the_network(tmp_path):
    """Weights, Adam moments and step, replay buffer and training draws come
    back exactly: the restored network's predictions equal the original's,
    and the restored search continues."""
    hs = _gpu()
    from paper_1605_03607_amd import search as S
    chains = 4
    cfg = S.SearchConfig(mode="surrogate", chains=chains, L=2, restarts=4, K=8, R=2, s_max=3000, proposals=6,
                         top=2, train_steps=2, train_batch=4)
    seeds = [workloads.couplings(2, "pm1", 43, c) for c in range(chains)]
    params = workloads.gnn_params(hs.lib().gnn_param_count(), hs.gnn_fan_ins())
    run = S.Search(cfg, seeds, surrogate_params=params)
    for _ in range(2):
        run.run_step(bars=(math.log(1.5),))
    path = str(tmp_path / "sur.npz")
    S.save_search(run, path)
    back = S.load_search(path, cfg)
    a, b = run.pool, back.pool
    for name in ("params", "m", "v"):
        assert np.array_equal(getattr(a.sur, name).cpu().numpy(), getattr(b.sur, name).cpu().numpy()), name
    assert a.sur.step == b.sur.step
    assert a.pairs_y == b.pairs_y and all(np.array_equal(x, y) for x, y in zip(a.pairs_J, b.pairs_J))
    assert a.rng.bit_generator.state == b.rng.bit_generator.state
    graphs = [(2, None, J) for J in run.J]
    assert np.array_equal(a.sur.forward(graphs), b.sur.forward(graphs))
    assert back.step == 2 and back.decisions == run.decisions and np.array_equal(back.ln, run.ln)
    back.run_step(bars=(math.log(1.5),))
    assert len(back.decisions) == 3 * chains


@pytest.mark.parametrize("direction", [1, -1])
def test_plain_search_replays_on_the_oracle(direction):
    """Algorithm 1 end to end on C4: the oracle replays every step (its own
    mutation, its own PT hardness of the candidate, its own acceptance) and
    reaches the same ln TTS, decisions and couplings as the GPU search."""
    hs = _gpu()
    from paper_1605_03607_amd import search as S
    chains, steps, L = 3, 5, 4
    cfg = S.SearchConfig(mode="plain", chains=chains, L=L, restarts=4, K=8, R=2, s_max=3000, direction=direction,
                         alphabet=S.ALPHABET_PM1 if direction < 0 else S.ALPHABET_PM7)
    seeds = [workloads.couplings(L, "pm1", 83, c) for c in range(chains)]
    run = S.Search(cfg, seeds)
    start = run.ln.copy()
    for _ in range(steps):
        run.run_step(bars=(math.log(1.5),))

    def hard(J, ch):
        return oracle.hardness_eval(L, None, J, ch, cfg.seed, cfg.restarts, cfg.K, cfg.R, cfg.beta,
                                    cfg.swap_interval, cfg.s_max)["ln_tts"]
    want = []
    for ch in range(chains):
        print(f"search replay on the oracle: chain {ch}", flush=True)
        J = np.array(seeds[ch], np.int8)
        ln = hard(J, ch)
        assert ln == start[ch]
        for k in range(steps):
            e, old, new, w = oracle.mutate(L, None, J, cfg.alphabet, ch, cfg.seed, k, 0)
            J2 = J.copy()
            J2[e] = new
            ln2 = hard(J2, ch)
            ok = oracle.rao_accept(direction * ln, direction * ln2, cfg.t_s, w)
            want.append((k, ch, ln, ln2, w, ok))
            if ok:
                J, ln = J2, ln2
        assert np.array_equal(run.J[ch], J) and run.ln[ch] == ln
    assert sorted(want) == sorted(run.decisions)


@pytest.mark.parametrize("direction", [1, -1])
def test_validation_during_the_search(direction):
    """A Validator re-scoring counted states on its own stream while two
    chain groups run: the search takes the decisions of a search without it,
    the fresh scores and counts equal validate()'s after the search, and a
    counted state's fresh score equals the oracle's hardness on the
    validation streams (its validation id and the validation seed)."""
    hs = _gpu()
    from paper_1605_03607_amd import search as S
    chains, L, steps = 6, 3, 4
    cfg = S.SearchConfig(mode="plain", chains=chains, L=L, restarts=4, K=8, R=2, s_max=3000, t_s=5.0,
                         direction=direction, alphabet=S.ALPHABET_PM1 if direction < 0 else S.ALPHABET_PM7)
    seeds = [workloads.couplings(L, "pm1", 89, c) for c in range(chains)]
    bars = (math.log(1.1),)
    bare = S.GroupedSearch(cfg, seeds, groups=2)
    bare.run(steps, bars=bars)
    run = S.GroupedSearch(cfg, seeds, groups=2)
    v = S.Validator(cfg, seeds, restarts=8, chunk=4, stream_index=2)
    run.attach(v)
    run.run(steps, bars=bars)
    got = v.finish(bars)
    assert run.decisions == bare.decisions and run.hard == bare.hard
    assert got["states"] == len(run.hard_J) > 0
    want = S.validate(run, seeds, bars, restarts=8)
    assert got["h0"] == want["h0"] and got["fresh"] == want["fresh"] and got["counts"] == want["counts"]
    k = sorted(run.hard_J)[0]
    print(f"validation on the oracle: state {k[:8]} (direction {direction})", flush=True)
    o = oracle.hardness_eval(L, None, run.hard_J[k], S.validation_id(k), S.validation_seed(cfg), 8, cfg.K, cfg.R,
                             cfg.beta, cfg.swap_interval, cfg.s_max)
    assert got["fresh"][k] == (o["ln_tts"], o["confirmed"])


def test_compute_units_set_aside_for_the_surrogate():
    """With CUs set aside for the surrogate (its kernels on a CU-masked
    stream, the groups' PT launches on the rest), a random-screened search
    takes exactly the decisions of one without the split, and a surrogate
    search runs its screen and training on the set-aside stream."""
    hs = _gpu()
    from paper_1605_03607_amd import search as S
    chains = 6
    cfg = S.SearchConfig(mode="random", chains=chains, L=3, restarts=4, K=8, R=2, s_max=4000, proposals=5, top=2)
    seeds = [workloads.couplings(3, "pm1", 97, c) for c in range(chains)]
    try:
        S.set_gnn_cus(0)
        plain = S.GroupedSearch(cfg, seeds, groups=2)
        plain.run(3, bars=(math.log(1.5),))
        S.set_gnn_cus(16)
        split = S.GroupedSearch(cfg, seeds, groups=2)
        split.run(3, bars=(math.log(1.5),))
        assert split.decisions == plain.decisions and np.array_equal(split.ln, plain.ln)
        scfg = S.SearchConfig(mode="surrogate", chains=chains, L=3, restarts=4, K=8, R=2, s_max=4000, proposals=5,
                              top=2, train_steps=2, train_batch=4)
        params = workloads.gnn_params(hs.lib().gnn_param_count(), hs.gnn_fan_ins())
        sur = S.GroupedSearch(scfg, seeds, groups=2, surrogate_params=params)
        sur.run(3, bars=(math.log(1.5),))
        assert len(sur.decisions) == 3 * chains and sur.pool.sur.step > 0
        assert np.isfinite(sur.pool.sur.params.cpu().numpy()).all()
    finally:
        S.set_gnn_cus(0)


def test_hardness_does_not_depend_on_the_launch_shape():
    """hardness_eval with 4-, 8- and 16-wavefront workgroups (the search's
    screened arms run with 8): identical ln TTS, ground-state energies,
    confirmations and per-restart sweep counts."""
    hs = _gpu()
    from paper_1605_03607_amd import search as S
    c = S.SearchConfig(L=3, restarts=6, K=8, R=2, s_max=4000)
    cands = [dict(L=3, J=workloads.couplings(3, "pm7", 101, i), live=None, instance_id=i) for i in range(6)]
    out = []
    for bw in (16, 8, 4):
        ln, det = hs.hardness_eval(cands, c.restarts, c.K, c.R, c.beta, c.swap_interval, c.s_max, c.seed,
                                   block_waves=bw)
        out.append((np.asarray(ln), [(d["e_gs"], d["confirmed"], d["restart_sweeps"].tolist()) for d in det]))
    for ln, det in out[1:]:
        assert np.array_equal(ln, out[0][0]) and det == out[0][1]
