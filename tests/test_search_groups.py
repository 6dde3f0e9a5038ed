"""Grouped search mechanics on the host: with a stand-in scorer (a fixed
function of the couplings and the chain index, as PT's ln TTS is for fixed
seeds), a plain or random-screened search split into concurrent chain groups
takes exactly the decisions of the single-group search, because every draw
is keyed by the chain's global index; H0 is the median over all chains."""
import contextlib
import hashlib
import math

import numpy as np
import pytest

import workloads


def _fake_eval(cands, n_restarts, K, R, beta, swap_interval, s_max, seed):
    ln, det = [], []
    for c in cands:
        h = hashlib.sha1(np.asarray(c["J"], np.int8).tobytes() + bytes([c["instance_id"] % 251])).digest()
        ln.append(5.0 + 4.0 * int.from_bytes(h[:4], "little") / 2.0**32)
        det.append(dict(e_gs=0, confirmed=True, n_censored=0, sweeps_total=100))
    return np.array(ln), det


class _NoStream:
    def synchronize(self):
        pass


@pytest.fixture
def S(monkeypatch):
    import paper_1605_03607_amd as hs
    hs.lib()
    from paper_1605_03607_amd import search
    monkeypatch.setattr(search, "hardness_eval", _fake_eval)
    monkeypatch.setattr(search, "_group_stream", lambda i: (_NoStream(), contextlib.nullcontext()))

    def untimed(cands, c):  # the scorer without device events
        ln, det = search.hardness_eval(cands, c.restarts, c.K, c.R, c.beta, c.swap_interval, c.s_max, c.seed)
        return ln, det, 0.0, 0
    monkeypatch.setattr(search, "_timed_hardness", untimed)

    def fresh_untimed(cands, c, restarts, seed_v):  # the validation scorer without device events
        ln, det = search.hardness_eval(cands, restarts, c.K, c.R, c.beta, c.swap_interval, c.s_max, seed_v)
        return ([float(v) for v in ln], [bool(d["confirmed"]) for d in det],
                sum(d["sweeps_total"] for d in det), 0, 0.0)
    monkeypatch.setattr(search, "_fresh_scores", fresh_untimed)
    return search


@pytest.mark.parametrize("mode", ["plain", "random"])
@pytest.mark.parametrize("groups", [2, 3, 7])
def test_groups_take_the_single_group_decisions(S, mode, groups):
    chains, steps = 7, 4
    cfg = S.SearchConfig(mode=mode, chains=chains, L=2, proposals=5, top=2, t_s=0.7)
    seeds = [workloads.couplings(2, "pm1", 41, c) for c in range(chains)]
    one = S.Search(cfg, seeds)
    for _ in range(steps):
        one.run_step(bars=(math.log(1.2),))
    many = S.GroupedSearch(cfg, seeds, groups=groups)
    assert many.h0 == one.h0
    sizes = [len(g.J) for g in many.groups]
    assert sum(sizes) == chains and max(sizes) - min(sizes) <= 1 and min(sizes) >= 1
    seen = []
    many.run(steps, bars=(math.log(1.2),), progress=lambda g, k: seen.append((g, k)))
    assert sorted(seen) == [(g, k) for g in range(groups) for k in range(1, steps + 1)]
    assert many.decisions == sorted(one.decisions)
    assert np.array_equal(many.ln, one.ln)
    assert all(np.array_equal(a, b) for a, b in zip(many.J, one.J))
    assert many.accepted == one.accepted
    assert many.hard == one.hard
    assert len(many.decisions) == chains * steps


def test_random_screen_is_keyed_by_chain_and_step(S):
    cfg = S.SearchConfig(mode="random", chains=3, L=2, proposals=6, top=2)
    seeds = [workloads.couplings(2, "pm1", 43, c) for c in range(3)]
    run = S.Search(cfg, seeds)
    picks = [run._random_screen(ch) for ch in range(3)]
    assert all(len(p) == 2 and len(set(p)) == 2 and all(0 <= x < 6 for x in p) for p in picks)
    again = S.Search(cfg, seeds[1:], chain_ids=[1, 2], ln=run.ln[1:], h0=run.h0)
    assert [again._random_screen(ch) for ch in range(2)] == picks[1:]


def test_group_failure_reaches_the_caller(S, monkeypatch):
    cfg = S.SearchConfig(mode="plain", chains=4, L=2)
    seeds = [workloads.couplings(2, "pm1", 47, c) for c in range(4)]
    many = S.GroupedSearch(cfg, seeds, groups=2)

    def boom(*a, **k):
        raise RuntimeError("scorer failed")
    monkeypatch.setattr(S, "hardness_eval", boom)
    with pytest.raises(RuntimeError, match="scorer failed"):
        many.run(2)


def test_group_count_is_checked(S):
    cfg = S.SearchConfig(mode="plain", chains=2, L=2)
    seeds = [workloads.couplings(2, "pm1", 53, c) for c in range(2)]
    with pytest.raises(ValueError):
        S.GroupedSearch(cfg, seeds, groups=3)


def test_grouped_lao_takes_the_single_group_decisions(S):
    cfg = S.SearchConfig(mode="plain", chains=5, L=2, t_s=0.7)
    one = S.LaoSearch(cfg, n_loops=14)
    for _ in range(4):
        one.run_step()
    many = S.GroupedLao(cfg, n_loops=14, groups=3)
    seen = []
    many.run(4, progress=lambda g, k: seen.append((g, k)))
    assert sorted(seen) == [(g, k) for g in range(3) for k in range(1, 5)]
    assert many.decisions == sorted(one.decisions)
    assert np.array_equal(many.ln, one.ln) and np.array_equal(many.ln0, one.ln0)
    assert all(np.array_equal(a["J"], b["J"]) for a, b in zip(many.inst, one.inst))
    assert (many.scored, many.voids, many.accepted) == (one.scored, one.voids, one.accepted)


@pytest.mark.parametrize("mode,groups_before,groups_after", [("plain", 1, 1), ("random", 3, 2), ("plain", 2, 1)])
def test_checkpoint_resume_is_exact(S, tmp_path, mode, groups_before, groups_after):
    chains, steps = 6, 4
    cfg = S.SearchConfig(mode=mode, chains=chains, L=2, proposals=5, top=2, t_s=0.7)
    seeds = [workloads.couplings(2, "pm1", 61, c) for c in range(chains)]
    bars = (math.log(1.2),)
    full = S.Search(cfg, seeds)
    for _ in range(steps):
        full.run_step(bars)
    run = S.GroupedSearch(cfg, seeds, groups=groups_before) if groups_before > 1 else S.Search(cfg, seeds)
    if groups_before > 1:
        run.run(2, bars)
    else:
        run.run_step(bars)
        run.run_step(bars)
    path = str(tmp_path / "search.npz")
    S.save_search(run, path)
    back = S.load_search(path, cfg, groups=groups_after)
    if groups_after > 1:
        back.run(steps - 2, bars)
    else:
        for _ in range(steps - 2):
            back.run_step(bars)
    assert sorted(back.decisions) == sorted(full.decisions)
    assert np.array_equal(back.ln, full.ln)
    assert all(np.array_equal(a, b) for a, b in zip(back.J, full.J))
    assert back.hard == full.hard and back.accepted == full.accepted
    if groups_before == groups_after == 1:
        assert back.pool.pairs_y == full.pool.pairs_y
        assert all(np.array_equal(a, b) for a, b in zip(back.pool.pairs_J, full.pool.pairs_J))
    else:  # concurrent groups add their pairs in the order they finish
        assert sorted(back.pool.pairs_y) == sorted(full.pool.pairs_y)


def test_checkpoint_rejects_another_configuration(S, tmp_path):
    cfg = S.SearchConfig(mode="plain", chains=3, L=2)
    seeds = [workloads.couplings(2, "pm1", 67, c) for c in range(3)]
    run = S.Search(cfg, seeds)
    run.run_step()
    path = str(tmp_path / "c.npz")
    S.save_search(run, path)
    other = S.SearchConfig(mode="plain", chains=3, L=2, t_s=0.9)
    with pytest.raises(ValueError, match="configuration"):
        S.load_search(path, other)


_CHILD = r"""
import math, os, signal, sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import numpy as np
import workloads
import paper_1605_03607_amd as hs
hs.lib()
from paper_1605_03607_amd import search as S
import test_search_groups as T
S.hardness_eval = T._fake_eval
def untimed(cands, c):
    ln, det = S.hardness_eval(cands, c.restarts, c.K, c.R, c.beta, c.swap_interval, c.s_max, c.seed)
    return ln, det, 0.0, 0
S._timed_hardness = untimed
cfg = S.SearchConfig(mode="random", chains=5, L=2, proposals=5, top=2, t_s=0.7)
run = S.Search(cfg, [workloads.couplings(2, "pm1", 71, c) for c in range(5)])
for k in range(3):
    run.run_step((math.log(1.2),))
    S.save_search(run, {path!r})
os.kill(os.getpid(), signal.SIGKILL)  # dies without any cleanup
"""


def test_resume_after_a_killed_process(S, tmp_path):
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    path = str(tmp_path / "killed.npz")
    code = _CHILD.format(root=root, tests=os.path.join(root, "tests"), path=path)
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, timeout=300)
    assert p.returncode == -9, p.stderr.decode()[-2000:]
    cfg = S.SearchConfig(mode="random", chains=5, L=2, proposals=5, top=2, t_s=0.7)
    seeds = [workloads.couplings(2, "pm1", 71, c) for c in range(5)]
    full = S.Search(cfg, seeds)
    for _ in range(5):
        full.run_step((math.log(1.2),))
    back = S.load_search(path, cfg)
    assert back.step == 3
    back.run_step((math.log(1.2),))
    back.run_step((math.log(1.2),))
    assert back.decisions == full.decisions
    assert np.array_equal(back.ln, full.ln)
    assert back.hard == full.hard


def test_checkpoint_needs_groups_at_one_step(S, tmp_path):
    cfg = S.SearchConfig(mode="plain", chains=4, L=2)
    seeds = [workloads.couplings(2, "pm1", 73, c) for c in range(4)]
    run = S.GroupedSearch(cfg, seeds, groups=2)
    run.run(1)
    run.groups[1].run_step()
    with pytest.raises(ValueError, match="different steps"):
        S.save_search(run, str(tmp_path / "x.npz"))


def test_validation_uses_restart_streams_disjoint_from_the_search(S, monkeypatch):
    """Counted states and the seed instances are re-scored with 64 restarts
    whose Philox keys (restart key, seed') all have seed' != the search's
    seed, so no validation stream is one the search used (every search key
    is (restart key, seed)); the validated counts come from those fresh
    scores, against the median fresh score of the seeds."""
    calls = []

    def recording(cands, n_restarts, K, R, beta, swap_interval, s_max, seed):
        calls.append((seed, n_restarts, len(cands)))
        return _fake_eval(cands, n_restarts, K, R, beta, swap_interval, s_max, seed)

    monkeypatch.setattr(S, "hardness_eval", recording)
    cfg = S.SearchConfig(mode="plain", chains=6, L=2, t_s=5.0)
    seeds = [workloads.couplings(2, "pm1", 47, c) for c in range(6)]
    run = S.GroupedSearch(cfg, seeds, groups=2)
    bars = (math.log(1.1), math.log(1.5))
    run.run(6, bars=bars)
    search_seeds = {sd for sd, _, _ in calls}
    assert search_seeds == {cfg.seed}
    n_calls = len(calls)
    assert run.hard_J and set(run.hard_J) == run.hard[bars[0]] | run.hard.get(bars[1], set())
    v = S.validate(run, seeds, bars)
    fresh_calls = calls[n_calls:]
    assert fresh_calls and all(sd == S.validation_seed(cfg) != cfg.seed and nr == 64 for sd, nr, _ in fresh_calls)
    assert sum(n for _, _, n in fresh_calls) == len(seeds) + len(run.hard_J)
    # the fake scorer depends on the instance id, as PT's ln TTS depends on
    # the restart streams: recompute the validated counts from its values
    fresh = [_fake_eval([dict(J=s, instance_id=i)], 0, 0, 0, 0, 0, 0, 0)[0][0] for i, s in enumerate(seeds)]
    h0v = float(np.median(fresh))
    assert v["h0"] == h0v
    keys = sorted(run.hard_J)
    ids = [S.validation_id(k) for k in keys]
    assert all(i >= 2**31 for i in ids) and len(set(ids)) == len(ids)
    for b in bars:
        want = 0
        for k in keys:
            y = _fake_eval([dict(J=run.hard_J[k], instance_id=S.validation_id(k))], 0, 0, 0, 0, 0, 0, 0)[0][0]
            want += int(y - h0v >= b)
        assert v["counts"][b] == want


@pytest.mark.parametrize("groups", [1, 3])
def test_validation_during_the_search_equals_validation_after_it(S, groups):
    """A Validator attached to the search re-scores each counted state as it
    is counted, on its own thread, in launches of whatever is waiting; it
    returns validate()'s H0', fresh scores and counts, and the search's
    decisions are those of a search without it."""
    cfg = S.SearchConfig(mode="random", chains=6, L=2, proposals=5, top=2, t_s=5.0)
    seeds = [workloads.couplings(2, "pm1", 53, c) for c in range(6)]
    bars = (math.log(1.1), math.log(1.5))
    bare = S.GroupedSearch(cfg, seeds, groups=groups)
    bare.run(6, bars=bars)
    run = S.GroupedSearch(cfg, seeds, groups=groups)
    val = S.Validator(cfg, seeds, chunk=3, stream_index=groups)
    run.attach(val)
    run.run(6, bars=bars)
    got = val.finish(bars)
    assert run.decisions == bare.decisions and run.hard == bare.hard
    want = S.validate(run, seeds, bars)
    assert got["overlapped"] and not want["overlapped"]
    assert got["h0"] == want["h0"] and got["fresh"] == want["fresh"] and got["counts"] == want["counts"]
    assert got["states"] == len(run.hard_J) > 3 and got["calls"] >= 2


def test_validator_failure_reaches_finish(S, monkeypatch):
    cfg = S.SearchConfig(mode="plain", chains=4, L=2, t_s=5.0)
    seeds = [workloads.couplings(2, "pm1", 59, c) for c in range(4)]

    def boom(*a, **k):
        raise RuntimeError("validation launch failed")
    monkeypatch.setattr(S, "_fresh_scores", boom)
    val = S.Validator(cfg, seeds)
    with pytest.raises(RuntimeError, match="validation launch failed"):
        val.finish((math.log(1.1),))


def test_checkpoint_keeps_the_counted_couplings(S, tmp_path):
    cfg = S.SearchConfig(mode="plain", chains=4, L=2, t_s=5.0)
    seeds = [workloads.couplings(2, "pm1", 49, c) for c in range(4)]
    run = S.Search(cfg, seeds)
    for _ in range(4):
        run.run_step(bars=(math.log(1.1),))
    assert run.hard_J
    path = str(tmp_path / "ck.npz")
    S.save_search(run, path)
    back = S.load_search(path, cfg)
    assert sorted(back.hard_J) == sorted(run.hard_J)
    assert all(np.array_equal(back.hard_J[k], run.hard_J[k]) for k in run.hard_J)


class _FakeSurrogate:
    """Stands in for the network: predictions from a hash of the couplings,
    and a record of every training call."""

    def __init__(self, params):
        self.calls = []
        self.step = 0

    def forward(self, graphs):
        return np.array([int(hashlib.sha1(np.asarray(g[2], np.int8).tobytes()).hexdigest()[:6], 16) / 2.0**24
                         for g in graphs], np.float32)

    def train_step(self, labels, graphs=None, lr=1e-3, ref=None, w_abs=1.0, **kw):
        self.calls.append((np.array(labels, np.float64), [np.array(g[2], np.int8) for g in graphs],
                           None if ref is None else np.array(ref), w_abs, lr))
        self.step += 1
        return 0.0, np.zeros(len(graphs), np.float32)


@pytest.mark.parametrize("loss", ["ranked", "plain"])
def test_surrogate_training_batches(S, monkeypatch, loss):
    """The ranked loss trains on (parent, proposal) pairs: every batch holds
    train_batch / 2 pairs, parent first, ref pointing each proposal at its
    parent; a proposal differs from its parent at one coupler, and both
    labels are the scores the search measured (the proposal's PT score, the
    chain's current score).  The plain loss draws single records."""
    monkeypatch.setattr(S, "Surrogate", _FakeSurrogate)
    cfg = S.SearchConfig(mode="surrogate", chains=6, L=2, proposals=5, top=2, t_s=0.7, train_steps=3,
                         train_batch=8, train_loss=loss)
    seeds = [workloads.couplings(2, "pm1", 61, c) for c in range(6)]
    run = S.Search(cfg, seeds, surrogate_params=np.zeros(4))
    for _ in range(3):
        run.run_step(bars=(math.log(1.2),))
    calls = run.pool.sur.calls
    assert len(calls) == 3 * 3
    for labels, graphs, ref, w_abs, lr in calls:
        assert lr == cfg.lr
        if loss == "plain":
            assert ref is None and len(graphs) == 8
            continue
        assert w_abs == cfg.w_abs and len(graphs) == 8
        assert ref.tolist() == [-1, 0, -1, 2, -1, 4, -1, 6]
        for k in range(0, 8, 2):
            assert int((graphs[k] != graphs[k + 1]).sum()) == 1  # one mutated coupler
            assert np.isfinite(labels[k]) and np.isfinite(labels[k + 1])
