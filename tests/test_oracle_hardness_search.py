"""Pins for the oracle's hardness evaluation (ground-state agreement,
Sec. III.B and Appendix B) and the RAO move/acceptance (Algorithm 1)."""
import math

import numpy as np
import pytest

import oracle
import workloads

BETAS = workloads.geometric_betas(0.1, 5.0, 8)


def _small_instance(seed, n_dead=10, alphabet="pm7"):
    L = 2
    N = 32
    J = workloads.couplings(L, alphabet, seed, 0)
    live = np.ones(N, np.uint8)
    live[np.random.default_rng(seed).choice(N, n_dead, replace=False)] = 0
    return L, live, J


@pytest.mark.parametrize("seed", range(3))
def test_ground_state_energy_matches_brute_force(seed):
    """The PT ground-state energy equals the exact minimum over all 2^22
    configurations (the cross-check of Sec. III.B)."""
    L, live, J = _small_instance(seed)
    levels, _, _ = oracle.enumerate_states(L, live, J)
    res = oracle.hardness_eval(L, live, J, 100 + seed, 9, 4, 8, 2, BETAS, 1, 20000)
    assert res["e_gs"] == levels[0]
    assert res["confirmed"]
    assert math.isfinite(res["ln_tts"]) and res["ln_tts"] >= 0.0
    assert np.all(res["r_sweeps"] <= 20000)


def test_unfrustrated_instance_reaches_minus_edge_count():
    L = 3
    ei, _ = oracle.edges(L)
    J = np.full(len(ei), -1, np.int8)
    res = oracle.hardness_eval(L, None, J, 1, 2, 5, 8, 2, BETAS, 1, 20000)
    assert res["e_gs"] == -len(ei)
    assert res["confirmed"]
    # TTS = restart sweeps per restart that reached E_gs (Appendix B's run
    # time per find of the minimum): at least the mean restart length
    n_hit = int(np.count_nonzero(res["r_tts"] > 0))
    assert n_hit >= 3 and np.all(res["r_tts"][res["r_tts"] > 0] >= 1)
    assert res["ln_tts"] == pytest.approx(math.log(res["r_sweeps"].sum() / n_hit))
    assert res["ln_tts"] >= math.log(res["r_sweeps"].mean()) - 1e-12


def test_sweep_cap_gives_the_closed_form():
    """With a sweep cap too short for agreement every restart runs exactly
    s_max sweeps, so TTS = n_restarts s_max / n_hit, finite since the best
    restart holds E_gs by definition."""
    L = 4
    J = workloads.couplings(L, "pm7", 31, 0)
    res = oracle.hardness_eval(L, None, J, 3, 4, 3, 4, 2, workloads.geometric_betas(0.1, 0.3, 4),
                               1, 3)
    assert np.all(res["r_sweeps"] == 3)
    n_hit = int(np.count_nonzero(res["r_emin"] == res["e_gs"]))
    assert 1 <= n_hit <= 3
    assert res["ln_tts"] == pytest.approx(math.log(3 * 3 / n_hit))
    assert res["r_emin"].min() == res["e_gs"]


@pytest.mark.parametrize("alphabet", ["pm1", "pm7"])
def test_mutation_invariants(alphabet):
    """Algorithm 1: one live edge changes, the new value is in the alphabet
    and differs from the old one; with {-1, +1} it is a sign flip."""
    L = 3
    A = workloads.ALPHABETS[alphabet]
    J = workloads.couplings(L, alphabet, 4, 0)
    live = workloads.missing_mask(L, 0.05, 4, 0)
    ei, ej = oracle.edges(L)
    lv = live.astype(bool)
    counts = np.zeros(len(ei), np.int64)
    for step in range(3000):
        e, old, new, w = oracle.mutate(L, live, J, A, 7, 99, step, step % 16)
        assert lv[ei[e]] and lv[ej[e]]
        assert old == J[e] and new in A and new != old
        if alphabet == "pm1":
            assert new == -old
        counts[e] += 1
    live_edges = lv[ei] & lv[ej]
    assert counts[~live_edges].sum() == 0
    # uniform over live edges (loose check on the spread)
    c = counts[live_edges]
    assert c.min() > 0 and c.max() < 6 * c.mean()


def test_rao_acceptance():
    """Delta >= 0 is always accepted; otherwise the acceptance rate is
    exp(Delta / T_s)."""
    rng = np.random.default_rng(5)
    for _ in range(100):
        w = int(rng.integers(0, 2 ** 32))
        assert oracle.rao_accept(1.0, 1.0 + rng.random(), 0.5, w)
    assert oracle.rao_accept(2.0, math.inf, 0.5, 2 ** 32 - 1)
    assert not oracle.rao_accept(math.inf, 2.0, 0.5, 0)
    delta = -0.3
    ws = rng.integers(0, 2 ** 32, size=20000)
    rate = np.mean([oracle.rao_accept(1.0, 1.0 + delta, 0.5, int(w)) for w in ws])
    assert rate == pytest.approx(math.exp(delta / 0.5), abs=0.015)
