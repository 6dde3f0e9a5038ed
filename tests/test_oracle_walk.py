"""Pins of the mixing-time oracle (Sec. III.B's tau of the temperature
random walk): brute force, a closed form for a square wave, the integrated
autocorrelation time of a two-state Markov chain, and invariants of the PT
walk itself."""
import numpy as np
import pytest

import oracle
import oracle.walk as W
import workloads


def test_sums_match_brute_force():
    rng = np.random.default_rng(3)
    K, T, C = 5, 37, 3
    traj = rng.integers(0, K, size=(T, C))
    S = W.acf_sums(traj, K, 40)
    for d in range(41):
        want = 0
        for c in range(C):
            for t in range(T - d):
                want += (2 * int(traj[t, c]) - (K - 1)) * (2 * int(traj[t + d, c]) - (K - 1))
        assert S[d] == want, d


def test_square_wave_closed_form():
    """g = +-A with half-period P over M periods: for d <= P,
    S(d) = A^2 (2 M P - (4 M - 1) d)."""
    K, P, M = 9, 7, 5
    A = K - 1
    one = np.array([K - 1] * P + [0] * P)
    traj = np.tile(one, M)[:, None]
    S = W.acf_sums(traj, K, P)
    for d in range(P + 1):
        assert S[d] == A * A * (2 * M * P - (4 * M - 1) * d)


def test_two_state_chain_tau():
    """A two-state chain that flips with probability p has rho(d) = (1-2p)^d
    and tau = 1/2 + (1-2p)/(2p) = (1-p)/(2p)."""
    rng = np.random.default_rng(11)
    p, T, K = 0.05, 400_000, 2
    flips = rng.random(T) < p
    state = np.cumsum(flips) % 2
    S = W.acf_sums(state[:, None], K, 400)
    tau, win, ok = W.tau_int(S, T)
    assert ok
    assert abs(tau - (1 - p) / (2 * p)) < 0.05 * (1 - p) / (2 * p), tau


def test_independent_draws_have_tau_one_half():
    rng = np.random.default_rng(5)
    T, K = 200_000, 8
    traj = rng.integers(0, K, size=(T, 2))
    S = W.acf_sums(traj, K, 50)
    tau, win, ok = W.tau_int(S, T)
    assert ok and abs(tau - 0.5) < 0.02


def test_hot_counts_and_criteria():
    traj = np.array([[0, 3], [1, 2], [3, 0], [2, 1], [0, 3]])
    hot = W.hot_counts(traj, 4)
    assert hot.tolist() == [3, 2]
    ok_i, ok_ii, share = W.criteria(hot, 5, 0.2)
    assert share == 0.4 and ok_i and ok_ii
    assert W.criteria(hot, 5, 1.0)[1] is False


def test_pt_walk_is_a_permutation_per_set():
    """After every EMCS each replica set's K configurations sit at K distinct
    temperatures, and configurations never leave their set."""
    L, K, R = 2, 6, 3
    J = workloads.couplings(L, "pm3", 4, 0)
    beta = workloads.geometric_betas(0.2, 3.0, K)
    traj, st = W.walk(L, None, J, K, R, beta, 9, 1605, 10, 40)
    assert traj.shape == (40, K * R)
    for e in range(40):
        for r in range(R):
            assert sorted(traj[e, r * K:(r + 1) * K].tolist()) == list(range(K))
    assert int(st.t[0]) == 400
