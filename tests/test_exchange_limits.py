"""The exchange pass by acceptance limits, checked on the CPU against the
definition of the pass (Sec. II: neighbouring temperatures, detailed balance).

The sweep kernel does not evaluate the test of pair (k, k+1) for each
configuration carried into slot k.  It turns the pair's uniform u into the
largest energy difference the pair accepts, D_k, and rejects a carried
configuration of energy E iff E > E_{k+1} + D_k.  That is exact because the
test "d <= 0 or u < T_k(d)" accepts a set of differences closed downwards:
T_k(d) = floor(2^32 exp(-(beta_{k+1} - beta_k) d)) does not grow with d.
These tests pin both facts with the oracle's thresholds.
"""
import numpy as np
import pytest

import oracle

LADDERS = {
    "geometric 0.1..5.0, K 32": np.geomspace(0.1, 5.0, 32),
    "geometric 0.2..3.0, K 16": np.geomspace(0.2, 3.0, 16),
    "closely spaced (steps of 1e-6)": 0.5 + 1e-6 * np.arange(8),
    "uneven steps": np.cumsum(np.random.default_rng(3).uniform(0.001, 0.8, 24)),
}


def _table(blo, bhi, dcap):
    return [oracle.swap_threshold(blo, bhi, d) for d in range(1, dcap + 1)]


@pytest.mark.parametrize("name", list(LADDERS))
def test_exchange_thresholds_do_not_grow_with_the_difference(name):
    beta = LADDERS[name]
    for k in range(len(beta) - 1):
        T = _table(beta[k], beta[k + 1], 400)
        assert all(a >= b for a, b in zip(T, T[1:])), f"{name}: pair {k}"


def _accepts(u, T, d):
    return d <= 0 or (d <= len(T) and u < T[d - 1])


def _sequential_pass(E, u, tables):
    """The definition: one ascending pass; pair k compares the configuration
    now at slot k (carried up by earlier acceptances) with the one at k+1."""
    K = len(E)
    E = list(E)
    slot = list(range(K))
    acc = [0] * (K - 1)
    for k in range(K - 1):
        if _accepts(u[k], tables[k], E[k] - E[k + 1]):
            E[k], E[k + 1] = E[k + 1], E[k]
            slot[k], slot[k + 1] = slot[k + 1], slot[k]
            acc[k] = 1
    return slot, acc


def _limit(u, T):
    D = 0
    while D < len(T) and u < T[D]:
        D += 1
    return D


def _pass_by_limits(E, u, tables):
    """Runs from the limits: the run from start x ends at the first pair
    k >= x with E_x > E_{k+1} + D_k; slot k of a run [x, e] receives the
    configuration from k + 1 if k < e and the carried one from x if k = e."""
    K = len(E)
    B = [E[k + 1] + _limit(u[k], tables[k]) for k in range(K - 1)]
    ends = []
    x = 0
    while x < K:
        e = next((k for k in range(x, K - 1) if E[x] > B[k]), K - 1)
        ends.append((x, e))
        x = e + 1
    slot = list(range(K))
    acc = [0] * (K - 1)
    for x, e in ends:
        for k in range(x, e):
            slot[k] = k + 1
            acc[k] = 1
        slot[e] = x
    return slot, acc


@pytest.mark.parametrize("name", list(LADDERS))
def test_pass_by_limits_equals_the_sequential_pass(name):
    beta = LADDERS[name]
    K = len(beta)
    rng = np.random.default_rng(11)
    dcap = 300
    tables = [_table(beta[k], beta[k + 1], dcap) for k in range(K - 1)]
    for trial in range(400):
        spread = [3, 40, 300][trial % 3]
        E = [int(x) for x in rng.integers(-spread, spread + 1, K)]
        u = [int(x) for x in rng.integers(0, 2**32, K - 1, dtype=np.uint64)]
        if trial % 4 == 0:
            # uniforms on and next to table entries, and the extremes
            for k in range(K - 1):
                T = tables[k]
                if T and rng.random() < 0.6:
                    d = int(rng.integers(1, len(T) + 1))
                    u[k] = min(max(T[d - 1] + int(rng.integers(-1, 2)), 0), 2**32 - 1)
                elif rng.random() < 0.3:
                    u[k] = [0, 2**32 - 1][int(rng.integers(0, 2))]
        assert _pass_by_limits(E, u, tables) == _sequential_pass(E, u, tables), f"{name}: trial {trial}"


def test_a_mistake_in_the_limit_is_caught():
    """An off-by-one limit (D_k + 1: accepting one difference too many)
    changes some pass, so the comparison above has teeth."""
    beta = LADDERS["geometric 0.1..5.0, K 32"]
    K = len(beta)
    tables = [_table(beta[k], beta[k + 1], 300) for k in range(K - 1)]
    rng = np.random.default_rng(5)
    differ = 0
    for _ in range(200):
        E = [int(x) for x in rng.integers(-40, 41, K)]
        u = [int(x) for x in rng.integers(0, 2**32, K - 1, dtype=np.uint64)]
        B = [E[k + 1] + _limit(u[k], tables[k]) + 1 for k in range(K - 1)]
        x, ends = 0, []
        while x < K:
            e = next((k for k in range(x, K - 1) if E[x] > B[k]), K - 1)
            ends.append(e)
            x = e + 1
        ref = _sequential_pass(E, u, tables)[1]
        got = [0 if k in ends else 1 for k in range(K - 1)]
        differ += got != ref
    assert differ > 0
