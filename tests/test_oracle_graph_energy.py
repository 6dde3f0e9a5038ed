"""Pins for the oracle's Chimera graph and Ising energy (Eq. 1; Appendix A)."""
import itertools

import numpy as np
import pytest

import oracle
import workloads


def site(L, r, c, u, k):
    return 8 * (L * r + c) + 4 * u + k


def coords(L, i):
    cell, rem = divmod(i, 8)
    u, k = divmod(rem, 4)
    r, c = divmod(cell, L)
    return r, c, u, k


@pytest.mark.parametrize("L", range(1, 13))
def test_edge_count_closed_form(L):
    ei, ej = oracle.edges(L)
    assert len(ei) == 16 * L * L + 8 * L * (L - 1) == workloads.num_edges(L)
    # canonical order: strictly ascending (min id, max id), no duplicates
    assert np.all(ei < ej)
    key = ei.astype(np.int64) * 100000 + ej
    assert np.all(np.diff(key) > 0)


@pytest.mark.parametrize("L", [1, 2, 3, 4])
def test_edges_match_brute_force_adjacency_rule(L):
    """Brute force over all site pairs with the adjacency rule of a Chimera
    graph: same cell and opposite sides (the K_{4,4}); or same side and same
    k in cells adjacent along that side's direction (u = 0 vertical,
    u = 1 horizontal)."""
    N = 8 * L * L
    want = set()
    for i, j in itertools.combinations(range(N), 2):
        ri, ci, ui, ki = coords(L, i)
        rj, cj, uj, kj = coords(L, j)
        if (ri, ci) == (rj, cj) and ui != uj:
            want.add((i, j))
        elif ui == uj == 0 and ki == kj and ci == cj and abs(ri - rj) == 1:
            want.add((i, j))
        elif ui == uj == 1 and ki == kj and ri == rj and abs(ci - cj) == 1:
            want.add((i, j))
    ei, ej = oracle.edges(L)
    assert set(zip(ei.tolist(), ej.tolist())) == want


@pytest.mark.parametrize("L", [1, 2, 8, 12])
def test_degree_and_two_colouring(L):
    ei, ej = oracle.edges(L)
    N = 8 * L * L
    deg = np.bincount(np.concatenate([ei, ej]), minlength=N)
    assert deg.max() <= 6  # Appendix A: degree 6 in the ideal graph
    if L >= 3:
        # interior cells have degree 6 everywhere; boundary vertices have 5
        interior = [site(L, 1, 1, u, k) for u in (0, 1) for k in range(4)]
        assert np.all(deg[interior] == 6)
        assert deg[site(L, 0, 1, 0, 0)] == 5  # top edge, vertical coupler missing
    # (r + c + u) mod 2 is a proper 2-colouring: every edge joins the colours
    col = np.array([(lambda r, c, u, k: (r + c + u) % 2)(*coords(L, i)) for i in range(N)])
    assert np.all(col[ei] != col[ej])


def _rand_J(L, seed, alphabet="pm7"):
    return workloads.couplings(L, alphabet, seed, 0)


def test_energy_all_up_is_sum_of_couplings():
    L = 3
    J = _rand_J(L, 5)
    N = 8 * L * L
    assert oracle.energy(L, None, J, np.zeros(N, np.uint8)) == int(J.astype(np.int64).sum())
    assert oracle.energy(L, None, J, np.ones(N, np.uint8)) == int(J.astype(np.int64).sum())


def test_energy_single_coupler_by_hand():
    L = 1
    ei, ej = oracle.edges(L)
    for e in (0, 7, 15):
        J = np.zeros(len(ei), np.int8)
        J[e] = 3
        b = np.zeros(8, np.uint8)
        assert oracle.energy(L, None, J, b) == 3  # s_i s_j = +1
        b[ei[e]] = 1
        assert oracle.energy(L, None, J, b) == -3  # s_i s_j = -1
        b[ej[e]] = 1
        assert oracle.energy(L, None, J, b) == 3


@pytest.mark.parametrize("seed", range(4))
def test_energy_gauge_and_flip_invariance(seed):
    """E_{gJg}(g.s) = E_J(s) for any gauge g (J'_ij = g_i g_j J_ij), and
    E(-s) = E(s) (Eq. 1 has no fields)."""
    L = 4
    N = 8 * L * L
    J = _rand_J(L, seed)
    live = workloads.missing_mask(L, 0.05, seed, 0)
    ei, ej = oracle.edges(L)
    g = np.random.default_rng(seed).integers(0, 2, N).astype(np.uint8)
    b = np.random.default_rng(seed + 50).integers(0, 2, N).astype(np.uint8)
    sg = 1 - 2 * g.astype(np.int64)
    Jg = (J * sg[ei] * sg[ej]).astype(np.int8)
    assert oracle.energy(L, live, Jg, b ^ g) == oracle.energy(L, live, J, b)
    assert oracle.energy(L, live, J, 1 - b) == oracle.energy(L, live, J, b)


@pytest.mark.parametrize("L,n_dead", [(1, 0), (2, 10)])
def test_ground_state_closed_forms(L, n_dead):
    """Bipartite graph, no frustration: all J = -1 (ferromagnet) and all
    J = +1 (antiferromagnet, Eq. 1 as printed) both have E_gs = -|E| with
    exactly two ground states; for J = +1 they are the two colour classes."""
    N = 8 * L * L
    live = None
    if n_dead:
        live = np.ones(N, np.uint8)
        live[np.random.default_rng(1).choice(N, n_dead, replace=False)] = 0
    ei, ej = oracle.edges(L)
    lv = np.ones(N, bool) if live is None else live.astype(bool)
    n_live_edges = int(np.count_nonzero(lv[ei] & lv[ej]))
    ids = np.nonzero(lv)[0]
    for sign in (-1, 1):
        J = np.full(len(ei), sign, np.int8)
        levels, counts, en = oracle.enumerate_states(L, live, J, want_energies=True)
        assert levels[0] == -n_live_edges
        assert counts[0] == 2 or n_live_edges == 0
        gs = np.nonzero(en == levels[0])[0]
        for s in gs:
            bits = np.zeros(N, np.uint8)
            bits[ids] = (int(s) >> np.arange(len(ids))) & 1
            if sign == 1:
                col = np.array([(coords(L, i)[0] + coords(L, i)[1] + coords(L, i)[2]) % 2
                                for i in range(N)], np.uint8)
                assert np.all((bits[ids] ^ col[ids]) == bits[ids[0]] ^ col[ids[0]])
            else:
                assert np.all(bits[ids] == bits[ids[0]])
        assert counts.sum() == 2 ** len(ids)


def test_enumeration_symmetric_spectrum():
    """Spin-flip symmetry of Eq. 1: every configuration and its negation have
    the same energy, so every level has even multiplicity."""
    L = 1
    J = _rand_J(L, 9)
    levels, counts, en = oracle.enumerate_states(L, None, J, want_energies=True)
    idx = np.arange(256)
    assert np.all(en[idx] == en[255 - idx])
    assert np.all(counts % 2 == 0)
