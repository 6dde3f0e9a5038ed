"""Pins of the planted-solution oracle (Sec. IV): cycle counts against the
closed forms of the Chimera geometry, brute-force ground states of small
planted instances, and the planted configuration's energy."""
import numpy as np
import pytest

import oracle
import oracle.lao as P


@pytest.mark.parametrize("L", [1, 2, 3])
def test_cycle_counts_follow_the_geometry(L):
    """4-cycles lie inside cells: 36 per K_{4,4}.  6-cycles: 96 inside each
    cell (16 K_{3,3} sub-graphs x 6 Hamiltonian cycles) and 96 through each
    pair of neighbouring cells (6 pairs {k, k'} x 4 x 4 connectors)."""
    c = P.cycles(L)
    assert len(c[4]) == 36 * L * L
    assert len(c[6]) == 96 * (L * L + 2 * L * (L - 1))


def test_cycles_are_simple_closed_paths():
    ei, ej = oracle.edges(2)
    for n, cs in P.cycles(2).items():
        for cyc in cs[::37]:
            deg = {}
            for e in cyc:
                for v in (ei[e], ej[e]):
                    deg[v] = deg.get(v, 0) + 1
            assert len(cyc) == n and len(deg) == n and all(d == 2 for d in deg.values())


def test_missing_sites_remove_their_cycles():
    live = np.ones(8 * 4, np.uint8)
    live[5] = 0
    full, cut = P.cycles(2), P.cycles(2, live)
    ei, ej = oracle.edges(2)
    for n in (4, 6):
        keep = [c for c in full[n] if all(ei[e] != 5 and ej[e] != 5 for e in c)]
        assert cut[n] == keep


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_planted_state_is_a_brute_force_ground_state(seed):
    L = 1
    inst = P.init(L, 6, chain=seed, seed=77)
    levels, counts, _ = oracle.enumerate_states(L, None, inst["J"])
    assert int(levels[0]) == inst["e_gs"]
    assert oracle.energy(L, None, inst["J"], inst["bits"]) == inst["e_gs"]
    assert np.all(np.abs(inst["J"]) <= 7)


def test_planted_energy_and_loop_frustration_on_c3():
    L = 3
    cyc = P.cycles(L)
    inst = P.init(L, 40, chain=5, seed=9, cyc=cyc)
    assert oracle.energy(L, None, inst["J"], inst["bits"]) == inst["e_gs"]
    s = 1 - 2 * inst["bits"].astype(np.int64)
    ei, ej = oracle.edges(L)
    for lp in inst["loops"]:
        idx, d = P.loop_couplings(L, lp, cyc, inst["bits"])
        # exactly one coupler of the loop is unsatisfied by the planted state
        assert int(np.sum(d * s[ei[idx]] * s[ej[idx]] > 0)) == 1
        # and the product of coupling signs marks the loop frustrated
        assert np.prod(np.sign(-d)) * np.prod(s[ei[idx]] * s[ej[idx]]) == -1


def test_move_replaces_one_loop():
    L = 2
    cyc = P.cycles(L)
    inst = P.init(L, 12, chain=3, seed=4, cyc=cyc)
    slot, lp, w, J2, e2 = P.move(L, inst, 3, 4, step=7, proposal=1, cyc=cyc)
    loops = list(inst["loops"])
    loops[slot] = lp
    J3, e3 = P.couplings(L, loops, cyc, inst["bits"])
    assert np.array_equal(J3, J2) and e3 == e2
    assert oracle.energy(L, None, J2, inst["bits"]) == e2
