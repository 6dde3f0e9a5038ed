"""Pins of the overlap oracle (Sec. III.B, Fig. 3): brute force on a C1
instance whose ground and first excited levels are enumerated exactly, the
spin-flip symmetry, and PT snapshots that respect their energy cap."""
import itertools

import numpy as np

import oracle
import oracle.overlap as O
import workloads


def test_summary_on_enumerated_levels():
    """All states of a C1 instance (8 spins): the summary of the complete
    ground and first-excited sets equals a direct brute-force computation."""
    L = 1
    J = workloads.couplings(L, "pm3", 12, 0)
    states = [np.array(b, np.uint8) for b in itertools.product((0, 1), repeat=8)]
    en = [oracle.energy(L, None, J, b) for b in states]
    levels = sorted(set(en))
    e0, e1 = levels[0], levels[1]
    cfg = [(e, b) for e, b in zip(en, states) if e in (e0, e1)]
    s = O.summary(cfg)
    g = [b for e, b in cfg if e == e0 and b[0] == 0]      # one representative per flip pair
    x = [b for e, b in cfg if e == e1 and b[0] == 0]
    q = lambda a, b: abs(1 - 2 * int(np.sum(a ^ b)) / 8)
    ge = sorted(q(a, b) for a in g for b in x)
    gg = sorted(q(g[i], g[j]) for i in range(len(g)) for j in range(i + 1, len(g)))
    assert (s["e0"], s["e1"], s["n_gs"], s["n_ex"]) == (e0, e1, len(g), len(x))
    assert s["med_ge"] == float(np.median(ge))
    assert s["med_gg"] == (float(np.median(gg)) if gg else 1.0)


def test_flipped_configuration_is_the_same_state():
    b = np.array([0, 1, 1, 0, 1, 0, 0, 0], np.uint8)
    s = O.summary([(-10, b), (-10, 1 - b), (-6, b ^ np.array([1, 0, 0, 0, 0, 0, 0, 0], np.uint8))])
    assert s["n_gs"] == 1 and s["med_gg"] == 1.0
    assert s["med_ge"] == abs(1 - 2 / 8)


def test_snapshots_respect_the_cap_and_match_lane_energies():
    L, K, R = 2, 8, 2
    J = workloads.couplings(L, "pm1", 3, 0)
    beta = workloads.geometric_betas(0.2, 3.0, K)
    snaps = O.snapshots(L, None, J, K, R, beta, 1, 7, 1, 5, 20, e_cap=-40)
    assert snaps
    for s, lane, e, bits in snaps:
        assert e <= -40
        assert oracle.energy(L, None, J, bits) == e
