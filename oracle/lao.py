"""Planted-solution instances and the loop moves of Loop Adaptive
Optimization (Sec. IV, Algorithm 2) -- TEST INFRASTRUCTURE ONLY (tests/,
the smoke check and bench.py's CPU baseline may use it; the product path
never does).

An instance is a sum of M loop Hamiltonians on the Chimera graph, each a
frustrated cycle whose couplings keep a planted configuration s* among its
ground states, so s* is a ground state of the sum and E_gs = sum over loops
of the loop's planted energy (Sec. IV).  Readings (the paper leaves them
open or gives them only for its figure):
  * loops are simple cycles of 4 or 6 couplers of the live graph, drawn
    uniformly from all such cycles, a 4-cycle with probability about 0.1
    (w0 < P4_THRESHOLD), else a 6-cycle (Fig. 6: 0.1 / 0.9);
  * loop weight w uniform in 1..5 (Fig. 6); every loop is frustrated: all
    its couplers are satisfied by s* (J += -w s_i s_j) except the f-th in
    the loop's ascending coupler order (J += +w s_i s_j), so s* pays
    -(n - 2) w on an n-loop, the loop minimum;
  * the engine takes |J| <= 7: a loop that would push a coupler past 7 is
    drawn again (next attempt counter), up to MAX_ATTEMPTS times.  Removing
    a loop can itself push a coupler past 7 (loops of opposite signs
    sharing it); a move is kept only if the whole new instance is within
    the cap, and a proposal with no such attempt is void (slot -1: the
    instance stays, as a rejected move);
  * a cycle is identified by its ascending tuple of canonical coupler
    indices; the candidates of one size are ordered by that tuple;
  * draws: planted bit i = bit 31 of word 0 of Philox((chain, seed),
    (i, 0, 1, 8)); initial loop m, attempt a: words (w0, w1, w2, w3) of
    Philox((chain, seed), (m, a, 0, 8)) -> size by w0, cycle index
    floor(w1 n_size / 2^32), weight 1 + floor(w2 5 / 2^32), frustrated
    coupler floor(w3 size / 2^32); a move (step, proposal) removes loop
    floor(w0 M / 2^32) and takes its acceptance uniform from w1 of
    Philox((chain, seed), (step, proposal, 0, 9)), and draws the new loop
    from Philox((chain, seed), (step, proposal, 1 + a, 9)) as above.
"""
import numpy as np

from . import edges, num_sites, philox

P4_THRESHOLD = 429496730  # ~0.1 * 2^32
W_MAX = 5
J_CAP = 7
MAX_ATTEMPTS = 64
D_INIT, D_MOVE = 8, 9


def cycles(L, live=None):
    """{4: [...], 6: [...]}: every simple cycle of 4 and of 6 couplers of
    the live graph, each an ascending tuple of coupler indices, sorted.
    Plain depth-first search from every site."""
    ei, ej = edges(L)
    N = num_sites(L)
    alive = np.ones(N, bool) if live is None else np.asarray(live).astype(bool)
    adj = [[] for _ in range(N)]
    for e, (i, j) in enumerate(zip(ei, ej)):
        if alive[i] and alive[j]:
            adj[i].append((j, e))
            adj[j].append((i, e))
    out = {4: set(), 6: set()}
    for start in range(N):
        if not alive[start]:
            continue
        stack = [(start, [start], [])]
        while stack:
            v, path, es = stack.pop()
            for w, e in adj[v]:
                if w == start and len(es) + 1 in (4, 6) and len(es) >= 3:
                    out[len(es) + 1].add(tuple(sorted(es + [e])))
                elif w > start and w not in path and len(es) + 1 < 6:
                    stack.append((w, path + [w], es + [e]))
    return {n: sorted(c) for n, c in out.items()}


def planted_bits(L, chain, seed):
    N = num_sites(L)
    return np.array([philox((i, 0, 1, D_INIT), (chain, seed))[0] >> 31 for i in range(N)], np.uint8)


def _loop_from_words(w, cyc):
    size = 4 if int(w[0]) < P4_THRESHOLD else 6
    n = len(cyc[size])
    if n == 0:
        return None
    cid = (int(w[1]) * n) >> 32
    weight = 1 + ((int(w[2]) * W_MAX) >> 32)
    flip = (int(w[3]) * size) >> 32
    return size, cid, weight, flip


def loop_couplings(L, loop, cyc, bits):
    """(coupler indices, coupling deltas) of one loop (size, cid, weight, flip)."""
    size, cid, weight, flip = loop
    ei, ej = edges(L)
    s = 1 - 2 * np.asarray(bits, np.int64)
    idx = np.array(cyc[size][cid], np.int64)
    d = -weight * s[ei[idx]] * s[ej[idx]]
    d[flip] = -d[flip]
    return idx, d


def couplings(L, loops, cyc, bits):
    """J (int64 over all canonical couplers) and E_gs = -sum (n - 2) w."""
    J = np.zeros(len(edges(L)[0]), np.int64)
    e_gs = 0
    for lp in loops:
        idx, d = loop_couplings(L, lp, cyc, bits)
        J[idx] += d
        e_gs -= (lp[0] - 2) * lp[2]
    return J, e_gs


def _fits(J, idx, d):
    return np.all(np.abs(J[idx] + d) <= J_CAP)


def init(L, n_loops, chain, seed, live=None, cyc=None):
    """Planted instance: dict(loops, bits, J (int8), e_gs)."""
    cyc = cyc or cycles(L, live)
    bits = planted_bits(L, chain, seed)
    if live is not None:
        bits = bits * np.asarray(live, np.uint8)
    J = np.zeros(len(edges(L)[0]), np.int64)
    loops = []
    for m in range(n_loops):
        for a in range(MAX_ATTEMPTS):
            lp = _loop_from_words(philox((m, a, 0, D_INIT), (chain, seed)), cyc)
            if lp is None:
                raise ValueError("no cycles")
            idx, d = loop_couplings(L, lp, cyc, bits)
            if _fits(J, idx, d):
                J[idx] += d
                loops.append(lp)
                break
        else:
            raise ValueError("loop does not fit under the coupling cap")
    J2, e_gs = couplings(L, loops, cyc, bits)
    assert np.array_equal(J, J2)
    return dict(loops=loops, bits=bits, J=J.astype(np.int8), e_gs=e_gs)


def move(L, inst, chain, seed, step, proposal, live=None, cyc=None):
    """(slot, new loop, w_accept, J' (int8), e_gs') of a proposal; slot -1
    (and the instance's own J, e_gs) when no attempt fits the cap."""
    cyc = cyc or cycles(L, live)
    M = len(inst["loops"])
    w = philox((step, proposal, 0, D_MOVE), (chain, seed))
    slot = (int(w[0]) * M) >> 32
    rest = [lp for k, lp in enumerate(inst["loops"]) if k != slot]
    J, _ = couplings(L, rest, cyc, inst["bits"])
    for a in range(MAX_ATTEMPTS):
        lp = _loop_from_words(philox((step, proposal, 1 + a, D_MOVE), (chain, seed)), cyc)
        idx, d = loop_couplings(L, lp, cyc, inst["bits"])
        J_try = J.copy()
        J_try[idx] += d
        if np.all(np.abs(J_try) <= J_CAP):
            loops = list(inst["loops"])
            loops[slot] = lp
            J2, e_gs = couplings(L, loops, cyc, inst["bits"])
            return slot, lp, int(w[1]), J2.astype(np.int8), e_gs
    return -1, None, int(w[1]), np.asarray(inst["J"], np.int8), inst["e_gs"]
