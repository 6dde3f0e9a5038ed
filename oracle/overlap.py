"""Ground-state / first-excited-state overlaps from PT snapshots (Sec.
III.B, Fig. 3) -- TEST INFRASTRUCTURE ONLY (tests/, the smoke check and
bench.py's CPU baseline may use it; the product path never does).

The paper compares the ground states of an instance with its dominant first
excited states through the overlap 1 - 2 h / N (h = Hamming distance) and
normalises the median ground/excited overlap by the median ground/ground
overlap.  Readings (the paper gives no sampling details):
  * snapshots: after every `interval` sweeps, every live lane whose energy is
    at most e_cap contributes its configuration;
  * without fields s and -s have the same energy, so overlaps are taken as
    |1 - 2 h / N_live| over live sites and configurations are distinct up to
    the global flip;
  * the ground level E0 is the lowest captured energy, the first excited
    level E1 the next captured one; "dominant" excited states are the
    distinct configurations captured at E1;
  * ratio = median over (ground, excited) pairs / median over pairs of
    distinct ground states (1 when there is one ground state up to flip).
"""
import numpy as np

from . import num_sites, pt_init, pt_run


def snapshots(L, live, J, K, R, beta, key0, key1, swap_interval, interval, n_snap, e_cap):
    """[(snapshot, lane, energy, bits uint8[N])] in (snapshot, lane) order."""
    st = pt_init(L, live, J, K, R, key0, key1)
    N = num_sites(L)
    out = []
    for s in range(n_snap):
        pt_run(L, live, J, K, R, beta, key0, key1, swap_interval, interval, st)
        for lane in range(K * R):
            e = int(st.energy[lane])
            if e <= e_cap:
                bits = np.array([(int(st.spins[i]) >> lane) & 1 for i in range(N)], np.uint8)
                out.append((s, lane, e, bits))
    return out


def hamming(a, b, live=None):
    d = np.asarray(a, np.uint8) ^ np.asarray(b, np.uint8)
    if live is not None:
        d = d & np.asarray(live, np.uint8)
    return int(d.sum())


def summary(configs, live=None):
    """dict(e0, e1, n_gs, n_ex, med_ge, med_gg, ratio) from (energy, bits)
    pairs; e1 and the medians are None without an excited level."""
    n_live = len(configs[0][1]) if live is None else int(np.count_nonzero(live))
    levels = sorted({e for e, _ in configs})
    def distinct(level):
        kept = []
        for e, b in configs:
            if e != level:
                continue
            if all(hamming(b, k, live) not in (0, n_live) for k in kept):
                kept.append(b)
        return kept
    gs = distinct(levels[0])
    q = lambda h: abs(1.0 - 2.0 * h / n_live)
    gg = [q(hamming(gs[i], gs[j], live)) for i in range(len(gs)) for j in range(i + 1, len(gs))]
    med_gg = float(np.median(gg)) if gg else 1.0
    if len(levels) < 2:
        return dict(e0=levels[0], e1=None, n_gs=len(gs), n_ex=0, med_ge=None, med_gg=med_gg, ratio=None)
    ex = distinct(levels[1])
    ge = [q(hamming(g, x, live)) for g in gs for x in ex]
    med_ge = float(np.median(ge))
    return dict(e0=levels[0], e1=levels[1], n_gs=len(gs), n_ex=len(ex), med_ge=med_ge, med_gg=med_gg,
                ratio=med_ge / med_gg)
