"""Snapshot capture and ground / first-excited overlaps on the GPU (Sec.
III.B, Fig. 3) against the oracle: captured configurations are bit-exact
(as a multiset: slots come from an atomic counter), the overlap summary is
identical, and a full buffer stops writing while still counting."""
import numpy as np
import pytest

import oracle.overlap as O
import workloads

pytestmark = pytest.mark.gpu

SEED = 1605


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1605_03607_amd as hs
    hs.lib()
    return hs, torch


def _insts():
    out = []
    for n, (L, K, R) in enumerate([(2, 8, 2), (3, 6, 3)]):
        out.append(dict(L=L, J=workloads.couplings(L, "pm1", 17, n), live=workloads.missing_mask(L, 0.03 * n, 17, n),
                        K=K, R=R, beta=workloads.geometric_betas(0.3, 3.0, K), instance_id=40 + n))
    return out


def _run(hs, torch, insts, caps, interval, n_snap, capacity):
    b = hs.PTBatch(insts, SEED, swap_interval=1)
    n_words = (8 * max(d["L"] for d in insts) ** 2 + 63) // 64
    configs = torch.zeros((capacity, n_words), dtype=torch.int64, device="cuda")
    meta = torch.zeros((capacity, 4), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    for _ in range(n_snap):
        b.sweep(interval)
        b.capture(caps, configs, meta, count)
    torch.cuda.synchronize()
    b.close()
    return configs.cpu().numpy().view(np.uint64), meta.cpu().numpy(), int(count.item()), n_words


def test_capture_and_overlaps_match_oracle():
    hs, torch = _gpu()
    insts = _insts()
    caps = [-46, -103]  # the two lowest levels of each instance
    configs, meta, count, n_words = _run(hs, torch, insts, caps, 5, 30, 4096)
    assert 0 < count <= 4096
    for n, d in enumerate(insts):
        snaps = O.snapshots(d["L"], d["live"], d["J"], d["K"], d["R"], d["beta"], d["instance_id"], SEED, 1, 5, 30,
                            caps[n])
        want = sorted(((s + 1) * 5, lane, e, tuple(hs.pack_sites(bits).tolist())) for s, lane, e, bits in snaps)
        rows = [i for i in range(count) if meta[i, 0] == n]
        got = sorted((int(meta[i, 3]), int(meta[i, 1]), int(meta[i, 2]),
                      tuple(int(x) for x in configs[i, :(8 * d["L"] ** 2 + 63) // 64])) for i in rows)
        assert got == want, f"instance {n}"
        if not got:
            continue
        live = np.ones(8 * d["L"] ** 2, np.uint8) if d["live"] is None else np.asarray(d["live"], np.uint8)
        mask = np.zeros(n_words, np.uint64)
        mask[:len(hs.pack_sites(live))] = hs.pack_sites(live)
        s = hs.overlap_analyze(configs[rows], meta[rows, 2], mask, int(live.sum()))
        o = O.summary([(e, bits) for _, _, e, bits in snaps], live)
        for k in ("e0", "e1", "n_gs", "n_ex", "med_gg", "med_ge", "ratio"):
            assert s[k] == o[k], (n, k, s[k], o[k])


def test_full_buffer_counts_but_stops_writing():
    hs, torch = _gpu()
    insts = _insts()
    configs, meta, count, _ = _run(hs, torch, insts, [10 ** 6, 10 ** 6], 3, 4, 20)
    lanes = sum(d["K"] * d["R"] for d in insts)
    assert count == 4 * lanes
    assert set(meta[:, 0].tolist()) <= {0, 1}


@pytest.mark.parametrize("L,n,n_levels,frac_missing", [(3, 300, 3, 0.0), (4, 257, 2, 0.05), (2, 40, 1, 0.0),
                                                      (2, 1, 1, 0.0), (3, 2, 2, 0.0)])
def test_overlap_summary_of_many_states_matches_oracle(L, n, n_levels, frac_missing):
    """Many distinct states, repeats and global flips on up to three levels
    (the medians run over thousands of pairs with many equal overlaps)."""
    hs, torch = _gpu()
    N = 8 * L * L
    g = np.random.default_rng([L, n, n_levels])
    live = workloads.missing_mask(L, frac_missing, 23, L)
    live = np.ones(N, np.uint8) if live is None else np.asarray(live, np.uint8)
    base = g.integers(0, 2, (n // 3 + 1, N), dtype=np.uint8) & live
    pick = g.integers(0, len(base), n)
    bits = base[pick].copy()
    flip = g.random(n) < 0.3
    bits[flip] ^= live
    energy = (-40 + 2 * (pick % n_levels)).astype(np.int32)
    n_words = (N + 63) // 64
    configs = np.stack([np.pad(hs.pack_sites(b), (0, n_words - len(hs.pack_sites(b)))) for b in bits])
    mask = np.zeros(n_words, np.uint64)
    mask[:len(hs.pack_sites(live))] = hs.pack_sites(live)
    s = hs.overlap_analyze(configs, energy, mask, int(live.sum()))
    o = O.summary(list(zip(energy.tolist(), bits)), live)
    for k in ("e0", "e1", "n_gs", "n_ex", "med_gg", "med_ge", "ratio"):
        assert s[k] == o[k], (k, s[k], o[k])


def test_overlap_rejects_a_wrong_live_count():
    hs, torch = _gpu()
    configs = np.zeros((2, 1), np.uint64)
    mask = np.array([np.uint64(0xFF)], np.uint64)
    with pytest.raises(hs.HardspinError, match="popcount"):
        hs.overlap_analyze(configs, np.array([0, 1], np.int32), mask, 9)
