"""Temperature-walk recording and mixing-time statistics on the GPU
(Sec. III.B) against the oracle: recorded walks are bit-exact, the
autocorrelation sums and hot-half counts are exact integers, and tau
agrees to rounding."""
import numpy as np
import pytest

import oracle.walk as W
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


def _instances():
    shapes = [(2, 8, 2, "pm3"), (3, 6, 4, "pm7"), (4, 16, 1, "pm1"), (1, 32, 2, "pm7")]
    out = []
    for n, (L, K, R, a) in enumerate(shapes):
        out.append(dict(L=L, J=workloads.couplings(L, a, 61, n), live=workloads.missing_mask(L, 0.02 * (n % 2), 61, n),
                        K=K, R=R, beta=workloads.geometric_betas(0.2, 4.0, K), instance_id=300 + n))
    return out


@pytest.mark.parametrize("si,n_emcs,cap", [(10, 60, 50), (1, 200, 256), (3, 40, 40)])
def test_recorded_walk_matches_oracle_and_sweeps_are_unchanged(si, n_emcs, cap):
    """Exchange every sweep, every 3rd and every 10th; a buffer shorter than
    the run (later passes are not written), longer, and exactly full."""
    hs, torch = _gpu()
    insts = _instances()
    b = hs.PTBatch(insts, SEED, swap_interval=si)
    walk = torch.full((len(insts), cap, 64), 0xEE, dtype=torch.uint8, device="cuda")
    b.sweep_record(si * n_emcs, walk)
    ref = hs.PTBatch(insts, SEED, swap_interval=si)
    ref.sweep(si * n_emcs)
    got = walk.cpu().numpy()
    for n, d in enumerate(insts):
        C = d["K"] * d["R"]
        traj, st = W.walk(d["L"], d["live"], d["J"], d["K"], d["R"], d["beta"], d["instance_id"], SEED, si, n_emcs)
        rec = min(cap, n_emcs)
        assert np.array_equal(got[n, :rec, :C], traj[:rec]), f"instance {n}"
        assert np.all(got[n, :, C:] == 0xEE)  # beyond K R: untouched
        assert np.all(got[n, rec:] == 0xEE)  # beyond the run: untouched
        a, r = b.state(n), ref.state(n)
        for name in ("spins", "perm", "energy", "emin", "thit", "swap_acc"):
            assert np.array_equal(a[name], r[name]), name
        assert np.array_equal(a["perm"], st.perm)
    b.close()
    ref.close()


@pytest.mark.parametrize("T,max_lag,K,R", [(3000, 300, 32, 2), (257, 64, 32, 2), (40, 100, 32, 2), (0, 5, 32, 2),
                                           (1031, 131, 6, 4), (515, 77, 16, 1), (3, 70, 64, 1)])
def test_autocorrelation_sums_are_exact(T, max_lag, K, R):
    """Synthetic walks spanning several time tiles and lag tiles with ragged
    ends, a lag range past the run, an empty run, and fewer than 64
    configurations (the rest of each 64-byte row is ignored)."""
    hs, torch = _gpu()
    rng = np.random.default_rng(T + max_lag)
    cap, n_inst = max(T, 1) + 3, 5
    host = rng.integers(0, K, size=(n_inst, cap, 64)).astype(np.uint8)
    walk = torch.from_numpy(host).cuda()
    acf, hot = hs.walk_autocorr(walk, T, K, R, max_lag)
    for n in range(n_inst):
        traj = host[n, :T, :K * R]
        assert np.array_equal(acf[n], W.acf_sums(traj, K, max_lag)), n
        want_hot = np.zeros(64, np.int64)
        want_hot[:K * R] = W.hot_counts(traj, K) if T else 0
        assert np.array_equal(hot[n], want_hot), n


def test_tau_from_a_recorded_run_matches_oracle():
    hs, torch = _gpu()
    L, K, R, si, n_emcs = 2, 12, 2, 10, 400
    d = dict(L=L, J=workloads.couplings(L, "pm3", 5, 1), live=None, K=K, R=R,
             beta=workloads.geometric_betas(0.2, 3.0, K), instance_id=9)
    b = hs.PTBatch([d], SEED, swap_interval=si)
    walk = torch.zeros((1, n_emcs, 64), dtype=torch.uint8, device="cuda")
    b.sweep_record(si * n_emcs, walk)
    acf, hot = hs.walk_autocorr(walk, n_emcs, K, R, 120)
    traj, _ = W.walk(L, None, d["J"], K, R, d["beta"], 9, SEED, si, n_emcs)
    S = W.acf_sums(traj, K, 120)
    assert np.array_equal(acf[0], S)
    got = hs.walk_tau(acf[0], n_emcs)
    want = W.tau_int(S, n_emcs)
    assert got[1:] == tuple(want[1:]) and abs(got[0] - want[0]) <= 1e-12 * want[0]
    assert np.array_equal(hot[0, :K * R], W.hot_counts(traj, K))
    b.close()
