"""GPU parity: the gfx950 PT kernels against the CPU oracle, bit-exact, on the
same seeded inputs (spins, slot permutations, energies, running minima,
first-hit sweeps, exchange counters, sweep counters)."""
import sys

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

SEED = 1605


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1605_03607_amd as hs
    hs.lib()
    return hs


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle_run(d, seed, swap_interval, n_sweeps, init_spins=None, stop=False, chunks=None):
    st = oracle.pt_init(d["L"], d.get("live"), d["J"], d["K"], d["R"], d["instance_id"], seed,
                        init_spins=init_spins)
    for n in (chunks or [n_sweeps]):
        oracle.pt_run(d["L"], d.get("live"), d["J"], d["K"], d["R"], d["beta"], d["instance_id"],
                      seed, swap_interval, n, st, stop_on_agreement=stop)
    return st


def _assert_same(g, o, what=""):
    K_R = len(o.perm)
    assert np.array_equal(g["spins"], o.spins), f"{what}: spins differ"
    assert np.array_equal(g["perm"], o.perm), f"{what}: perm differs"
    assert np.array_equal(g["energy"], o.energy), f"{what}: energy differs"
    assert np.array_equal(g["emin"], o.emin), f"{what}: emin differs"
    assert np.array_equal(g["thit"], o.thit), f"{what}: thit differs"
    if K_R and len(o.swap_acc) > 1 or o.swap_acc[0] != 0:
        assert np.array_equal(g["swap_acc"][:len(o.swap_acc)], o.swap_acc), f"{what}: swap_acc"
    assert g["t"] == int(o.t[0]), f"{what}: t"
    assert g["stopped"] == int(o.stopped[0]), f"{what}: stopped"


def test_c4_parity_config_full_length():
    """One C4 instance, J in {+-1}, K = 16 (0.2..3.0), R = 1, an exchange
    pass after every sweep, 10^4 sweeps: identical at several checkpoints."""
    hs = _gpu()
    cfg = workloads.parity_c4()
    insts = workloads.make_batch(cfg)
    d = insts[0]
    b = hs.PTBatch(insts, SEED, swap_interval=1)
    o = oracle.pt_init(d["L"], None, d["J"], d["K"], d["R"], d["instance_id"], SEED)
    _assert_same(b.state(0), o, "init")
    done = 0
    for target in (1, 2, 7, 100, 1000, cfg["sweeps"]):
        _say(f"C4 parity: sweeps {done} -> {target}")
        b.sweep(target - done)
        oracle.pt_run(d["L"], None, d["J"], d["K"], d["R"], d["beta"], d["instance_id"], SEED, 1,
                      target - done, o)
        done = target
        _assert_same(b.state(0), o, f"after {target} sweeps")
    assert b.measure() == 0
    b.close()


def _uneven_instances():
    rng = np.random.default_rng(7)
    shapes = [(1, 2, 1), (1, 4, 16), (2, 8, 8), (3, 5, 3), (4, 64, 1), (5, 24, 2), (7, 31, 2),
              (8, 32, 2), (9, 13, 4), (12, 48, 1), (6, 1, 64), (11, 2, 32), (2, 1, 1)]
    insts = []
    for n, (L, K, R) in enumerate(shapes):
        alphabet = ["pm1", "pm3", "pm7"][n % 3]
        insts.append(dict(L=L, J=workloads.couplings(L, alphabet, 99, n),
                          live=workloads.missing_mask(L, 0.02 * (n % 3), 99, n), K=K, R=R,
                          beta=workloads.geometric_betas(0.1 + 0.05 * n, 2.0 + 0.5 * n, K),
                          instance_id=1000 + n))
    return insts


@pytest.mark.parametrize("swap_interval", [1, 3])
def test_uneven_batch_parity(swap_interval):
    """Mixed sizes C1..C12, odd cell counts, missing spins, K R from 2 to 64,
    in one persistent launch; every instance matches the oracle."""
    hs = _gpu()
    insts = _uneven_instances()
    b = hs.PTBatch(insts, SEED, swap_interval=swap_interval)
    n_sweeps = 120
    b.sweep(50)
    b.sweep(n_sweeps - 50)
    for n, d in enumerate(insts):
        _say(f"uneven parity: instance {n} L={d['L']} K={d['K']} R={d['R']}")
        o = _oracle_run(d, SEED, swap_interval, n_sweeps)
        _assert_same(b.state(n), o, f"instance {n}")
    assert b.measure() == 0
    b.close()


@pytest.mark.parametrize("waves", [1, 2, 4, 8, 16])
def test_launch_shape_does_not_change_results(waves):
    hs = _gpu()
    insts = workloads.make_batch(workloads.batch_c8(), 3)
    b = hs.PTBatch(insts, SEED, swap_interval=2, block_waves=waves)
    b.sweep(40)
    for n, d in enumerate(insts):
        o = _oracle_run(d, SEED, 2, 40)
        _assert_same(b.state(n), o, f"waves={waves} instance {n}")
    b.close()


@pytest.mark.parametrize("waves,K,R", [(3, 48, 1), (5, 32, 2), (6, 32, 2), (7, 32, 2), (12, 20, 3), (16, 1, 7)])
def test_exchange_walkers_and_hand_over_shapes(waves, K, R):
    """Launch shapes at the edges of the exchange pass's work split: one
    walking wavefront per replica set, and other wavefronts handing over the
    walkers' next draws only when there are at least three wavefronts per
    walker (on with 3 for one set and 6 or 7 for two, off with 5, and never
    with three sets); one-temperature sets have no pairs.  An exchange pass
    after every sweep; bit-exact against the oracle."""
    hs = _gpu()
    insts = []
    for n, L in enumerate((4, 5, 3)):
        insts.append(dict(L=L, J=workloads.couplings(L, "pm7", 77, n), live=workloads.missing_mask(L, 0.02, 77, n),
                          K=K, R=R, beta=workloads.geometric_betas(0.1, 5.0, K), instance_id=4200 + n))
    b = hs.PTBatch(insts, SEED, swap_interval=1, block_waves=waves)
    assert b.launch_shape()[1] == waves
    _say(f"walker shapes: {waves} wavefronts, K={K} R={R}")
    b.sweep(60)
    assert b.measure() == 0
    for n, d in enumerate(insts):
        _assert_same(b.state(n), _oracle_run(d, SEED, 1, 60), f"waves={waves} K={K} R={R} instance {n}")
    b.close()


def test_init_from_buffer_and_gauge_images():
    """Caller-provided initial spins; and the gauge transform (J', s0') =
    (gJg, g.s0) gives s'(t) = g.s(t) with identical energies and perms."""
    hs = _gpu()
    L, K, R = 6, 16, 4
    N = 8 * L * L
    J = workloads.couplings(L, "pm7", 5, 0)
    live = workloads.missing_mask(L, 0.02, 5, 0)
    ei, ej = oracle.edges(L)
    g = workloads.gauge_vector(N, 5)
    sg = 1 - 2 * g.astype(np.int64)
    Jg = (J * sg[ei] * sg[ej]).astype(np.int8)
    beta = workloads.geometric_betas(0.2, 3.0, K)
    s0 = workloads.random_spins(N, K * R, 5, 0)
    lv = live.astype(bool)
    s0[~lv] = 0
    gw = np.where(g == 1, np.uint64((1 << 64) - 1), np.uint64(0)).astype(np.uint64)
    lane_mask = np.uint64((1 << (K * R)) - 1)
    d1 = dict(L=L, J=J, live=live, K=K, R=R, beta=beta, instance_id=3)
    d2 = dict(d1, J=Jg)
    s1 = (s0 ^ gw) & lane_mask
    s1[~lv] = 0
    b = hs.PTBatch([d1, d2], SEED, swap_interval=1, flags=hs.HS_INIT_FROM_BUFFER,
                   init_spins=np.concatenate([s0, s1]))
    b.sweep(200)
    a, c = b.state(0), b.state(1)
    o = _oracle_run(d1, SEED, 1, 200, init_spins=s0)
    _assert_same(a, o, "from buffer")
    assert np.array_equal((a["spins"] ^ gw)[lv] & lane_mask, c["spins"][lv])
    for name in ("perm", "energy", "emin", "thit", "swap_acc"):
        assert np.array_equal(a[name], c[name]), name
    b.close()


def test_extra_exchange_pass_matches_oracle():
    hs = _gpu()
    insts = workloads.make_batch(workloads.batch_c8(), 2)
    b = hs.PTBatch(insts, SEED, swap_interval=0)
    b.sweep(30)
    b.swap()
    b.sweep(5)
    for n, d in enumerate(insts):
        st = oracle.pt_init(d["L"], None, d["J"], d["K"], d["R"], d["instance_id"], SEED)
        oracle.pt_run(d["L"], None, d["J"], d["K"], d["R"], d["beta"], d["instance_id"], SEED, 0,
                      30, st)
        oracle.pt_swap_extra(d["L"], None, d["J"], d["K"], d["R"], d["beta"], d["instance_id"],
                             SEED, st)
        oracle.pt_run(d["L"], None, d["J"], d["K"], d["R"], d["beta"], d["instance_id"], SEED, 0,
                      5, st)
        _assert_same(b.state(n), st, f"instance {n}")
    b.close()


def test_stop_on_agreement_matches_oracle():
    hs = _gpu()
    insts = []
    for n in range(6):
        L = 2 + n % 3
        insts.append(dict(L=L, J=workloads.couplings(L, "pm3", 41, n), live=None, K=8, R=2,
                          beta=workloads.geometric_betas(0.1, 5.0, 8), instance_id=50 + n))
    b = hs.PTBatch(insts, SEED, swap_interval=1, flags=hs.HS_STOP_ON_AGREEMENT)
    b.sweep(5000)
    for n, d in enumerate(insts):
        o = _oracle_run(d, SEED, 1, 5000, stop=True)
        _assert_same(b.state(n), o, f"instance {n}")
        assert o.stopped[0] == 1
    b.close()


def test_zero_sweeps_and_empty_batch():
    hs = _gpu()
    insts = workloads.make_batch(workloads.parity_c4())
    b = hs.PTBatch(insts, SEED)
    b.sweep(0)
    d = insts[0]
    o = oracle.pt_init(d["L"], None, d["J"], d["K"], d["R"], d["instance_id"], SEED)
    _assert_same(b.state(0), o, "zero sweeps")
    b.close()
    e = hs.PTBatch([], SEED)
    e.sweep(10)
    e.close()


def test_free_spins_and_ferromagnet_match_oracle():
    """Degenerate couplings: J = 0 (every attempt accepted, energy stays 0)
    and the all-ferromagnetic instance (ground states all-up and all-down,
    E = -|E|), bit-exact against the oracle, and hardness_eval finds the
    closed-form ground energies."""
    hs = _gpu()
    L, K, R = 3, 8, 2
    n_e = 24 * L * L - 8 * L
    beta = workloads.geometric_betas(0.2, 4.0, K)
    insts = [dict(L=L, J=np.zeros(n_e, np.int8), live=None, K=K, R=R, beta=beta, instance_id=51),
             dict(L=L, J=np.full(n_e, -1, np.int8), live=None, K=K, R=R, beta=beta, instance_id=52)]
    b = hs.PTBatch(insts, SEED, swap_interval=1)
    b.sweep(300)
    for n, d in enumerate(insts):
        _say(f"degenerate couplings: instance {n}")
        o = oracle.pt_init(L, None, d["J"], K, R, d["instance_id"], SEED)
        oracle.pt_run(L, None, d["J"], K, R, beta, d["instance_id"], SEED, 1, 300, o)
        _assert_same(b.state(n), o, f"instance {n}")
    assert np.all(b.state(0)["energy"][:K * R] == 0)
    assert b.measure() == 0
    b.close()
    cands = [dict(L=L, J=d["J"], live=None, instance_id=d["instance_id"]) for d in insts]
    ln, det = hs.hardness_eval(cands, 4, K, R, beta, 1, 5000, 77)
    assert det[0]["e_gs"] == 0 and det[1]["e_gs"] == -n_e
    assert all(np.isfinite(ln))


def test_hardness_eval_matches_oracle():
    hs = _gpu()
    beta = workloads.geometric_betas(0.1, 5.0, 8)
    cands = []
    for n in range(4):
        L = 2 + n % 2
        cands.append(dict(L=L, J=workloads.couplings(L, "pm7", 61, n),
                          live=workloads.missing_mask(L, 0.05, 61, n), instance_id=700 + n))
    ln, det = hs.hardness_eval(cands, 6, 8, 2, beta, 1, 4000, 77)
    for n, c in enumerate(cands):
        _say(f"hardness parity: candidate {n}")
        o = oracle.hardness_eval(c["L"], c["live"], c["J"], c["instance_id"], 77, 6, 8, 2, beta,
                                 1, 4000)
        assert det[n]["e_gs"] == o["e_gs"]
        assert det[n]["confirmed"] == o["confirmed"]
        assert det[n]["sweeps_total"] == int(o["r_sweeps"].sum())
        assert np.array_equal(det[n]["restart_sweeps"], o["r_sweeps"])
        assert (ln[n] == o["ln_tts"]) or (np.isinf(ln[n]) and np.isinf(o["ln_tts"]))


@pytest.mark.parametrize("swap_interval", [1, 10])
def test_full_size_c8_batch_sampled(swap_interval):
    """The 256-instance C8 batch in the benchmark's launch configuration
    (exchange every sweep, and every 10th sweep as in the elementary Monte
    Carlo step): sampled instances re-run one by one on the oracle match
    bit-exactly, and every instance's incremental energies equal the
    recomputed ones."""
    hs = _gpu()
    cfg = workloads.batch_c8()
    insts = workloads.make_batch(cfg)
    b = hs.PTBatch(insts, cfg["seed"], swap_interval=swap_interval)
    n_sweeps = 150
    b.sweep(n_sweeps)
    assert b.measure() == 0
    for n in (0, 137, 255):
        _say(f"C8 full-batch parity (swap_interval {swap_interval}): instance {n}")
        o = _oracle_run(insts[n], cfg["seed"], swap_interval, n_sweeps)
        _assert_same(b.state(n), o, f"instance {n}")
    b.close()


def test_full_size_c8_batch_every_instance_prefix():
    """All 256 instances of the benchmark batch after a 10^3-sweep prefix of
    the benchmark launch (one persistent launch, exchange every sweep),
    each re-run on the oracle in a pool of host threads: bit-exact."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    hs = _gpu()
    cfg = workloads.batch_c8()
    insts = workloads.make_batch(cfg)
    n_sweeps = 1000
    b = hs.PTBatch(insts, cfg["seed"], swap_interval=1)
    b.sweep(n_sweeps)
    assert b.measure() == 0
    got = [b.state(n) for n in range(len(insts))]
    b.close()
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(workers) as pool:
        futs = [pool.submit(_oracle_run, d, cfg["seed"], 1, n_sweeps) for d in insts]
        for n, f in enumerate(futs):
            if n % 32 == 0:
                _say(f"C8 every-instance prefix: instance {n} of {len(insts)}")
            _assert_same(got[n], f.result(), f"instance {n}")


@pytest.mark.parametrize("K,R", [(32, 2), (64, 1), (1, 64), (2, 32)])
def test_largest_lattice_parity(K, R):
    """C16 (the largest lattice the engine takes, N = 2048) with 2% missing
    spins and 64 lanes: the launch picks the most compact LDS layout that
    fits (the largest R needs the most room for run ends), and every shape
    matches the oracle."""
    hs = _gpu()
    L = 16
    d = dict(L=L, J=workloads.couplings(L, "pm7", 21, K), live=workloads.missing_mask(L, 0.02, 21, K),
             K=K, R=R, beta=workloads.geometric_betas(0.1, 5.0, K),
             instance_id=77)
    _say(f"C16 parity: K={K} R={R}")
    b = hs.PTBatch([d], SEED, swap_interval=1)
    b.sweep(30)
    o = _oracle_run(d, SEED, 1, 30)
    _assert_same(b.state(0), o, f"C16 K={K} R={R}")
    assert b.measure() == 0
    b.close()
