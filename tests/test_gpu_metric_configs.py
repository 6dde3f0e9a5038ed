"""GPU parity at the sizes and in the launch configurations the benchmarks
measure, against the CPU oracle:

  * the uneven batch (1024 instances C4..C12, 2% missing spins, K 24..48)
    exactly as the benchmark launches it: autotuned workgroup shape, one
    persistent launch held in a HIP graph; every instance re-run on the
    oracle after a 200-sweep prefix;
  * several thousand small instances of mixed K and R, three times the
    grid, so that every workgroup takes several instances from the queue
    (each reloads the LDS state of a new instance);
  * the 256 x C8 batch for one full 10^5-sweep benchmark step (one launch),
    sampled instances against oracle results stored by
    tests/golden/make_metric_configs.py;
  * hardness_eval at the search's configuration (32 restarts of K32 x R2,
    beta 0.1..5.0, stop on agreement or 10^5 sweeps), with the 64 seed
    instances in one launch, against stored oracle scores.
"""
import json
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import workloads
from test_gpu_parity import _assert_same, _gpu, _oracle_run, _say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "metric_configs.json")


def _workers():
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _check_all(b, insts, seed, swap_interval, n_sweeps, what):
    got = [b.state(n) for n in range(len(insts))]
    with ThreadPoolExecutor(_workers()) as pool:
        futs = [pool.submit(_oracle_run, d, seed, swap_interval, n_sweeps) for d in insts]
        for n, f in enumerate(futs):
            if n % 128 == 0:
                _say(f"{what}: instance {n} of {len(insts)}")
            _assert_same(got[n], f.result(), f"{what}: instance {n}")


def test_uneven_batch_as_benchmarked():
    """1024 instances of mixed size, the autotuner's shape, a HIP-graph
    replay of one persistent launch (the grid is smaller than the batch, so
    workgroups take several instances of different sizes from the queue):
    every instance bit-exact against the oracle."""
    import torch
    hs = _gpu()
    cfg = workloads.uneven_batch()
    insts = cfg["instances"]
    bw, us = hs.autotune(insts, cfg["seed"], swap_interval=cfg["swap_interval"], trial_sweeps=200)
    _say(f"uneven batch: autotuned block_waves={bw} ({us:.1f} us per sweep)")
    b = hs.PTBatch(insts, cfg["seed"], swap_interval=cfg["swap_interval"], block_waves=bw)
    grid, waves, lds, items, _ = b.launch_shape()
    _say(f"uneven batch: grid {grid}, {waves} wavefronts, {lds} LDS bytes per workgroup")
    assert waves == bw and grid < len(insts)
    n_sweeps = 200
    g = b.graph(n_sweeps)
    g.launch()
    torch.cuda.synchronize()
    assert b.measure() == 0
    _check_all(b, insts, cfg["seed"], cfg["swap_interval"], n_sweeps, "uneven batch")
    g.close()
    b.close()


def test_small_instances_three_times_the_grid():
    """C1..C3 instances with K R from 2 to 64: three times as many as the
    grid holds, so each workgroup runs at least three instances in turn;
    every instance bit-exact and every incremental energy exact."""
    hs = _gpu()
    rng = np.random.default_rng(2026)
    shapes = [(8, 2), (16, 1), (4, 4), (32, 2), (5, 3), (64, 1), (1, 2), (12, 5)]

    def make(n):
        out = []
        for i in range(n):
            L = int(rng.integers(1, 4))
            K, R = shapes[i % len(shapes)]
            out.append(dict(L=L, J=workloads.couplings(L, ["pm1", "pm3", "pm7"][i % 3], 4040, i),
                            live=workloads.missing_mask(L, 0.05 * (i % 2), 4040, i), K=K, R=R,
                            beta=workloads.geometric_betas(0.1, 4.0, K), instance_id=9000 + i))
        return out

    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    # at most 8 such workgroups fit on a compute unit (32 wavefronts of 8)
    insts = make(3 * 8 * cus)
    b = hs.PTBatch(insts, 77, swap_interval=2)
    grid, waves, _, _, _ = b.launch_shape()
    _say(f"small instances: {len(insts)} instances, grid {grid}, {waves} wavefronts")
    assert len(insts) >= 3 * grid
    n_sweeps = 150
    b.sweep(n_sweeps)
    assert b.measure() == 0
    _check_all(b, insts, 77, 2, n_sweeps, "small instances")
    b.close()


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_c8_batch_full_benchmark_step():
    """One 10^5-sweep step of the 256 x C8 benchmark (one persistent launch,
    exchange every sweep): instances 0, 85, 170, 255 equal the oracle's
    stored states, and every incremental energy equals the recomputed one."""
    hs = _gpu()
    gold = _golden()["c8_long"]
    cfg = workloads.batch_c8()
    assert gold["seed"] == cfg["seed"] and gold["sweeps"] == cfg["sweeps"] == 100_000
    insts = workloads.make_batch(cfg)
    b = hs.PTBatch(insts, cfg["seed"], swap_interval=1)
    _say("C8 full step: 10^5 sweeps of 256 instances")
    b.sweep(cfg["sweeps"])
    assert b.measure() == 0
    for rec in gold["instances"]:
        n = rec["index"]
        g = b.state(n)
        _say(f"C8 full step: instance {n}")
        assert np.array_equal(g["spins"], np.array(rec["spins"], np.uint64)), f"instance {n}: spins"
        assert g["perm"].tolist() == rec["perm"], f"instance {n}: perm"
        assert g["energy"].tolist() == rec["energy"], f"instance {n}: energy"
        assert g["emin"].tolist() == rec["emin"] and g["thit"].tolist() == rec["thit"], f"instance {n}: minima"
        assert g["swap_acc"].tolist() == rec["swap_acc"], f"instance {n}: swap_acc"
        assert g["t"] == rec["t"] == 100_000
    b.close()


def test_hardness_at_the_search_configuration():
    """hardness_eval as the search calls it (SearchConfig's defaults: 32
    restarts, K32 x R2, beta 0.1..5.0, exchange every sweep, 10^5-sweep
    cap): the 64 seed instances in one launch of 2048 runs (more runs than
    the grid, so workgroups take several from the queue); the candidates
    stored from the oracle match in ln TTS, E_gs, confirmation and every
    restart's sweep count."""
    hs = _gpu()
    from paper_1605_03607_amd.search import SearchConfig
    gold = _golden()["hardness"]
    c = SearchConfig()
    assert (c.restarts, c.K, c.R, c.swap_interval, c.s_max, c.seed) == (
        gold["restarts"], gold["K"], gold["R"], gold["swap_interval"], gold["s_max"], gold["seed"])
    assert np.array_equal(c.beta, workloads.geometric_betas(gold["beta"][0], gold["beta"][1], gold["K"]))
    seeds = workloads.search_seeds(64)
    cands = [dict(L=8, J=J, live=None, instance_id=i) for i, J in enumerate(seeds)]
    _say(f"hardness at the search configuration: {len(cands)} candidates x {c.restarts} restarts")
    ln, det = hs.hardness_eval(cands, c.restarts, c.K, c.R, c.beta, c.swap_interval, c.s_max, c.seed)
    for rec in gold["candidates"]:
        n = int(rec["name"][len("seed"):])
        assert cands[n]["instance_id"] == rec["instance_id"]
        _say(f"hardness: candidate {rec['name']} ln TTS {ln[n]:.4f} (oracle {rec['ln_tts']:.4f})")
        assert det[n]["e_gs"] == rec["e_gs"]
        assert int(det[n]["confirmed"]) == rec["confirmed"]
        assert det[n]["restart_sweeps"].tolist() == rec["r_sweeps"]
        assert ln[n] == rec["ln_tts"]


def test_uneven_batch_packed_lanes():
    """The uneven batch with HS_PACK_LANES: instances of one lattice size
    share a workgroup's 64 lanes (the queue hands out fewer work items than
    instances), and every instance is still bit-exact against the oracle,
    through a HIP-graph replay."""
    import torch
    hs = _gpu()
    cfg = workloads.uneven_batch()
    insts = cfg["instances"]
    b = hs.PTBatch(insts, cfg["seed"], swap_interval=cfg["swap_interval"], flags=hs.HS_PACK_LANES)
    grid, waves, lds, items, _ = b.launch_shape()
    _say(f"uneven batch packed: {items} packs for {len(insts)} instances, grid {grid}, {waves} wavefronts, "
         f"{lds} LDS bytes")
    assert items < len(insts)
    n_sweeps = 200
    g = b.graph(n_sweeps)
    g.launch()
    torch.cuda.synchronize()
    assert b.measure() == 0
    _check_all(b, insts, cfg["seed"], cfg["swap_interval"], n_sweeps, "uneven batch packed")
    g.close()
    b.close()


@pytest.mark.parametrize("swap_interval", [1, 3])
def test_packed_members_of_mixed_shapes(swap_interval):
    """Packs whose members differ in K, R, couplings, missing spins and
    ladders (including one-lane and one-temperature members), with the
    recorded temperature walk: bit-exact, and the walk equals the unpacked
    launch's."""
    import torch
    hs = _gpu()
    shapes = [(3, 32, 1), (3, 24, 1), (3, 8, 4), (3, 16, 2), (3, 1, 1), (3, 63, 1), (2, 5, 3), (2, 40, 1),
              (2, 12, 2), (2, 1, 7), (4, 20, 1), (4, 44, 1)]
    insts = []
    for n, (L, K, R) in enumerate(shapes):
        insts.append(dict(L=L, J=workloads.couplings(L, ["pm1", "pm3", "pm7"][n % 3], 123, n),
                          live=workloads.missing_mask(L, 0.03 * (n % 2), 123, n), K=K, R=R,
                          beta=workloads.geometric_betas(0.1 + 0.03 * n, 3.0 + 0.2 * n, K), instance_id=500 + n))
    n_sweeps = 90
    walks = []
    for flags in (hs.HS_PACK_LANES, 0):
        b = hs.PTBatch(insts, 31, swap_interval=swap_interval, flags=flags)
        items = b.launch_shape()[3]
        _say(f"mixed packs (swap interval {swap_interval}, flags {flags}): {items} work items")
        assert (items < len(insts)) == (flags != 0)
        cap = n_sweeps // swap_interval + 1
        walk = torch.full((len(insts), cap, 64), 255, dtype=torch.uint8, device="cuda")
        b.sweep_record(n_sweeps, walk)
        torch.cuda.synchronize()
        walks.append(walk.cpu().numpy())
        assert b.measure() == 0
        if flags:
            _check_all(b, insts, 31, swap_interval, n_sweeps, "mixed packs")
        b.close()
    assert np.array_equal(walks[0], walks[1])
