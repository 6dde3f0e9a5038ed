"""Throughput benchmark: spin-flip attempts/s of batched parallel tempering.

Workload: 256 independent Chimera C8 instances (N = 512, 1472 couplers),
J uniform in {+-1..+-7}, K = 32 temperatures (beta geometric 0.1..5.0) x
R = 2 replica sets = 64 lanes per instance, an exchange pass after every
Metropolis sweep (--swap-interval 10 gives the elementary Monte Carlo step of
Sec. III.B).  One step = 10^5 sweeps of the whole batch (Metropolis sweeps,
exchange passes, running minima) in one persistent launch, continuing the
same chains.

Prints one JSON line (rank 0, N = 1 GPU) with the roofline of the sweep kernel
(integer VALU issue bound) and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

# Op count and peak of the sweep kernel's roofline (integer VALU issue), fixed
# in roofline_opcount.json: the reported frac uses the reference count (22 ops
# per attempt, the minimal formulation fixed before tuning); the count of the
# formulation this kernel runs (15.5) is reported beside it.
with open(os.path.join(ROOT, "roofline_opcount.json")) as _f:
    OPCOUNT = json.load(_f)
PEAK_INT32_OPS = float(OPCOUNT["peak_lane_ops_per_s"])
A_OPS = float(OPCOUNT["reference"]["ops_per_attempt"])
A_OPS_IMPL = float(OPCOUNT["implemented"]["ops_per_attempt"])
ISSUE_RATES_FILE = os.path.join(ROOT, "profiles", "isa_issue_rates.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1605_03607_amd", "csrc", "hs_pt.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pt_sweep_c8x256_traffic.json")


def kernel_fingerprint():
    """Hash of the sweep-kernel source without comments and blank lines, so
    that edits of comments alone keep the committed counters valid."""
    import hashlib
    import re
    with open(KERNEL_SOURCE) as f:
        src = f.read()
    token = re.compile(r'"(?:\\.|[^"\\])*"|//[^\n]*|/\*.*?\*/', re.S)
    code = token.sub(lambda m: m.group(0) if m.group(0).startswith('"') else " ", src)
    lines = [" ".join(l.split()) for l in code.splitlines()]
    return hashlib.sha256("\n".join(l for l in lines if l).encode()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per sweep-kernel launch from the committed counter summary,
    or None if the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_fingerprint") != kernel_fingerprint():
        return None
    return t.get("bytes_per_launch")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--sweeps", type=int, default=None, help="sweeps per step (default 10^5)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--block-waves", type=int, default=0)
    p.add_argument("--instances", type=int, default=256,
                   help="batch workload: number of instances (256: the benchmark)")
    p.add_argument("--lattice", type=int, default=8,
                   help="batch workload: Chimera side L of the 256 instances (8: the C8 benchmark; other sizes show "
                        "how the per-sweep costs amortise)")
    p.add_argument("--swap-interval", type=int, default=None,
                   help="sweeps between exchange passes (default: the workload's)")
    p.add_argument("--copy-mib", type=int, default=0,
                   help="after the timed steps, run one plain device copy of this many MiB "
                        "(reference kernel for scaling HBM byte counters)")
    p.add_argument("--workload", choices=["c8", "uneven", "search", "search-reverse", "surrogate", "tau", "lao",
                                          "overlap"],
                   default="c8",
                   help="c8: the 256 x C8 batch (default); uneven: 1024 instances C4..C12, "
                        "autotuned shape, HIP-graph replay, live attempts/s; search: bounded "
                        "plain / surrogate-screened / random-screened instance search")
    p.add_argument("--pack", choices=["auto", "on", "off"], default="auto",
                   help="uneven workload: lane packing of instances of one size (auto: the tuner decides)")
    p.add_argument("--tune-cache", default=None,
                   help="uneven workload: JSON file caching the tuned launch plan by the batch's size classes")
    p.add_argument("--search-steps", type=int, default=20)
    p.add_argument("--search-chains", type=int, default=64)
    p.add_argument("--search-groups", type=int, default=4,
                   help="chain groups stepping concurrently on their own streams (search workloads)")
    p.add_argument("--search-top", type=int, default=2,
                   help="screened arms: proposals per chain scored by PT after the screen")
    p.add_argument("--search-log", default=None,
                   help="search workloads: write every acceptance decision as a JSON line to this file")
    p.add_argument("--validate", choices=["during", "after"], default="during",
                   help="search workloads: re-score counted states on a stream of their own while the search "
                        "runs (during), or after its last step")
    p.add_argument("--search-block-waves", default="auto",
                   help="search workload: wavefronts per PT workgroup of hardness_eval, 0 for the library's choice "
                        "(16 at C8), or auto: 16 for the plain arm, whose steps wait for their slowest restart, and "
                        "8 for the screened arms, which score twice the restarts per step and gain more from two "
                        "workgroups per CU than they lose on the slowest restart (measured)")
    p.add_argument("--gnn-cus", type=int, default=0,
                   help="surrogate arm: compute units set aside for the surrogate's kernels (0: none); the arm's PT "
                        "launches use the others")
    p.add_argument("--hw-queues", type=int, default=8,
                   help="search workloads: hardware queues of the process (GPU_MAX_HW_QUEUES, at most 32); "
                        "the chain groups and the validation stream each need one")
    p.add_argument("--tau-emcs", type=int, default=20000, help="EMCS of the --workload tau run")
    p.add_argument("--probe", action="store_true",
                   help="also measure instruction issue rates (libhsprobe.so)")
    return p.parse_args()


def cpu_baseline(cfg, insts, budget_s):
    """The CPU oracle, as it stands, on the host's cores: one instance per
    thread, a prefix of the sweeps, scaled to attempts/s."""
    import oracle
    cores = host_cores()
    lanes = cfg["K"] * cfg["R"]
    n_sites = 8 * cfg["L"] ** 2
    # calibrate: one instance, a few sweeps
    d = insts[0]
    st = oracle.pt_init(d["L"], None, d["J"], d["K"], d["R"], d["instance_id"], cfg["seed"])
    t0 = time.perf_counter()
    oracle.pt_run(d["L"], None, d["J"], d["K"], d["R"], d["beta"], d["instance_id"], cfg["seed"],
                  cfg["swap_interval"], 5, st)
    per_sweep = (time.perf_counter() - t0) / 5
    sweeps = max(10, int(budget_s / per_sweep))
    done = []

    def work(i):
        d = insts[i]
        s = oracle.pt_init(d["L"], None, d["J"], d["K"], d["R"], d["instance_id"], cfg["seed"])
        oracle.pt_run(d["L"], None, d["J"], d["K"], d["R"], d["beta"], d["instance_id"],
                      cfg["seed"], cfg["swap_interval"], sweeps, s)
        done.append(i)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(cores)]
    t0 = time.perf_counter()
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    el = time.perf_counter() - t0
    attempts = cores * sweeps * n_sites * lanes
    return {"value": attempts / el, "unit": "spin-flip attempts/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{cores} C8 instances x {sweeps} sweeps (one per thread), "
                      f"{el:.1f} s wall"}


# Host threads the CPU baselines use at most: 16, a per-GPU share of a
# many-core host, whatever count the operating system reports for the whole
# machine (the count actually used is recorded with every baseline).
HOST_THREAD_CAP = 16


def host_cores(limit=HOST_THREAD_CAP):
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return max(1, min(cores, limit))


def host_info():
    """What the host reports about its CPUs, recorded with every CPU baseline."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"host_cpu_model": model, "host_nproc": os.cpu_count(), "host_affinity_cpus": aff,
            "thread_cap": HOST_THREAD_CAP,
            "thread_cap_reason": "at most 16 threads, a per-GPU share of the host; cores = min(affinity CPUs, cap, "
                                 "instances in the sample)"}


def emit(line):
    """Prints the benchmark's JSON line; a CPU baseline carries what the host
    reports about its CPUs."""
    if isinstance(line.get("cpu_baseline"), dict):
        line["cpu_baseline"].update(host_info())
    print(json.dumps(line), flush=True)


def measured_issue_rates():
    """Issue rates of single instruction classes measured on an MI355X
    (bench.py --probe), from the committed summary, or None."""
    try:
        with open(ISSUE_RATES_FILE) as f:
            return json.load(f).get("lane_ops_per_s")
    except (OSError, ValueError):
        return None


def alu_roofline(attempts, kernel_s):
    """The int32-VALU roofline fields of a sweep-kernel launch: achieved
    lane operations per second at the reference op count, its fraction of
    the peak, and the same at the implemented op count."""
    per_s = attempts / kernel_s if kernel_s > 0 else 0.0
    return {"bound": "alu", "achieved": per_s * A_OPS / 1e12, "peak": PEAK_INT32_OPS / 1e12,
            "unit": "Tops/s (int32 lane operations)", "frac": per_s * A_OPS / PEAK_INT32_OPS,
            "ops_per_attempt": A_OPS, "ops_per_attempt_implemented": A_OPS_IMPL,
            "frac_implemented_ops": per_s * A_OPS_IMPL / PEAK_INT32_OPS,
            "peak_derivation": OPCOUNT["peak_derivation"], "opcount_file": "roofline_opcount.json"}


def pt_roofline(attempts, kernel_ms, launches, kernel, wall_s=None):
    """Roofline object of the sweep kernel from the attempts of `launches`
    launches and their summed device time (HIP events on the launch
    streams): algorithmic int32 lane operations per launch over the mean
    launch duration.  With wall_s, also the whole chip's share over that
    wall time (launches of concurrent groups overlap, so their durations
    add up to more than the time they span)."""
    out = alu_roofline(attempts, kernel_ms / 1e3)
    out.update({"traffic": None, "kernel_ms_avg": kernel_ms / max(1, launches), "launches": launches,
                "kernel": kernel})
    if wall_s:
        out["chip_frac_over_wall"] = attempts * A_OPS / wall_s / PEAK_INT32_OPS
        out["wall_s"] = wall_s
    return out


def mixed_cpu_baseline(insts, seed, swap_interval, budget_s):
    """The CPU oracle, as it stands, on a mixed batch: one instance per
    host thread, taken evenly across the batch (each with its own size,
    missing spins and ladder), a prefix of the sweeps sized to the budget
    from the slowest of them; live spin-flip attempts per second."""
    import oracle
    cores = min(host_cores(), len(insts))
    pick = [insts[(i * len(insts)) // cores] for i in range(cores)]
    per_sweep = 0.0
    for d in pick:
        st = oracle.pt_init(d["L"], d["live"], d["J"], d["K"], d["R"], d["instance_id"], seed)
        oracle.pt_run(d["L"], d["live"], d["J"], d["K"], d["R"], d["beta"], d["instance_id"], seed,
                      swap_interval, 2, st)
        t0 = time.perf_counter()
        oracle.pt_run(d["L"], d["live"], d["J"], d["K"], d["R"], d["beta"], d["instance_id"], seed,
                      swap_interval, 10, st)
        per_sweep = max(per_sweep, (time.perf_counter() - t0) / 10)
    sweeps = max(5, int(budget_s / per_sweep))

    def work(i):
        d = pick[i]
        st = oracle.pt_init(d["L"], d["live"], d["J"], d["K"], d["R"], d["instance_id"], seed)
        oracle.pt_run(d["L"], d["live"], d["J"], d["K"], d["R"], d["beta"], d["instance_id"], seed,
                      swap_interval, sweeps, st)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(cores)]
    t0 = time.perf_counter()
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    el = time.perf_counter() - t0
    live = sum(int(d["K"]) * int(d["R"]) * int(np.count_nonzero(d["live"])) for d in pick) * sweeps
    return {"value": live / el, "unit": "spin-flip attempts/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} instances spread over the batch (one per thread) x {sweeps} sweeps, "
                      f"{el:.1f} s wall"}


def search_cpu_baseline(cfg, seeds, budget_s, sweeps_per_step, what="plain search step"):
    """The CPU oracle's hardness_eval, as it stands, on the host's cores: one
    seed instance per thread, two restarts each with the sweep cap lowered so
    the sample fits the budget (the cost per sweep does not depend on the
    cap), scaled to the seconds one step's PT sweeps take."""
    import oracle
    cores = min(host_cores(), len(seeds))
    t0 = time.perf_counter()
    r = oracle.hardness_eval(cfg.L, None, seeds[0], 0, cfg.seed, 1, cfg.K, cfg.R, cfg.beta, cfg.swap_interval, 20)
    per_sweep = (time.perf_counter() - t0) / max(1, int(r["r_sweeps"].sum()))
    s_cap = int(max(50, min(cfg.s_max, budget_s / per_sweep / 2)))
    sweeps = [0] * cores

    def work(i):
        out = oracle.hardness_eval(cfg.L, None, seeds[i], i, cfg.seed, 2, cfg.K, cfg.R, cfg.beta,
                                   cfg.swap_interval, s_cap)
        sweeps[i] = int(out["r_sweeps"].sum())

    threads = [threading.Thread(target=work, args=(i,)) for i in range(cores)]
    t0 = time.perf_counter()
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    el = time.perf_counter() - t0
    rate = sum(sweeps) / el
    return {"value": sweeps_per_step / rate, "unit": f"s per {what} (PT sweeps only)", "cores": cores,
            "kind": "oracle", "sweeps_per_s": rate,
            "sample": f"hardness_eval of {cores} seed instances (one per thread), 2 restarts each, "
                      f"sweep cap {s_cap}: {sum(sweeps)} sweeps in {el:.1f} s wall; scaled to "
                      f"{sweeps_per_step:.3g} sweeps per {what}"}


def _products(T, M):
    """Products g(t) g(t + d) of the autocorrelation sums over lags 0..M of a
    run of T passes, per configuration."""
    M = min(M, T - 1)
    return (M + 1) * T - M * (M + 1) // 2


def walk_cpu_baseline(insts, seed, K, R, beta, si, T, max_lag, budget_s):
    """The CPU oracle's recorded temperature walk and autocorrelation sums,
    as they stand, on the host's cores: one instance per thread for a prefix
    of the run (its cost per EMCS is constant), then the sums of one prefix
    scaled by the count of products to the full run and window.  Returns the
    seconds per EMCS and per instance's sums on one core, and the sample."""
    import oracle.walk as W
    cores = min(host_cores(), len(insts))
    d = insts[0]
    t0 = time.perf_counter()
    W.walk(d["L"], None, d["J"], K, R, beta, 0, seed, si, 2)
    per_emcs = (time.perf_counter() - t0) / 2
    n_s = int(max(8, 0.8 * budget_s / per_emcs))
    trajs = [None] * cores

    def work(i):
        trajs[i], _ = W.walk(insts[i]["L"], None, insts[i]["J"], K, R, beta, i, seed, si, n_s)

    threads = [threading.Thread(target=work, args=(i,)) for i in range(cores)]
    t0 = time.perf_counter()
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    el_walk = time.perf_counter() - t0
    # the sums' cost does not depend on the values: time the first lags of
    # a full-length run of random indices, scale by the product count
    traj = np.random.default_rng(7).integers(0, K, (T, K * R)).astype(np.uint8)
    t0 = time.perf_counter()
    W.acf_sums(traj, K, 9)
    m_s = int(min(max_lag, max(9, 10 * 0.15 * budget_s / max(1e-6, time.perf_counter() - t0) - 1)))
    t0 = time.perf_counter()
    W.acf_sums(traj, K, m_s)
    el_acf = time.perf_counter() - t0
    acf_full = el_acf * _products(T, max_lag) / _products(T, m_s)
    sample = (f"walk of {cores} C8 instances (one per thread) x {n_s} EMCS in {el_walk:.1f} s wall, scaled to "
              f"{T} EMCS; sums over the first {m_s + 1} lags of a {T}-pass run in {el_acf:.2f} s, scaled by the "
              f"product count to {max_lag + 1} lags ({acf_full:.1f} s)")
    return {"per_emcs": el_walk / n_s, "acf": acf_full, "cores": cores, "sample": sample}


def uneven(args):
    """1024 instances of mixed size (C4..C12, 2% missing spins, K 24..48):
    the workgroup shape chosen by the autotuner, each step one replay of a
    HIP graph holding the persistent launch.  Counts live attempts only
    (live sites x K R lanes)."""
    import torch

    import paper_1605_03607_amd as hs
    cfg = workloads.uneven_batch()
    if args.swap_interval is not None:
        cfg["swap_interval"] = args.swap_interval
    insts = cfg["instances"]
    sweeps = args.sweeps or cfg["sweeps"]
    live_per_sweep = sum(int(d["K"]) * int(d["R"]) * int(np.count_nonzero(d["live"])) for d in insts)
    # the tuner times the workgroup shapes of the plain plan (one instance per
    # workgroup) and of the packed plan (instances of one size sharing lanes),
    # cached by the batch's size classes
    from paper_1605_03607_amd import tuning
    t0 = time.perf_counter()
    if args.block_waves or args.pack != "auto":
        bw = args.block_waves or 16
        flags = hs.HS_PACK_LANES if args.pack == "on" else 0
        plan = {"tried": [], "cached": False, "us_per_sweep": None}
    else:
        bw, flags, plan = tuning.tuned_plan(insts, cfg["seed"], cfg["swap_interval"], cache_path=args.tune_cache)
    us = plan.get("us_per_sweep")
    tried = [(t["us_per_sweep"], t["block_waves"], hs.HS_PACK_LANES if t["packed"] else 0)
             for t in plan.get("tried", [])]
    tune_s = time.perf_counter() - t0
    print(f"# autotune: {plan} -> block_waves={bw}, flags={flags} ({tune_s:.1f} s)", file=sys.stderr, flush=True)
    batch = hs.PTBatch(insts, cfg["seed"], swap_interval=cfg["swap_interval"], block_waves=bw, flags=flags)
    _, _, _, items, lane_slots = batch.launch_shape()
    graph = batch.graph(sweeps)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        graph.launch()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s in range(args.steps):
        ev[s][0].record(stream)
        graph.launch()
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in ev]
    mism = batch.measure()
    attempts = live_per_sweep * sweeps
    k_avg_s = float(np.mean(kernel_ms)) / 1e3
    out = {
        "metric": "live spin-flip attempts/s (uneven batch)",
        "value": attempts * args.steps / wall,
        "unit": "spin-flip attempts/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": cfg["name"], "instances": len(insts), "sweeps_per_step": sweeps,
                   "swap_interval": cfg["swap_interval"], "block_waves": bw,
                   "packed_lanes": bool(flags & hs.HS_PACK_LANES), "work_items": items,
                   "autotune_us_per_sweep": us, "autotune_cached": plan.get("cached"),
                   "autotune_tried": [{"us_per_sweep": t[0], "block_waves": t[1],
                                       "packed_lanes": bool(t[2] & hs.HS_PACK_LANES)} for t in tried],
                   "live_attempts_per_sweep": live_per_sweep,
                   "live_fraction_of_lane_slots": live_per_sweep / lane_slots},
        "roofline": dict(alu_roofline(attempts, k_avg_s), traffic=None, kernel_ms_avg=float(np.mean(kernel_ms))),
        "energy_mismatches": mism,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = mixed_cpu_baseline(insts, cfg["seed"], cfg["swap_interval"], args.cpu_seconds)
    graph.close()
    batch.close()
    emit(out)


def _write_decisions(args, arm, run, mode="a"):
    """One JSON line per acceptance decision of a search arm."""
    if not args.search_log:
        return
    with open(args.search_log, mode) as f:
        for step, chain, ln_cur, ln_new, w, ok in run.decisions:
            f.write(json.dumps({"arm": arm, "step": step, "chain": chain, "ln_tts_current": ln_cur,
                                "ln_tts_candidate": ln_new, "w": w, "accepted": ok}) + "\n")


def _search_progress(name, args):
    def report(group, step):
        print(f"# {name}: group {group + 1}/{args.search_groups} step {step}/{args.search_steps}",
              file=sys.stderr, flush=True)
    return report


# The time-to-solution every search line reports, next to its numbers.
TTS_READING = ("ln TTS = ln(sweeps of all restarts / restarts whose minimum is the ground-state energy), the run time "
               "per find of the ground state after Appendix B, in sweeps; not the median over restarts that the "
               "workload description names")


def _search_block_waves(args, mode):
    if args.search_block_waves == "auto":
        return 16 if mode == "plain" or args.search_top < 2 else 8
    return int(args.search_block_waves)


def _run_validated(args, S, run, seeds, bars, name):
    """The timed steps of a search and the validation of its counted states:
    during the search (a Validator on the stream after the groups' ones) or
    after it.  Returns (search wall s, validation dict); the validated rate's
    hour is the wall plus val["seconds"] (the wait for the last validation
    launches, or the whole validation when it runs after the search)."""
    t0 = time.perf_counter()
    v = None
    if args.validate == "during":
        v = S.Validator(run.cfg, seeds, stream_index=args.search_groups)
        run.attach(v)
    run.run(args.search_steps, bars=bars, progress=_search_progress(name, args))
    wall = time.perf_counter() - t0
    print(f"# {name}: validating {len(run.hard_J)} counted states ({args.validate} the search)",
          file=sys.stderr, flush=True)
    val = v.finish(bars) if v is not None else S.validate(run, seeds, bars)
    return wall, val


def _validation_record(val, rule):
    return {"h0_fresh_ln_tts": val["h0"], "states": val["states"], "restarts": val["restarts"],
            "seconds": val["seconds"], "pt_sweeps": val["sweeps"], "pt_attempts": int(val["attempts"]),
            "pt_device_ms": val["device_ms"], "overlapped_with_search": val["overlapped"], "rule": rule}


def _chip_share(attempts, seconds):
    """Spin-flip attempts x the reference op count over `seconds`, as a
    fraction of the ALU peak."""
    return attempts * A_OPS / seconds / PEAK_INT32_OPS if seconds > 0 else None


def search(args):
    """Hard instances per hour of the instance search (Algorithm 1) on C8:
    plain chains, surrogate-screened chains and the random-screen ablation,
    each for a bounded number of steps from the same seed instances."""
    import math

    import paper_1605_03607_amd as hs
    from paper_1605_03607_amd import search as S
    seeds = workloads.search_seeds(args.search_chains)
    bars = {"ln3": math.log(3.0), "ln10": math.log(10.0), "ln30": math.log(30.0)}
    arms = {}
    for mode in ("plain", "surrogate", "random"):
        S.set_gnn_cus(args.gnn_cus if mode == "surrogate" else 0)
        cfg = S.SearchConfig(mode=mode, chains=args.search_chains, top=args.search_top,
                             block_waves=_search_block_waves(args, mode))
        params = workloads.gnn_params(hs.lib().gnn_param_count(), hs.gnn_fan_ins())
        t0 = time.perf_counter()
        run = S.GroupedSearch(cfg, seeds, groups=args.search_groups,
                              surrogate_params=params if mode == "surrogate" else None)
        t_init = time.perf_counter() - t0
        wall, val = _run_validated(args, S, run, seeds, tuple(bars.values()), mode)
        hours = wall / 3600.0
        hard = {name: len(run.hard.get(b, set())) for name, b in bars.items()}
        _write_decisions(args, mode, run, "w" if mode == "plain" else "a")
        v_wall = wall + val["seconds"]
        v_hours = v_wall / 3600.0
        finite = np.isfinite(run.ln)
        arms[mode] = {
            "steps": args.search_steps, "seconds": wall, "s_per_step": wall / args.search_steps,
            "init_seconds": t_init, "pt_seconds": run.pt_seconds, "gnn_seconds": run.gnn_seconds,
            "pt_sweeps": int(run.pt_sweeps), "accepted": run.accepted, "h0_ln_tts": run.h0,
            "pt_device_ms": run.pt_device_ms, "pt_attempts": int(run.pt_attempts), "pt_calls": run.pt_calls,
            "pt_block_waves": cfg.block_waves,
            "validated_hard_instances": {name: val["counts"][b] for name, b in bars.items()},
            "validated_hard_instances_per_hour": {name: val["counts"][b] / v_hours for name, b in bars.items()},
            "validation": _validation_record(
                val, "a counted state is re-scored with 64 restarts on streams disjoint from the search's and "
                     "kept if its fresh ln TTS >= H0' + bar (H0' = median fresh ln TTS of the seeds) and its "
                     "ground state is confirmed; the hour includes this re-scoring"),
            "chip_share_search": _chip_share(run.pt_attempts, wall),
            "chip_share_with_validation": _chip_share(run.pt_attempts + val["attempts"], v_wall),
            "hard_instances": hard,
            "hard_instances_per_hour": {k: v / hours for k, v in hard.items()},
            "final_median_ln_tts_finite": float(np.median(run.ln[finite])) if finite.any() else None,
            "final_censored_chains": int((~finite).sum()),
        }
    rate = lambda m: arms[m]["validated_hard_instances_per_hour"]["ln10"]
    raw = lambda m: arms[m]["hard_instances_per_hour"]["ln10"]
    out = {
        "metric": "hard instances/hour, surrogate vs plain",
        "value": rate("surrogate"),
        "unit": "validated hard instances/hour (fresh ln TTS >= H0' + ln 10)",
        "tts_reading": TTS_READING,
        "n_gpus": 1, "steps": args.search_steps, "warmup": 0,
        "ms_per_step": arms["surrogate"]["s_per_step"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32 (PT) / bf16-fp32 (surrogate)", "data": "synthetic",
        "config": {"workload": f"instance search, {args.search_chains} C8 chains, +-1 seeds, "
                               "mutations in +-1..+-7, 32 restarts K32 R2, T_s 0.5",
                   "bounded_steps": args.search_steps, "chain_groups": args.search_groups,
                   "screen": f"16 proposals, top {args.search_top} scored by PT",
                   "validation": args.validate, "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"),
                   "surrogate_cus": args.gnn_cus, "pt_block_waves": args.search_block_waves},
        "chip_share_note": "chip shares are spin-flip attempts x 22 ops over the wall, as a fraction of the "
                           "ALU peak; the sweep kernel's own full-batch fraction (C8 benchmark) bounds them",
        "surrogate_over_plain": (rate("surrogate") / rate("plain")) if rate("plain") > 0 else None,
        "surrogate_over_plain_unvalidated": (raw("surrogate") / raw("plain")) if raw("plain") > 0 else None,
        "random_over_plain": (rate("random") / rate("plain")) if rate("plain") > 0 else None,
        "surrogate_over_plain_by_bar": {
            b: (arms["surrogate"]["validated_hard_instances_per_hour"][b] /
                arms["plain"]["validated_hard_instances_per_hour"][b])
            if arms["plain"]["validated_hard_instances_per_hour"][b] > 0 else None for b in bars},
        "arms": arms,
        "roofline": pt_roofline(sum(a["pt_attempts"] for a in arms.values()),
                                sum(a["pt_device_ms"] for a in arms.values()),
                                sum(a["pt_calls"] for a in arms.values()),
                                "k_pt_sweep<false> in hardness_eval (stop on agreement), all launches of the "
                                "three arms; concurrent groups share the chip",
                                sum(a["seconds"] for a in arms.values())),
    }
    if not args.no_cpu_baseline:
        plain = S.SearchConfig(mode="plain", chains=args.search_chains)
        out["cpu_baseline"] = search_cpu_baseline(plain, seeds, args.cpu_seconds,
                                                  arms["plain"]["pt_sweeps"] / args.search_steps)
    emit(out)


def search_reverse(args):
    """The reversed search (Sec. II.B): plain chains that favour shorter TTS,
    from the same +-1 seeds with sign-flip mutations (Algorithm 1's move);
    easy instances per hour and the drop of the median ln TTS (the paper
    lowers TTS about tenfold below random instances)."""
    import math

    from paper_1605_03607_amd import search as S
    seeds = workloads.search_seeds(args.search_chains)
    bars = {"ln3": math.log(3.0), "ln10": math.log(10.0)}
    cfg = S.SearchConfig(mode="plain", chains=args.search_chains, direction=-1, alphabet=S.ALPHABET_PM1)
    run = S.GroupedSearch(cfg, seeds, groups=args.search_groups)
    h0 = run.h0
    wall, val = _run_validated(args, S, run, seeds, tuple(bars.values()), "reverse")
    easy = {name: len(run.hard.get(b, set())) for name, b in bars.items()}
    _write_decisions(args, "reverse", run, "w")
    v_easy = {name: val["counts"][b] for name, b in bars.items()}
    med = float(np.median(run.ln))
    out = {
        "metric": "easy instances/hour (reversed search)",
        "value": v_easy["ln3"] / ((wall + val["seconds"]) / 3600.0),
        "unit": "validated easy instances/hour (fresh ln TTS <= H0' - ln 3)",
        "tts_reading": TTS_READING,
        "unvalidated_easy_instances_per_hour": easy["ln3"] / (wall / 3600.0),
        "validated_easy_instances": v_easy,
        "validation": _validation_record(
            val, "a counted state is re-scored with 64 restarts on streams disjoint from the search's and kept "
                 "if its fresh ln TTS <= H0' - bar (H0' = median fresh ln TTS of the seeds) and its ground state "
                 "is confirmed; the hour includes this re-scoring"),
        "chip_share_search": _chip_share(run.pt_attempts, wall),
        "chip_share_with_validation": _chip_share(run.pt_attempts + val["attempts"], wall + val["seconds"]),
        "n_gpus": 1, "steps": args.search_steps, "warmup": 0,
        "ms_per_step": wall * 1e3 / args.search_steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32 (PT)", "data": "synthetic",
        "config": {"workload": f"reversed instance search, {args.search_chains} C8 chains, +-1 seeds, "
                               "sign-flip mutations (J stays +-1), 32 restarts K32 R2, T_s 0.5",
                   "bounded_steps": args.search_steps, "chain_groups": args.search_groups,
                   "validation": args.validate, "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES")},
        "easy_instances": easy, "h0_ln_tts": h0, "final_median_ln_tts": med,
        "median_drop_ln": h0 - med, "accepted": run.accepted, "pt_sweeps": int(run.pt_sweeps),
        "roofline": pt_roofline(run.pt_attempts, run.pt_device_ms, run.pt_calls,
                                "k_pt_sweep<false> in hardness_eval (stop on agreement), all launches; "
                                "concurrent groups share the chip", wall),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = search_cpu_baseline(cfg, seeds, args.cpu_seconds,
                                                  run.pt_sweeps / args.search_steps, "reversed search step")
    emit(out)


def tau(args):
    """Mixing time of the temperature random walk (Sec. III.B) for 256 C8
    instances with +-1 couplings: K = 32 temperatures (beta 0.1..5.0) x R = 2
    chains, EMCS = 10 sweeps + one exchange pass, a bounded run of
    --tau-emcs EMCS recorded on the device, then exact autocorrelation sums,
    the automatic-window tau and the paper's two acceptance criteria."""
    import torch

    import paper_1605_03607_amd as hs
    n_inst, K, R, si = 256, 32, 2, 10
    T = args.tau_emcs
    max_lag = min(65535, max(1, T // 4))
    beta = workloads.geometric_betas(0.1, 5.0, K)
    insts = [dict(L=8, J=workloads.couplings(8, "pm1", 2024, n), live=None, K=K, R=R, beta=beta,
                  instance_id=n) for n in range(n_inst)]
    b = hs.PTBatch(insts, 2024, swap_interval=si)
    walk = torch.zeros((n_inst, T, 64), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    b.sweep_record(T * si, walk)
    e1.record(stream)
    acf, hot = hs.walk_autocorr(walk, T, K, R, max_lag)
    e2.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_pt, ms_acf = e0.elapsed_time(e1), e1.elapsed_time(e2)
    acf_products = n_inst * K * R * _products(T, max_lag)
    taus, ok_i, ok_ii, conv = [], 0, 0, 0
    for n in range(n_inst):
        t_emcs, win, c = hs.walk_tau(acf[n], T)
        share = float(hot[n, :K * R].min()) / T
        taus.append(t_emcs * si)
        ok_i += share >= 0.2
        ok_ii += T >= 20 * t_emcs
        conv += c
    attempts = n_inst * K * R * 512 * T * si
    out = {
        "metric": "mixing time of the temperature walk (instances per hour)",
        "value": n_inst / (wall / 3600.0),
        "unit": "instances with tau estimated per hour (bounded run)",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": wall * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32 (PT) / int64 (sums)", "data": "synthetic",
        "config": {"workload": f"tau, {n_inst} C8 instances J=+-1, K{K} R{R} beta 0.1..5.0, EMCS = {si} sweeps + "
                               f"1 exchange, {T} EMCS", "max_lag_emcs": max_lag},
        "pt_attempts_per_s": attempts / (ms_pt / 1e3), "pt_ms": ms_pt, "acf_ms": ms_acf,
        "roofline": pt_roofline(attempts, ms_pt, 1, "k_pt_sweep<true> (walk recording), one launch"),
        "acf": {"kernel": "k_walk_acf", "products": acf_products,
                "int32_lane_ops_per_s": 2 * acf_products / (ms_acf / 1e3),
                "frac_of_alu_peak": 2 * acf_products / (ms_acf / 1e3) / PEAK_INT32_OPS},
        "tau_sweeps": {"median": float(np.median(taus)), "p90": float(np.percentile(taus, 90)),
                       "max": float(np.max(taus))},
        "window_converged": int(conv), "criterion_hot_half": int(ok_i), "criterion_20_tau": int(ok_ii),
        "energy_mismatches": b.measure(),
    }
    b.close()
    if not args.no_cpu_baseline:
        c = walk_cpu_baseline(insts, 2024, K, R, beta, si, T, max_lag, args.cpu_seconds)
        per_inst = c["per_emcs"] * T + c["acf"]
        out["cpu_baseline"] = {"value": c["cores"] * 3600.0 / per_inst, "unit": out["unit"], "cores": c["cores"],
                               "kind": "oracle", "sample": c["sample"]}
    emit(out)


def lao(args):
    """Loop Adaptive Optimization (Sec. IV, Algorithm 2) on planted-solution
    C8 instances: 64 chains of 350 frustrated loops (weights 1..5, 4-cycles
    with probability 0.1), one loop replaced per step, scored by PT; the
    ratio of final TTS to the mean initial TTS (the paper's Fig. 6 measure)
    and how often PT reached the planted ground state."""
    from paper_1605_03607_amd import search as S
    cfg = S.SearchConfig(mode="plain", chains=args.search_chains)
    t0 = time.perf_counter()
    run = S.GroupedLao(cfg, n_loops=350, groups=args.search_groups)
    t_init = time.perf_counter() - t0
    sweeps0 = run.pt_sweeps
    t0 = time.perf_counter()
    run.run(args.search_steps, progress=_search_progress("lao", args))
    wall = time.perf_counter() - t0
    tts0, tts = np.exp(run.ln0), np.exp(run.ln)
    _write_decisions(args, "lao", run, "w")
    ratio = tts / float(np.mean(tts0))
    out = {
        "metric": "LAO: final TTS / mean initial TTS (planted C8)",
        "value": float(np.mean(ratio)),
        "unit": "ratio (mean over chains)",
        "n_gpus": 1, "steps": args.search_steps, "warmup": 0,
        "ms_per_step": wall * 1e3 / args.search_steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32 (PT)", "data": "synthetic",
        "config": {"workload": f"LAO, {args.search_chains} planted C8 chains, 350 loops (weights 1..5, "
                               "P(4-cycle) 0.1), 32 restarts K32 R2, T_s 0.5",
                   "bounded_steps": args.search_steps, "chain_groups": args.search_groups,
                   "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES")},
        "ratio_median": float(np.median(ratio)), "ratio_max": float(np.max(ratio)),
        "initial_mean_ln_tts": float(np.mean(run.ln0)), "final_mean_ln_tts": float(np.mean(run.ln)),
        "accepted": run.accepted, "scored": run.scored, "pt_ground_state_equals_planted": run.gs_found,
        "init_seconds": t_init, "pt_seconds": run.pt_seconds, "pt_sweeps": int(run.pt_sweeps),
        "roofline": pt_roofline(run.pt_attempts, run.pt_device_ms, run.pt_calls,
                                "k_pt_sweep<false> in hardness_eval (stop on agreement), all launches",
                                t_init + wall),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = search_cpu_baseline(cfg, [i["J"] for i in run.inst], args.cpu_seconds,
                                                  (run.pt_sweeps - sweeps0) / args.search_steps, "LAO step")
    emit(out)


def overlap(args):
    """Fig. 3's two hardness measures on the same runs: 256 C8 instances
    (J = +-1, K32 R2, EMCS = 10 sweeps + one exchange pass) run --tau-emcs
    EMCS with the temperature walk recorded (tau), then 300 more EMCS with
    a snapshot after each, capturing every lane within 4 of the instance's
    lowest energy so far; per instance the ground / first-excited median
    overlap ratio, and the rank correlation of ratio and tau over the
    instances whose tau window converged."""
    import torch

    import paper_1605_03607_amd as hs
    n_inst, K, R, si, L = 256, 32, 2, 10, 8
    T = args.tau_emcs
    max_lag = min(65535, max(1, T // 4))
    beta = workloads.geometric_betas(0.1, 5.0, K)
    insts = [dict(L=L, J=workloads.couplings(L, "pm1", 3033, n), live=None, K=K, R=R, beta=beta, instance_id=n)
             for n in range(n_inst)]
    b = hs.PTBatch(insts, 3033, swap_interval=si)
    walk = torch.zeros((n_inst, T, 64), dtype=torch.uint8, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    b.sweep_record(T * si, walk)
    e1.record()
    acf, hot = hs.walk_autocorr(walk, T, K, R, max_lag)
    del walk
    taus = [hs.walk_tau(acf[n], T) for n in range(n_inst)]
    e_min = [int(b.state(n)["emin"].min()) for n in range(n_inst)]
    n_words, capacity, n_snap = (8 * L * L + 63) // 64, 1 << 22, 300
    configs = torch.zeros((capacity, n_words), dtype=torch.int64, device="cuda")
    meta = torch.zeros((capacity, 4), dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    caps = [e + 4 for e in e_min]
    for _ in range(n_snap):
        b.sweep(si)
        b.capture(caps, configs, meta, count)
    torch.cuda.synchronize()
    t_pt = time.perf_counter() - t0
    n_cap = min(int(count.item()), capacity)
    cfg_h = configs[:n_cap].cpu().numpy().view(np.uint64)
    meta_h = meta[:n_cap].cpu().numpy()
    mask = np.full(n_words, np.uint64(0xFFFFFFFFFFFFFFFF), np.uint64)
    t1 = time.perf_counter()
    ratios, analysed = [], []
    by_inst = np.argsort(meta_h[:, 0], kind="stable")  # capture order within each instance
    bounds = np.searchsorted(meta_h[by_inst, 0], np.arange(n_inst + 1))
    for n in range(n_inst):
        rows = by_inst[bounds[n]:bounds[n + 1]]
        if len(rows) == 0:
            ratios.append(None)
            continue
        # repeated snapshots of one configuration change nothing in the analysis
        key = np.concatenate([meta_h[rows, 2:3].astype(np.uint64), cfg_h[rows]], axis=1)
        _, first = np.unique(key, axis=0, return_index=True)
        sel = rows[np.sort(first)][:2000]
        analysed.append(len(sel))
        s = hs.overlap_analyze(cfg_h[sel], meta_h[sel, 2], mask, 8 * L * L)
        ratios.append(s["ratio"])
    t_ov = time.perf_counter() - t1
    pairs = [(taus[n][0] * si, ratios[n]) for n in range(n_inst) if taus[n][2] and ratios[n] is not None]
    rho = None
    if len(pairs) >= 3:
        a = np.argsort(np.argsort([p[0] for p in pairs])).astype(float)
        c = np.argsort(np.argsort([p[1] for p in pairs])).astype(float)
        rho = float(np.corrcoef(a, c)[0, 1])
    valid = [r for r in ratios if r is not None]
    out = {
        "metric": "ground / first-excited overlap ratio and mixing time (Fig. 3)",
        "value": float(np.median(valid)) if valid else None,
        "unit": "median over instances of (median GS-ES overlap / median GS-GS overlap)",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": (t_pt + t_ov) * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32 (PT) / int64 (sums)", "data": "synthetic",
        "config": {"workload": f"overlap + tau, {n_inst} C8 instances J=+-1, K{K} R{R}, EMCS = {si} sweeps + 1 exchange, "
                               f"{T} EMCS walk then {n_snap} snapshot EMCS, cap E_min + 4"},
        "captured": int(count.item()), "stored": n_cap, "instances_with_excited_level": len(valid),
        "tau_converged": int(sum(t[2] for t in taus)),
        "spearman_tau_vs_ratio": rho, "pairs": len(pairs),
        "pt_seconds": t_pt, "overlap_seconds": t_ov,
        "roofline": pt_roofline(n_inst * K * R * 8 * L * L * T * si, e0.elapsed_time(e1), 1,
                                "k_pt_sweep<true> (walk recording), the walk launch"),
    }
    b.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = overlap_cpu_baseline(insts, K, R, beta, si, T, max_lag, n_snap,
                                                   float(np.mean(analysed)) if analysed else 0.0, args.cpu_seconds)
    emit(out)


def overlap_cpu_baseline(insts, K, R, beta, si, T, max_lag, n_snap, n_analysed, budget_s):
    """The CPU oracle on the overlap workload, as it stands: the walk and its
    sums (walk_cpu_baseline) plus the snapshot EMCS at the walk's cost per
    EMCS, and the oracle's overlap summary timed on 120 synthetic
    configurations of two levels and scaled by the pair count to the mean
    number analysed per instance here (the snapshot capture itself is not
    counted); seconds for all instances over the host's cores."""
    import oracle.overlap as O
    c = walk_cpu_baseline(insts, 3033, K, R, beta, si, T, max_lag, 0.7 * budget_s)
    N = 8 * insts[0]["L"] ** 2
    g = np.random.default_rng(5)
    n_s = 120
    cfgs = [(int(-700 + 4 * (i % 2)), g.integers(0, 2, N, dtype=np.uint8)) for i in range(n_s)]
    t0 = time.perf_counter()
    O.summary(cfgs)
    el = time.perf_counter() - t0
    summ = el * (n_analysed / n_s) ** 2
    per_inst = c["per_emcs"] * (T + n_snap) + c["acf"] + summ
    return {"value": len(insts) * per_inst / c["cores"], "unit": "s per workload", "cores": c["cores"],
            "kind": "oracle",
            "sample": c["sample"] + f"; summary of {n_s} configurations in {el:.2f} s, scaled to "
                                    f"{n_analysed:.0f} per instance ({summ:.1f} s)"}


def surrogate(args):
    """Surrogate step times on C8 graphs: a training step (forward, backward,
    Adam) on the 16-graph batch and the forward pass that screens 1024
    proposals (64 chains x 16), with the MFMA-priced FLOP rate."""
    import torch

    import paper_1605_03607_amd as hs
    n_par = hs.lib().gnn_param_count()
    sur = hs.Surrogate(workloads.gnn_params(n_par, hs.gnn_fan_ins()))
    L = 8
    E = 24 * L * L - 8 * L
    N = 8 * L * L

    def flops(G):  # matrix products of one forward pass
        ne, nn = 2 * E * G, N * G
        return 3 * 2 * 64 * (ne * 192 + nn * 128)

    out = {}
    for G, what in ((16, "train"), (1024, "forward")):
        gr = [(L, None, workloads.couplings(L, "pm7", 99, g)) for g in range(G)]
        sur.prepare(gr)
        labels = np.linspace(5.0, 12.0, G)
        reps = 20 if what == "train" else 5
        for _ in range(2):
            sur.train_step(labels, update=False) if what == "train" else sur.forward()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            if what == "train":
                sur.train_step(labels)
            else:
                sur.forward()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        f = flops(G) * (3 if what == "train" else 1)
        out[what] = {"graphs": G, "ms": dt * 1e3, "tflops": f / dt / 1e12}
    res = {"metric": "surrogate step time (C8 graphs)", "value": out["train"]["ms"], "unit": "ms per training step",
           "n_gpus": 1, "steps": 20, "warmup": 2, "higher_is_better": False, "dtype": "bf16 (fp32 accumulate)",
           "data": "synthetic", "config": {"workload": "surrogate, 16-graph training batch, 1024-graph screen"},
           "detail": out, "mfma_peak_tflops_bf16": 2500.0,
           "roofline": {"bound": "mfma", "achieved": out["train"]["tflops"], "peak": 2500.0, "unit": "TFLOP/s",
                        "frac": out["train"]["tflops"] / 2500.0, "traffic": None,
                        "kernel": "training step (all of its kernels: rows, gathers, weight gradients, Adam); "
                                  "matrix-product FLOPs over the step's time",
                        "kernel_ms_avg": out["train"]["ms"]}}
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = surrogate_cpu_baseline(n_par, L, args.cpu_seconds)
    emit(res)


def surrogate_cpu_baseline(n_par, L, budget_s):
    """The CPU oracle's surrogate (fp64 numpy, as it stands): training steps
    (loss, gradient, Adam) on the same 16-graph batch shape, for about the
    budget; ms per training step on one process."""
    import oracle.gnn as G

    import paper_1605_03607_amd as hs
    theta = workloads.gnn_params(n_par, hs.gnn_fan_ins()).astype(np.float64)
    B = G.batch([(L, None, workloads.couplings(L, "pm7", 99, g)) for g in range(16)])
    labels = np.linspace(5.0, 12.0, 16)
    m, v = np.zeros_like(theta), np.zeros_like(theta)
    steps, t0 = 0, time.perf_counter()
    while True:
        _, grad = G.loss_and_grad(theta, B, labels)[:2]
        theta, m, v = G.adam(theta, m, v, grad, steps + 1, 3e-3)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 200:
            break
    return {"value": el * 1e3 / steps, "unit": "ms per training step", "cores": 1, "kind": "oracle",
            "sample": f"{steps} training steps of 16 C8 graphs in {el:.1f} s (numpy fp64, one process)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.workload in ("search", "search-reverse", "lao"):
        if not 1 <= args.hw_queues <= 32:
            print(json.dumps({"error": "--hw-queues must be in 1..32"}))
            sys.exit(2)
        # read by the HIP runtime when it starts, which is after this point
        # (nothing has touched the GPU yet)
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    if args.workload == "uneven":
        uneven(args)
        return
    if args.workload == "overlap":
        overlap(args)
        return
    if args.workload == "lao":
        lao(args)
        return
    if args.workload == "tau":
        tau(args)
        return
    if args.workload == "search-reverse":
        search_reverse(args)
        return
    if args.workload == "search":
        search(args)
        return
    if args.workload == "surrogate":
        surrogate(args)
        return
    import torch

    import paper_1605_03607_amd as hs
    cfg = workloads.batch_c8()
    if args.lattice != 8:
        if not 1 <= args.lattice <= 16:
            print(json.dumps({"error": "--lattice must be in 1..16"}))
            sys.exit(2)
        cfg.update(L=args.lattice, name=f"C{args.lattice} x256, K32 R2, +-7")
    if args.instances != 256:
        if args.instances < 1:
            print(json.dumps({"error": "--instances must be positive"}))
            sys.exit(2)
        cfg.update(n_inst=args.instances, name=cfg["name"].replace("x256", f"x{args.instances}"))
    if args.swap_interval is not None:
        cfg["swap_interval"] = args.swap_interval
    sweeps = args.sweeps or cfg["sweeps"]
    insts = workloads.make_batch(cfg)
    n_inst = len(insts)
    lanes = cfg["K"] * cfg["R"]
    n_sites = 8 * cfg["L"] ** 2
    attempts_per_step = n_inst * lanes * n_sites * sweeps

    batch = hs.PTBatch(insts, cfg["seed"], swap_interval=cfg["swap_interval"],
                       block_waves=args.block_waves)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        batch.sweep(sweeps)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s in range(args.steps):
        ev[s][0].record(stream)
        batch.sweep(sweeps)
        ev[s][1].record(stream)
        print(f"# step {s + 1}/{args.steps} enqueued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in ev]
    mism = batch.measure()
    if args.copy_mib:
        src = torch.ones(args.copy_mib * (1 << 20) // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ms_per_step = wall * 1e3 / args.steps
    value = attempts_per_step * args.steps / wall
    k_avg_s = float(np.mean(kernel_ms)) / 1e3
    roof = alu_roofline(attempts_per_step, k_avg_s)
    roof.update({"traffic": measured_traffic() if (cfg["L"], n_inst) == (8, 256) else None,
                 "kernel_ms_avg": float(np.mean(kernel_ms)),
                 "kernel": "hs::dev::k_pt_sweep", "kernel_fingerprint": kernel_fingerprint(),
                 "issue_rates_measured_lane_ops_per_s": measured_issue_rates()})
    out = {
        "metric": f"spin-flip attempts/s (C{cfg['L']} PT batch)",
        "value": value,
        "unit": "spin-flip attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "instances": n_inst, "L": cfg["L"], "N": n_sites,
                   "couplers": 24 * cfg["L"] ** 2 - 8 * cfg["L"], "K": cfg["K"], "R": cfg["R"],
                   "sweeps_per_step": sweeps,
                   "swap_interval": cfg["swap_interval"], "alphabet": "+-1..+-7"},
        "roofline": roof,
        "energy_mismatches": mism,
    }
    if args.probe:
        out["isa_probe_lane_ops_per_s"] = hs.probe_rates()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, insts, args.cpu_seconds)
    batch.close()
    emit(out)


if __name__ == "__main__":
    main()
