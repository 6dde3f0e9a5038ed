"""Writes tests/golden/metric_configs.json: CPU-oracle results at the sizes the
benchmarks run, too long for the oracle to recompute inside a GPU test.

  c8_long    four instances (0, 85, 170, 255) of the 256 x C8 batch (J uniform
             over +-1..+-7, K = 32 with beta geometric 0.1..5.0, R = 2, an
             exchange pass after every sweep) after 10^5 sweeps from the
             Philox initial state: the full PT state.
  hardness   three C8 candidates scored as the instance search scores them
             (32 restarts of K = 32 x R = 2, beta 0.1..5.0, exchange every
             sweep, stop on agreement or 10^5 sweeps, seed 1605): the first
             three +-1 seed instances (chain ids 0, 1 and 2).

Calls only oracle/ and the seeded input generators.  Run from the repository
root: python tests/golden/make_metric_configs.py  (about 10 minutes on 8 cores).
"""
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "metric_configs.json")
C8_PICK = (0, 85, 170, 255)
C8_SWEEPS = 100_000
HARD_SEED = 1605
HARD_RESTARTS = 32
HARD_K, HARD_R = 32, 2
HARD_SMAX = 100_000


def hardness_candidates():
    seeds = workloads.search_seeds(64)
    return [dict(name=f"seed{i}", J=seeds[i], instance_id=i) for i in range(3)]


def _c8(n, insts, seed):
    d = insts[n]
    st = oracle.pt_init(d["L"], None, d["J"], d["K"], d["R"], d["instance_id"], seed)
    oracle.pt_run(d["L"], None, d["J"], d["K"], d["R"], d["beta"], d["instance_id"], seed, 1, C8_SWEEPS, st)
    return dict(index=n, spins=[int(x) for x in st.spins], perm=st.perm.tolist(), energy=st.energy.tolist(),
                emin=st.emin.tolist(), thit=st.thit.tolist(), swap_acc=st.swap_acc.tolist(), t=int(st.t[0]))


def _hard(c, beta):
    r = oracle.hardness_eval(8, None, c["J"], c["instance_id"], HARD_SEED, HARD_RESTARTS, HARD_K, HARD_R, beta, 1,
                             HARD_SMAX)
    return dict(name=c["name"], instance_id=c["instance_id"], ln_tts=float(r["ln_tts"]), e_gs=int(r["e_gs"]),
                confirmed=int(r["confirmed"]), r_emin=r["r_emin"].tolist(), r_sweeps=r["r_sweeps"].tolist())


def main():
    cfg = workloads.batch_c8()
    insts = workloads.make_batch(cfg)
    beta = workloads.geometric_betas(0.1, 5.0, HARD_K)
    t0 = time.time()
    with ThreadPoolExecutor(8) as pool:
        hard = [pool.submit(_hard, c, beta) for c in hardness_candidates()]
        c8 = [pool.submit(_c8, n, insts, cfg["seed"]) for n in C8_PICK]
        out = dict(
            c8_long=dict(seed=cfg["seed"], sweeps=C8_SWEEPS, swap_interval=1, instances=[f.result() for f in c8]),
            hardness=dict(seed=HARD_SEED, restarts=HARD_RESTARTS, K=HARD_K, R=HARD_R, beta=[0.1, 5.0],
                          swap_interval=1, s_max=HARD_SMAX, candidates=[f.result() for f in hard]))
    with open(OUT + ".tmp", "w") as f:
        json.dump(out, f, separators=(",", ":"))
    os.replace(OUT + ".tmp", OUT)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
