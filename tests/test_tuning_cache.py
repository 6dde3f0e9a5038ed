"""The launch-plan tuner's JSON cache, on the host with a stand-in for the
library's timing: the plain and the packed plan are both timed, the faster
is kept, and a batch with the same size classes (lattice side, lanes) is
answered from the cache without timing; another make-up is timed again."""
import numpy as np

import workloads


def _batch(n, K, L=3):
    return [dict(L=L, J=workloads.couplings(L, "pm1", 5, i), live=None, K=K, R=1,
                 beta=workloads.geometric_betas(0.1, 3.0, K), instance_id=i) for i in range(n)]


def test_plan_cache(tmp_path):
    import paper_1605_03607_amd as hs
    from paper_1605_03607_amd import tuning
    calls = []

    def fake(insts, seed, swap_interval=1, flags=0, trial_sweeps=200):
        calls.append(flags)
        return (8, 5.0) if flags & hs.HS_PACK_LANES else (16, 7.0)

    path = str(tmp_path / "plans.json")
    bw, flags, rec = tuning.tuned_plan(_batch(6, 24), 1, 1, cache_path=path, tuner=fake, device_name="dev")
    assert (bw, flags, rec["cached"]) == (8, hs.HS_PACK_LANES, False) and len(calls) == 2
    assert {t["packed"] for t in rec["tried"]} == {True, False}
    # same size classes, other couplings: from the cache
    other = _batch(6, 24)
    for d in other:
        d["J"] = -d["J"]
    bw2, flags2, rec2 = tuning.tuned_plan(other, 1, 1, cache_path=path, tuner=fake, device_name="dev")
    assert (bw2, flags2, rec2["cached"]) == (8, hs.HS_PACK_LANES, True) and len(calls) == 2
    # another make-up, another interval or device: timed again
    tuning.tuned_plan(_batch(6, 32), 1, 1, cache_path=path, tuner=fake, device_name="dev")
    tuning.tuned_plan(_batch(6, 24), 1, 10, cache_path=path, tuner=fake, device_name="dev")
    tuning.tuned_plan(_batch(6, 24), 1, 1, cache_path=path, tuner=fake, device_name="other")
    assert len(calls) == 8
    # stop-on-agreement batches cannot pack: only the plain plan is timed
    bw3, flags3, rec3 = tuning.tuned_plan(_batch(2, 8), 1, 1, tuner=fake, flags=hs.HS_STOP_ON_AGREEMENT,
                                          device_name="dev")
    assert flags3 == hs.HS_STOP_ON_AGREEMENT and len(rec3["tried"]) == 1


def test_batch_key_is_the_size_class_histogram():
    from paper_1605_03607_amd import tuning
    a = _batch(3, 24) + _batch(2, 32, L=4)
    b = list(reversed(a))
    assert tuning.batch_key(a, 1, "d") == tuning.batch_key(b, 1, "d")
    assert tuning.batch_key(a, 1, "d") != tuning.batch_key(a[:-1], 1, "d")
    assert np.all([k in tuning.batch_key(a, 1, "d") for k in ("3x24:3", "4x32:2")])
