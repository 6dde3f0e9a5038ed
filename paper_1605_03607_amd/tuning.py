"""Launch-plan tuning of PT batches with a JSON cache.

pt_autotune (libhardspin) times the workgroup shapes of one launch plan on
scratch buffers.  tuned_plan() asks it for the plain plan (one instance per
workgroup) and, where instances of one lattice size can share a workgroup's
64 lanes, for the packed plan (HS_PACK_LANES), and keeps the faster.  The
choice depends on the batch only through its size classes -- how many
instances of each (lattice side, lanes K R) it holds -- the exchange
interval and the device, so it is cached under that key in a JSON file and
reused by later batches of the same make-up.
"""
import json
import os
import threading

from . import HS_PACK_LANES, autotune

_LOCK = threading.Lock()


def batch_key(insts, swap_interval, device_name):
    """Cache key: size-class histogram (L, K R) -> count, exchange interval,
    device."""
    hist = {}
    for d in insts:
        c = (int(d["L"]), int(d["K"]) * int(d["R"]))
        hist[c] = hist.get(c, 0) + 1
    classes = ";".join(f"{L}x{lanes}:{n}" for (L, lanes), n in sorted(hist.items()))
    return f"{device_name}|si={int(swap_interval)}|{classes}"


def _device_name():
    import torch
    return torch.cuda.get_device_name(torch.cuda.current_device())


def tuned_plan(insts, seed, swap_interval=1, cache_path=None, trial_sweeps=200, flags=0, tuner=None,
               device_name=None):
    """(block_waves, flags, record) for the batch: flags carries HS_PACK_LANES
    when the packed plan timed faster.  record lists what was timed (or that
    the cache answered).  `tuner` stands in for the library's autotune (same
    signature); `flags` holds the caller's other flags (never
    HS_STOP_ON_AGREEMENT with packing: then only the plain plan is timed)."""
    tuner = tuner or autotune
    name = device_name or _device_name()
    key = batch_key(insts, swap_interval, name)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with _LOCK, open(cache_path) as f:
            try:
                cache = json.load(f)
            except ValueError:
                cache = {}
    if key in cache:
        hit = cache[key]
        return int(hit["block_waves"]), (flags & ~HS_PACK_LANES) | (HS_PACK_LANES if hit["packed"] else 0), \
            dict(hit, cached=True)
    plans = [flags & ~HS_PACK_LANES]
    if not flags & 2:  # HS_STOP_ON_AGREEMENT cannot pack
        plans.append(plans[0] | HS_PACK_LANES)
    tried = []
    for f in plans:
        bw, us = tuner(insts, seed, swap_interval=swap_interval, flags=f, trial_sweeps=trial_sweeps)
        tried.append(dict(us_per_sweep=float(us), block_waves=int(bw), packed=bool(f & HS_PACK_LANES)))
    best = min(tried, key=lambda t: t["us_per_sweep"])
    rec = dict(block_waves=best["block_waves"], packed=best["packed"], us_per_sweep=best["us_per_sweep"],
               tried=tried)
    if cache_path:
        with _LOCK:
            cache = {}
            if os.path.exists(cache_path):
                with open(cache_path) as f:
                    try:
                        cache = json.load(f)
                    except ValueError:
                        cache = {}
            cache[key] = rec
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1, sort_keys=True)
            os.replace(tmp, cache_path)
    return best["block_waves"], plans[0] | (HS_PACK_LANES if best["packed"] else 0), dict(rec, cached=False)
