"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

ctypes view of liboracle.so (oracle.c), the plain scalar reference for the
parallel-tempering hot path.  Only tests/, the smoke check and the
CPU-baseline leg of bench.py may import this package; the product path never
does.  See oracle.c for what each function follows in the paper.

An instance is (L, live, J): Chimera side L, live-site mask (uint8[N] or
None for all live) and couplings int8 over the full canonical edge list.
"""
import ctypes as C
import math
import os

import numpy as np

from . import build as _build

_lib = None

_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        L.or_philox.argtypes = [_u32p, _u32p, _u32p]
        L.or_philox.restype = None
        L.or_num_sites.argtypes = [C.c_int]
        L.or_edges.argtypes = [C.c_int, C.c_void_p, C.c_void_p]
        L.or_energy.argtypes = [C.c_int, C.c_void_p, _i8p, _u8p]
        L.or_energy.restype = C.c_int64
        L.or_metro_threshold.argtypes = [C.c_double, C.c_int]
        L.or_metro_threshold.restype = C.c_uint64
        L.or_swap_threshold.argtypes = [C.c_double, C.c_double, C.c_int64]
        L.or_swap_threshold.restype = C.c_uint64
        L.or_pt_init.argtypes = [C.c_int, C.c_void_p, _i8p, C.c_int, C.c_int, C.c_uint32,
                                 C.c_uint32, C.c_void_p, _u64p, _u8p, _i32p, _i32p, _i64p, _u32p]
        L.or_pt_run.argtypes = [C.c_int, C.c_void_p, _i8p, C.c_int, C.c_int, _f64p, C.c_uint32,
                                C.c_uint32, C.c_int, C.c_int64, C.c_int, C.c_void_p, _u64p, _u8p,
                                _i32p, _i32p, _i64p, _u32p, _i64p, _i32p]
        L.or_pt_swap_extra.argtypes = [C.c_int, C.c_void_p, _i8p, C.c_int, C.c_int, _f64p,
                                       C.c_uint32, C.c_uint32, _u64p, _u8p, _i32p, _u32p,
                                       C.c_int64]
        L.or_lane_energies.argtypes = [C.c_int, C.c_void_p, _i8p, C.c_int, _u64p, _i32p]
        L.or_hardness_eval.argtypes = [C.c_int, C.c_void_p, _i8p, C.c_uint32, C.c_uint32, C.c_int,
                                       C.c_int, C.c_int, _f64p, C.c_int, C.c_int64, _f64p, _i32p,
                                       _i32p, _i32p, _i64p, _i64p]
        L.or_mutate.argtypes = [C.c_int, C.c_void_p, _i8p, _i8p, C.c_int, C.c_uint32, C.c_uint32,
                                C.c_uint32, C.c_uint32, _i32p, _i8p, _i8p, _u32p]
        L.or_rao_accept.argtypes = [C.c_double, C.c_double, C.c_double, C.c_uint32]
        L.or_enumerate.argtypes = [C.c_int, C.c_void_p, _i8p, C.c_void_p, _i32p, _i64p, C.c_int,
                                   _i32p]
        _lib = L
    return _lib


def _live_ptr(live):
    if live is None:
        return None, None
    arr = np.ascontiguousarray(live, dtype=np.uint8)
    return arr, arr.ctypes.data


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed (rc={rc})")


def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().or_philox(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def num_sites(L):
    return 8 * L * L


def edges(L):
    n = lib().or_edges(L, None, None)
    ei = np.zeros(n, np.int32)
    ej = np.zeros(n, np.int32)
    lib().or_edges(L, ei.ctypes.data, ej.ctypes.data)
    return ei, ej


def energy(L, live, J, bits):
    keep, lp = _live_ptr(live)
    return int(lib().or_energy(L, lp, np.ascontiguousarray(J, np.int8),
                               np.ascontiguousarray(bits, np.uint8)))


def metro_threshold(beta, m):
    return int(lib().or_metro_threshold(beta, m))


def swap_threshold(beta_lo, beta_hi, d):
    return int(lib().or_swap_threshold(beta_lo, beta_hi, d))


class PTState:
    """State of one PT run (see oracle.c): spins word-major uint64[N],
    perm uint8[K*R], energy int32[64], emin int32[R], thit int64[R],
    swap_acc uint32[(K-1)*R], t (completed sweeps), stopped."""

    def __init__(self, N, K, R):
        self.spins = np.zeros(N, np.uint64)
        self.perm = np.zeros(K * R, np.uint8)
        self.energy = np.zeros(64, np.int32)
        self.emin = np.zeros(R, np.int32)
        self.thit = np.zeros(R, np.int64)
        self.swap_acc = np.zeros(max(1, (K - 1) * R), np.uint32)
        self.t = np.zeros(1, np.int64)
        self.stopped = np.zeros(1, np.int32)

    def copy(self):
        s = PTState.__new__(PTState)
        for k, v in self.__dict__.items():
            setattr(s, k, v.copy())
        return s


def pt_init(L, live, J, K, R, key0, key1, init_spins=None):
    st = PTState(num_sites(L), K, R)
    keep, lp = _live_ptr(live)
    ini = None
    ip = None
    if init_spins is not None:
        ini = np.ascontiguousarray(init_spins, np.uint64)
        ip = ini.ctypes.data
    _check(lib().or_pt_init(L, lp, np.ascontiguousarray(J, np.int8), K, R, key0, key1, ip,
                            st.spins, st.perm, st.energy, st.emin, st.thit, st.swap_acc),
           "pt_init")
    return st


def pt_run(L, live, J, K, R, beta, key0, key1, swap_interval, n_sweeps, state,
           stop_on_agreement=False, site_order=None):
    """Advances `state` in place by up to n_sweeps sweeps; returns it."""
    keep, lp = _live_ptr(live)
    order = None
    op = None
    if site_order is not None:
        order = np.ascontiguousarray(site_order, np.int32)
        op = order.ctypes.data
    _check(lib().or_pt_run(L, lp, np.ascontiguousarray(J, np.int8), K, R,
                           np.ascontiguousarray(beta, np.float64), key0, key1, swap_interval,
                           n_sweeps, 1 if stop_on_agreement else 0, op, state.spins, state.perm,
                           state.energy, state.emin, state.thit, state.swap_acc, state.t,
                           state.stopped), "pt_run")
    return state


def pt_swap_extra(L, live, J, K, R, beta, key0, key1, state):
    """One exchange pass outside the schedule (use 3, counter = completed sweeps)."""
    keep, lp = _live_ptr(live)
    _check(lib().or_pt_swap_extra(L, lp, np.ascontiguousarray(J, np.int8), K, R,
                                  np.ascontiguousarray(beta, np.float64), key0, key1,
                                  state.spins, state.perm, state.energy, state.swap_acc,
                                  int(state.t[0])), "pt_swap_extra")
    return state


def lane_energies(L, live, J, lanes, spins):
    out = np.zeros(64, np.int32)
    keep, lp = _live_ptr(live)
    _check(lib().or_lane_energies(L, lp, np.ascontiguousarray(J, np.int8), lanes,
                                  np.ascontiguousarray(spins, np.uint64), out), "lane_energies")
    return out


def hardness_eval(L, live, J, instance_id, seed, n_restarts, K, R, beta, swap_interval, s_max):
    """Returns dict(ln_tts, e_gs, confirmed, r_emin, r_tts, r_sweeps); ln_tts = ln(sum r_sweeps /
    restarts reaching e_gs); r_tts = first-hit sweep, -1 if the restart never reached e_gs."""
    keep, lp = _live_ptr(live)
    ln = np.zeros(1, np.float64)
    egs = np.zeros(1, np.int32)
    conf = np.zeros(1, np.int32)
    r_emin = np.zeros(n_restarts, np.int32)
    r_tts = np.zeros(n_restarts, np.int64)
    r_sw = np.zeros(n_restarts, np.int64)
    _check(lib().or_hardness_eval(L, lp, np.ascontiguousarray(J, np.int8), instance_id, seed,
                                  n_restarts, K, R, np.ascontiguousarray(beta, np.float64),
                                  swap_interval, s_max, ln, egs, conf, r_emin, r_tts, r_sw),
           "hardness_eval")
    return dict(ln_tts=float(ln[0]), e_gs=int(egs[0]), confirmed=bool(conf[0]),
                r_emin=r_emin, r_tts=r_tts, r_sweeps=r_sw)


def mutate(L, live, J, alphabet, chain, seed, step, proposal):
    """Returns (edge index in the full canonical list, old J, new J, accept uniform)."""
    keep, lp = _live_ptr(live)
    e = np.zeros(1, np.int32)
    o = np.zeros(1, np.int8)
    n = np.zeros(1, np.int8)
    w = np.zeros(1, np.uint32)
    alpha = np.ascontiguousarray(alphabet, np.int8)
    _check(lib().or_mutate(L, lp, np.ascontiguousarray(J, np.int8), alpha, len(alpha), chain,
                           seed, step, proposal, e, o, n, w), "mutate")
    return int(e[0]), int(o[0]), int(n[0]), int(w[0])


def rao_accept(ln_cur, ln_new, t_s, w):
    return bool(lib().or_rao_accept(ln_cur, ln_new, t_s, w))


def enumerate_states(L, live, J, want_energies=False):
    """Brute force.  Returns (levels, counts, energies-or-None); energies are
    indexed by the bits of the live sites in ascending order."""
    keep, lp = _live_ptr(live)
    n_live = num_sites(L) if live is None else int(np.count_nonzero(live))
    en = np.zeros(1 << n_live, np.int32) if want_energies else None
    cap = 20000
    he = np.zeros(cap, np.int32)
    hn = np.zeros(cap, np.int64)
    nl = np.zeros(1, np.int32)
    _check(lib().or_enumerate(L, lp, np.ascontiguousarray(J, np.int8),
                              en.ctypes.data if en is not None else None, he, hn, cap, nl),
           "enumerate")
    k = int(nl[0])
    return he[:k].copy(), hn[:k].copy(), en


def ln(x):
    return math.log(x)
