"""The C-ABI library loads, exports every declared entry point, and its
host-only functions agree with the oracle (no GPU needed)."""
import math
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hardspin.h")
GNN_HEADER = os.path.join(ROOT, "include", "hs_gnn.h")
PROBE_HEADER = os.path.join(ROOT, "include", "hs_probe.h")
WALK_HEADER = os.path.join(ROOT, "include", "hs_walk.h")


def _hs():
    import paper_1605_03607_amd as hs
    if not os.path.exists(hs.LIB_PATH):
        pytest.skip("libhardspin.so not built")
    return hs


def _declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:int|const char \*)\s*\**\s*([a-z_]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for want in ("pt_init", "pt_sweep", "pt_swap", "pt_measure", "instance_mutate",
                 "hardness_eval", "pt_destroy", "hs_last_error", "pt_workspace_bytes",
                 "hs_version"):
        assert want in names


def test_library_exports_every_declared_symbol():
    hs = _hs()
    out = subprocess.run(["nm", "-D", "--defined-only", hs.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    declared = _declared_functions() + _declared_functions(GNN_HEADER) + _declared_functions(WALK_HEADER)
    assert {"pt_sweep_record", "walk_autocorr", "walk_tau"} <= set(declared)
    missing = [n for n in declared if n not in exported]
    assert not missing, missing
    lib = hs.lib()
    assert lib.hs_version() >= 10000
    for n in declared:
        assert hasattr(lib, n)


def test_probe_library_exports_its_entry_point():
    hs = _hs()
    path = os.path.join(os.path.dirname(hs.LIB_PATH), "libhsprobe.so")
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    names = _declared_functions(PROBE_HEADER)
    assert names and all(n in exported for n in names)


def test_gnn_host_entry_points():
    """Parameter count matches the oracle's layout; the workspace grows with
    the batch; malformed arguments are rejected without a GPU."""
    import ctypes as C
    import oracle.gnn as G
    hs = _hs()
    lib = hs.lib()
    assert lib.gnn_param_count() == G.n_params()
    a, b = C.c_size_t(0), C.c_size_t(0)
    assert lib.gnn_workspace_bytes(1, 8, C.byref(a)) == 0
    assert lib.gnn_workspace_bytes(16, 8, C.byref(b)) == 0
    assert b.value > 10 * a.value > 0
    assert lib.gnn_workspace_bytes(0, 8, C.byref(a)) == -1
    assert lib.gnn_workspace_bytes(1, 17, C.byref(a)) == -1
    # the ranked step needs its parent indices and a finite w_abs >= 0
    dummy = C.c_void_p(16)
    assert lib.gnn_train_step_ranked(dummy, 1, 8, dummy, None, 0.1, dummy, 1, None, dummy, dummy, None,
                                     None) == -1
    assert b"NULL ref" in lib.hs_last_error()
    for w in (-0.5, float("nan"), float("inf")):
        assert lib.gnn_train_step_ranked(dummy, 1, 8, dummy, dummy, w, dummy, 1, None, dummy, dummy, None,
                                         None) == -1
        assert b"w_abs" in lib.hs_last_error()


def test_cu_stream_entry_points_check_their_arguments():
    """hs_stream_create_cus needs somewhere to put the stream; destroying
    NULL is a no-op (no GPU needed for either)."""
    hs = _hs()
    lib = hs.lib()
    assert lib.hs_stream_create_cus(0, 8, None) == -1
    assert b"NULL stream" in lib.hs_last_error()
    assert lib.hs_stream_destroy(None) == 0


def test_library_has_gfx950_code():
    hs = _hs()
    # the embedded offload bundle names its target
    data = open(hs.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in data


@pytest.mark.parametrize("alphabet", ["pm1", "pm7"])
def test_instance_mutate_matches_oracle(alphabet):
    hs = _hs()
    L = 4
    A = workloads.ALPHABETS[alphabet]
    J = workloads.couplings(L, alphabet, 3, 0)
    live = workloads.missing_mask(L, 0.02, 3, 0)
    inst = dict(L=L, J=J, live=live)
    for step in range(300):
        for prop in (0, 5, 15):
            got = hs.instance_mutate(inst, A, 11, 2016, step, prop)
            want = oracle.mutate(L, live, J, A, 11, 2016, step, prop)
            assert got == want


def test_rao_accept_matches_oracle():
    hs = _hs()
    rng = np.random.default_rng(4)
    cases = [(1.0, 2.0), (2.0, 1.0), (3.0, 2.5), (math.inf, 4.0), (4.0, math.inf),
             (math.inf, math.inf)]
    for cur, new in cases:
        for w in rng.integers(0, 2 ** 32, size=200):
            assert hs.rao_accept(cur, new, 0.5, int(w)) == oracle.rao_accept(cur, new, 0.5, int(w))


def test_invalid_descriptors_are_rejected():
    hs = _hs()
    import ctypes as C
    base = dict(L=4, J=workloads.couplings(4, "pm1", 1, 0), live=None, K=4, R=2,
                beta=workloads.geometric_betas(0.1, 1.0, 4), instance_id=0)
    bad = [
        dict(base, L=17),                        # L > 16
        dict(base, K=40, R=2),                   # K R > 64
        dict(base, beta=np.array([0.1, 0.2, 0.2, 0.3])),  # not strictly ascending
        dict(base, beta=np.array([-0.1, 0.2, 0.3, 0.4])),
        dict(base, J=np.full(352, 9, np.int8)),  # |J| > 7
    ]
    for inst in bad:
        hi = hs._HostInstances([inst])
        desc = hs.hs_pt_desc(1, C.cast(hi.arr, C.POINTER(hs.hs_instance)), 1, 1, 0, 0)
        nb = C.c_size_t(0)
        rc = hs.lib().pt_workspace_bytes(C.byref(desc), C.byref(nb))
        assert rc in (-1, -3), inst
        assert hs.lib().hs_last_error()
    hi = hs._HostInstances([dict(base, R=1)])
    desc = hs.hs_pt_desc(1, C.cast(hi.arr, C.POINTER(hs.hs_instance)), 1, 1,
                         hs.HS_STOP_ON_AGREEMENT, 0)
    nb = C.c_size_t(0)
    assert hs.lib().pt_workspace_bytes(C.byref(desc), C.byref(nb)) == -1


def test_workspace_grows_with_batch():
    hs = _hs()
    import ctypes as C
    sizes = []
    for n in (1, 4, 16):
        insts = workloads.make_batch(workloads.batch_c8(), n)
        hi = hs._HostInstances(insts)
        desc = hs.hs_pt_desc(n, C.cast(hi.arr, C.POINTER(hs.hs_instance)), 1, 10, 0, 0)
        nb = C.c_size_t(0)
        assert hs.lib().pt_workspace_bytes(C.byref(desc), C.byref(nb)) == 0
        sizes.append(nb.value)
    assert sizes[0] < sizes[1] < sizes[2]


def test_walk_tau_matches_oracle():
    """The library's window rule and tau against the oracle's, on the sums
    of a seeded two-state chain, of independent draws and of a short run."""
    import oracle.walk as W
    hs = _hs()
    rng = np.random.default_rng(8)
    cases = []
    for p, T in ((0.05, 50_000), (0.3, 20_000), (0.5, 3)):
        st = np.cumsum(rng.random(T) < p) % 2
        cases.append((W.acf_sums(st[:, None], 2, 200), T))
    cases.append((W.acf_sums(rng.integers(0, 6, size=(5000, 4)), 6, 40), 5000))
    cases.append((np.zeros(5, np.int64), 100))
    for S, T in cases:
        got = hs.walk_tau(S, T)
        want = W.tau_int(S, T)
        assert got[1:] == tuple(want[1:])
        assert abs(got[0] - want[0]) <= 1e-12 * max(1.0, abs(want[0]))


def test_walk_entry_points_reject_bad_sizes():
    hs = _hs()
    import ctypes as C
    lib = hs.lib()
    acf = np.zeros(4, np.int64)
    tau, win, conv = C.c_double(), C.c_int(), C.c_int()
    assert lib.walk_tau(None, 3, 10, 6.0, C.byref(tau), C.byref(win), C.byref(conv)) == -1
    assert lib.walk_tau(acf.ctypes.data, -1, 10, 6.0, C.byref(tau), C.byref(win), C.byref(conv)) == -1
    for args in ((0, 4, 5, 8, 2, 10), (0, 4, 2, 0, 2, 10), (0, 4, 2, 8, 9, 10), (0, 4, 2, 8, 2, -1),
                 (-1, 4, 2, 8, 2, 10)):
        n, cap, T, K, R, lag = args
        assert lib.walk_autocorr(None, n, cap, T, K, R, lag, None, None, None) == -1, args
    assert lib.walk_autocorr(None, 0, 4, 2, 8, 2, 10, None, None, None) == 0
    assert lib.pt_sweep_record(None, 10, None, 0) == -1


@pytest.mark.parametrize("L,missing", [(1, 0.0), (2, 0.0), (3, 0.05)])
def test_lao_matches_oracle(L, missing):
    """Planted instances and loop moves of the library equal the oracle's:
    cycle counts, loops, planted bits, couplings, ground-state energies."""
    import oracle.lao as P
    hs = _hs()
    live = workloads.missing_mask(L, missing, 13, L) if missing else None
    cyc = P.cycles(L, live)
    for n in (4, 6):
        assert hs.lao_cycle_count(L, n, live) == len(cyc[n])
    M = {1: 5, 2: 14, 3: 40}[L]
    for chain in range(3):
        got = hs.lao_init(L, M, chain, 21, live)
        want = P.init(L, M, chain, 21, live=live, cyc=cyc)
        assert [tuple(r) for r in got["loops"].tolist()] == [tuple(x) for x in want["loops"]]
        assert np.array_equal(got["bits"], want["bits"])
        assert np.array_equal(got["J"], want["J"]) and got["e_gs"] == want["e_gs"]
        for step in range(4):
            g = hs.lao_move(L, got, chain, 21, step, 1, live)
            w = P.move(L, want, chain, 21, step, 1, live=live, cyc=cyc)
            assert g[0] == w[0] and g[2] == w[2]
            assert g[0] < 0 or g[1] == tuple(w[1])
            assert np.array_equal(g[3], w[3]) and g[4] == w[4]


def test_lao_rejects_bad_arguments():
    hs = _hs()
    with pytest.raises(RuntimeError):
        hs.lao_init(0, 5, 0, 0)
    with pytest.raises(RuntimeError):
        hs.lao_init(2, 0, 0, 0)
    with pytest.raises(RuntimeError):
        hs.lao_cycle_count(2, 5)
    inst = hs.lao_init(2, 6, 0, 0)
    bad = dict(inst, loops=inst["loops"].copy())
    bad["loops"][2, 1] = 10 ** 6
    with pytest.raises(RuntimeError):
        hs.lao_move(2, bad, 0, 0, 1, 0)


def test_lao_moves_keep_the_cap_and_match_oracle_on_dense_c4():
    """Dense loops (120 on C4): removing a loop can push a shared coupler
    past |J| = 7, so some proposals are void; every candidate stays within
    the cap and library and oracle agree move by move."""
    import oracle.lao as P
    hs = _hs()
    cyc = P.cycles(4)
    g = hs.lao_init(4, 120, 2, 8)
    o = P.init(4, 120, 2, 8, cyc=cyc)
    voids = 0
    for step in range(60):
        a = hs.lao_move(4, g, 2, 8, step, 0)
        b = P.move(4, o, 2, 8, step, 0, cyc=cyc)
        assert a[0] == b[0] and np.array_equal(a[3], b[3]) and a[4] == b[4]
        assert int(np.abs(a[3].astype(int)).max()) <= 7
        if a[0] < 0:
            voids += 1
            assert np.array_equal(a[3], g["J"])
            continue
        g = dict(g, loops=g["loops"].copy(), J=a[3], e_gs=a[4])
        g["loops"][a[0]] = a[1]
        o = dict(o, loops=list(o["loops"]), J=b[3], e_gs=b[4])
        o["loops"][b[0]] = b[1]
        J, e = P.couplings(4, o["loops"], cyc, o["bits"])
        assert np.array_equal(J, a[3]) and e == a[4]
    assert voids > 0


def test_mutation_rejects_alphabets_that_are_not_sets_holding_the_value():
    """Algorithm 1 replaces a coupler's value by another value of the
    alphabet: an alphabet with a repeated letter, or one without the chosen
    coupler's current value, is an error in the library and in the oracle
    (never an out-of-range read)."""
    hs = _hs()
    L = 2
    J = workloads.couplings(L, "pm1", 3, 0)
    inst = dict(L=L, J=J, live=None)
    bad = [np.array([-1, 1, 1], np.int8), np.array([-1, -1], np.int8), np.array([2, 3, 4], np.int8)]
    for A in bad:
        with pytest.raises(RuntimeError):
            hs.instance_mutate(inst, A, 0, 1, 0, 0)
        with pytest.raises(ValueError):
            oracle.mutate(L, None, J, A, 0, 1, 0, 0)
    good = np.array([-1, 1], np.int8)
    assert hs.instance_mutate(inst, good, 0, 1, 0, 0) == oracle.mutate(L, None, J, good, 0, 1, 0, 0)


def test_closely_spaced_ladder_keeps_the_exchange_table_bounded():
    """Exchange thresholds are tabulated only up to the largest energy
    difference an instance allows (2 sum |J|): a ladder with a spacing of
    1e-9 (where floor(2^32 e^{-d dbeta}) stays positive for ~2e10 entries)
    is accepted at once with a small workspace."""
    hs = _hs()
    import ctypes as C
    import time
    L = 4
    J = workloads.couplings(L, "pm7", 5, 0)
    d = dict(L=L, J=J, live=None, K=2, R=1, beta=np.array([1.0, 1.0 + 1e-9]), instance_id=0)
    hi = hs._HostInstances([d])
    desc = hs.hs_pt_desc(1, C.cast(hi.arr, C.POINTER(hs.hs_instance)), 1, 1, 0, 0)
    nb = C.c_size_t(0)
    t0 = time.perf_counter()
    assert hs.lib().pt_workspace_bytes(C.byref(desc), C.byref(nb)) == 0
    assert time.perf_counter() - t0 < 5.0
    two_sum_j = 2 * int(np.abs(J.astype(np.int64)).sum())
    assert nb.value < 64 * 1024 + 8 * two_sum_j


def test_destroy_of_a_null_handle_is_a_no_op():
    hs = _hs()
    assert hs.lib().pt_destroy(None) == 0
    assert hs.lib().pt_launch_shape(None, None, None, None, None, None) == -1
