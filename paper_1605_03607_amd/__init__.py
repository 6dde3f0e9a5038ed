"""Python binding of libhardspin (argument marshalling only).

Every step of the parallel-tempering path runs in the library's gfx950
kernels; this module only converts numpy / torch arguments into the C ABI of
include/hardspin.h.  PyTorch is used for device memory and streams.  The
library must have been built (`python -m paper_1605_03607_amd.build`);
importing the binding fails loudly otherwise.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhardspin.so")

HS_INIT_FROM_BUFFER = 1
HS_STOP_ON_AGREEMENT = 2
HS_PACK_LANES = 4

_ERRORS = {-1: "HS_EINVAL", -2: "HS_ENOSPACE", -3: "HS_EUNSUPPORTED", -4: "HS_EHIP",
           -5: "HS_EMISMATCH"}


class HardspinError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class hs_instance(C.Structure):
    _fields_ = [("L", C.c_int32), ("live", C.c_void_p), ("J", C.c_void_p),
                ("instance_id", C.c_uint32), ("K", C.c_int32), ("R", C.c_int32),
                ("beta", C.c_void_p)]


class hs_pt_desc(C.Structure):
    _fields_ = [("n_inst", C.c_int32), ("inst", C.POINTER(hs_instance)), ("seed", C.c_uint32),
                ("swap_interval", C.c_int32), ("flags", C.c_uint32), ("block_waves", C.c_int32)]


class hs_buffers(C.Structure):
    _fields_ = [("spins", C.c_void_p), ("perm", C.c_void_p), ("energy", C.c_void_p),
                ("emin", C.c_void_p), ("thit", C.c_void_p), ("swap_acc", C.c_void_p),
                ("t", C.c_void_p), ("stopped", C.c_void_p), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t)]


class hs_mutation(C.Structure):
    _fields_ = [("edge", C.c_int32), ("old_j", C.c_int8), ("new_j", C.c_int8),
                ("w_accept", C.c_uint32)]


class hs_hardness_params(C.Structure):
    _fields_ = [("n_restarts", C.c_int32), ("K", C.c_int32), ("R", C.c_int32),
                ("beta", C.c_void_p), ("swap_interval", C.c_int32), ("s_max", C.c_int64),
                ("seed", C.c_uint32), ("block_waves", C.c_int32), ("restart_sweeps", C.c_void_p)]


class hs_gnn_batch(C.Structure):
    _fields_ = [("n_graphs", C.c_int32), ("L", C.c_int32), ("live", C.c_void_p), ("J", C.c_void_p)]


class hs_adam(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("step", C.c_int64), ("m", C.c_void_p), ("v", C.c_void_p)]


class hs_tts_detail(C.Structure):
    _fields_ = [("e_gs", C.c_int32), ("confirmed", C.c_int32), ("n_censored", C.c_int32),
                ("sweeps_total", C.c_int64)]


_lib = None


def lib():
    """The loaded libhardspin.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1605_03607_amd.build`")
        # torch ships its own HIP runtime under the same soname: load it first so
        # that the library and torch share one runtime
        _torch()
        L = C.CDLL(LIB_PATH)
        L.hs_version.restype = C.c_int
        L.hs_last_error.restype = C.c_char_p
        L.pt_workspace_bytes.argtypes = [C.POINTER(hs_pt_desc), C.POINTER(C.c_size_t)]
        L.pt_init.argtypes = [C.POINTER(C.c_void_p), C.POINTER(hs_pt_desc), C.POINTER(hs_buffers),
                              C.c_void_p]
        L.pt_sweep.argtypes = [C.c_void_p, C.c_int64]
        L.pt_sweep_record.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int64]
        L.walk_autocorr.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_int, C.c_int, C.c_int,
                                    C.c_void_p, C.c_void_p, C.c_void_p]
        L.pt_capture.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int]
        L.overlap_analyze.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_void_p,
                                      C.c_void_p, C.POINTER(hs_overlap)]
        L.lao_cycle_count.argtypes = [C.c_int, C.c_void_p, C.c_int, C.POINTER(C.c_int64)]
        L.lao_init.argtypes = [C.c_int, C.c_void_p, C.c_int, C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p,
                               C.c_void_p, C.POINTER(C.c_int64)]
        L.lao_move.argtypes = [C.c_int, C.c_void_p, C.c_int, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                               C.c_void_p, C.c_void_p, C.POINTER(C.c_int32), C.c_void_p, C.POINTER(C.c_uint32),
                               C.c_void_p, C.POINTER(C.c_int64)]
        L.walk_tau.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.c_double, C.POINTER(C.c_double),
                               C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.pt_swap.argtypes = [C.c_void_p]
        L.pt_measure.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]
        L.pt_destroy.argtypes = [C.c_void_p]
        L.pt_launch_shape.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        L.pt_graph_create.argtypes = [C.c_void_p, C.c_int64, C.POINTER(C.c_void_p)]
        L.pt_graph_launch.argtypes = [C.c_void_p]
        L.pt_graph_destroy.argtypes = [C.c_void_p]
        L.pt_autotune.argtypes = [C.POINTER(hs_pt_desc), C.POINTER(hs_buffers), C.c_void_p, C.c_int64,
                                  C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.instance_mutate.argtypes = [C.POINTER(hs_instance), C.c_void_p, C.c_int, C.c_uint32,
                                      C.c_uint32, C.c_uint32, C.c_uint32, C.POINTER(hs_mutation)]
        L.hs_rao_accept.argtypes = [C.c_double, C.c_double, C.c_double, C.c_uint32]
        L.hardness_workspace_bytes.argtypes = [C.POINTER(hs_instance), C.c_int,
                                               C.POINTER(hs_hardness_params),
                                               C.POINTER(C.c_size_t)]
        L.hardness_eval.argtypes = [C.POINTER(hs_instance), C.c_int, C.POINTER(hs_hardness_params),
                                    C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(hs_tts_detail),
                                    C.c_void_p]
        L.hardness_eval_static.argtypes = [C.POINTER(hs_instance), C.c_int, C.POINTER(hs_hardness_params),
                                           C.c_void_p, C.POINTER(hs_tts_detail), C.c_void_p]
        L.gnn_param_count.restype = C.c_int
        L.gnn_workspace_bytes.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]
        L.gnn_prepare.argtypes = [C.POINTER(hs_gnn_batch), C.c_void_p, C.c_size_t, C.c_void_p]
        L.gnn_forward.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                  C.c_void_p]
        L.gnn_train_step.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                     C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.POINTER(hs_adam), C.c_void_p]
        L.hs_stream_create_cus.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_void_p)]
        L.hs_stream_destroy.argtypes = [C.c_void_p]
        L.gnn_train_step_ranked.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_float,
                                            C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p,
                                            C.POINTER(hs_adam), C.c_void_p]
        _lib = L
    return _lib


PROBE_NAMES = ["v_add_u32", "v_bitop3_b32", "v_mad_u64_u32", "v_mul_hi_u32", "v_mul_lo_u32",
               "v_dot4_i32_i8", "v_mad_i32_i24"]


def probe_rates(iters=2000):
    """Measured lane-ops/s of each instruction class (libhsprobe.so)."""
    torch = _torch()
    lib()
    path = os.path.join(HERE, "libhsprobe.so")
    P = C.CDLL(path)
    P.hs_probe_rate.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_double), C.c_void_p]
    scratch = torch.zeros(16, dtype=torch.int32, device="cuda")
    out = {}
    for w, name in enumerate(PROBE_NAMES):
        r = C.c_double(0)
        _check(P.hs_probe_rate(w, iters, C.byref(r), C.c_void_p(scratch.data_ptr())))
        out[name] = r.value
    return out


def exported_symbols():
    return ["hs_version", "hs_last_error", "pt_workspace_bytes", "pt_init", "pt_sweep", "pt_swap",
            "pt_measure", "pt_destroy", "pt_graph_create", "pt_graph_launch", "pt_graph_destroy",
            "pt_autotune", "instance_mutate", "hs_rao_accept", "hardness_workspace_bytes",
            "hardness_eval", "gnn_param_count", "gnn_workspace_bytes", "gnn_prepare", "gnn_forward",
            "gnn_train_step", "pt_sweep_record", "walk_autocorr", "walk_tau", "lao_cycle_count", "lao_init",
            "lao_move", "pt_capture", "overlap_analyze", "pt_launch_shape", "hardness_eval_static",
            "gnn_train_step_ranked", "hs_stream_create_cus", "hs_stream_destroy"]


def _check(rc):
    if rc != 0:
        raise HardspinError(rc, lib().hs_last_error().decode())


class hs_overlap(C.Structure):
    _fields_ = [("e0", C.c_int32), ("e1", C.c_int32), ("n_gs", C.c_int32), ("n_ex", C.c_int32),
                ("has_excited", C.c_int32), ("pad_", C.c_int32), ("med_gg", C.c_double),
                ("med_ge", C.c_double), ("ratio", C.c_double)]


class _HostInstances:
    """Keeps the numpy arrays behind an hs_instance[] alive."""

    def __init__(self, insts):
        self.keep = []
        self.arr = (hs_instance * max(1, len(insts)))()
        for n, d in enumerate(insts):
            J = np.ascontiguousarray(d["J"], np.int8)
            beta = np.ascontiguousarray(d["beta"], np.float64)
            live = d.get("live")
            live = None if live is None else np.ascontiguousarray(live, np.uint8)
            self.keep += [J, beta, live]
            x = self.arr[n]
            x.L = int(d["L"])
            x.J = J.ctypes.data
            x.beta = beta.ctypes.data
            x.live = None if live is None else live.ctypes.data
            x.instance_id = int(d.get("instance_id", n))
            x.K = int(d["K"])
            x.R = int(d["R"])


def _torch():
    import torch
    return torch


def cu_stream(cu_first, cu_count):
    """A torch stream (wrapping hs_stream_create_cus) whose kernels run only
    on CUs cu_first .. cu_first + cu_count - 1.  The stream lives as long as
    the process (torch's caching allocator keeps blocks per stream)."""
    torch = _torch()
    h = C.c_void_p()
    _check(lib().hs_stream_create_cus(int(cu_first), int(cu_count), C.byref(h)))
    return torch.cuda.ExternalStream(h.value)


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class PTBatch:
    """A batch of PT instances in device memory (pt_init .. pt_destroy).

    insts: list of dicts with L, J, live (or None), K, R, beta, instance_id.
    """

    def __init__(self, insts, seed, swap_interval=1, flags=0, block_waves=0, init_spins=None,
                 device="cuda", stream=None):
        torch = _torch()
        self.torch = torch
        self.insts = insts
        self.n = len(insts)
        self.Ns = [8 * int(d["L"]) ** 2 for d in insts]
        self.offsets = np.concatenate([[0], np.cumsum(self.Ns)]).astype(np.int64)
        self.hi = _HostInstances(insts)
        self.desc = hs_pt_desc(self.n, C.cast(self.hi.arr, C.POINTER(hs_instance)), seed,
                               swap_interval, flags, block_waves)
        nb = C.c_size_t(0)
        _check(lib().pt_workspace_bytes(C.byref(self.desc), C.byref(nb)))
        _alloc_buffers(self, torch.device(device), self.n, int(self.offsets[-1]), nb.value)
        if init_spins is not None:
            self.spins.copy_(torch.from_numpy(np.ascontiguousarray(init_spins).view(np.int64)))
        self.recomputed = torch.zeros((max(1, self.n), 64), dtype=torch.int32, device=self.spins.device)
        self.stream = stream
        h = C.c_void_p()
        _check(lib().pt_init(C.byref(h), C.byref(self.desc), C.byref(self.bufs),
                             _stream_ptr(stream)))
        self.h = h

    def sweep(self, n_sweeps):
        _check(lib().pt_sweep(self.h, int(n_sweeps)))

    def sweep_record(self, n_sweeps, walk):
        """pt_sweep that writes the temperature walk into `walk` (a uint8
        device tensor [n_inst, capacity, 64]): entry [n, e, c] = temperature
        index of configuration c after the e-th exchange pass of this call."""
        torch = _torch()
        if walk.dtype != torch.uint8 or walk.dim() != 3 or walk.shape[0] < max(1, self.n) or \
                walk.shape[2] != 64 or not walk.is_contiguous() or not walk.is_cuda:
            raise ValueError("walk must be a contiguous CUDA uint8 tensor [n_inst, capacity, 64]")
        _check(lib().pt_sweep_record(self.h, int(n_sweeps), C.c_void_p(walk.data_ptr()), int(walk.shape[1])))

    def capture(self, e_cap, configs, meta, count):
        """pt_capture into device tensors: configs int64 [capacity, n_words],
        meta int32 [capacity, 4], count int32 [1] (cleared by the caller);
        e_cap: energy cap per instance (sequence of ints)."""
        torch = _torch()
        cap = torch.as_tensor(np.ascontiguousarray(e_cap, np.int32)).to(self.spins.device)
        self._cap_keep = cap
        for t, dt in ((configs, torch.int64), (meta, torch.int32), (count, torch.int32)):
            if t.dtype != dt or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("capture buffers: contiguous CUDA int64 configs, int32 meta and count")
        _check(lib().pt_capture(self.h, C.c_void_p(cap.data_ptr()), C.c_void_p(configs.data_ptr()),
                                C.c_void_p(meta.data_ptr()), C.c_void_p(count.data_ptr()), int(configs.shape[0]),
                                int(configs.shape[1])))

    def graph(self, n_sweeps):
        """A captured HIP graph whose replay runs n_sweeps more sweeps."""
        return SweepGraph(self, n_sweeps)

    def swap(self):
        _check(lib().pt_swap(self.h))

    def launch_shape(self):
        """(workgroups in the grid, wavefronts per workgroup, LDS bytes per
        workgroup, work items of the queue, lane slots per sweep) of the
        persistent sweep launch."""
        g, w, b, n, ls = C.c_int32(0), C.c_int32(0), C.c_int32(0), C.c_int32(0), C.c_int64(0)
        _check(lib().pt_launch_shape(self.h, C.byref(g), C.byref(w), C.byref(b), C.byref(n), C.byref(ls)))
        return g.value, w.value, b.value, n.value, ls.value

    def measure(self):
        """Recomputes energies on the device; returns the mismatch count."""
        mm = C.c_int32(0)
        rc = lib().pt_measure(self.h, C.c_void_p(self.recomputed.data_ptr()), C.byref(mm))
        if rc not in (0, -5):
            _check(rc)
        return int(mm.value)

    def state(self, n):
        """Host copy of instance n's state, in the oracle's PTState layout."""
        self.torch.cuda.synchronize()
        d = self.insts[n]
        K, R = int(d["K"]), int(d["R"])
        a, b = int(self.offsets[n]), int(self.offsets[n + 1])
        return dict(
            spins=self.spins[a:b].cpu().numpy().view(np.uint64).copy(),
            perm=self.perm[n, :K * R].cpu().numpy().copy(),
            energy=self.energy[n].cpu().numpy().copy(),
            emin=self.emin[n, :R].cpu().numpy().copy(),
            thit=self.thit[n, :R].cpu().numpy().copy(),
            swap_acc=self.swap_acc[n, :max(1, (K - 1) * R)].cpu().numpy().view(np.uint32).copy()
            if K > 1 else np.zeros(1, np.uint32),
            t=int(self.t[n].item()),
            stopped=int(self.stopped[n].item()),
        )

    def close(self):
        if getattr(self, "h", None):
            lib().pt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SweepGraph:
    """pt_graph_create / pt_graph_launch / pt_graph_destroy."""

    def __init__(self, batch, n_sweeps):
        self.batch = batch
        g = C.c_void_p()
        _check(lib().pt_graph_create(batch.h, int(n_sweeps), C.byref(g)))
        self.g = g

    def launch(self):
        _check(lib().pt_graph_launch(self.g))

    def close(self):
        if getattr(self, "g", None):
            lib().pt_graph_destroy(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _alloc_buffers(obj, dev, n_inst, total_spins, workspace_bytes):
    """Device buffers of a batch (hs_buffers layout) as torch tensors on obj."""
    torch = _torch()
    n = max(1, n_inst)
    obj.spins = torch.zeros(max(1, total_spins), dtype=torch.int64, device=dev)
    obj.perm = torch.zeros((n, 64), dtype=torch.uint8, device=dev)
    obj.energy = torch.zeros((n, 64), dtype=torch.int32, device=dev)
    obj.emin = torch.zeros((n, 64), dtype=torch.int32, device=dev)
    obj.thit = torch.zeros((n, 64), dtype=torch.int64, device=dev)
    obj.swap_acc = torch.zeros((n, 64), dtype=torch.int32, device=dev)
    obj.t = torch.zeros(n, dtype=torch.int64, device=dev)
    obj.stopped = torch.zeros(n, dtype=torch.int32, device=dev)
    obj.workspace = torch.zeros(max(16, workspace_bytes), dtype=torch.uint8, device=dev)
    obj.bufs = hs_buffers(obj.spins.data_ptr(), obj.perm.data_ptr(), obj.energy.data_ptr(),
                          obj.emin.data_ptr(), obj.thit.data_ptr(), obj.swap_acc.data_ptr(),
                          obj.t.data_ptr(), obj.stopped.data_ptr(), obj.workspace.data_ptr(),
                          workspace_bytes)


def autotune(insts, seed, swap_interval=1, flags=0, trial_sweeps=200, device="cuda", stream=None):
    """pt_autotune on scratch buffers: returns (block_waves, microseconds per sweep)."""
    hi = _HostInstances(insts)
    desc = hs_pt_desc(len(insts), C.cast(hi.arr, C.POINTER(hs_instance)), seed, swap_interval,
                      flags, 0)
    need = 0
    for bw in (2, 4, 8, 16):
        desc.block_waves = bw
        nb = C.c_size_t(0)
        _check(lib().pt_workspace_bytes(C.byref(desc), C.byref(nb)))
        need = max(need, nb.value)
    desc.block_waves = 0

    class _Scratch:
        pass

    sc = _Scratch()
    total = sum(8 * int(d["L"]) ** 2 for d in insts)
    _alloc_buffers(sc, _torch().device(device), len(insts), total, need)
    bw = C.c_int32(0)
    us = C.c_double(0)
    _check(lib().pt_autotune(C.byref(desc), C.byref(sc.bufs), _stream_ptr(stream), int(trial_sweeps),
                             C.byref(bw), C.byref(us)))
    return int(bw.value), float(us.value)


def instance_mutate(inst, alphabet, chain, seed, step, proposal):
    hi = _HostInstances([dict(inst, K=inst.get("K", 1), R=inst.get("R", 1),
                              beta=inst.get("beta", np.ones(1)))])
    alpha = np.ascontiguousarray(alphabet, np.int8)
    out = hs_mutation()
    _check(lib().instance_mutate(C.byref(hi.arr[0]), alpha.ctypes.data, len(alpha), chain, seed,
                                 step, proposal, C.byref(out)))
    return int(out.edge), int(out.old_j), int(out.new_j), int(out.w_accept)


def rao_accept(ln_cur, ln_new, t_s, w):
    return bool(lib().hs_rao_accept(ln_cur, ln_new, t_s, w))


def hardness_eval(cands, n_restarts, K, R, beta, swap_interval, s_max, seed, block_waves=0,
                  stream=None):
    """ln TTS per candidate (dicts with L, J, live, instance_id) plus details
    (restart_sweeps: the sweeps t of every restart)."""
    torch = _torch()
    hi = _HostInstances([dict(c, K=K, R=R, beta=beta) for c in cands])
    beta_arr = np.ascontiguousarray(beta, np.float64)
    rs = np.zeros((max(1, len(cands)), n_restarts), np.int64)
    p = hs_hardness_params(n_restarts, K, R, beta_arr.ctypes.data, swap_interval, s_max, seed,
                           block_waves, rs.ctypes.data)
    nb = C.c_size_t(0)
    _check(lib().hardness_workspace_bytes(hi.arr, len(cands), C.byref(p), C.byref(nb)))
    # hardness_eval writes every scratch byte its launch reads: no fill kernel
    # (which would wait for CUs held by other streams' persistent launches)
    scratch = torch.empty(max(16, nb.value), dtype=torch.uint8, device="cuda")
    ln = np.zeros(len(cands), np.float64)
    det = (hs_tts_detail * max(1, len(cands)))()
    _check(lib().hardness_eval(hi.arr, len(cands), C.byref(p), C.c_void_p(scratch.data_ptr()),
                               nb.value, ln.ctypes.data, det, _stream_ptr(stream)))
    details = [dict(e_gs=det[i].e_gs, confirmed=bool(det[i].confirmed),
                    n_censored=det[i].n_censored, sweeps_total=det[i].sweeps_total,
                    restart_sweeps=rs[i].copy())
               for i in range(len(cands))]
    return ln, details


HS_STATIC_SCRATCH_BYTES = 64 << 20


def hardness_eval_static(cands, n_restarts, K, R, beta, swap_interval, s_max, seed, block_waves=0,
                         stream=None):
    """hardness_eval through hardness_eval_static: the library's static
    device scratch instead of a buffer allocated here (nothing is allocated
    on the device)."""
    hi = _HostInstances([dict(c, K=K, R=R, beta=beta) for c in cands])
    beta_arr = np.ascontiguousarray(beta, np.float64)
    rs = np.zeros((max(1, len(cands)), n_restarts), np.int64)
    p = hs_hardness_params(n_restarts, K, R, beta_arr.ctypes.data, swap_interval, s_max, seed,
                           block_waves, rs.ctypes.data)
    ln = np.zeros(len(cands), np.float64)
    det = (hs_tts_detail * max(1, len(cands)))()
    _check(lib().hardness_eval_static(hi.arr, len(cands), C.byref(p), ln.ctypes.data, det, _stream_ptr(stream)))
    details = [dict(e_gs=det[i].e_gs, confirmed=bool(det[i].confirmed),
                    n_censored=det[i].n_censored, sweeps_total=det[i].sweeps_total,
                    restart_sweeps=rs[i].copy())
               for i in range(len(cands))]
    return ln, details


# ---------------------------------------------------------------------------
# Ground / first-excited overlaps (hardspin.h).
def overlap_analyze(configs, energies, live_bits_words, n_live, stream=None):
    """configs: host uint64 [n, n_words] of one instance; energies: [n];
    live_bits_words: host uint64 [n_words] mask of live sites."""
    torch = _torch()
    cfg = torch.from_numpy(np.ascontiguousarray(configs, np.uint64).view(np.int64)).cuda()
    mask = torch.from_numpy(np.ascontiguousarray(live_bits_words, np.uint64).view(np.int64)).cuda()
    e = np.ascontiguousarray(energies, np.int32)
    n, w = cfg.shape
    scratch = torch.zeros(max(1, n * n), dtype=torch.int32, device=cfg.device)
    out = hs_overlap()
    _check(lib().overlap_analyze(C.c_void_p(cfg.data_ptr()), e.ctypes.data, int(n), int(w),
                                 C.c_void_p(mask.data_ptr()), int(n_live), C.c_void_p(scratch.data_ptr()),
                                 _stream_ptr(stream), C.byref(out)))
    return dict(e0=out.e0, e1=out.e1 if out.has_excited else None, n_gs=out.n_gs, n_ex=out.n_ex,
                med_gg=out.med_gg, med_ge=out.med_ge if out.has_excited else None,
                ratio=out.ratio if out.has_excited else None)


def pack_sites(bits):
    """uint8 [N] site bits -> uint64 words, bit b of word w = site 64 w + b."""
    b = np.asarray(bits, np.uint8)
    words = np.zeros((len(b) + 63) // 64, np.uint64)
    for i in np.nonzero(b)[0]:
        words[i // 64] |= np.uint64(1) << np.uint64(i % 64)
    return words


# ---------------------------------------------------------------------------
# Planted-solution instances and LAO moves (hardspin.h).
def _n_couplers(L):
    return 24 * L * L - 8 * L


def _live_arg(live):
    if live is None:
        return None, None
    a = np.ascontiguousarray(live, np.uint8)
    return a, C.c_void_p(a.ctypes.data)


def lao_cycle_count(L, size, live=None):
    keep, lp = _live_arg(live)
    n = C.c_int64(0)
    _check(lib().lao_cycle_count(int(L), lp, int(size), C.byref(n)))
    return n.value


def lao_init(L, n_loops, chain, seed, live=None):
    """Planted instance: dict(loops int32 [n_loops, 4] = (size, cycle,
    weight, flip), bits uint8 [N], J int8, e_gs)."""
    keep, lp = _live_arg(live)
    loops = np.zeros((n_loops, 4), np.int32)
    bits = np.zeros(8 * L * L, np.uint8)
    J = np.zeros(_n_couplers(L), np.int8)
    e = C.c_int64(0)
    _check(lib().lao_init(int(L), lp, int(n_loops), int(chain), int(seed), loops.ctypes.data, bits.ctypes.data,
                          J.ctypes.data, C.byref(e)))
    return dict(loops=loops, bits=bits, J=J, e_gs=e.value)


def lao_move(L, inst, chain, seed, step, proposal, live=None):
    """(slot, new loop (size, cycle, weight, flip), w_accept, J', e_gs')."""
    keep, lp = _live_arg(live)
    loops = np.ascontiguousarray(inst["loops"], np.int32)
    bits = np.ascontiguousarray(inst["bits"], np.uint8)
    slot, w = C.c_int32(0), C.c_uint32(0)
    new = np.zeros(4, np.int32)
    J = np.zeros(_n_couplers(L), np.int8)
    e = C.c_int64(0)
    _check(lib().lao_move(int(L), lp, len(loops), int(chain), int(seed), int(step), int(proposal), loops.ctypes.data,
                          bits.ctypes.data, C.byref(slot), new.ctypes.data, C.byref(w), J.ctypes.data, C.byref(e)))
    return slot.value, tuple(int(x) for x in new), w.value, J, e.value


# ---------------------------------------------------------------------------
# Mixing time of the temperature walk (include/hs_walk.h).
def walk_autocorr(walk, n_steps, K, R, max_lag, stream=None):
    """Exact autocorrelation sums S(d) (int64 [n_inst, max_lag + 1]) and
    hot-half passes (int64 [n_inst, 64]) of a walk tensor written by
    PTBatch.sweep_record; returned as numpy arrays."""
    torch = _torch()
    n_inst, cap = int(walk.shape[0]), int(walk.shape[1])
    acf = torch.zeros((max(1, n_inst), max_lag + 1), dtype=torch.int64, device=walk.device)
    hot = torch.zeros((max(1, n_inst), 64), dtype=torch.int64, device=walk.device)
    _check(lib().walk_autocorr(C.c_void_p(walk.data_ptr()), n_inst, cap, int(n_steps), int(K), int(R),
                               int(max_lag), C.c_void_p(acf.data_ptr()), C.c_void_p(hot.data_ptr()),
                               _stream_ptr(stream)))
    return acf.cpu().numpy()[:n_inst], hot.cpu().numpy()[:n_inst]


def walk_tau(acf_row, n_steps, c_window=6.0):
    """(tau in exchange passes, window, converged) from one row of S(d)."""
    a = np.ascontiguousarray(acf_row, np.int64)
    tau, win, conv = C.c_double(0), C.c_int(0), C.c_int(0)
    _check(lib().walk_tau(a.ctypes.data, len(a) - 1, int(n_steps), float(c_window), C.byref(tau), C.byref(win),
                          C.byref(conv)))
    return tau.value, win.value, bool(conv.value)


# ---------------------------------------------------------------------------
# Hardness surrogate (include/hs_gnn.h).
GNN_WIDTH = 64


def gnn_fan_ins():
    """(size, fan_in) of every parameter block, in the library's order."""
    D = GNN_WIDTH
    blocks = [(D * 5, 5), (D, 0), (D * 4, 4), (D, 0)]
    for _ in range(3):
        blocks += [(D * 3 * D, 3 * D), (D, 0), (D * 2 * D, 2 * D), (D, 0)]
    return blocks + [(D, D), (1, 0)]


class Surrogate:
    """Parameters, Adam state and workspace of the surrogate on one device.

    graphs: list of (L, live or None, J) with one L per call."""

    def __init__(self, params, device="cuda", stream=None):
        torch = _torch()
        self.torch = torch
        n = lib().gnn_param_count()
        params = np.ascontiguousarray(params, np.float32)
        if params.size != n:
            raise ValueError(f"expected {n} parameters")
        dev = torch.device(device)
        self.params = torch.from_numpy(params.copy()).to(dev)
        self.m = torch.zeros(n, dtype=torch.float32, device=dev)
        self.v = torch.zeros(n, dtype=torch.float32, device=dev)
        self.grad = torch.zeros(n, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.step = 0
        self.stream = stream
        self.ws = None
        self.shape = None

    def prepare(self, graphs):
        torch = self.torch
        G = len(graphs)
        L = int(graphs[0][0])
        if any(int(g[0]) != L for g in graphs):
            raise ValueError("one L per batch")
        nb = C.c_size_t(0)
        _check(lib().gnn_workspace_bytes(G, L, C.byref(nb)))
        if self.ws is None or self.ws.numel() < nb.value:
            self.ws = torch.zeros(nb.value, dtype=torch.uint8, device=self.params.device)
        N = 8 * L * L
        J = np.ascontiguousarray(np.concatenate([np.asarray(g[2], np.int8) for g in graphs]))
        lives = [g[1] for g in graphs]
        live = None
        if any(x is not None for x in lives):
            live = np.ascontiguousarray(np.concatenate(
                [np.ones(N, np.uint8) if x is None else np.asarray(x, np.uint8) for x in lives]))
        b = hs_gnn_batch(G, L, None if live is None else live.ctypes.data, J.ctypes.data)
        _check(lib().gnn_prepare(C.byref(b), C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                 _stream_ptr(self.stream)))
        self.shape = (G, L)

    def forward(self, graphs=None):
        """y_hat (numpy float32) of the prepared (or given) batch."""
        if graphs is not None:
            self.prepare(graphs)
        G, L = self.shape
        y = self.torch.zeros(G, dtype=self.torch.float32, device=self.params.device)
        _check(lib().gnn_forward(C.c_void_p(self.params.data_ptr()), G, L, C.c_void_p(self.ws.data_ptr()),
                                 self.ws.numel(), C.c_void_p(y.data_ptr()), _stream_ptr(self.stream)))
        return y.cpu().numpy()

    def train_step(self, labels, graphs=None, lr=1e-3, update=True, betas=(0.9, 0.999), eps=1e-8, ref=None,
                   w_abs=1.0):
        """One step on the prepared (or given) batch: (loss, y_hat); the
        gradient stays in self.grad.  update=False leaves the parameters.
        With ref (the index of each graph's parent in the batch, -1 for
        none) the step takes the ranked loss (gnn_train_step_ranked) with
        weight w_abs on the plain term."""
        torch = self.torch
        if graphs is not None:
            self.prepare(graphs)
        G, L = self.shape
        lab = torch.from_numpy(np.ascontiguousarray(labels, np.float32)).to(self.params.device)
        y = torch.zeros(G, dtype=torch.float32, device=self.params.device)
        adam = None
        if update:
            self.step += 1
            adam = hs_adam(lr, betas[0], betas[1], eps, self.step, self.m.data_ptr(), self.v.data_ptr())
        tail = (C.c_void_p(self.ws.data_ptr()), self.ws.numel(), C.c_void_p(y.data_ptr()),
                C.c_void_p(self.loss.data_ptr()), C.c_void_p(self.grad.data_ptr()),
                None if adam is None else C.byref(adam), _stream_ptr(self.stream))
        if ref is None:
            _check(lib().gnn_train_step(C.c_void_p(self.params.data_ptr()), G, L, C.c_void_p(lab.data_ptr()),
                                        *tail))
        else:
            r = np.ascontiguousarray(ref, np.int32)
            if r.shape != (G,):
                raise ValueError("one parent index per graph")
            rd = torch.from_numpy(r).to(self.params.device)
            _check(lib().gnn_train_step_ranked(C.c_void_p(self.params.data_ptr()), G, L,
                                               C.c_void_p(lab.data_ptr()), C.c_void_p(rd.data_ptr()),
                                               float(w_abs), *tail))
        return float(self.loss.item()), y.cpu().numpy()
