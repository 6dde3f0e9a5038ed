"""Instance-space search driven by the gfx950 engine (Algorithm 1, Sec. II.A).

Every chain holds one instance J.  A step proposes coupler mutations
(instance_mutate over `alphabet`: +-1..+-7 by default, +-1 for Algorithm 1's
sign flips), scores candidates with hardness_eval (ln of the PT run time per
find of the ground state over independent restarts, in sweeps; Appendix B)
and accepts by Metropolis in ln TTS at search temperature t_s
(hs_rao_accept).  Three modes:

  plain      one proposal per chain, scored by PT (Algorithm 1 as written)
  surrogate  `proposals` mutations per chain ranked by the surrogate network;
             the `top` best go to PT, the one with the larger PT score (ties:
             lower proposal index) enters the acceptance test; the network
             is trained online on every PT-scored (J, ln TTS) pair
  random     as surrogate, but the `top` candidates are chosen at random
             (the ablation: what ranking by the network gains)

PT scores every instance that can be accepted.  A hard instance is an
accepted state with ln TTS >= H0 + ln(bar), H0 = median ln TTS of the seed
instances; distinct hard instances are counted by their couplings.

direction = -1 is the reversed search of Sec. II.B: the acceptance test runs
on -ln TTS (shorter times are favoured), the screen keeps the proposals with
the lowest predicted ln TTS, the better of the PT-scored candidates is the
one with the lower ln TTS, and the counted states are the easy ones,
ln TTS <= H0 - ln(bar).  Every acceptance decision is logged in `decisions`
as (step, chain, ln_cur, ln_new, w, accepted).

GroupedSearch runs the chains of one search as G groups, each group stepping
in its own host thread on its own stream.  One PT launch lasts as long as its
slowest restart, and the runs that stop early leave most of the chip idle
during that tail; launches of the other groups fill it.  The groups share the
surrogate and its replay buffer (under a lock).  Chains keep their global
indices, so every random draw (PT streams, mutations, the random screen) is
the one the single-group search makes: plain and random searches take the
same decisions under any grouping; the surrogate arm's training order, and
with it its screen, depends on the order in which groups finish.
"""
import hashlib
import math
import queue
import threading
import time

import numpy as np

from . import Surrogate, hardness_eval, instance_mutate, rao_accept

ALPHABET_PM7 = np.array([-7, -6, -5, -4, -3, -2, -1, 1, 2, 3, 4, 5, 6, 7], np.int8)
ALPHABET_PM1 = np.array([-1, 1], np.int8)  # Algorithm 1's sign flips


def _launch(c):
    """hardness_eval's launch shape for config c: the wavefronts per
    workgroup when set (results do not depend on it), else the library's
    choice."""
    return {"block_waves": c.block_waves} if c.block_waves else {}


def _timed_hardness(cands, c):
    """hardness_eval on the calling thread's current stream, with the device
    span of the call from events recorded on that stream: (ln, details, ms,
    spin-flip attempts)."""
    import torch
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    ln, det = hardness_eval(cands, c.restarts, c.K, c.R, c.beta, c.swap_interval, c.s_max, c.seed, **_launch(c))
    end.record()
    end.synchronize()
    lanes_sites = c.K * c.R * 8 * c.L * c.L
    return ln, det, start.elapsed_time(end), sum(d["sweeps_total"] for d in det) * lanes_sites


def _geometric(lo, hi, k):
    if k == 1:
        return np.array([float(lo)])
    return lo * (hi / lo) ** (np.arange(k) / (k - 1))


class SearchConfig:
    def __init__(self, mode="plain", chains=64, L=8, restarts=32, K=32, R=2, beta=(0.1, 5.0),
                 swap_interval=1, s_max=100_000, t_s=0.5, seed=1605, proposals=16, top=2,
                 train_steps=32, train_batch=32, lr=3e-3, replay=4096, screen_chunk=128, direction=1,
                 alphabet=ALPHABET_PM7, train_loss="ranked", w_abs=0.1, block_waves=0):
        if direction not in (1, -1):
            raise ValueError("direction is +1 (harder) or -1 (easier)")
        self.mode = mode
        self.direction = direction
        self.alphabet = np.ascontiguousarray(alphabet, np.int8)
        self.chains, self.L, self.restarts, self.K, self.R = chains, L, restarts, K, R
        self.beta = _geometric(beta[0], beta[1], K)
        self.swap_interval, self.s_max, self.t_s, self.seed = swap_interval, s_max, t_s, seed
        self.proposals = 1 if mode == "plain" else proposals
        self.top = 1 if mode == "plain" else top
        self.train_steps, self.train_batch, self.lr = train_steps, train_batch, lr
        self.replay, self.screen_chunk = replay, screen_chunk
        if train_loss not in ("ranked", "plain"):
            raise ValueError("train_loss is 'ranked' or 'plain'")
        self.train_loss, self.w_abs = train_loss, float(w_abs)
        # wavefronts per PT workgroup (0: the library's choice); a launch
        # shape, so it changes no result and is not part of a checkpoint
        self.block_waves = int(block_waves)


def _key(J):
    return hashlib.sha1(np.ascontiguousarray(J, np.int8).tobytes()).hexdigest()


class _Pool:
    """What the chain groups of one search share: the surrogate, the replay
    buffer of PT-scored (J, ln TTS) records and the training draws.  A
    record of a scored proposal also keeps the instance it was made from and
    that instance's score (the chain's current state, scored on the same
    restart streams), for the ranked loss; a seed's record has none."""

    def __init__(self, cfg, surrogate_params):
        self.sur = Surrogate(surrogate_params) if cfg.mode == "surrogate" else None
        self.pairs_J, self.pairs_y = [], []
        self.parent_J, self.parent_y = [], []  # None / nan for records without a parent
        self.rng = np.random.default_rng(cfg.seed + 77)
        self.lock = threading.Lock()
        self.gnn_seconds = 0.0
        self.replay = cfg.replay

    def add(self, cands, ln, parents=None):
        """parents: (J, ln TTS) of each candidate's parent, or None."""
        with self.lock:
            for i, (cd, y) in enumerate(zip(cands, ln)):
                if math.isfinite(y):
                    self.pairs_J.append(np.array(cd["J"], np.int8))
                    self.pairs_y.append(float(y))
                    pj, py = parents[i] if parents is not None else (None, math.nan)
                    ok = pj is not None and math.isfinite(py)
                    self.parent_J.append(np.array(pj, np.int8) if ok else None)
                    self.parent_y.append(float(py) if ok else math.nan)
            if len(self.pairs_J) > self.replay:
                self.pairs_J = self.pairs_J[-self.replay:]
                self.pairs_y = self.pairs_y[-self.replay:]
                self.parent_J = self.parent_J[-self.replay:]
                self.parent_y = self.parent_y[-self.replay:]


class Search:
    """One search over `seeds`.  chain_ids (default 0..n-1) are the chains'
    global indices, which key every random draw; a group of a GroupedSearch
    passes its slice of them with the shared pool and the seeds' scores."""

    def __init__(self, cfg, seeds, surrogate_params=None, chain_ids=None, pool=None, ln=None, h0=None):
        self.cfg = cfg
        self.J = [np.array(s, np.int8) for s in seeds]
        self.ids = list(range(len(self.J))) if chain_ids is None else [int(i) for i in chain_ids]
        if len(self.ids) != len(self.J):
            raise ValueError("one chain id per seed")
        self.step = 0
        self.pt_seconds = 0.0
        self.pt_sweeps = 0
        self.pt_device_ms = 0.0   # summed device spans of the hardness_eval calls
        self.pt_attempts = 0      # spin-flip attempts they made
        self.pt_calls = 0
        self.pool = _Pool(cfg, surrogate_params) if pool is None else pool
        # training steps per step in proportion to the chains this search holds
        self.train_steps = max(1, round(cfg.train_steps * len(self.J) / cfg.chains))
        if ln is None:
            ln = self._score(self._seed_cands())
        self.ln = np.array(ln, np.float64)
        self.h0 = float(np.median(self.ln)) if h0 is None else float(h0)
        self.accepted = 0
        self.hard = {}
        self.hard_J = {}  # couplings of every counted state, by key
        self.decisions = []
        self.on_count = None  # called as on_count(key, J) once per newly counted state

    @property
    def gnn_seconds(self):
        return self.pool.gnn_seconds

    @property
    def sur(self):
        return self.pool.sur

    def _seed_cands(self):
        return [dict(L=self.cfg.L, J=J, live=None, instance_id=i) for i, J in zip(self.ids, self.J)]

    def _score(self, cands, keep=True, parents=None):
        """ln TTS of the candidates; keep=True adds them (with their parents)
        to the replay buffer."""
        c = self.cfg
        t0 = time.perf_counter()
        ln, det, ms, att = _timed_hardness(cands, c)
        self.pt_seconds += time.perf_counter() - t0
        self.pt_sweeps += sum(d["sweeps_total"] for d in det)
        self.pt_device_ms += ms
        self.pt_attempts += att
        self.pt_calls += 1
        if keep:
            self.pool.add(cands, ln, parents)
        return ln

    def _proposals(self, chain):
        c = self.cfg
        out = []
        for p in range(c.proposals):
            e, old, new, w = instance_mutate(dict(L=c.L, J=self.J[chain], live=None), c.alphabet, self.ids[chain],
                                             c.seed, self.step, p)
            J2 = self.J[chain].copy()
            J2[e] = new
            out.append((J2, w, p))
        return out

    def _rank(self, props):
        """Surrogate predictions for every (chain, proposal)."""
        c = self.cfg
        flat = [J for pr in props for (J, _, _) in pr]
        pool = self.pool
        pred = []
        with pool.lock, _gnn_context():  # every call ends with a host copy: nothing is left in flight
            t0 = time.perf_counter()
            for a in range(0, len(flat), c.screen_chunk):
                pred.append(pool.sur.forward([(c.L, None, J) for J in flat[a:a + c.screen_chunk]]))
            pool.gnn_seconds += time.perf_counter() - t0
        return np.concatenate(pred).reshape(len(props), c.proposals)

    def _train(self):
        c = self.cfg
        pool = self.pool
        if pool.sur is None:
            return
        with pool.lock, _gnn_context():
            t0 = time.perf_counter()
            if c.train_loss == "ranked":
                # batches of train_batch / 2 (parent, proposal) pairs: the
                # network learns how much one mutation changes ln TTS
                linked = [i for i, pj in enumerate(pool.parent_J) if pj is not None]
                half = c.train_batch // 2
                if len(linked) < half:
                    return
                ref = np.array([-1 if k % 2 == 0 else k - 1 for k in range(2 * half)], np.int32)  # parent, child
                for _ in range(self.train_steps):
                    idx = pool.rng.choice(len(linked), size=half, replace=False)
                    graphs, labels = [], []
                    for i in (linked[j] for j in idx):
                        graphs += [(c.L, None, pool.parent_J[i]), (c.L, None, pool.pairs_J[i])]
                        labels += [pool.parent_y[i], pool.pairs_y[i]]
                    pool.sur.train_step(np.array(labels), graphs=graphs, lr=c.lr, ref=ref, w_abs=c.w_abs)
            else:
                if len(pool.pairs_J) < c.train_batch:
                    return
                for _ in range(self.train_steps):
                    idx = pool.rng.choice(len(pool.pairs_J), size=c.train_batch, replace=False)
                    pool.sur.train_step(np.array([pool.pairs_y[i] for i in idx]),
                                        graphs=[(c.L, None, pool.pairs_J[i]) for i in idx], lr=c.lr)
            pool.gnn_seconds += time.perf_counter() - t0

    def _random_screen(self, chain):
        """The ablation's `top` proposals of one chain at this step, drawn from
        a generator keyed by (seed, step, global chain index)."""
        c = self.cfg
        g = np.random.default_rng([c.seed, 0x5C4EE7, self.step, self.ids[chain]])
        return sorted(g.choice(c.proposals, size=c.top, replace=False).tolist())

    def run_step(self, bars=(math.log(3.0), math.log(10.0), math.log(30.0))):
        c = self.cfg
        n = len(self.J)
        props = [self._proposals(ch) for ch in range(n)]
        if c.mode == "plain":
            chosen = [[0] for _ in range(n)]
        elif c.mode == "surrogate":
            pred = self._rank(props) * c.direction
            chosen = [sorted(np.argsort(-pred[ch], kind="stable")[:c.top].tolist()) for ch in range(n)]
        else:
            chosen = [self._random_screen(ch) for ch in range(n)]
        cands, owner, parents = [], [], []
        for ch in range(n):
            for p in chosen[ch]:
                J2, _, _ = props[ch][p]
                cands.append(dict(L=c.L, J=J2, live=None, instance_id=self.ids[ch]))
                owner.append((ch, p))
                parents.append((self.J[ch], float(self.ln[ch])))
        ln = self._score(cands, parents=parents)
        best = {}
        d = c.direction
        for (ch, p), y in zip(owner, ln):
            if ch not in best or d * y > d * best[ch][1]:  # ties keep the lower proposal index
                best[ch] = (p, y)
        for ch in range(n):
            p, y = best[ch]
            J2, w, _ = props[ch][p]
            ok = rao_accept(d * self.ln[ch], d * y, c.t_s, w)
            self.decisions.append((self.step, self.ids[ch], float(self.ln[ch]), float(y), int(w), bool(ok)))
            if ok:
                self.J[ch] = J2
                self.ln[ch] = y
                self.accepted += 1
                for b in bars:
                    if d * (y - self.h0) >= b:
                        k = _key(J2)
                        self.hard.setdefault(b, set()).add(k)
                        if k not in self.hard_J:
                            self.hard_J[k] = J2
                            if self.on_count is not None:
                                self.on_count(k, J2)
        self._train()
        self.step += 1


_STREAMS = {}
_STREAMS_LOCK = threading.Lock()
_GNN_CUS = 0  # compute units set aside for the surrogate's kernels (0: none)


def set_gnn_cus(n):
    """Sets aside the device's last n compute units for the surrogate: the
    streams made afterwards for chain groups and validation run their PT
    launches on the other CUs, and the surrogate's screen and training run
    on these n (0: every stream uses every CU).  A persistent PT launch
    holds each CU it reaches until its queue is empty, so without this the
    surrogate's small kernels wait for the other groups' launches to drain.
    Measured on the C8 search, the PT launches lose more on the remaining
    CUs than the surrogate gains, so the default is 0."""
    global _GNN_CUS
    _GNN_CUS = int(n)


def _stream(kind, i):
    import torch
    from . import cu_stream
    key = (kind, i, _GNN_CUS)
    with _STREAMS_LOCK:
        if key not in _STREAMS:
            if _GNN_CUS:
                n = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
                if not 0 < _GNN_CUS < n:
                    raise ValueError(f"cannot set aside {_GNN_CUS} of {n} CUs")
                _STREAMS[key] = cu_stream(n - _GNN_CUS, _GNN_CUS) if kind == "gnn" else cu_stream(0, n - _GNN_CUS)
            else:
                _STREAMS[key] = torch.cuda.Stream()
        return _STREAMS[key]


def _group_stream(i):
    """Stream i (default priority) and the context that makes it the calling
    thread's current one.  Streams are kept for the process: the caching
    allocator keeps freed blocks per stream, so a later search reuses the
    memory of an earlier one instead of allocating afresh while other
    groups' kernels run."""
    import torch
    s = _stream("pt", i)
    return s, torch.cuda.stream(s)


def _gnn_context():
    """Context for the surrogate's calls: its own stream on the CUs set aside
    by set_gnn_cus, else the caller's current stream."""
    import contextlib
    if not _GNN_CUS:
        return contextlib.nullcontext()
    import torch
    return torch.cuda.stream(_stream("gnn", 0))


def _in_groups(n, fn):
    """fn(i, failed) for i < n, each in a host thread on stream i; failed is
    set once any call raises, and the first exception is raised here."""
    errors = []
    failed = threading.Event()
    streams = [_group_stream(i) for i in range(n)]

    def work(i):
        stream, current = streams[i]
        try:
            with current:
                fn(i, failed)
            stream.synchronize()
        except BaseException as e:  # noqa: BLE001 - handed to the caller
            errors.append(e)
            failed.set()

    threads = [threading.Thread(target=work, args=(i,)) for i in range(n)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    if errors:
        raise errors[0]


class GroupedSearch:
    """The chains of one search in `groups` contiguous groups that step
    concurrently, each in a host thread with a stream of its own (default
    priority).  Groups beyond the process's hardware queues (4 by default)
    share a queue, and a launch then waits behind another's tail.  Each group scores its own seeds, concurrently; H0 is the
    median over all chains and the seeds enter the replay buffer in chain
    order, as in Search.  The attributes mirror Search's, merged over the
    groups; pt_seconds sums the groups' (overlapping) PT calls."""

    def __init__(self, cfg, seeds, groups=4, surrogate_params=None):
        n = len(seeds)
        if not 1 <= groups <= n:
            raise ValueError("need 1 <= groups <= chains")
        self.cfg = cfg
        self.pool = _Pool(cfg, surrogate_params)
        cuts = [round(g * n / groups) for g in range(groups + 1)]
        nan = np.full(n, np.nan)
        self.groups = [Search(cfg, seeds[a:b], chain_ids=range(a, b), pool=self.pool, ln=nan[a:b], h0=np.nan)
                       for a, b in zip(cuts[:-1], cuts[1:])]

        def score(i, failed):
            g = self.groups[i]
            g.ln = np.array(g._score(g._seed_cands(), keep=False), np.float64)

        _in_groups(groups, score)
        for g in self.groups:
            self.pool.add(g._seed_cands(), g.ln)
        self.h0 = float(np.median(self.ln))
        self.init_pt_seconds = max(g.pt_seconds for g in self.groups)
        self.init_pt_sweeps = sum(g.pt_sweeps for g in self.groups)
        for g in self.groups:
            g.h0 = self.h0
            g.pt_seconds, g.pt_sweeps, g.pt_device_ms, g.pt_attempts, g.pt_calls = 0.0, 0, 0.0, 0, 0

    def run(self, steps, bars=(math.log(3.0), math.log(10.0), math.log(30.0)), progress=None):
        """Every group takes `steps` steps; progress(group, step) is called
        after each.  The first failure of any group is raised here."""

        def walk(i, failed):
            g = self.groups[i]
            for _ in range(steps):
                if failed.is_set():
                    return
                g.run_step(bars)
                if progress is not None:
                    progress(i, g.step)

        _in_groups(len(self.groups), walk)

    def attach(self, validator):
        """Hand every newly counted state of every group to validator.submit
        (a Validator re-scoring them while the search runs)."""
        for g in self.groups:
            g.on_count = validator.submit

    @property
    def ln(self):
        return np.concatenate([g.ln for g in self.groups])

    @property
    def J(self):
        return [J for g in self.groups for J in g.J]

    @property
    def decisions(self):
        return sorted(d for g in self.groups for d in g.decisions)

    @property
    def hard(self):
        out = {}
        for g in self.groups:
            for b, keys in g.hard.items():
                out.setdefault(b, set()).update(keys)
        return out

    @property
    def hard_J(self):
        out = {}
        for g in self.groups:
            out.update(g.hard_J)
        return out

    @property
    def accepted(self):
        return sum(g.accepted for g in self.groups)

    @property
    def pt_seconds(self):
        return sum(g.pt_seconds for g in self.groups)

    @property
    def pt_sweeps(self):
        return sum(g.pt_sweeps for g in self.groups)

    @property
    def pt_device_ms(self):
        return sum(g.pt_device_ms for g in self.groups)

    @property
    def pt_attempts(self):
        return sum(g.pt_attempts for g in self.groups)

    @property
    def pt_calls(self):
        return sum(g.pt_calls for g in self.groups)

    @property
    def gnn_seconds(self):
        return self.pool.gnn_seconds


# ---------------------------------------------------------------------------
# Validation of counted states.  The search scores every candidate of a chain
# with the same restart streams (instance_id = the chain's index), a common
# random number choice that makes decisions reproducible and compares
# proposals on equal terms; but a state can then look hard only because these
# streams are slow on it.  Appendix B re-measures a final instance with many
# independent runs: here every counted state, and every seed instance (for
# H0), is scored again with VALIDATION_RESTARTS restarts whose Philox keys
# carry a second word (seed XOR VALIDATION_SEED_XOR) that no search stream
# uses, so the validation streams are disjoint from the search's.

VALIDATION_SEED_XOR = 0x7A11DA7E
VALIDATION_RESTARTS = 64


def validation_seed(cfg):
    return (int(cfg.seed) ^ VALIDATION_SEED_XOR) & 0xFFFFFFFF


def validation_id(key):
    """instance_id of a counted state in its validation run, from the key of
    its couplings: the same whichever order states are counted or validated
    in, and with the top bit set, so that no state shares the ids 0..n-1 of
    the n seeds."""
    return 0x80000000 | (int(key[:8], 16) & 0x7FFFFFFF)


def _fresh_scores(cands, c, restarts, seed_v):
    """hardness_eval of validation candidates on the current stream: (ln,
    confirmed, sweeps, spin-flip attempts, device ms)."""
    import torch
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    y, det = hardness_eval(cands, restarts, c.K, c.R, c.beta, c.swap_interval, c.s_max, seed_v, **_launch(c))
    end.record()
    end.synchronize()
    sweeps = sum(int(dd["sweeps_total"]) for dd in det)
    return ([float(v) for v in y], [bool(dd["confirmed"]) for dd in det], sweeps,
            sweeps * c.K * c.R * 8 * c.L * c.L, start.elapsed_time(end))


def _tally(h0v, fresh, bars, direction):
    """Validated count per bar: states whose fresh score is confirmed and
    clears H0' + bar (below H0' - bar for the reversed search)."""
    return {b: sum(1 for y, ok in fresh.values() if ok and direction * (y - h0v) >= b) for b in bars}


def validate(run, seeds, bars, restarts=VALIDATION_RESTARTS, chunk=256):
    """Re-scores the seed instances and every counted state of `run` (a
    Search or GroupedSearch) with independent restart streams, after the
    search.  A state is validated at bar b when its fresh ln TTS clears
    H0' + b (H0' = median fresh ln TTS of the seeds; below H0' - b for the
    reversed search) and its ground state is confirmed.  Returns a dict with
    H0', the validated counts per bar, the fresh scores and the seconds
    spent."""
    c = run.cfg
    states = run.hard_J
    keys = sorted(states)
    cands = [dict(L=c.L, J=np.asarray(J, np.int8), live=None, instance_id=i) for i, J in enumerate(seeds)]
    cands += [dict(L=c.L, J=states[k], live=None, instance_id=validation_id(k)) for k in keys]
    seed_v = validation_seed(c)
    t0 = time.perf_counter()
    ln, conf, sweeps, attempts, ms = [], [], 0, 0, 0.0
    for a in range(0, len(cands), chunk):
        y, ok, sw, att, t = _fresh_scores(cands[a:a + chunk], c, restarts, seed_v)
        ln += y
        conf += ok
        sweeps += sw
        attempts += att
        ms += t
    seconds = time.perf_counter() - t0
    h0v = float(np.median(ln[:len(seeds)]))
    fresh = {k: (ln[len(seeds) + i], conf[len(seeds) + i]) for i, k in enumerate(keys)}
    return dict(h0=h0v, counts=_tally(h0v, fresh, bars, c.direction), fresh=fresh, seconds=seconds,
                sweeps=sweeps, attempts=attempts, device_ms=ms, restarts=restarts, seed=seed_v,
                states=len(keys), overlapped=False)


class Validator:
    """validate() while the search runs.  A host thread on a stream of its
    own scores the seeds first, then takes the states the search counts as
    they arrive (GroupedSearch.attach or Search.on_count hand them over) and
    scores everything waiting, up to `chunk` states, in one hardness_eval
    call.  Its launches fill the chip while the search's launches wait for
    their slowest restarts.  Every state keeps the instance id validate()
    gives it, and a candidate's score does not depend on the launch it
    shares, so finish() returns what validate() returns for the same states,
    with `seconds` the time finish() waited for the last launches."""

    def __init__(self, cfg, seeds, restarts=VALIDATION_RESTARTS, chunk=256, stream_index=0):
        self.cfg = cfg
        self.restarts = restarts
        self.chunk = chunk
        self.seed = validation_seed(cfg)
        self._seeds = [np.array(J, np.int8) for J in seeds]
        self._queue = queue.Queue()
        self._seen = set()
        self._lock = threading.Lock()
        self._error = None
        self.fresh = {}
        self.h0 = None
        self.sweeps = 0
        self.attempts = 0
        self.device_ms = 0.0
        self.calls = 0
        self._stream = _group_stream(stream_index)  # made here: the list of streams is not thread-safe
        self._thread = threading.Thread(target=self._run, daemon=True)
        self._thread.start()

    def submit(self, key, J):
        """Queue one counted state (called from any search thread)."""
        with self._lock:
            if key in self._seen:
                return
            self._seen.add(key)
        self._queue.put((key, np.array(J, np.int8)))

    def _score(self, cands):
        y, ok, sw, att, ms = _fresh_scores(cands, self.cfg, self.restarts, self.seed)
        self.sweeps += sw
        self.attempts += att
        self.device_ms += ms
        self.calls += 1
        return y, ok

    def _run(self):
        stream, current = self._stream
        c = self.cfg
        try:
            with current:
                y, _ = self._score([dict(L=c.L, J=J, live=None, instance_id=i) for i, J in enumerate(self._seeds)])
                self.h0 = float(np.median(y))
                done = False
                while not done:
                    batch = [self._queue.get()]
                    while len(batch) < self.chunk and batch[-1] is not None:
                        try:
                            batch.append(self._queue.get_nowait())
                        except queue.Empty:
                            break
                    if batch[-1] is None:
                        batch.pop()
                        done = True
                    if batch:
                        y, ok = self._score([dict(L=c.L, J=J, live=None, instance_id=validation_id(k))
                                             for k, J in batch])
                        for (k, _), v, conf in zip(batch, y, ok):
                            self.fresh[k] = (v, conf)
            stream.synchronize()
        except BaseException as e:  # noqa: BLE001 - raised by finish()
            self._error = e

    def finish(self, bars):
        """Waits for every queued state and returns validate()'s dict."""
        t0 = time.perf_counter()
        self._queue.put(None)
        self._thread.join()
        seconds = time.perf_counter() - t0
        if self._error is not None:
            raise self._error
        return dict(h0=self.h0, counts=_tally(self.h0, self.fresh, bars, self.cfg.direction),
                    fresh=dict(self.fresh), seconds=seconds, sweeps=self.sweeps, attempts=self.attempts,
                    device_ms=self.device_ms, restarts=self.restarts, seed=self.seed, states=len(self.fresh),
                    overlapped=True, calls=self.calls)


class LaoSearch:
    """Loop Adaptive Optimization (Sec. IV, Algorithm 2) on planted-solution
    instances: every chain starts from lao_init's instance of n_loops
    frustrated loops; a step replaces one loop (lao_move), scores the
    candidate with hardness_eval and accepts by Metropolis in ln TTS
    (hs_rao_accept).  The planted ground-state energy travels with the
    instance; `gs_found` counts scored candidates whose PT ground state
    (minimum over restarts) reached it, `voids` counts proposals with no
    replacement loop under the coupling cap (kept as rejected moves), and
    `decisions` logs (step, chain, ln_cur, ln_new, w, accepted)."""

    def __init__(self, cfg, n_loops, seed_chain0=0, score=True):
        from . import lao_init
        self.cfg = cfg
        self.n_loops = n_loops
        self.inst = [lao_init(cfg.L, n_loops, seed_chain0 + ch, cfg.seed) for ch in range(cfg.chains)]
        self.chain_id = [seed_chain0 + ch for ch in range(cfg.chains)]
        self.step = 0
        self.pt_seconds = 0.0
        self.pt_sweeps = 0
        self.pt_device_ms = 0.0
        self.pt_attempts = 0
        self.pt_calls = 0
        self.scored = 0
        self.gs_found = 0
        self.accepted = 0
        self.voids = 0
        self.decisions = []
        self.ln = self.ln0 = None
        if score:
            self.score_initial()

    def score_initial(self):
        self.ln = self._score([(ch, i["J"], i["e_gs"]) for ch, i in enumerate(self.inst)])
        self.ln0 = self.ln.copy()

    def _score(self, cands):
        c = self.cfg
        t0 = time.perf_counter()
        ln, det, ms, att = _timed_hardness(
            [dict(L=c.L, J=J, live=None, instance_id=self.chain_id[ch]) for ch, J, _ in cands], c)
        self.pt_seconds += time.perf_counter() - t0
        self.pt_sweeps += sum(d["sweeps_total"] for d in det)
        self.pt_device_ms += ms
        self.pt_attempts += att
        self.pt_calls += 1
        for (_, _, e_gs), d in zip(cands, det):
            self.scored += 1
            self.gs_found += int(d["e_gs"] == e_gs)
        return np.asarray(ln, np.float64)

    def run_step(self):
        from . import lao_move
        c = self.cfg
        moves = [lao_move(c.L, self.inst[ch], self.chain_id[ch], c.seed, self.step, 0) for ch in range(c.chains)]
        live = [ch for ch, m in enumerate(moves) if m[0] >= 0]  # void proposals are rejected moves
        scores = self._score([(ch, moves[ch][3], moves[ch][4]) for ch in live]) if live else []
        ln = dict(zip(live, scores))
        for ch, (slot, lp, w, J2, e2) in enumerate(moves):
            if slot < 0:
                self.voids += 1
                continue
            ok = rao_accept(self.ln[ch], ln[ch], c.t_s, w)
            self.decisions.append((self.step, self.chain_id[ch], float(self.ln[ch]), float(ln[ch]), int(w),
                                   bool(ok)))
            if ok:
                inst = self.inst[ch]
                inst["loops"] = inst["loops"].copy()
                inst["loops"][slot] = lp
                inst["J"] = J2
                inst["e_gs"] = e2
                self.ln[ch] = ln[ch]
                self.accepted += 1
        self.step += 1


class GroupedLao:
    """LaoSearch's chains in `groups` contiguous groups stepping concurrently
    on their own streams, as GroupedSearch does for Algorithm 1.  Chains
    keep their global indices (planted instances, moves and PT streams are
    keyed by them), so every decision is the one-group search's."""

    def __init__(self, cfg, n_loops, groups=4):
        import copy
        n = cfg.chains
        if not 1 <= groups <= n:
            raise ValueError("need 1 <= groups <= chains")
        self.cfg = cfg
        cuts = [round(g * n / groups) for g in range(groups + 1)]
        self.groups = []
        for a, b in zip(cuts[:-1], cuts[1:]):
            cg = copy.copy(cfg)
            cg.chains = b - a
            self.groups.append(LaoSearch(cg, n_loops, seed_chain0=a, score=False))
        _in_groups(groups, lambda i, failed: self.groups[i].score_initial())
        self.init_pt_seconds = max(g.pt_seconds for g in self.groups)

    def run(self, steps, progress=None):
        def walk(i, failed):
            g = self.groups[i]
            for _ in range(steps):
                if failed.is_set():
                    return
                g.run_step()
                if progress is not None:
                    progress(i, g.step)

        _in_groups(len(self.groups), walk)

    def _sum(self, name):
        return sum(getattr(g, name) for g in self.groups)

    ln = property(lambda self: np.concatenate([g.ln for g in self.groups]))
    ln0 = property(lambda self: np.concatenate([g.ln0 for g in self.groups]))
    inst = property(lambda self: [i for g in self.groups for i in g.inst])
    decisions = property(lambda self: sorted(d for g in self.groups for d in g.decisions))
    accepted = property(lambda self: self._sum("accepted"))
    scored = property(lambda self: self._sum("scored"))
    gs_found = property(lambda self: self._sum("gs_found"))
    voids = property(lambda self: self._sum("voids"))
    pt_seconds = property(lambda self: self._sum("pt_seconds"))
    pt_sweeps = property(lambda self: self._sum("pt_sweeps"))
    pt_device_ms = property(lambda self: self._sum("pt_device_ms"))
    pt_attempts = property(lambda self: self._sum("pt_attempts"))
    pt_calls = property(lambda self: self._sum("pt_calls"))


# ---------------------------------------------------------------------------
# Checkpoint and resume.  A search is saved between whole steps: the chains'
# couplings, ln TTS, the step, the counted states, the decision log and the
# shared pool (replay buffer, training draws, surrogate weights and Adam
# state).  Every other draw is keyed by (seed, step, chain), so nothing else
# is needed to continue exactly.  The file is a numpy archive without pickled
# objects, written to a temporary name and renamed, so a process killed while
# saving leaves the previous checkpoint intact.

_CKPT_VERSION = 3
_CFG_KEYS = ("mode", "direction", "chains", "L", "restarts", "K", "R", "swap_interval", "s_max", "t_s", "seed",
             "proposals", "top", "train_steps", "train_batch", "lr", "replay", "train_loss", "w_abs")


def _cfg_record(cfg):
    rec = {k: getattr(cfg, k) for k in _CFG_KEYS}
    rec["beta"] = [float(b) for b in cfg.beta]
    rec["alphabet"] = [int(a) for a in cfg.alphabet]
    return rec


def save_search(run, path):
    """Checkpoint of a Search or GroupedSearch (all groups at the same step)."""
    import json
    import os
    groups = run.groups if isinstance(run, GroupedSearch) else [run]
    steps = {g.step for g in groups}
    if len(steps) != 1:
        raise ValueError("groups are at different steps")
    pool = groups[0].pool
    cfg = groups[0].cfg
    hard = {}
    for g in groups:
        for b, keys in g.hard.items():
            hard.setdefault(repr(float(b)), set()).update(keys)
    dec = sorted(d for g in groups for d in g.decisions)
    meta = {"version": _CKPT_VERSION, "cfg": _cfg_record(cfg), "step": steps.pop(),
            "h0": groups[0].h0, "accepted": sum(g.accepted for g in groups),
            "hard": {b: sorted(k) for b, k in hard.items()},
            "rng": pool.rng.bit_generator.state, "sur_step": pool.sur.step if pool.sur is not None else 0}
    arrays = {
        "ids": np.array([i for g in groups for i in g.ids], np.int64),
        "J": np.stack([J for g in groups for J in g.J]).astype(np.int8),
        "ln": np.concatenate([g.ln for g in groups]).astype(np.float64),
        "decisions": np.array([[d[0], d[1], d[2], d[3], d[4], float(d[5])] for d in dec], np.float64).reshape(-1, 6),
        "pairs_J": (np.stack(pool.pairs_J).astype(np.int8) if pool.pairs_J
                    else np.zeros((0, len(groups[0].J[0])), np.int8)),
        "pairs_y": np.array(pool.pairs_y, np.float64),
        "parent_J": (np.stack([np.zeros_like(J) if pj is None else pj for pj, J in zip(pool.parent_J, pool.pairs_J)])
                     .astype(np.int8) if pool.pairs_J else np.zeros((0, len(groups[0].J[0])), np.int8)),
        "parent_y": np.array(pool.parent_y, np.float64),
    }
    hard_J = {}
    for g in groups:
        hard_J.update(g.hard_J)
    hk = sorted(hard_J)
    meta["hard_J_keys"] = hk
    arrays["hard_J"] = (np.stack([hard_J[k] for k in hk]).astype(np.int8) if hk
                        else np.zeros((0, len(groups[0].J[0])), np.int8))
    if pool.sur is not None:
        arrays["sur_params"] = pool.sur.params.cpu().numpy()
        arrays["sur_m"] = pool.sur.m.cpu().numpy()
        arrays["sur_v"] = pool.sur.v.cpu().numpy()
    arrays["meta"] = np.frombuffer(json.dumps(meta).encode(), np.uint8)
    tmp = path + ".tmp.npz"
    np.savez(tmp, **arrays)
    os.replace(tmp, path)


def load_search(path, cfg, groups=1):
    """Resume a checkpoint as a Search (groups = 1) or a GroupedSearch.  cfg
    must equal the saved configuration; the grouping may differ, since no
    decision depends on it."""
    import json
    with np.load(path, allow_pickle=False) as z:
        a = {k: z[k] for k in z.files}
    meta = json.loads(a["meta"].tobytes().decode())
    if meta["version"] != _CKPT_VERSION:
        raise ValueError("unknown checkpoint version")
    if meta["cfg"] != json.loads(json.dumps(_cfg_record(cfg))):
        raise ValueError("checkpoint was written with another search configuration")
    n = len(a["ids"])
    if not 1 <= groups <= n:
        raise ValueError("need 1 <= groups <= chains")
    pool = _Pool(cfg, a["sur_params"] if "sur_params" in a else None)
    pool.pairs_J = [row.copy() for row in a["pairs_J"]]
    pool.pairs_y = [float(y) for y in a["pairs_y"]]
    pool.parent_y = [float(y) for y in a["parent_y"]]
    pool.parent_J = [row.copy() if math.isfinite(y) else None for row, y in zip(a["parent_J"], pool.parent_y)]
    pool.rng.bit_generator.state = meta["rng"]
    if pool.sur is not None:
        torch = pool.sur.torch
        pool.sur.m.copy_(torch.from_numpy(a["sur_m"]))
        pool.sur.v.copy_(torch.from_numpy(a["sur_v"]))
        pool.sur.step = int(meta["sur_step"])
    cuts = [round(g * n / groups) for g in range(groups + 1)]
    parts = []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        g = Search(cfg, [a["J"][i] for i in range(lo, hi)], chain_ids=a["ids"][lo:hi].tolist(), pool=pool,
                   ln=a["ln"][lo:hi], h0=meta["h0"])
        g.step = int(meta["step"])
        parts.append(g)
    owner = {int(i): g for g in parts for i in g.ids}
    for row in a["decisions"]:
        d = (int(row[0]), int(row[1]), float(row[2]), float(row[3]), int(row[4]), bool(row[5]))
        owner[d[1]].decisions.append(d)
    parts[0].accepted = int(meta["accepted"])
    parts[0].hard = {float(b): set(keys) for b, keys in meta["hard"].items()}
    parts[0].hard_J = {k: a["hard_J"][i].copy() for i, k in enumerate(meta["hard_J_keys"])}
    if groups == 1:
        return parts[0]
    run = GroupedSearch.__new__(GroupedSearch)
    run.cfg, run.pool, run.groups, run.h0 = cfg, pool, parts, float(meta["h0"])
    run.init_pt_seconds, run.init_pt_sweeps = 0.0, 0
    return run
