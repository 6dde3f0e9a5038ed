"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws inputs (couplings, missing-spin masks, sizes, ladders);
it holds none of the method's arithmetic, so both the CPU oracle and the GPU
library can be fed from it without sharing any code with each other.

The paper's own instances (the RAO hardness groups, the hardest instance and
the DW2 dead-qubit map) are not available, so every workload is synthetic:
Chimera C_L couplings drawn uniformly from a fixed alphabet with numpy's
PCG64 seeded by (seed, instance index), and missing qubits drawn uniformly
without replacement.
"""
import numpy as np

ALPHABETS = {
    "pm1": np.array([-1, 1], np.int8),
    "pm3": np.array([-3, -2, -1, 1, 2, 3], np.int8),
    "pm7": np.array([-7, -6, -5, -4, -3, -2, -1, 1, 2, 3, 4, 5, 6, 7], np.int8),
}


def num_sites(L):
    return 8 * L * L


def num_edges(L):
    """Couplers of the full Chimera C_L: 16 per K_{4,4} cell plus 4 per
    neighbouring cell pair."""
    return 16 * L * L + 8 * L * (L - 1)


def rng(seed, index):
    return np.random.default_rng([int(seed), int(index)])


def couplings(L, alphabet, seed, index):
    """J over the full canonical edge list of C_L, uniform over `alphabet`."""
    a = ALPHABETS[alphabet] if isinstance(alphabet, str) else np.asarray(alphabet, np.int8)
    g = rng(seed, index)
    return a[g.integers(0, len(a), size=num_edges(L))].astype(np.int8)


def missing_mask(L, frac, seed, index):
    """uint8 live mask with exactly round(frac * N) sites removed (None if frac == 0)."""
    N = num_sites(L)
    n_dead = int(round(frac * N))
    if n_dead == 0:
        return None
    g = rng(seed + 7919, index)
    live = np.ones(N, np.uint8)
    live[g.choice(N, size=n_dead, replace=False)] = 0
    return live


def geometric_betas(beta_min, beta_max, K):
    """Inverse temperatures beta_k = beta_min (beta_max / beta_min)^(k / (K-1)), ascending."""
    if K == 1:
        return np.array([beta_min], np.float64)
    k = np.arange(K, dtype=np.float64)
    return beta_min * (beta_max / beta_min) ** (k / (K - 1))


def random_spins(N, lanes, seed, index):
    """Word-major uint64 spins: bit l of word i is lane l's spin bit at site i."""
    g = rng(seed + 104729, index)
    lo = g.integers(0, 2 ** 32, size=N, dtype=np.uint64)
    hi = g.integers(0, 2 ** 32, size=N, dtype=np.uint64)
    w = (hi << np.uint64(32)) | lo
    if lanes < 64:
        w &= np.uint64((1 << lanes) - 1)
    return w


def gauge_vector(N, seed):
    """Random +-1 gauge (as spin bits, 1 <-> -1) for the gauge-invariance test."""
    return rng(seed + 15485863, 0).integers(0, 2, size=N).astype(np.uint8)


# The five workloads.  Names describe what they are; sizes are the full sizes.
def parity_c4():
    """One C4 instance, J in {-1,+1}, K = 16 (beta 0.2..3.0), R = 1, 10^4 sweeps."""
    return dict(name="C4 x1, K16 R1, +-1", L=4, alphabet="pm1", seed=1605, n_inst=1,
                K=16, R=1, beta=(0.2, 3.0), sweeps=10_000, swap_interval=1, missing=0.0)


def batch_c8():
    """256 C8 instances, J in {+-1..+-7}, K = 32 (beta 0.1..5.0) x R = 2, 10^5 sweeps,
    an exchange pass after every sweep.  (The elementary Monte Carlo step of
    Sec. III.B, 10 sweeps per exchange pass, is swap_interval = 10.)"""
    return dict(name="C8 x256, K32 R2, +-7", L=8, alphabet="pm7", seed=1605, n_inst=256,
                K=32, R=2, beta=(0.1, 5.0), sweeps=100_000, swap_interval=1, missing=0.0)


def uneven_batch(n_inst=1024, seed=1606):
    """1024 instances, L ~ U{4..12}, 2% missing spins, J in {+-1,+-2,+-3},
    K ~ U{24..48}, R = 1, beta 0.1..5.0."""
    g = rng(seed, 999_999)
    Ls = g.integers(4, 13, size=n_inst)
    Ks = g.integers(24, 49, size=n_inst)
    insts = []
    for n in range(n_inst):
        L = int(Ls[n])
        insts.append(dict(L=L, J=couplings(L, "pm3", seed, n), live=missing_mask(L, 0.02, seed, n),
                          K=int(Ks[n]), R=1, beta=geometric_betas(0.1, 5.0, int(Ks[n])),
                          instance_id=n))
    return dict(name=f"uneven x{n_inst}, C4..C12, 2% missing, K24..48 R1, +-3",
                seed=seed, sweeps=100_000, swap_interval=1, instances=insts)


def make_batch(cfg, n_inst=None):
    """Materialises a uniform-size workload as a list of instance dicts."""
    n = cfg["n_inst"] if n_inst is None else n_inst
    beta = geometric_betas(cfg["beta"][0], cfg["beta"][1], cfg["K"])
    out = []
    for i in range(n):
        out.append(dict(L=cfg["L"], J=couplings(cfg["L"], cfg["alphabet"], cfg["seed"], i),
                        live=missing_mask(cfg["L"], cfg["missing"], cfg["seed"], i),
                        K=cfg["K"], R=cfg["R"], beta=beta, instance_id=i))
    return out


def search_seeds(n_chains=64, L=8, seed=2016):
    """Random +-1 seed instances for the instance-hardness search (Algorithm 1)."""
    return [couplings(L, "pm1", seed, c) for c in range(n_chains)]


def gnn_params(n_params, fan_ins, seed=1605):
    """Initial surrogate weights: uniform in +-sqrt(6 / (fan_in + 64)) per
    block (fan_ins: list of (size, fan_in), fan_in 0 = zeros), float32."""
    g = rng(seed, 777_777)
    out = np.zeros(n_params, np.float32)
    o = 0
    for size, fan_in in fan_ins:
        if fan_in > 0:
            a = np.sqrt(6.0 / (fan_in + 64))
            out[o:o + size] = g.uniform(-a, a, size).astype(np.float32)
        o += size
    assert o == n_params
    return out
