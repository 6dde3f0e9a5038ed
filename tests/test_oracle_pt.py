"""Pins for the oracle's parallel tempering (Sec. II; Sec. III.B): Boltzmann
statistics against brute-force enumeration, limits with closed-form results,
the checkerboard order contract, checkpoint/resume, and energy bookkeeping."""
import numpy as np
import pytest
from scipy import stats

import oracle
import workloads

SEED = 77


def _one_cell_instance(seed=3):
    L = 1
    return L, None, workloads.couplings(L, "pm3", seed, 0)


def _state_index(spins, lane):
    """Configuration of `lane` at the 8 sites of a one-cell instance, as an
    integer whose bit n is the spin bit of site n."""
    bits = (spins >> np.uint64(lane)) & np.uint64(1)
    return int(np.sum(bits.astype(np.int64) << np.arange(len(spins))))


def _chi2_pvalue(counts, probs):
    """Pearson chi^2 over bins with expected count >= 5 (rest pooled)."""
    exp = probs * counts.sum()
    big = exp >= 5
    obs = np.append(counts[big], counts[~big].sum())
    e = np.append(exp[big], exp[~big].sum())
    keep = e > 0
    obs, e = obs[keep], e[keep]
    chi2 = float(((obs - e) ** 2 / e).sum())
    return stats.chi2.sf(chi2, len(obs) - 1)


def _boltzmann(en, beta):
    w = np.exp(-beta * (en - en.min()))
    return w / w.sum()


@pytest.mark.parametrize("beta", [0.25, 0.8])
def test_single_temperature_metropolis_samples_boltzmann(beta):
    """64 independent Metropolis chains (K = 1, R = 64) on one K_{4,4} cell:
    the histogram over the 256 configurations matches exp(-beta E)/Z."""
    L, live, J = _one_cell_instance()
    _, _, en = oracle.enumerate_states(L, live, J, want_energies=True)
    probs = _boltzmann(en.astype(np.float64), beta)
    K, R = 1, 64
    st = oracle.pt_init(L, live, J, K, R, 11, SEED)
    betas = np.array([beta])
    counts = np.zeros(256, np.int64)
    oracle.pt_run(L, live, J, K, R, betas, 11, SEED, 0, 20, st)  # burn-in
    for _ in range(600):
        oracle.pt_run(L, live, J, K, R, betas, 11, SEED, 0, 2, st)
        for lane in range(64):
            counts[_state_index(st.spins, lane)] += 1
    # A single-temperature chain crosses between a configuration and its
    # global spin flip (equal weight, Eq. 1 has no fields) only slowly at low
    # temperature, so compare over flip classes {s, ~s}.
    idx = np.arange(128)
    folded = counts[idx] + counts[255 - idx]
    p = _chi2_pvalue(folded, probs[idx] + probs[255 - idx])
    assert p > 1e-4, p


def test_parallel_tempering_marginals_are_boltzmann():
    """PT with K = 4 temperatures and 16 replica sets on one cell, exchanges
    every sweep: the configuration held at each temperature slot follows the
    Boltzmann distribution of that slot's beta (detailed balance of both
    the Metropolis and the exchange moves)."""
    L, live, J = _one_cell_instance(seed=8)
    _, _, en = oracle.enumerate_states(L, live, J, want_energies=True)
    K, R = 4, 16
    betas = workloads.geometric_betas(0.2, 1.5, K)
    st = oracle.pt_init(L, live, J, K, R, 5, SEED)
    oracle.pt_run(L, live, J, K, R, betas, 5, SEED, 1, 20, st)
    counts = np.zeros((K, 256), np.int64)
    for _ in range(500):
        oracle.pt_run(L, live, J, K, R, betas, 5, SEED, 1, 2, st)
        for k in range(K):
            for r in range(R):
                counts[k, _state_index(st.spins, int(st.perm[k * R + r]))] += 1
    for k in range(K):
        p = _chi2_pvalue(counts[k], _boltzmann(en.astype(np.float64), betas[k]))
        assert p > 1e-4, (k, p)
    assert st.swap_acc.sum() > 0


def test_infinite_temperature_limit_flips_everything():
    """As beta -> 0 every Metropolis move is accepted (min(1, e^0) = 1), so a
    full sweep flips every live spin of every lane."""
    L = 2
    J = workloads.couplings(L, "pm7", 4, 0)
    live = workloads.missing_mask(L, 0.1, 4, 0)
    K, R = 2, 3
    st = oracle.pt_init(L, live, J, K, R, 9, SEED)
    before = st.spins.copy()
    oracle.pt_run(L, live, J, K, R, np.array([1e-13, 2e-13]), 9, SEED, 0, 1, st)
    mask = np.uint64((1 << (K * R)) - 1)
    lv = np.ones(8 * L * L, bool) if live is None else live.astype(bool)
    assert np.all(st.spins[lv] == (before[lv] ^ mask))
    assert np.all(st.spins[~lv] == 0)


def test_zero_temperature_quench_never_goes_uphill():
    """At very large beta no uphill move is accepted: every lane's energy is
    non-increasing sweep by sweep, and ends in a local minimum."""
    L = 3
    J = workloads.couplings(L, "pm7", 6, 0)
    K, R = 2, 8
    betas = np.array([40.0, 50.0])
    st = oracle.pt_init(L, None, J, K, R, 2, SEED)
    prev = st.energy.copy()
    for _ in range(30):
        oracle.pt_run(L, None, J, K, R, betas, 2, SEED, 0, 1, st)
        assert np.all(st.energy[:K * R] <= prev[:K * R])
        prev = st.energy.copy()


def test_incremental_energy_matches_recomputed():
    L = 4
    J = workloads.couplings(L, "pm7", 1, 0)
    live = workloads.missing_mask(L, 0.03, 1, 0)
    K, R = 8, 4
    betas = workloads.geometric_betas(0.1, 3.0, K)
    st = oracle.pt_init(L, live, J, K, R, 17, SEED)
    assert np.array_equal(st.energy, oracle.lane_energies(L, live, J, K * R, st.spins))
    oracle.pt_run(L, live, J, K, R, betas, 17, SEED, 1, 200, st)
    assert np.array_equal(st.energy, oracle.lane_energies(L, live, J, K * R, st.spins))
    # emin per replica set equals the minimum lane energy ever seen; at least
    # not above the current minimum
    for r in range(R):
        assert st.emin[r] <= st.energy[r * K:(r + 1) * K].min()


def test_site_order_within_colour_is_irrelevant():
    """Same-colour sites share no edge, so any visiting order inside a colour
    phase gives identical trajectories (the checkerboard contract)."""
    L = 4
    J = workloads.couplings(L, "pm7", 2, 0)
    K, R = 8, 2
    betas = workloads.geometric_betas(0.2, 3.0, K)
    a = oracle.pt_init(L, None, J, K, R, 3, SEED)
    b = a.copy()
    oracle.pt_run(L, None, J, K, R, betas, 3, SEED, 1, 300, a)
    order = np.random.default_rng(0).permutation(8 * L * L).astype(np.int32)
    oracle.pt_run(L, None, J, K, R, betas, 3, SEED, 1, 300, b, site_order=order)
    for name in ("spins", "perm", "energy", "emin", "thit", "swap_acc", "t"):
        assert np.array_equal(getattr(a, name), getattr(b, name)), name


def test_checkpoint_resume_is_bit_exact():
    L = 3
    J = workloads.couplings(L, "pm7", 3, 0)
    K, R = 16, 4
    betas = workloads.geometric_betas(0.1, 5.0, K)
    a = oracle.pt_init(L, None, J, K, R, 4, SEED)
    b = a.copy()
    oracle.pt_run(L, None, J, K, R, betas, 4, SEED, 3, 400, a)
    oracle.pt_run(L, None, J, K, R, betas, 4, SEED, 3, 150, b)
    oracle.pt_run(L, None, J, K, R, betas, 4, SEED, 3, 250, b)
    for name in ("spins", "perm", "energy", "emin", "thit", "swap_acc", "t"):
        assert np.array_equal(getattr(a, name), getattr(b, name)), name


def test_philox_initial_state_is_balanced_and_buffer_init_is_exact():
    L = 4
    J = workloads.couplings(L, "pm1", 5, 0)
    K, R = 16, 4
    st = oracle.pt_init(L, None, J, K, R, 8, SEED)
    bits = np.unpackbits(st.spins.view(np.uint8)).mean()
    assert abs(bits - 0.5) < 0.03
    init = workloads.random_spins(8 * L * L, K * R, 3, 0)
    st2 = oracle.pt_init(L, None, J, K, R, 8, SEED, init_spins=init)
    assert np.array_equal(st2.spins, init)
    assert np.array_equal(st2.perm, np.array([r * K + k for k in range(K) for r in range(R)],
                                             np.uint8))


def test_gauge_transformed_trajectories_are_gauge_images():
    """The draws depend on neither J nor the spins and every dE and exchange
    d is gauge invariant, so (J', s0') = (gJg, g.s0) yields s'(t) = g.s(t)
    with identical energies and slot permutations."""
    L = 4
    N = 8 * L * L
    J = workloads.couplings(L, "pm7", 12, 0)
    live = workloads.missing_mask(L, 0.03, 12, 0)
    ei, ej = oracle.edges(L)
    g = workloads.gauge_vector(N, 12)
    sg = 1 - 2 * g.astype(np.int64)
    Jg = (J * sg[ei] * sg[ej]).astype(np.int8)
    K, R = 8, 8
    lanes = K * R
    betas = workloads.geometric_betas(0.2, 3.0, K)
    s0 = workloads.random_spins(N, lanes, 12, 0)
    gw = np.where(g == 1, np.uint64((1 << 64) - 1), np.uint64(0)).astype(np.uint64)
    a = oracle.pt_init(L, live, J, K, R, 6, SEED, init_spins=s0)
    b = oracle.pt_init(L, live, Jg, K, R, 6, SEED, init_spins=s0 ^ gw)
    oracle.pt_run(L, live, J, K, R, betas, 6, SEED, 1, 150, a)
    oracle.pt_run(L, live, Jg, K, R, betas, 6, SEED, 1, 150, b)
    lv = np.ones(N, bool) if live is None else live.astype(bool)
    assert np.array_equal(a.spins[lv] ^ gw[lv], b.spins[lv])
    for name in ("perm", "energy", "emin", "thit", "swap_acc"):
        assert np.array_equal(getattr(a, name), getattr(b, name)), name
