"""Pins of the oracle against what the paper and the mathematics fix, written
independently of the oracle's own code:

  * time-to-solution and the agreement stop (Appendix B, Sec. III.B):
    closed forms for free couplings, and a zero-temperature limit in which
    every trajectory is a deterministic greedy descent, recomputed here from
    the definitions (Chimera graph of Appendix A, Eq. 1, the checkerboard
    order, the stop rule, TTS = restart sweeps per restart reaching E_gs);
  * Metropolis and exchange thresholds within 2^-32 of the exact
    exponentials (Sec. II: acceptance probabilities min(1, e^{-beta dE}) and
    the detailed-balance exchange ratio), the exponentials evaluated in
    50-digit decimal arithmetic, not with libm;
  * Boltzmann statistics on the two-cell (16-spin) graph, and the joint
    distribution of (temperature slot, configuration) under parallel
    tempering: stationary product of Boltzmann marginals (Sec. II, detailed
    balance), against brute-force enumeration;
  * the RAO move (Algorithm 1): one coupler drawn uniformly among the live
    ones, its new value uniform over the other letters of the alphabet;
  * the surrogate oracle's forward and backward pass against torch autograd.
"""
import decimal
import math

import numpy as np
import pytest
from scipy import stats

import oracle
import workloads

SEED = 91


# ---------------------------------------------------------------------------
# Chimera graph and energies written from the definitions (Appendix A, Eq. 1)
def _chimera(L):
    def sid(r, c, u, k):
        return 8 * (L * r + c) + 4 * u + k

    edges = []
    for r in range(L):
        for c in range(L):
            edges += [(sid(r, c, 0, a), sid(r, c, 1, b)) for a in range(4) for b in range(4)]
            for k in range(4):
                if r + 1 < L:
                    edges.append((sid(r, c, 0, k), sid(r + 1, c, 0, k)))
                if c + 1 < L:
                    edges.append((sid(r, c, 1, k), sid(r, c + 1, 1, k)))
    edges.sort()
    return np.array(edges, np.int64)


def _colour(L, N):
    i = np.arange(N)
    cell = i // 8
    return ((cell // L) + (cell % L) + (i // 4) % 2) % 2


def _coupling_matrix(L, live, J):
    N = 8 * L * L
    E = _chimera(L)
    lv = np.ones(N, bool) if live is None else np.asarray(live, bool)
    M = np.zeros((N, N), np.int64)
    for (a, b), j in zip(E, np.asarray(J, np.int64)):
        if lv[a] and lv[b]:
            M[a, b] = M[b, a] = j
    return M, lv


def _philox_bit(ctr, key, word):
    return int(oracle.philox(ctr, key)[word]) >> 31


def _greedy_restart(L, live, J, K, R, key, seed, s_max):
    """Zero-temperature PT restart: every uphill move is rejected (its
    threshold floor(2^32 e^{-beta dE}) is 0 at these betas), so sweep t is a
    checkerboard greedy descent (flip iff dE <= 0) in every lane, whatever
    slot it sits at; the running minimum of a replica set is over its lanes.
    Returns (per-set minima, per-set first-hit sweeps, sweeps run)."""
    M, lv = _coupling_matrix(L, live, J)
    N = M.shape[0]
    col = _colour(L, N)
    lanes = K * R
    s = np.ones((lanes, N), np.int64)
    for r in range(R):
        for k in range(K):
            for i in range(N):
                if lv[i] and _philox_bit([0, i // 4, (k << 8) | r, 2], [key, seed], i % 4):
                    s[r * K + k, i] = -1

    def energies():
        return ((s @ M) * s).sum(axis=1) // 2

    e = energies()
    emin = [int(e[r * K:(r + 1) * K].min()) for r in range(R)]
    thit = [0] * R
    t = 0
    while t < s_max:
        for p in (0, 1):
            h = s @ M
            flip = (-2 * s * h <= 0) & (col == p)[None, :] & lv[None, :]
            s[flip] *= -1
        t += 1
        e = energies()
        for r in range(R):
            m = int(e[r * K:(r + 1) * K].min())
            if m < emin[r]:
                emin[r], thit[r] = m, t
        if len(set(emin)) == 1 and t >= 2 * max(thit):
            break
    return emin, thit, t


def _hardness_reference(L, live, J, iid, seed, n_restarts, K, R, s_max):
    """E_gs, ln TTS (Appendix B: sweeps of all restarts per restart that
    ended at E_gs), confirmation and per-restart results, from the greedy
    restarts above."""
    res = []
    for rho in range(n_restarts):
        key = int(oracle.philox([rho, 0, 0, 5], [iid, seed])[0])
        res.append(_greedy_restart(L, live, J, K, R, key, seed, s_max))
    gs = min(min(em) for em, _, _ in res)
    hits = [rho for rho, (em, _, _) in enumerate(res) if min(em) == gs]
    sweeps = sum(t for _, _, t in res)
    r_tts = []
    for em, th, _ in res:
        at = [th[r] for r in range(R) if em[r] == gs]
        r_tts.append(max(1, min(at)) if at else -1)
    confirmed = len(hits) >= 2 or any(sum(1 for x in em if x == gs) >= 2 for em, _, _ in res)
    return dict(e_gs=gs, ln_tts=math.log(sweeps / len(hits)), confirmed=confirmed,
                r_emin=[min(em) for em, _, _ in res], r_sweeps=[t for _, _, t in res], r_tts=r_tts)


ZERO_T_BETAS = workloads.geometric_betas(12.0, 768.0, 4)


def test_zero_temperature_thresholds_are_zero():
    """The premise of the greedy reference: at beta >= 12 no uphill move of
    dE >= 2 and no exchange against d >= 1 has a nonzero threshold."""
    for b in ZERO_T_BETAS:
        assert oracle.metro_threshold(float(b), 1) == 0
    for k in range(len(ZERO_T_BETAS) - 1):
        assert oracle.swap_threshold(float(ZERO_T_BETAS[k]), float(ZERO_T_BETAS[k + 1]), 1) == 0


def test_hardness_equals_greedy_reference_at_zero_temperature():
    """Restart by restart, the oracle's hardness_eval equals the greedy
    reference: minima, sweeps run (agreement stop t >= 2 max t_hit, else
    the cap), first hits, E_gs, confirmation and ln TTS.  The cases cover
    restarts that stop on agreement and restarts that run to the cap."""
    stopped, capped = 0, 0
    cases = [(2, None, workloads.couplings(2, "pm1", 5, n), 300 + n, 2) for n in range(4)]
    cases += [(2, workloads.missing_mask(2, 0.1, 6, 0), workloads.couplings(2, "pm3", 6, 0), 400, 3),
              (3, None, np.full(len(_chimera(3)), -1, np.int8), 500, 2),
              (2, None, workloads.couplings(2, "pm7", 7, 1), 600, 2)]
    s_max = 40
    for L, live, J, iid, R in cases:
        want = _hardness_reference(L, live, J, iid, SEED, 6, 4, R, s_max)
        got = oracle.hardness_eval(L, live, J, iid, SEED, 6, 4, R, ZERO_T_BETAS, 1, s_max)
        assert got["e_gs"] == want["e_gs"]
        assert got["r_emin"].tolist() == want["r_emin"]
        assert got["r_sweeps"].tolist() == want["r_sweeps"], (iid, got["r_sweeps"], want["r_sweeps"])
        assert got["r_tts"].tolist() == want["r_tts"]
        assert got["confirmed"] == want["confirmed"]
        assert got["ln_tts"] == want["ln_tts"]
        stopped += sum(1 for t in want["r_sweeps"] if t < s_max)
        capped += sum(1 for t in want["r_sweeps"] if t == s_max)
    assert stopped > 0 and capped > 0, (stopped, capped)


@pytest.mark.parametrize("L,R", [(2, 2), (3, 3)])
def test_free_couplings_stop_after_one_sweep(L, R):
    """J = 0: every energy is 0 from the start, the running minima agree
    with first hit 0, so every restart stops after its first sweep
    (1 >= 2 * 0): sweeps = n_restarts, every restart finds E_gs = 0, and
    ln TTS = ln(n / n) = 0 exactly."""
    J = np.zeros(len(_chimera(L)), np.int8)
    res = oracle.hardness_eval(L, None, J, 7, SEED, 5, 6, R, workloads.geometric_betas(0.1, 5.0, 6), 1, 1000)
    assert res["e_gs"] == 0 and res["confirmed"]
    assert res["r_sweeps"].tolist() == [1] * 5
    assert res["r_tts"].tolist() == [1] * 5
    assert res["ln_tts"] == 0.0


# ---------------------------------------------------------------------------
# Thresholds against the exact exponentials (50-digit decimal arithmetic)
_CTX = decimal.Context(prec=50)


def _exact_scaled(x):
    """2^32 e^{-x} for a double x >= 0, to 50 significant digits."""
    return _CTX.multiply(_CTX.exp(_CTX.minus(decimal.Decimal(x))), decimal.Decimal(2 ** 32))


def _ladders():
    out = [workloads.geometric_betas(0.2, 3.0, 16), workloads.geometric_betas(0.1, 5.0, 32),
           workloads.geometric_betas(0.1, 5.0, 8)]
    out += [workloads.geometric_betas(0.1, 5.0, K) for K in (24, 37, 48)]
    return out


def _check_floor(T, exact):
    """T = floor(exact) up to a 2^-16 allowance for the double-precision
    exponential: 0 <= exact - T < 1, i.e. |T / 2^32 - e^{-x}| < 2^-32."""
    diff = exact - decimal.Decimal(T)
    tol = decimal.Decimal(2) ** -16
    assert -tol <= diff < 1 + tol, (T, exact)


def test_metropolis_thresholds_are_floors_of_the_exact_acceptance():
    """Accepting iff a uniform 32-bit u < T gives probability T / 2^32; with
    T = floor(2^32 e^{-beta dE}) and dE = 2m this is e^{-beta dE} within
    2^-32 (Sec. II, Metropolis).  A rounding instead of a floor, or beta m in
    place of beta 2m, fails here."""
    n = 0
    for ladder in _ladders():
        for b in ladder:
            for m in range(1, 43):
                _check_floor(oracle.metro_threshold(float(b), m), _exact_scaled(2 * m * float(b)))
                n += 1
    assert n > 5000


def test_exchange_thresholds_are_floors_of_the_detailed_balance_ratio():
    """Exchange of x at beta_k with y at beta_{k+1}: the ratio of the joint
    Boltzmann weights after and before is e^{-(beta_{k+1} - beta_k)(E_x - E_y)}
    (Sec. II); T = floor(2^32 of it) for d = E_x - E_y >= 1, until it reaches
    0.  A swapped sign or a missing factor fails here."""
    for ladder in _ladders()[:4]:
        for k in range(len(ladder) - 1):
            lo, hi = float(ladder[k]), float(ladder[k + 1])
            db = hi - lo
            assert db == float(decimal.Decimal(hi) - decimal.Decimal(lo))  # exact (Sterbenz)
            last = int(22.2 / db) + 2
            ds = list(range(1, 120)) + list(range(120, last, 37)) + [last]
            for d in ds:
                T = oracle.swap_threshold(lo, hi, d)
                _check_floor(T, _exact_scaled(db * d))


# ---------------------------------------------------------------------------
# Boltzmann statistics against brute-force enumeration
def _chi2_pvalue(counts, probs, min_expected=5.0):
    exp = probs * counts.sum()
    big = exp >= min_expected
    obs = np.append(counts[big], counts[~big].sum())
    e = np.append(exp[big], exp[~big].sum())
    keep = e > 0
    obs, e = obs[keep], e[keep]
    return stats.chi2.sf(float(((obs - e) ** 2 / e).sum()), len(obs) - 1)


def _boltzmann(en, beta):
    w = np.exp(-beta * (en - en.min()))
    return w / w.sum()


def _lane_states(spins, lanes, n_sites):
    """Integer index of each lane's configuration over sites 0..n_sites-1
    (bit n = spin bit of site n)."""
    bits = (spins[:n_sites, None] >> np.arange(lanes, dtype=np.uint64)[None, :]) & np.uint64(1)
    return (bits.astype(np.int64) << np.arange(n_sites)[:, None]).sum(axis=0)


def test_two_cell_graph_samples_boltzmann():
    """64 independent Metropolis chains on the 16-spin graph of two
    neighbouring cells (the other two cells of C2 missing): the histograms of
    energies and of configurations (folded by the global flip, a symmetry of
    Eq. 1 without fields) match exp(-beta E) / Z from enumeration."""
    L = 2
    live = np.zeros(32, np.uint8)
    live[:16] = 1                     # cells (0,0) and (0,1)
    J = workloads.couplings(L, "pm3", 17, 0)
    _, _, en = oracle.enumerate_states(L, live, J, want_energies=True)
    beta = 0.3
    probs = _boltzmann(en.astype(np.float64), beta)
    K, R = 1, 64
    st = oracle.pt_init(L, live, J, K, R, 23, SEED)
    b = np.array([beta])
    oracle.pt_run(L, live, J, K, R, b, 23, SEED, 0, 50, st)
    counts = np.zeros(1 << 16, np.int64)
    for _ in range(3000):
        oracle.pt_run(L, live, J, K, R, b, 23, SEED, 0, 3, st)
        np.add.at(counts, _lane_states(st.spins, 64, 16), 1)
    idx = np.arange(1 << 15)
    flip = (1 << 16) - 1 - idx
    p_conf = _chi2_pvalue(counts[idx] + counts[flip], probs[idx] + probs[flip])
    levels = np.unique(en)
    pos = np.searchsorted(levels, en)
    c_lev = np.bincount(pos, weights=counts, minlength=len(levels))
    p_lev = np.bincount(pos, weights=probs, minlength=len(levels))
    p_energy = _chi2_pvalue(c_lev, p_lev)
    assert p_conf > 1e-4 and p_energy > 1e-4, (p_conf, p_energy)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_joint_slot_and_configuration_distribution(K):
    """Parallel tempering on one K_{4,4} cell with K temperatures and 16
    replica sets, an exchange pass after every sweep.  In the stationary
    state (detailed balance of both moves, Sec. II) every configuration
    copy sits at each slot with probability 1/K and, given slot k, follows
    Boltzmann at beta_k; the energies held at the K slots are independent.
    Both joint distributions are compared with the enumerated product form."""
    L = 1
    J = workloads.couplings(L, "pm3", 30 + K, 0)
    _, _, en = oracle.enumerate_states(L, None, J, want_energies=True)
    betas = workloads.geometric_betas(0.2, 1.2, K)
    R = 16
    st = oracle.pt_init(L, None, J, K, R, 40 + K, SEED)
    oracle.pt_run(L, None, J, K, R, betas, 40 + K, SEED, 1, 30, st)
    lanes = K * R
    slot_conf = np.zeros((K, 256), np.int64)
    levels = np.unique(en)
    nlev = len(levels)
    tuples = np.zeros(nlev ** K, np.int64)
    for _ in range(1500):
        oracle.pt_run(L, None, J, K, R, betas, 40 + K, SEED, 1, 2, st)
        conf = _lane_states(st.spins, lanes, 8)
        perm = st.perm.reshape(K, R)             # perm[k R + r] = lane at slot (k, r)
        for k in range(K):
            np.add.at(slot_conf[k], conf[perm[k]], 1)
        lev = np.searchsorted(levels, en[conf[perm]])   # [K, R] level index per slot
        code = np.zeros(R, np.int64)
        for k in range(K):
            code = code * nlev + lev[k]
        np.add.at(tuples, code, 1)
    # (slot, configuration): 1/K x Boltzmann(beta_k), folded by the global flip
    idx = np.arange(128)
    want = np.concatenate([_boltzmann(en.astype(np.float64), b)[idx] + _boltzmann(en.astype(np.float64), b)[255 - idx]
                           for b in betas]) / K
    got = np.concatenate([slot_conf[k][idx] + slot_conf[k][255 - idx] for k in range(K)])
    p_joint = _chi2_pvalue(got, want)
    # energies across slots: product of the per-slot level distributions
    pos = np.searchsorted(levels, en)
    marg = [np.bincount(pos, weights=_boltzmann(en.astype(np.float64), b), minlength=nlev) for b in betas]
    prod = marg[0]
    for k in range(1, K):
        prod = np.multiply.outer(prod, marg[k]).ravel()
    p_prod = _chi2_pvalue(tuples, prod)
    assert p_joint > 1e-4 and p_prod > 1e-4, (p_joint, p_prod)


# ---------------------------------------------------------------------------
# The RAO move (Algorithm 1)
def test_mutation_is_uniform_over_live_couplers_and_other_letters():
    """Over many (step, proposal) draws the pair (coupler, new value) is
    uniform over the live couplers times the alphabet letters other than the
    coupler's current value: every cell of that grid is hit at the same
    rate (chi^2), and nothing outside it is ever drawn."""
    L = 2
    A = workloads.ALPHABETS["pm3"]
    J = workloads.couplings(L, "pm3", 8, 0)
    live = workloads.missing_mask(L, 0.1, 8, 0)
    E = _chimera(L)
    lv = live.astype(bool)
    live_e = np.nonzero(lv[E[:, 0]] & lv[E[:, 1]])[0]
    pos = {int(e): n for n, e in enumerate(live_e)}
    counts = np.zeros((len(live_e), len(A)), np.int64)
    for step in range(4000):
        for prop in range(8):
            e, old, new, _ = oracle.mutate(L, live, J, A, 3, 77, step, prop)
            assert e in pos and old == J[e] and new != old
            counts[pos[e], int(np.nonzero(A == new)[0][0])] += 1
    allowed = np.array([[a != J[e] for a in A] for e in live_e])
    assert counts[~allowed].sum() == 0
    obs = counts[allowed]
    p = stats.chisquare(obs).pvalue
    assert p > 1e-4, p


# ---------------------------------------------------------------------------
# Surrogate oracle against torch autograd
def test_surrogate_oracle_matches_torch_autograd():
    """The float64 forward pass and hand-written backward pass of
    oracle/gnn.py equal torch's autograd of the same network, written here
    from its definition (edge message passing, 3 layers, width 64, mean
    readout over live sites, MSE over finite labels), on a batch with
    missing sites and an infinite label."""
    torch = pytest.importorskip("torch")
    import oracle.gnn as G
    graphs = []
    for g in range(3):
        graphs.append((2, workloads.missing_mask(2, 0.1, 12, g), workloads.couplings(2, "pm7", 12, g)))
    B = G.batch(graphs)
    labels = np.array([1.5, np.inf, -0.25])
    theta = np.random.default_rng(4).normal(0.0, 0.15, G.n_params())
    loss_o, grad_o, y_o = G.loss_and_grad(theta, B, labels)

    t = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    P, o = {}, 0
    for name, shp in G.param_shapes():
        n = int(np.prod(shp))
        P[name] = t[o:o + n].reshape(shp)
        o += n
    xn = torch.tensor(B["xn"])
    xe = torch.tensor(B["xe"])
    src = torch.tensor(B["src"])
    dst = torch.tensor(B["dst"])
    n_nodes = xn.shape[0]
    h = xn @ P["W_en"].T + P["b_en"]
    m = (xe @ P["W_ee"].T + P["b_ee"]).repeat_interleave(2, dim=0)   # directions 2q, 2q+1
    for l in range(3):
        m = torch.relu(torch.cat([h[src], h[dst], m], dim=1) @ P[f"W_m{l}"].T + P[f"b_m{l}"])
        s = torch.zeros(n_nodes, 64, dtype=torch.float64).index_add(0, dst, m)
        h = torch.relu(torch.cat([h, s], dim=1) @ P[f"W_h{l}"].T + P[f"b_h{l}"])
    live = torch.tensor(B["live"]).reshape(B["G"], B["N"])
    mean = (h.reshape(B["G"], B["N"], 64) * live[:, :, None]).sum(dim=1) / live.sum(dim=1)[:, None]
    y = mean @ P["w_out"] + P["b_out"][0]
    ok = torch.tensor(np.isfinite(labels))
    lab = torch.tensor(np.where(np.isfinite(labels), labels, 0.0))
    loss = ((y - lab)[ok] ** 2).sum() / ok.sum()
    loss.backward()
    assert np.allclose(y.detach().numpy(), y_o, rtol=1e-12, atol=1e-12)
    assert abs(loss.item() - loss_o) <= 1e-12 * max(1.0, abs(loss_o))
    g = t.grad.numpy()
    assert np.allclose(grad_o, g, rtol=1e-9, atol=1e-12), float(np.abs(grad_o - g).max())
