"""Temperature random walk of parallel tempering and its mixing time --
TEST INFRASTRUCTURE ONLY (tests/, the smoke check and bench.py's CPU
baseline may use it; the product path never does).

Sec. III.B defines the classical hardness as the mixing time tau of the
temperature random walk that each system copy performs under PT.  The
elementary Monte Carlo step (EMCS) is 10 Metropolis sweeps followed by one
exchange pass, and a tau is accepted when (i) the copy that spends the
least time in the hot half (the K/2 highest temperatures) spends at least
20 % of the run there, and (ii) the run spans at least 20 tau.

The paper takes the estimator from a reference that is not reproduced in
it.  Reading used here: the integrated autocorrelation time of the
temperature index (Sokal's lecture notes, which the paper cites) in units
of EMCS, with
  g_c(t) = 2 k_c(t) - (K - 1)      (temperature index about its stationary
                                    mean (K - 1) / 2: a copy visits every
                                    temperature equally often at equilibrium)
  S(d)   = sum over copies c and t < T - d of g_c(t) g_c(t + d)   (exact)
  rho(d) = [S(d) / (T - d)] / [S(0) / T]
  tau(W) = 1/2 + sum_{d=1..W} rho(d),  W = the smallest window with
           W >= c tau(W)  (Sokal's automatic window, c = 6).
tau in Metropolis sweeps is tau(W) times the sweeps per EMCS.
"""
import numpy as np

from . import pt_init, pt_run

HOT_FRACTION_MIN = 0.2   # criterion (i)
RUN_OVER_TAU_MIN = 20.0  # criterion (ii)


def walk(L, live, J, K, R, beta, key0, key1, sweeps_per_emcs, n_emcs, state=None):
    """Temperature index of every configuration after each of n_emcs
    EMCS (sweeps_per_emcs sweeps, the last followed by the exchange pass):
    uint8 [n_emcs][K R], plus the final state.  Configuration c belongs to
    replica set c // K for the whole run."""
    st = state if state is not None else pt_init(L, live, J, K, R, key0, key1)
    out = np.zeros((n_emcs, K * R), np.uint8)
    for e in range(n_emcs):
        pt_run(L, live, J, K, R, beta, key0, key1, sweeps_per_emcs, sweeps_per_emcs, st)
        for k in range(K):
            for r in range(R):
                out[e, st.perm[k * R + r]] = k  # perm[k R + r] = configuration at slot (k, r)
    return out, st


def acf_sums(traj, K, max_lag):
    """S(d) for d = 0..max_lag (int64, exact); lags at or beyond the run
    length are 0."""
    g = 2 * np.asarray(traj, np.int64) - (K - 1)
    T = g.shape[0]
    S = np.zeros(max_lag + 1, np.int64)
    for d in range(min(max_lag, T - 1) + 1):
        S[d] = int(np.sum(g[:T - d] * g[d:]))
    return S


def hot_counts(traj, K):
    """EMCS each configuration spent in the hot half: temperature index
    k < K // 2 (the ladder is ordered by ascending beta, so small k is hot)."""
    return (np.asarray(traj) < K // 2).sum(axis=0).astype(np.int64)


def tau_int(S, T, c=6.0):
    """(tau in EMCS, window W, converged) from the sums S over a run of T
    EMCS.  Not converged when no window up to len(S) - 1 satisfies
    W >= c tau(W); tau(max window) is returned then."""
    S = np.asarray(S, np.float64)
    if T < 2 or S[0] <= 0:
        return 0.5, 0, False
    c0 = S[0] / T
    tau = 0.5
    for W in range(1, len(S)):
        if W >= T:
            break
        tau += (S[W] / (T - W)) / c0
        if W >= c * tau:
            return tau, W, True
    return tau, min(len(S) - 1, T - 1), False


def criteria(hot, T, tau_emcs):
    """(i) least hot-half share over the copies >= 0.2 and (ii) T >= 20 tau."""
    share = float(np.min(hot)) / T if T else 0.0
    return share >= HOT_FRACTION_MIN, T >= RUN_OVER_TAU_MIN * tau_emcs, share
