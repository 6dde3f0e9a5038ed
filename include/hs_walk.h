/*
 * hs_walk -- C ABI of the mixing-time statistics of the temperature random
 * walk (Sec. III.B: the classical hardness of an instance is the mixing time
 * tau of the walk that every PT copy performs over the temperature ladder;
 * EMCS = 10 Metropolis sweeps and one exchange pass; a tau counts when the
 * copy that spends the least time in the hot half (the K/2 highest
 * temperatures) spends at least 20 % of the run there, and when the run spans
 * at least 20 tau).  The walks come from pt_sweep_record (hardspin.h).
 *
 * The estimator of the paper's cited reference is not reproduced in the
 * paper.  This library uses the integrated autocorrelation time of the
 * temperature index, with the stationary mean (K - 1) / 2 taken as known:
 *   g_c(t) = 2 k_c(t) - (K - 1)
 *   S(d)   = sum over configurations c < K R and t < T - d of g_c(t) g_c(t+d)
 *   rho(d) = [S(d) / (T - d)] / [S(0) / T]
 *   tau(W) = 1/2 + sum_{d=1..W} rho(d), W = the smallest window with
 *            W >= c tau(W) (automatic window; c = 6 is customary)
 * in units of exchange passes (EMCS).
 *
 * Memory: device pointers are the caller's and must stay valid until the
 * stream has finished; the library allocates no device memory.  Errors are
 * HS_* codes of hardspin.h with a thread-local message (hs_last_error).
 */
#ifndef HS_WALK_H
#define HS_WALK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Enqueues on `stream` (hipStream_t, NULL = default), for every instance n <
 * n_inst of a walk buffer laid out as pt_sweep_record writes it (capacity
 * passes per instance, the first n_steps of them used):
 *   acf[n (max_lag + 1) + d] = S(d), d = 0..max_lag (0 when d >= n_steps),
 *   hot[n 64 + c] = passes t < n_steps with k_c(t) < K / 2 (0 for c >= K R).
 * acf (int64) and hot (int64) are device buffers.  Sums are exact.
 * HS_EINVAL unless 0 <= n_steps <= capacity, 1 <= K, 1 <= R, K R <= 64,
 * 0 <= max_lag <= 65535 and the pointers are non-NULL when n_inst > 0. */
int walk_autocorr(const uint8_t *walk, int n_inst, int64_t capacity, int64_t n_steps, int K, int R,
                  int max_lag, int64_t *acf, int64_t *hot, void *stream);

/* Host only: tau(W) in exchange passes from S(0..max_lag) (host array) of a
 * walk of n_steps passes, with window constant c_window.  *window = W and
 * *converged = 1 when some W <= min(max_lag, n_steps - 1) satisfies
 * W >= c_window tau(W); otherwise *converged = 0 and tau is the sum over
 * that largest window.  S(0) <= 0 or n_steps < 2 gives tau = 1/2, W = 0,
 * not converged.  HS_EINVAL for NULL pointers or max_lag < 0. */
int walk_tau(const int64_t *acf, int max_lag, int64_t n_steps, double c_window, double *tau, int *window,
             int *converged);

#ifdef __cplusplus
}
#endif

#endif
