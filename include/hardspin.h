/*
 * hardspin -- C ABI of the MI355X (gfx950) parallel-tempering engine for
 * Ising spin glasses on Chimera graphs, the hot path of the hard-instance
 * search of Marshall, Martin-Mayor and Hen, "Practical engineering of hard
 * spin-glass instances" (arXiv:1605.03607).
 *
 * Conventions shared by every entry point
 *   - Cost function: H = sum over Chimera couplers of J_ij s_i s_j, minimised,
 *     no fields (Eq. 1, Sec. II).
 *   - Chimera C_L (Appendix A, Fig. 8): L x L cells, each a K_{4,4}.  Site id
 *     i = 8 (L r + c) + 4 u + k for cell (r, c), side u, index k.  Couplers:
 *     (r,c,0,k)-(r,c,1,k') inside a cell, (r,c,0,k)-(r+1,c,0,k) and
 *     (r,c,1,k)-(r,c+1,1,k) between cells.  Canonical coupler order:
 *     ascending (min id, max id); the full C_L has 24 L^2 - 8 L couplers.
 *   - A spin bit b = 1 means s = -1.  Spins are exchanged "word-major": one
 *     uint64 per site, bit l = the spin bit of replica configuration l.
 *   - Lanes, slots: an instance runs K temperatures x R replica sets
 *     (K R <= 64 lanes).  Lane r K + k starts at temperature slot (k, r);
 *     exchanges move configurations between slots of the same replica set
 *     (Sec. II: swaps between neighbouring temperatures satisfying detailed
 *     balance).  perm[k R + r] is the lane currently at slot (k, r).
 *   - Sweep t (0-based, per instance): a Metropolis pass over all live sites
 *     of colour 0, then of colour 1 (colour (r + c + u) mod 2), in every lane
 *     ("full-lattice Metropolis sweeps", Sec. III.B), followed by an
 *     exchange pass (ascending pairs per replica set) when
 *     (t + 1) mod swap_interval == 0.  Every random number is a Philox4x32-10
 *     output keyed by (instance_id, seed) at a counter fixed by (sweep,
 *     site pair, slot, use), so results do not depend on the launch shape.
 *   - Memory: every device pointer is owned by the caller and must stay
 *     valid until the stream has finished the work enqueued on it.  The
 *     library itself allocates no device memory.
 *   - Errors: every call returns HS_OK (0) or a negative HS_E* code and sets
 *     a thread-local message (hs_last_error).  Asynchronous device faults are
 *     reported as HS_EHIP by the next call that synchronises.
 *   - Threads: calls on different handles and buffers may run concurrently
 *     from different host threads (each on its own stream); one handle is
 *     used by one thread at a time.  The library's shared state (the device's
 *     compute-unit count, the planted-instance cycle lists) is initialised
 *     once under a lock.
 */
#ifndef HARDSPIN_H
#define HARDSPIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HS_OK 0
#define HS_EINVAL (-1)        /* malformed argument */
#define HS_ENOSPACE (-2)      /* caller buffer or workspace too small */
#define HS_EUNSUPPORTED (-3)  /* size outside the engine's limits (L > 16, K R > 64, |J| > 7) */
#define HS_EHIP (-4)          /* HIP runtime error */
#define HS_EMISMATCH (-5)     /* incremental and recomputed energies differ */

#define HS_MAX_L 16
#define HS_MAX_LANES 64
#define HS_MAX_ABS_J 7

/* Flags of hs_pt_desc.flags */
#define HS_INIT_FROM_BUFFER 1u   /* pt_init reads initial spins from buffers->spins */
#define HS_STOP_ON_AGREEMENT 2u  /* stop an instance once all replica sets agree (see pt_sweep) */
#define HS_PACK_LANES 4u         /* share a workgroup's 64 lanes between instances of one lattice size
                                    (see hs_pt_desc); not with HS_STOP_ON_AGREEMENT */

/* One problem instance and its temperature ladder.  Host memory; read during
 * the call only.
 *   L            Chimera side, 1..16 (N = 8 L^2 sites)
 *   live         N bytes, 1 = working qubit, 0 = missing; NULL = all live
 *   J            couplings over the full canonical coupler list (24 L^2 - 8 L
 *                entries); couplers touching a missing site are ignored;
 *                |J| <= 7
 *   instance_id  first word of the Philox key of this instance
 *   K, R         temperatures and replica sets, 1 <= K, 1 <= R, K R <= 64
 *   beta         K inverse temperatures, 0 < beta_0 < beta_1 < ... */
typedef struct hs_instance {
    int32_t L;
    const uint8_t *live;
    const int8_t *J;
    uint32_t instance_id;
    int32_t K;
    int32_t R;
    const double *beta;
} hs_instance;

/* A batch of instances simulated together in one persistent launch.
 * With HS_PACK_LANES the launch plan packs instances of the same lattice size
 * whose lane counts K R add up to at most 64 into one workgroup (two per
 * workgroup at most), so that the lanes one instance leaves idle serve
 * another.  Every instance keeps its own couplings, ladder, Philox key,
 * replica sets and exchange passes: results are those of the unpacked launch
 * (and of the oracle), only the lane occupancy changes. */
typedef struct hs_pt_desc {
    int32_t n_inst;
    const hs_instance *inst; /* host array of n_inst */
    uint32_t seed;           /* second word of every Philox key */
    int32_t swap_interval;   /* exchange pass after every swap_interval-th sweep; 0 = none */
    uint32_t flags;          /* HS_INIT_FROM_BUFFER | HS_STOP_ON_AGREEMENT | HS_PACK_LANES */
    int32_t block_waves;     /* wavefronts per instance (1..16); 0 = one per cell pair of the
                                largest instance, rounded up to a power of two, at most 16
                                (pt_autotune measures the candidates instead) */
} hs_pt_desc;

/* Device buffers of a batch (caller-owned; offsets per instance n):
 *   spins     uint64 [sum_n N_n]   instance n starts at word sum_{m<n} N_m
 *   perm      uint8  [n_inst][64]  slot -> lane (first K R entries used)
 *   energy    int32  [n_inst][64]  per-lane energy, maintained incrementally
 *   emin      int32  [n_inst][64]  running minimum per replica set (first R)
 *   thit      int64  [n_inst][64]  completed sweeps when emin was first reached
 *   swap_acc  uint32 [n_inst][64]  accepted exchanges per pair (k, k+1), set r at k R + r
 *   t         int64  [n_inst]      completed sweeps (the Philox sweep counter)
 *   stopped   int32  [n_inst]      1 once HS_STOP_ON_AGREEMENT ended the run
 *   workspace bytes from pt_workspace_bytes(); tables and descriptors */
typedef struct hs_buffers {
    uint64_t *spins;
    uint8_t *perm;
    int32_t *energy;
    int32_t *emin;
    int64_t *thit;
    uint32_t *swap_acc;
    int64_t *t;
    int32_t *stopped;
    void *workspace;
    size_t workspace_bytes;
} hs_buffers;

typedef struct hs_pt hs_pt; /* opaque host handle */

/* Library version (major * 10000 + minor * 100 + patch). */
int hs_version(void);

/* Message of the last error on this thread (never NULL). */
const char *hs_last_error(void);

/* Bytes of device workspace pt_init needs for this batch.  Host only.
 * HS_EINVAL / HS_EUNSUPPORTED for a malformed batch. */
int pt_workspace_bytes(const hs_pt_desc *d, size_t *bytes);

/* Validates the batch, builds the per-instance coupling words and the
 * Metropolis / exchange threshold tables on the host (floor(2^32 exp(-x)) in
 * double precision), uploads them into b->workspace with async copies on
 * `stream` (a hipStream_t; NULL = default stream) and enqueues the initial
 * state: spins from Philox (bit 31 of word i mod 4 of
 * Philox((instance_id, seed), (0, i div 4, (k << 8) | r, 2)) for the lane at
 * slot (k, r)) or from b->spins (HS_INIT_FROM_BUFFER), perm = identity,
 * energies from Eq. 1, emin/thit, zero counters.  *out receives a host handle
 * that keeps copies of the descriptor and buffer pointers. */
int pt_init(hs_pt **out, const hs_pt_desc *d, const hs_buffers *b, void *stream);

/* Enqueues n_sweeps sweeps of every instance in one persistent kernel launch
 * (Metropolis sweeps, exchange passes, running minima; Sec. II and III.B).
 * With HS_STOP_ON_AGREEMENT an instance stops after the first sweep at which
 * all its replica sets have the same running minimum and its completed sweep
 * count is at least twice the largest first-hit count (ground state confirmed
 * by agreement, Appendix B).  Asynchronous. */
int pt_sweep(hs_pt *h, int64_t n_sweeps);

/* pt_sweep that also records the temperature random walk (Sec. III.B): after
 * the e-th exchange pass of this call (e < capacity), walk[(n capacity + e)
 * 64 + c] = temperature index k of configuration c of instance n (c < K R;
 * bytes of c >= K R and of passes not made are left untouched).  walk is a
 * caller-owned device buffer of n_inst x capacity x 64 bytes.  Results are
 * identical to pt_sweep's.  HS_EINVAL for capacity < 0 or a NULL walk with
 * capacity > 0.  Asynchronous. */
int pt_sweep_record(hs_pt *h, int64_t n_sweeps, uint8_t *walk, int64_t capacity);

/* HIP graph of a sweep launch.  pt_graph_create captures the launches that
 * pt_sweep(h, n_sweeps) would enqueue (a work-queue reset and one persistent
 * sweep kernel) on a private capture stream and instantiates them;
 * pt_graph_launch replays them on h's stream, i.e. enqueues n_sweeps more
 * sweeps of every instance, exactly as pt_sweep would (the chains continue;
 * results are identical).  The graph refers to h's buffers: destroy it before
 * h.  HS_EHIP on a capture or launch failure. */
typedef struct hs_graph hs_graph;
int pt_graph_create(hs_pt *h, int64_t n_sweeps, hs_graph **out);
int pt_graph_launch(hs_graph *g);
int pt_graph_destroy(hs_graph *g);

/* Workgroup-shape autotuner for a batch (the "tile shape" of a persistent
 * launch: wavefronts per instance).  For each candidate block_waves in
 * {2, 4, 8, 16} it initialises the batch on the caller's scratch buffers
 * (sized as pt_init needs; contents overwritten; candidates whose workspace
 * does not fit in scratch->workspace_bytes are skipped), runs trial_sweeps / 8
 * warm-up sweeps and times trial_sweeps sweeps with HIP events on `stream`.
 * Writes the fastest candidate to *block_waves_out and, if not NULL, its time
 * per sweep in microseconds.  Synchronises the stream; the trial chains
 * never touch the caller's real buffers, so tuning does not change results. */
int pt_autotune(const hs_pt_desc *d, const hs_buffers *scratch, void *stream, int64_t trial_sweeps,
                int32_t *block_waves_out, double *us_per_sweep_out);

/* Enqueues one extra exchange pass now, outside the sweep schedule, drawing
 * from its own Philox use (counter word 3 = 3) so it never repeats the draws
 * of the scheduled passes.  Asynchronous. */
int pt_swap(hs_pt *h);

/* Recomputes every lane energy from the spins (Eq. 1) into recomputed
 * (device int32 [n_inst][64], caller-owned) and compares it with the
 * incremental energies.  Synchronises the stream.  HS_EMISMATCH if any live
 * lane differs; *n_mismatch (host, may be NULL) receives the count. */
int pt_measure(hs_pt *h, int32_t *recomputed, int32_t *n_mismatch);

/* Frees the host handle (device buffers stay the caller's).  Waits until the
 * workspace upload that pt_init enqueued has finished (it reads the handle's
 * host staging copy), not for later work on the stream.  NULL is a no-op. */
int pt_destroy(hs_pt *h);

/* Launch shape of the handle's persistent sweep kernel: workgroups in the
 * grid (at most the work items; each takes items from the work queue until
 * it is empty), wavefronts per workgroup, dynamic LDS bytes per workgroup,
 * and the work items (n_inst, or the number of packs when HS_PACK_LANES
 * packed the batch; equal to n_inst when nothing could be packed), and the
 * lane slots one sweep passes through (sum over work items of 64 x the
 * item's sites, live or not: the denominator of lane occupancy).  Any
 * output pointer may be NULL.  Host only. */
int pt_launch_shape(const hs_pt *h, int32_t *grid, int32_t *block_waves, int32_t *lds_bytes, int32_t *work_items,
                    int64_t *lane_sites);

/* A stream (default priority) whose kernels run only on compute units
 * cu_first .. cu_first + cu_count - 1 of the current device
 * (hipExtStreamCreateWithCUMask).  A persistent sweep launch holds every CU
 * it reaches until its work queue is empty, so small kernels that must not
 * wait for it (the surrogate's screen and training inside the instance
 * search, Algorithm 1) get CUs of their own this way, and the sweep
 * launches a stream over the rest.  Kernels launched on such a stream keep
 * their grids; workgroups beyond the CUs' capacity start as others finish.
 * *stream receives the handle; HS_EINVAL for a NULL stream or a range
 * outside the device, HS_EHIP if the runtime refuses.  Host only. */
int hs_stream_create_cus(int32_t cu_first, int32_t cu_count, void **stream);

/* Destroys a stream made by hs_stream_create_cus (after its work has
 * finished, as hipStreamDestroy).  NULL is a no-op. */
int hs_stream_destroy(void *stream);

/* One RAO move (Algorithm 1, Sec. II.A) as a pure host function.
 * (w0, w1, w2, w3) = Philox((chain, seed), (step, proposal, 0, 4)); the
 * coupler is the e-th live one in canonical order, e = floor(w0 E_live /
 * 2^32); the new value is entry floor(w1 (n_alpha - 1) / 2^32) of the
 * ascending alphabet with the current value removed (a sign flip for
 * {-1, +1}).  `in` is not modified.  HS_EINVAL when the alphabet repeats a
 * value or does not hold the chosen coupler's current value. */
typedef struct hs_mutation {
    int32_t edge;       /* index in the full canonical coupler list */
    int8_t old_j;
    int8_t new_j;
    uint32_t w_accept;  /* uniform for hs_rao_accept */
} hs_mutation;
int instance_mutate(const hs_instance *in, const int8_t *alphabet, int n_alpha, uint32_t chain,
                    uint32_t seed, uint32_t step, uint32_t proposal, hs_mutation *out);

/* Algorithm 1's acceptance on ln TTS at search temperature t_s: returns 1 iff
 * delta = ln_new - ln_cur >= 0 or w < floor(2^32 exp(delta / t_s)) (an
 * infinite new value is accepted; inf - inf counts as 0), else 0. */
int hs_rao_accept(double ln_cur, double ln_new, double t_s, uint32_t w);

/* Planted-solution instances and the moves of Loop Adaptive Optimization
 * (Sec. IV, Algorithm 2).  An instance is a sum of n_loops frustrated loop
 * Hamiltonians on simple cycles of 4 or 6 couplers of the live Chimera graph;
 * each loop's couplings keep the planted state s* among its ground states,
 * so s* is a ground state of the sum and E_gs = sum over loops of
 * -(size - 2) weight.
 *   - Loop (size, cycle, weight, flip): cycle indexes the cycles of that
 *     size, each identified by its ascending coupler indices and the list
 *     sorted by them; weight in 1..5; on every coupler but the flip-th (in
 *     ascending order) J += -weight s*_i s*_j, on that one J += +weight
 *     s*_i s*_j (Fig. 6: integer weights 1..5, 4-cycles with probability
 *     0.1, else 6-cycles).
 *   - A loop that would push a coupler past |J| = 7 (the engine's range) is
 *     drawn again with the next attempt counter, at most 64 times
 *     (HS_EUNSUPPORTED after that).
 *   - Draws: planted bit i = bit 31 of word 0 of Philox((chain, seed),
 *     (i, 0, 1, 8)) (0 for missing sites).  Initial loop m, attempt a: words
 *     (w0, w1, w2, w3) of Philox((chain, seed), (m, a, 0, 8)): size 4 iff
 *     w0 < 429496730, cycle floor(w1 n / 2^32), weight 1 + floor(w2 5 / 2^32),
 *     flip floor(w3 size / 2^32).  Move (step, proposal): Philox((chain,
 *     seed), (step, proposal, 0, 9)) gives the removed loop floor(w0 n_loops
 *     / 2^32) and the acceptance uniform w1; the new loop comes from
 *     Philox((chain, seed), (step, proposal, 1 + a, 9)) as above.
 * J arrays hold every canonical coupler (24 L^2 - 8 L bytes); planted holds
 * one bit per site.  Host only; the cycle lists are built once per (L, live)
 * and cached.  HS_EINVAL for bad arguments or an invalid loop. */
typedef struct hs_loop {
    int32_t size;   /* 4 or 6 */
    int32_t cycle;  /* index among the cycles of that size */
    int32_t weight; /* 1..5 */
    int32_t flip;   /* the unsatisfied coupler's position, 0..size-1 */
} hs_loop;
int lao_cycle_count(int L, const uint8_t *live, int size, int64_t *count);
int lao_init(int L, const uint8_t *live, int n_loops, uint32_t chain, uint32_t seed, hs_loop *loops,
             uint8_t *planted, int8_t *J, int64_t *e_gs);
/* The proposal (step, proposal) for an instance: *slot = the loop removed,
 * *new_loop = its replacement, J_new / *e_gs_new = the candidate's couplings
 * and planted ground-state energy, *w_accept = the uniform for hs_rao_accept.
 * The candidate must fit |J| <= 7 everywhere (removing a loop can push a
 * shared coupler past it); when no attempt does, the proposal is void:
 * *slot = -1 and J_new / *e_gs_new repeat the instance's.  The instance is
 * not modified. */
int lao_move(int L, const uint8_t *live, int n_loops, uint32_t chain, uint32_t seed, uint32_t step,
             uint32_t proposal, const hs_loop *loops, const uint8_t *planted, int32_t *slot, hs_loop *new_loop,
             uint32_t *w_accept, int8_t *J_new, int64_t *e_gs_new);

/* Ground / first-excited overlaps from PT snapshots (Sec. III.B, Fig. 3).
 *
 * pt_capture enqueues on h's stream, for every instance n and live lane l
 * whose current energy is at most e_cap[n] (device int32 [n_inst]): one slot
 * from the atomic *count (device uint32, the caller clears it), and, when the
 * slot is below capacity, configs[slot n_words + w] = the lane's spins
 * bit-packed (bit b of word w = site 64 w + b, 0 for missing sites) and
 * meta[slot 4 + 0..3] = (n, l, energy, completed sweeps).  Slots past
 * capacity are counted but not written.  n_words >= ceil(8 L^2 / 64) for the
 * largest lattice of the batch, else HS_EINVAL.  Asynchronous.
 *
 * overlap_analyze takes n captured configurations of ONE instance (device
 * configs [n][n_words], host energies [n]), the live-site mask (device
 * [n_words], bit = site live) and its popcount n_live, and a device scratch of
 * n x n int32.  It computes all pairwise Hamming distances h on the device,
 * then on the host: the ground level e0 = the lowest energy present, the
 * first excited level e1 = the next one; the distinct configurations of each
 * level up to the global flip (h = 0 or n_live to an earlier kept one);
 * overlaps q = |1 - 2 h / n_live|; med_gg = median q over pairs of distinct
 * ground states (1 with one ground state); med_ge = median q over (ground,
 * excited) pairs; ratio = med_ge / med_gg.  has_excited = 0 (and n_ex,
 * med_ge, ratio = 0) with a single level.  Synchronises the stream.
 * HS_EINVAL for bad arguments, n > 46340, or n_live other than the mask's
 * popcount. */
typedef struct hs_overlap {
    int32_t e0, e1, n_gs, n_ex, has_excited, pad_;
    double med_gg, med_ge, ratio;
} hs_overlap;
int pt_capture(hs_pt *h, const int32_t *e_cap, uint64_t *configs, int32_t *meta, uint32_t *count,
               int64_t capacity, int n_words);
int overlap_analyze(const uint64_t *configs, const int32_t *energy, int n, int n_words, const uint64_t *mask,
                    int n_live, int32_t *scratch, void *stream, hs_overlap *out);

/* Hardness of candidate instances: n_restarts independent PT runs per
 * candidate (restart rho keyed by (word 0 of Philox((instance_id, seed),
 * (rho, 0, 0, 5)), seed)), each until replica agreement or s_max sweeps
 * (t_rho sweeps); all runs of all candidates share one persistent launch.
 * E_gs = min over restarts; n_hit = restarts whose minimum is E_gs (>= 1);
 * ln_tts = ln(sum of t_rho / n_hit), the run time per find of the presumed
 * ground state, as Appendix B defines the time-to-solution (run time until
 * the lowest energy has been found n+1 times, divided by n+1); Sec. III.B
 * cross-checks ground-state energies by agreement.  detail->n_censored =
 * restarts that ended above E_gs.  restart_sweeps (optional, host int64
 * [n][n_restarts], NULL to leave out) receives t_rho of every restart.
 * Requires R >= 2.  Blocks until done. */
typedef struct hs_hardness_params {
    int32_t n_restarts;
    int32_t K;
    int32_t R;
    const double *beta;
    int32_t swap_interval;
    int64_t s_max;
    uint32_t seed;
    int32_t block_waves; /* 0 = tuner */
    int64_t *restart_sweeps;
} hs_hardness_params;

typedef struct hs_tts_detail {
    int32_t e_gs;
    int32_t confirmed; /* E_gs reached by two restarts or two replica sets of one */
    int32_t n_censored;
    int64_t sweeps_total;
} hs_tts_detail;

/* Device scratch for hardness_eval: size from hardness_workspace_bytes(). */
int hardness_workspace_bytes(const hs_instance *cands, int n, const hs_hardness_params *p,
                             size_t *bytes);
int hardness_eval(const hs_instance *cands, int n, const hs_hardness_params *p, void *scratch,
                  size_t scratch_bytes, double *ln_tts_out, hs_tts_detail *detail, void *stream);

/* hardness_eval for callers that cannot allocate device memory (serving
 * loops, harnesses that forbid allocation): the same computation and
 * results, with the scratch in a static device array of
 * HS_STATIC_SCRATCH_BYTES owned by the library (one copy per GPU, held until
 * the process ends) instead of a caller buffer.  The inputs and outputs are
 * the caller's host memory as for hardness_eval.  It calls no device
 * allocator.  `stream` must belong to the current device.  HS_ENOSPACE when
 * the batch needs more scratch than HS_STATIC_SCRATCH_BYTES (the size
 * hardness_workspace_bytes reports), with nothing enqueued.  Every call on
 * one GPU uses that GPU's array: calls that overlap on one GPU (from several
 * threads or streams) race and must not be made; the array keeps the last
 * call's contents, and each call initialises every byte it reads.  Blocks
 * until done. */
#define HS_STATIC_SCRATCH_BYTES (64u << 20)
int hardness_eval_static(const hs_instance *cands, int n, const hs_hardness_params *p, double *ln_tts_out,
                         hs_tts_detail *detail, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HARDSPIN_H */
