/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, scalar C implementation of the parallel-tempering (PT)
 * Metropolis hot path of "Practical engineering of hard spin-glass
 * instances" (Marshall, Martin-Mayor, Hen, arXiv:1605.03607).  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or constant generator with the GPU
 * library: it has its own Chimera builder, its own Philox, and it evaluates
 * every Metropolis / exchange threshold directly from the formula at the
 * point of use (no tables).
 *
 * What it computes, with the passage it follows:
 *   - Ising cost H = sum_<ij> J_ij s_i s_j over Chimera couplers, minimised,
 *     no local fields (Eq. 1, Sec. II).
 *   - Chimera graph C_L: L x L unit cells, each a K_{4,4}; vertex degree <= 6
 *     (Appendix A, caption of Fig. 8).
 *   - PT: N_T copies at temperatures T_1 < ... < T_NT, independent Metropolis
 *     updates in each copy, temperature swaps between neighbouring
 *     temperatures with probabilities satisfying detailed balance (Sec. II);
 *     "full-lattice Metropolis sweeps" followed by a temperature-exchange
 *     sweep (Sec. III.B).
 *   - Ground-state agreement as the stopping rule for a time-to-solution
 *     (Appendix B: halt after the lowest energy agrees n+1 times; Sec. III.B
 *     cross-check of PT ground-state energies).
 *   - RAO move and acceptance (Algorithm 1, Sec. II.A).
 *   - Brute-force enumeration of all 2^N configurations (definition of the
 *     ground state of Eq. 1; used only to pin the above).
 *
 * Readings where the paper is silent:
 *   spin bit b = 1 <-> s = -1; checkerboard sweep order (colour (r+c+u) mod 2,
 *   colour 0 first); Philox4x32-10 (Salmon et al., SC'11) with the counter
 *   layout below; a 32-bit uniform u = (hi16 << 16) | lo16 drawn from two
 *   Philox domains; accept iff dE <= 0 or u < floor(2^32 exp(-beta dE));
 *   one ascending exchange pass per replica set after every swap_interval-th
 *   sweep; time-to-solution = restart sweeps per restart that reached the
 *   ground state (Appendix B's run time per find of the minimum).
 *
 * Parity status: every function here is pinned by the not-gpu tests
 * against things other than itself: brute force, closed forms, Boltzmann
 * statistics (one and two cells, and the joint slot / configuration
 * distribution of PT), gauge invariance, Random123 known-answer vectors and
 * rocRAND's independent Philox, thresholds against 50-digit exponentials,
 * and for or_hardness_eval a zero-temperature limit recomputed from the
 * definitions (greedy descent, agreement stop, TTS) plus the free-coupling
 * closed form.  or_mutate's draws are pinned by their joint uniformity over
 * (live coupler, other letter).  Search trajectories as a whole are pinned
 * only through these parts.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Philox counter word 3 ("domain") values: every use of randomness has its
 * own domain, so no two uses can share a counter. */
#define OR_D_METRO_HI 0u
#define OR_D_SWAP 1u
#define OR_D_INIT 2u
#define OR_D_SWAP_EXTRA 3u
#define OR_D_MUTATE 4u
#define OR_D_RESTART 5u
#define OR_D_METRO_LO 7u

#define OR_MAX_LANES 64
#define OR_MAX_L 16

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as   */
/* easy as 1, 2, 3", SC'11).  Ten rounds of the 4x32 S-box with the two      */
/* published multipliers and the two Weyl key increments.                    */
/* ------------------------------------------------------------------------ */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        x0 = n0;
        x1 = n1;
        x2 = n2;
        x3 = n3;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

static uint32_t philox_word(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                            uint32_t key0, uint32_t key1, int word)
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {key0, key1};
    uint32_t out[4];
    or_philox(ctr, key, out);
    return out[word];
}

/* ------------------------------------------------------------------------ */
/* Chimera C_L (Appendix A, Fig. 8): unit cell (r, c), side u in {0, 1},    */
/* index k in [0, 4).  Site id i = 8 (L r + c) + 4 u + k.                    */
/*   intra-cell: (r,c,0,k) - (r,c,1,k') for all k, k'  (the K_{4,4})          */
/*   inter-cell: (r,c,0,k) - (r+1,c,0,k) and (r,c,1,k) - (r,c+1,1,k)          */
/* Canonical edge order: ascending (min id, max id).                         */
/* ------------------------------------------------------------------------ */
int or_num_sites(int L) { return 8 * L * L; }

static int site_id(int L, int r, int c, int u, int k) { return 8 * (L * r + c) + 4 * u + k; }

static int cmp_edge(const void *a, const void *b)
{
    const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
    if (x[0] != y[0]) return x[0] < y[0] ? -1 : 1;
    if (x[1] != y[1]) return x[1] < y[1] ? -1 : 1;
    return 0;
}

/* Writes the edges of the full C_L in canonical order into ei/ej (either may
 * be NULL to only count); returns the number of edges. */
int or_edges(int L, int32_t *ei, int32_t *ej)
{
    if (L < 1 || L > OR_MAX_L) return -1;
    int cap = 32 * L * L;
    int32_t *pairs = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)cap);
    int n = 0;
    for (int r = 0; r < L; ++r)
        for (int c = 0; c < L; ++c) {
            for (int k = 0; k < 4; ++k)
                for (int k2 = 0; k2 < 4; ++k2) {
                    pairs[2 * n] = site_id(L, r, c, 0, k);
                    pairs[2 * n + 1] = site_id(L, r, c, 1, k2);
                    ++n;
                }
            for (int k = 0; k < 4; ++k) {
                if (r + 1 < L) {
                    pairs[2 * n] = site_id(L, r, c, 0, k);
                    pairs[2 * n + 1] = site_id(L, r + 1, c, 0, k);
                    ++n;
                }
                if (c + 1 < L) {
                    pairs[2 * n] = site_id(L, r, c, 1, k);
                    pairs[2 * n + 1] = site_id(L, r, c + 1, 1, k);
                    ++n;
                }
            }
        }
    qsort(pairs, (size_t)n, 2 * sizeof(int32_t), cmp_edge);
    for (int e = 0; e < n; ++e) {
        if (ei) ei[e] = pairs[2 * e];
        if (ej) ej[e] = pairs[2 * e + 1];
    }
    free(pairs);
    return n;
}

/* Checkerboard colour of a site: (r + c + u) mod 2. */
static int site_colour(int L, int i)
{
    int cell = i / 8, u = (i / 4) % 2;
    int r = cell / L, c = cell % L;
    return (r + c + u) % 2;
}

/* An instance with its adjacency lists (edges touching a dead site dropped). */
typedef struct {
    int L, N, E;
    int32_t *ei, *ej;
    const int8_t *J;    /* over the full edge list */
    const uint8_t *live; /* N bytes, 1 = live; NULL = all live */
    int deg[8 * OR_MAX_L * OR_MAX_L];
    int nbr[8 * OR_MAX_L * OR_MAX_L][6];
    int jn[8 * OR_MAX_L * OR_MAX_L][6];
} Inst;

static int is_live(const Inst *g, int i) { return g->live == NULL || g->live[i] != 0; }

static Inst *inst_new(int L, const uint8_t *live, const int8_t *J)
{
    if (L < 1 || L > OR_MAX_L) return NULL;
    Inst *g = (Inst *)calloc(1, sizeof(Inst));
    g->L = L;
    g->N = or_num_sites(L);
    g->E = or_edges(L, NULL, NULL);
    g->ei = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->E);
    g->ej = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->E);
    or_edges(L, g->ei, g->ej);
    g->J = J;
    g->live = live;
    for (int e = 0; e < g->E; ++e) {
        int i = g->ei[e], j = g->ej[e];
        if (!is_live(g, i) || !is_live(g, j)) continue;
        g->nbr[i][g->deg[i]] = j;
        g->jn[i][g->deg[i]] = J[e];
        g->deg[i]++;
        g->nbr[j][g->deg[j]] = i;
        g->jn[j][g->deg[j]] = J[e];
        g->deg[j]++;
    }
    return g;
}

static void inst_free(Inst *g)
{
    if (!g) return;
    free(g->ei);
    free(g->ej);
    free(g);
}

/* Eq. 1 for one configuration: bits b[i] (1 <-> s_i = -1), sum over live
 * edges of J_e s_i s_j. */
static int64_t energy_bits(const Inst *g, const uint8_t *b)
{
    int64_t E = 0;
    for (int e = 0; e < g->E; ++e) {
        int i = g->ei[e], j = g->ej[e];
        if (!is_live(g, i) || !is_live(g, j)) continue;
        int si = b[i] ? -1 : 1, sj = b[j] ? -1 : 1;
        E += (int64_t)g->J[e] * si * sj;
    }
    return E;
}

int64_t or_energy(int L, const uint8_t *live, const int8_t *J, const uint8_t *bits)
{
    Inst *g = inst_new(L, live, J);
    if (!g) return INT64_MIN;
    int64_t E = energy_bits(g, bits);
    inst_free(g);
    return E;
}

/* ------------------------------------------------------------------------ */
/* Metropolis and exchange thresholds, evaluated from the formula each time. */
/* ------------------------------------------------------------------------ */

/* floor(2^32 * exp(-beta * dE)) for dE = 2m > 0; returned as uint64. */
uint64_t or_metro_threshold(double beta, int m)
{
    double x = exp(-(double)(2 * m) * beta);
    return (uint64_t)floor(ldexp(x, 32));
}

/* floor(2^32 * exp(-(beta_hi - beta_lo) * d)) for d > 0. */
uint64_t or_swap_threshold(double beta_lo, double beta_hi, int64_t d)
{
    double dbeta = beta_hi - beta_lo;
    double x = exp(-dbeta * (double)d);
    return (uint64_t)floor(ldexp(x, 32));
}

/* ------------------------------------------------------------------------ */
/* PT state (flat arrays so that Python can hold it):                       */
/*   spins[N]  word-major: bit l of spins[i] = spin bit of lane l at site i  */
/*   perm[K*R] perm[k*R + r] = lane currently at temperature slot (k, r)    */
/*   energy[64] per lane                                                     */
/*   emin[R], thit[R]: running minimum over the lanes of replica set r and  */
/*             the number of completed sweeps when it was first reached      */
/*   swap_acc[(K-1)*R] accepted exchanges per pair (k, k+1) and set r        */
/* Lane l belongs to replica set l / K for ever (exchanges stay in a set).   */
/* ------------------------------------------------------------------------ */

typedef struct {
    const Inst *g;
    int K, R, lanes;
    const double *beta;
    uint32_t key0, key1;
    uint8_t *b; /* [lanes][N] spin bits */
    uint8_t *perm;
    int64_t E[OR_MAX_LANES];
} PT;

static void unpack_spins(PT *p, const uint64_t *spins)
{
    int N = p->g->N;
    for (int l = 0; l < p->lanes; ++l)
        for (int i = 0; i < N; ++i)
            p->b[(size_t)l * N + i] = is_live(p->g, i) ? (uint8_t)((spins[i] >> l) & 1u) : 0;
}

static void pack_spins(const PT *p, uint64_t *spins)
{
    int N = p->g->N;
    for (int i = 0; i < N; ++i) {
        uint64_t w = 0;
        for (int l = 0; l < p->lanes; ++l)
            if (p->b[(size_t)l * N + i]) w |= (uint64_t)1 << l;
        spins[i] = w;
    }
}

/* Initial state.  Lane r*K + k starts at slot (k, r).  Bits come from the
 * caller (init_spins != NULL, word-major) or from Philox:
 *   bit 31 of word (i mod 4) of Philox(key, (0, i div 4, (k << 8) | r, D_INIT)).
 * Dead sites hold 0.  Energies are computed from Eq. 1. */
int or_pt_init(int L, const uint8_t *live, const int8_t *J, int K, int R,
               uint32_t key0, uint32_t key1, const uint64_t *init_spins,
               uint64_t *spins, uint8_t *perm, int32_t *energy, int32_t *emin,
               int64_t *thit, uint32_t *swap_acc)
{
    if (K < 1 || R < 1 || K * R > OR_MAX_LANES) return -1;
    Inst *g = inst_new(L, live, J);
    if (!g) return -1;
    int N = g->N;
    uint8_t *b = (uint8_t *)calloc((size_t)K * R * N, 1);
    for (int r = 0; r < R; ++r)
        for (int k = 0; k < K; ++k) {
            int l = r * K + k;
            perm[k * R + r] = (uint8_t)l;
            for (int i = 0; i < N; ++i) {
                if (!is_live(g, i)) continue;
                uint32_t bit;
                if (init_spins)
                    bit = (uint32_t)((init_spins[i] >> l) & 1u);
                else
                    bit = philox_word(0u, (uint32_t)(i / 4), ((uint32_t)k << 8) | (uint32_t)r,
                                      OR_D_INIT, key0, key1, i % 4) >> 31;
                b[(size_t)l * N + i] = (uint8_t)bit;
            }
        }
    for (int l = 0; l < OR_MAX_LANES; ++l) energy[l] = 0;
    for (int l = 0; l < K * R; ++l) energy[l] = (int32_t)energy_bits(g, b + (size_t)l * N);
    for (int r = 0; r < R; ++r) {
        int32_t m = energy[r * K];
        for (int k = 1; k < K; ++k)
            if (energy[r * K + k] < m) m = energy[r * K + k];
        emin[r] = m;
        thit[r] = 0;
    }
    for (int q = 0; q < (K - 1) * R; ++q) swap_acc[q] = 0;
    for (int i = 0; i < N; ++i) {
        uint64_t w = 0;
        for (int l = 0; l < K * R; ++l)
            if (b[(size_t)l * N + i]) w |= (uint64_t)1 << l;
        spins[i] = w;
    }
    free(b);
    inst_free(g);
    return 0;
}

/* One Metropolis update of live site i for the lane at slot (k, r) during
 * phase p of sweep t.  dE = E(after) - E(before) = -2 s_i h_i with
 * h_i = sum_j J_ij s_j (Eq. 1).  The uniform u is 32 bits:
 *   pair = (i div 8) div 2 (two neighbouring cells share one Philox call),
 *   q    = 4 * ((i div 8) mod 2) + (i mod 4) selects a 16-bit half,
 *   hi16 = half q of Philox(key, (t, 2 pair + p, (k << 8) | r, D_METRO_HI)),
 *   lo16 = half q of Philox(key, (t, 2 pair + p, (k << 8) | r, D_METRO_LO)),
 *   u    = hi16 * 2^16 + lo16.
 * Accept iff dE <= 0 or u < floor(2^32 exp(-beta_k dE)). */
static void metropolis_site(PT *p, int i, int k, int r, uint32_t t, int phase)
{
    const Inst *g = p->g;
    int N = g->N;
    int l = p->perm[k * p->R + r];
    uint8_t *b = p->b + (size_t)l * N;
    int si = b[i] ? -1 : 1;
    int h = 0;
    for (int d = 0; d < g->deg[i]; ++d) {
        int j = g->nbr[i][d];
        int sj = b[j] ? -1 : 1;
        h += g->jn[i][d] * sj;
    }
    int dE = -2 * si * h;
    int accept;
    if (dE <= 0) {
        accept = 1;
    } else {
        int cell = i / 8;
        uint32_t pair = (uint32_t)(cell / 2);
        int q = 4 * (cell % 2) + (i % 4);
        uint32_t c1 = 2u * pair + (uint32_t)phase;
        uint32_t c2 = ((uint32_t)k << 8) | (uint32_t)r;
        uint32_t whi = philox_word(t, c1, c2, OR_D_METRO_HI, p->key0, p->key1, q / 2);
        uint32_t wlo = philox_word(t, c1, c2, OR_D_METRO_LO, p->key0, p->key1, q / 2);
        uint32_t hi16 = (q % 2) ? (whi >> 16) : (whi & 0xFFFFu);
        uint32_t lo16 = (q % 2) ? (wlo >> 16) : (wlo & 0xFFFFu);
        uint64_t u = ((uint64_t)hi16 << 16) | (uint64_t)lo16;
        accept = u < or_metro_threshold(p->beta[k], dE / 2);
    }
    if (accept) {
        b[i] ^= 1u;
        p->E[l] += dE;
    }
}

/* Exchange sweep after sweep t: for each replica set r, one ascending pass
 * over neighbouring slot pairs (k, k+1).  With x at slot k, y at slot k+1 and
 * d = E_x - E_y, the swap is accepted iff d <= 0 or
 * u < floor(2^32 exp(-(beta_{k+1} - beta_k) d)), u = word 0 of
 * Philox(key, (t, k, r, D_SWAP)).  This ratio is the detailed-balance
 * acceptance for exchanging the two copies (Sec. II). */
static void swap_sweep(PT *p, uint32_t t, uint32_t use, uint32_t *swap_acc)
{
    for (int r = 0; r < p->R; ++r)
        for (int k = 0; k + 1 < p->K; ++k) {
            int x = p->perm[k * p->R + r], y = p->perm[(k + 1) * p->R + r];
            int64_t d = p->E[x] - p->E[y];
            int accept;
            if (d <= 0) {
                accept = 1;
            } else {
                uint32_t u = philox_word(t, (uint32_t)k, (uint32_t)r, use, p->key0, p->key1, 0);
                accept = (uint64_t)u < or_swap_threshold(p->beta[k], p->beta[k + 1], d);
            }
            if (accept) {
                p->perm[k * p->R + r] = (uint8_t)y;
                p->perm[(k + 1) * p->R + r] = (uint8_t)x;
                swap_acc[k * p->R + r]++;
            }
        }
}

/* Runs n_sweeps sweeps from the given state (all arrays are updated in
 * place; *t counts completed sweeps and is the Philox sweep counter).
 * site_order (optional, a permutation of 0..N-1) fixes the order in which the
 * sites of one colour are visited; any order gives identical results because
 * same-colour sites share no edge.  With stop_on_agreement the run ends after
 * the first sweep at which all replica sets have the same running minimum
 * and the completed sweep count is at least twice the largest first-hit
 * count (requires R >= 2); *stopped is then 1. */
int or_pt_run(int L, const uint8_t *live, const int8_t *J, int K, int R,
              const double *beta, uint32_t key0, uint32_t key1, int swap_interval,
              int64_t n_sweeps, int stop_on_agreement, const int32_t *site_order,
              uint64_t *spins, uint8_t *perm, int32_t *energy, int32_t *emin,
              int64_t *thit, uint32_t *swap_acc, int64_t *t, int32_t *stopped)
{
    if (K < 1 || R < 1 || K * R > OR_MAX_LANES) return -1;
    if (stop_on_agreement && R < 2) return -1;
    Inst *g = inst_new(L, live, J);
    if (!g) return -1;
    int N = g->N;
    PT p;
    p.g = g;
    p.K = K;
    p.R = R;
    p.lanes = K * R;
    p.beta = beta;
    p.key0 = key0;
    p.key1 = key1;
    p.b = (uint8_t *)calloc((size_t)p.lanes * N, 1);
    p.perm = perm;
    unpack_spins(&p, spins);
    for (int l = 0; l < OR_MAX_LANES; ++l) p.E[l] = l < p.lanes ? energy[l] : 0;
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    for (int i = 0; i < N; ++i) order[i] = site_order ? site_order[i] : i;
    *stopped = 0;

    for (int64_t s = 0; s < n_sweeps; ++s) {
        uint32_t tt = (uint32_t)*t;
        for (int phase = 0; phase < 2; ++phase)
            for (int oi = 0; oi < N; ++oi) {
                int i = order[oi];
                if (!is_live(g, i) || site_colour(L, i) != phase) continue;
                for (int r = 0; r < R; ++r)
                    for (int k = 0; k < K; ++k) metropolis_site(&p, i, k, r, tt, phase);
            }
        if (swap_interval > 0 && ((*t + 1) % swap_interval) == 0) swap_sweep(&p, tt, OR_D_SWAP, swap_acc);
        *t += 1;
        /* running minimum per replica set, after the sweep (and exchanges) */
        for (int r = 0; r < R; ++r) {
            int64_t m = p.E[r * K];
            for (int k = 1; k < K; ++k)
                if (p.E[r * K + k] < m) m = p.E[r * K + k];
            if (m < emin[r]) {
                emin[r] = (int32_t)m;
                thit[r] = *t;
            }
        }
        if (stop_on_agreement) {
            int agree = 1;
            int64_t tmax = 0;
            for (int r = 0; r < R; ++r) {
                if (emin[r] != emin[0]) agree = 0;
                if (thit[r] > tmax) tmax = thit[r];
            }
            if (agree && *t >= 2 * tmax) {
                *stopped = 1;
                break;
            }
        }
    }
    pack_spins(&p, spins);
    for (int l = 0; l < OR_MAX_LANES; ++l) energy[l] = l < p.lanes ? (int32_t)p.E[l] : 0;
    free(order);
    free(p.b);
    inst_free(g);
    return 0;
}

/* One exchange pass outside the sweep schedule, with its own Philox use
 * (counter word 3 = 3) and counter word 0 = the completed sweep count; the
 * lane energies are unchanged, so are the running minima. */
int or_pt_swap_extra(int L, const uint8_t *live, const int8_t *J, int K, int R,
                     const double *beta, uint32_t key0, uint32_t key1, uint64_t *spins,
                     uint8_t *perm, int32_t *energy, uint32_t *swap_acc, int64_t t)
{
    if (K < 1 || R < 1 || K * R > OR_MAX_LANES) return -1;
    Inst *g = inst_new(L, live, J);
    if (!g) return -1;
    PT p;
    p.g = g;
    p.K = K;
    p.R = R;
    p.lanes = K * R;
    p.beta = beta;
    p.key0 = key0;
    p.key1 = key1;
    p.b = NULL;
    p.perm = perm;
    (void)spins;
    for (int l = 0; l < OR_MAX_LANES; ++l) p.E[l] = l < p.lanes ? energy[l] : 0;
    swap_sweep(&p, (uint32_t)t, OR_D_SWAP_EXTRA, swap_acc);
    inst_free(g);
    return 0;
}

/* Energy of every lane recomputed from the packed spins (Eq. 1). */
int or_lane_energies(int L, const uint8_t *live, const int8_t *J, int lanes,
                     const uint64_t *spins, int32_t *energy)
{
    Inst *g = inst_new(L, live, J);
    if (!g) return -1;
    uint8_t *b = (uint8_t *)malloc((size_t)g->N);
    for (int l = 0; l < lanes; ++l) {
        for (int i = 0; i < g->N; ++i) b[i] = is_live(g, i) ? (uint8_t)((spins[i] >> l) & 1u) : 0;
        energy[l] = (int32_t)energy_bits(g, b);
    }
    free(b);
    inst_free(g);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Hardness: time-to-solution from independent PT restarts.                 */
/* Restart rho of a candidate with id `instance_id` uses the Philox key     */
/* (word 0 of Philox((instance_id, seed), (rho, 0, 0, D_RESTART)), seed),   */
/* starts from the Philox initial state and runs until agreement or s_max   */
/* sweeps (t_rho).  E_gs = min over restarts.  ln_tts = ln(sum t_rho /      */
/* n_hit), n_hit = restarts whose minimum is E_gs (Appendix B's run time    */
/* per repeated find of the presumed minimum).  r_tts: first sweep at which */
/* restart rho held E_gs (max 1), -1 if it never did (censored).            */
/* confirmed = 1 when E_gs was reached by two restarts, or by two replica   */
/* sets of one restart.                                                     */
/* ------------------------------------------------------------------------ */

int or_hardness_eval(int L, const uint8_t *live, const int8_t *J, uint32_t instance_id,
                     uint32_t seed, int n_restarts, int K, int R, const double *beta,
                     int swap_interval, int64_t s_max, double *ln_tts, int32_t *e_gs,
                     int32_t *confirmed, int32_t *r_emin, int64_t *r_tts, int64_t *r_sweeps)
{
    if (n_restarts < 1 || R < 2 || K * R > OR_MAX_LANES) return -1;
    int N = or_num_sites(L);
    uint64_t *spins = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)N);
    uint8_t perm[OR_MAX_LANES];
    int32_t energy[OR_MAX_LANES];
    int32_t emin[OR_MAX_LANES];
    int64_t thit[OR_MAX_LANES];
    uint32_t swap_acc[OR_MAX_LANES * OR_MAX_LANES];
    int32_t *rset_emin = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_restarts * R);
    int64_t *rset_thit = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_restarts * R);
    for (int rho = 0; rho < n_restarts; ++rho) {
        uint32_t rk = philox_word((uint32_t)rho, 0u, 0u, OR_D_RESTART, instance_id, seed, 0);
        if (or_pt_init(L, live, J, K, R, rk, seed, NULL, spins, perm, energy, emin, thit, swap_acc))
            return -1;
        int64_t t = 0;
        int32_t stopped = 0;
        if (or_pt_run(L, live, J, K, R, beta, rk, seed, swap_interval, s_max, 1, NULL, spins, perm,
                      energy, emin, thit, swap_acc, &t, &stopped))
            return -1;
        int32_t m = emin[0];
        for (int r = 0; r < R; ++r) {
            if (emin[r] < m) m = emin[r];
            rset_emin[rho * R + r] = emin[r];
            rset_thit[rho * R + r] = thit[r];
        }
        r_emin[rho] = m;
        r_sweeps[rho] = t;
    }
    int32_t gs = r_emin[0];
    for (int rho = 1; rho < n_restarts; ++rho)
        if (r_emin[rho] < gs) gs = r_emin[rho];
    int hits = 0, double_hit = 0;
    for (int rho = 0; rho < n_restarts; ++rho) {
        int64_t best = -1;
        int sets = 0;
        for (int r = 0; r < R; ++r)
            if (rset_emin[rho * R + r] == gs) {
                ++sets;
                if (best < 0 || rset_thit[rho * R + r] < best) best = rset_thit[rho * R + r];
            }
        if (sets >= 2) double_hit = 1;
        if (best >= 0) {
            ++hits;
            if (best < 1) best = 1;
            r_tts[rho] = best;
        } else {
            r_tts[rho] = -1;
        }
    }
    /* Appendix B: the time-to-solution is the run time spent until the
     * presumed minimum has been found n+1 times, divided by n+1.  Each
     * restart is one independent search that ends at its own presumed
     * minimum (replica agreement); so TTS = sweeps of all restarts / number
     * of restarts whose minimum is E_gs (at least one). */
    int64_t total = 0;
    for (int rho = 0; rho < n_restarts; ++rho) total += r_sweeps[rho];
    *ln_tts = log((double)(total > 0 ? total : 1) / (double)hits);
    *e_gs = gs;
    *confirmed = (hits >= 2 || double_hit) ? 1 : 0;
    free(rset_emin);
    free(rset_thit);
    free(spins);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* RAO move and acceptance (Algorithm 1, Sec. II.A).                        */
/* (w0, w1, w2, w3) = Philox((chain, seed), (step, proposal, 0, D_MUTATE)). */
/* Edge: the e-th live edge in canonical order, e = floor(w0 E_live / 2^32). */
/* New value: element floor(w1 (|A|-1) / 2^32) of the ascending alphabet A  */
/* with the current value removed.  With A = {-1, +1} this is the sign flip */
/* of Algorithm 1.  w2 is the uniform for the acceptance test.              */
/* ------------------------------------------------------------------------ */
int or_mutate(int L, const uint8_t *live, const int8_t *J, const int8_t *alphabet, int n_alpha,
              uint32_t chain, uint32_t seed, uint32_t step, uint32_t proposal, int32_t *edge,
              int8_t *old_j, int8_t *new_j, uint32_t *w_accept)
{
    if (n_alpha < 2 || n_alpha > 255) return -1;
    for (int a = 0; a < n_alpha; ++a)
        for (int b = 0; b < a; ++b)
            if (alphabet[a] == alphabet[b]) return -1; /* the alphabet is a set */
    Inst *g = inst_new(L, live, J);
    if (!g) return -1;
    uint32_t ctr[4] = {step, proposal, 0u, OR_D_MUTATE};
    uint32_t key[2] = {chain, seed};
    uint32_t w[4];
    or_philox(ctr, key, w);
    int n_live = 0;
    for (int e = 0; e < g->E; ++e)
        if (is_live(g, g->ei[e]) && is_live(g, g->ej[e])) ++n_live;
    if (n_live == 0) {
        inst_free(g);
        return -1;
    }
    int pick = (int)(((uint64_t)w[0] * (uint64_t)n_live) >> 32);
    int e_sel = -1;
    for (int e = 0, seen = 0; e < g->E; ++e) {
        if (!(is_live(g, g->ei[e]) && is_live(g, g->ej[e]))) continue;
        if (seen == pick) {
            e_sel = e;
            break;
        }
        ++seen;
    }
    int8_t cur = J[e_sel];
    int8_t rest[256];
    int nr = 0;
    for (int a = 0; a < n_alpha; ++a)
        if (alphabet[a] != cur) rest[nr++] = alphabet[a];
    /* the move replaces the current value by another value of the alphabet,
       so the current value must be one of its letters */
    if (nr != n_alpha - 1) {
        inst_free(g);
        return -1;
    }
    int idx = (int)(((uint64_t)w[1] * (uint64_t)(n_alpha - 1)) >> 32);
    *edge = e_sel;
    *old_j = cur;
    *new_j = rest[idx];
    *w_accept = w[2];
    inst_free(g);
    return 0;
}

/* Algorithm 1's acceptance with TTS replaced by ln TTS and beta = 1 / t_s:
 * accept iff delta >= 0 or w < floor(2^32 exp(delta / t_s)).  An infinite
 * (censored) new value is always accepted; infinite minus infinite counts as
 * delta = 0. */
int or_rao_accept(double ln_cur, double ln_new, double t_s, uint32_t w)
{
    double delta;
    if (isinf(ln_cur) && isinf(ln_new))
        delta = 0.0;
    else
        delta = ln_new - ln_cur;
    if (delta >= 0.0) return 1;
    double x = exp(delta / t_s);
    uint64_t th = (uint64_t)floor(ldexp(x, 32));
    return (uint64_t)w < th;
}

/* ------------------------------------------------------------------------ */
/* Brute force over all 2^N_live configurations (N_live <= 26).            */
/* energies: optional, receives E for every configuration, indexed by the   */
/* bits of the live sites in ascending site order (bit n of the index is    */
/* the n-th live site).  hist_e / hist_n: distinct energy levels ascending  */
/* and their multiplicities (capacity hist_cap).                            */
/* ------------------------------------------------------------------------ */
int or_enumerate(int L, const uint8_t *live, const int8_t *J, int32_t *energies,
                 int32_t *hist_e, int64_t *hist_n, int hist_cap, int32_t *n_levels)
{
    Inst *g = inst_new(L, live, J);
    if (!g) return -1;
    int N = g->N;
    int ids[8 * OR_MAX_L * OR_MAX_L];
    int nl = 0;
    for (int i = 0; i < N; ++i)
        if (is_live(g, i)) ids[nl++] = i;
    if (nl > 26) {
        inst_free(g);
        return -1;
    }
    /* energy levels lie in [-sum|J|, +sum|J|]: count them in a dense array */
    int64_t jsum = 0;
    for (int e = 0; e < g->E; ++e)
        if (is_live(g, g->ei[e]) && is_live(g, g->ej[e])) jsum += abs(g->J[e]);
    int64_t *count = (int64_t *)calloc((size_t)(2 * jsum + 1), sizeof(int64_t));
    uint8_t *b = (uint8_t *)calloc((size_t)N, 1);
    uint64_t total = (uint64_t)1 << nl;
    for (uint64_t s = 0; s < total; ++s) {
        for (int n = 0; n < nl; ++n) b[ids[n]] = (uint8_t)((s >> n) & 1u);
        int64_t E = energy_bits(g, b);
        if (energies) energies[s] = (int32_t)E;
        count[E + jsum]++;
    }
    int nlev = 0;
    for (int64_t v = 0; v <= 2 * jsum; ++v) {
        if (count[v] == 0) continue;
        if (nlev < hist_cap) {
            hist_e[nlev] = (int32_t)(v - jsum);
            hist_n[nlev] = count[v];
        }
        ++nlev;
    }
    *n_levels = nlev;
    free(count);
    free(b);
    inst_free(g);
    return 0;
}
