/* Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
 * CPU oracle (oracle/oracle.c): calls every entry point on small Chimera
 * instances, with missing sites, up to 64 lanes, the agreement stop, extra
 * exchange passes, brute force, mutation (valid and invalid alphabets) and
 * hardness evaluation.  Exits 0 when every call behaves; the sanitizers
 * abort on the first invalid access or undefined operation. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int or_num_sites(int L);
int or_edges(int L, int32_t *ei, int32_t *ej);
int64_t or_energy(int L, const uint8_t *live, const int8_t *J, const uint8_t *bits);
uint64_t or_metro_threshold(double beta, int m);
uint64_t or_swap_threshold(double beta_lo, double beta_hi, int64_t d);
int or_pt_init(int L, const uint8_t *live, const int8_t *J, int K, int R, uint32_t key0, uint32_t key1,
               const uint64_t *init_spins, uint64_t *spins, uint8_t *perm, int32_t *energy, int32_t *emin,
               int64_t *thit, uint32_t *swap_acc);
int or_pt_run(int L, const uint8_t *live, const int8_t *J, int K, int R, const double *beta, uint32_t key0,
              uint32_t key1, int swap_interval, int64_t n_sweeps, int stop_on_agreement, const int32_t *site_order,
              uint64_t *spins, uint8_t *perm, int32_t *energy, int32_t *emin, int64_t *thit, uint32_t *swap_acc,
              int64_t *t, int32_t *stopped);
int or_pt_swap_extra(int L, const uint8_t *live, const int8_t *J, int K, int R, const double *beta, uint32_t key0,
                     uint32_t key1, uint64_t *spins, uint8_t *perm, int32_t *energy, uint32_t *swap_acc, int64_t t);
int or_lane_energies(int L, const uint8_t *live, const int8_t *J, int lanes, const uint64_t *spins, int32_t *energy);
int or_hardness_eval(int L, const uint8_t *live, const int8_t *J, uint32_t instance_id, uint32_t seed,
                     int n_restarts, int K, int R, const double *beta, int swap_interval, int64_t s_max,
                     double *ln_tts, int32_t *e_gs, int32_t *confirmed, int32_t *r_emin, int64_t *r_tts,
                     int64_t *r_sweeps);
int or_mutate(int L, const uint8_t *live, const int8_t *J, const int8_t *alphabet, int n_alpha, uint32_t chain,
              uint32_t seed, uint32_t step, uint32_t proposal, int32_t *edge, int8_t *old_j, int8_t *new_j,
              uint32_t *w_accept);
int or_rao_accept(double ln_cur, double ln_new, double t_s, uint32_t w);
int or_enumerate(int L, const uint8_t *live, const int8_t *J, int32_t *energies, int32_t *hist_e, int64_t *hist_n,
                 int hist_cap, int32_t *n_levels);

static int fails = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++fails;                                                     \
        }                                                                \
    } while (0)

static uint32_t lcg(uint32_t *s)
{
    *s = *s * 1664525u + 1013904223u;
    return *s >> 8;
}

static void ladder(int K, double lo, double hi, double *b)
{
    for (int k = 0; k < K; ++k) b[k] = K == 1 ? lo : lo + (hi - lo) * k / (K - 1);
}

int main(void)
{
    uint32_t s = 12345;
    static const int shapes[][3] = {{1, 1, 64}, {1, 64, 1}, {2, 8, 2}, {3, 5, 3}, {4, 16, 4}, {2, 32, 2}};
    for (size_t n = 0; n < sizeof(shapes) / sizeof(shapes[0]); ++n) {
        const int L = shapes[n][0], K = shapes[n][1], R = shapes[n][2];
        const int N = or_num_sites(L), E = or_edges(L, NULL, NULL);
        CHECK(E == 24 * L * L - 8 * L);
        int32_t *ei = malloc(sizeof(int32_t) * E), *ej = malloc(sizeof(int32_t) * E);
        CHECK(or_edges(L, ei, ej) == E);
        int8_t *J = malloc(E);
        uint8_t *live = malloc(N), *bits = malloc(N);
        const int8_t pm7[14] = {-7, -6, -5, -4, -3, -2, -1, 1, 2, 3, 4, 5, 6, 7};
        for (int e = 0; e < E; ++e) J[e] = pm7[lcg(&s) % 14];
        for (int i = 0; i < N; ++i) {
            live[i] = (lcg(&s) % 10) != 0;
            bits[i] = lcg(&s) & 1;
        }
        (void)or_energy(L, live, J, bits);
        (void)or_energy(L, NULL, J, bits);
        double beta[64];
        ladder(K, 0.1, 3.0, beta);
        uint64_t *spins = calloc(N, 8);
        uint8_t perm[64];
        int32_t energy[64], emin[64], re[64];
        int64_t thit[64], t = 0;
        uint32_t sacc[64 * 64];
        int32_t stopped = 0;
        CHECK(or_pt_init(L, live, J, K, R, 7, 9, NULL, spins, perm, energy, emin, thit, sacc) == 0);
        CHECK(or_pt_run(L, live, J, K, R, beta, 7, 9, 1, 25, 0, NULL, spins, perm, energy, emin, thit, sacc, &t,
                        &stopped) == 0);
        CHECK(or_pt_swap_extra(L, live, J, K, R, beta, 7, 9, spins, perm, energy, sacc, t) == 0);
        CHECK(or_lane_energies(L, live, J, K * R, spins, re) == 0);
        for (int l = 0; l < K * R; ++l) CHECK(re[l] == energy[l]);
        if (R >= 2) {
            CHECK(or_pt_run(L, live, J, K, R, beta, 7, 9, 3, 200, 1, NULL, spins, perm, energy, emin, thit, sacc,
                            &t, &stopped) == 0);
            double ln;
            int32_t gs, conf, r_emin[3];
            int64_t r_tts[3], r_sw[3];
            CHECK(or_hardness_eval(L, live, J, 3, 4, 3, K, R, beta, 1, 300, &ln, &gs, &conf, r_emin, r_tts, r_sw) ==
                  0);
        }
        const int8_t rep[3] = {-1, 1, 1};
        int32_t edge;
        int8_t oj, nj;
        uint32_t w;
        for (int step = 0; step < 50; ++step) {
            CHECK(or_mutate(L, live, J, pm7, 14, 1, 2, step, 0, &edge, &oj, &nj, &w) == 0);
            CHECK(oj == J[edge] && nj != oj);
            CHECK(or_mutate(L, live, J, rep, 3, 1, 2, step, 0, &edge, &oj, &nj, &w) == -1);
        }
        free(ei);
        free(ej);
        free(J);
        free(live);
        free(bits);
        free(spins);
    }
    {
        const int L = 1, E = 16;
        int8_t J[16];
        for (int e = 0; e < E; ++e) J[e] = (int8_t)((int)(lcg(&s) % 7) - 3);
        int32_t *en = malloc(sizeof(int32_t) * 256), he[300], nl = 0;
        int64_t hn[300];
        CHECK(or_enumerate(L, NULL, J, en, he, hn, 300, &nl) == 0 && nl > 0);
        free(en);
    }
    for (int m = 1; m <= 42; ++m) CHECK(or_metro_threshold(0.1, m) < (1ull << 32));
    CHECK(or_swap_threshold(0.1, 0.2, 1) > 0);
    CHECK(or_rao_accept(1.0, 2.0, 0.5, 0xFFFFFFFFu) == 1);
    uint32_t ctr[4] = {0, 0, 0, 0}, key[2] = {0, 0}, out[4];
    or_philox(ctr, key, out);
    if (fails) return 1;
    printf("oracle sanitizer driver: ok\n");
    return 0;
}
