// Host side of libhardspin: Chimera graph, per-instance coupling words,
// Metropolis / exchange threshold tables, the RAO move and acceptance.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "hs_internal.h"

namespace hs {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// products with the published multipliers, key bumped by the Weyl constants.
void philox_host(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t ka = key[0], kb = key[1];
    for (int i = 0; i < 10; ++i) {
        const uint64_t a = uint64_t(0xD2511F53u) * c[0];
        const uint64_t b = uint64_t(0xCD9E8D57u) * c[2];
        const uint32_t n0 = uint32_t(b >> 32) ^ c[1] ^ ka;
        const uint32_t n2 = uint32_t(a >> 32) ^ c[3] ^ kb;
        c[1] = uint32_t(b);
        c[3] = uint32_t(a);
        c[0] = n0;
        c[2] = n2;
        ka += 0x9E3779B9u;
        kb += 0xBB67AE85u;
    }
    std::memcpy(out, c, sizeof(c));
}

static inline int sid(int L, int r, int c, int u, int k) { return 8 * (L * r + c) + 4 * u + k; }

void chimera_edges(int L, std::vector<int32_t> &ei, std::vector<int32_t> &ej)
{
    std::vector<std::pair<int32_t, int32_t>> e;
    e.reserve(size_t(24 * L * L));
    for (int r = 0; r < L; ++r)
        for (int c = 0; c < L; ++c) {
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) e.emplace_back(sid(L, r, c, 0, a), sid(L, r, c, 1, b));
            for (int k = 0; k < 4; ++k) {
                if (r + 1 < L) e.emplace_back(sid(L, r, c, 0, k), sid(L, r + 1, c, 0, k));
                if (c + 1 < L) e.emplace_back(sid(L, r, c, 1, k), sid(L, r, c + 1, 1, k));
            }
        }
    std::sort(e.begin(), e.end());
    ei.resize(e.size());
    ej.resize(e.size());
    for (size_t n = 0; n < e.size(); ++n) {
        ei[n] = e[n].first;
        ej[n] = e[n].second;
    }
}

static inline uint32_t put_byte(uint32_t w, int byte, int v)
{
    return w | (uint32_t(uint8_t(int8_t(v))) << (8 * byte));
}

int build_instance(const hs_instance &in, HostInstance &out, std::string &err)
{
    const int L = in.L;
    if (L < 1 || L > HS_MAX_L) {
        err = "L must be in 1..16";
        return HS_EUNSUPPORTED;
    }
    if (in.J == nullptr) {
        err = "J is NULL";
        return HS_EINVAL;
    }
    std::vector<int32_t> ei, ej;
    chimera_edges(L, ei, ej);
    const int N = 8 * L * L, E = int(ei.size());
    auto live = [&](int i) { return in.live == nullptr || in.live[i] != 0; };
    // coupling of site i to each neighbour, 0 if absent
    std::vector<int> jmap(size_t(N) * 6, 0), nmap(size_t(N) * 6, -1), deg(N, 0);
    std::vector<uint32_t> edges;
    for (int e = 0; e < E; ++e) {
        const int j = in.J[e];
        if (j < -HS_MAX_ABS_J || j > HS_MAX_ABS_J) {
            err = "|J| > 7 is not supported";
            return HS_EUNSUPPORTED;
        }
        const int a = ei[e], b = ej[e];
        if (!live(a) || !live(b)) continue;
        nmap[size_t(a) * 6 + deg[a]] = b;
        jmap[size_t(a) * 6 + deg[a]++] = j;
        nmap[size_t(b) * 6 + deg[b]] = a;
        jmap[size_t(b) * 6 + deg[b]++] = j;
        edges.push_back(uint32_t(a) | (uint32_t(b) << 12) | (uint32_t(uint8_t(int8_t(j))) << 24));
    }
    auto coupling = [&](int i, int j) {
        for (int d = 0; d < deg[i]; ++d)
            if (nmap[size_t(i) * 6 + d] == j) return jmap[size_t(i) * 6 + d];
        return 0;
    };
    out.L = L;
    out.N = N;
    out.E = E;
    out.ncell = L * L;
    out.jw.assign(size_t(out.ncell) * 16, 0u);
    out.live.assign(size_t(out.ncell) * 2, 0u);
    out.edges = std::move(edges);
    for (int r = 0; r < L; ++r)
        for (int c = 0; c < L; ++c) {
            const int cell = L * r + c;
            for (int u = 0; u < 2; ++u) {
                uint32_t *w = &out.jw[size_t(cell * 2 + u) * 8];
                uint32_t lm = 0;
                // neighbour cells along this side's direction (A before, B after)
                const int ra = u == 0 ? r - 1 : r, ca = u == 0 ? c : c - 1;
                const int rb = u == 0 ? r + 1 : r, cb = u == 0 ? c : c + 1;
                for (int k = 0; k < 4; ++k) {
                    const int i = sid(L, r, c, u, k);
                    if (live(i)) lm |= 0xFEu << (8 * k);
                    uint32_t jin = 0;
                    for (int k2 = 0; k2 < 4; ++k2)
                        jin = put_byte(jin, k2, -4 * coupling(i, sid(L, r, c, 1 - u, k2)));
                    int ja = 0, jb = 0;
                    if (ra >= 0 && ca >= 0) ja = coupling(i, sid(L, ra, ca, u, k));
                    if (rb < L && cb < L) jb = coupling(i, sid(L, rb, cb, u, k));
                    // vertical / horizontal neighbours are read from the perm'd
                    // word [A.k0, A.k1, B.k0, B.k1] (k in {0,1}) or
                    // [A.k2, A.k3, B.k2, B.k3] (k in {2,3})
                    const int lo = k & 1;
                    uint32_t jv = 0;
                    jv = put_byte(jv, lo, -4 * ja);
                    jv = put_byte(jv, 2 + lo, -4 * jb);
                    w[k] = jin;
                    w[4 + k] = jv;
                }
                out.live[size_t(cell * 2 + u)] = lm;
            }
        }
    return HS_OK;
}

// Wavefront task table of an L x L lattice processed by nwaves wavefronts:
// wavefront w, phase p, iteration i updates cell pair j = w + i nwaves
// (cells 2j, 2j+1 in row-major order).  Entry (16 words): Philox counter word
// (j << 1 | p), quad indices q0 | q1 << 16 (q1 = 0xFFFF without a second
// cell), then for each cell the LDS byte offsets (row x 256) of the spin rows
// own, opposite, neighbour A and neighbour B (row 2 L^2 is the zero row);
// byte offsets, so the kernel adds them to its column address as they are.
void build_tasks(int L, int nwaves, std::vector<uint32_t> &out, int &iters)
{
    const int ncell = L * L, npairs = (ncell + 1) / 2, zero = 2 * ncell;
    iters = (npairs + nwaves - 1) / nwaves;
    out.assign(size_t(nwaves) * 2 * iters * 16, 0u);
    for (int w = 0; w < nwaves; ++w)
        for (int p = 0; p < 2; ++p)
            for (int it = 0; it < iters; ++it) {
                const int j = w + it * nwaves;
                if (j >= npairs) continue;
                uint32_t *e = &out[((size_t(w) * 2 + p) * iters + it) * 16];
                e[0] = (uint32_t(j) << 1) | uint32_t(p);
                uint32_t qs[2] = {0xFFFFu, 0xFFFFu};
                for (int h = 0; h < 2; ++h) {
                    const int cell = 2 * j + h;
                    if (cell >= ncell) continue;
                    const int r = cell / L, c = cell % L, u = (r + c + p) & 1;
                    const int own = cell * 2 + u, oth = cell * 2 + 1 - u;
                    const int a = u == 0 ? (r > 0 ? (cell - L) * 2 : zero) : (c > 0 ? (cell - 1) * 2 + 1 : zero);
                    const int b = u == 0 ? (r + 1 < L ? (cell + L) * 2 : zero) : (c + 1 < L ? (cell + 1) * 2 + 1 : zero);
                    qs[h] = uint32_t(own);
                    e[2 + 4 * h] = uint32_t(own) * 256u;
                    e[3 + 4 * h] = uint32_t(oth) * 256u;
                    e[4 + 4 * h] = uint32_t(a) * 256u;
                    e[5 + 4 * h] = uint32_t(b) * 256u;
                }
                e[1] = qs[0] | (qs[1] << 16);
            }
}

uint64_t metro_threshold(double beta, int m)
{
    const double x = std::exp(-double(2 * m) * beta);
    return uint64_t(std::floor(std::ldexp(x, 32)));
}

uint64_t swap_threshold(double beta_lo, double beta_hi, int64_t d)
{
    const double db = beta_hi - beta_lo;
    const double x = std::exp(-db * double(d));
    return uint64_t(std::floor(std::ldexp(x, 32)));
}

// d_cap bounds the exchange tables: no two configurations of any instance
// using this ladder differ in energy by more than d_cap (2 sum |J| over its
// live couplers), so entries beyond it are never read and a closely spaced
// ladder cannot make the table grow without bound.
void build_tables(int K, const double *beta, int64_t d_cap, HostTables &t)
{
    t.K = K;
    t.beta.assign(beta, beta + K);
    t.thi.assign(size_t(K) * kMRow, 0);
    t.tfull.assign(size_t(K) * kMRow, 0);
    for (int k = 0; k < K; ++k)
        for (int m = -kMaxM; m <= kMaxM; ++m) {
            const size_t at = size_t(k) * kMRow + size_t(m + kMaxM);
            if (m <= 0) {
                t.thi[at] = kAlways;
                t.tfull[at] = 0xFFFFFFFFu;
            } else {
                const uint64_t T = metro_threshold(beta[k], m);
                t.thi[at] = uint32_t(T >> 16);
                t.tfull[at] = uint32_t(T);
            }
        }
    t.ts_row.assign(K, 0);
    t.ts_dhi.assign(K, 0);
    t.ts_dmax.assign(K, 0);
    t.ts_full_row.assign(K, 0);
    t.ts_rate.assign(K, 0.0f);
    t.ts_hi.clear();
    t.ts_full.clear();
    for (int k = 0; k + 1 < K; ++k) {
        t.ts_row[k] = int32_t(t.ts_hi.size());
        t.ts_full_row[k] = int32_t(t.ts_full.size());
        t.ts_rate[k] = float(std::log(2.0) / (beta[k + 1] - beta[k]));
        int64_t d = 1;
        for (; d <= d_cap; ++d) {
            const uint64_t T = swap_threshold(beta[k], beta[k + 1], d);
            if (T == 0) break;
            t.ts_full.push_back(uint32_t(T));
            if ((T >> 16) > 0) {
                t.ts_hi.push_back(uint16_t(T >> 16));
                t.ts_dhi[k] = int32_t(d);
            }
        }
        t.ts_dmax[k] = int32_t(d - 1);
    }
    t.ts_hi.push_back(0);                          // a clamped read of an empty last row stays inside
    if (t.ts_hi.size() % 2) t.ts_hi.push_back(0);  // keep uint32 alignment
}

}  // namespace hs

using namespace hs;

extern "C" {

int hs_version(void) { return 10000; }

const char *hs_last_error(void) { return g_err.c_str(); }

int instance_mutate(const hs_instance *in, const int8_t *alphabet, int n_alpha, uint32_t chain,
                    uint32_t seed, uint32_t step, uint32_t proposal, hs_mutation *out)
{
    if (in == nullptr || alphabet == nullptr || out == nullptr || n_alpha < 2 || n_alpha > 255)
        return fail(HS_EINVAL, "instance_mutate: bad arguments");
    if (in->L < 1 || in->L > HS_MAX_L || in->J == nullptr)
        return fail(HS_EINVAL, "instance_mutate: bad instance");
    for (int a = 0; a < n_alpha; ++a)
        for (int b = 0; b < a; ++b)
            if (alphabet[a] == alphabet[b]) return fail(HS_EINVAL, "instance_mutate: repeated alphabet value");
    std::vector<int32_t> ei, ej;
    chimera_edges(in->L, ei, ej);
    auto live = [&](int i) { return in->live == nullptr || in->live[i] != 0; };
    std::vector<int32_t> live_edges;
    for (size_t e = 0; e < ei.size(); ++e)
        if (live(ei[e]) && live(ej[e])) live_edges.push_back(int32_t(e));
    if (live_edges.empty()) return fail(HS_EINVAL, "instance_mutate: no live coupler");
    const uint32_t ctr[4] = {step, proposal, 0u, kUseMutate};
    const uint32_t key[2] = {chain, seed};
    uint32_t w[4];
    philox_host(ctr, key, w);
    const size_t pick = size_t((uint64_t(w[0]) * live_edges.size()) >> 32);
    const int e = live_edges[pick];
    const int8_t cur = in->J[e];
    std::vector<int8_t> rest;
    for (int a = 0; a < n_alpha; ++a)
        if (alphabet[a] != cur) rest.push_back(alphabet[a]);
    // the alphabet minus the current value must have n_alpha - 1 entries:
    // distinct letters, one of them the current value
    if (rest.size() + 1 != size_t(n_alpha))
        return fail(HS_EINVAL, "instance_mutate: the alphabet must hold distinct values, one of them the "
                               "coupler's current value");
    const size_t idx = size_t((uint64_t(w[1]) * uint64_t(n_alpha - 1)) >> 32);
    out->edge = e;
    out->old_j = cur;
    out->new_j = rest[idx];
    out->w_accept = w[2];
    return HS_OK;
}

int hs_rao_accept(double ln_cur, double ln_new, double t_s, uint32_t w)
{
    const double delta = (std::isinf(ln_cur) && std::isinf(ln_new)) ? 0.0 : ln_new - ln_cur;
    if (delta >= 0.0) return 1;
    const uint64_t th = uint64_t(std::floor(std::ldexp(std::exp(delta / t_s), 32)));
    return uint64_t(w) < th ? 1 : 0;
}

}  // extern "C"
