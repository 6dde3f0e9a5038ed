// Planted-solution instances and loop moves of Loop Adaptive Optimization
// (Sec. IV, Algorithm 2).  Host code: the loops are a few hundred small
// cycles, and parallel tempering (the device path) scores the instances.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hs_internal.h"

namespace hs {
namespace {

constexpr uint32_t kUseLaoInit = 8;
constexpr uint32_t kUseLaoMove = 9;
constexpr uint32_t kP4Threshold = 429496730u;  // a 4-cycle with probability ~0.1
constexpr int kWeightMax = 5;
constexpr int kJCap = 7;
constexpr int kMaxAttempts = 64;

struct Cycles {
    std::vector<std::vector<int32_t>> c4, c6;  // ascending coupler indices, sorted
};

// Cycles of 4 and 6 couplers of the live Chimera graph, from its geometry:
// 4-cycles inside a cell (two sites on each side); 6-cycles inside a cell
// (a K_{3,3}'s Hamiltonian cycles) and through two neighbouring cells (two
// inter-cell couplers k, k' joined by one site of the other side in each cell).
Cycles build_cycles(int L, const uint8_t *live)
{
    std::vector<int32_t> ei, ej;
    chimera_edges(L, ei, ej);
    std::map<std::pair<int, int>, int32_t> eid;
    for (size_t e = 0; e < ei.size(); ++e) eid[{ei[e], ej[e]}] = int32_t(e);
    auto site = [&](int r, int c, int u, int k) { return 8 * (L * r + c) + 4 * u + k; };
    auto alive = [&](int i) { return live == nullptr || live[i] != 0; };
    auto edge = [&](int a, int b) { return eid.at({std::min(a, b), std::max(a, b)}); };
    std::vector<std::vector<int32_t>> c4, c6;
    auto add = [&](std::vector<std::vector<int32_t>> &dst, const std::vector<int> &path) {
        for (int v : path)
            if (!alive(v)) return;
        std::vector<int32_t> es;
        for (size_t p = 0; p < path.size(); ++p) es.push_back(edge(path[p], path[(p + 1) % path.size()]));
        std::sort(es.begin(), es.end());
        dst.push_back(es);
    };
    for (int r = 0; r < L; ++r)
        for (int c = 0; c < L; ++c) {
            for (int k1 = 0; k1 < 4; ++k1)
                for (int k2 = k1 + 1; k2 < 4; ++k2)
                    for (int x1 = 0; x1 < 4; ++x1)
                        for (int x2 = x1 + 1; x2 < 4; ++x2)
                            add(c4, {site(r, c, 0, k1), site(r, c, 1, x1), site(r, c, 0, k2), site(r, c, 1, x2)});
            // K_{3,3} Hamiltonian cycles a-p-b-q-d-s-a (duplicates removed below)
            for (int skip0 = 0; skip0 < 4; ++skip0)
                for (int skip1 = 0; skip1 < 4; ++skip1) {
                    std::vector<int> A, X;
                    for (int k = 0; k < 4; ++k) {
                        if (k != skip0) A.push_back(k);
                        if (k != skip1) X.push_back(k);
                    }
                    std::vector<int> perm = X;
                    do {
                        add(c6, {site(r, c, 0, A[0]), site(r, c, 1, perm[0]), site(r, c, 0, A[1]),
                                 site(r, c, 1, perm[1]), site(r, c, 0, A[2]), site(r, c, 1, perm[2])});
                        add(c6, {site(r, c, 0, A[0]), site(r, c, 1, perm[0]), site(r, c, 0, A[2]),
                                 site(r, c, 1, perm[1]), site(r, c, 0, A[1]), site(r, c, 1, perm[2])});
                    } while (std::next_permutation(perm.begin(), perm.end()));
                }
            for (int dir = 0; dir < 2; ++dir) {  // dir 0: (r+1, c) through side 0; dir 1: (r, c+1) through side 1
                const int r2 = r + (dir == 0), c2 = c + (dir == 1);
                if (r2 >= L || c2 >= L) continue;
                const int u = dir, o = 1 - dir;
                for (int k = 0; k < 4; ++k)
                    for (int k2 = k + 1; k2 < 4; ++k2)
                        for (int x = 0; x < 4; ++x)
                            for (int y = 0; y < 4; ++y)
                                add(c6, {site(r, c, u, k), site(r2, c2, u, k), site(r2, c2, o, x), site(r2, c2, u, k2),
                                         site(r, c, u, k2), site(r, c, o, y)});
            }
        }
    for (auto *v : {&c4, &c6}) {
        std::sort(v->begin(), v->end());
        v->erase(std::unique(v->begin(), v->end()), v->end());
    }
    return Cycles{std::move(c4), std::move(c6)};
}

const Cycles &cycles_of(int L, const uint8_t *live)
{
    static std::mutex mu;
    static std::map<std::string, Cycles> cache;
    std::string key = std::to_string(L) + ":";
    if (live != nullptr) key.append(reinterpret_cast<const char *>(live), size_t(8 * L * L));
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it == cache.end()) it = cache.emplace(key, build_cycles(L, live)).first;
    return it->second;
}

bool loop_from_words(const uint32_t w[4], const Cycles &cy, hs_loop &lp)
{
    lp.size = w[0] < kP4Threshold ? 4 : 6;
    const auto &list = lp.size == 4 ? cy.c4 : cy.c6;
    if (list.empty()) return false;
    lp.cycle = int32_t((uint64_t(w[1]) * list.size()) >> 32);
    lp.weight = 1 + int32_t((uint64_t(w[2]) * kWeightMax) >> 32);
    lp.flip = int32_t((uint64_t(w[3]) * uint32_t(lp.size)) >> 32);
    return true;
}

// Coupling changes of one loop: -w s_i s_j on each coupler but the flip-th.
void loop_deltas(const hs_loop &lp, const Cycles &cy, const std::vector<int32_t> &ei, const std::vector<int32_t> &ej,
                 const uint8_t *bits, std::vector<std::pair<int32_t, int>> &out)
{
    out.clear();
    const auto &es = (lp.size == 4 ? cy.c4 : cy.c6)[size_t(lp.cycle)];
    for (int p = 0; p < int(es.size()); ++p) {
        const int e = es[size_t(p)];
        const int s = (bits[ei[size_t(e)]] ^ bits[ej[size_t(e)]]) ? -1 : 1;  // s_i s_j
        const int d = -lp.weight * s;
        out.push_back({e, p == lp.flip ? -d : d});
    }
}

bool valid_loop(const hs_loop &lp, const Cycles &cy)
{
    if (lp.size != 4 && lp.size != 6) return false;
    const size_t n = (lp.size == 4 ? cy.c4 : cy.c6).size();
    return lp.cycle >= 0 && size_t(lp.cycle) < n && lp.weight >= 1 && lp.weight <= kWeightMax && lp.flip >= 0 &&
           lp.flip < lp.size;
}

}  // namespace
}  // namespace hs

using namespace hs;

extern "C" {

int lao_cycle_count(int L, const uint8_t *live, int size, int64_t *count)
{
    if (L < 1 || L > HS_MAX_L || (size != 4 && size != 6) || count == nullptr)
        return fail(HS_EINVAL, "lao_cycle_count: bad arguments");
    const Cycles &cy = cycles_of(L, live);
    *count = int64_t((size == 4 ? cy.c4 : cy.c6).size());
    return HS_OK;
}

int lao_init(int L, const uint8_t *live, int n_loops, uint32_t chain, uint32_t seed, hs_loop *loops, uint8_t *planted,
             int8_t *J, int64_t *e_gs)
{
    if (L < 1 || L > HS_MAX_L || n_loops < 1 || loops == nullptr || planted == nullptr || J == nullptr ||
        e_gs == nullptr)
        return fail(HS_EINVAL, "lao_init: bad arguments");
    const Cycles &cy = cycles_of(L, live);
    std::vector<int32_t> ei, ej;
    chimera_edges(L, ei, ej);
    const int N = 8 * L * L;
    const uint32_t key[2] = {chain, seed};
    for (int i = 0; i < N; ++i) {
        const uint32_t ctr[4] = {uint32_t(i), 0u, 1u, kUseLaoInit};
        uint32_t w[4];
        philox_host(ctr, key, w);
        planted[i] = (live == nullptr || live[i]) ? uint8_t(w[0] >> 31) : uint8_t(0);
    }
    std::vector<int> acc(ei.size(), 0);
    std::vector<std::pair<int32_t, int>> d;
    int64_t e = 0;
    for (int m = 0; m < n_loops; ++m) {
        bool placed = false;
        for (int a = 0; a < kMaxAttempts && !placed; ++a) {
            const uint32_t ctr[4] = {uint32_t(m), uint32_t(a), 0u, kUseLaoInit};
            uint32_t w[4];
            philox_host(ctr, key, w);
            hs_loop lp;
            if (!loop_from_words(w, cy, lp)) return fail(HS_EUNSUPPORTED, "lao_init: no cycle of the drawn size");
            loop_deltas(lp, cy, ei, ej, planted, d);
            bool fits = true;
            for (auto &x : d) fits = fits && std::abs(acc[size_t(x.first)] + x.second) <= kJCap;
            if (!fits) continue;
            for (auto &x : d) acc[size_t(x.first)] += x.second;
            loops[m] = lp;
            e -= int64_t(lp.size - 2) * lp.weight;
            placed = true;
        }
        if (!placed) return fail(HS_EUNSUPPORTED, "lao_init: no loop fits under |J| <= 7");
    }
    for (size_t k = 0; k < ei.size(); ++k) J[k] = int8_t(acc[k]);
    *e_gs = e;
    return HS_OK;
}

int lao_move(int L, const uint8_t *live, int n_loops, uint32_t chain, uint32_t seed, uint32_t step, uint32_t proposal,
             const hs_loop *loops, const uint8_t *planted, int32_t *slot, hs_loop *new_loop, uint32_t *w_accept,
             int8_t *J_new, int64_t *e_gs_new)
{
    if (L < 1 || L > HS_MAX_L || n_loops < 1 || loops == nullptr || planted == nullptr || slot == nullptr ||
        new_loop == nullptr || w_accept == nullptr || J_new == nullptr || e_gs_new == nullptr)
        return fail(HS_EINVAL, "lao_move: bad arguments");
    const Cycles &cy = cycles_of(L, live);
    for (int m = 0; m < n_loops; ++m)
        if (!valid_loop(loops[m], cy)) return fail(HS_EINVAL, "lao_move: invalid loop in the instance");
    std::vector<int32_t> ei, ej;
    chimera_edges(L, ei, ej);
    const uint32_t key[2] = {chain, seed};
    uint32_t w[4];
    {
        const uint32_t ctr[4] = {step, proposal, 0u, kUseLaoMove};
        philox_host(ctr, key, w);
    }
    const int s = int((uint64_t(w[0]) * uint32_t(n_loops)) >> 32);
    std::vector<int> acc(ei.size(), 0);
    std::vector<std::pair<int32_t, int>> d;
    int64_t e = 0;
    for (int m = 0; m < n_loops; ++m) {
        if (m == s) continue;
        loop_deltas(loops[m], cy, ei, ej, planted, d);
        for (auto &x : d) acc[size_t(x.first)] += x.second;
        e -= int64_t(loops[m].size - 2) * loops[m].weight;
    }
    for (int a = 0; a < kMaxAttempts; ++a) {
        const uint32_t ctr[4] = {step, proposal, uint32_t(1 + a), kUseLaoMove};
        uint32_t v[4];
        philox_host(ctr, key, v);
        hs_loop lp;
        if (!loop_from_words(v, cy, lp)) return fail(HS_EUNSUPPORTED, "lao_move: no cycle of the drawn size");
        loop_deltas(lp, cy, ei, ej, planted, d);
        // the whole instance must fit: removing a loop can itself push a
        // coupler past the cap
        std::vector<int> trial = acc;
        for (auto &x : d) trial[size_t(x.first)] += x.second;
        bool fits = true;
        for (int v : trial) fits = fits && std::abs(v) <= kJCap;
        if (!fits) continue;
        for (size_t k = 0; k < ei.size(); ++k) J_new[k] = int8_t(trial[k]);
        *slot = s;
        *new_loop = lp;
        *w_accept = w[1];
        *e_gs_new = e - int64_t(lp.size - 2) * lp.weight;
        return HS_OK;
    }
    // void proposal: the instance stays (a rejected move)
    for (int m = 0; m < n_loops; ++m) {
        loop_deltas(loops[m], cy, ei, ej, planted, d);
        if (m == s)
            for (auto &x : d) acc[size_t(x.first)] += x.second;
    }
    for (size_t k = 0; k < ei.size(); ++k) J_new[k] = int8_t(acc[k]);
    *slot = -1;
    *new_loop = loops[s];
    *w_accept = w[1];
    *e_gs_new = e - int64_t(loops[s].size - 2) * loops[s].weight;
    return HS_OK;
}

}  // extern "C"
