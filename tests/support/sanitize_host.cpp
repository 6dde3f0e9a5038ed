// Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
// host-side C++ of libhardspin (hs_host.cpp, hs_lao.cpp): Chimera graphs,
// coupling words, threshold tables (including a closely spaced ladder),
// wavefront task tables, the RAO move with valid and invalid alphabets, and
// the planted-instance cycles, instances and loop moves.  Exits 0 when every
// call behaves; the sanitizers abort on the first invalid access or
// undefined operation.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../paper_1605_03607_amd/csrc/hs_internal.h"

static int fails = 0;
#define CHECK(c)                                                           \
    do {                                                                   \
        if (!(c)) {                                                        \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++fails;                                                       \
        }                                                                  \
    } while (0)

int main()
{
    uint32_t s = 777;
    auto lcg = [&] {
        s = s * 1664525u + 1013904223u;
        return s >> 8;
    };
    const int8_t pm7[14] = {-7, -6, -5, -4, -3, -2, -1, 1, 2, 3, 4, 5, 6, 7};
    for (int L = 1; L <= 16; L += (L < 4 ? 1 : 6)) {
        std::vector<int32_t> ei, ej;
        hs::chimera_edges(L, ei, ej);
        const int N = 8 * L * L, E = int(ei.size());
        CHECK(E == 24 * L * L - 8 * L);
        std::vector<int8_t> J(E);
        std::vector<uint8_t> live(N);
        for (auto &j : J) j = pm7[lcg() % 14];
        for (auto &v : live) v = (lcg() % 20) != 0;
        std::vector<double> beta(24);
        for (int k = 0; k < 24; ++k) beta[k] = 0.1 * (1.0 + 0.2 * k);
        hs_instance in{L, live.data(), J.data(), 5u, 24, 2, beta.data()};
        hs::HostInstance hi;
        std::string err;
        CHECK(hs::build_instance(in, hi, err) == HS_OK);
        in.live = nullptr;
        CHECK(hs::build_instance(in, hi, err) == HS_OK);
        for (int w : {1, 2, 4, 16}) {
            std::vector<uint32_t> tk;
            int iters = 0;
            hs::build_tasks(L, w, tk, iters);
            CHECK(iters >= 1);
        }
        for (int step = 0; step < 40; ++step) {
            hs_mutation m{};
            CHECK(instance_mutate(&in, pm7, 14, 1, 2, uint32_t(step), 3, &m) == HS_OK);
            CHECK(m.new_j != m.old_j);
            const int8_t rep[3] = {-1, 1, 1};
            CHECK(instance_mutate(&in, rep, 3, 1, 2, uint32_t(step), 3, &m) == HS_EINVAL);
        }
    }
    {
        hs::HostTables t;
        const double close[2] = {1.0, 1.0 + 1e-9};
        hs::build_tables(2, close, 2 * 7 * 1472, t);
        CHECK(t.ts_full.size() <= size_t(2 * 7 * 1472));
        std::vector<double> b(32);
        for (int k = 0; k < 32; ++k) b[k] = 0.1 * std::pow(50.0, k / 31.0);
        hs::build_tables(32, b.data(), 1 << 20, t);
        CHECK(!t.ts_hi.empty());
    }
    CHECK(hs_rao_accept(1.0, 0.5, 0.5, 0u) == 1);
    for (int L = 1; L <= 3; ++L) {
        int64_t n4 = 0, n6 = 0;
        CHECK(lao_cycle_count(L, nullptr, 4, &n4) == HS_OK);
        CHECK(lao_cycle_count(L, nullptr, 6, &n6) == HS_OK);
        const int loops = 4 * L * L;
        std::vector<hs_loop> lp(loops);
        std::vector<uint8_t> planted(8 * L * L);
        std::vector<int8_t> J(24 * L * L - 8 * L), J2(J.size());
        int64_t e_gs = 0, e2 = 0;
        CHECK(lao_init(L, nullptr, loops, 3, 4, lp.data(), planted.data(), J.data(), &e_gs) == HS_OK);
        for (int step = 0; step < 10; ++step) {
            int32_t slot = 0;
            hs_loop nl{};
            uint32_t w = 0;
            CHECK(lao_move(L, nullptr, loops, 3, 4, uint32_t(step), 0, lp.data(), planted.data(), &slot, &nl, &w,
                           J2.data(), &e2) == HS_OK);
        }
    }
    if (fails) return 1;
    std::printf("host sanitizer driver: ok\n");
    return 0;
}
