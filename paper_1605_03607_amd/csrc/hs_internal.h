// Internal data layout shared by the host side (hs_host.cpp) and the gfx950
// kernels (hs_pt.hip) of libhardspin.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hardspin.h"

namespace hs {

// Philox counter word 3 ("use") values.
constexpr uint32_t kUseMetroHi = 0;
constexpr uint32_t kUseSwap = 1;
constexpr uint32_t kUseInit = 2;
constexpr uint32_t kUseSwapExtra = 3;
constexpr uint32_t kUseMutate = 4;
constexpr uint32_t kUseRestart = 5;
constexpr uint32_t kUseMetroLo = 7;

// Local-field range: |h| <= 6 neighbours * 7 = 42, so m = dE / 2 in [-42, 42].
constexpr int kMaxM = 42;
constexpr int kMRow = 2 * kMaxM + 1;  // 85 table entries per temperature

// Per-instance descriptor in device memory (all offsets in elements of the
// array they index, relative to the workspace base).
struct alignas(16) InstDev {
    int32_t L, ncell, npairs, K;
    int32_t R, nlanes, n_sites, tab;  // tab = index of the TableDev this instance uses
    uint32_t key0, key1;
    int64_t spin_off;   // first uint64 spin word of this instance in buffers.spins
    int64_t jw_off;     // uint32 offset of the coupling words [ncell][2][8]
    int64_t live_off;   // uint32 offset of the flip masks [ncell][2] (byte k = 0xFE if site k is live)
    int64_t edge_off;   // uint32 offset of packed live couplers (i | j << 12 | (J & 0xff) << 24)
    int32_t n_live_edges, task_iters;  // task_iters: pair iterations per wavefront and phase
    int64_t task_off;   // uint32 offset of the wavefront task table of this lattice size
    int64_t cost;       // sweeps x cells, used to order the work queue
    int32_t tri;        // (K - 1) K / 2: exchange tests (start j <= pair k) per replica set
    uint32_t tri_m;     // ceil(2^32 / tri) for tri >= 2: q / tri = mul_hi(q, tri_m) for q < 2^12
    uint32_t k_m;       // ceil(2^16 / K): l / K = (l k_m) >> 16 for l < 64
    int32_t pad_;
};

// Instances sharing one workgroup's 64 lanes (HS_PACK_LANES): member m holds
// lanes lane0[m] .. lane0[m] + nlanes(m) - 1; its replica sets are segments
// of K consecutive lanes.  An unpacked launch has one member per pack.
constexpr int kMaxPack = 2;

struct alignas(16) PackDev {
    int32_t n_mem;            // members, 1..kMaxPack
    int32_t nlanes;           // lanes used by all members
    int32_t n_seg;            // replica sets of all members
    int32_t mem[kMaxPack];    // instance indices
    int32_t lane0[kMaxPack];  // first lane of each member
    int64_t cost;             // cells, used to order the work queue
};

// Metropolis and exchange tables of one temperature ladder.
struct alignas(16) TableDev {
    int32_t K, lds_ts_entries;     // entries of the exchange fast table held in LDS
    int64_t thi_off;               // uint32 [K][85]: fast Metropolis threshold (see below)
    int64_t tfull_off;             // uint32 [K][85]: exact floor(2^32 e^{-2 beta m}) for m >= 1
    int64_t ts_row_off;            // int32 [K]: start of row k in the exchange tables
    int64_t ts_dhi_off;            // int32 [K]: rows of the 16-bit exchange table (d = 1..dhi)
    int64_t ts_dmax_off;           // int32 [K]: rows of the exact exchange table (d = 1..dmax)
    int64_t ts_hi_off;             // uint16 as uint32 pairs: fast exchange thresholds (high 16 bits)
    int64_t ts_full_off;           // uint32: exact exchange thresholds
    int64_t ts_full_row_off;       // int32 [K]: start of row k in the exact table
    int64_t ts_rate_off;           // float [K]: ln 2 / (beta_{k+1} - beta_k) of pair (k, k+1)
};

// Fast Metropolis threshold: thi = T >> 16 for m >= 1, 0x10000 for m <= 0
// ("always").  With u = hi16 * 2^16 + lo16:  hi16 < thi -> accept,
// hi16 > thi -> reject, hi16 == thi -> decide with the exact table (rare).
constexpr uint32_t kAlways = 0x10000u;

struct HostTables {
    int K = 0;
    std::vector<double> beta;
    std::vector<uint32_t> thi, tfull;       // [K][85]
    std::vector<int32_t> ts_row, ts_dhi, ts_dmax, ts_full_row;
    std::vector<uint16_t> ts_hi;            // concatenated rows
    std::vector<uint32_t> ts_full;          // concatenated rows
    std::vector<float> ts_rate;             // [K]: ln 2 / (beta_{k+1} - beta_k)
};

struct HostInstance {
    int L = 0, N = 0, E = 0, ncell = 0;
    std::vector<uint32_t> jw;    // [ncell][2][8]
    std::vector<uint32_t> live;  // [ncell][2] flip masks: byte k = 0xFE if site k is live
    std::vector<uint32_t> edges; // packed live couplers
};

// Host-side builders (hs_host.cpp).
void chimera_edges(int L, std::vector<int32_t> &ei, std::vector<int32_t> &ej);
int build_instance(const hs_instance &in, HostInstance &out, std::string &err);
void build_tables(int K, const double *beta, int64_t d_cap, HostTables &out);
void build_tasks(int L, int nwaves, std::vector<uint32_t> &out, int &iters);
uint64_t metro_threshold(double beta, int m);
uint64_t swap_threshold(double beta_lo, double beta_hi, int64_t d);
void philox_host(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

// pt_init with the upload event optional (hs_pt.hip).
int pt_init_ex(hs_pt **out, const hs_pt_desc *d, const hs_buffers *b, void *stream, bool track_upload);

void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

}  // namespace hs
