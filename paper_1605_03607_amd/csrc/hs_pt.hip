// gfx950 kernels and C ABI of the parallel-tempering engine (libhardspin).
//
// Layout on the device (one workgroup per instance, persistent work queue):
//   * Spins live in LDS in 64 columns, one per replica configuration, and
//     the four spins of one side of one K_{4,4} cell are the four bytes of
//     one dword (byte = +1 or -1, i.e. 0x01 / 0xFF).  S[cell][side][column].
//     Lane l of every wavefront is slot l = r K + k (temperature k of replica
//     set r) for the whole launch and updates column perm[l], the
//     configuration currently at that temperature.
//   * The local field of a site is two v_dot4_i32_i8: the four spins of the
//     opposite side of the cell times four coupling bytes, plus the two
//     inter-cell neighbours (v_perm'd into one dword) times two coupling
//     bytes.  Coupling bytes are -4 J, so the product with the site's own spin
//     is 4 m = 2 dE directly (m = -s h, dE = 2 m).
//   * Randomness: Philox4x32-10, one call per (sweep, phase, cell pair, slot)
//     gives eight 16-bit halves, the high halves of the eight 32-bit
//     Metropolis uniforms of the pair's two updated cell sides.  The low
//     halves come from a second Philox use and are computed only when a lane
//     ties on the high half (probability 2^-16 per attempt).
//   * Thresholds: fast table thi[k][m] = T >> 16 (0x10000 for m <= 0), held
//     in LDS as one column per slot (lane), biased by 0x8000 so that packed
//     signed 16-bit arithmetic compares it with the uniforms; with 4-byte
//     columns the per-lane gather is free of bank conflicts.  The exact table
//     T = floor(2^32 exp(-2 beta m)) stays in global memory for ties.
//   * Exchange passes: one wavefront per replica set turns each pair's
//     uniform into the largest energy difference the pair accepts, walks the
//     runs of accepted exchanges and rewrites perm.  (pt_swap evaluates the
//     acceptance tests of pair (k, k+1) for every configuration that can be
//     carried into slot k first, then links the runs.)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "hs_internal.h"

namespace hs {
namespace dev {

constexpr uint32_t M0 = 0xD2511F53u;
constexpr uint32_t M1 = 0xCD9E8D57u;
constexpr uint32_t W0 = 0x9E3779B9u;
constexpr uint32_t W1 = 0xBB67AE85u;

// a ^ b ^ k in one v_bitop3_b32 (truth table 0x96).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t k)
{
    uint32_t d;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(d) : "v"(a), "v"(b), "v"(k));
    return d;
}

// Read-only workspace data through the constant address space: uniform
// addresses then compile to scalar loads (the workspace is never written while
// a kernel reads it).
template <class T>
using cptr = const __attribute__((address_space(4))) T *;

template <class T>
__device__ __forceinline__ cptr<T> to_const(const T *p)
{
    return (cptr<T>)(p);
}

// A descriptor copied word by word through scalar loads.
template <class T>
__device__ __forceinline__ T load_desc(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "descriptor size");
    const cptr<uint32_t> src = (cptr<uint32_t>)(p);
    uint32_t w[sizeof(T) / 4];
#pragma unroll
    for (int i = 0; i < int(sizeof(T) / 4); ++i) w[i] = src[i];
    T out;
    __builtin_memcpy(&out, w, sizeof(T));
    return out;
}

__device__ __forceinline__ void mul_hilo(uint32_t a, uint32_t b, uint32_t &hi, uint32_t &lo)
{
    const uint64_t p = uint64_t(a) * uint64_t(b);
    hi = uint32_t(p >> 32);
    lo = uint32_t(p);
}

// A wave-uniform value held in a vector register (keeps scalar registers
// free; v_bitop3 reads three vector operands without a constant-bus slot).
__device__ __forceinline__ uint32_t in_vgpr(uint32_t s)
{
    uint32_t v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(__builtin_amdgcn_readfirstlane(s)));
    return v;
}

// The ten round keys of Philox4x32-10 for key (k0, k1): (k0 + r W0, k1 + r W1).
// Bias that maps unsigned 16-bit halves onto signed ones with the same order.
constexpr uint32_t kBias16 = 0x80008000u;

struct RoundKeys {
    uint32_t a[10], b[10];
};

__device__ __forceinline__ RoundKeys round_keys(uint32_t k0, uint32_t k1)
{
    RoundKeys K;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        K.a[r] = in_vgpr(k0 + uint32_t(r) * W0);
        K.b[r] = in_vgpr(k1 + uint32_t(r) * W1);
    }
    return K;
}

// Rounds r0..9 (0-based) of Philox4x32-10 on state x.
__device__ __forceinline__ void philox_rounds(uint32_t &x0, uint32_t &x1, uint32_t &x2, uint32_t &x3,
                                              const RoundKeys &K, int r0)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r < r0) continue;
        uint32_t h0, l0, h1, l1;
        mul_hilo(x0, M0, h0, l0);
        mul_hilo(x2, M1, h1, l1);
        const uint32_t n0 = xor3(h1, x1, K.a[r]);
        const uint32_t n2 = xor3(h0, x3, K.b[r]);
        x0 = n0;
        x1 = l1;
        x2 = n2;
        x3 = l0;
    }
}

// (the key must be the same in every lane of the wavefront)
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
{
    const RoundKeys K = round_keys(k0, k1);
    philox_rounds(c0, c1, c2, c3, K, 0);
    return make_uint4(c0, c1, c2, c3);
}

// Round keys of a key that differs between lanes (packed launches: the
// members' instances have their own first key word).
__device__ __forceinline__ RoundKeys round_keys_lane(uint32_t k0, uint32_t k1)
{
    RoundKeys K;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        K.a[r] = k0 + uint32_t(r) * W0;
        K.b[r] = in_vgpr(k1 + uint32_t(r) * W1);
    }
    return K;
}

// Philox4x32-10 with a key that may differ between lanes.
__device__ __forceinline__ uint4 philox_lane(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                             uint32_t k1)
{
    const RoundKeys K = round_keys_lane(k0, k1);
    philox_rounds(c0, c1, c2, c3, K, 0);
    return make_uint4(c0, c1, c2, c3);
}

// Parts of a Metropolis Philox call that do not depend on the cell pair.
// Counter = (t, c1, slot, use).  Round 0 multiplies the uniform sweep word t
// and the per-lane slot word; round 1 multiplies one uniform word.
struct MetroUniform {
    uint32_t y0u;  // xor into the lane's low slot product -> round-2 x0
    uint32_t y1;   // round-2 x1 (uniform)
    uint32_t y2u;  // xor into the per-call high product -> round-2 x2
};

__device__ __forceinline__ MetroUniform metro_uniform(uint32_t t, uint32_t use, uint32_t k0, uint32_t k1)
{
    uint32_t h0, l0;
    mul_hilo(t, M0, h0, l0);
    const uint32_t x2 = h0 ^ use ^ k1;
    uint32_t qh, ql;
    mul_hilo(x2, M1, qh, ql);
    MetroUniform u;
    u.y0u = qh ^ (k0 + W0);
    u.y1 = ql;
    u.y2u = l0 ^ (k1 + W1);
    return u;
}

// Per-lane slot products: (hi, lo) of M1 * slot.
struct MetroLane {
    uint32_t a;  // hi(M1 slot) ^ k0  -> round-0 x0 before the xor with c1
    uint32_t lo; // lo(M1 slot)       -> round-1 x1
};

__device__ __forceinline__ uint4 metro_call(const MetroLane &ml, const MetroUniform &mu, uint32_t c1,
                                            const RoundKeys &K)
{
    const uint32_t x0 = ml.a ^ c1;
    uint32_t qh, ql;
    mul_hilo(x0, M0, qh, ql);
    uint32_t y0 = ml.lo ^ mu.y0u, y1 = mu.y1, y2 = qh ^ mu.y2u, y3 = ql;
    philox_rounds(y0, y1, y2, y3, K, 2);
    return make_uint4(y0, y1, y2, y3);
}

__device__ __forceinline__ uint32_t half16(uint4 w, int q)
{
    const uint32_t word = (q >> 1) == 0 ? w.x : (q >> 1) == 1 ? w.y : (q >> 1) == 2 ? w.z : w.w;
    return (q & 1) ? (word >> 16) : (word & 0xFFFFu);
}

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

// ---------------------------------------------------------------------------
// Dynamic LDS layout of the sweep kernel.
struct LdsLayout {
    uint32_t S, ths, tshi, Eacc, perm, sacc, xrow, lim, misc, total;
    // packed launches only: replica-set segments, the members' coupling
    // words and flip masks, threshold-row offsets
    uint32_t seg, jwl, lml, thia;
    // the first two Metropolis draws of the next sweep for the (at most two)
    // wavefronts that walk the exchange runs
    uint32_t hand;
};

// mode bit 0: 2-byte threshold columns (else 4-byte: no two lanes share a
// bank).  mode bit 1: packed launch (instances sharing the lanes; the
// exchange tables stay in global memory).
constexpr int kLdsPacked = 2;
// mode bit 2: room for the exchange walkers' hand-over of their first two
// draws of the next sweep
constexpr int kLdsHand = 4;

__host__ __device__ inline LdsLayout lds_layout(int ncell_max, int tshi_max, int r_max, int mode)
{
    LdsLayout l;
    uint32_t o = 0;
    l.S = o;
    o += (uint32_t(ncell_max) * 2 + 1) * 64 * 4;  // spin rows, then one zero row
    l.ths = o;
    o += uint32_t(kMRow) * 64 * ((mode & 1) ? 2 : 4);  // 16-bit thresholds, one column per slot
    l.tshi = o;
    o += ((uint32_t(tshi_max) * 2 + 15) / 16) * 16;
    l.Eacc = o;
    o += 2 * 64 * 4;                              // slot energies (set-major), double-buffered by sweep parity
    l.perm = o;
    o += 64 * 4;                                  // slot (set-major) -> configuration column
    l.sacc = o;
    o += 64 * 4;
    l.xrow = o;
    // exchange-table row start and length of pair (k, k+1), the exact
    // table's row start and length (packed launches: by the pair's lower
    // slot), and ln 2 / (beta_{k+1} - beta_k)
    o += 5 * 64 * 4;
    l.lim = o;
    // limits D of the due exchange pass's pairs, by lane (64 used; sized by
    // the replica sets, which keeps the sweep kernel's registers as measured)
    o += uint32_t(r_max) * 64 * 4;
    l.misc = o;
    o += 16 * 4;
    l.seg = l.jwl = l.lml = l.thia = l.hand = o;
    if (mode & kLdsHand) {
        o = (o + 15u) & ~15u;
        l.hand = o;
        o += 4 * 64 * 16;                         // uint4 [walker][draw][lane]
    }
    if (mode & kLdsPacked) {
        l.seg = o;
        o += 2 * 64 * 4;                          // first slot and K of every replica set
        l.thia = o;
        o += 64 * 4;                              // Metropolis threshold row of every slot
        l.jwl = o;
        o += uint32_t(kMaxPack) * uint32_t(ncell_max) * 16 * 4;  // coupling words [member][cell][2][8]
        l.lml = o;
        o += uint32_t(kMaxPack) * uint32_t(ncell_max) * 2 * 4;   // flip masks [member][cell][2]
    }
    l.total = o;
    return l;
}

struct SweepArgs {
    const InstDev *inst;
    const TableDev *tabs;
    const PackDev *packs;     // packed launches: the packs the queue hands out
    const uint32_t *ws32;     // workspace viewed as uint32
    const int32_t *order;     // processing order of instances (of packs when packed), descending cost
    uint32_t *queue;          // work-queue counter
    uint64_t *spins;
    uint8_t *perm;
    int32_t *energy;
    int32_t *emin;
    int64_t *thit;
    uint32_t *swap_acc;
    int64_t *t;
    int32_t *stopped;
    int32_t n_inst;
    int32_t n_items;          // work items of the queue: instances, or packs when packed
    int32_t swap_interval;
    int64_t n_sweeps;
    uint32_t flags;
    int32_t ncell_max, tshi_max, r_max;
    int32_t lds_ts_ok;        // 1 if every ladder's fast exchange table fits in LDS
    int32_t lds_mode;         // lds_layout mode
    uint8_t *walk;            // optional: temperature index per configuration after each exchange pass
    int64_t walk_cap;         // exchange passes the walk buffer holds per instance
};

// Exchange decisions (detailed balance, Sec. II) for configuration x at
// slot k and y at slot k + 1: d = E_x - E_y, accept iff d <= 0 or
// u < floor(2^32 exp(-(beta_{k+1} - beta_k) d)).  A 16-bit table (the high
// halves of the thresholds for d = 1..dhi(k)) decides unless the high halves
// tie; ties are settled with the exact 32-bit table.

// The uniforms of one exchange pass: lane p < (K-1) R gets word 0 of
// Philox(key, (t, k, r, use)) for pair p = r (K-1) + k.
__device__ __forceinline__ uint32_t exchange_uniform(uint32_t t, uint32_t use, int K, int R, uint32_t key0,
                                                     uint32_t key1)
{
    const int lane = threadIdx.x & 63;
    const int km1 = max(K - 1, 1);
    const int r = lane / km1, k = lane - r * km1;
    const uint32_t u = philox(t, uint32_t(k), uint32_t(r), use, key0, key1).x;
    return lane < (K - 1) * R ? u : 0u;
}

// An exchange pass is one ascending sweep over the pairs (k, k+1) of each
// replica set.  The configuration at slot k when pair k is tested is the one
// that started at the beginning j of the current run of accepted exchanges
// (a rejection at k starts a new run at k + 1).
//
// Slots are numbered set-major, s = r K + k (set r, temperature k); Es[s] is
// the energy of the configuration at slot s.
//
// Step 1 (every wavefront): for each set r and start j, stop(j) = the first
// pair k >= j rejected when slot k holds the configuration from slot j
// (K - 1 if none).  The R (K-1) K / 2 tests (r, j <= k) are spread one per
// lane over the workgroup, q = r T + k (k + 1) / 2 + j, and rejections are
// merged into stopv[r][j] (K - 1 beforehand) with an LDS atomic minimum.

// Row start and 16-bit row length of the exchange table of pair (k, k + 1),
// k = i < K - 1 (xrow[i], xrow[64 + i]).
__device__ __forceinline__ void load_xrows(int32_t *xrow, const TableDev &tb, const uint32_t *ws32, int K,
                                           int i)
{
    if (i < 64) {
        const bool ok = i < K - 1;
        xrow[i] = ok ? int32_t(ws32[tb.ts_row_off + i]) : 0;
        xrow[64 + i] = ok ? int32_t(ws32[tb.ts_dhi_off + i]) : 0;
    }
}

// Test q = r T + k (k + 1) / 2 + j (T = tri = (K-1) K / 2, tri_m = ceil(2^32 / T)
// for T >= 2) packed as r << 16 | k << 8 | j.
__device__ __forceinline__ uint32_t exchange_test(int q, int tri, uint32_t tri_m)
{
    const int r = tri == 1 ? q : int(__umulhi(uint32_t(q), tri_m));
    const int rem = q - r * tri;
    int k = int((__fsqrt_rn(float(8 * rem + 1)) - 1.0f) * 0.5f);
    k += ((k + 1) * (k + 2) / 2 <= rem) ? 1 : 0;
    k -= (k * (k + 1) / 2 > rem) ? 1 : 0;
    const int j = rem - k * (k + 1) / 2;
    return (uint32_t(r) << 16) | (uint32_t(k) << 8) | uint32_t(j);
}

// dec0 = exchange_test(min(wave * 64 + lane, ntest - 1)), computed once per
// instance by the caller; later rounds (more tests than lanes) decode here.
template <bool kLds>
__device__ void exchange_stops(int K, int R, int tri, uint32_t tri_m, int wave, int nwaves, uint32_t dec0,
                               const int32_t *Es, const uint32_t *ux, const int32_t *xrow, int32_t *stopv,
                               const TableDev &tb, const uint32_t *ws32, const uint16_t *tshi)
{
    const int lane = threadIdx.x & 63;
    const int ntest = tri * R;
    if (wave * 64 >= ntest) return;
    const uint16_t *ghi = reinterpret_cast<const uint16_t *>(ws32 + tb.ts_hi_off);
    for (int base = wave * 64; base < ntest; base += nwaves * 64) {
        const uint32_t dec = base == wave * 64 ? dec0 : exchange_test(min(base + lane, ntest - 1), tri, tri_m);
        const int r = int(dec >> 16), k = int((dec >> 8) & 0xFFu), j = int(dec & 0xFFu);
        const int ex = Es[r * K + j];
        const int ey = Es[r * K + k + 1];
        const uint32_t u = ux[r * (K - 1) + k];
        const int row = xrow[k], dh = xrow[64 + k];
        const int d = ex - ey;
        const int at = row + min(max(d, 1), max(dh, 1)) - 1;  // clamped into the row
        uint32_t h;
        if constexpr (kLds)
            h = tshi[at];
        else
            h = ghi[at];
        const uint32_t th = d <= dh ? h : 0u;
        const uint32_t u16 = u >> 16;
        bool rej = d > 0 && u16 > th;
        const bool tie = d > 0 && u16 == th;
        if (__any(tie)) {  // rare: exact table
            if (tie) {
                const int dmx = int(ws32[tb.ts_dmax_off + k]);
                const uint32_t tf = d <= dmx ? ws32[tb.ts_full_off + ws32[tb.ts_full_row_off + k] + d - 1] : 0u;
                rej = !(u < tf);
            }
        }
        if (rej && base + lane < ntest) atomicMin(&stopv[r * 64 + j], k);
    }
}

// Step 2 (wavefront r mod nwaves for set r, lane j): the run ends of set r
// are stop(0), stop(stop(0) + 1), ... up to K - 1, found by a scalar walk
// that reads stop(j) from lane j, two runs per step.  Slot k of the run [x, e] receives the
// configuration from slot k + 1 if k < e (accepted) and the carried
// configuration from slot x if k = e.  perm maps slot (set-major) -> the
// configuration's column and sacc counts accepted exchanges by pair k R + r.
// Sets are disjoint, so the wavefronts of different sets touch disjoint
// entries.
__device__ void exchange_apply(int K, int R, int wave, int nwaves, int32_t *perm, uint32_t *sacc, int32_t *stopv)
{
    const int j = threadIdx.x & 63;
    for (int r = wave; r < R; r += nwaves) {
        const int base = r * K;
        int st = K - 1;
        if (j < K - 1) {
            st = stopv[r * 64 + j];
            stopv[r * 64 + j] = K - 1;  // ready for the next pass
        }
        // two runs per step: st2(j) = stop(stop(j) + 1) ends the run after j's
        // (K - 1 when j's run is the last)
        const int st2 = __shfl(st, min(st + 1, K - 1), 64);
        uint64_t ends = 0;
        int x0 = 0;
        do {
            const int e1 = __builtin_amdgcn_readlane(st, x0);  // stop(x0) >= x0
            const int e2 = __builtin_amdgcn_readlane(st2, x0);
            ends |= (1ull << e1) | (1ull << e2);
            x0 = max(e2, x0) + 1;
        } while (x0 < K);
        if (j < K) {
            const int e = j + __ffsll(static_cast<long long>(ends >> j)) - 1;  // end of j's run
            const uint64_t below = ends & ((1ull << j) - 1ull);
            const int x = below ? 64 - __clzll(static_cast<long long>(below)) : 0;  // start of j's run
            const int ox = perm[base + x];
            const int on = perm[base + min(j + 1, K - 1)];
            const int np = j == e ? ox : on;
            perm[base + j] = np;
            if (j < K - 1 && j != e) atomicAdd(&sacc[j * R + r], 1u);
        }
    }
}

// The exchange pass by critical energy differences (packed launches use the
// same, through pair_limit_packed and exchange_walk_packed below).  For
// pair (k, k+1) with uniform u the test "d <= 0 or u < T_k(d)" accepts a set
// of differences closed downwards, since T_k(d) = floor(2^32 e^{-(beta_{k+1} -
// beta_k) d}) does not grow with d (0 beyond the table): it accepts exactly
// d <= D_k, D_k >= 0 the largest difference it accepts.  A configuration of
// energy E carried into slot k therefore moves on iff E <= B_k = E_{k+1} + D_k,
// and one wavefront per replica set finds the runs of the ascending pass by a
// scalar walk: the run from x ends at the first pair k >= x with E_x > B_k.
// D_k needs no energies, so one wavefront computes the limits of a pass
// before the phase barrier that precedes it.  It starts from the real bound
// (u < 2^32 e^{-db d} iff d < (32 - log2 u) ln 2 / db) and is settled on the
// integer tables, so every decision equals the test's.
//
// xrow: [k] fast-table row start, [64 + k] its length dhi, [128 + k] exact
// table row start, [192 + k] its length dmax, [256 + k] ln 2 / (beta_{k+1} -
// beta_k) (float bits).
__device__ __forceinline__ void load_xrows_walk(int32_t *xrow, const TableDev &tb, const uint32_t *ws32, int K,
                                                int i)
{
    if (i < 64) {
        const bool ok = i < K - 1;
        xrow[i] = ok ? int32_t(ws32[tb.ts_row_off + i]) : 0;
        xrow[64 + i] = ok ? int32_t(ws32[tb.ts_dhi_off + i]) : 0;
        xrow[128 + i] = ok ? int32_t(ws32[tb.ts_full_row_off + i]) : 0;
        xrow[192 + i] = ok ? int32_t(ws32[tb.ts_dmax_off + i]) : 0;
        xrow[256 + i] = ok ? int32_t(ws32[tb.ts_rate_off + i]) : 0;
    }
}

// D_k for pair k (0 <= k < K - 1) and uniform u: the largest difference the
// pair accepts.
template <bool kLds>
__device__ __forceinline__ int pair_limit(uint32_t u, int k, const int32_t *xrow, const TableDev &tb,
                                          const uint32_t *ws32, const uint16_t *tshi)
{
    const uint16_t *hi = kLds ? tshi : reinterpret_cast<const uint16_t *>(ws32 + tb.ts_hi_off);
    const uint32_t *full = ws32 + tb.ts_full_off;
    const int row = xrow[k], dh = xrow[64 + k], frow = xrow[128 + k], dmax = xrow[192 + k];
    const float rate = __int_as_float(xrow[256 + k]);
    // u < T(d) for 1 <= d <= dmax: the 16-bit table decides unless the high
    // halves tie (h = the table's entry d, 0 beyond its length)
    const uint32_t u16 = u >> 16;
    auto acc = [&](int d, uint32_t h) -> bool { return u16 != h ? u16 < h : u < full[frow + d - 1]; };
    auto hi_at = [&](int d) -> uint32_t {
        return d <= dh ? uint32_t(hi[row + min(max(d, 1), max(dh, 1)) - 1]) : 0u;
    };
    // log2(0) = -inf gives +inf, clamped to the table
    const float x = fminf(fmaxf((32.0f - __builtin_amdgcn_logf(float(u))) * rate, 0.0f), float(dmax) + 1.0f);
    int D = min(max(int(ceilf(x)) - 1, 0), dmax);
    // entries D + 1 and D, read together
    const uint32_t h1 = hi_at(D + 1), h0 = hi_at(D);
    const bool a1 = D < dmax && acc(D + 1, h1);
    const bool a0 = D == 0 || acc(D, h0);
    if (a1) {
        ++D;
        while (D < dmax && acc(D + 1, hi_at(D + 1))) ++D;
    } else if (!a0) {
        --D;
        while (D > 0 && !acc(D, hi_at(D))) --D;
    }
    return D;
}

// The runs of one exchange pass and the new perm, from xd[r (K-1) + k] = D_k
// of every pair (wavefront r mod nwaves for set r, lane j = slot).
__device__ void exchange_walk(int K, int R, int wave, int nwaves, const int32_t *Es, const int32_t *xd,
                              int32_t *perm, uint32_t *sacc)
{
    const int j = threadIdx.x & 63;
    const bool pair = j < K - 1;
    for (int r = wave; r < R; r += nwaves) {
        const int base = r * K;
        const int e = Es[base + min(j, K - 1)];
        // pairs reject a carried energy above b = E_{k+1} + D_k; other lanes never do
        const int b = pair ? Es[base + j + 1] + xd[r * (K - 1) + j] : INT32_MAX;
        // run ends: bit k of `ends` set iff slot k keeps the carried configuration
        uint64_t ends = 0;
        int x0 = 0;
        do {
            const int ec = __builtin_amdgcn_readlane(e, x0);  // the configuration carried from slot x0
            // lanes with ec > b, straight from the compare (every lane is
            // active here); the wait states cover ec, just written by a VALU
            // instruction
            uint64_t gt;
            asm volatile("s_nop 1\n\tv_cmp_gt_i32_e64 %0, %1, %2" : "=s"(gt) : "s"(ec), "v"(b));
            const uint64_t rej = gt & (~0ull << x0);
            const int st = rej ? int(__builtin_ctzll(rej)) : K - 1;
            ends |= 1ull << st;
            x0 = st + 1;
        } while (x0 < K);
        if (j < K) {
            const int en = j + __builtin_ctzll(ends >> j);  // end of j's run
            const uint64_t below = ends & ((1ull << j) - 1ull);
            const int xs = below ? 64 - __builtin_clzll(below) : 0;  // start of j's run
            const int ox = perm[base + xs];
            const int on = perm[base + min(j + 1, K - 1)];
            perm[base + j] = j == en ? ox : on;
            if (pair && j != en) sacc[j * R + r] += 1u;
        }
    }
}

// Packed launches: D for the pair at slot l (its lower slot), with the
// tables indexed from the workspace base: xrow[l] the 16-bit row (uint16
// index), [64 + l] its length, [128 + l] the exact row (uint32 index),
// [192 + l] its length, [256 + l] ln 2 / (beta_{k+1} - beta_k).
__device__ __forceinline__ int pair_limit_packed(uint32_t u, int l, const int32_t *xrow, const uint32_t *ws32)
{
    const uint16_t *hi = reinterpret_cast<const uint16_t *>(ws32);
    const int row = xrow[l], dh = xrow[64 + l], frow = xrow[128 + l], dmax = xrow[192 + l];
    const float rate = __int_as_float(xrow[256 + l]);
    const uint32_t u16 = u >> 16;
    auto acc = [&](int d, uint32_t h) -> bool { return u16 != h ? u16 < h : u < ws32[frow + d - 1]; };
    auto hi_at = [&](int d) -> uint32_t {
        return d <= dh ? uint32_t(hi[row + min(max(d, 1), max(dh, 1)) - 1]) : 0u;
    };
    const float x = fminf(fmaxf((32.0f - __builtin_amdgcn_logf(float(u))) * rate, 0.0f), float(dmax) + 1.0f);
    int D = min(max(int(ceilf(x)) - 1, 0), dmax);
    const uint32_t h1 = hi_at(D + 1), h0 = hi_at(D);
    const bool a1 = D < dmax && acc(D + 1, h1);
    const bool a0 = D == 0 || acc(D, h0);
    if (a1) {
        ++D;
        while (D < dmax && acc(D + 1, hi_at(D + 1))) ++D;
    } else if (!a0) {
        --D;
        while (D > 0 && !acc(D, hi_at(D))) --D;
    }
    return D;
}

// Packed launches: the walk of each replica set (segment s: slots
// seg_base[s] .. seg_base[s] + K_s - 1), as exchange_walk, with the limit
// and the counter of pair (k, k+1) at its lower slot.
__device__ void exchange_walk_packed(int n_seg, const int32_t *seg_base, const int32_t *seg_k, int wave, int nwaves,
                                     const int32_t *Es, const int32_t *xd, int32_t *perm, uint32_t *sacc)
{
    const int j = threadIdx.x & 63;
    for (int sg = wave; sg < n_seg; sg += nwaves) {
        const int base = __builtin_amdgcn_readfirstlane(seg_base[sg]);
        const int K = __builtin_amdgcn_readfirstlane(seg_k[sg]);
        const bool pair = j < K - 1;
        const int e = Es[base + min(j, K - 1)];
        const int b = pair ? Es[base + j + 1] + xd[base + j] : INT32_MAX;
        uint64_t ends = 0;
        int x0 = 0;
        do {
            const int ec = __builtin_amdgcn_readlane(e, x0);
            // wait states for ec as in exchange_walk
            uint64_t gt;
            asm volatile("s_nop 1\n\tv_cmp_gt_i32_e64 %0, %1, %2" : "=s"(gt) : "s"(ec), "v"(b));
            const uint64_t rej = gt & (~0ull << x0);
            const int st = rej ? int(__builtin_ctzll(rej)) : K - 1;
            ends |= 1ull << st;
            x0 = st + 1;
        } while (x0 < K);
        if (j < K) {
            const int en = j + __builtin_ctzll(ends >> j);
            const uint64_t below = ends & ((1ull << j) - 1ull);
            const int xs = below ? 64 - __builtin_clzll(below) : 0;
            const int ox = perm[base + xs];
            const int on = perm[base + min(j + 1, K - 1)];
            perm[base + j] = j == en ? ox : on;
            if (pair && j != en) sacc[base + j] += 1u;
        }
    }
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int64_t wave_max64(int64_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const int64_t w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

// Quad table entry: LDS byte offsets of the spin rows of an updated cell
// side (own), of the opposite side of its cell (oth) and of the same side of
// the two neighbouring cells along that side's direction (a, b; the zero
// row when absent), plus the side's index q for the coupling words.
struct QuadRows {
    uint32_t own, oth, a, b;
};

__host__ __device__ inline QuadRows quad_rows(int cell, int p, int Lc, int ncell)
{
    const int r = cell / Lc, c = cell - r * Lc;
    const int u = (r + c + p) & 1;
    const int zero = ncell * 2;
    QuadRows x;
    x.own = uint32_t(cell * 2 + u) * 256u;
    x.oth = uint32_t(cell * 2 + 1 - u) * 256u;
    x.a = uint32_t(u == 0 ? (r > 0 ? (cell - Lc) * 2 : zero) : (c > 0 ? (cell - 1) * 2 + 1 : zero)) * 256u;
    x.b = uint32_t(u == 0 ? (r + 1 < Lc ? (cell + Lc) * 2 : zero) : (c + 1 < Lc ? (cell + 1) * 2 + 1 : zero)) *
          256u;
    return x;
}

// Dot products and the spin multiply use the compiler builtins, not inline
// assembly: the wait states a dot-instruction result needs before a dependent
// read are inserted only for instructions the compiler itself generates.
// The clamp flag selects the three-operand encoding, whose zero accumulator
// is an inline constant; the sums here are far from saturating.
__device__ __forceinline__ int dot4_0(uint32_t a, uint32_t b)
{
    return __builtin_amdgcn_sdot4(int(a), int(b), 0, true);
}

__device__ __forceinline__ int dot4_acc(uint32_t a, uint32_t b, int c)
{
    return __builtin_amdgcn_sdot4(int(a), int(b), c, false);
}

// (sign-extended byte K of own) * h4
template <int K>
__device__ __forceinline__ int mul_spin(uint32_t own, int h4)
{
    return __mul24(int(int8_t(uint8_t(own >> (8 * K)))), h4);
}

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

// Per 16-bit half: saturating t' - u' of sign-flipped thresholds and
// uniforms (t' = t ^ 0x8000, so the signed difference has the sign of t - u
// and is zero iff t == u).
__device__ __forceinline__ uint32_t sub_sat16x2(uint32_t a, uint32_t b)
{
    s16x2 x, y;
    __builtin_memcpy(&x, &a, 4);
    __builtin_memcpy(&y, &b, 4);
    const s16x2 d = __builtin_elementwise_sub_sat(x, y);
    uint32_t r;
    __builtin_memcpy(&r, &d, 4);
    return r;
}

__device__ __forceinline__ uint32_t min_u16x2(uint32_t a, uint32_t b)
{
    u16x2 x, y;
    __builtin_memcpy(&x, &a, 4);
    __builtin_memcpy(&y, &b, 4);
    const u16x2 d = __builtin_elementwise_min(x, y);
    uint32_t r;
    __builtin_memcpy(&r, &d, 4);
    return r;
}

// 4 m = 2 dE of site k of a cell side: h4 = -4 h from the opposite side
// (coupling bytes jin) and the two inter-cell neighbours (perm'd word xv,
// coupling bytes jv); m4 = s h4.
template <int K>
__device__ __forceinline__ int site_m4(uint32_t own, uint32_t oth, uint32_t xv, uint32_t jin, uint32_t jv)
{
    return mul_spin<K>(own, dot4_acc(oth, jin, dot4_0(xv, jv)));
}

// The eight coupling words of cell side q (bytes -4 J towards the opposite
// side, then towards the neighbouring cells) and its flip mask: scalar loads
// from the workspace, or in a packed launch the copies of the lane's member
// in LDS (lanes of different members read different words).
template <bool kPacked>
__device__ __forceinline__ uint32_t coupling_words(cptr<uint32_t> jw, cptr<uint32_t> livew, const uint32_t *jwl,
                                                   const uint32_t *lml, uint32_t q, uint32_t (&jq)[8])
{
    if constexpr (kPacked) {
        const uint4 lo = *reinterpret_cast<const uint4 *>(jwl + q * 8);
        const uint4 hi = *reinterpret_cast<const uint4 *>(jwl + q * 8 + 4);
        jq[0] = lo.x;
        jq[1] = lo.y;
        jq[2] = lo.z;
        jq[3] = lo.w;
        jq[4] = hi.x;
        jq[5] = hi.y;
        jq[6] = hi.z;
        jq[7] = hi.w;
        return lml[q];
    } else {
#pragma unroll
        for (int w = 0; w < 8; ++w) jq[w] = jw[q * 8 + w];
        return livew[q];
    }
}

// ---------------------------------------------------------------------------
// The persistent sweep kernel.
//
// Per sweep: colour phase 0, barrier, colour phase 1, barrier.  Every coupler
// joins a colour-0 and a colour-1 site, so the energy after the sweep is
// sum over colour-1 sites of s_i' h_i (Eq. 1), with h_i the local field seen
// in phase 1 and s_i' the spin after its update: phase 1 alone yields the
// slot energies, accumulated in LDS with atomics.  Every wavefront then keeps
// its own copy of the running minima (identical in all wavefronts) and, when
// an exchange pass is due, the two exchange steps add two barriers.
// kRecord: also write the temperature walk (pt_sweep_record); a separate
// instantiation keeps the plain sweep free of the recording code.
template <bool kRecord, bool kPacked>
__global__ void __launch_bounds__(1024) k_pt_sweep(SweepArgs a)
{
    extern __shared__ __align__(16) char lds[];
    const LdsLayout L = lds_layout(a.ncell_max, a.tshi_max, a.r_max, a.lds_mode);
    const uint32_t ths_sh = (a.lds_mode & 1) ? 5u : 6u;  // entry m of a column at byte (4 m) << ths_sh
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nwaves = __builtin_amdgcn_readfirstlane(int(blockDim.x >> 6));
    uint32_t *S = reinterpret_cast<uint32_t *>(lds + L.S);
    uint16_t *THS = reinterpret_cast<uint16_t *>(lds + L.ths);
    int32_t *Eacc = reinterpret_cast<int32_t *>(lds + L.Eacc);
    int32_t *perm = reinterpret_cast<int32_t *>(lds + L.perm);
    uint32_t *sacc = reinterpret_cast<uint32_t *>(lds + L.sacc);
    int32_t *xrow = reinterpret_cast<int32_t *>(lds + L.xrow);
    int32_t *lim = reinterpret_cast<int32_t *>(lds + L.lim);
    int32_t *misc = reinterpret_cast<int32_t *>(lds + L.misc);
    uint16_t *tshi = reinterpret_cast<uint16_t *>(lds + L.tshi);
    const bool stop_mode = (a.flags & HS_STOP_ON_AGREEMENT) != 0;
    const int si = a.swap_interval;

    for (;;) {
        if (tid == 0) misc[0] = int32_t(atomicAdd(a.queue, 1u));
        __syncthreads();
        const int qi = __builtin_amdgcn_readfirstlane(misc[0]);
        __syncthreads();
        if (qi >= a.n_items) break;
        const int item = __builtin_amdgcn_readfirstlane(to_const(a.order)[qi]);
        // The first member (the only one unless packed) gives the lattice and
        // the task tables; K, R, the Philox key and the tables of a lane come
        // from the lane's own member.
        PackDev pk{};
        if constexpr (kPacked) {
            pk = load_desc(a.packs + item);
        } else {
            pk.n_mem = 1;
            pk.mem[0] = item;
        }
        const int n = pk.mem[0];
        const InstDev d = load_desc(a.inst + n);
        const TableDev tb = load_desc(a.tabs + d.tab);
        const int ncell = d.ncell;
        const uint32_t key1 = d.key1;
        const cptr<uint32_t> ws4 = to_const(a.ws32);
        const cptr<uint32_t> jw = ws4 + d.jw_off;     // coupling words [ncell][2][8]
        const cptr<uint32_t> livew = ws4 + d.live_off; // flip masks [ncell][2]
        // the lane's member: the second one from lane0[1] on (packed launches)
        const InstDev e = kPacked && pk.n_mem > 1 ? load_desc(a.inst + pk.mem[1]) : d;
        const TableDev te = kPacked && pk.n_mem > 1 ? load_desc(a.tabs + e.tab) : tb;
        const int mi = (kPacked && pk.n_mem > 1 && lane >= pk.lane0[1]) ? 1 : 0;
        const int K = mi ? e.K : d.K, R = mi ? e.R : d.R;
        const int nlanes = kPacked ? pk.nlanes : d.nlanes;
        const uint32_t key0 = mi ? e.key0 : d.key0;
        const int lane0 = mi ? pk.lane0[1] : 0;  // first lane of this lane's member
        const int nm = mi ? pk.mem[1] : n;       // this lane's instance
        const int64_t spin_off = mi ? e.spin_off : d.spin_off;
        const int64_t live_off = mi ? e.live_off : d.live_off;
        const int64_t tfull_off = mi ? te.tfull_off : tb.tfull_off;
        // packed: this lane's member's coupling words and flip masks in LDS
        const uint32_t *jwl = reinterpret_cast<const uint32_t *>(lds + L.jwl) + mi * a.ncell_max * 16;
        const uint32_t *lml = reinterpret_cast<const uint32_t *>(lds + L.lml) + mi * a.ncell_max * 2;
        int32_t *seg_base = reinterpret_cast<int32_t *>(lds + L.seg);
        int32_t *seg_k = seg_base + 64;
        if constexpr (kPacked) {
            // the members' coupling words and flip masks
            for (int m = 0; m < pk.n_mem; ++m) {
                const InstDev &x = m ? e : d;
                uint32_t *jd = reinterpret_cast<uint32_t *>(lds + L.jwl) + m * a.ncell_max * 16;
                uint32_t *ld = reinterpret_cast<uint32_t *>(lds + L.lml) + m * a.ncell_max * 2;
                for (int i = tid; i < ncell * 16; i += blockDim.x) jd[i] = a.ws32[x.jw_off + i];
                for (int i = tid; i < ncell * 2; i += blockDim.x) ld[i] = a.ws32[x.live_off + i];
            }
            if (tid < 64) {
                // per slot l: threshold row, exchange-table rows of pair (k, k+1), perm, counters
                const int l = tid;
                const bool lv = l < pk.nlanes;
                const int ll = l - lane0;
                const int kk = lv ? ll % K : 0, rr = lv ? ll / K : 0;
                const TableDev &tl = mi ? te : tb;
                uint32_t *thia = reinterpret_cast<uint32_t *>(lds + L.thia);
                thia[l] = uint32_t(tl.thi_off + kk * kMRow);
                const bool pair = lv && kk < K - 1;
                xrow[l] = pair ? int32_t(tl.ts_hi_off * 2 + a.ws32[tl.ts_row_off + kk]) : 0;
                xrow[64 + l] = pair ? int32_t(a.ws32[tl.ts_dhi_off + kk]) : 0;
                xrow[128 + l] = pair ? int32_t(tl.ts_full_off + a.ws32[tl.ts_full_row_off + kk]) : 0;
                xrow[192 + l] = pair ? int32_t(a.ws32[tl.ts_dmax_off + kk]) : 0;
                xrow[256 + l] = pair ? int32_t(a.ws32[tl.ts_rate_off + kk]) : 0;
                // perm in LDS is set-major (slot lane0 + r K + k, configuration columns of
                // the member from lane0 on); the buffers hold slot k R + r
                perm[l] = lv ? lane0 + int(a.perm[nm * 64 + kk * R + rr]) : l;
                sacc[l] = pair ? a.swap_acc[nm * 64 + kk * R + rr] : 0u;
                if (lv && kk == 0) {  // first slot of a replica set: its segment
                    const int sg = (mi ? d.R : 0) + rr;
                    seg_base[sg] = l;
                    seg_k[sg] = K;
                }
            }
            if (tid == 0) misc[1] = 0;
            __syncthreads();
        }
        const uint64_t *sp = a.spins + spin_off;

        // ---- load state ----
        for (int q = wave; q < ncell * 2; q += nwaves) {
            const uint32_t lm = kPacked ? a.ws32[live_off + q] : livew[q];
            uint32_t w = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint64_t word = sp[q * 4 + k];
                const bool in = !kPacked || lane < nlanes;
                const uint32_t bit =
                    (in && ((lm >> (8 * k + 1)) & 1u)) ? uint32_t((word >> (lane - lane0)) & 1ull) : 0u;
                w |= (bit ? 0xFFu : 0x01u) << (8 * k);
            }
            S[q * 64 + lane] = w;
        }
        if (wave == 0) S[ncell * 2 * 64 + lane] = 0u;  // zero row for absent neighbours
        // threshold column r K + k holds the row of temperature k: the lanes of
        // a replica set occupy one block of columns, so each half-wavefront
        // gathers from distinct banks
        for (int i = tid; i < kMRow * 64; i += blockDim.x) {
            const int m = i >> 6, sx = i & 63;
            uint32_t th;
            if constexpr (kPacked) {
                th = a.ws32[reinterpret_cast<const uint32_t *>(lds + L.thia)[sx] + m];
            } else {
                const int k = sx < nlanes ? sx % K : 0;
                th = a.ws32[tb.thi_off + k * kMRow + m];
            }
            // 0x10000 ("always", m <= 0) becomes 0xFFFF: a uniform of 0xFFFF then
            // ties and the exact pass accepts
            THS[(uint32_t(i) << ths_sh) >> 5] = uint16_t((th >= 0x10000u ? 0xFFFFu : th) ^ 0x8000u);
        }
        if constexpr (!kPacked) {
            if (a.lds_ts_ok) {
                const uint32_t *src = a.ws32 + tb.ts_hi_off;
                uint32_t *dst = reinterpret_cast<uint32_t *>(tshi);
                for (int i = tid; i < (tb.lds_ts_entries + 1) / 2; i += blockDim.x) dst[i] = src[i];
            }
            load_xrows_walk(xrow, tb, a.ws32, K, tid);
            if (tid < 64) {
                // perm in LDS is set-major (slot r K + k); the buffer holds slot k R + r
                const int src = tid < K * R ? (tid % K) * R + tid / K : tid;
                perm[tid] = a.perm[n * 64 + src];
                sacc[tid] = a.swap_acc[n * 64 + tid];
            }
            if (tid == 0) misc[1] = a.stopped[n];
        }
        __syncthreads();

        // Lane l is slot l = r K + k (temperature k of replica set r) in every
        // wavefront; the configuration it updates is spin column perm[l],
        // which changes only in exchange passes.  Dead lanes keep their own
        // (unused) column.
        const bool live = lane < nlanes;
        const int kslot = live ? (lane - lane0) % K : 0;
        const uint32_t sword = live ? (uint32_t(kslot) << 8) | uint32_t((lane - lane0) / K) : 0u;
        // threshold column of this lane's temperature
        // (with 4-byte columns every lane of a gather reads its own bank)
        const uint32_t thl_base = L.ths + ((uint32_t(kMaxM) * 4u) << ths_sh) + ((uint32_t(lane) << ths_sh) >> 4);
        MetroLane ml;
        {
            uint32_t h, l;
            mul_hilo(sword, M1, h, l);
            ml.a = h ^ key0;
            ml.lo = l;
        }
        int col = live ? perm[lane] : lane;
        int Es = live ? a.energy[nm * 64 + col - lane0] : 0;  // energy of slot `lane` after the last sweep
        int col_e = col;                                       // the column Es belongs to
        const int set = live ? (lane - lane0) / K : 0;          // the lane's replica set in its instance
        const int seg_lo = lane0 + set * K, seg_hi = seg_lo + K;
        int em = a.emin[nm * 64 + set];
        int64_t th = a.thit[nm * 64 + set];
        int agree = 0;
        int64_t tmax = 0;
        if (stop_mode) {
            agree = wave_min(live ? em : INT32_MAX) == wave_max(live ? em : INT32_MIN);
            tmax = wave_max64(live ? th : int64_t(0));
        }

        int64_t t = a.t[n];
        bool stopped = __builtin_amdgcn_readfirstlane(misc[1]) != 0;
        // sweeps left until the next exchange pass (0: after this sweep)
        int cd = si > 0 ? int((int64_t(si) - (t + 1) % si) % si) : -1;
        const int npairs = d.npairs;
        const int iters = d.task_iters;
        // pair tasks of this wavefront per phase: it = 0 .. nt-1 with wave + it nwaves < npairs
        const int nt = wave < npairs ? min(iters, (npairs - wave + nwaves - 1) / nwaves) : 0;
        const cptr<uint32_t> task = ws4 + d.task_off;
        // Metropolis draws: the last round's keys carry the bias kBias16 of
        // the 16-bit comparisons, so words 0 and 2 come out biased (the exact
        // pass removes it again)
        RoundKeys RK = kPacked ? round_keys_lane(key0, key1) : round_keys(key0, key1);
        RK.a[9] ^= kBias16;
        RK.b[9] ^= kBias16;

        // Philox draws do not depend on the exchange passes, since a lane's
        // slot is fixed.  The draws of the first two pairs of phase 0 are made
        // ahead (pre0, pre1), during the previous sweep's exchange pass by the
        // wavefronts that do not walk the runs.  Every other draw (the next
        // pair of the phase, or the first pair of phase 1) is computed while
        // the spin rows of the current pair are being read.
        const int nwalk = min(kPacked ? pk.n_seg : R, nwaves);  // wavefronts of the exchange walk
        // unpacked launches with at most two walkers: other wavefronts make the
        // walkers' first draws of the next sweep during the walk
        const bool hand_ok = (a.lds_mode & kLdsHand) && nwalk <= 2 && nwaves >= 3 * nwalk;
        uint4 *hand = reinterpret_cast<uint4 *>(lds + L.hand);
        uint4 pre0 = make_uint4(0u, 0u, 0u, 0u), pre1 = pre0;
        auto predraw = [&](const MetroUniform &m) {
            if (nt > 0) pre0 = metro_call(ml, m, task[(wave * 2) * iters * 16], RK);
            if (nt > 1) pre1 = metro_call(ml, m, task[((wave * 2) * iters + 1) * 16], RK);
        };
        predraw(metro_uniform(uint32_t(t), kUseMetroHi, key0, key1));
        int64_t n_ex = 0;  // exchange passes made in this launch (recording only)
        // Unpacked launches: the limits D_k of a due exchange pass (they depend
        // only on the pass's uniforms) into lim, made at the end of phase 1
        // by wavefront 0, which walks and leaves its phase-1 tasks early.
        auto make_limits = [&](uint32_t tp) {
            const uint32_t u = exchange_uniform(tp, kUseSwap, K, R, key0, key1);
            const int km1 = max(K - 1, 1);
            const int kp = lane - (lane / km1) * km1;
            if (lane < (K - 1) * R)
                lim[lane] = a.lds_ts_ok ? pair_limit<true>(u, kp, xrow, tb, a.ws32, tshi)
                                          : pair_limit<false>(u, kp, xrow, tb, a.ws32, tshi);
        };

        for (int64_t sw = 0; sw < a.n_sweeps && !stopped; ++sw) {
            const uint32_t tt = uint32_t(t);
            const uint32_t s_base = L.S + uint32_t(col) * 4u;
            const MetroUniform mu = metro_uniform(tt, kUseMetroHi, key0, key1);
            const MetroUniform mu_next = metro_uniform(tt + 1u, kUseMetroHi, key0, key1);
            int32_t *Eb = Eacc + (tt & 1u) * 64u;
            if (wave == 0) Eb[lane] = 0;
            int e4 = 0;        // phase 1: sum of (m4 ^ s) over this wavefront's sites
            uint32_t nrej = 0; // phase 1: 8 x rejected sites
            uint4 rw_next = pre0;
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                // Fair share of the SIMD between the phase's wavefronts: each
                // finished pair task lowers the wavefront's issue priority, so
                // wavefronts that are behind catch up and all reach the
                // barrier at about the same time.
                __builtin_amdgcn_s_setprio(3);
                for (int it = 0; it < nt; ++it) {
                    // task entry: counter word, quad indices, spin rows (scalar loads)
                    const cptr<uint32_t> te = task + ((wave * 2 + p) * iters + it) * 16;
                    const uint32_t c1 = te[0];
                    const uint32_t qq = te[1];
                    const bool second = (qq >> 16) != 0xFFFFu;
                    uint32_t orow[2], o0[2], oth[2], A[2], B[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        orow[h] = s_base + te[2 + 4 * h];
                        o0[h] = *reinterpret_cast<const uint32_t *>(lds + orow[h]);
                        oth[h] = *reinterpret_cast<const uint32_t *>(lds + s_base + te[3 + 4 * h]);
                        A[h] = *reinterpret_cast<const uint32_t *>(lds + s_base + te[4 + 4 * h]);
                        B[h] = *reinterpret_cast<const uint32_t *>(lds + s_base + te[5 + 4 * h]);
                    }
                    const uint4 rw = rw_next;
                    {
                        const bool last = it + 1 == nt;
                        if (p == 0 && it == 0 && !last) {
                            rw_next = pre1;
                        } else if (p == 0 || !last) {
                            const uint32_t c1n = !last ? te[16] : task[((wave * 2 + 1) * iters) * 16];
                            rw_next = metro_call(ml, mu, c1n, RK);
                        }
                    }
                    uint32_t nw[2];
                    const int e4_save = e4;
                    const uint32_t nrej_save = nrej;
                    uint32_t tmin = 0xFFFFFFFFu;
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const uint32_t q = (h == 0 || !second) ? (qq & 0xFFFFu) : (qq >> 16);
                        uint32_t jq[8];
                        const uint32_t fm = coupling_words<kPacked>(jw, livew, jwl, lml, q, jq);
                        const uint32_t x01 = __builtin_amdgcn_perm(B[h], A[h], 0x05040100u);
                        const uint32_t x23 = __builtin_amdgcn_perm(B[h], A[h], 0x07060302u);
                        const int m0 = site_m4<0>(o0[h], oth[h], x01, jq[0], jq[4]);
                        const int m1 = site_m4<1>(o0[h], oth[h], x01, jq[1], jq[5]);
                        const int m2 = site_m4<2>(o0[h], oth[h], x23, jq[2], jq[6]);
                        const int m3 = site_m4<3>(o0[h], oth[h], x23, jq[3], jq[7]);
                        // sign-flipped 16-bit thresholds of the four sites
                        const uint32_t t0 = *reinterpret_cast<const uint16_t *>(lds + thl_base + (uint32_t(m0) << ths_sh));
                        const uint32_t t1 = *reinterpret_cast<const uint16_t *>(lds + thl_base + (uint32_t(m1) << ths_sh));
                        const uint32_t t2 = *reinterpret_cast<const uint16_t *>(lds + thl_base + (uint32_t(m2) << ths_sh));
                        const uint32_t t3 = *reinterpret_cast<const uint16_t *>(lds + thl_base + (uint32_t(m3) << ths_sh));
                        const uint32_t u01 = h == 0 ? rw.x : rw.z;  // biased by the key
                        const uint32_t u23 = (h == 0 ? rw.y : rw.w) ^ kBias16;
                        // per site d = t - u (16-bit, saturated): accept iff d > 0, tie iff d == 0
                        const uint32_t d01 = sub_sat16x2(t0 | (t1 << 16), u01);
                        const uint32_t d23 = sub_sat16x2(t2 | (t3 << 16), u23);
                        tmin = min_u16x2(tmin, min_u16x2(d01, d23));
                        // reject bytes (0xFF where d < 0): the sign bits of bytes 1, 3, 5, 7
                        const uint32_t rej = __builtin_amdgcn_perm(d23, d01, 0x0B0A0908u);
                        if (p == 1 && (h == 0 || second)) {
                            // (m4 ^ s) - s = m4 if accepted, -m4 if rejected (s = -1 on reject)
                            e4 += (m0 ^ int(int8_t(rej))) + (m1 ^ int(int8_t(rej >> 8))) +
                                  (m2 ^ int(int8_t(rej >> 16))) + (m3 ^ int(int8_t(rej >> 24)));
                            nrej += __builtin_popcount(rej);
                        }
                        // flip = ~R & fm (fm = 0xFE per live site)
                        nw[h] = o0[h] ^ (~rej & fm);
                    }
                    if (__any((tmin & 0xFFFFu) == 0u || (tmin >> 16) == 0u)) {
                        // exact pass for this pair: full 32-bit uniforms
                        const MetroUniform mlo = metro_uniform(tt, kUseMetroLo, key0, key1);
                        const uint4 rlb = metro_call(ml, mlo, c1, RK);
                        const uint4 rl = make_uint4(rlb.x ^ kBias16, rlb.y, rlb.z ^ kBias16, rlb.w);
                        const uint4 rh = make_uint4(rw.x ^ kBias16, rw.y, rw.z ^ kBias16, rw.w);
                        const uint32_t *tfull = a.ws32 + tfull_off + kslot * kMRow + kMaxM;
                        e4 = e4_save;
                        nrej = nrej_save;
                        for (int h = 0; h < 2; ++h) {
                            const uint32_t q = (h == 0 || !second) ? (qq & 0xFFFFu) : (qq >> 16);
                            uint32_t jq[8];
                            const uint32_t fmq = coupling_words<kPacked>(jw, livew, jwl, lml, q, jq);
                            const uint32_t x01 = __builtin_amdgcn_perm(B[h], A[h], 0x05040100u);
                            const uint32_t x23 = __builtin_amdgcn_perm(B[h], A[h], 0x07060302u);
                            int m[4];
                            m[0] = site_m4<0>(o0[h], oth[h], x01, jq[0], jq[4]);
                            m[1] = site_m4<1>(o0[h], oth[h], x01, jq[1], jq[5]);
                            m[2] = site_m4<2>(o0[h], oth[h], x23, jq[2], jq[6]);
                            m[3] = site_m4<3>(o0[h], oth[h], x23, jq[3], jq[7]);
                            uint32_t flip = 0;
                            int ev = 0;
                            for (int k = 0; k < 4; ++k) {
                                const uint32_t uu = (half16(rh, 4 * h + k) << 16) | half16(rl, 4 * h + k);
                                const bool acc = m[k] <= 0 || uu < tfull[m[k] >> 2];
                                flip |= acc ? (0xFEu << (8 * k)) : 0u;
                                ev += acc ? m[k] : -m[k];
                            }
                            if (p == 1 && (h == 0 || second)) e4 += ev;
                            nw[h] = o0[h] ^ (flip & fmq);  // flip bytes 0xFE, fm bytes 0xFE
                        }
                    }
                    *reinterpret_cast<uint32_t *>(lds + orow[0]) = nw[0];
                    if (second) *reinterpret_cast<uint32_t *>(lds + orow[1]) = nw[1];
                    if (it == 0)
                        __builtin_amdgcn_s_setprio(2);
                    else if (it == 1)
                        __builtin_amdgcn_s_setprio(1);
                    else
                        __builtin_amdgcn_s_setprio(0);
                }
                if (p == 1 && live) atomicAdd(&Eb[lane], (e4 + int(nrej >> 3)) >> 2);
                // the uniforms of a due exchange pass (packed launches: drawn by the
                // last wavefront, by slot: pair (k, k+1) of a set at its lower
                // slot), or its limits
                if constexpr (kPacked) {
                    // by slot: pair (k, k+1) of a set at its lower slot
                    if (p == 1 && cd == 0 && wave == 0 && live && kslot < K - 1)
                        lim[lane] = pair_limit_packed(
                            philox_lane(tt, uint32_t(kslot), uint32_t(set), kUseSwap, key0, key1).x, lane, xrow,
                            a.ws32);
                } else {
                    if (p == 1 && cd == 0 && wave == 0) make_limits(tt);
                }
                __syncthreads();
            }
            // ---- energies, running minima, agreement, exchange ----
            Es = Eb[lane];  // slot `lane`: lanes seg_lo .. seg_hi - 1 are one set
            col_e = col;
            if (__any(live && Es < em)) {
                // minimum over the lane's replica set (slots seg_lo .. seg_hi - 1)
                int v = live ? Es : INT32_MAX;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const int w = __shfl(v, (lane + o) & 63, 64);
                    if (lane + o < seg_hi) v = min(v, w);
                }
                const int mn = __shfl(v, seg_lo, 64);
                if (live && mn < em) {
                    em = mn;
                    th = t + 1;
                }
                if (stop_mode) {
                    agree = wave_min(live ? em : INT32_MAX) == wave_max(live ? em : INT32_MIN);
                    tmax = wave_max64(live ? th : int64_t(0));
                }
            }
            const bool stop_now = stop_mode && agree && (t + 1) >= 2 * tmax;
            if (cd == 0) {
                if (wave >= nwalk) {
                    predraw(mu_next);
                    // helpers nwalk .. 3 nwalk - 1 also make the walkers' two draws
                    const int h = wave - nwalk;
                    if (hand_ok && h < 2 * nwalk) {
                        const int w = h >> 1, i = h & 1;
                        const int ntw = w < npairs ? min(iters, (npairs - w + nwaves - 1) / nwaves) : 0;
                        if (ntw > i)
                            hand[(w * 2 + i) * 64 + lane] =
                                metro_call(ml, mu_next, task[((w * 2) * iters + i) * 16], RK);
                    }
                }
                // the walk is the pass's critical path: its wavefronts issue first
                if (wave < nwalk) __builtin_amdgcn_s_setprio(3);
                if constexpr (kPacked)
                    exchange_walk_packed(pk.n_seg, seg_base, seg_k, wave, nwaves, Eb, lim, perm, sacc);
                else
                    exchange_walk(K, R, wave, nwaves, Eb, lim, perm, sacc);
                __syncthreads();
                if (wave < nwalk) {
                    if (hand_ok) {
                        if (nt > 0) pre0 = hand[(wave * 2) * 64 + lane];
                        if (nt > 1) pre1 = hand[(wave * 2 + 1) * 64 + lane];
                    } else {
                        predraw(mu_next);
                    }
                }
                col = live ? perm[lane] : lane;
                if constexpr (kRecord) {
                    // temperature walk: configuration col now sits at temperature kslot
                    if (wave == nwaves - 1 && n_ex < a.walk_cap && live)
                        a.walk[(int64_t(nm) * a.walk_cap + n_ex) * 64 + col - lane0] = uint8_t(kslot);
                    ++n_ex;
                }
            } else {
                predraw(mu_next);
            }
            if (si > 0) cd = cd == 0 ? si - 1 : cd - 1;
            stopped = stop_now;
            t += 1;
        }

        // ---- store state ----
        if constexpr (kPacked) {
            for (int m = 0; m < pk.n_mem; ++m) {
                // member m's lanes lane0[m] .. lane0[m] + K R - 1, its own words
                const InstDev x = load_desc(a.inst + pk.mem[m]);
                const int l0 = pk.lane0[m];
                uint64_t *spm = a.spins + x.spin_off;
                const cptr<uint32_t> lvm = ws4 + x.live_off;
                const uint64_t mmask = x.nlanes >= 64 ? ~0ull : ((1ull << x.nlanes) - 1ull);
                for (int q = wave; q < ncell * 2; q += nwaves) {
                    const uint32_t w = S[q * 64 + lane];
                    const uint32_t lm = lvm[q];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const uint64_t bits = (__ballot(((w >> (8 * k)) & 0xFFu) == 0xFFu) >> l0) & mmask;
                        if (lane == k) spm[q * 4 + k] = ((lm >> (8 * k + 1)) & 1u) ? bits : 0ull;
                    }
                }
            }
            if (wave == 0) {
                if (live) {
                    const int rr = (lane - lane0) / K;
                    a.energy[nm * 64 + col_e - lane0] = Es;
                    a.perm[nm * 64 + kslot * R + rr] = uint8_t(perm[lane] - lane0);
                    if (kslot < K - 1) a.swap_acc[nm * 64 + kslot * R + rr] = sacc[lane];
                    if (kslot == 0) {
                        a.emin[nm * 64 + rr] = em;
                        a.thit[nm * 64 + rr] = th;
                    }
                }
                if (lane < pk.n_mem) {
                    a.t[pk.mem[lane]] = t;
                    a.stopped[pk.mem[lane]] = 0;
                }
            }
            __syncthreads();
            continue;
        }
        uint64_t *spw = a.spins + d.spin_off;
        const uint64_t lane_mask = nlanes >= 64 ? ~0ull : ((1ull << nlanes) - 1ull);
        for (int q = wave; q < ncell * 2; q += nwaves) {
            const uint32_t w = S[q * 64 + lane];
            const uint32_t lm = livew[q];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint64_t bits = __ballot(((w >> (8 * k)) & 0xFFu) == 0xFFu) & lane_mask;
                if (lane == k) spw[q * 4 + k] = ((lm >> (8 * k + 1)) & 1u) ? bits : 0ull;
            }
        }
        if (wave == 0) {
            const int head = min(lane, R - 1) * K;
            const int emh = __shfl(em, head, 64);
            const int64_t thh = __shfl(th, head, 64);
            a.energy[n * 64 + (live ? col_e : lane)] = live ? Es : 0;
            a.perm[n * 64 + lane] = uint8_t(perm[lane < K * R ? (lane % R) * K + lane / R : lane]);
            a.swap_acc[n * 64 + lane] = sacc[lane];
            if (lane < R) {
                a.emin[n * 64 + lane] = emh;
                a.thit[n * 64 + lane] = thh;
            }
            if (lane == 0) {
                a.t[n] = t;
                a.stopped[n] = stopped ? 1 : 0;
            }
        }
        __syncthreads();
    }
}

__global__ void k_reset_queue(uint32_t *q) { *q = 0u; }

// ---------------------------------------------------------------------------
// Initial state: one workgroup (one wavefront) per instance.
struct InitArgs {
    const InstDev *inst;
    const uint32_t *ws32;
    uint64_t *spins;
    uint8_t *perm;
    int32_t *energy;
    int32_t *emin;
    int64_t *thit;
    uint32_t *swap_acc;
    int64_t *t;
    int32_t *stopped;
    int32_t from_buffer;
};

__device__ int lane_energy(const InstDev &d, const uint32_t *ws32, const uint64_t *sp, int lane)
{
    const uint32_t *ed = ws32 + d.edge_off;
    int e = 0;
    for (int x = 0; x < d.n_live_edges; ++x) {
        const uint32_t w = ed[x];
        const int i = int(w & 0xFFFu), j = int((w >> 12) & 0xFFFu);
        const int J = int(int8_t(uint8_t(w >> 24)));
        const int bi = int((sp[i] >> lane) & 1ull), bj = int((sp[j] >> lane) & 1ull);
        e += (bi ^ bj) ? -J : J;
    }
    return e;
}

__global__ void __launch_bounds__(64) k_pt_init(InitArgs a)
{
    const int n = blockIdx.x;
    const int lane = threadIdx.x;
    const InstDev d = a.inst[n];
    const uint32_t *livew = a.ws32 + d.live_off;
    uint64_t *sp = a.spins + d.spin_off;
    const int K = d.K, R = d.R, nlanes = d.nlanes;
    const uint64_t lane_mask = nlanes >= 64 ? ~0ull : ((1ull << nlanes) - 1ull);
    const int kk = lane % max(K, 1), rr = lane / max(K, 1);
    for (int q = 0; q < d.ncell * 2; ++q) {
        const uint32_t lm = livew[q];
        uint4 w = make_uint4(0, 0, 0, 0);
        if (!a.from_buffer && lane < nlanes)
            w = philox(0u, uint32_t(q), (uint32_t(kk) << 8) | uint32_t(rr), kUseInit, d.key0, d.key1);
        const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
        for (int k = 0; k < 4; ++k) {
            uint64_t bits;
            if (a.from_buffer)
                bits = sp[q * 4 + k] & lane_mask;
            else
                bits = __ballot(lane < nlanes && (ww[k] >> 31) != 0u) & lane_mask;
            if (!((lm >> (8 * k + 1)) & 1u)) bits = 0ull;
            if (lane == 0) sp[q * 4 + k] = bits;
        }
    }
    __syncthreads();
    const int ev = lane < nlanes ? lane_energy(d, a.ws32, sp, lane) : 0;
    a.energy[n * 64 + lane] = ev;
    a.perm[n * 64 + lane] = lane < K * R ? uint8_t((lane % R) * K + lane / R) : uint8_t(0);
    int em = 0;
    for (int r = 0; r < R; ++r) {
        const bool mine = lane >= r * K && lane < (r + 1) * K;
        const int mn = wave_min(mine ? ev : INT32_MAX);
        if (lane == r) em = mn;
    }
    a.emin[n * 64 + lane] = lane < R ? em : 0;
    a.thit[n * 64 + lane] = 0;
    a.swap_acc[n * 64 + lane] = 0u;
    if (lane == 0) {
        a.t[n] = 0;
        a.stopped[n] = 0;
    }
}

// Recomputed lane energies (Eq. 1) and count of mismatches.
__global__ void __launch_bounds__(64) k_energy(const InstDev *inst, const uint32_t *ws32,
                                               const uint64_t *spins, const int32_t *energy,
                                               int32_t *out, int32_t *mismatch)
{
    const int n = blockIdx.x, lane = threadIdx.x;
    const InstDev d = inst[n];
    const int ev = lane < d.nlanes ? lane_energy(d, ws32, spins + d.spin_off, lane) : 0;
    out[n * 64 + lane] = ev;
    if (lane < d.nlanes && ev != energy[n * 64 + lane]) atomicAdd(mismatch, 1);
}

// Configurations of the live lanes whose energy is at most e_cap[n]
// (pt_capture), one wavefront per instance and thread per lane: each
// selected lane takes an output slot from an atomic counter and writes its
// spins bit-packed (bit b of word w = site 64 w + b) and (n, lane, energy, t).
__global__ void __launch_bounds__(64) k_capture(const InstDev *inst, const uint64_t *spins, const int32_t *energy,
                                                const int64_t *tsweep, const int32_t *e_cap, uint64_t *configs,
                                                int32_t *meta, uint32_t *count, int64_t capacity, int n_words)
{
    const int n = blockIdx.x, lane = threadIdx.x;
    const InstDev d = inst[n];
    const int e = energy[n * 64 + lane];
    if (lane >= d.nlanes || e > e_cap[n]) return;
    const uint32_t at = atomicAdd(count, 1u);
    if (int64_t(at) >= capacity) return;
    const uint64_t *sp = spins + d.spin_off;
    for (int w = 0; w < n_words; ++w) {
        uint64_t word = 0;
        for (int b = 0; b < 64; ++b) {
            const int i = 64 * w + b;
            if (i < d.n_sites) word |= ((sp[i] >> lane) & 1ull) << b;
        }
        configs[int64_t(at) * n_words + w] = word;
    }
    meta[int64_t(at) * 4 + 0] = n;
    meta[int64_t(at) * 4 + 1] = lane;
    meta[int64_t(at) * 4 + 2] = e;
    meta[int64_t(at) * 4 + 3] = int32_t(tsweep[n]);
}

// One extra exchange pass per instance (pt_swap), one wavefront each.
__global__ void __launch_bounds__(64) k_swap_extra(const InstDev *inst, const TableDev *tabs,
                                                   const uint32_t *ws32, uint8_t *perm_g,
                                                   const int32_t *energy, uint32_t *swap_acc,
                                                   const int64_t *t)
{
    __shared__ int32_t E[64], perm[64], xrow[128], stopv[64 * 64];
    __shared__ uint32_t sacc[64], ux[64];
    const int n = blockIdx.x, lane = threadIdx.x;
    const InstDev d = inst[n];
    const TableDev tb = tabs[d.tab];
    const bool valid = lane < d.K * d.R;
    perm[lane] = perm_g[n * 64 + (valid ? (lane % d.K) * d.R + lane / d.K : lane)];  // set-major
    E[lane] = valid ? energy[n * 64 + perm[lane]] : 0;                                  // by slot
    sacc[lane] = swap_acc[n * 64 + lane];
    for (int i = lane; i < d.R * 64; i += 64) stopv[i] = d.K - 1;
    load_xrows(xrow, tb, ws32, d.K, lane);
    ux[lane] = exchange_uniform(uint32_t(t[n]), kUseSwapExtra, d.K, d.R, d.key0, d.key1);
    __syncthreads();
    const uint32_t dec0 = exchange_test(min(lane, d.tri * d.R - 1), d.tri, d.tri_m);
    exchange_stops<false>(d.K, d.R, d.tri, d.tri_m, 0, 1, dec0, E, ux, xrow, stopv, tb, ws32, nullptr);
    __syncthreads();
    exchange_apply(d.K, d.R, 0, 1, perm, sacc, stopv);
    __syncthreads();
    perm_g[n * 64 + lane] = uint8_t(perm[valid ? (lane % d.R) * d.K + lane / d.R : lane]);
    swap_acc[n * 64 + lane] = sacc[lane];
}

}  // namespace dev
}  // namespace hs

// ===========================================================================
// Host side of the ABI.
using namespace hs;

struct hs_pt {
    int n_inst = 0;
    hs_buffers buf{};
    hipStream_t stream = nullptr;
    uint32_t flags = 0;
    int32_t swap_interval = 0;
    int nwaves = 16;
    int grid = 0;
    int ncell_max = 0, tshi_max = 0, r_max = 1;
    int lds_ts_ok = 1;
    int lds_mode = 0;
    bool packed = false;  // the queue hands out packs of instances sharing the lanes
    int n_items = 0;      // work items of the queue
    int64_t lane_sites = 0;  // sum over work items of 64 x sites: the lane slots of one sweep
    size_t lds_bytes = 0;
    // workspace layout (uint32 offsets)
    size_t off_inst = 0, off_tabs = 0, off_order = 0, off_queue = 0, off_packs = 0;
    std::vector<uint32_t> host_ws;  // staging image of the workspace (kept until destroy)
    hipEvent_t uploaded = nullptr;  // recorded after the upload of host_ws on `stream`
};

namespace {

constexpr size_t kLdsTsBudget = 48 * 1024;  // bytes of LDS for the 16-bit exchange table
constexpr size_t kLdsLimit = 160 * 1024;    // LDS of one gfx950 workgroup

struct Plan {
    std::vector<HostInstance> hi;
    std::vector<HostTables> ht;
    std::vector<int> tab_of;
    std::vector<InstDev> idev;
    std::vector<TableDev> tdev;
    std::vector<int32_t> order;
    std::vector<PackDev> packs;   // packed launches only
    std::vector<uint32_t> image;  // workspace image in uint32 words
    int nwaves = 16;
    size_t off_inst = 0, off_tabs = 0, off_order = 0, off_queue = 0, off_packs = 0;
    int ncell_max = 0, K_max = 0, tshi_max = 0, r_max = 1;
    int lds_ts_ok = 1;
    int lds_mode = 0;
    bool packed = false;
    size_t total_words = 0;
};

// Packs of instances sharing a workgroup's lanes: within each lattice size,
// the instance with the most lanes is paired with the one with the fewest
// if their lanes fit into 64 together, else it runs alone (a two-pointer
// pass over the lane counts, which pairs as many as pairing can).
void make_packs(const std::vector<InstDev> &idev, std::vector<PackDev> &packs)
{
    packs.clear();
    for (int L = 1; L <= HS_MAX_L; ++L) {
        std::vector<int> ids;
        for (int i = 0; i < int(idev.size()); ++i)
            if (idev[i].L == L) ids.push_back(i);
        std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return idev[a].nlanes < idev[b].nlanes; });
        int lo = 0, hi = int(ids.size()) - 1;
        while (lo <= hi) {
            PackDev pk;
            std::memset(&pk, 0, sizeof(pk));
            const InstDev &big = idev[ids[hi]];
            pk.mem[0] = ids[hi];
            pk.n_mem = 1;
            pk.nlanes = big.nlanes;
            pk.n_seg = big.R;
            if (lo < hi && big.nlanes + idev[ids[lo]].nlanes <= HS_MAX_LANES) {
                const InstDev &sm = idev[ids[lo]];
                pk.mem[1] = ids[lo];
                pk.lane0[1] = big.nlanes;
                pk.n_mem = 2;
                pk.nlanes += sm.nlanes;
                pk.n_seg += sm.R;
                ++lo;
            }
            pk.cost = int64_t(big.ncell);
            packs.push_back(pk);
            --hi;
        }
    }
}

size_t align16w(size_t w) { return (w + 3) & ~size_t(3); }

template <class T>
size_t append(std::vector<uint32_t> &img, const T *p, size_t count)
{
    const size_t at = align16w(img.size());
    img.resize(at);
    const size_t words = (count * sizeof(T) + 3) / 4;
    img.resize(at + words, 0u);
    if (count) std::memcpy(img.data() + at, p, count * sizeof(T));
    return at;
}

int validate_inst(const hs_instance &in, std::string &err)
{
    if (in.K < 1 || in.R < 1 || in.K * in.R > HS_MAX_LANES) {
        err = "need K >= 1, R >= 1, K*R <= 64";
        return HS_EUNSUPPORTED;
    }
    if (in.beta == nullptr) {
        err = "beta is NULL";
        return HS_EINVAL;
    }
    for (int k = 0; k < in.K; ++k) {
        if (!(in.beta[k] > 0.0) || !std::isfinite(in.beta[k])) {
            err = "beta must be positive and finite";
            return HS_EINVAL;
        }
        if (k > 0 && !(in.beta[k] > in.beta[k - 1])) {
            err = "beta must be strictly ascending";
            return HS_EINVAL;
        }
    }
    return HS_OK;
}

int make_plan(const hs_pt_desc &d, Plan &P, std::string &err)
{
    if (d.n_inst < 0 || (d.n_inst > 0 && d.inst == nullptr)) {
        err = "bad instance array";
        return HS_EINVAL;
    }
    if (d.swap_interval < 0) {
        err = "swap_interval must be >= 0";
        return HS_EINVAL;
    }
    if (d.block_waves < 0 || d.block_waves > 16) {
        err = "block_waves must be in 0..16";
        return HS_EINVAL;
    }
    if ((d.flags & HS_PACK_LANES) && (d.flags & HS_STOP_ON_AGREEMENT)) {
        err = "HS_PACK_LANES cannot be combined with HS_STOP_ON_AGREEMENT";
        return HS_EINVAL;
    }
    const int n = d.n_inst;
    P.hi.resize(n);
    P.tab_of.resize(n);
    // largest energy difference between two configurations of any instance:
    // 2 sum |J| over its live couplers (bounds the exchange tables)
    int64_t d_cap = 0;
    for (int i = 0; i < n; ++i) {
        const hs_instance &in = d.inst[i];
        int rc = validate_inst(in, err);
        if (rc) return rc;
        rc = build_instance(in, P.hi[i], err);
        if (rc) return rc;
        if ((d.flags & HS_STOP_ON_AGREEMENT) && in.R < 2) {
            err = "HS_STOP_ON_AGREEMENT needs R >= 2";
            return HS_EINVAL;
        }
        int64_t sum_j = 0;
        for (uint32_t e : P.hi[i].edges) sum_j += std::abs(int(int8_t(uint8_t(e >> 24))));
        d_cap = std::max(d_cap, 2 * sum_j);
    }
    for (int i = 0; i < n; ++i) {
        const hs_instance &in = d.inst[i];
        // share tables between instances with the same ladder
        int found = -1;
        for (size_t t = 0; t < P.ht.size(); ++t)
            if (P.ht[t].K == in.K && std::memcmp(P.ht[t].beta.data(), in.beta, sizeof(double) * in.K) == 0) {
                found = int(t);
                break;
            }
        if (found < 0) {
            P.ht.emplace_back();
            build_tables(in.K, in.beta, d_cap, P.ht.back());
            if (P.ht.back().ts_full.size() > (size_t(1) << 24)) {
                err = "temperature ladder too dense for the exchange tables";
                return HS_EUNSUPPORTED;
            }
            found = int(P.ht.size()) - 1;
        }
        P.tab_of[i] = found;
        P.ncell_max = std::max(P.ncell_max, P.hi[i].ncell);
        P.K_max = std::max(P.K_max, in.K);
        P.r_max = std::max(P.r_max, in.R);
    }
    // wavefronts per workgroup: one per cell pair of the largest instance, up to 16
    if (d.block_waves > 0) {
        P.nwaves = d.block_waves;
    } else {
        const int pairs = (P.ncell_max + 1) / 2;
        P.nwaves = 1;
        while (P.nwaves < pairs && P.nwaves < 16) P.nwaves *= 2;
    }
    // workspace image: [InstDev][TableDev][order][queue][per-instance data][tables]
    std::vector<uint32_t> &img = P.image;
    img.clear();
    P.idev.resize(n);
    P.tdev.resize(P.ht.size());
    P.off_inst = 0;
    img.resize(align16w(sizeof(InstDev) * n / 4 + 4));
    P.off_tabs = img.size();
    img.resize(align16w(P.off_tabs + sizeof(TableDev) * P.tdev.size() / 4 + 4));
    P.off_order = img.size();
    img.resize(align16w(P.off_order + n + 4));
    P.off_queue = img.size();
    img.resize(align16w(P.off_queue + 4));
    int64_t spin_off = 0;
    int64_t task_off[HS_MAX_L + 1];
    int task_iters[HS_MAX_L + 1];
    for (int l = 0; l <= HS_MAX_L; ++l) task_off[l] = -1;
    for (int i = 0; i < n; ++i) {
        const int Lx = d.inst[i].L;
        if (task_off[Lx] >= 0) continue;
        std::vector<uint32_t> tk;
        build_tasks(Lx, P.nwaves, tk, task_iters[Lx]);
        task_off[Lx] = int64_t(append(img, tk.data(), tk.size()));
    }
    for (int i = 0; i < n; ++i) {
        const hs_instance &in = d.inst[i];
        InstDev &x = P.idev[i];
        std::memset(&x, 0, sizeof(x));
        x.L = in.L;
        x.ncell = in.L * in.L;
        x.npairs = (x.ncell + 1) / 2;
        x.K = in.K;
        x.R = in.R;
        x.nlanes = in.K * in.R;
        x.n_sites = 8 * in.L * in.L;
        x.tab = P.tab_of[i];
        x.key0 = in.instance_id;
        x.key1 = d.seed;
        x.spin_off = spin_off;
        spin_off += x.n_sites;
        x.jw_off = int64_t(append(img, P.hi[i].jw.data(), P.hi[i].jw.size()));
        x.live_off = int64_t(append(img, P.hi[i].live.data(), P.hi[i].live.size()));
        x.edge_off = int64_t(append(img, P.hi[i].edges.data(), P.hi[i].edges.size()));
        x.n_live_edges = int32_t(P.hi[i].edges.size());
        x.task_off = task_off[in.L];
        x.task_iters = task_iters[in.L];
        x.cost = int64_t(x.ncell);
        x.tri = (in.K - 1) * in.K / 2;
        x.tri_m = x.tri > 1 ? uint32_t(((uint64_t(1) << 32) + uint64_t(x.tri) - 1) / uint64_t(x.tri)) : 0u;
        x.k_m = uint32_t((65536 + in.K - 1) / in.K);
    }
    for (size_t t = 0; t < P.ht.size(); ++t) {
        const HostTables &h = P.ht[t];
        TableDev &x = P.tdev[t];
        std::memset(&x, 0, sizeof(x));
        x.K = h.K;
        x.lds_ts_entries = int32_t(h.ts_hi.size());
        x.thi_off = int64_t(append(img, h.thi.data(), h.thi.size()));
        x.tfull_off = int64_t(append(img, h.tfull.data(), h.tfull.size()));
        x.ts_row_off = int64_t(append(img, h.ts_row.data(), h.ts_row.size()));
        x.ts_dhi_off = int64_t(append(img, h.ts_dhi.data(), h.ts_dhi.size()));
        x.ts_dmax_off = int64_t(append(img, h.ts_dmax.data(), h.ts_dmax.size()));
        x.ts_hi_off = int64_t(append(img, h.ts_hi.data(), h.ts_hi.size()));
        x.ts_full_off = int64_t(append(img, h.ts_full.data(), h.ts_full.size()));
        x.ts_full_row_off = int64_t(append(img, h.ts_full_row.data(), h.ts_full_row.size()));
        x.ts_rate_off = int64_t(append(img, h.ts_rate.data(), h.ts_rate.size()));
        P.tshi_max = std::max(P.tshi_max, int(h.ts_hi.size()));
    }
    // Packed launch: the packs, their LDS layout (exchange tables stay in
    // global memory); kept only if it fits, packs something, and every
    // workspace offset fits the 32-bit indices of the packed exchange tables
    if (d.flags & HS_PACK_LANES) {
        make_packs(P.idev, P.packs);
        int nseg = 1;
        for (const PackDev &pk : P.packs) nseg = std::max(nseg, pk.n_seg);
        // the walkers' hand-over if it fits
        const int modes[4] = {dev::kLdsHand, 0, dev::kLdsHand | 1, 1};
        for (int m : modes)
            if (!P.packed && P.packs.size() < size_t(n) &&
                dev::lds_layout(P.ncell_max, 0, nseg, m | dev::kLdsPacked).total <= kLdsLimit &&
                img.size() < (size_t(1) << 29)) {
                P.packed = true;
                P.lds_mode = m | dev::kLdsPacked;
                P.lds_ts_ok = 0;
                P.tshi_max = 0;
                P.r_max = nseg;
            }
        if (!P.packed) P.packs.clear();
    }
    // LDS layout: the fast exchange table in LDS first, then 4-byte threshold
    // columns, whichever fit
    if (!P.packed) {
        // 4-byte threshold columns first, with the walkers' hand-over if it fits
        const int modes[4] = {dev::kLdsHand, 0, dev::kLdsHand | 1, 1};
        bool found = false;
        if (size_t(P.tshi_max) * 2 <= kLdsTsBudget) {
            for (int m : modes)
                if (!found && dev::lds_layout(P.ncell_max, P.tshi_max, P.r_max, m).total <= kLdsLimit) {
                    P.lds_mode = m;
                    found = true;
                }
        }
        if (!found) {
            P.lds_ts_ok = 0;
            P.tshi_max = 0;
            for (int m : modes)
                if (!found && dev::lds_layout(P.ncell_max, 0, P.r_max, m).total <= kLdsLimit) {
                    P.lds_mode = m;
                    found = true;
                }
        }
        if (!found) {
            err = "instance too large for one workgroup's LDS";
            return HS_EUNSUPPORTED;
        }
    }
    // order: most expensive first (instances, or packs)
    const int items = P.packed ? int(P.packs.size()) : n;
    P.order.resize(items);
    std::iota(P.order.begin(), P.order.end(), 0);
    if (P.packed)
        std::stable_sort(P.order.begin(), P.order.end(),
                         [&](int a, int b) { return P.packs[a].cost > P.packs[b].cost; });
    else
        std::stable_sort(P.order.begin(), P.order.end(),
                         [&](int a, int b) { return P.idev[a].cost > P.idev[b].cost; });
    if (P.packed) P.off_packs = append(img, P.packs.data(), P.packs.size());
    std::memcpy(img.data() + P.off_inst, P.idev.data(), sizeof(InstDev) * n);
    std::memcpy(img.data() + P.off_tabs, P.tdev.data(), sizeof(TableDev) * P.tdev.size());
    std::memcpy(img.data() + P.off_order, P.order.data(), sizeof(int32_t) * items);
    P.total_words = align16w(img.size());
    img.resize(P.total_words, 0u);
    return HS_OK;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(HS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                  \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return hip_fail(_e, #expr); \
    } while (0)

int device_cus()
{
    static const int cus = [] {  // thread-safe one-time initialisation
        int dev = 0, n = 1;
        if (hipGetDevice(&dev) != hipSuccess) return 1;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
        return n;
    }();
    return cus;
}

}  // namespace

extern "C" {

int pt_workspace_bytes(const hs_pt_desc *d, size_t *bytes)
{
    if (d == nullptr || bytes == nullptr) return fail(HS_EINVAL, "pt_workspace_bytes: NULL argument");
    Plan P;
    std::string err;
    int rc = make_plan(*d, P, err);
    if (rc) return fail(rc, "pt_workspace_bytes: " + err);
    *bytes = P.total_words * 4;
    return HS_OK;
}

int pt_init(hs_pt **out, const hs_pt_desc *d, const hs_buffers *b, void *stream)
{
    return hs::pt_init_ex(out, d, b, stream, true);
}

}  // extern "C"

// track_upload = false: no event is created; the caller synchronises the
// stream before pt_destroy (the upload reads the handle's host copy).
int hs::pt_init_ex(hs_pt **out, const hs_pt_desc *d, const hs_buffers *b, void *stream, bool track_upload)
{
    if (out == nullptr || d == nullptr || b == nullptr) return fail(HS_EINVAL, "pt_init: NULL argument");
    *out = nullptr;
    Plan P;
    std::string err;
    int rc = make_plan(*d, P, err);
    if (rc) return fail(rc, "pt_init: " + err);
    if (d->n_inst > 0 && (b->spins == nullptr || b->perm == nullptr || b->energy == nullptr ||
                          b->emin == nullptr || b->thit == nullptr || b->swap_acc == nullptr ||
                          b->t == nullptr || b->stopped == nullptr || b->workspace == nullptr))
        return fail(HS_EINVAL, "pt_init: NULL device buffer");
    if (b->workspace_bytes < P.total_words * 4)
        return fail(HS_ENOSPACE, "pt_init: workspace too small (need " + std::to_string(P.total_words * 4) +
                                     " bytes)");
    auto h = new hs_pt();
    h->n_inst = d->n_inst;
    h->buf = *b;
    h->stream = reinterpret_cast<hipStream_t>(stream);
    h->flags = d->flags;
    h->swap_interval = d->swap_interval;
    h->nwaves = P.nwaves;
    h->ncell_max = P.ncell_max;
    h->tshi_max = P.tshi_max;
    h->r_max = P.r_max;
    h->lds_ts_ok = P.lds_ts_ok;
    h->lds_mode = P.lds_mode;
    h->packed = P.packed;
    h->n_items = P.packed ? int(P.packs.size()) : d->n_inst;
    if (P.packed)
        for (const PackDev &pk : P.packs) h->lane_sites += 64 * int64_t(P.idev[pk.mem[0]].n_sites);
    else
        for (const InstDev &x : P.idev) h->lane_sites += 64 * int64_t(x.n_sites);
    h->off_inst = P.off_inst;
    h->off_tabs = P.off_tabs;
    h->off_order = P.off_order;
    h->off_queue = P.off_queue;
    h->off_packs = P.off_packs;
    h->lds_bytes = dev::lds_layout(h->ncell_max, h->tshi_max, h->r_max, h->lds_mode).total;
    h->host_ws = std::move(P.image);
    if (h->n_inst == 0) {
        *out = h;
        return HS_OK;
    }
    hipError_t e = hipMemcpyAsync(b->workspace, h->host_ws.data(), h->host_ws.size() * 4,
                                  hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess && track_upload) e = hipEventCreateWithFlags(&h->uploaded, hipEventDisableTiming);
    if (e == hipSuccess && track_upload) e = hipEventRecord(h->uploaded, h->stream);
    // after an error once the upload is enqueued: wait for it (it reads
    // h->host_ws), then free the handle
    auto abort_init = [&](int rc) {
        (void)hipStreamSynchronize(h->stream);
        pt_destroy(h);
        return rc;
    };
    if (e != hipSuccess) return abort_init(hip_fail(e, "pt_init: upload"));
    const char *ws = reinterpret_cast<const char *>(b->workspace);
    dev::InitArgs ia;
    ia.inst = reinterpret_cast<const InstDev *>(ws + h->off_inst * 4);
    ia.ws32 = reinterpret_cast<const uint32_t *>(ws);
    ia.spins = b->spins;
    ia.perm = b->perm;
    ia.energy = b->energy;
    ia.emin = b->emin;
    ia.thit = b->thit;
    ia.swap_acc = b->swap_acc;
    ia.t = b->t;
    ia.stopped = b->stopped;
    ia.from_buffer = (d->flags & HS_INIT_FROM_BUFFER) ? 1 : 0;
    hipLaunchKernelGGL(dev::k_pt_init, dim3(h->n_inst), dim3(64), 0, h->stream, ia);
    e = hipGetLastError();
    if (e != hipSuccess) return abort_init(hip_fail(e, "pt_init: launch"));
    const void *kfn = h->packed ? reinterpret_cast<const void *>(&dev::k_pt_sweep<false, true>)
                                : reinterpret_cast<const void *>(&dev::k_pt_sweep<false, false>);
    const void *kfn_rec = h->packed ? reinterpret_cast<const void *>(&dev::k_pt_sweep<true, true>)
                                    : reinterpret_cast<const void *>(&dev::k_pt_sweep<true, false>);
    if (h->lds_bytes > 64 * 1024) {
        e = hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, int(h->lds_bytes));
        if (e == hipSuccess)
            e = hipFuncSetAttribute(kfn_rec, hipFuncAttributeMaxDynamicSharedMemorySize, int(h->lds_bytes));
        if (e != hipSuccess) return abort_init(hip_fail(e, "pt_init: LDS size"));
    }
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, h->nwaves * 64, h->lds_bytes);
    if (e != hipSuccess || per_cu < 1)
        return abort_init(fail(HS_EUNSUPPORTED, "pt_init: instances too large for one workgroup's LDS"));
    h->grid = std::min(h->n_items, per_cu * device_cus());
    *out = h;
    return HS_OK;
}

namespace {

// Enqueues the work-queue reset and the persistent sweep kernel on `stream`.
int sweep_launch(hs_pt *h, int64_t n_sweeps, hipStream_t stream, uint8_t *walk = nullptr,
                 int64_t walk_cap = 0)
{
    char *ws = reinterpret_cast<char *>(h->buf.workspace);
    dev::SweepArgs a;
    a.inst = reinterpret_cast<const InstDev *>(ws + h->off_inst * 4);
    a.tabs = reinterpret_cast<const TableDev *>(ws + h->off_tabs * 4);
    a.packs = reinterpret_cast<const PackDev *>(ws + h->off_packs * 4);
    a.ws32 = reinterpret_cast<const uint32_t *>(ws);
    a.order = reinterpret_cast<const int32_t *>(ws + h->off_order * 4);
    a.queue = reinterpret_cast<uint32_t *>(ws + h->off_queue * 4);
    a.spins = h->buf.spins;
    a.perm = h->buf.perm;
    a.energy = h->buf.energy;
    a.emin = h->buf.emin;
    a.thit = h->buf.thit;
    a.swap_acc = h->buf.swap_acc;
    a.t = h->buf.t;
    a.stopped = h->buf.stopped;
    a.n_inst = h->n_inst;
    a.n_items = h->n_items;
    a.swap_interval = h->swap_interval;
    a.n_sweeps = n_sweeps;
    a.flags = h->flags;
    a.ncell_max = h->ncell_max;
    a.tshi_max = h->tshi_max;
    a.r_max = h->r_max;
    a.lds_ts_ok = h->lds_ts_ok;
    a.lds_mode = h->lds_mode;
    a.walk = walk;
    a.walk_cap = walk_cap;
    hipLaunchKernelGGL(dev::k_reset_queue, dim3(1), dim3(1), 0, stream, a.queue);
    const dim3 grid(h->grid), block(h->nwaves * 64);
    if (walk != nullptr && h->packed)
        hipLaunchKernelGGL((dev::k_pt_sweep<true, true>), grid, block, h->lds_bytes, stream, a);
    else if (walk != nullptr)
        hipLaunchKernelGGL((dev::k_pt_sweep<true, false>), grid, block, h->lds_bytes, stream, a);
    else if (h->packed)
        hipLaunchKernelGGL((dev::k_pt_sweep<false, true>), grid, block, h->lds_bytes, stream, a);
    else
        hipLaunchKernelGGL((dev::k_pt_sweep<false, false>), grid, block, h->lds_bytes, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "pt_sweep: launch");
    return HS_OK;
}

}  // namespace

struct hs_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t stream = nullptr;
};

extern "C" {

int pt_sweep(hs_pt *h, int64_t n_sweeps)
{
    if (h == nullptr || n_sweeps < 0) return fail(HS_EINVAL, "pt_sweep: bad arguments");
    if (h->n_inst == 0 || n_sweeps == 0) return HS_OK;
    return sweep_launch(h, n_sweeps, h->stream);
}

int pt_sweep_record(hs_pt *h, int64_t n_sweeps, uint8_t *walk, int64_t capacity)
{
    if (h == nullptr || n_sweeps < 0 || capacity < 0 || (walk == nullptr && capacity > 0))
        return fail(HS_EINVAL, "pt_sweep_record: bad arguments");
    if (h->n_inst == 0 || n_sweeps == 0) return HS_OK;
    return sweep_launch(h, n_sweeps, h->stream, walk, capacity);
}

int pt_graph_create(hs_pt *h, int64_t n_sweeps, hs_graph **out)
{
    if (h == nullptr || out == nullptr || n_sweeps < 0) return fail(HS_EINVAL, "pt_graph_create: bad arguments");
    *out = nullptr;
    hipGraph_t g = nullptr;
    if (h->n_inst == 0 || n_sweeps == 0) {
        HIP_TRY(hipGraphCreate(&g, 0));
    } else {
        // capture on a private stream (the handle's stream may be the legacy default stream)
        hipStream_t cs = nullptr;
        HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            (void)hipStreamDestroy(cs);
            return hip_fail(e, "pt_graph_create: begin capture");
        }
        const int rc = sweep_launch(h, n_sweeps, cs);
        const hipError_t e2 = hipStreamEndCapture(cs, &g);
        (void)hipStreamDestroy(cs);
        if (rc != HS_OK || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return rc != HS_OK ? rc : hip_fail(e2, "pt_graph_create: end capture");
        }
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "pt_graph_create: instantiate");
    }
    auto G = new hs_graph();
    G->graph = g;
    G->exec = ex;
    G->stream = h->stream;
    *out = G;
    return HS_OK;
}

int pt_graph_launch(hs_graph *g)
{
    if (g == nullptr) return fail(HS_EINVAL, "pt_graph_launch: NULL graph");
    HIP_TRY(hipGraphLaunch(g->exec, g->stream));
    return HS_OK;
}

int pt_graph_destroy(hs_graph *g)
{
    if (g == nullptr) return HS_OK;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return HS_OK;
}

int pt_autotune(const hs_pt_desc *d, const hs_buffers *scratch, void *stream, int64_t trial_sweeps,
                int32_t *block_waves_out, double *us_per_sweep_out)
{
    if (d == nullptr || scratch == nullptr || block_waves_out == nullptr || trial_sweeps < 1)
        return fail(HS_EINVAL, "pt_autotune: bad arguments");
    const int cand[] = {2, 4, 8, 16};
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int best = 0;
    double best_us = 0.0;
    int rc = HS_OK;
    for (int c : cand) {
        hs_pt_desc dc = *d;
        dc.block_waves = c;
        dc.flags &= ~HS_INIT_FROM_BUFFER;
        size_t need = 0;
        rc = pt_workspace_bytes(&dc, &need);
        if (rc != HS_OK) break;
        if (need > scratch->workspace_bytes) continue;
        hs_pt *h = nullptr;
        rc = pt_init(&h, &dc, scratch, stream);
        if (rc != HS_OK) break;
        rc = pt_sweep(h, std::max<int64_t>(1, trial_sweeps / 8));  // warm-up
        hipError_t e = hipSuccess;
        if (rc == HS_OK) e = hipEventRecord(e0, st);
        if (rc == HS_OK && e == hipSuccess) rc = pt_sweep(h, trial_sweeps);
        if (rc == HS_OK && e == hipSuccess) e = hipEventRecord(e1, st);
        if (rc == HS_OK && e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (rc == HS_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        pt_destroy(h);
        if (rc != HS_OK) break;
        if (e != hipSuccess) {
            rc = hip_fail(e, "pt_autotune: timing");
            break;
        }
        const double us = double(ms) * 1e3 / double(trial_sweeps);
        if (best == 0 || us < best_us) {
            best = c;
            best_us = us;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != HS_OK) return rc;
    if (best == 0) return fail(HS_ENOSPACE, "pt_autotune: scratch workspace too small for every candidate");
    *block_waves_out = best;
    if (us_per_sweep_out) *us_per_sweep_out = best_us;
    return HS_OK;
}

int pt_swap(hs_pt *h)
{
    if (h == nullptr) return fail(HS_EINVAL, "pt_swap: NULL handle");
    if (h->n_inst == 0) return HS_OK;
    char *ws = reinterpret_cast<char *>(h->buf.workspace);
    hipLaunchKernelGGL(dev::k_swap_extra, dim3(h->n_inst), dim3(64), 0, h->stream,
                       reinterpret_cast<const InstDev *>(ws + h->off_inst * 4),
                       reinterpret_cast<const TableDev *>(ws + h->off_tabs * 4),
                       reinterpret_cast<const uint32_t *>(ws), h->buf.perm, h->buf.energy,
                       h->buf.swap_acc, h->buf.t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "pt_swap: launch");
    return HS_OK;
}

int pt_measure(hs_pt *h, int32_t *recomputed, int32_t *n_mismatch)
{
    if (h == nullptr || recomputed == nullptr) return fail(HS_EINVAL, "pt_measure: bad arguments");
    if (n_mismatch) *n_mismatch = 0;
    if (h->n_inst == 0) return HS_OK;
    char *ws = reinterpret_cast<char *>(h->buf.workspace);
    // mismatch counter lives in the queue slot's neighbour word
    int32_t *mm = reinterpret_cast<int32_t *>(ws + h->off_queue * 4) + 1;
    hipLaunchKernelGGL(dev::k_reset_queue, dim3(1), dim3(1), 0, h->stream, reinterpret_cast<uint32_t *>(mm));
    hipLaunchKernelGGL(dev::k_energy, dim3(h->n_inst), dim3(64), 0, h->stream,
                       reinterpret_cast<const InstDev *>(ws + h->off_inst * 4),
                       reinterpret_cast<const uint32_t *>(ws), h->buf.spins, h->buf.energy, recomputed, mm);
    HIP_TRY(hipGetLastError());
    int32_t host_mm = 0;
    HIP_TRY(hipMemcpyAsync(&host_mm, mm, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (n_mismatch) *n_mismatch = host_mm;
    if (host_mm != 0) return fail(HS_EMISMATCH, "pt_measure: incremental and recomputed energies differ");
    return HS_OK;
}

int pt_capture(hs_pt *h, const int32_t *e_cap, uint64_t *configs, int32_t *meta, uint32_t *count, int64_t capacity,
               int n_words)
{
    if (h == nullptr || e_cap == nullptr || configs == nullptr || meta == nullptr || count == nullptr ||
        capacity < 0 || n_words < (8 * h->ncell_max + 63) / 64)
        return fail(HS_EINVAL, "pt_capture: bad arguments");
    if (h->n_inst == 0) return HS_OK;
    char *ws = reinterpret_cast<char *>(h->buf.workspace);
    hipLaunchKernelGGL(dev::k_capture, dim3(h->n_inst), dim3(64), 0, h->stream,
                       reinterpret_cast<const InstDev *>(ws + h->off_inst * 4), h->buf.spins, h->buf.energy, h->buf.t,
                       e_cap, configs, meta, count, capacity, n_words);
    HIP_TRY(hipGetLastError());
    return HS_OK;
}

int pt_destroy(hs_pt *h)
{
    if (h == nullptr) return HS_OK;
    int rc = HS_OK;
    if (h->uploaded != nullptr) {
        // the upload reads host_ws asynchronously: wait for it before freeing
        const hipError_t e = hipEventSynchronize(h->uploaded);
        if (e != hipSuccess) rc = hip_fail(e, "pt_destroy: waiting for the workspace upload");
        (void)hipEventDestroy(h->uploaded);
    }
    delete h;
    return rc;
}

int pt_launch_shape(const hs_pt *h, int32_t *grid, int32_t *block_waves, int32_t *lds_bytes, int32_t *work_items,
                    int64_t *lane_sites)
{
    if (h == nullptr) return fail(HS_EINVAL, "pt_launch_shape: NULL handle");
    if (grid) *grid = h->grid;
    if (block_waves) *block_waves = h->nwaves;
    if (lds_bytes) *lds_bytes = int32_t(h->lds_bytes);
    if (work_items) *work_items = h->n_items;
    if (lane_sites) *lane_sites = h->lane_sites;
    return HS_OK;
}

}  // extern "C"
