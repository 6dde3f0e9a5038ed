// Mixing-time statistics of the PT temperature random walk (Sec. III.B):
// exact autocorrelation sums of the centred temperature index and hot-half
// residency per configuration, from the walks pt_sweep_record writes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "../../include/hs_walk.h"
#include "hs_internal.h"

namespace hs {
namespace dev {

constexpr int kLagTile = 64;    // lags per workgroup: 4 runs of 16 consecutive lags
constexpr int kTimeTile = 256;  // passes per LDS tile (a multiple of 4)
constexpr int kBaseW = kTimeTile / 4 + 1;                 // words per configuration row (odd: no bank clash)
constexpr int kShiftW = (kTimeTile + kLagTile) / 4 + 1;   // the lag window needs one word past the tile

// Centred index g = 2 k - (K - 1) as a byte (|g| <= 63); 0 past the run and
// for configurations beyond K R.
__device__ __forceinline__ uint32_t g_byte(const uint8_t *src, int64_t t, int64_t T, int cc, int C, int K)
{
    if (t >= T || cc >= C) return 0u;
    return uint32_t(uint8_t(int8_t(2 * int(src[t * 64 + cc]) - (K - 1))));
}

// Workgroup (n, lag tile): 256 threads = 64 configurations x 4 runs of 16
// lags; thread (c, j) sums lags d = d0 + 16 j + i, i < 16.  A tile stages,
// per configuration row, g of passes [t0, t0 + kTimeTile) (base) and
// [t0 + d0, t0 + d0 + kTimeTile + kLagTile + 4) (shifted) packed four passes
// to a word (byte b of word w = pass 4 w + b).  For four passes t .. t + 3
// the products g(t + u) g(t + u + d) of one lag are one 4-way signed byte
// dot product of the base word and the shifted bytes at offset t + d,
// aligned out of two neighbouring words; a window of five shifted words
// serves the 16 lags and slides by one word per four passes.
__global__ void __launch_bounds__(256) k_walk_acf(const uint8_t *walk, int64_t cap, int64_t T, int K, int C,
                                                  int max_lag, int64_t *acf)
{
    __shared__ uint32_t base[64 * kBaseW];
    __shared__ uint32_t shifted[64 * kShiftW];
    const int n = blockIdx.x;
    const int d0 = blockIdx.y * kLagTile;
    const int c = threadIdx.x & 63, j = threadIdx.x >> 6;
    const uint8_t *src = walk + int64_t(n) * cap * 64;
    int64_t acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0;
    for (int64_t t0 = 0; t0 < T - d0; t0 += kTimeTile) {
        __syncthreads();
        // lane c of each wavefront reads configuration c: 64-byte rows of the walk
        for (int w = j; w < kTimeTile / 4; w += 4) {
            const int64_t t = t0 + 4 * w;
            base[c * kBaseW + w] = g_byte(src, t, T, c, C, K) | (g_byte(src, t + 1, T, c, C, K) << 8) |
                                   (g_byte(src, t + 2, T, c, C, K) << 16) | (g_byte(src, t + 3, T, c, C, K) << 24);
        }
        for (int w = j; w < kShiftW; w += 4) {
            const int64_t t = t0 + d0 + 4 * w;
            shifted[c * kShiftW + w] = g_byte(src, t, T, c, C, K) | (g_byte(src, t + 1, T, c, C, K) << 8) |
                                       (g_byte(src, t + 2, T, c, C, K) << 16) |
                                       (g_byte(src, t + 3, T, c, C, K) << 24);
        }
        __syncthreads();
        int32_t part[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) part[i] = 0;
        const uint32_t *brow = base + c * kBaseW;
        const uint32_t *srow = shifted + c * kShiftW + 4 * j;
        uint32_t win[5];
#pragma unroll
        for (int k = 0; k < 4; ++k) win[k] = srow[k];
#pragma unroll 4
        for (int q = 0; q < kTimeTile / 4; ++q) {
            win[4] = srow[q + 4];
            const int32_t b = int32_t(brow[q]);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const uint32_t h = (i & 3) == 0 ? win[i >> 2] : __builtin_amdgcn_alignbyte(win[(i >> 2) + 1], win[i >> 2], i & 3);
                part[i] = __builtin_amdgcn_sdot4(b, int32_t(h), part[i], false);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) win[k] = win[k + 1];
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] += part[i];
    }
    // sum over the 64 configurations of this wavefront's lanes
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        int64_t v = acc[i];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
        const int d = d0 + 16 * j + i;
        if (c == 0 && d <= max_lag) acf[int64_t(n) * (max_lag + 1) + d] = v;
    }
}

// One wavefront per instance: passes with k < K / 2 per configuration.
__global__ void __launch_bounds__(64) k_walk_hot(const uint8_t *walk, int64_t cap, int64_t T, int K, int C,
                                                 int64_t *hot)
{
    const int n = blockIdx.x, c = threadIdx.x;
    const uint8_t *src = walk + int64_t(n) * cap * 64;
    int64_t h = 0;
    if (c < C)
        for (int64_t t = 0; t < T; ++t) h += src[t * 64 + c] < uint8_t(K / 2) ? 1 : 0;
    hot[int64_t(n) * 64 + c] = h;
}

}  // namespace dev
}  // namespace hs

using namespace hs;

extern "C" {

int walk_autocorr(const uint8_t *walk, int n_inst, int64_t capacity, int64_t n_steps, int K, int R,
                  int max_lag, int64_t *acf, int64_t *hot, void *stream)
{
    if (n_inst < 0 || n_steps < 0 || n_steps > capacity || K < 1 || R < 1 || K * R > 64 || max_lag < 0 ||
        max_lag > 65535)
        return fail(HS_EINVAL, "walk_autocorr: bad sizes");
    if (n_inst == 0) return HS_OK;
    if (walk == nullptr || acf == nullptr || hot == nullptr) return fail(HS_EINVAL, "walk_autocorr: NULL buffer");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const dim3 grid(unsigned(n_inst), unsigned((max_lag + dev::kLagTile) / dev::kLagTile));
    hipLaunchKernelGGL(dev::k_walk_acf, grid, dim3(256), 0, s, walk, capacity, n_steps, K, K * R, max_lag, acf);
    hipLaunchKernelGGL(dev::k_walk_hot, dim3(unsigned(n_inst)), dim3(64), 0, s, walk, capacity, n_steps, K, K * R,
                       hot);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(HS_EHIP, std::string("walk_autocorr: launch: ") + hipGetErrorString(e));
    return HS_OK;
}

int walk_tau(const int64_t *acf, int max_lag, int64_t n_steps, double c_window, double *tau, int *window,
             int *converged)
{
    if (acf == nullptr || tau == nullptr || window == nullptr || converged == nullptr || max_lag < 0)
        return fail(HS_EINVAL, "walk_tau: bad arguments");
    *tau = 0.5;
    *window = 0;
    *converged = 0;
    if (n_steps < 2 || acf[0] <= 0) return HS_OK;
    const double c0 = double(acf[0]) / double(n_steps);
    double t = 0.5;
    int64_t w_max = std::min<int64_t>(max_lag, n_steps - 1);
    for (int64_t w = 1; w <= w_max; ++w) {
        t += (double(acf[w]) / double(n_steps - w)) / c0;
        if (double(w) >= c_window * t) {
            *tau = t;
            *window = int(w);
            *converged = 1;
            return HS_OK;
        }
    }
    *tau = t;
    *window = int(w_max);
    return HS_OK;
}

}  // extern "C"
