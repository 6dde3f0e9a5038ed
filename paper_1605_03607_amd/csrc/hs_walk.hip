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

constexpr int kLagTile = 64;    // lags per workgroup (16 per thread, 4 lag phases)
constexpr int kTimeTile = 256;  // passes per LDS tile

// Workgroup (n, lag tile): 256 threads = 64 configurations x 4 lag phases;
// thread (j, c) sums lags d0 + j + 4 i, i < 16.  Each tile stages the centred
// indices g of passes [t0, t0 + kTimeTile) and [t0 + d0, t0 + d0 + kTimeTile
// + kLagTile) as int8 (|g| <= 63; zero beyond the run and for dead
// configurations), so every product reads LDS only.
__global__ void __launch_bounds__(256) k_walk_acf(const uint8_t *walk, int64_t cap, int64_t T, int K, int C,
                                                  int max_lag, int64_t *acf)
{
    __shared__ int8_t base[kTimeTile * 64];
    __shared__ int8_t shifted[(kTimeTile + kLagTile) * 64];
    const int n = blockIdx.x;
    const int d0 = blockIdx.y * kLagTile;
    const int c = threadIdx.x & 63, j = threadIdx.x >> 6;
    const uint8_t *src = walk + int64_t(n) * cap * 64;
    auto gval = [&](int64_t t, int cc) -> int8_t {
        if (t >= T || cc >= C) return 0;
        return int8_t(2 * int(src[t * 64 + cc]) - (K - 1));
    };
    int64_t acc[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0;
    for (int64_t t0 = 0; t0 < T - d0; t0 += kTimeTile) {
        __syncthreads();
        for (int i = threadIdx.x; i < kTimeTile * 64; i += 256) base[i] = gval(t0 + (i >> 6), i & 63);
        for (int i = threadIdx.x; i < (kTimeTile + kLagTile) * 64; i += 256)
            shifted[i] = gval(t0 + d0 + (i >> 6), i & 63);
        __syncthreads();
        int32_t part[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) part[i] = 0;
        for (int t = 0; t < kTimeTile; ++t) {
            const int32_t gb = base[t * 64 + c];
#pragma unroll
            for (int i = 0; i < 16; ++i) part[i] += gb * int32_t(shifted[(t + j + 4 * i) * 64 + c]);
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
        const int d = d0 + j + 4 * i;
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
