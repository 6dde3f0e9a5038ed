// Issue-rate probes for the integer VALU instructions the sweep kernel uses.
// Each thread runs 8 independent dependency chains of one instruction; the
// grid oversubscribes every SIMD, so the rate is the issue limit, not latency.
#include <hip/hip_runtime.h>

#include "../../include/hs_probe.h"

namespace {

constexpr int kChains = 8;
constexpr int kUnroll = 16;

#define CHAIN_LOOP(BODY)                                 \
    for (int it = 0; it < iters; ++it) {                 \
        _Pragma("unroll") for (int u = 0; u < kUnroll; ++u) { BODY }   \
    }

__global__ void __launch_bounds__(256) p_add(int iters, uint32_t *out)
{
    uint32_t x[kChains];
    for (int c = 0; c < kChains; ++c) x[c] = threadIdx.x * 7u + c;
    CHAIN_LOOP(for (int c = 0; c < kChains; ++c) asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[c]) : "v"(x[(c + 1) % kChains]));)
    uint32_t s = 0;
    for (int c = 0; c < kChains; ++c) s ^= x[c];
    if (s == 0x12345678u) out[0] = s;
}

__global__ void __launch_bounds__(256) p_bitop3(int iters, uint32_t *out)
{
    uint32_t x[kChains];
    for (int c = 0; c < kChains; ++c) x[c] = threadIdx.x * 7u + c;
    CHAIN_LOOP(for (int c = 0; c < kChains; ++c) asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(x[c]) : "v"(x[(c + 1) % kChains]), "v"(x[(c + 2) % kChains]));)
    uint32_t s = 0;
    for (int c = 0; c < kChains; ++c) s ^= x[c];
    if (s == 0x12345678u) out[0] = s;
}

__global__ void __launch_bounds__(256) p_mad64(int iters, uint32_t *out)
{
    uint32_t lo[kChains], hi[kChains];
    for (int c = 0; c < kChains; ++c) {
        lo[c] = threadIdx.x * 7u + c;
        hi[c] = c;
    }
    const uint32_t m = 0xD2511F53u;
    CHAIN_LOOP(for (int c = 0; c < kChains; ++c) {
        uint64_t r;
        asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, 0" : "=v"(r) : "v"(lo[c]), "v"(m) : "vcc");
        lo[c] = uint32_t(r);
    })
    uint32_t s = 0;
    for (int c = 0; c < kChains; ++c) s ^= lo[c] ^ hi[c];
    if (s == 0x12345678u) out[0] = s;
}

__global__ void __launch_bounds__(256) p_mulhi(int iters, uint32_t *out)
{
    uint32_t x[kChains];
    for (int c = 0; c < kChains; ++c) x[c] = threadIdx.x * 7u + c;
    const uint32_t m = 0xD2511F53u;
    CHAIN_LOOP(for (int c = 0; c < kChains; ++c) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(x[c]) : "v"(m));)
    uint32_t s = 0;
    for (int c = 0; c < kChains; ++c) s ^= x[c];
    if (s == 0x12345678u) out[0] = s;
}

__global__ void __launch_bounds__(256) p_mullo(int iters, uint32_t *out)
{
    uint32_t x[kChains];
    for (int c = 0; c < kChains; ++c) x[c] = threadIdx.x * 7u + c;
    const uint32_t m = 0xD2511F53u;
    CHAIN_LOOP(for (int c = 0; c < kChains; ++c) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x[c]) : "v"(m));)
    uint32_t s = 0;
    for (int c = 0; c < kChains; ++c) s ^= x[c];
    if (s == 0x12345678u) out[0] = s;
}

__global__ void __launch_bounds__(256) p_dot4(int iters, uint32_t *out)
{
    uint32_t x[kChains];
    for (int c = 0; c < kChains; ++c) x[c] = threadIdx.x * 7u + c;
    const uint32_t m = 0x01FF01FFu;
    CHAIN_LOOP(for (int c = 0; c < kChains; ++c) asm volatile("v_dot4_i32_i8 %0, %1, %2, %0" : "+v"(x[c]) : "v"(m), "v"(x[(c + 1) % kChains]));)
    uint32_t s = 0;
    for (int c = 0; c < kChains; ++c) s ^= x[c];
    if (s == 0x12345678u) out[0] = s;
}

__global__ void __launch_bounds__(256) p_mul24(int iters, uint32_t *out)
{
    uint32_t x[kChains];
    for (int c = 0; c < kChains; ++c) x[c] = threadIdx.x * 7u + c;
    CHAIN_LOOP(for (int c = 0; c < kChains; ++c) asm volatile("v_mad_i32_i24 %0, %0, %1, %2" : "+v"(x[c]) : "v"(x[(c + 1) % kChains]), "v"(x[(c + 3) % kChains]));)
    uint32_t s = 0;
    for (int c = 0; c < kChains; ++c) s ^= x[c];
    if (s == 0x12345678u) out[0] = s;
}

}  // namespace

extern "C" int hs_probe_rate(int which, int iters, double *ops_per_s, void *scratch)
{
    if (which < 0 || which > 6 || iters < 1 || !ops_per_s || !scratch) return -1;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -4;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -4;
    const int blocks = cus * 8, threads = 256;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -4;
    uint32_t *out = reinterpret_cast<uint32_t *>(scratch);
    auto launch = [&](int n) {
        switch (which) {
        case 0: hipLaunchKernelGGL(p_add, dim3(blocks), dim3(threads), 0, nullptr, n, out); break;
        case 1: hipLaunchKernelGGL(p_bitop3, dim3(blocks), dim3(threads), 0, nullptr, n, out); break;
        case 2: hipLaunchKernelGGL(p_mad64, dim3(blocks), dim3(threads), 0, nullptr, n, out); break;
        case 3: hipLaunchKernelGGL(p_mulhi, dim3(blocks), dim3(threads), 0, nullptr, n, out); break;
        case 4: hipLaunchKernelGGL(p_mullo, dim3(blocks), dim3(threads), 0, nullptr, n, out); break;
        case 5: hipLaunchKernelGGL(p_dot4, dim3(blocks), dim3(threads), 0, nullptr, n, out); break;
        default: hipLaunchKernelGGL(p_mul24, dim3(blocks), dim3(threads), 0, nullptr, n, out); break;
        }
    };
    launch(1);
    (void)hipEventRecord(a, nullptr);
    launch(iters);
    (void)hipEventRecord(b, nullptr);
    if (hipEventSynchronize(b) != hipSuccess) return -4;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    const double ops = double(blocks) * threads * iters * kUnroll * kChains;
    *ops_per_s = ops / (double(ms) * 1e-3);
    return 0;
}
