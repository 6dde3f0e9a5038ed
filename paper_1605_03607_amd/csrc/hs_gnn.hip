// gfx950 kernels and C ABI of the hardness surrogate (include/hs_gnn.h).
//
// Layout: node rows v = g N + site, directed edge rows e = g 2E + 2q + d.
// Node states H, edge states M and message sums S are bfloat16 rows of 64;
// pre-activations Z and all gradients are float32.  The matrix products are
// v_mfma_f32_16x16x32_bf16 tiles (16 rows x 16 columns x 32 deep, one
// wavefront): lane l holds A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e]
// [l % 16] (e = 0..7) and receives D[4 (l / 16) + i][l % 16] (i = 0..3).
//   * row products  Y = X W^T (+ b): X rows gathered from up to three row
//     tables (edge update [h_src; h_dst; m], node update [h; s], and the
//     input gradient dZ W), one wavefront per 16 rows, every output column
//   * weight gradients dW = dZ^T X: 32-row slices of dZ and X staged in LDS,
//     read as transposed fragments, summed over the rows of a workgroup, then
//     added to the gradient with float atomics
// The sums over the at most six edges of a node are gathers, not atomics.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hs_gnn.h"
#include "hs_internal.h"

namespace hs {
namespace gnn {

constexpr int D = 64;
constexpr int kLayers = 3;
constexpr int kNodeF = 5, kEdgeF = 4;
// parameter offsets (floats)
constexpr int kWen = 0, kBen = kWen + D * kNodeF, kWee = kBen + D, kBee = kWee + D * kEdgeF;
constexpr int kLayer0 = kBee + D;
constexpr int kWm = 0, kBm = kWm + D * 3 * D, kWh = kBm + D, kBh = kWh + D * 2 * D, kLayerSize = kBh + D;
constexpr int kWout = kLayer0 + kLayers * kLayerSize, kBout = kWout + D;
constexpr int kParams = kBout + 1;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite values)
    return uint16_t(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

__device__ __forceinline__ bf16x8 load8(const uint16_t *p)
{
    bf16x8 v;
    const uint4 w = *reinterpret_cast<const uint4 *>(p);
    __builtin_memcpy(&v, &w, 16);
    return v;
}

// ---------------------------------------------------------------------------
// Small element-wise kernels.
__global__ void k_fill(float *p, int64_t n, float v)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

// bfloat16 copies of W_m, W_h (row-major, out x in) and of their transposes.
struct WeightsBf {
    uint16_t *wm[kLayers], *wh[kLayers], *wmT[kLayers], *whT[kLayers];
};

__global__ void k_cast_weights(const float *P, WeightsBf w)
{
    const int l = blockIdx.y;
    const float *L_ = P + kLayer0 + l * kLayerSize;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < D * 3 * D; i += gridDim.x * blockDim.x) {
        const int o = i / (3 * D), c = i % (3 * D);
        const uint16_t b = f2bf(L_[kWm + i]);
        w.wm[l][i] = b;
        w.wmT[l][c * D + o] = b;
        if (i < D * 2 * D) {
            const int o2 = i / (2 * D), c2 = i % (2 * D);
            const uint16_t b2 = f2bf(L_[kWh + i]);
            w.wh[l][i] = b2;
            w.whT[l][c2 * D + o2] = b2;
        }
    }
}

__global__ void k_embed(const float *P, const float *xn, const float *xe, uint16_t *H0, uint16_t *M0, int nn,
                        int nq)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int d = int(i % D);
    const int64_t r = i / D;
    if (r < nn) {
        float h = P[kBen + d];
        for (int f = 0; f < kNodeF; ++f) h += P[kWen + d * kNodeF + f] * xn[r * 8 + f];
        H0[r * D + d] = f2bf(h);
    } else if (r < nn + int64_t(nq)) {
        const int64_t q = r - nn;
        float m = P[kBee + d];
        for (int f = 0; f < kEdgeF; ++f) m += P[kWee + d * kEdgeF + f] * xe[q * kEdgeF + f];
        const uint16_t b = f2bf(m);
        M0[(2 * q) * D + d] = b;
        M0[(2 * q + 1) * D + d] = b;
    }
}

// ---------------------------------------------------------------------------
// Row products: Y[r][n] = sum_k X[r][k] Wt[n][k] (+ bias[n]), X = the
// concatenation of NSEG gathered 64-wide rows, n < 16 NCB.  Z (float) and
// Yb = bf16(relu(Z)) are optional outputs.
struct Seg {
    const uint16_t *base[3];  // bf16 row tables, 64 per row
    const int32_t *idx[3];    // row index per output row, or null (identity)
};

template <int NSEG, int NCB>
__global__ void __launch_bounds__(256) k_rows(int rows, Seg X, const uint16_t *Wt, const float *bias, float *Z,
                                              uint16_t *Yb)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row0 = (blockIdx.x * 4 + wave) * 16;
    if (row0 >= rows) return;
    const int ar = row0 + (lane & 15), kq = lane >> 4;
    constexpr int K = 64 * NSEG;
    f32x4 acc[NCB];
#pragma unroll
    for (int c = 0; c < NCB; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < NSEG; ++s) {
        int64_t src = -1;
        if (ar < rows) src = X.idx[s] ? int64_t(X.idx[s][ar]) : int64_t(ar);
#pragma unroll
        for (int kk = 0; kk < 2; ++kk) {
            bf16x8 a;
            if (src >= 0)
                a = load8(X.base[s] + src * D + kk * 32 + kq * 8);
            else
                a = bf16x8{};
#pragma unroll
            for (int c = 0; c < NCB; ++c) {
                const bf16x8 b = load8(Wt + int64_t(c * 16 + (lane & 15)) * K + s * 64 + kk * 32 + kq * 8);
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
        const int n = c * 16 + (lane & 15);
        const float bn = bias ? bias[n] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = row0 + kq * 4 + i;
            if (r < rows) {
                const float z = acc[c][i] + bn;
                if (Z) Z[int64_t(r) * (16 * NCB) + n] = z;
                if (Yb) Yb[int64_t(r) * (16 * NCB) + n] = f2bf(fmaxf(z, 0.f));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient: gW[o][k] += sum_r dZ[r][o] X[r][k], o < 64, k < 64 NSEG,
// over the rows of this workgroup (kRowsPerBlock, 32 per step), added to gW
// with one atomic per element and workgroup.  Fewer rows per workgroup fill
// more CUs but add atomics to the same addresses; 256 was the fastest of
// 128..1024 for C8 batches.
constexpr int kRowsPerBlock = 256;

template <int NSEG>
__global__ void __launch_bounds__(256) k_wgrad(int rows, const uint16_t *dZ, Seg X, float *gW)
{
    __shared__ uint16_t zt[32 * D];
    __shared__ uint16_t xt[32 * 64 * NSEG];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kq = lane >> 4, cl = lane & 15;
    constexpr int K = 64 * NSEG;
    // wavefront w owns column blocks nb = w + 4 j (j < NSEG) and every row block
    f32x4 acc[4][NSEG];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int j = 0; j < NSEG; ++j) acc[mb][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int rbeg = blockIdx.x * kRowsPerBlock;
    const int rend = min(rows, rbeg + kRowsPerBlock);
    // 32-row slices of dZ (32 x 64) and of X (32 x 64 NSEG), 16 bytes per
    // thread and chunk; the next slice is loaded into registers while the
    // current one is multiplied out of LDS
    const int rr = tid >> 3, ch = tid & 7;  // row in slice, 16-byte chunk in a 64-wide row
    uint4 zn, xn[NSEG];
    auto fetch = [&](int r0) {
        const int r = r0 + rr;
        zn = uint4{0u, 0u, 0u, 0u};
        if (r < rend) zn = *reinterpret_cast<const uint4 *>(dZ + int64_t(r) * D + ch * 8);
#pragma unroll
        for (int s = 0; s < NSEG; ++s) {
            xn[s] = uint4{0u, 0u, 0u, 0u};
            if (r < rend) {
                const int64_t src = X.idx[s] ? int64_t(X.idx[s][r]) : int64_t(r);
                xn[s] = *reinterpret_cast<const uint4 *>(X.base[s] + src * D + ch * 8);
            }
        }
    };
    if (rbeg < rend) fetch(rbeg);
    for (int r0 = rbeg; r0 < rend; r0 += 32) {
        *reinterpret_cast<uint4 *>(zt + rr * D + ch * 8) = zn;
#pragma unroll
        for (int s = 0; s < NSEG; ++s) *reinterpret_cast<uint4 *>(xt + rr * K + s * 64 + ch * 8) = xn[s];
        __syncthreads();
        if (r0 + 32 < rend) fetch(r0 + 32);
        bf16x8 a[4];
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            uint16_t t[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) t[e] = zt[(kq * 8 + e) * D + mb * 16 + cl];
            __builtin_memcpy(&a[mb], t, 16);
        }
#pragma unroll
        for (int j = 0; j < NSEG; ++j) {
            const int nb = wave + 4 * j;
            uint16_t t[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) t[e] = xt[(kq * 8 + e) * K + nb * 16 + cl];
            bf16x8 b;
            __builtin_memcpy(&b, t, 16);
#pragma unroll
            for (int mb = 0; mb < 4; ++mb) acc[mb][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mb], b, acc[mb][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int j = 0; j < NSEG; ++j) {
            const int nb = wave + 4 * j;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int o = mb * 16 + kq * 4 + i, k = nb * 16 + cl;
                atomicAdd(&gW[o * K + k], acc[mb][j][i]);
            }
        }
}

// ---------------------------------------------------------------------------
// Message sums S_v = bf16(sum of M over the edges into v); the edges into v
// are the reverses (e ^ 1) of its out-edges.  One thread per node and 8
// features (16-byte loads and store); each feature is summed over the
// out-edge slots in order.
__global__ void k_gather_sum(const uint16_t *M, const int32_t *outE, uint16_t *S, int nn)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= int64_t(nn) * (D / 8)) return;
    const int64_t v = i / (D / 8);
    const int c = int(i % (D / 8));
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int j = 0; j < 6; ++j) {
        const int e = outE[v * 6 + j];
        if (e >= 0) {
            const uint4 w = *reinterpret_cast<const uint4 *>(M + int64_t(e ^ 1) * D + c * 8);
            const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s[2 * k] += bf2f(uint16_t(u[k] & 0xFFFFu));
                s[2 * k + 1] += bf2f(uint16_t(u[k] >> 16));
            }
        }
    }
    uint4 o;
    o.x = uint32_t(f2bf(s[0])) | (uint32_t(f2bf(s[1])) << 16);
    o.y = uint32_t(f2bf(s[2])) | (uint32_t(f2bf(s[3])) << 16);
    o.z = uint32_t(f2bf(s[4])) | (uint32_t(f2bf(s[5])) << 16);
    o.w = uint32_t(f2bf(s[6])) | (uint32_t(f2bf(s[7])) << 16);
    *reinterpret_cast<uint4 *>(S + v * D + c * 8) = o;
}

// Readout in two passes.  k_readout_part: workgroup (g, p) sums the live h
// rows of nodes [p n / S, (p + 1) n / S) of graph g (S = kReadSplit) into
// rpart[g][p][64].  k_readout_fin: 64 threads per graph add the S partial
// sums in order, take the mean over live nodes and form y_hat.
constexpr int kReadSplit = 8;
__global__ void __launch_bounds__(256) k_readout_part(const uint16_t *H, const float *live, int n, float *rpart)
{
    __shared__ float part[4][D];
    const int g = blockIdx.x, p = blockIdx.y, t = threadIdx.x, d = t & 63, q = t >> 6;
    const int lo = int(int64_t(p) * n / kReadSplit), hi = int(int64_t(p + 1) * n / kReadSplit);
    float s = 0.f;
    for (int v = lo + q; v < hi; v += 4) {
        const int64_t row = int64_t(g) * n + v;
        s += live[row] * bf2f(H[row * D + d]);
    }
    part[q][d] = s;
    __syncthreads();
    if (t < D) rpart[(int64_t(g) * kReadSplit + p) * D + d] = part[0][d] + part[1][d] + part[2][d] + part[3][d];
}

__global__ void __launch_bounds__(64) k_readout_fin(const float *rpart, const float *nlive, const float *P,
                                                    float *mean, float *y)
{
    __shared__ float red[D];
    const int g = blockIdx.x, d = threadIdx.x;
    float s = 0.f;
    for (int p = 0; p < kReadSplit; ++p) s += rpart[(int64_t(g) * kReadSplit + p) * D + d];
    const float m = s / nlive[g];
    mean[g * D + d] = m;
    red[d] = m * P[kWout + d];
    __syncthreads();
    if (d == 0) {
        float acc = P[kBout];
        for (int k = 0; k < D; ++k) acc += red[k];
        y[g] = acc;
    }
}

// Loss, d loss / d y_hat and the readout-parameter gradient (one workgroup of 64).
__global__ void k_loss(const float *y, const float *labels, const float *mean, int G, float *dy, float *loss,
                       float *grad)
{
    const int t = threadIdx.x;
    __shared__ int nvalid;
    if (t == 0) {
        int c = 0;
        for (int g = 0; g < G; ++g) c += isfinite(labels[g]) ? 1 : 0;
        nvalid = c > 0 ? c : 1;
    }
    __syncthreads();
    const float inv = 1.f / float(nvalid);
    for (int g = t; g < G; g += blockDim.x) dy[g] = isfinite(labels[g]) ? 2.f * (y[g] - labels[g]) * inv : 0.f;
    __syncthreads();
    float gw = 0.f;
    for (int g = 0; g < G; ++g) gw += dy[g] * mean[g * D + t];
    grad[kWout + t] = gw;
    if (t == 0) {
        float l = 0.f, gb = 0.f;
        for (int g = 0; g < G; ++g) {
            if (isfinite(labels[g])) {
                const float df = y[g] - labels[g];
                l += df * df;
            }
            gb += dy[g];
        }
        *loss = l * inv;
        grad[kBout] = gb;
    }
}

// The ranked loss (a child graph against its parent ref[g], plus w_abs times
// the plain loss), d loss / d y_hat and the readout-parameter gradient (one
// workgroup of 64).  A pair term needs 0 <= ref[g] < G, ref[g] != g and both
// labels finite; each thread sums its own graphs' terms in graph order, so
// the result does not depend on thread timing.
__global__ void k_loss_ranked(const float *y, const float *labels, const int32_t *ref, float w_abs,
                              const float *mean, int G, float *dy, float *loss, float *grad)
{
    const int t = threadIdx.x;
    __shared__ int nvalid, npair;
    auto paired = [&](int g) {
        const int p = ref[g];
        return p >= 0 && p < G && p != g && isfinite(labels[g]) && isfinite(labels[p]);
    };
    if (t == 0) {
        int c = 0, q = 0;
        for (int g = 0; g < G; ++g) {
            c += isfinite(labels[g]) ? 1 : 0;
            q += paired(g) ? 1 : 0;
        }
        nvalid = c > 0 ? c : 1;
        npair = q > 0 ? q : 1;
    }
    __syncthreads();
    const float inv = 1.f / float(nvalid), invp = 1.f / float(npair);
    auto pair_d = [&](int g) { return (y[g] - y[ref[g]]) - (labels[g] - labels[ref[g]]); };
    for (int g = t; g < G; g += blockDim.x) {
        float v = isfinite(labels[g]) ? w_abs * 2.f * (y[g] - labels[g]) * inv : 0.f;
        if (paired(g)) v += 2.f * pair_d(g) * invp;
        for (int h = 0; h < G; ++h)
            if (ref[h] == g && paired(h)) v -= 2.f * pair_d(h) * invp;
        dy[g] = v;
    }
    __syncthreads();
    float gw = 0.f;
    for (int g = 0; g < G; ++g) gw += dy[g] * mean[g * D + t];
    grad[kWout + t] = gw;
    if (t == 0) {
        float l = 0.f, lp = 0.f, gb = 0.f;
        for (int g = 0; g < G; ++g) {
            if (isfinite(labels[g])) {
                const float df = y[g] - labels[g];
                l += df * df;
            }
            if (paired(g)) {
                const float d = pair_d(g);
                lp += d * d;
            }
            gb += dy[g];
        }
        *loss = w_abs * l * inv + lp * invp;
        grad[kBout] = gb;
    }
}

__global__ void k_readout_bwd(const float *dy, const float *P, const float *live, const float *nlive, float *dH,
                              int nn, int n)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= int64_t(nn) * D) return;
    const int64_t v = i / D;
    const int g = int(v / n);
    dH[i] = live[v] * dy[g] * P[kWout + int(i % D)] / nlive[g];
}

// dZ = dY * (Z > 0) as bfloat16, and the bias gradient (float).  For edges
// dY = dM (from the layer above, column 128.. of its input gradient; none
// for the top layer) + dS of the edge's destination (column 64.. of the node
// input gradient).  Each workgroup stores its 64 partial bias sums in
// bpart[blockIdx.x][64]; k_bias_sum adds them up (no atomics on the 64 shared
// addresses, and the same sum on every run).
constexpr unsigned kReluBlocks = 2048;
__global__ void __launch_bounds__(256) k_relu_bwd(int rows, const float *dY, int ldY, int offY, const float *dS,
                                                  const int32_t *dst, const float *Z, uint16_t *dZb, float *bpart)
{
    __shared__ float part[4][D];
    const int t = threadIdx.x, d = t & 63, q = t >> 6;
    float s = 0.f;
    for (int r = blockIdx.x * 4 + q; r < rows; r += gridDim.x * 4) {
        float y = dY ? dY[int64_t(r) * ldY + offY + d] : 0.f;
        if (dS) y += dS[int64_t(dst[r]) * 128 + 64 + d];
        const float z = Z[int64_t(r) * D + d] > 0.f ? y : 0.f;
        dZb[int64_t(r) * D + d] = f2bf(z);
        s += z;
    }
    part[q][d] = s;
    __syncthreads();
    if (t < D) bpart[int64_t(blockIdx.x) * D + d] = part[0][d] + part[1][d] + part[2][d] + part[3][d];
}

// gb[d] += sum over the nb rows of bpart[.][d]: one workgroup per column, a
// fixed reduction tree.
__global__ void __launch_bounds__(256) k_bias_sum(const float *bpart, int nb, float *gb)
{
    __shared__ float red[256];
    const int d = blockIdx.x, t = threadIdx.x;
    float s = 0.f;
    for (int b = t; b < nb; b += 256) s += bpart[int64_t(b) * D + d];
    red[t] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t == 0) gb[d] += red[0];
}

// dH_v = dXn[v][0..63] + sum over out-edges e of dXe[e][0..63] + sum over
// in-edges (e ^ 1) of dXe[e ^ 1][64..127].
__global__ void k_node_collect(const float *dXn, const float *dXe, const int32_t *outE, float *dH, int nn)
{
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= int64_t(nn) * D) return;
    const int64_t v = i / D;
    const int d = int(i % D);
    float s = dXn[v * 128 + d];
    for (int j = 0; j < 6; ++j) {
        const int e = outE[v * 6 + j];
        if (e >= 0) s += dXe[int64_t(e) * 192 + d] + dXe[int64_t(e ^ 1) * 192 + 64 + d];
    }
    dH[i] = s;
}

// Embedding gradients: node (W_en, b_en) from dH0, edge (W_ee, b_ee) from
// dM0 = column 128.. of the first layer's edge input gradient, summed over
// the two directions of each coupler.
// Workgroup (x, y) of a kEmbBlocks x 2 grid (y = 0 nodes, 1 couplers) stores
// its partial sums in epart[y][x][64][6]; k_embed_sum adds them up.
constexpr int kEmbBlocks = 512;
__global__ void __launch_bounds__(256) k_embed_bwd(const float *dH0, const float *dXe0, const float *xn,
                                                   const float *xe, int nn, int nq, float *epart)
{
    __shared__ float part[4][D][6];
    const int t = threadIdx.x, d = t & 63, q = t >> 6;
    float a[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (blockIdx.y == 0) {
        for (int v = blockIdx.x * 4 + q; v < nn; v += gridDim.x * 4) {
            const float g = dH0[int64_t(v) * D + d];
            for (int f = 0; f < kNodeF; ++f) a[f] += g * xn[int64_t(v) * 8 + f];
            a[5] += g;
        }
    } else {
        for (int c = blockIdx.x * 4 + q; c < nq; c += gridDim.x * 4) {
            const float g = dXe0[int64_t(2 * c) * 192 + 128 + d] + dXe0[int64_t(2 * c + 1) * 192 + 128 + d];
            for (int f = 0; f < kEdgeF; ++f) a[f] += g * xe[int64_t(c) * kEdgeF + f];
            a[5] += g;
        }
    }
    for (int f = 0; f < 6; ++f) part[q][d][f] = a[f];
    __syncthreads();
    if (t < D) {
        float *o = epart + ((int64_t(blockIdx.y) * gridDim.x + blockIdx.x) * D + d) * 6;
        for (int f = 0; f < 6; ++f) o[f] = part[0][d][f] + part[1][d][f] + part[2][d][f] + part[3][d][f];
    }
}

// Embedding gradients from the partial sums: workgroup (d, y) adds the nb
// workgroups' 6 sums of feature d with a fixed tree.
__global__ void __launch_bounds__(256) k_embed_sum(const float *epart, int nb, float *grad)
{
    __shared__ float red[6][256];
    const int d = blockIdx.x, y = blockIdx.y, t = threadIdx.x;
    float s[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int b = t; b < nb; b += 256) {
        const float *p = epart + ((int64_t(y) * nb + b) * D + d) * 6;
        for (int f = 0; f < 6; ++f) s[f] += p[f];
    }
    for (int f = 0; f < 6; ++f) red[f][t] = s[f];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int f = 0; f < 6; ++f) red[f][t] += red[f][t + w];
        __syncthreads();
    }
    if (t == 0) {
        if (y == 0) {
            for (int f = 0; f < kNodeF; ++f) grad[kWen + d * kNodeF + f] += red[f][0];
            grad[kBen + d] += red[5][0];
        } else {
            for (int f = 0; f < kEdgeF; ++f) grad[kWee + d * kEdgeF + f] += red[f][0];
            grad[kBee + d] += red[5][0];
        }
    }
}

__global__ void k_adam(float *P, const float *g, float *m, float *v, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float mi = b1 * m[i] + (1.f - b1) * g[i];
    const float vi = b2 * v[i] + (1.f - b2) * g[i] * g[i];
    m[i] = mi;
    v[i] = vi;
    P[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace gnn
}  // namespace hs

// ===========================================================================
// Host side.
using namespace hs;
using namespace hs::gnn;

namespace {

struct Layout {
    int G = 0, L = 0, N = 0, E = 0;
    int64_t nn = 0, nq = 0, ne = 0;
    size_t xn, xe, live, nlive, src, dst, outE, wb, H, M, S, Zm, Zh, mean, y, dy, dZ, dXe, dXn, dH, bpart, rpart,
        epart, total;
};

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

bool make_layout(int G, int L, Layout &o)
{
    if (G < 1 || L < 1 || L > HS_MAX_L) return false;
    o.G = G;
    o.L = L;
    o.N = 8 * L * L;
    o.E = 24 * L * L - 8 * L;
    o.nn = int64_t(G) * o.N;
    o.nq = int64_t(G) * o.E;
    o.ne = 2 * o.nq;
    size_t p = 0;
    auto take = [&](size_t bytes) {
        const size_t at = p;
        p = al(p + bytes);
        return at;
    };
    o.xn = take(size_t(o.nn) * 8 * 4);
    o.xe = take(size_t(o.nq) * kEdgeF * 4);
    o.live = take(size_t(o.nn) * 4);
    o.nlive = take(size_t(G) * 4);
    o.src = take(size_t(o.ne) * 4);
    o.dst = take(size_t(o.ne) * 4);
    o.outE = take(size_t(o.nn) * 6 * 4);
    o.wb = take(size_t(kLayers) * (2 * D * 3 * D + 2 * D * 2 * D) * 2);
    o.H = take(size_t(kLayers + 1) * o.nn * D * 2);
    o.M = take(size_t(kLayers + 1) * o.ne * D * 2);
    o.S = take(size_t(kLayers) * o.nn * D * 2);
    o.Zm = take(size_t(kLayers) * o.ne * D * 4);
    o.Zh = take(size_t(kLayers) * o.nn * D * 4);
    o.mean = take(size_t(G) * D * 4);
    o.y = take(size_t(G) * 4);
    o.dy = take(size_t(G) * 4);
    o.dZ = take(size_t(o.ne) * D * 2);
    o.dXe = take(size_t(2) * o.ne * 192 * 4);
    o.dXn = take(size_t(o.nn) * 128 * 4);
    o.dH = take(size_t(o.nn) * D * 4);
    o.bpart = take(size_t(kReluBlocks) * D * 4);
    o.rpart = take(size_t(G) * kReadSplit * D * 4);
    o.epart = take(size_t(2) * kEmbBlocks * D * 6 * 4);
    o.total = p;
    return true;
}

int hip_err(hipError_t e, const std::string &what) { return fail(HS_EHIP, what + ": " + hipGetErrorString(e)); }

struct Bufs {
    float *xn, *xe, *live, *nlive, *mean, *y, *dy, *dXe[2], *dXn, *dH, *bpart, *rpart, *epart, *Zm[kLayers], *Zh[kLayers];
    int32_t *src, *dst, *outE;
    uint16_t *H[kLayers + 1], *M[kLayers + 1], *S[kLayers], *dZ;
    WeightsBf wb;
};

Bufs views(const Layout &o, void *ws)
{
    char *b = reinterpret_cast<char *>(ws);
    Bufs v;
    v.xn = reinterpret_cast<float *>(b + o.xn);
    v.xe = reinterpret_cast<float *>(b + o.xe);
    v.live = reinterpret_cast<float *>(b + o.live);
    v.nlive = reinterpret_cast<float *>(b + o.nlive);
    v.src = reinterpret_cast<int32_t *>(b + o.src);
    v.dst = reinterpret_cast<int32_t *>(b + o.dst);
    v.outE = reinterpret_cast<int32_t *>(b + o.outE);
    uint16_t *w = reinterpret_cast<uint16_t *>(b + o.wb);
    for (int l = 0; l < kLayers; ++l) {
        v.wb.wm[l] = w;
        w += D * 3 * D;
        v.wb.wmT[l] = w;
        w += D * 3 * D;
        v.wb.wh[l] = w;
        w += D * 2 * D;
        v.wb.whT[l] = w;
        w += D * 2 * D;
    }
    for (int l = 0; l <= kLayers; ++l) {
        v.H[l] = reinterpret_cast<uint16_t *>(b + o.H) + size_t(l) * o.nn * D;
        v.M[l] = reinterpret_cast<uint16_t *>(b + o.M) + size_t(l) * o.ne * D;
    }
    for (int l = 0; l < kLayers; ++l) {
        v.S[l] = reinterpret_cast<uint16_t *>(b + o.S) + size_t(l) * o.nn * D;
        v.Zm[l] = reinterpret_cast<float *>(b + o.Zm) + size_t(l) * o.ne * D;
        v.Zh[l] = reinterpret_cast<float *>(b + o.Zh) + size_t(l) * o.nn * D;
    }
    v.mean = reinterpret_cast<float *>(b + o.mean);
    v.y = reinterpret_cast<float *>(b + o.y);
    v.dy = reinterpret_cast<float *>(b + o.dy);
    v.dZ = reinterpret_cast<uint16_t *>(b + o.dZ);
    v.dXe[0] = reinterpret_cast<float *>(b + o.dXe);
    v.dXe[1] = v.dXe[0] + size_t(o.ne) * 192;
    v.dXn = reinterpret_cast<float *>(b + o.dXn);
    v.dH = reinterpret_cast<float *>(b + o.dH);
    v.bpart = reinterpret_cast<float *>(b + o.bpart);
    v.rpart = reinterpret_cast<float *>(b + o.rpart);
    v.epart = reinterpret_cast<float *>(b + o.epart);
    return v;
}

unsigned blocks_for(int64_t n, int per) { return unsigned((n + per - 1) / per); }

// Forward pass into the workspace (y_hat in v.y).  keep_z: also store the
// float pre-activations the backward pass needs (a forward-only call skips
// those writes).
int forward_pass(const float *P, const Layout &o, const Bufs &v, hipStream_t st, bool keep_z)
{
    hipLaunchKernelGGL(k_cast_weights, dim3(48, kLayers), dim3(256), 0, st, P, v.wb);
    hipLaunchKernelGGL(k_embed, dim3(blocks_for((o.nn + o.nq) * D, 256)), dim3(256), 0, st, P, v.xn, v.xe,
                       v.H[0], v.M[0], int(o.nn), int(o.nq));
    const int ne = int(o.ne), nn = int(o.nn);
    for (int l = 0; l < kLayers; ++l) {
        const float *Ls = P + kLayer0 + l * kLayerSize;
        Seg xe{{v.H[l], v.H[l], v.M[l]}, {v.src, v.dst, nullptr}};
        hipLaunchKernelGGL((k_rows<3, 4>), dim3(blocks_for(ne, 64)), dim3(256), 0, st, ne, xe, v.wb.wm[l],
                           Ls + kBm, keep_z ? v.Zm[l] : nullptr, v.M[l + 1]);
        hipLaunchKernelGGL(k_gather_sum, dim3(blocks_for(o.nn * (D / 8), 256)), dim3(256), 0, st, v.M[l + 1],
                           v.outE, v.S[l], nn);
        Seg xn{{v.H[l], v.S[l], nullptr}, {nullptr, nullptr, nullptr}};
        hipLaunchKernelGGL((k_rows<2, 4>), dim3(blocks_for(nn, 64)), dim3(256), 0, st, nn, xn, v.wb.wh[l],
                           Ls + kBh, keep_z ? v.Zh[l] : nullptr, v.H[l + 1]);
    }
    hipLaunchKernelGGL(k_readout_part, dim3(o.G, kReadSplit), dim3(256), 0, st, v.H[kLayers], v.live, o.N,
                       v.rpart);
    hipLaunchKernelGGL(k_readout_fin, dim3(o.G), dim3(64), 0, st, v.rpart, v.nlive, P, v.mean, v.y);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? HS_OK : hip_err(e, "gnn forward: launch");
}

int check_ws(int G, int L, size_t bytes, Layout &o, const char *who)
{
    if (!make_layout(G, L, o)) return fail(HS_EINVAL, std::string(who) + ": bad n_graphs or L");
    if (bytes < o.total) return fail(HS_ENOSPACE, std::string(who) + ": workspace too small");
    return HS_OK;
}

}  // namespace

extern "C" {

int gnn_param_count(void) { return kParams; }

int gnn_workspace_bytes(int32_t n_graphs, int32_t L, size_t *bytes)
{
    Layout o;
    if (bytes == nullptr || !make_layout(n_graphs, L, o)) return fail(HS_EINVAL, "gnn_workspace_bytes: bad arguments");
    *bytes = o.total;
    return HS_OK;
}

int gnn_prepare(const hs_gnn_batch *b, void *workspace, size_t workspace_bytes, void *stream)
{
    if (b == nullptr || b->J == nullptr || workspace == nullptr) return fail(HS_EINVAL, "gnn_prepare: NULL argument");
    Layout o;
    int rc = check_ws(b->n_graphs, b->L, workspace_bytes, o, "gnn_prepare");
    if (rc) return rc;
    const int L = o.L, N = o.N, E = o.E, G = o.G;
    std::vector<int32_t> ei, ej;
    chimera_edges(L, ei, ej);
    if (int(ei.size()) != E) return fail(HS_EINVAL, "gnn_prepare: coupler count");
    std::vector<float> xn(size_t(o.nn) * 8, 0.f), xe(size_t(o.nq) * kEdgeF), live(o.nn), nlive(G);
    std::vector<int32_t> src(o.ne), dst(o.ne), outE(size_t(o.nn) * 6, -1);
    std::vector<int> deg(o.nn, 0);
    for (int g = 0; g < G; ++g) {
        const uint8_t *lv = b->live ? b->live + size_t(g) * N : nullptr;
        int cnt = 0;
        for (int i = 0; i < N; ++i) {
            const int cell = i / 8, u = (i / 4) % 2, k = i % 4, r = cell / L, c = cell % L;
            const size_t row = size_t(g) * N + i;
            const float alive = (lv == nullptr || lv[i]) ? 1.f : 0.f;
            xn[row * 8 + 0] = float(r) / float(L);
            xn[row * 8 + 1] = float(c) / float(L);
            xn[row * 8 + 2] = float(u);
            xn[row * 8 + 3] = float(k) / 3.f;
            xn[row * 8 + 4] = alive;
            live[row] = alive;
            cnt += alive > 0.f ? 1 : 0;
        }
        if (cnt == 0) return fail(HS_EINVAL, "gnn_prepare: a graph without live sites");
        nlive[g] = float(cnt);
        for (int q = 0; q < E; ++q) {
            const int i = ei[q], j = ej[q];
            const bool on = lv == nullptr || (lv[i] && lv[j]);
            const int J = int(b->J[size_t(g) * E + q]);
            const size_t row = size_t(g) * E + q;
            const int ci = i / 8, cj = j / 8;
            xe[row * 4 + 0] = on ? float(J) / 7.f : 0.f;
            xe[row * 4 + 1] = ci == cj ? 1.f : 0.f;
            xe[row * 4 + 2] = (ci != cj && ((i / 4) % 2) == 0) ? 1.f : 0.f;
            xe[row * 4 + 3] = (ci != cj && ((i / 4) % 2) == 1) ? 1.f : 0.f;
            const int64_t vi = int64_t(g) * N + i, vj = int64_t(g) * N + j;
            const int64_t e0 = 2 * int64_t(row);
            src[e0] = int32_t(vi);
            dst[e0] = int32_t(vj);
            src[e0 + 1] = int32_t(vj);
            dst[e0 + 1] = int32_t(vi);
            if (deg[vi] >= 6 || deg[vj] >= 6) return fail(HS_EINVAL, "gnn_prepare: degree above 6");
            outE[vi * 6 + deg[vi]++] = int32_t(e0);
            outE[vj * 6 + deg[vj]++] = int32_t(e0 + 1);
        }
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char *w = reinterpret_cast<char *>(workspace);
    auto up = [&](size_t off, const void *src_, size_t bytes) {
        return hipMemcpyAsync(w + off, src_, bytes, hipMemcpyHostToDevice, st);
    };
    hipError_t e = up(o.xn, xn.data(), xn.size() * 4);
    if (e == hipSuccess) e = up(o.xe, xe.data(), xe.size() * 4);
    if (e == hipSuccess) e = up(o.live, live.data(), live.size() * 4);
    if (e == hipSuccess) e = up(o.nlive, nlive.data(), nlive.size() * 4);
    if (e == hipSuccess) e = up(o.src, src.data(), src.size() * 4);
    if (e == hipSuccess) e = up(o.dst, dst.data(), dst.size() * 4);
    if (e == hipSuccess) e = up(o.outE, outE.data(), outE.size() * 4);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // the host vectors end with this call
    return e == hipSuccess ? HS_OK : hip_err(e, "gnn_prepare: upload");
}

int gnn_forward(const float *params, int32_t n_graphs, int32_t L, void *workspace, size_t workspace_bytes,
                float *y_hat, void *stream)
{
    if (params == nullptr || workspace == nullptr || y_hat == nullptr) return fail(HS_EINVAL, "gnn_forward: NULL argument");
    Layout o;
    int rc = check_ws(n_graphs, L, workspace_bytes, o, "gnn_forward");
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const Bufs v = views(o, workspace);
    rc = forward_pass(params, o, v, st, false);
    if (rc) return rc;
    const hipError_t e = hipMemcpyAsync(y_hat, v.y, size_t(o.G) * 4, hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? HS_OK : hip_err(e, "gnn_forward: copy");
}

}  // extern "C"

namespace {

// Forward pass, loss (plain, or ranked when ref is not NULL), backward pass
// and the optional Adam update of one training step.
int train_step(const char *who, float *params, int32_t n_graphs, int32_t L, const float *labels,
               const int32_t *ref, float w_abs, void *workspace, size_t workspace_bytes, float *y_hat, float *loss,
               float *grad, const hs_adam *adam, void *stream)
{
    if (params == nullptr || labels == nullptr || workspace == nullptr || loss == nullptr || grad == nullptr)
        return fail(HS_EINVAL, std::string(who) + ": NULL argument");
    if (adam && (adam->m == nullptr || adam->v == nullptr || adam->step < 1))
        return fail(HS_EINVAL, std::string(who) + ": bad Adam state");
    Layout o;
    int rc = check_ws(n_graphs, L, workspace_bytes, o, who);
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const Bufs v = views(o, workspace);
    rc = forward_pass(params, o, v, st, true);
    if (rc) return rc;
    const int ne = int(o.ne), nn = int(o.nn);
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(kParams, 256)), dim3(256), 0, st, grad, int64_t(kParams), 0.f);
    if (ref)
        hipLaunchKernelGGL(k_loss_ranked, dim3(1), dim3(64), 0, st, v.y, labels, ref, w_abs, v.mean, o.G, v.dy,
                           loss, grad);
    else
        hipLaunchKernelGGL(k_loss, dim3(1), dim3(64), 0, st, v.y, labels, v.mean, o.G, v.dy, loss, grad);
    hipLaunchKernelGGL(k_readout_bwd, dim3(blocks_for(o.nn * D, 256)), dim3(256), 0, st, v.dy, params, v.live,
                       v.nlive, v.dH, nn, o.N);
    const float *dXe_above = nullptr;
    int cur = 0;
    for (int l = kLayers - 1; l >= 0; --l) {
        float *gl = grad + kLayer0 + l * kLayerSize;
        // node update
        const unsigned gn = std::min<unsigned>(blocks_for(nn, 4), kReluBlocks);
        hipLaunchKernelGGL(k_relu_bwd, dim3(gn), dim3(256), 0, st, nn, v.dH, D, 0, nullptr, nullptr, v.Zh[l], v.dZ,
                           v.bpart);
        hipLaunchKernelGGL(k_bias_sum, dim3(D), dim3(256), 0, st, v.bpart, int(gn), gl + kBh);
        Seg xn{{v.H[l], v.S[l], nullptr}, {nullptr, nullptr, nullptr}};
        hipLaunchKernelGGL(k_wgrad<2>, dim3(blocks_for(nn, kRowsPerBlock)), dim3(256), 0, st, nn, v.dZ, xn,
                           gl + kWh);
        Seg dzn{{v.dZ, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
        hipLaunchKernelGGL((k_rows<1, 8>), dim3(blocks_for(nn, 64)), dim3(256), 0, st, nn, dzn, v.wb.whT[l],
                           nullptr, v.dXn, nullptr);
        // edge update
        const unsigned ge = std::min<unsigned>(blocks_for(ne, 4), kReluBlocks);
        hipLaunchKernelGGL(k_relu_bwd, dim3(ge), dim3(256), 0, st, ne, dXe_above, 192, 128, v.dXn, v.dst, v.Zm[l],
                           v.dZ, v.bpart);
        hipLaunchKernelGGL(k_bias_sum, dim3(D), dim3(256), 0, st, v.bpart, int(ge), gl + kBm);
        Seg xe{{v.H[l], v.H[l], v.M[l]}, {v.src, v.dst, nullptr}};
        hipLaunchKernelGGL(k_wgrad<3>, dim3(blocks_for(ne, kRowsPerBlock)), dim3(256), 0, st, ne, v.dZ, xe,
                           gl + kWm);
        Seg dze{{v.dZ, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
        hipLaunchKernelGGL((k_rows<1, 12>), dim3(blocks_for(ne, 64)), dim3(256), 0, st, ne, dze, v.wb.wmT[l],
                           nullptr, v.dXe[cur], nullptr);
        hipLaunchKernelGGL(k_node_collect, dim3(blocks_for(o.nn * D, 256)), dim3(256), 0, st, v.dXn, v.dXe[cur],
                           v.outE, v.dH, nn);
        dXe_above = v.dXe[cur];
        cur ^= 1;
    }
    hipLaunchKernelGGL(k_embed_bwd, dim3(kEmbBlocks, 2), dim3(256), 0, st, v.dH, dXe_above, v.xn, v.xe, nn,
                       int(o.nq), v.epart);
    hipLaunchKernelGGL(k_embed_sum, dim3(D, 2), dim3(256), 0, st, v.epart, kEmbBlocks, grad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_err(e, std::string(who) + ": launch");
    if (y_hat) {
        e = hipMemcpyAsync(y_hat, v.y, size_t(o.G) * 4, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_err(e, std::string(who) + ": copy");
    }
    if (adam) {
        const double t = double(adam->step);
        const float c1 = float(1.0 - std::pow(double(adam->beta1), t));
        const float c2 = float(1.0 - std::pow(double(adam->beta2), t));
        hipLaunchKernelGGL(k_adam, dim3(blocks_for(kParams, 256)), dim3(256), 0, st, params, grad, adam->m,
                           adam->v, kParams, adam->lr, adam->beta1, adam->beta2, adam->eps, c1, c2);
        e = hipGetLastError();
        if (e != hipSuccess) return hip_err(e, std::string(who) + ": Adam");
    }
    return HS_OK;
}

}  // namespace

extern "C" {

int gnn_train_step(float *params, int32_t n_graphs, int32_t L, const float *labels, void *workspace,
                   size_t workspace_bytes, float *y_hat, float *loss, float *grad, const hs_adam *adam,
                   void *stream)
{
    return train_step("gnn_train_step", params, n_graphs, L, labels, nullptr, 1.f, workspace, workspace_bytes,
                      y_hat, loss, grad, adam, stream);
}

int gnn_train_step_ranked(float *params, int32_t n_graphs, int32_t L, const float *labels, const int32_t *ref,
                          float w_abs, void *workspace, size_t workspace_bytes, float *y_hat, float *loss,
                          float *grad, const hs_adam *adam, void *stream)
{
    if (ref == nullptr) return fail(HS_EINVAL, "gnn_train_step_ranked: NULL ref");
    if (!(w_abs >= 0.f) || !std::isfinite(w_abs)) return fail(HS_EINVAL, "gnn_train_step_ranked: w_abs");
    return train_step("gnn_train_step_ranked", params, n_graphs, L, labels, ref, w_abs, workspace,
                      workspace_bytes, y_hat, loss, grad, adam, stream);
}

}  // extern "C"
