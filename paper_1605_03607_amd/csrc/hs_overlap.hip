// Overlaps between captured ground and first-excited configurations (Sec.
// III.B, Fig. 3): all-pairs Hamming distances on the device, then the
// distinct states (up to the global flip) and the median overlaps on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/hardspin.h"
#include "hs_internal.h"

namespace hs {
namespace dev {

// out[i n + j] = popcount((c_i ^ c_j) & mask) over n_words words; one thread per j.
__global__ void __launch_bounds__(256) k_hamming(const uint64_t *configs, int n, int n_words, const uint64_t *mask,
                                                 int32_t *out)
{
    const int i = blockIdx.x;
    const int j = blockIdx.y * 256 + threadIdx.x;
    if (j >= n) return;
    const uint64_t *a = configs + int64_t(i) * n_words, *b = configs + int64_t(j) * n_words;
    int h = 0;
    for (int w = 0; w < n_words; ++w) h += __popcll((a[w] ^ b[w]) & mask[w]);
    out[int64_t(i) * n + j] = h;
}

}  // namespace dev

namespace {

// Median of the overlaps q(h) = |1 - 2h/n_live| of a multiset of Hamming
// distances given as counts per distance h = 0..n_live: the distances are
// visited in ascending order of q, the value itself, so the element(s) found
// at the middle rank are those a sort of all the pair overlaps would give.
double median_q(const std::vector<int64_t> &count, int n_live)
{
    std::vector<double> qv(size_t(n_live) + 1);
    std::vector<int> order(size_t(n_live) + 1);
    int64_t total = 0;
    for (int h = 0; h <= n_live; ++h) {
        qv[h] = std::fabs(1.0 - 2.0 * double(h) / n_live);
        order[h] = h;
        total += count[h];
    }
    std::sort(order.begin(), order.end(), [&](int a, int b) { return qv[a] < qv[b]; });
    auto at = [&](int64_t rank) {  // the element of 0-based rank in ascending order
        int64_t cum = 0;
        for (int h : order) {
            cum += count[h];
            if (cum > rank) return qv[h];
        }
        return qv[order.back()];
    };
    const int64_t m = total / 2;
    return total % 2 ? at(m) : 0.5 * (at(m - 1) + at(m));
}

}  // namespace
}  // namespace hs

using namespace hs;

extern "C" {

int overlap_analyze(const uint64_t *configs, const int32_t *energy, int n, int n_words, const uint64_t *mask,
                    int n_live, int32_t *scratch, void *stream, hs_overlap *out)
{
    if (configs == nullptr || energy == nullptr || mask == nullptr || scratch == nullptr || out == nullptr || n < 1 ||
        n > 46340 || n_words < 1 || n_live < 1)
        return fail(HS_EINVAL, "overlap_analyze: bad arguments");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // every distance is at most popcount(mask): n_live must be that count
    std::vector<uint64_t> mh(size_t(n_words), 0);
    hipError_t em = hipMemcpyAsync(mh.data(), mask, mh.size() * 8, hipMemcpyDeviceToHost, s);
    if (em == hipSuccess) em = hipStreamSynchronize(s);
    if (em != hipSuccess) return fail(HS_EHIP, std::string("overlap_analyze: ") + hipGetErrorString(em));
    int live = 0;
    for (uint64_t w : mh) live += __builtin_popcountll(w);
    if (live != n_live) return fail(HS_EINVAL, "overlap_analyze: n_live is not the popcount of the mask");
    hipLaunchKernelGGL(dev::k_hamming, dim3(unsigned(n), unsigned((n + 255) / 256)), dim3(256), 0, s, configs, n,
                       n_words, mask, scratch);
    std::vector<int32_t> h(size_t(n) * size_t(n));
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), scratch, h.size() * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(HS_EHIP, std::string("overlap_analyze: ") + hipGetErrorString(e));
    // levels present
    std::vector<int32_t> lv(energy, energy + n);
    std::sort(lv.begin(), lv.end());
    lv.erase(std::unique(lv.begin(), lv.end()), lv.end());
    // distinct configurations of one level, up to the global flip, in index order
    auto distinct = [&](int32_t level) {
        std::vector<int> kept;
        for (int i = 0; i < n; ++i) {
            if (energy[i] != level) continue;
            bool dup = false;
            for (int k : kept) {
                const int32_t d = h[size_t(i) * n + size_t(k)];
                dup = dup || d == 0 || d == n_live;
            }
            if (!dup) kept.push_back(i);
        }
        return kept;
    };
    const std::vector<int> gs = distinct(lv[0]);
    std::vector<int64_t> gg(size_t(n_live) + 1, 0);
    for (size_t a = 0; a < gs.size(); ++a)
        for (size_t b = a + 1; b < gs.size(); ++b) ++gg[h[size_t(gs[a]) * n + size_t(gs[b])]];
    out->e0 = lv[0];
    out->n_gs = int32_t(gs.size());
    out->med_gg = gs.size() < 2 ? 1.0 : median_q(gg, n_live);
    out->has_excited = lv.size() > 1 ? 1 : 0;
    out->e1 = lv.size() > 1 ? lv[1] : lv[0];
    out->n_ex = 0;
    out->med_ge = 0.0;
    out->ratio = 0.0;
    if (lv.size() > 1) {
        const std::vector<int> ex = distinct(lv[1]);
        std::vector<int64_t> ge(size_t(n_live) + 1, 0);
        for (int g : gs)
            for (int x : ex) ++ge[h[size_t(g) * n + size_t(x)]];
        out->n_ex = int32_t(ex.size());
        out->med_ge = median_q(ge, n_live);
        out->ratio = out->med_ge / out->med_gg;
    }
    return HS_OK;
}

}  // extern "C"
