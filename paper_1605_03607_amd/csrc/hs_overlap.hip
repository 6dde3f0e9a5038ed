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

double median(std::vector<double> v)
{
    std::sort(v.begin(), v.end());
    const size_t m = v.size() / 2;
    return v.size() % 2 ? v[m] : 0.5 * (v[m - 1] + v[m]);
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
    auto q = [&](int i, int j) { return std::fabs(1.0 - 2.0 * double(h[size_t(i) * n + size_t(j)]) / n_live); };
    const std::vector<int> gs = distinct(lv[0]);
    std::vector<double> gg;
    for (size_t a = 0; a < gs.size(); ++a)
        for (size_t b = a + 1; b < gs.size(); ++b) gg.push_back(q(gs[a], gs[b]));
    out->e0 = lv[0];
    out->n_gs = int32_t(gs.size());
    out->med_gg = gg.empty() ? 1.0 : median(gg);
    out->has_excited = lv.size() > 1 ? 1 : 0;
    out->e1 = lv.size() > 1 ? lv[1] : lv[0];
    out->n_ex = 0;
    out->med_ge = 0.0;
    out->ratio = 0.0;
    if (lv.size() > 1) {
        const std::vector<int> ex = distinct(lv[1]);
        std::vector<double> ge;
        for (int g : gs)
            for (int x : ex) ge.push_back(q(g, x));
        out->n_ex = int32_t(ex.size());
        out->med_ge = median(ge);
        out->ratio = out->med_ge / out->med_gg;
    }
    return HS_OK;
}

}  // extern "C"
