// hardness_eval: time-to-solution of candidate instances from independent PT
// restarts that stop on ground-state agreement (Sec. III.B cross-check of PT
// ground-state energies; Appendix B agreement rule), all restarts of all
// candidates in one persistent launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "hs_internal.h"

using namespace hs;

// Device scratch of hardness_eval_static: one copy per GPU, held until the
// process ends.  In host code `scratch` names a host-side stand-in, never the
// device memory: host code uses the per-device address from
// hipGetSymbolAddress (static_scratch below).
static __device__ __align__(256) unsigned char scratch[HS_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

// Address of the current device's copy of `scratch`, looked up once per
// device with that device current.
int static_scratch(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(HS_EHIP, std::string("hardness_eval_static: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(HS_EUNSUPPORTED, "hardness_eval_static: device index >= 64");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_addr[dev] == nullptr) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(HS_EHIP, std::string("hardness_eval_static: scratch address: ") + hipGetErrorString(e));
        g_scratch_addr[dev] = p;
    }
    *out = g_scratch_addr[dev];
    return HS_OK;
}

struct HardnessLayout {
    size_t spins, perm, energy, emin, thit, sacc, t, stopped, ws, total, ws_bytes;
};

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

int build_batch(const hs_instance *cands, int n, const hs_hardness_params *p,
                std::vector<hs_instance> &runs, hs_pt_desc &d)
{
    if (cands == nullptr || p == nullptr || n < 0) return fail(HS_EINVAL, "hardness: bad arguments");
    if (p->n_restarts < 1 || p->R < 2 || p->s_max < 0 || p->beta == nullptr)
        return fail(HS_EINVAL, "hardness: need n_restarts >= 1, R >= 2, s_max >= 0, beta");
    runs.clear();
    for (int c = 0; c < n; ++c)
        for (int rho = 0; rho < p->n_restarts; ++rho) {
            hs_instance x = cands[c];
            const uint32_t ctr[4] = {uint32_t(rho), 0u, 0u, kUseRestart};
            const uint32_t key[2] = {cands[c].instance_id, p->seed};
            uint32_t w[4];
            philox_host(ctr, key, w);
            x.instance_id = w[0];
            x.K = p->K;
            x.R = p->R;
            x.beta = p->beta;
            runs.push_back(x);
        }
    d.n_inst = int32_t(runs.size());
    d.inst = runs.data();
    d.seed = p->seed;
    d.swap_interval = p->swap_interval;
    d.flags = HS_STOP_ON_AGREEMENT;
    d.block_waves = p->block_waves;
    return HS_OK;
}

int layout(const std::vector<hs_instance> &runs, const hs_pt_desc &d, HardnessLayout &L)
{
    size_t sites = 0;
    for (const auto &r : runs) sites += size_t(8) * r.L * r.L;
    const size_t m = std::max<size_t>(1, runs.size());
    size_t o = 0;
    L.spins = o;
    o = up256(o + sites * 8);
    L.perm = o;
    o = up256(o + m * 64);
    L.energy = o;
    o = up256(o + m * 64 * 4);
    L.emin = o;
    o = up256(o + m * 64 * 4);
    L.thit = o;
    o = up256(o + m * 64 * 8);
    L.sacc = o;
    o = up256(o + m * 64 * 4);
    L.t = o;
    o = up256(o + m * 8);
    L.stopped = o;
    o = up256(o + m * 4);
    L.ws = o;
    size_t wsb = 0;
    if (!runs.empty()) {
        int rc = pt_workspace_bytes(&d, &wsb);
        if (rc) return rc;
    }
    L.ws_bytes = wsb;
    L.total = up256(o + wsb);
    return HS_OK;
}

}  // namespace

extern "C" {

int hardness_workspace_bytes(const hs_instance *cands, int n, const hs_hardness_params *p, size_t *bytes)
{
    if (bytes == nullptr) return fail(HS_EINVAL, "hardness_workspace_bytes: NULL");
    std::vector<hs_instance> runs;
    hs_pt_desc d{};
    int rc = build_batch(cands, n, p, runs, d);
    if (rc) return rc;
    HardnessLayout L{};
    rc = layout(runs, d, L);
    if (rc) return rc;
    *bytes = L.total;
    return HS_OK;
}

}  // extern "C"

namespace {

// Every restart of every candidate in one persistent launch on the device
// memory at `base` (L.total bytes laid out by `layout`); pt_init writes every
// byte the launch reads (workspace image, initial state), so nothing has to
// be cleared beforehand.
int run_hardness(int n, const hs_hardness_params *p, std::vector<hs_instance> &runs,
                 const hs_pt_desc &d, const HardnessLayout &L, char *base, double *ln_tts_out, hs_tts_detail *detail,
                 void *stream)
{
    int rc = HS_OK;
    hs_buffers b{};
    b.spins = reinterpret_cast<uint64_t *>(base + L.spins);
    b.perm = reinterpret_cast<uint8_t *>(base + L.perm);
    b.energy = reinterpret_cast<int32_t *>(base + L.energy);
    b.emin = reinterpret_cast<int32_t *>(base + L.emin);
    b.thit = reinterpret_cast<int64_t *>(base + L.thit);
    b.swap_acc = reinterpret_cast<uint32_t *>(base + L.sacc);
    b.t = reinterpret_cast<int64_t *>(base + L.t);
    b.stopped = reinterpret_cast<int32_t *>(base + L.stopped);
    b.workspace = base + L.ws;
    b.workspace_bytes = L.ws_bytes;
    hs_pt *h = nullptr;
    // the stream is synchronised below before pt_destroy: no upload event
    rc = pt_init_ex(&h, &d, &b, stream, false);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    rc = pt_sweep(h, p->s_max);
    if (rc) {
        (void)hipStreamSynchronize(s);  // the upload reads the handle's host copy
        pt_destroy(h);
        return rc;
    }
    const size_t m = runs.size();
    std::vector<int32_t> emin(m * 64);
    std::vector<int64_t> thit(m * 64), t(m);
    hipError_t e = hipMemcpyAsync(emin.data(), b.emin, m * 64 * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(thit.data(), b.thit, m * 64 * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(t.data(), b.t, m * 8, hipMemcpyDeviceToHost, s);
    const hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess) e = es;
    pt_destroy(h);
    if (e != hipSuccess) return fail(HS_EHIP, std::string("hardness_eval: ") + hipGetErrorString(e));
    const int nr = p->n_restarts, R = p->R;
    for (int c = 0; c < n; ++c) {
        int32_t gs = INT32_MAX;
        for (int rho = 0; rho < nr; ++rho)
            for (int r = 0; r < R; ++r) gs = std::min(gs, emin[(size_t(c) * nr + rho) * 64 + r]);
        int hits = 0, double_hit = 0, censored = 0;
        int64_t sweeps = 0;
        for (int rho = 0; rho < nr; ++rho) {
            const size_t run = size_t(c) * nr + rho;
            sweeps += t[run];
            if (p->restart_sweeps) p->restart_sweeps[size_t(c) * nr + rho] = t[run];
            int sets = 0;
            for (int r = 0; r < R; ++r) sets += emin[run * 64 + r] == gs ? 1 : 0;
            if (sets >= 2) double_hit = 1;
            if (sets > 0)
                ++hits;
            else
                ++censored;
        }
        // run time per find of the presumed minimum (Appendix B): all restart
        // sweeps over the restarts that ended at E_gs (at least one does)
        ln_tts_out[c] = std::log(double(std::max<int64_t>(sweeps, 1)) / double(hits));
        if (detail) {
            detail[c].e_gs = gs;
            detail[c].confirmed = (hits >= 2 || double_hit) ? 1 : 0;
            detail[c].n_censored = censored;
            detail[c].sweeps_total = sweeps;
        }
    }
    return HS_OK;
}

}  // namespace

extern "C" {

int hardness_eval(const hs_instance *cands, int n, const hs_hardness_params *p, void *scratch_buf,
                  size_t scratch_bytes, double *ln_tts_out, hs_tts_detail *detail, void *stream)
{
    if (ln_tts_out == nullptr || (n > 0 && scratch_buf == nullptr))
        return fail(HS_EINVAL, "hardness_eval: NULL argument");
    std::vector<hs_instance> runs;
    hs_pt_desc d{};
    int rc = build_batch(cands, n, p, runs, d);
    if (rc) return rc;
    if (n == 0) return HS_OK;
    HardnessLayout L{};
    rc = layout(runs, d, L);
    if (rc) return rc;
    if (scratch_bytes < L.total) return fail(HS_ENOSPACE, "hardness_eval: scratch too small");
    return run_hardness(n, p, runs, d, L, reinterpret_cast<char *>(scratch_buf), ln_tts_out, detail, stream);
}

int hs_stream_create_cus(int32_t cu_first, int32_t cu_count, void **stream)
{
    if (stream == nullptr) return fail(HS_EINVAL, "hs_stream_create_cus: NULL stream");
    int dev = 0, n = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return fail(HS_EHIP, std::string("hs_stream_create_cus: ") + hipGetErrorString(e));
    if (cu_first < 0 || cu_count < 1 || int64_t(cu_first) + cu_count > n)
        return fail(HS_EINVAL, "hs_stream_create_cus: CU range outside the device's " + std::to_string(n));
    std::vector<uint32_t> mask((n + 31) / 32, 0u);
    for (int c = cu_first; c < cu_first + cu_count; ++c) mask[c / 32] |= 1u << (c % 32);
    hipStream_t st = nullptr;
    e = hipExtStreamCreateWithCUMask(&st, uint32_t(mask.size()), mask.data());
    if (e != hipSuccess) return fail(HS_EHIP, std::string("hs_stream_create_cus: ") + hipGetErrorString(e));
    *stream = st;
    return HS_OK;
}

int hs_stream_destroy(void *stream)
{
    if (stream == nullptr) return HS_OK;
    const hipError_t e = hipStreamDestroy(reinterpret_cast<hipStream_t>(stream));
    return e == hipSuccess ? HS_OK : fail(HS_EHIP, std::string("hs_stream_destroy: ") + hipGetErrorString(e));
}

int hardness_eval_static(const hs_instance *cands, int n, const hs_hardness_params *p, double *ln_tts_out,
                         hs_tts_detail *detail, void *stream)
{
    if (ln_tts_out == nullptr) return fail(HS_EINVAL, "hardness_eval_static: NULL argument");
    std::vector<hs_instance> runs;
    hs_pt_desc d{};
    int rc = build_batch(cands, n, p, runs, d);
    if (rc) return rc;
    if (n == 0) return HS_OK;
    HardnessLayout L{};
    rc = layout(runs, d, L);
    if (rc) return rc;
    if (L.total > size_t(HS_STATIC_SCRATCH_BYTES))
        return fail(HS_ENOSPACE, "hardness_eval_static: the batch needs " + std::to_string(L.total) +
                                     " bytes of scratch, more than the static " +
                                     std::to_string(size_t(HS_STATIC_SCRATCH_BYTES)) +
                                     "; use hardness_eval with a caller buffer");
    void *base = nullptr;
    rc = static_scratch(&base);
    if (rc) return rc;
    return run_hardness(n, p, runs, d, L, reinterpret_cast<char *>(base), ln_tts_out, detail, stream);
}

}  // extern "C"
