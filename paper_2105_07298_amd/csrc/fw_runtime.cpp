// fw_runtime.cpp -- host side of the C ABI: argument checks, padding, the round
// loop of the blocked method (paper Sect. 2.2; one round per block of k, three
// dependent launches per round as in Sect. 3.2), status codes and timing hooks.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/fw_apsp.h"
#include "fw_internal.h"

namespace {

thread_local char g_err[512] = "";

fw_status_t fail(fw_status_t st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

fw_status_t hip_fail(hipError_t e, const char *what) {
    return fail(FW_EHIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

// ---- last-phase timing hooks ------------------------------------------------
// When enabled, each last-phase launch is bracketed by two events on its
// stream; fw_prof_read() synchronizes them and returns the count and summed time.
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<hipEvent_t> g_ev_pool;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_ev_used;
hipEvent_t g_pending = nullptr;

hipEvent_t take_event() {
    if (!g_ev_pool.empty()) {
        hipEvent_t e = g_ev_pool.back();
        g_ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

constexpr int64_t kMaxN = int64_t(1) << 20;
constexpr int32_t kMaxBatchedN = 4096;
constexpr int32_t kMaxBackwardN = 4096;

// Pinned staging for the batched job table.
std::mutex g_stage_mu;
void *g_stage = nullptr;
size_t g_stage_cap = 0;
hipEvent_t g_stage_ev = nullptr;

struct TuneEntry { int f64, path; long long n_lo, n_hi; int block, tile_m, tile_n; };
struct TuneBatchedEntry { int f64, path, small_max_n; };
#include "tune_table.inc"

fw::TileCfg default_cfg(fw_dtype_t dt, int64_t n, bool path) { return fw::tuned_config(dt == FW_F64, path, n); }

template <typename T>
fw_status_t run_apsp(int64_t n, T *dist, int32_t *path, fw::TileCfg cfg, hipStream_t s) {
    if (!fw::config_supported<T>(cfg))
        return fail(FW_EUNSUPPORTED, "block %d / tile %d x %d not compiled in", cfg.block, cfg.tile_m, cfg.tile_n);
    const int64_t unit = cfg.tile_m > cfg.tile_n ? cfg.tile_m : cfg.tile_n;
    const int64_t npad = (n + unit - 1) / unit * unit;
    const bool aligned = ((uintptr_t)dist % 16 == 0) && (path == nullptr || (uintptr_t)path % 16 == 0);
    hipError_t e;
    T *D = dist;
    int32_t *P = path;
    void *scratch = nullptr;
    if (npad != n || !aligned) {
        const size_t dbytes = (size_t)(npad * npad) * sizeof(T);
        const size_t pbytes = path ? (size_t)(npad * npad) * sizeof(int32_t) : 0;
        e = hipMallocAsync(&scratch, dbytes + pbytes, s);
        if (e != hipSuccess) return fail(FW_ENOMEM, "scratch of %zu bytes: %s", dbytes + pbytes, hipGetErrorString(e));
        D = (T *)scratch;
        P = path ? (int32_t *)((char *)scratch + dbytes) : nullptr;
        if ((e = fw::launch_pad_in<T>(dist, n, D, npad, s)) != hipSuccess) return hip_fail(e, "pad");
    }
    if (P && (e = fw::launch_fill_i32(P, npad * npad, -1, s)) != hipSuccess) return hip_fail(e, "path init");
    // Path mode scratch: pending marks L (uint16, zeroed), then the transpose of
    // D for the label resolution.
    void *ps = nullptr;
    uint16_t *L = nullptr;
    const size_t lbytes = (size_t)(npad * npad) * sizeof(uint16_t), tbytes = (size_t)(npad * npad) * sizeof(T);
    if (P) {
        e = hipMallocAsync(&ps, lbytes + tbytes, s);
        if (e != hipSuccess) return fail(FW_ENOMEM, "label scratch of %zu bytes: %s", lbytes + tbytes, hipGetErrorString(e));
        L = (uint16_t *)ps;
        if ((e = fw::launch_fill_i32((int32_t *)L, npad * npad / 2, 0, s)) != hipSuccess) return hip_fail(e, "mark init");
    }
    const int R = (int)(npad / cfg.block);
    for (int r = 0; r < R; ++r)
        if ((e = fw::launch_round<T>(D, P, L, npad, r, cfg, s)) != hipSuccess) return hip_fail(e, "round launch");
    if (P) {
        e = fw::launch_resolve<T>(D, (T *)((char *)ps + lbytes), L, P, npad, cfg.block, s);
        hipError_t e2 = hipFreeAsync(ps, s);
        if (e != hipSuccess) return hip_fail(e, "label resolution");
        if (e2 != hipSuccess) return hip_fail(e2, "label scratch free");
    }
    if (scratch) {
        if ((e = fw::launch_pad_out<T>(D, npad, dist, n, s)) != hipSuccess) return hip_fail(e, "unpad");
        if (path && (e = fw::launch_pad_out<int32_t>(P, npad, path, n, s)) != hipSuccess) return hip_fail(e, "unpad P");
        if ((e = hipFreeAsync(scratch, s)) != hipSuccess) return hip_fail(e, "scratch free");
    }
    return FW_OK;
}

fw_status_t check_common(fw_dtype_t dt, int64_t n, const void *dist) {
    if (dt != FW_F32 && dt != FW_F64) return fail(FW_EINVAL, "unknown dtype %d", (int)dt);
    if (n < 1 || n > kMaxN) return fail(FW_EINVAL, "n = %lld outside [1, %lld]", (long long)n, (long long)kMaxN);
    if (dist == nullptr) return fail(FW_EINVAL, "dist is NULL");
    return FW_OK;
}

}  // namespace

namespace fw {
TileCfg tuned_config(bool f64, bool path, int64_t n) {
    for (const TuneEntry &t : kTuneApsp)
        if (t.f64 == (int)f64 && t.path == (int)path && n >= t.n_lo && n < t.n_hi) return {t.block, t.tile_m, t.tile_n};
    return {64, 64, 64};
}
int tuned_batched_small_max_n(bool f64, bool path) {
    for (const TuneBatchedEntry &t : kTuneBatched)
        if (t.f64 == (int)f64 && t.path == (int)path) return t.small_max_n;
    return 0;
}

void prof_begin_p4(hipStream_t s) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_pending = take_event();
    if (g_pending) (void)hipEventRecord(g_pending, s);
}
void prof_end_p4(hipStream_t s) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_pending) return;
    hipEvent_t e = take_event();
    if (!e) return;
    (void)hipEventRecord(e, s);
    g_ev_used.push_back({g_pending, e});
    g_pending = nullptr;
}
}  // namespace fw

extern "C" {

fw_status_t fw_apsp_config(fw_dtype_t dt, int64_t n, void *dist, int32_t *path, const fw_config_t *cfg, void *stream) {
    g_err[0] = 0;
    fw_status_t st = check_common(dt, n, dist);
    if (st != FW_OK) return st;
    fw::TileCfg tc = default_cfg(dt, n, path != nullptr);
    if (cfg) {
        if (cfg->reserved) return fail(FW_EINVAL, "reserved config field must be 0");
        if (cfg->block) tc.block = cfg->block;
        if (cfg->tile_m) tc.tile_m = cfg->tile_m;
        if (cfg->tile_n) tc.tile_n = cfg->tile_n;
        if (tc.block <= 0 || tc.tile_m <= 0 || tc.tile_n <= 0 || tc.tile_m % tc.block || tc.tile_n % tc.block)
            return fail(FW_EINVAL, "tile edges must be multiples of block");
    }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipStream_t s = (hipStream_t)stream;
    if (dt == FW_F32) return run_apsp<float>(n, (float *)dist, path, tc, s);
    return run_apsp<double>(n, (double *)dist, path, tc, s);
}

fw_status_t fw_query_config(fw_dtype_t dt, int64_t n, int32_t path, fw_config_t *out) {
    g_err[0] = 0;
    if (dt != FW_F32 && dt != FW_F64) return fail(FW_EINVAL, "unknown dtype %d", (int)dt);
    if (n < 1 || n > kMaxN) return fail(FW_EINVAL, "n = %lld outside [1, %lld]", (long long)n, (long long)kMaxN);
    if (!out) return fail(FW_EINVAL, "out is NULL");
    const fw::TileCfg c = default_cfg(dt, n, path != 0);
    out->block = c.block;
    out->tile_m = c.tile_m;
    out->tile_n = c.tile_n;
    out->reserved = 0;
    return FW_OK;
}

fw_status_t fw_apsp(fw_dtype_t dt, int64_t n, void *dist, int32_t *path, void *stream) {
    return fw_apsp_config(dt, n, dist, path, nullptr, stream);
}

fw_status_t fw_apsp_batched_config(fw_dtype_t dt, int32_t batch, const int32_t *n_host, const int64_t *off_host,
                                   void *dist, int32_t *path, const fw_batched_config_t *cfg, void *stream) {
    g_err[0] = 0;
    if (cfg && (cfg->reserved0 || cfg->reserved1 || cfg->reserved2)) return fail(FW_EINVAL, "reserved config fields must be 0");
    if (dt != FW_F32 && dt != FW_F64) return fail(FW_EINVAL, "unknown dtype %d", (int)dt);
    if (batch < 1) return fail(FW_EINVAL, "batch = %d < 1", batch);
    if (!n_host || !off_host || !dist) return fail(FW_EINVAL, "NULL argument");
    for (int32_t b = 0; b < batch; ++b) {
        if (n_host[b] < 1 || n_host[b] > kMaxBatchedN)
            return fail(FW_EINVAL, "n[%d] = %d outside [1, %d]", b, n_host[b], kMaxBatchedN);
        if (off_host[b] < 0) return fail(FW_EINVAL, "offset[%d] < 0", b);
    }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipStream_t s = (hipStream_t)stream;
    const int small_max_n = (cfg && cfg->small_max_n >= 0) ? cfg->small_max_n
                                                          : fw::tuned_batched_small_max_n(dt == FW_F64, path != nullptr);
    // Queue in order of decreasing n (longest job first); counter slot first.
    std::vector<int32_t> order((size_t)batch);
    for (int32_t b = 0; b < batch; ++b) order[(size_t)b] = b;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return n_host[x] > n_host[y]; });
    const size_t words = 1 + 2 * (size_t)batch, bytes = words * sizeof(int64_t);
    void *djobs = nullptr;
    e = hipMallocAsync(&djobs, bytes, s);
    if (e != hipSuccess) return fail(FW_ENOMEM, "job table of %zu bytes: %s", bytes, hipGetErrorString(e));
    {
        // Pinned staging buffer, reused across calls once its previous upload is done.
        std::lock_guard<std::mutex> lk(g_stage_mu);
        if (g_stage_ev && (e = hipEventSynchronize(g_stage_ev)) != hipSuccess) return hip_fail(e, "staging wait");
        if (g_stage_cap < bytes) {
            if (g_stage) (void)hipHostFree(g_stage);
            g_stage = nullptr;
            g_stage_cap = 0;
            if ((e = hipHostMalloc(&g_stage, bytes, 0)) != hipSuccess) return fail(FW_ENOMEM, "pinned staging: %s", hipGetErrorString(e));
            g_stage_cap = bytes;
        }
        int64_t *tab = (int64_t *)g_stage;
        tab[0] = 0;
        for (int32_t q = 0; q < batch; ++q) {
            tab[1 + 2 * q] = off_host[order[(size_t)q]];
            tab[2 + 2 * q] = n_host[order[(size_t)q]];
        }
        if ((e = hipMemcpyAsync(djobs, g_stage, bytes, hipMemcpyHostToDevice, s)) != hipSuccess) return hip_fail(e, "job upload");
        if (!g_stage_ev && (e = hipEventCreateWithFlags(&g_stage_ev, hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "event");
        if ((e = hipEventRecord(g_stage_ev, s)) != hipSuccess) return hip_fail(e, "event record");
    }
    int cus = 0;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return hip_fail(e, "CU count");
    const bool p = path != nullptr;
    const int occ = dt == FW_F32 ? fw::batched_occupancy<float>(p) : fw::batched_occupancy<double>(p);
    int grid = cus * occ;
    if (grid > batch) grid = batch;
    e = dt == FW_F32 ? fw::launch_batched<float>((float *)dist, path, (int64_t *)djobs, batch, small_max_n, grid, s)
                     : fw::launch_batched<double>((double *)dist, path, (int64_t *)djobs, batch, small_max_n, grid, s);
    hipError_t e2 = hipFreeAsync(djobs, s);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    if (e2 != hipSuccess) return hip_fail(e2, "job table free");
    return FW_OK;
}

fw_status_t fw_apsp_batched(fw_dtype_t dt, int32_t batch, const int32_t *n_host, const int64_t *off_host, void *dist,
                            int32_t *path, void *stream) {
    return fw_apsp_batched_config(dt, batch, n_host, off_host, dist, path, nullptr, stream);
}

fw_status_t fw_apsp_backward(fw_dtype_t dt, int64_t n, int32_t batch, const void *dist, const int32_t *path,
                             const void *grad_dist, void *grad_w, void *stream) {
    g_err[0] = 0;
    if (dt != FW_F32 && dt != FW_F64) return fail(FW_EINVAL, "unknown dtype %d", (int)dt);
    if (n < 1 || n > kMaxBackwardN) return fail(FW_EINVAL, "n = %lld outside [1, %d]", (long long)n, kMaxBackwardN);
    if (batch < 1 || batch > 65535) return fail(FW_EINVAL, "batch = %d outside [1, 65535]", batch);
    if (!dist || !path || !grad_dist || !grad_w) return fail(FW_EINVAL, "NULL argument (path is required)");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipStream_t s = (hipStream_t)stream;
    e = dt == FW_F32 ? fw::launch_backward<float>((const float *)dist, path, (const float *)grad_dist,
                                                  (float *)grad_w, (int)n, batch, s)
                     : fw::launch_backward<double>((const double *)dist, path, (const double *)grad_dist,
                                                   (double *)grad_w, (int)n, batch, s);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    return FW_OK;
}

const char *fw_status_string(int st) {
    switch (st) {
    case FW_OK: return "ok";
    case FW_EINVAL: return "invalid argument";
    case FW_ENOMEM: return "out of device memory";
    case FW_EHIP: return "HIP runtime error";
    case FW_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *fw_last_error(void) { return g_err; }

const char *fw_version(void) { return "fwapsp 0.1 gfx950"; }

// Timing hooks for the benchmark: enable/disable bracketing of last-phase
// launches with events, and read (count, summed milliseconds) since the last
// reset.  fw_prof_read synchronizes on the recorded events.
void fw_prof_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
}

int fw_prof_read(int64_t *count, double *total_ms, int reset) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    double tot = 0.0;
    int64_t cnt = 0;
    for (auto &pr : g_ev_used) {
        if (hipEventSynchronize(pr.second) != hipSuccess) return FW_EHIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess) return FW_EHIP;
        tot += ms;
        ++cnt;
    }
    if (count) *count = cnt;
    if (total_ms) *total_ms = tot;
    if (reset) {
        for (auto &pr : g_ev_used) {
            g_ev_pool.push_back(pr.first);
            g_ev_pool.push_back(pr.second);
        }
        g_ev_used.clear();
    }
    return FW_OK;
}

}  // extern "C"
