// fw_runtime.cpp -- host side of the C ABI: argument checks, padding, the round
// loop of the blocked method (paper Sect. 2.2; one round per block of k, three
// dependent launches per round as in Sect. 3.2), status codes and timing hooks.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <vector>

#include "../../include/fw_apsp.h"
#include "fw_internal.h"
#include "fw_route.h"
#include "fw_plan.h"

static_assert(fw::FW_VARIANT_PANELS == FW_P4_PANELS && fw::FW_VARIANT_WAVEROWS == FW_P4_WAVEROWS,
              "variant codes of the C ABI");
static_assert(fw::FW_SCHEDULE_SERIAL == FW_SCHED_SERIAL && fw::FW_SCHEDULE_LOOKAHEAD == FW_SCHED_LOOKAHEAD &&
                  fw::FW_SCHEDULE_PAIRS == FW_SCHED_PAIRS &&
                  fw::FW_SCHEDULE_PAIRS_LOOKAHEAD == FW_SCHED_PAIRS_LOOKAHEAD,
              "schedule codes of the C ABI");
static_assert(FW_F32 == 0 && FW_F64 == 1 && FW_F16 == 2, "dtype codes of the tuning table");

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
// When enabled, each bulk last-phase launch (every tile outside the round's
// block, or the caller-stream part of a pair of rounds) is bracketed by two
// events on its stream; fw_prof_read() synchronizes them and returns the count,
// the summed time and the summed algorithmic updates.
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<hipEvent_t> g_ev_pool;
struct ProfRec {
    hipEvent_t begin, end;
    int64_t updates;
};
std::vector<ProfRec> g_ev_used;
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

struct TuneEntry { int dtype, path; long long n_lo, n_hi; int block, tile_m, tile_n, variant, schedule; };
struct TuneBatchedEntry { int dtype, path; unsigned long long tile64; };
#include "tune_table.inc"

fw::TileCfg default_cfg(fw_dtype_t dt, int64_t n, bool path) { return fw::tuned_config((int)dt, path, n); }

bool supported_for(fw_dtype_t dt, fw::TileCfg c) {
    return dt == FW_F32 ? fw::config_supported<float>(c)
                        : dt == FW_F64 ? fw::config_supported<double>(c) : fw::config_supported<_Float16>(c);
}

// ---- lookahead ---------------------------------------------------------------
// Phases 1-3 of round r + 1 only read and write block row and column r + 1.  The
// last phase of round r is therefore split: a small "cross" launch finishes
// block row and column r + 1, and a "rest" launch does every other tile.  The
// two are independent (disjoint tiles, read-only panels), and cross(r) only
// needs rest(r - 1).  The caller's stream runs the rest launches back to back;
// an auxiliary stream runs cross(r), then phases 1-3 of round r + 1, which the
// caller's stream waits for before rest(r + 1):
//   main: ... rest(r-1) -> [wait p23(r)]   rest(r)    -> [wait p23(r+1)] rest(r+1) ...
//   aux:  ... [wait rest(r-1)] cross(r) -> p1(r+1) -> p23(r+1) -> [wait rest(r)] cross(r+1) ...
// Events alternate between two per direction, so a wait never sees a record
// from a later round.  The auxiliary streams (default priority, non-blocking)
// and their events are kept per device and reused; one call holds one at a time.
struct Aux {
    int dev;
    hipStream_t st;
    // The lookahead schedule uses ev[0..1] (rest done), ev[2..3] (phases 2+3
    // done) and ev[6] (start); the pairs-with-lookahead plan all seven (fw_plan.h).
    hipEvent_t ev[fw::kPlanEvents];
    bool busy;
};
std::mutex g_aux_mu;
std::vector<Aux *> g_aux;  // never freed: streams live until the process ends

Aux *acquire_aux(int dev) {
    std::lock_guard<std::mutex> lk(g_aux_mu);
    for (Aux *a : g_aux)
        if (a->dev == dev && !a->busy) {
            a->busy = true;
            return a;
        }
    Aux *a = new Aux{dev, nullptr, {}, true};
    bool ok = hipStreamCreateWithFlags(&a->st, hipStreamNonBlocking) == hipSuccess;
    for (hipEvent_t &e : a->ev) ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        for (hipEvent_t &e : a->ev)
            if (e) (void)hipEventDestroy(e);
        if (a->st) (void)hipStreamDestroy(a->st);
        delete a;
        return nullptr;
    }
    g_aux.push_back(a);
    return a;
}

void release_aux(Aux *a) {
    std::lock_guard<std::mutex> lk(g_aux_mu);
    a->busy = false;
}

// Rounds with lookahead need at least 3 blocks (else there is nothing to overlap).
constexpr int kLookaheadMinRounds = 3;

template <typename T>
hipError_t run_rounds(T *D, int32_t *P, uint16_t *L, int64_t ld, fw::TileCfg cfg, hipStream_t s) {
    using fw::P4Mode;
    const int R = (int)(ld / cfg.block);
    const bool path = P != nullptr;
    hipError_t e;
    int dev = -1;
    Aux *aux = nullptr;
    if (cfg.schedule == fw::FW_SCHEDULE_PAIRS && R >= 2 && fw::pairs_supported(cfg)) {
        // Pairs of rounds on one stream: round r's last phase on block r + 1,
        // phases 1-3 of round r + 1, both rounds' last phase on every other tile
        // in one pass, then round r + 1's on block r (after that pass has read
        // block r as round r's panels).
        for (int r = 0; r < R; r += 2) {
            if ((e = fw::launch_phase123<T>(D, P, L, ld, r, cfg.block, s)) != hipSuccess) return e;
            if (r + 1 == R) return fw::launch_phase4<T>(D, L, path, ld, r, cfg, P4Mode::all, s);
            if ((e = fw::launch_phase4<T>(D, L, path, ld, r, cfg, P4Mode::cross, s)) != hipSuccess) return e;
            if ((e = fw::launch_phase123<T>(D, P, L, ld, r + 1, cfg.block, s)) != hipSuccess) return e;
            if ((e = fw::launch_phase4<T>(D, L, path, ld, r, cfg, P4Mode::pair, s)) != hipSuccess) return e;
            if ((e = fw::launch_phase4<T>(D, L, path, ld, r + 1, cfg, P4Mode::crossprev, s)) != hipSuccess) return e;
        }
        return hipSuccess;
    }
    if (cfg.schedule == fw::FW_SCHEDULE_PAIRS_LOOKAHEAD && R >= kLookaheadMinRounds && fw::pairs_supported(cfg) &&
        hipGetDevice(&dev) == hipSuccess && (aux = acquire_aux(dev)) != nullptr) {
        // The plan of fw_plan.h, enqueued op by op (stream 1 = the auxiliary stream).
        hipError_t err = hipSuccess;
        fw::plan_pairs_lookahead(R, [&](const fw::PlanOp &op) {
            if (err != hipSuccess) return;
            hipStream_t st = op.stream ? aux->st : s;
            switch (op.kind) {
            case fw::PlanKind::p123: err = fw::launch_phase123<T>(D, P, L, ld, op.r, cfg.block, st); break;
            case fw::PlanKind::p4: err = fw::launch_phase4<T>(D, L, path, ld, op.r, cfg, op.mode, st); break;
            case fw::PlanKind::record: err = hipEventRecord(aux->ev[op.ev], st); break;
            case fw::PlanKind::wait: err = hipStreamWaitEvent(st, aux->ev[op.ev], 0); break;
            }
        });
        release_aux(aux);
        return err;
    }
    if (cfg.schedule == fw::FW_SCHEDULE_LOOKAHEAD && R >= kLookaheadMinRounds && fw::lookahead_supported(cfg) &&
        hipGetDevice(&dev) == hipSuccess)
        aux = acquire_aux(dev);
    if (!aux) {
        for (int r = 0; r < R; ++r) {
            if ((e = fw::launch_phase123<T>(D, P, L, ld, r, cfg.block, s)) != hipSuccess) return e;
            if ((e = fw::launch_phase4<T>(D, L, path, ld, r, cfg, P4Mode::all, s)) != hipSuccess) return e;
        }
        return hipSuccess;
    }
    hipStream_t a = aux->st;
    auto body = [&]() -> hipError_t {
        hipError_t e;
        if ((e = hipEventRecord(aux->ev[fw::kEvStart], s)) != hipSuccess) return e;  // after the caller's earlier work
        if ((e = hipStreamWaitEvent(a, aux->ev[fw::kEvStart], 0)) != hipSuccess) return e;
        if ((e = fw::launch_phase123<T>(D, P, L, ld, 0, cfg.block, a)) != hipSuccess) return e;
        if ((e = hipEventRecord(aux->ev[2], a)) != hipSuccess) return e;
        for (int r = 0; r + 1 < R; ++r) {
            // main stream: the bulk of round r
            if ((e = hipStreamWaitEvent(s, aux->ev[2 + (r & 1)], 0)) != hipSuccess) return e;
            if ((e = fw::launch_phase4<T>(D, L, path, ld, r, cfg, P4Mode::rest, s)) != hipSuccess) return e;
            if ((e = hipEventRecord(aux->ev[r & 1], s)) != hipSuccess) return e;
            // auxiliary stream: block row / column r + 1, then phases 1-3 of round r + 1
            if (r > 0 && (e = hipStreamWaitEvent(a, aux->ev[(r - 1) & 1], 0)) != hipSuccess) return e;
            if ((e = fw::launch_phase4<T>(D, L, path, ld, r, cfg, P4Mode::cross, a)) != hipSuccess) return e;
            if ((e = fw::launch_phase123<T>(D, P, L, ld, r + 1, cfg.block, a)) != hipSuccess) return e;
            if ((e = hipEventRecord(aux->ev[2 + ((r + 1) & 1)], a)) != hipSuccess) return e;
        }
        // last round: one launch on the main stream, after everything on the auxiliary one
        if ((e = hipStreamWaitEvent(s, aux->ev[2 + ((R - 1) & 1)], 0)) != hipSuccess) return e;
        return fw::launch_phase4<T>(D, L, path, ld, R - 1, cfg, P4Mode::all, s);
    };
    e = body();
    release_aux(aux);
    return e;
}

// Test hook (fw_debug_fail_next): the next call of the named entry point
// returns an injected error right after its scratch allocations, through the
// same clean-up path as a real failure.
std::atomic<int> g_fail_next{0};
bool take_injected_failure(int where) {
    int expect = where;
    return where != 0 && g_fail_next.compare_exchange_strong(expect, 0);
}

// Stream-ordered scratch of one call, freed on the caller's stream on every
// return path (hipFreeAsync is ordered after the launches that use it).
struct StreamScratch {
    hipStream_t s;
    void *p[2] = {nullptr, nullptr};
    explicit StreamScratch(hipStream_t st) : s(st) {}
    hipError_t alloc(int slot, size_t bytes) { return hipMallocAsync(&p[slot], bytes, s); }
    hipError_t release() {
        hipError_t first = hipSuccess;
        for (void *&q : p) {
            if (!q) continue;
            hipError_t e = hipFreeAsync(q, s);
            if (first == hipSuccess) first = e;
            q = nullptr;
        }
        return first;
    }
    ~StreamScratch() { (void)release(); }
};

template <typename T>
fw_status_t run_apsp(int64_t n, T *dist, int32_t *path, fw::TileCfg cfg, hipStream_t s) {
    if (!fw::config_supported<T>(cfg))
        return fail(FW_EUNSUPPORTED, "block %d / tile %d x %d / variant %d not compiled in", cfg.block, cfg.tile_m,
                    cfg.tile_n, cfg.variant);
    const int64_t unit = std::max(cfg.block, std::max(cfg.tile_m, cfg.tile_n));  // powers of two
    const int64_t npad = (n + unit - 1) / unit * unit;
    const bool aligned = ((uintptr_t)dist % 16 == 0) && (path == nullptr || (uintptr_t)path % 16 == 0);
    hipError_t e;
    T *D = dist;
    int32_t *P = path;
    StreamScratch scr(s);  // [0] padded copies, [1] path-mode marks and transpose
    const bool padded = npad != n || !aligned;
    if (padded) {
        const size_t dbytes = (size_t)(npad * npad) * sizeof(T);
        const size_t pbytes = path ? (size_t)(npad * npad) * sizeof(int32_t) : 0;
        if ((e = scr.alloc(0, dbytes + pbytes)) != hipSuccess)
            return fail(FW_ENOMEM, "scratch of %zu bytes: %s", dbytes + pbytes, hipGetErrorString(e));
        D = (T *)scr.p[0];
        P = path ? (int32_t *)((char *)scr.p[0] + dbytes) : nullptr;
    }
    // Path mode scratch: pending marks L (uint16, zeroed), then the transpose of
    // D for the label resolution.
    uint16_t *L = nullptr;
    const size_t lbytes = (size_t)(npad * npad) * sizeof(uint16_t), tbytes = (size_t)(npad * npad) * sizeof(T);
    if (P) {
        if ((e = scr.alloc(1, lbytes + tbytes)) != hipSuccess)
            return fail(FW_ENOMEM, "label scratch of %zu bytes: %s", lbytes + tbytes, hipGetErrorString(e));
        L = (uint16_t *)scr.p[1];
    }
    if (take_injected_failure(1)) return fail(FW_EHIP, "injected failure after the scratch allocations");
    if (padded && (e = fw::launch_pad_in<T>(dist, n, D, npad, s)) != hipSuccess) return hip_fail(e, "pad");
    if (P && (e = fw::launch_fill_i32(P, npad * npad, -1, s)) != hipSuccess) return hip_fail(e, "path init");
    if (L && (e = fw::launch_fill_i32((int32_t *)L, npad * npad / 2, 0, s)) != hipSuccess)
        return hip_fail(e, "mark init");
    if ((e = run_rounds<T>(D, P, L, npad, cfg, s)) != hipSuccess) return hip_fail(e, "round launch");
    if (P && (e = fw::launch_resolve<T>(D, (T *)((char *)scr.p[1] + lbytes), L, P, npad, cfg.block, s)) != hipSuccess)
        return hip_fail(e, "label resolution");
    if (padded) {
        if ((e = fw::launch_pad_out<T>(D, npad, dist, n, s)) != hipSuccess) return hip_fail(e, "unpad");
        if (path && (e = fw::launch_pad_out<int32_t>(P, npad, path, n, s)) != hipSuccess) return hip_fail(e, "unpad P");
    }
    if ((e = scr.release()) != hipSuccess) return hip_fail(e, "scratch free");
    return FW_OK;
}

// dt codes accepted by the single-graph entry points (and, when two_only, by
// the ones that have no binary16 form).
fw_status_t check_dtype(fw_dtype_t dt, bool two_only) {
    if (dt == FW_F32 || dt == FW_F64) return FW_OK;
    if (dt == FW_F16 && !two_only) return FW_OK;
    if (dt == FW_F16) return fail(FW_EINVAL, "FW_F16 is supported by fw_apsp / fw_apsp_config only");
    return fail(FW_EINVAL, "unknown dtype %d", (int)dt);
}

fw_status_t check_common(fw_dtype_t dt, int64_t n, const void *dist, bool two_only) {
    if (fw_status_t st = check_dtype(dt, two_only); st != FW_OK) return st;
    if (n < 1 || n > kMaxN) return fail(FW_EINVAL, "n = %lld outside [1, %lld]", (long long)n, (long long)kMaxN);
    if (dist == nullptr) return fail(FW_EINVAL, "dist is NULL");
    return FW_OK;
}

}  // namespace

namespace fw {
TileCfg tuned_config(int dtype, bool path, int64_t n) {
    for (const TuneEntry &t : kTuneApsp)
        if (t.dtype == dtype && t.path == (int)path && n >= t.n_lo && n < t.n_hi)
            return {t.block, t.tile_m, t.tile_n, t.variant, t.schedule};
    if (dtype == FW_F16) return {64, 64, 128, FW_VARIANT_PANELS, FW_SCHEDULE_SERIAL};
    return {64, 64, 64, FW_VARIANT_PANELS, FW_SCHEDULE_SERIAL};
}
BatchedTiles tuned_batched_tiles(bool f64, bool path) {
    for (const TuneBatchedEntry &t : kTuneBatched)
        if (t.dtype == (f64 ? FW_F64 : FW_F32) && t.path == (int)path) return {0, (uint64_t)t.tile64};
    // untuned: 64-tiles above 768 vertices, and above 64 wherever they pad no
    // further than 32-tiles
    return {0, 0xFFFFFFFFFFAAAAA8ull};
}

void prof_begin_p4(hipStream_t s) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_pending = take_event();
    if (g_pending) (void)hipEventRecord(g_pending, s);
}
void prof_end_p4(hipStream_t s, int64_t updates) {
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_pending) return;
    hipEvent_t e = take_event();
    if (!e) return;
    (void)hipEventRecord(e, s);
    g_ev_used.push_back({g_pending, e, updates});
    g_pending = nullptr;
}
}  // namespace fw

extern "C" {

fw_status_t fw_apsp_config(fw_dtype_t dt, int64_t n, void *dist, int32_t *path, const fw_config_t *cfg, void *stream) {
    g_err[0] = 0;
    fw_status_t st = check_common(dt, n, dist, false);
    if (st != FW_OK) return st;
    fw::TileCfg tc = default_cfg(dt, n, path != nullptr);
    if (cfg) {
        if (cfg->block < 0 || cfg->tile_m < 0 || cfg->tile_n < 0 || cfg->variant < 0 ||
            cfg->variant > FW_P4_WAVEROWS || cfg->schedule < 0 || cfg->schedule > FW_SCHED_PAIRS_LOOKAHEAD)
            return fail(FW_EINVAL, "config fields must be 0 (tuned) or positive, variant at most %d, schedule at most %d",
                        FW_P4_WAVEROWS, FW_SCHED_PAIRS_LOOKAHEAD);
        if (cfg->block) tc.block = cfg->block;
        if (cfg->tile_m) tc.tile_m = cfg->tile_m;
        if (cfg->tile_n) tc.tile_n = cfg->tile_n;
        if (cfg->variant) tc.variant = cfg->variant;
        if (cfg->schedule) tc.schedule = cfg->schedule;
    }
    if (!supported_for(dt, tc))
        return fail(FW_EUNSUPPORTED, "block %d / tile %d x %d / variant %d not compiled in", tc.block, tc.tile_m,
                    tc.tile_n, tc.variant);
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipStream_t s = (hipStream_t)stream;
    if (dt == FW_F32) return run_apsp<float>(n, (float *)dist, path, tc, s);
    if (dt == FW_F16) return run_apsp<_Float16>(n, (_Float16 *)dist, path, tc, s);
    return run_apsp<double>(n, (double *)dist, path, tc, s);
}

fw_status_t fw_query_config(fw_dtype_t dt, int64_t n, int32_t path, fw_config_t *out) {
    g_err[0] = 0;
    if (fw_status_t st = check_dtype(dt, false); st != FW_OK) return st;
    if (n < 1 || n > kMaxN) return fail(FW_EINVAL, "n = %lld outside [1, %lld]", (long long)n, (long long)kMaxN);
    if (!out) return fail(FW_EINVAL, "out is NULL");
    const fw::TileCfg c = default_cfg(dt, n, path != 0);
    out->block = c.block;
    out->tile_m = c.tile_m;
    out->tile_n = c.tile_n;
    out->variant = c.variant;
    out->schedule = c.schedule;
    return FW_OK;
}

int32_t fw_list_configs(fw_dtype_t dt, fw_config_t *out, int32_t cap) {
    g_err[0] = 0;
    if (fw_status_t st = check_dtype(dt, false); st != FW_OK) return st;
    if (cap < 0 || (cap > 0 && !out)) return fail(FW_EINVAL, "out must hold cap >= 0 entries");
    auto list = [dt](fw::TileCfg *o, int c) {
        return dt == FW_F32 ? fw::list_configs<float>(o, c)
                            : dt == FW_F64 ? fw::list_configs<double>(o, c) : fw::list_configs<_Float16>(o, c);
    };
    std::vector<fw::TileCfg> all((size_t)list(nullptr, 0));
    const int total = list(all.data(), (int)all.size());
    for (int k = 0; k < total && k < cap; ++k) out[k] = {all[k].block, all[k].tile_m, all[k].tile_n, all[k].variant, 0};
    return total;
}

int64_t fw_ooc_superblock(fw_dtype_t dt, int64_t n, int32_t path, size_t device_bytes) {
    g_err[0] = 0;
    if (fw_status_t st = check_dtype(dt, true); st != FW_OK) return st;
    if (n < 1 || n > kMaxN) return fail(FW_EINVAL, "n = %lld outside [1, %lld]", (long long)n, (long long)kMaxN);
    if (device_bytes == 0) {
        size_t free_b = 0, total_b = 0;
        hipError_t e = hipMemGetInfo(&free_b, &total_b);
        if (e != hipSuccess) return hip_fail(e, "hipMemGetInfo");
        device_bytes = free_b / 10 * 9;
    }
    const size_t es = dt == FW_F32 ? 4 : 8;
    constexpr int64_t unit = 256;
    for (int64_t S = (n + unit - 1) / unit * unit; S >= unit; S -= unit)
        if (fw::ooc_working_bytes(n, S, es, path != 0) <= device_bytes) return S;
    return fail(FW_ENOMEM, "%zu device bytes hold no working set for n = %lld (need %zu for 256-vertex super-blocks)",
                device_bytes, (long long)n, fw::ooc_working_bytes(n, unit, es, path != 0));
}

fw_status_t fw_apsp_ooc(fw_dtype_t dt, int64_t n, void *dist_host, int32_t *path_host, size_t device_bytes,
                        void *stream) {
    g_err[0] = 0;
    fw_status_t st = check_common(dt, n, dist_host, true);
    if (st != FW_OK) return st;
    const int64_t S = fw_ooc_superblock(dt, n, path_host != nullptr, device_bytes);
    if (S < 0) return (fw_status_t)S;
    const char *what = "";
    hipError_t e = dt == FW_F32 ? fw::run_ooc<float>(n, (float *)dist_host, path_host, S, (hipStream_t)stream, &what)
                                : fw::run_ooc<double>(n, (double *)dist_host, path_host, S, (hipStream_t)stream, &what);
    if (e != hipSuccess) return hip_fail(e, what);
    return FW_OK;
}

fw_status_t fw_validate_input(fw_dtype_t dt, int64_t n, const void *dist, void *stream) {
    g_err[0] = 0;
    if (fw_status_t st = check_common(dt, n, dist, false); st != FW_OK) return st;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipStream_t s = (hipStream_t)stream;
    StreamScratch scr(s);
    if ((e = scr.alloc(0, sizeof(unsigned long long))) != hipSuccess)
        return fail(FW_ENOMEM, "validation word: %s", hipGetErrorString(e));
    unsigned long long *first = (unsigned long long *)scr.p[0];
    e = dt == FW_F32 ? fw::launch_validate<float>((const float *)dist, n, first, s)
                     : dt == FW_F64 ? fw::launch_validate<double>((const double *)dist, n, first, s)
                                    : fw::launch_validate<_Float16>((const _Float16 *)dist, n, first, s);
    if (e != hipSuccess) return hip_fail(e, "validation launch");
    unsigned long long idx = 0;
    if ((e = hipMemcpyAsync(&idx, first, sizeof idx, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_fail(e, "validation read-back");
    if ((e = scr.release()) != hipSuccess) return hip_fail(e, "validation word free");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "validation wait");
    if (idx == ~0ull) return FW_OK;
    const size_t es = dt == FW_F32 ? 4 : dt == FW_F64 ? 8 : 2;
    unsigned char raw[8] = {};
    if ((e = hipMemcpy(raw, (const char *)dist + idx * es, es, hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "validation entry read-back");
    double v = 0.0;
    if (dt == FW_F32) v = *(float *)raw;
    if (dt == FW_F64) v = *(double *)raw;
    if (dt == FW_F16) v = (double)*(_Float16 *)raw;
    const long long i = (long long)(idx / (unsigned long long)n), j = (long long)(idx % (unsigned long long)n);
    return fail(FW_EINPUT, "entry (%lld, %lld) = %g: %s", i, j, v,
                v != v ? "NaN" : (i == j ? "diagonal entry is not 0" : "negative weight"));
}

fw_status_t fw_apsp(fw_dtype_t dt, int64_t n, void *dist, int32_t *path, void *stream) {
    return fw_apsp_config(dt, n, dist, path, nullptr, stream);
}

fw_status_t fw_apsp_batched_config(fw_dtype_t dt, int32_t batch, const int32_t *n_host, const int64_t *off_host,
                                   void *dist, int32_t *path, const fw_batched_config_t *cfg, void *stream) {
    g_err[0] = 0;
    if (cfg && (cfg->reserved1 || cfg->reserved2)) return fail(FW_EINVAL, "reserved config fields must be 0");
    if (cfg && cfg->route < -1) return fail(FW_EINVAL, "route = %d < -1", cfg->route);
    if (fw_status_t st = check_dtype(dt, true); st != FW_OK) return st;
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
    const fw::BatchedTiles tiles = (cfg && cfg->small_max_n >= 0) ? fw::BatchedTiles{cfg->small_max_n, ~0ull}
                                                                  : fw::tuned_batched_tiles(dt == FW_F64, path != nullptr);
    int cus = 0;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return hip_fail(e, "CU count");
    const bool p = path != nullptr;
    const int occ = dt == FW_F32 ? fw::batched_occupancy<float>(p) : fw::batched_occupancy<double>(p);
    // Graphs far above their share of the work go to fw_apsp (the whole GPU
    // per graph), one after another on the same stream, before the launch.
    std::vector<uint8_t> routed((size_t)batch);
    fw::batched_route(n_host, batch, (int64_t)cus * occ, cfg ? cfg->route : 0, routed.data());
    const size_t esize = dt == FW_F32 ? sizeof(float) : sizeof(double);
    std::vector<int32_t> order;
    order.reserve((size_t)batch);
    for (int32_t b = 0; b < batch; ++b) {
        if (!routed[(size_t)b]) {
            order.push_back(b);
            continue;
        }
        if (fw_status_t st = fw_apsp_config(dt, n_host[b], (char *)dist + off_host[b] * esize,
                                            path ? path + off_host[b] : nullptr, nullptr, stream);
            st != FW_OK)
            return st;
    }
    g_err[0] = 0;
    if (order.empty()) return FW_OK;
    const int32_t njobs = (int32_t)order.size();
    // Queue in order of decreasing n (longest job first); counter slot first.
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return n_host[x] > n_host[y]; });
    const size_t words = 2 + 2 * (size_t)njobs, bytes = words * sizeof(int64_t);
    StreamScratch scr(s);
    if ((e = scr.alloc(0, bytes)) != hipSuccess)
        return fail(FW_ENOMEM, "job table of %zu bytes: %s", bytes, hipGetErrorString(e));
    void *djobs = scr.p[0];
    if (take_injected_failure(2)) return fail(FW_EHIP, "injected failure after the job table allocation");
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
        tab[1] = njobs;
        for (int32_t q = 0; q < njobs; ++q) {
            tab[2 + 2 * q] = off_host[order[(size_t)q]];
            tab[3 + 2 * q] = n_host[order[(size_t)q]];
        }
        if ((e = hipMemcpyAsync(djobs, g_stage, bytes, hipMemcpyHostToDevice, s)) != hipSuccess) return hip_fail(e, "job upload");
        if (!g_stage_ev && (e = hipEventCreateWithFlags(&g_stage_ev, hipEventDisableTiming)) != hipSuccess)
            return hip_fail(e, "event");
        if ((e = hipEventRecord(g_stage_ev, s)) != hipSuccess) return hip_fail(e, "event record");
    }
    int grid = cus * occ;
    if (grid > njobs) grid = njobs;
    e = dt == FW_F32 ? fw::launch_batched<float>((float *)dist, path, (int64_t *)djobs, tiles, grid, s)
                     : fw::launch_batched<double>((double *)dist, path, (int64_t *)djobs, tiles, grid, s);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    if ((e = scr.release()) != hipSuccess) return hip_fail(e, "job table free");
    return FW_OK;
}

// The device-array form: the job table is built on the device (k_build_jobs)
// into `jobs` (2 + 2*batch int64), then the persistent launch reads it.
static fw_status_t batched_device_common(fw_dtype_t dt, int32_t batch, const int32_t *n_dev, const int64_t *off_dev,
                                         void *dist, int32_t *path, int64_t *jobs, hipStream_t s, int dev) {
    hipError_t e;
    int cus = 0;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return hip_fail(e, "CU count");
    const bool p = path != nullptr;
    const int occ = dt == FW_F32 ? fw::batched_occupancy<float>(p) : fw::batched_occupancy<double>(p);
    const fw::BatchedTiles tiles = fw::tuned_batched_tiles(dt == FW_F64, p);
    int grid = cus * occ;
    if (grid > batch) grid = batch;
    if ((e = fw::launch_build_jobs(n_dev, off_dev, batch, jobs, s)) != hipSuccess) return hip_fail(e, "job table build");
    e = dt == FW_F32 ? fw::launch_batched<float>((float *)dist, path, jobs, tiles, grid, s)
                     : fw::launch_batched<double>((double *)dist, path, jobs, tiles, grid, s);
    if (e != hipSuccess) return hip_fail(e, "batched launch");
    return FW_OK;
}

static fw_status_t batched_device_check(fw_dtype_t dt, int32_t batch, const int32_t *n_dev, const int64_t *off_dev,
                                        const void *dist, int *dev) {
    if (fw_status_t st = check_dtype(dt, true); st != FW_OK) return st;
    if (batch < 1) return fail(FW_EINVAL, "batch = %d < 1", batch);
    if (!n_dev || !off_dev || !dist) return fail(FW_EINVAL, "NULL argument");
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    return FW_OK;
}

fw_status_t fw_apsp_batched_device(fw_dtype_t dt, int32_t batch, const int32_t *n_dev, const int64_t *off_dev,
                                   void *dist, int32_t *path, void *stream) {
    g_err[0] = 0;
    int dev = -1;
    if (fw_status_t st = batched_device_check(dt, batch, n_dev, off_dev, dist, &dev); st != FW_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    StreamScratch scr(s);
    const size_t bytes = (2 + 2 * (size_t)batch) * sizeof(int64_t);
    hipError_t e;
    if ((e = scr.alloc(0, bytes)) != hipSuccess)
        return fail(FW_ENOMEM, "job table of %zu bytes: %s", bytes, hipGetErrorString(e));
    if (fw_status_t st = batched_device_common(dt, batch, n_dev, off_dev, dist, path, (int64_t *)scr.p[0], s, dev);
        st != FW_OK)
        return st;
    if ((e = scr.release()) != hipSuccess) return hip_fail(e, "job table free");
    return FW_OK;
}

fw_status_t fw_apsp_batched_device_noalloc(fw_dtype_t dt, int32_t batch, const int32_t *n_dev,
                                           const int64_t *off_dev, void *dist, int32_t *path, void *stream) {
    g_err[0] = 0;
    int dev = -1;
    if (fw_status_t st = batched_device_check(dt, batch, n_dev, off_dev, dist, &dev); st != FW_OK) return st;
    if (batch > fw::kNoAllocMaxBatch)
        return fail(FW_EINVAL, "batch = %d above the %d graphs the static job table holds", batch,
                    fw::kNoAllocMaxBatch);
    int64_t *jobs = nullptr;
    hipError_t e = fw::noalloc_jobs(dev, &jobs);
    if (e != hipSuccess) return hip_fail(e, "job table address (hipGetSymbolAddress)");
    return batched_device_common(dt, batch, n_dev, off_dev, dist, path, jobs, (hipStream_t)stream, dev);
}

fw_status_t fw_apsp_batched(fw_dtype_t dt, int32_t batch, const int32_t *n_host, const int64_t *off_host, void *dist,
                            int32_t *path, void *stream) {
    return fw_apsp_batched_config(dt, batch, n_host, off_host, dist, path, nullptr, stream);
}

fw_status_t fw_apsp_backward(fw_dtype_t dt, int64_t n, int32_t batch, const void *dist, const int32_t *path,
                             const void *grad_dist, void *grad_w, void *stream) {
    g_err[0] = 0;
    if (fw_status_t st = check_dtype(dt, true); st != FW_OK) return st;
    if (n < 1 || n > kMaxBackwardN) return fail(FW_EINVAL, "n = %lld outside [1, %d]", (long long)n, kMaxBackwardN);
    if (batch < 1 || batch > 65535) return fail(FW_EINVAL, "batch = %d outside [1, 65535]", batch);
    if (!dist || !path || !grad_dist || !grad_w) return fail(FW_EINVAL, "NULL argument (path is required)");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipStream_t s = (hipStream_t)stream;
    StreamScratch scr(s);
    const size_t bytes = fw::backward_scratch_bytes((int)n, batch);
    if ((e = scr.alloc(0, bytes)) != hipSuccess)
        return fail(FW_ENOMEM, "backward scratch of %zu bytes: %s", bytes, hipGetErrorString(e));
    e = dt == FW_F32 ? fw::launch_backward<float>((const float *)dist, path, (const float *)grad_dist,
                                                  (float *)grad_w, (int)n, batch, scr.p[0], s)
                     : fw::launch_backward<double>((const double *)dist, path, (const double *)grad_dist,
                                                   (double *)grad_w, (int)n, batch, scr.p[0], s);
    if (e != hipSuccess) return hip_fail(e, "backward launch");
    if ((e = scr.release()) != hipSuccess) return hip_fail(e, "backward scratch free");
    return FW_OK;
}

const char *fw_status_string(int st) {
    switch (st) {
    case FW_OK: return "ok";
    case FW_EINVAL: return "invalid argument";
    case FW_ENOMEM: return "out of device memory";
    case FW_EHIP: return "HIP runtime error";
    case FW_EUNSUPPORTED: return "unsupported";
    case FW_EINPUT: return "input outside the contract";
    }
    return "unknown status";
}

const char *fw_last_error(void) { return g_err; }

void fw_debug_fail_next(int where) { g_fail_next.store(where == 1 || where == 2 ? where : 0); }

const char *fw_version(void) { return "fwapsp 0.1 gfx950"; }

// Timing hooks for the benchmark: enable/disable bracketing of last-phase
// launches with events, and read (count, summed milliseconds, summed updates)
// since the last reset.  fw_prof_read synchronizes on the recorded events.
void fw_prof_enable(int on) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
}

int fw_prof_read(int64_t *count, double *total_ms, int64_t *updates, int reset) {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    double tot = 0.0;
    int64_t cnt = 0, upd = 0;
    for (auto &pr : g_ev_used) {
        if (hipEventSynchronize(pr.end) != hipSuccess) return FW_EHIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, pr.begin, pr.end) != hipSuccess) return FW_EHIP;
        tot += ms;
        upd += pr.updates;
        ++cnt;
    }
    if (count) *count = cnt;
    if (total_ms) *total_ms = tot;
    if (updates) *updates = upd;
    if (reset) {
        for (auto &pr : g_ev_used) {
            g_ev_pool.push_back(pr.begin);
            g_ev_pool.push_back(pr.end);
        }
        g_ev_used.clear();
    }
    return FW_OK;
}

}  // extern "C"
