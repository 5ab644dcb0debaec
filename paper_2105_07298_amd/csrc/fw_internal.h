// fw_internal.h -- declarations shared by the host runtime and the kernel file.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fw_tiles.h"

namespace fw {

// Last-phase kernels: both operand panels in LDS, or one column-panel row per
// wave in scalar registers and the row panel in LDS.
constexpr int FW_VARIANT_PANELS = 1;
constexpr int FW_VARIANT_WAVEROWS = 2;
// Round schedules: one stream, lookahead on an auxiliary stream, rounds in
// pairs, or rounds in pairs with lookahead (fw_plan.h).
constexpr int FW_SCHEDULE_SERIAL = 1;
constexpr int FW_SCHEDULE_LOOKAHEAD = 2;
constexpr int FW_SCHEDULE_PAIRS = 3;
constexpr int FW_SCHEDULE_PAIRS_LOOKAHEAD = 4;

// Round depth (the paper's TB), last-phase output tile (rows x columns),
// last-phase kernel and round schedule.
struct TileCfg {
    int block;
    int tile_m;
    int tile_n;
    int variant;
    int schedule;
};

// Launches of round r of the blocked method, enqueued on `s`.  D, P are the
// padded matrices (leading dimension ld, a multiple of the block and of both
// tile edges); P may be null (distances only).  L (path mode) marks entries
// whose label is pending from a round of the last phase (r + 1; 0 = current),
// zero-initialised.  Each returns hipSuccess or the launch error.
//
// Phases 1-3: the diagonal block of round r, then its row and column panels.
template <typename T>
hipError_t launch_phase123(T *D, int32_t *P, uint16_t *L, int64_t ld, int r, int block, hipStream_t s);

// Phase 4 of round r over a selection of its tiles (P4Mode, in fw_tiles.h).
// cross, rest, crossprev and pair need lookahead_supported(cfg) and a next
// round (crossprev: r >= 1); the pair and *_band / *_rest modes need
// pairs_supported(cfg).
template <typename T>
hipError_t launch_phase4(T *D, uint16_t *L, bool path, int64_t ld, int r, TileCfg cfg, P4Mode mode, hipStream_t s);

// Tiles exactly one block wide and at most one block tall, so that block row
// and column r + 1 are whole tiles.
bool lookahead_supported(TileCfg cfg);

// LDS-panel tiles exactly one block square: the fused pair launch exists.
bool pairs_supported(TileCfg cfg);

// Compiled (block, tile_m, tile_n, variant) combinations for element type T.
template <typename T>
bool config_supported(TileCfg cfg);

// Writes up to cap of them to out (may be null) and returns their number.
template <typename T>
int list_configs(TileCfg *out, int cap);

// Path mode, after the last round: resolve the labels the last phase left
// pending (marked in L).  DT (ld*ld elements) is scratch for the transpose of D.
template <typename T>
hipError_t launch_resolve(const T *D, T *DT, const uint16_t *L, int32_t *P, int64_t ld, int block, hipStream_t s);

// Persistent batched launch (one workgroup per graph at a time).  jobs is a
// device table of 2 + 2*njobs int64: [0] the queue counter (must be 0), [1]
// njobs, then (element offset, n) per queue slot in processing order.  The tile
// of a graph: 32 x 32 when n <= tiles.small_max_n, else by its size class
// c = (n - 1) / 32: 64 x 64 when c >= 64 or bit c of tiles.tile64 is set, 32 x 32
// otherwise.
struct BatchedTiles {
    int small_max_n;
    uint64_t tile64;
};
template <typename T>
hipError_t launch_batched(T *dist, int32_t *path, int64_t *jobs, BatchedTiles tiles, int grid, hipStream_t s);

// The same table built on the device from device arrays nv[batch] (vertex
// counts) and off[batch] (element offsets), ordered by decreasing n; graphs
// with n outside [1, 4096] or a negative offset are left out.  jobs holds
// 2 + 2*batch int64.
hipError_t launch_build_jobs(const int32_t *nv, const int64_t *off, int batch, int64_t *jobs, hipStream_t s);

// Largest batch of fw_apsp_batched_device_noalloc, whose job table is a static
// device array (2 + 2*kNoAllocMaxBatch int64 = 4 MiB per GPU), and that array's
// address on device dev (looked up on the first call with dev current).
constexpr int kNoAllocMaxBatch = 262144;
hipError_t noalloc_jobs(int dev, int64_t **out);

// Workgroups of the batched kernel that fit on one CU at once.
template <typename T>
int batched_occupancy(bool path);

// Tuning table lookup (tune_table.inc): tile configuration for fw_apsp and the
// per-size-class tile choice of fw_apsp_batched.
TileCfg tuned_config(int dtype, bool path, int64_t n);  // dtype: an fw_dtype_t code
BatchedTiles tuned_batched_tiles(bool f64, bool path);

// Gradient dL/dW (every entry written) from (D, P) and G = dL/dD for batch
// graphs of n vertices each (contiguous, stride n*n), n <= 4096.  scratch holds
// backward_scratch_bytes(n, batch) bytes: per (graph, source, column) the
// predecessor (int16) and the subtree sum (double).
inline size_t backward_scratch_split(int n, int batch) {  // bytes of the int16 part, 256-aligned
    return ((size_t)n * n * batch * sizeof(int16_t) + 255) / 256 * 256;
}
inline size_t backward_scratch_bytes(int n, int batch) {
    return backward_scratch_split(n, batch) + (size_t)n * n * batch * sizeof(double);
}
template <typename T>
hipError_t launch_backward(const T *D, const int32_t *P, const T *G, T *gW, int n, int batch, void *scratch,
                           hipStream_t s);

// C <- min(C, A (x) B): C is M x N (leading dimension ldc), A is M x K (lda), B
// is K x N (ldb); M, N, K multiples of 64, pointers and leading dimensions
// 16-byte aligned.  Distances only (no labels).
template <typename T>
hipError_t launch_minplus(T *C, int64_t ldc, const T *A, int64_t lda, const T *B, int64_t ldb, int64_t M, int64_t N,
                          int64_t K, hipStream_t s);

// (C, PC) <- lexicographic minimum with A (x) B carrying labels: candidate k
// has length A[i][k] + B[k][j] and label max(PA[i][k], kbase + k, PB[k][j]).
// M, N multiples of 64, K of 32.
template <typename T>
hipError_t launch_minplus_lex(T *C, int32_t *PC, int64_t ldc, const T *A, const int32_t *PA, int64_t lda, const T *B,
                              const int32_t *PB, int64_t ldb, int64_t M, int64_t N, int64_t K, int32_t kbase,
                              hipStream_t s);

// P[x] <- base + Plocal[x] where Plocal[x] >= 0 (count entries).
hipError_t launch_merge_labels(int32_t *P, const int32_t *Plocal, int64_t count, int32_t base, hipStream_t s);

// rows x cols block (leading dimension ld) set to +inf, with 0 on the diagonal
// if zero_diag (a block of isolated vertices).
template <typename T>
hipError_t launch_fill_blank(T *p, int64_t ld, int64_t rows, int64_t cols, bool zero_diag, hipStream_t s);

// Out of core: distances of the n x n matrix H in host memory, super-blocks of
// edge S (a multiple of 256); returns when H holds the result.  *what names the
// failing step on error.
template <typename T>
hipError_t run_ooc(int64_t n, T *H, int32_t *HP, int64_t S, hipStream_t user, const char **what);
// Device bytes of the working set for super-block edge S (with labels if path).
size_t ooc_working_bytes(int64_t n, int64_t S, size_t es, bool path);

// Fill n int32 with v.
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);

// Copy a user matrix (n x n, leading dim n) into a padded one (npad x npad);
// padding entries become +inf off the diagonal and 0 on it.
template <typename T>
hipError_t launch_pad_in(const T *src, int64_t n, T *dst, int64_t npad, hipStream_t s);

// Copy the leading n x n block of a padded matrix back (T = float, double, int32_t).
template <typename T>
hipError_t launch_pad_out(const T *src, int64_t npad, T *dst, int64_t n, hipStream_t s);

// Input contract check: *first <- the smallest flat index of an entry of the
// n x n matrix D that is NaN, negative, or a non-zero diagonal entry (~0 if none).
template <typename T>
hipError_t launch_validate(const T *D, int64_t n, unsigned long long *first, hipStream_t s);

// Kernel-class timing hooks: events around the last-phase launches of kind
// all / rest, with the algorithmic min-plus updates each performs.
void prof_begin_p4(hipStream_t s);
void prof_end_p4(hipStream_t s, int64_t updates);

}  // namespace fw
