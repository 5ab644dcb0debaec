// fw_internal.h -- declarations shared by the host runtime and the kernel file.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fw {

// Round depth (the paper's TB) and last-phase output tile (rows x columns, each
// a multiple of the block).
struct TileCfg {
    int block;
    int tile_m;
    int tile_n;
};

// One round of the blocked method, enqueued on `s`.  D, P are the padded
// matrices (leading dimension ld, a multiple of both tile edges); P may be null
// (distances only).  L (path mode) marks entries whose label is pending from a
// round of the last phase (r + 1; 0 = current), zero-initialised.
// Returns hipSuccess or the launch error.
template <typename T>
hipError_t launch_round(T *D, int32_t *P, uint16_t *L, int64_t ld, int r, TileCfg cfg, hipStream_t s);

// Compiled (block, tile_m, tile_n) combinations for element type T.
template <typename T>
bool config_supported(TileCfg cfg);

// Path mode, after the last round: resolve the labels the last phase left
// pending (marked in L).  DT (ld*ld elements) is scratch for the transpose of D.
template <typename T>
hipError_t launch_resolve(const T *D, T *DT, const uint16_t *L, int32_t *P, int64_t ld, int block, hipStream_t s);

// Persistent batched launch (one workgroup per graph at a time).  jobs is a
// device table of 1 + 2*njobs int64: [0] the queue counter (must be 0), then
// (element offset, n) per queue slot in processing order.  Graphs with
// n <= small_max_n, or that 64-tiles would pad further than 32-tiles, use
// 32 x 32 tiles; the others 64 x 64.
template <typename T>
hipError_t launch_batched(T *dist, int32_t *path, int64_t *jobs, int njobs, int small_max_n, int grid,
                          hipStream_t s);

// Workgroups of the batched kernel that fit on one CU at once.
template <typename T>
int batched_occupancy(bool path);

// Tuning table lookup (tune_table.inc): tile configuration for fw_apsp and the
// small-graph split of fw_apsp_batched.
TileCfg tuned_config(bool f64, bool path, int64_t n);
int tuned_batched_small_max_n(bool f64, bool path);

// Gradient dL/dW (zeroed here) from (D, P) and G = dL/dD for batch graphs of n
// vertices each (contiguous, stride n*n), n <= 4096.
template <typename T>
hipError_t launch_backward(const T *D, const int32_t *P, const T *G, T *gW, int n, int batch, hipStream_t s);

// Fill n int32 with v.
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);

// Copy a user matrix (n x n, leading dim n) into a padded one (npad x npad);
// padding entries become +inf off the diagonal and 0 on it.
template <typename T>
hipError_t launch_pad_in(const T *src, int64_t n, T *dst, int64_t npad, hipStream_t s);

// Copy the leading n x n block of a padded matrix back (T = float, double, int32_t).
template <typename T>
hipError_t launch_pad_out(const T *src, int64_t npad, T *dst, int64_t n, hipStream_t s);

// Kernel-class timing hooks (events around the last-phase launches).
void prof_begin_p4(hipStream_t s);
void prof_end_p4(hipStream_t s);

}  // namespace fw
