/*
 * fw_apsp.h -- C ABI of the MI355X (gfx950) blocked Floyd-Warshall library.
 *
 * Problem (paper Sect. 2.2, "FW Algorithm"): a dense n x n distance matrix D
 * (D[i][j] = weight of edge i->j, +infinity when there is no edge, 0 on the
 * diagonal) is replaced by the all-pairs shortest distances, and a path matrix
 * P records, for every pair, the intermediate vertex of a shortest path.  The
 * library computes it with the blocked three-phase method of the same section
 * ("Blocked FW Algorithm": diagonal block, then its row and column panels, then
 * every remaining block, for each block of k).
 *
 * Conventions shared by every entry point
 *   - Matrices are row-major with leading dimension n (element (i, j) at i*n + j).
 *   - dist, path, grad_* are DEVICE pointers (hipMalloc'd or torch tensors) owned
 *     by the caller.  Host arrays are marked "host" below.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).  Calls are
 *     asynchronous: results are ready when the stream reaches this point.
 *     Argument errors are reported synchronously before anything is enqueued.
 *   - Input contract: dist[i][i] = 0; off-diagonal weights >= 0 or +inf; no NaN.
 *     Negative weights or cycles are outside the contract (results undefined).
 *   - path[i][j] = -1 when i == j, when j is unreachable from i, or when the direct
 *     edge is a shortest path; otherwise the largest interior vertex of a shortest
 *     path, chosen as the smallest such value over all shortest paths.  This is
 *     what the classic loop with a strict update test stores, and does not depend
 *     on the block size.  For real-valued weights, rounding may resolve
 *     near-ties differently from a float64 computation.
 *   - Return value: FW_OK or a negative fw_status_t; nothing throws.  The text of
 *     the last failure on the calling thread is available from fw_last_error().
 *   - The library allocates stream-ordered scratch (hipMallocAsync) only where an
 *     entry point says so, and frees it on the same stream before returning.
 */
#ifndef FW_APSP_H
#define FW_APSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element type of the distance matrix.  FW_F16 (IEEE binary16, _Float16) is the
 * half-width variant for small integer weights: the last phase updates two
 * entries per packed instruction.  Binary16 holds every integer up to 2048
 * exactly, so when weights are integers (or multiples of one power of two, in
 * units where they are integers) and every finite shortest distance is below
 * 2048 units, D and P equal those of the exact computation; larger lengths are
 * rounded and may change which candidates tie.  FW_F16 is accepted by fw_apsp,
 * fw_apsp_config, fw_query_config and fw_list_configs only (FW_EINVAL
 * elsewhere). */
typedef enum { FW_F32 = 0, FW_F64 = 1, FW_F16 = 2 } fw_dtype_t;

typedef enum {
    FW_OK = 0,
    FW_EINVAL = -1,       /* bad argument (size, pointer, dtype, layout)         */
    FW_ENOMEM = -2,       /* scratch allocation failed                           */
    FW_EHIP = -3,         /* a HIP runtime call failed (no device, launch error) */
    FW_EUNSUPPORTED = -4, /* valid but not supported by this build               */
    FW_EINPUT = -5        /* fw_validate_input: the matrix breaks the contract    */
} fw_status_t;

/*
 * All-pairs shortest paths of one graph, in place (paper Sect. 2.2, Algorithm 1
 * and the blocked method).
 *   dt    FW_F32 (float), FW_F64 (double) or FW_F16 (_Float16): element type
 *         of dist.
 *   n     vertex count, 1 <= n <= 2^20.
 *   dist  device, n*n elements: W on entry, shortest distances on exit.
 *   path  device, n*n int32: receives P; NULL computes distances only.
 * When n is not a multiple of the block size or dist is not 16-byte aligned, the
 * call copies the matrices into padded stream-ordered scratch (padding vertices
 * are isolated, so they change nothing) and back.
 */
fw_status_t fw_apsp(fw_dtype_t dt, int64_t n, void *dist, int32_t *path, void *stream);

/*
 * Checks a weight matrix against the input contract of the problem statement
 * (paper Sect. 2.2: 0 on the diagonal, a weight >= 0 or +inf off it; no NaN),
 * which the other entry points assume without checking (they compute nothing
 * meaningful otherwise: a negative cycle has no shortest path).
 *   dt, n, dist  as for fw_apsp (device, n*n elements, row-major); not modified.
 * Waits for `stream` (the check's launch and its one-word read-back are ordered
 * after earlier work on it).  Returns FW_OK, or FW_EINPUT with the first
 * offending entry in row-major order, its value and the broken rule in
 * fw_last_error().  Allocates one 8-byte stream-ordered word.
 */
fw_status_t fw_validate_input(fw_dtype_t dt, int64_t n, const void *dist, void *stream);

/*
 * Tile configuration of fw_apsp, for tuning and for the tests that show results
 * do not depend on it.
 *   block    round depth (the paper's TB), 32 or 64.
 *   variant  the last-phase kernel:
 *            FW_P4_PANELS    both operand panels staged in LDS; tile_m and
 *                            tile_n each 64 or 128 and a multiple of block
 *                            (FW_F16: tile_n 128 or 256, tile_m 32 to 128).
 *            FW_P4_WAVEROWS  each wave of 4 takes tile_m / 4 rows of the tile
 *                            and reads their column-panel values with scalar
 *                            loads; only the row panel is staged in LDS.
 *                            tile_m divides block; tile_n = 64 x columns per
 *                            lane (64 to 256).
 *   tile_m x tile_n  the output tile one workgroup updates in the last phase.
 *   schedule FW_SCHED_SERIAL: the three phases of each round one after the
 *            other on the caller's stream.  FW_SCHED_LOOKAHEAD (tiles one
 *            block wide, tile_m dividing block, at least 3 rounds; otherwise
 *            serial): block row and column r + 1 of round r's last phase and
 *            then phases 1-3 of round r + 1 run on an auxiliary stream of the
 *            library, concurrently with the rest of round r's last phase on
 *            the caller's stream, which waits for them before round r + 1.
 *            The call stays stream-ordered on the caller's stream.
 *            FW_SCHED_PAIRS (LDS-panel tiles exactly one block square;
 *            otherwise serial, which includes every FW_F16 configuration):
 *            rounds in pairs on the caller's stream; the last phase of both
 *            rounds of a pair is applied to every tile outside their two blocks
 *            in one pass, so those tiles move through memory once per two
 *            rounds.  FW_SCHED_PAIRS_LOOKAHEAD (same tiles, at least 3 rounds;
 *            otherwise serial): the same pairs, with phases 1-3 of the next
 *            pair, the tiles they read and the cross launches on an auxiliary
 *            stream of the library while the caller's stream runs the bulk of
 *            the current pair; stream-ordered on the caller's stream.
 * Fields set to 0 keep the tuned choice (a table of timings on gfx950 per
 * element type, path mode and size range).  The resulting combination must be
 * one the library compiles (fw_apsp_config returns FW_EUNSUPPORTED otherwise).
 */
enum { FW_P4_PANELS = 1, FW_P4_WAVEROWS = 2 };
enum { FW_SCHED_SERIAL = 1, FW_SCHED_LOOKAHEAD = 2, FW_SCHED_PAIRS = 3, FW_SCHED_PAIRS_LOOKAHEAD = 4 };
typedef struct {
    int32_t block;
    int32_t tile_m;
    int32_t tile_n;
    int32_t variant;
    int32_t schedule;
} fw_config_t;

/* fw_apsp with an explicit configuration (cfg may be NULL = library choice).
 * FW_EUNSUPPORTED if the combination is not compiled in. */
fw_status_t fw_apsp_config(fw_dtype_t dt, int64_t n, void *dist, int32_t *path,
                           const fw_config_t *cfg, void *stream);

/* Every (block, tile_m, tile_n, variant) compiled in for dt, with schedule 0
 * (either schedule runs with any of them): writes the first min(cap, count)
 * to out (host memory; may be NULL when cap is 0) and returns count, or
 * FW_EINVAL (negative) for a bad dtype or cap.  Host only; launches nothing. */
int32_t fw_list_configs(fw_dtype_t dt, fw_config_t *out, int32_t cap);

/* The configuration fw_apsp uses for (dt, n, path != 0) -- the tuned table's
 * entry -- written to *out.  Host only; launches nothing. */
fw_status_t fw_query_config(fw_dtype_t dt, int64_t n, int32_t path, fw_config_t *out);

/*
 * All-pairs shortest paths for a matrix larger than the device memory to be
 * used (out of core: the paper leaves this as future work for its GPU runs,
 * where the matrix had to fit in device memory).  dist_host is HOST memory,
 * n*n elements row-major, W on entry and D on exit; path_host (HOST, n*n int32)
 * receives P, or is NULL for distances only.  Pinned memory (hipHostMalloc)
 * lets the transfers overlap the computation.  The blocked method runs over
 * super-blocks of edge S (fw_ooc_superblock): each super-round closes its
 * diagonal super-block in device memory with fw_apsp, updates its row and
 * column bands, updates the next super-round's bands in place on the device,
 * and streams every other S x S super-tile through the device once.  P follows the same lexicographic rule as fw_apsp, so both give the
 * same P for the same D.  device_bytes bounds the device working set (0: 90%
 * of the free memory).  Ordered after earlier work on `stream`; returns when
 * the host arrays hold the result.  FW_ENOMEM if device_bytes cannot hold even
 * 256-vertex super-blocks.
 */
fw_status_t fw_apsp_ooc(fw_dtype_t dt, int64_t n, void *dist_host, int32_t *path_host, size_t device_bytes,
                        void *stream);

/* The super-block edge fw_apsp_ooc uses for (dt, n, path != 0, device_bytes):
 * the largest multiple of 256 whose working set fits -- 4*S^2 + 4*S*ceil(n/S)*S
 * elements (four blocks and two sets of row and column bands), plus as many
 * int32 labels and S^2 more with the path matrix -- or
 * a negative status.  Host only. */
int64_t fw_ooc_superblock(fw_dtype_t dt, int64_t n, int32_t path, size_t device_bytes);

/*
 * Many independent graphs of uneven size in one persistent launch.
 *   batch      number of graphs, >= 1.
 *   n_host     host [batch]: vertex count of each graph, 1 <= n <= 4096.
 *   off_host   host [batch]: element offset of graph b's matrix in dist/path
 *              (graph b occupies n_b*n_b elements from there, row-major).
 *   dist, path device, ragged concatenation; path may be NULL.
 * Same per-graph semantics and results as fw_apsp on each graph.  Allocates a
 * small stream-ordered job table.  In the launch one workgroup solves one
 * graph, so a graph that alone holds much more than its share of the batch's
 * work would finish long after the rest: a graph with n >= 256 whose n^3 is
 * above 4 times the batch's sum of n^3 per resident workgroup is solved by
 * fw_apsp instead, on the same stream, before the launch (see the route field
 * of fw_batched_config_t).
 */
fw_status_t fw_apsp_batched(fw_dtype_t dt, int32_t batch, const int32_t *n_host,
                            const int64_t *off_host, void *dist, int32_t *path, void *stream);

/*
 * Choices of fw_apsp_batched, for tuning and for the tests that show results
 * do not depend on them.
 *   small_max_n  tile choice: k >= 0 processes a graph in 32 x 32 tiles when
 *                n <= k and in 64 x 64 tiles otherwise; -1 keeps the tuned
 *                choice (made per size class of 32 vertices, n in
 *                (32c, 32c + 32], from timings of both tilings; 64 x 64 above
 *                2048 vertices).
 *   route        which graphs fw_apsp solves instead of the persistent launch:
 *                0 the rule given at fw_apsp_batched, -1 none, k > 0 every
 *                graph with n >= k.
 * Reserved fields must be 0.
 */
typedef struct { int32_t small_max_n; int32_t route; int32_t reserved1; int32_t reserved2; } fw_batched_config_t;

/* fw_apsp_batched with explicit choices (cfg may be NULL = tuned tiles, route 0). */
fw_status_t fw_apsp_batched_config(fw_dtype_t dt, int32_t batch, const int32_t *n_host,
                                   const int64_t *off_host, void *dist, int32_t *path,
                                   const fw_batched_config_t *cfg, void *stream);

/*
 * fw_apsp_batched with the vertex counts and offsets in DEVICE memory, for
 * callers whose batch description is produced on the GPU (same per-graph
 * semantics and results, paper Sect. 2.2 per graph).
 *   n_dev    device [batch] int32: vertex count of each graph.
 *   off_dev  device [batch] int64: element offset of each graph in dist / path
 *            (an array of batch + 1 offsets, whose last entry is the end, may be
 *            passed as is; only the first batch entries are read).
 * The device arrays are read by the launches, so they must stay valid until the
 * stream reaches this point.  Their values are not seen by the host: a graph
 * whose n is outside [1, 4096] or whose offset is negative is skipped on the
 * device (left untouched, no error reported).  The queue (ordered by decreasing
 * n) is built on the device into a stream-ordered job table of 16 (batch + 1)
 * bytes.  Every graph runs in the persistent launch (no routing of large
 * graphs to fw_apsp, which needs n on the host).  FW_F32 and FW_F64.
 */
fw_status_t fw_apsp_batched_device(fw_dtype_t dt, int32_t batch, const int32_t *n_dev,
                                   const int64_t *off_dev, void *dist, int32_t *path, void *stream);

/*
 * fw_apsp_batched_device for callers that cannot allocate memory (code under
 * HIP graph capture, tight serving loops): the same launches and results, with
 * the job table in a static device array of the library (one per GPU, 4 MiB,
 * held until the process ends) instead of stream-ordered scratch.  Calls no
 * allocation routine.  batch is at most 262144 (FW_EINVAL above).  Every call on
 * one GPU uses that GPU's one table: calls that overlap on one GPU (different
 * streams, or host threads, without ordering between them) race and must not
 * be issued; calls ordered on one stream are safe (the table is rebuilt by the
 * first launch of each call).
 */
fw_status_t fw_apsp_batched_device_noalloc(fw_dtype_t dt, int32_t batch, const int32_t *n_dev,
                                           const int64_t *off_dev, void *dist, int32_t *path, void *stream);

/*
 * Gradient of a loss L(D) with respect to the weights W, given the forward
 * outputs.  D is piecewise linear in W: dD[i][j]/dW[u][v] = 1 when edge u->v is
 * on the path P encodes for (i, j), else 0 (the subgradient along that path at
 * ties).  Hence grad_w[u][v] = sum of grad_dist[i][j] over the pairs whose path
 * uses u->v, computed per source i as subtree sums over its shortest-path tree.
 *   n, batch   1 <= batch <= 65535 graphs of 1 <= n <= 4096 vertices each,
 *              contiguous with stride n*n.
 *   dist, path forward outputs (device); path must not be NULL.
 *   grad_dist  device, dL/dD (same layout/type as dist).
 *   grad_w     device, output dL/dW (same layout/type), overwritten.
 * Diagonal and unused edges get 0.  Requires positive off-diagonal weights and
 * a path matrix produced by this library for the same dist; a label outside
 * [-1, n) or a chain of labels that does not end within n steps makes the pair
 * count as unreachable (no contribution).  Each source's contributions are
 * summed per column in a fixed order, in double, and rounded once: the result
 * is the same bit for bit on every run.  Allocates stream-ordered scratch of
 * 10 bytes per (graph, source, column).
 */
fw_status_t fw_apsp_backward(fw_dtype_t dt, int64_t n, int32_t batch, const void *dist,
                             const int32_t *path, const void *grad_dist, void *grad_w,
                             void *stream);

/* Static description of a status code. */
const char *fw_status_string(int status);

/* Text of the last failure on the calling thread ("" if none). */
const char *fw_last_error(void);

/* Library version string. */
const char *fw_version(void);

/*
 * Test hook for the error paths.  where = 1: the next fw_apsp / fw_apsp_config
 * call in the process returns FW_EHIP right after allocating its scratch, before
 * launching anything; where = 2: the same for the next fw_apsp_batched /
 * fw_apsp_batched_config call after its job table allocation; 0 clears a pending
 * request.  The call frees its scratch on its stream like any failing call, so
 * later calls on that stream run normally.  Host only; launches nothing.
 */
void fw_debug_fail_next(int where);

/*
 * Timing hooks for benchmarks.  While enabled, every bulk launch of the
 * last-phase kernel (the register-blocked min-plus tile update: each round's
 * whole last phase, or with lookahead its part outside the next round's block
 * row and column) is bracketed by two HIP events recorded on the stream it runs
 * on.  fw_prof_read waits for the recorded events and returns the number of
 * bracketed launches, their summed duration in milliseconds and their summed
 * algorithmic min-plus updates (entries updated x block) since the last reset
 * (reset != 0 starts a new window).  Any output pointer may be NULL.
 */
void fw_prof_enable(int on);
int fw_prof_read(int64_t *count, double *total_ms, int64_t *updates, int reset);

#ifdef __cplusplus
}
#endif

#endif /* FW_APSP_H */
