// fw_batched.hip -- many independent graphs of uneven size in one persistent
// launch.
//
// Every workgroup loops: take the next job from a device queue (one atomic add
// on a counter), run the whole blocked Floyd-Warshall method (paper Sect. 2.2:
// per block of k, the diagonal block, then its row and column panels, then all
// remaining blocks) on that graph alone, repeat until the queue is empty.  The
// host orders the queue by decreasing n (longest job first), so the largest
// graphs start first and the small ones fill the gaps at the end.
//
// Inside a workgroup a graph is processed TB x TB tile by tile through LDS (TB =
// 32 or 64 per graph, by size, from the tuning table): the
// diagonal block is closed by TB sequential k-steps; panel and remaining tiles
// are min-plus products of two LDS-resident operand tiles with the old tile
// held in registers.  Every step applies the lexicographic label rule
// (length, max(P[i][k], k, P[k][j])), so D and P equal the single-graph result
// (and the classic loop's, for exact weights) whatever TB is.  Graphs are stored
// unpadded (leading dimension n, any offset), so tile loads are guarded: rows
// and columns beyond n read as isolated padding vertices (+inf off the
// diagonal, 0 on it, label -1) and are never written.
#include "fw_internal.h"
#include "fw_lex.h"

namespace fw {
namespace {

constexpr int NT = 256;

template <typename T> __device__ __forceinline__ T inf_b();
template <> __device__ __forceinline__ float inf_b<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double inf_b<double>() { return __builtin_inf(); }

// One graph's tile machinery.  Thread (ty, tx) of the 16 x 16 layout owns rows
// ty + 16*ii and columns tx + 16*jj of a TB x TB tile (RM = TB/16 per side).
template <typename T, int TB, bool PATH>
struct GraphTiles {
    static constexpr int TS = 16, RM = TB / TS, ST = TB + 1;
    T *D;
    int32_t *P;
    int n;

    // Lengths pass through canon() in path mode (lex_take_u's key needs +0.0).
    __device__ T ld_d(int i, int j) const {
        if (i < n && j < n) return PATH ? canon(D[(int64_t)i * n + j]) : D[(int64_t)i * n + j];
        return i == j ? (T)0 : inf_b<T>();
    }
    // Labels are held as label + 1 between load and store.
    __device__ uint32_t ld_p(int i, int j) const {
        return (i < n && j < n) ? (uint32_t)(P[(int64_t)i * n + j] + 1) : 0u;
    }
    // Stage tile (I0, J0) into LDS (values, and labels in path mode).
    __device__ void stage(T *sd, uint32_t *sp, int I0, int J0) const {
        for (int q = threadIdx.x; q < TB * TB; q += NT) {
            const int rr = q / TB, cc = q % TB;
            sd[rr * ST + cc] = ld_d(I0 + rr, J0 + cc);
            if (PATH) sp[rr * ST + cc] = ld_p(I0 + rr, J0 + cc);
        }
    }
    __device__ void load_regs(T (&d)[RM][RM], uint32_t (&p)[RM][RM], int I0, int J0, int tx, int ty) const {
#pragma unroll
        for (int ii = 0; ii < RM; ++ii)
#pragma unroll
            for (int jj = 0; jj < RM; ++jj) {
                d[ii][jj] = ld_d(I0 + ty + TS * ii, J0 + tx + TS * jj);
                if (PATH) p[ii][jj] = ld_p(I0 + ty + TS * ii, J0 + tx + TS * jj);
            }
    }
    __device__ void store_regs(const T (&d)[RM][RM], const uint32_t (&p)[RM][RM], int I0, int J0, int tx,
                               int ty) const {
#pragma unroll
        for (int ii = 0; ii < RM; ++ii)
#pragma unroll
            for (int jj = 0; jj < RM; ++jj) {
                const int i = I0 + ty + TS * ii, j = J0 + tx + TS * jj;
                if (i < n && j < n) {
                    D[(int64_t)i * n + j] = d[ii][jj];
                    if (PATH) P[(int64_t)i * n + j] = (int32_t)p[ii][jj] - 1;
                }
            }
    }
};

template <typename T, bool PATH>
__device__ __forceinline__ void take(T &d, uint32_t &p, T s, uint32_t m) {
    if (PATH)
        lex_take_u(d, p, s, m);
    else
        d = s < d ? s : d;
}

// One graph, whole method, by the calling workgroup.
template <typename T, int TB, bool PATH>
__device__ void solve_graph(GraphTiles<T, TB, PATH> g, T *sa, T *sb, uint32_t *spa, uint32_t *spb) {
    using G = GraphTiles<T, TB, PATH>;
    constexpr int TS = G::TS, RM = G::RM, ST = G::ST;
    const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
    const int n = g.n;
    if (PATH) {
        for (int64_t x = threadIdx.x; x < (int64_t)n * n; x += NT) g.P[x] = -1;
    }
    __syncthreads();
    const int R = (n + TB - 1) / TB;
    T d[RM][RM];
    uint32_t p[RM][RM];
    for (int r = 0; r < R; ++r) {
        const int k0 = r * TB;
        // Phase 1: close the diagonal block in LDS.  Row k and column k do not
        // change at step k (D[k][k] = 0: their candidates equal the current
        // value with a label that is not smaller), so updating in place while
        // others read them is safe; one barrier per k orders the steps.
        g.stage(sa, spa, k0, k0);
        __syncthreads();
        g.load_regs(d, p, k0, k0, tx, ty);
        for (int k = 0; k < TB; ++k) {
            T a[RM], b[RM];
            uint32_t pa[RM], pb[RM];
#pragma unroll
            for (int ii = 0; ii < RM; ++ii) {
                a[ii] = sa[(ty + TS * ii) * ST + k];
                if (PATH) pa[ii] = spa[(ty + TS * ii) * ST + k];
            }
#pragma unroll
            for (int jj = 0; jj < RM; ++jj) {
                b[jj] = sa[k * ST + tx + TS * jj];
                if (PATH) pb[jj] = spa[k * ST + tx + TS * jj];
            }
#pragma unroll
            for (int ii = 0; ii < RM; ++ii)
#pragma unroll
                for (int jj = 0; jj < RM; ++jj) {
                    const T s = a[ii] + b[jj];
                    const uint32_t m = PATH ? max(max(pa[ii], pb[jj]), (uint32_t)(k0 + k + 1)) : 0u;
                    const T d0 = d[ii][jj];
                    const uint32_t p0 = p[ii][jj];
                    take<T, PATH>(d[ii][jj], p[ii][jj], s, m);
                    if (d[ii][jj] != d0 || (PATH && p[ii][jj] != p0)) {
                        sa[(ty + TS * ii) * ST + tx + TS * jj] = d[ii][jj];
                        if (PATH) spa[(ty + TS * ii) * ST + tx + TS * jj] = p[ii][jj];
                    }
                }
            __syncthreads();
        }
        g.store_regs(d, p, k0, k0, tx, ty);
        // The closed diagonal block stays in sa/spa for the panels.
        __syncthreads();
        // Phases 2 and 3: each panel tile is one product with the closed block.
        for (int t = 0; t < 2 * (R - 1); ++t) {
            const bool rowp = t < R - 1;
            const int o0 = rowp ? t : t - (R - 1);
            const int o = o0 < r ? o0 : o0 + 1;
            const int I0 = rowp ? k0 : o * TB, J0 = rowp ? o * TB : k0;
            // the old panel tile goes to sb (it is the B operand of a row panel
            // and the A operand of a column panel)
            g.stage(sb, spb, I0, J0);
            g.load_regs(d, p, I0, J0, tx, ty);
            __syncthreads();
            const T *A = rowp ? sa : sb;
            const T *B = rowp ? sb : sa;
            const uint32_t *PA = rowp ? spa : spb;
            const uint32_t *PB = rowp ? spb : spa;
            for (int k = 0; k < TB; ++k) {
                T a[RM], b[RM];
                uint32_t pa[RM], pb[RM];
#pragma unroll
                for (int ii = 0; ii < RM; ++ii) {
                    a[ii] = A[(ty + TS * ii) * ST + k];
                    if (PATH) pa[ii] = max(PA[(ty + TS * ii) * ST + k], (uint32_t)(k0 + k + 1));
                }
#pragma unroll
                for (int jj = 0; jj < RM; ++jj) {
                    b[jj] = B[k * ST + tx + TS * jj];
                    if (PATH) pb[jj] = PB[k * ST + tx + TS * jj];
                }
#pragma unroll
                for (int ii = 0; ii < RM; ++ii)
#pragma unroll
                    for (int jj = 0; jj < RM; ++jj)
                        take<T, PATH>(d[ii][jj], p[ii][jj], a[ii] + b[jj], PATH ? max(pa[ii], pb[jj]) : 0u);
            }
            g.store_regs(d, p, I0, J0, tx, ty);
            __syncthreads();
        }
        // Phase 4: every other tile, product of its final column-panel and
        // row-panel tiles (staged per tile; the panels are not written here).
        for (int t = 0; t < (R - 1) * (R - 1); ++t) {
            const int bi0 = t / (R - 1), bj0 = t % (R - 1);
            const int bi = bi0 < r ? bi0 : bi0 + 1, bj = bj0 < r ? bj0 : bj0 + 1;
            const int I0 = bi * TB, J0 = bj * TB;
            g.stage(sa, spa, I0, k0);
            g.stage(sb, spb, k0, J0);
            g.load_regs(d, p, I0, J0, tx, ty);
            __syncthreads();
            for (int k = 0; k < TB; ++k) {
                T a[RM], b[RM];
                uint32_t pa[RM], pb[RM];
#pragma unroll
                for (int ii = 0; ii < RM; ++ii) {
                    a[ii] = sa[(ty + TS * ii) * ST + k];
                    if (PATH) pa[ii] = max(spa[(ty + TS * ii) * ST + k], (uint32_t)(k0 + k + 1));
                }
#pragma unroll
                for (int jj = 0; jj < RM; ++jj) {
                    b[jj] = sb[k * ST + tx + TS * jj];
                    if (PATH) pb[jj] = spb[k * ST + tx + TS * jj];
                }
#pragma unroll
                for (int ii = 0; ii < RM; ++ii)
#pragma unroll
                    for (int jj = 0; jj < RM; ++jj)
                        take<T, PATH>(d[ii][jj], p[ii][jj], a[ii] + b[jj], PATH ? max(pa[ii], pb[jj]) : 0u);
            }
            g.store_regs(d, p, I0, J0, tx, ty);
            __syncthreads();
        }
    }
}

// Persistent batched kernel.  jobs[0] holds the queue counter (set to 0 by the
// host copy that uploads the table); jobs[1 + 2q], jobs[2 + 2q] = offset and n
// of queue slot q.  A graph uses 64 x 64 tiles when n > small_max_n (from the
// tuning table) and 64-tiles pad it to no more vertices than 32-tiles would
// (n mod 64 = 0 or > 32); otherwise 32 x 32 tiles.  Both share the LDS arrays,
// sized for 64.
template <typename T, bool PATH>
__global__ void __launch_bounds__(NT) k_batched(T *__restrict__ dist, int32_t *__restrict__ path,
                                               int64_t *__restrict__ jobs, int njobs, int small_max_n) {
    constexpr int ST = 64 + 1;
    __shared__ T sa[64 * ST];
    __shared__ T sb[64 * ST];
    __shared__ uint32_t spa[PATH ? 64 * ST : 1];  // labels + 1
    __shared__ uint32_t spb[PATH ? 64 * ST : 1];
    __shared__ int s_job;
    unsigned long long *counter = (unsigned long long *)jobs;
    for (;;) {
        if (threadIdx.x == 0) s_job = (int)atomicAdd(counter, 1ull);
        __syncthreads();
        const int q = s_job;
        __syncthreads();
        if (q >= njobs) return;
        const int64_t off = jobs[1 + 2 * q];
        const int n = (int)jobs[2 + 2 * q];
        const bool small = (n <= small_max_n) || (((n + 63) & ~63) != ((n + 31) & ~31));
        if (small) {
            GraphTiles<T, 32, PATH> g{dist + off, PATH ? path + off : nullptr, n};
            solve_graph<T, 32, PATH>(g, sa, sb, spa, spb);
        } else {
            GraphTiles<T, 64, PATH> g{dist + off, PATH ? path + off : nullptr, n};
            solve_graph<T, 64, PATH>(g, sa, sb, spa, spb);
        }
    }
}

}  // namespace

template <typename T>
hipError_t launch_batched(T *dist, int32_t *path, int64_t *jobs, int njobs, int small_max_n, int grid,
                          hipStream_t s) {
    if (path)
        hipLaunchKernelGGL((k_batched<T, true>), dim3(grid), dim3(NT), 0, s, dist, path, jobs, njobs, small_max_n);
    else
        hipLaunchKernelGGL((k_batched<T, false>), dim3(grid), dim3(NT), 0, s, dist, path, jobs, njobs, small_max_n);
    return hipGetLastError();
}

template <typename T>
int batched_occupancy(bool path) {
    int nb = 0;
    hipError_t e = path ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batched<T, true>, NT, 0)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batched<T, false>, NT, 0);
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

template int batched_occupancy<float>(bool);
template int batched_occupancy<double>(bool);
template hipError_t launch_batched<float>(float *, int32_t *, int64_t *, int, int, int, hipStream_t);
template hipError_t launch_batched<double>(double *, int32_t *, int64_t *, int, int, int, hipStream_t);

}  // namespace fw
