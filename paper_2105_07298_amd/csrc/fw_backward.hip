// fw_backward.hip -- gradient of a loss L(D) with respect to the weights W,
// from the forward outputs (D, P) and G = dL/dD, with no per-k record.
//
// D is piecewise linear in W: D[i][j] is the sum of the weights on the path P
// encodes for (i, j), so dD[i][j]/dW[u][v] is 1 when edge u->v lies on that
// path and 0 otherwise, and dL/dW[u][v] = sum of G[i][j] over the pairs whose
// path uses u->v.  For a fixed source i the encoded paths form a tree rooted at
// i: the path to j is the path to pred_i(j) followed by the edge
// pred_i(j) -> j.  Hence, with S(j) = G[i][j] + sum of S over j's children,
// source i contributes S(j) to dL/dW[pred_i(j)][j] for every j it reaches.
//
// k_backward_tree, one workgroup per (graph, source i):
//   1. pred_i(j): the last edge of path(i, j) is the last edge of
//      path(P[i][j], j), so follow a <- P[a][j] from a = i while it is >= 0; the
//      vertex reached is pred_i(j).
//   2. depth_i(j) (edges on the path): depth of pred_i(j) plus one, settled
//      level by level.
//   3. subtree sums, deepest level first, by the first wave alone: a level's
//      vertices are taken 64 at a time in increasing order; within such a
//      group the lanes that share a parent are summed in lane order by the
//      lowest of them, which adds that sum to the parent's (double, in LDS).
//      A level is complete before the next shallower one starts, and every
//      addition happens in an order fixed by the vertex numbers.
//   4. row i of two scratch matrices: U[i][j] = pred_i(j) (-1 where source i
//      contributes nothing to column j) and S[i][j] = S(j) in double.
// k_backward_columns, one wave per (graph, column j): dL/dW[u][j] is the sum of
// S[i][j] over the sources i with U[i][j] = u.  The wave takes the sources 64 at
// a time; lanes with equal u are summed in lane order by the lowest of them,
// which then adds the group's sum to an LDS accumulator per u.  Every addition
// happens in an order fixed by (i, lane), so the gradient is the same bit for
// bit from run to run (no atomics), and it is accumulated in double before the
// one rounding to T.
#include "fw_internal.h"

namespace fw {
namespace {

constexpr int NT = 256;

template <typename T> __device__ __forceinline__ T inf_w();
template <> __device__ __forceinline__ float inf_w<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double inf_w<double>() { return __builtin_inf(); }

// LDS layout (dynamic): S double[n], pred int16[n], depth int16[n].
template <typename T>
__global__ void __launch_bounds__(NT) k_backward_tree(const T *__restrict__ D, const int32_t *__restrict__ P,
                                                     const T *__restrict__ G, int16_t *__restrict__ U,
                                                     double *__restrict__ SV, int n) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    double *S = (double *)lds;
    int16_t *pred = (int16_t *)(S + n);
    int16_t *depth = pred + n;
    __shared__ int s_changed;
    const int i = blockIdx.x;
    const int64_t base = (int64_t)blockIdx.y * n * n;
    const T *Drow = D + base + (int64_t)i * n;
    const T *Grow = G + base + (int64_t)i * n;
    const int32_t *Pg = P + base;
    constexpr int16_t UNSET = -1, NONE = -2;

    // 1. predecessor of every reachable j (the chain has at most n links for a
    //    valid path matrix; a longer one, or a label outside [-1, n), is
    //    treated as unreachable).
    for (int j = threadIdx.x; j < n; j += NT) {
        int16_t pr = -1, dp = NONE;
        double s = 0.0;
        if (j != i && Drow[j] != inf_w<T>()) {
            int a = i, steps = 0;
            int32_t m = Pg[(int64_t)a * n + j];
            while (m >= 0 && m < n && steps < n) {
                a = m;
                m = Pg[(int64_t)a * n + j];
                ++steps;
            }
            if (m == -1) {
                pr = (int16_t)a;
                dp = UNSET;
                s = (double)Grow[j];
            }
        }
        if (j == i) dp = 0;
        pred[j] = pr;
        depth[j] = dp;
        S[j] = s;
    }
    __syncthreads();
    // 2. depths, one level per pass.  The flag is read into a register and a
    //    barrier separates that read from the next pass's reset, so every wave
    //    sees the same value and leaves the loop at the same level.
    int maxd = 0;
    for (int lev = 1;; ++lev) {
        if (threadIdx.x == 0) s_changed = 0;
        __syncthreads();
        for (int j = threadIdx.x; j < n; j += NT) {
            if (depth[j] == UNSET && depth[pred[j]] == lev - 1) {
                depth[j] = (int16_t)lev;
                s_changed = 1;
            }
        }
        __syncthreads();
        const int changed = s_changed;
        __syncthreads();
        if (!changed) {
            maxd = lev - 1;
            break;
        }
    }
    // 3. subtree sums from the deepest level up (level-1 vertices hang off i,
    //    whose own sum is not needed).  One wave: its LDS accesses take effect
    //    in program order, so a level's additions are seen by the next level.
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        for (int lev = maxd; lev >= 2; --lev) {
            for (int j0 = 0; j0 < n; j0 += 64) {
                const int j = j0 + lane;
                const bool on = j < n && depth[j] == lev;
                uint64_t mask = __ballot(on);
                if (mask == 0) continue;
                const int par = on ? (int)pred[j] : -1;
                const double s = on ? S[j] : 0.0;
                const uint64_t sb = __builtin_bit_cast(uint64_t, s);
                const int slo = (int)(uint32_t)sb, shi = (int)(uint32_t)(sb >> 32);
                double sum = 0.0;
                bool leader = on;
                while (mask) {
                    const int l = __builtin_ctzll(mask);
                    mask &= mask - 1;
                    const int pl = __builtin_amdgcn_readlane(par, l);
                    const uint64_t bl = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(shi, l) << 32) |
                                        (uint32_t)__builtin_amdgcn_readlane(slo, l);
                    const bool same = pl == par;
                    sum += same ? __builtin_bit_cast(double, bl) : 0.0;
                    leader = leader && !(same && l < lane);
                }
                if (on && leader) S[par] += sum;  // one leader per parent in this group
            }
        }
    }
    __syncthreads();
    // 4. this source's row of the (pred, subtree sum) scratch.
    const int64_t row = base + (int64_t)i * n;
    for (int j = threadIdx.x; j < n; j += NT) {
        U[row + j] = depth[j] >= 1 ? pred[j] : (int16_t)-1;
        SV[row + j] = S[j];
    }
}

// One wave per (graph, column j); LDS: acc double[n], owner int16[n].  Consecutive workgroups
// are dispatched round-robin over the 8 XCDs, so workgroup x takes column
// (x mod 8) * per + x / 8: each XCD walks a contiguous range of columns, whose
// strided reads of U and S share cache lines in that XCD's L2.
template <typename T>
__global__ void __launch_bounds__(64) k_backward_columns(const int16_t *__restrict__ U, const double *__restrict__ SV,
                                                        T *__restrict__ gW, int n, int per) {
    extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
    double *acc = (double *)lds;
    int16_t *owner = (int16_t *)(acc + n);
    const int x = blockIdx.x;
    const int j = (x % 8) * per + x / 8;
    if (j >= n) return;
    const int lane = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.y * n * n;
    for (int u = lane; u < n; u += 64) acc[u] = 0.0;
    __syncthreads();
    for (int i0 = 0; i0 < n; i0 += 64) {
        const int i = i0 + lane;
        int u = -1;
        double s = 0.0;
        if (i < n) {
            u = U[base + (int64_t)i * n + j];
            s = SV[base + (int64_t)i * n + j];
        }
        // Fast path: when no two lanes of this group share a predecessor, every
        // acc[u] gets at most one addition from the group, so the order is fixed
        // without the lane loop.  A clash is detected by every lane writing its
        // number to owner[u] and reading it back (one wave: the read follows the
        // write); whichever lane's write lands, a lane that shares u with another
        // reads a number not its own.
        if (u >= 0) owner[u] = (int16_t)lane;
        // The read must go to LDS (another lane may have written the same word):
        // the compiler barrier keeps it from being forwarded from this lane's
        // own store.  LDS instructions of one wave complete in order.
        asm volatile("" ::: "memory");
        const bool clash = u >= 0 && owner[u] != (int16_t)lane;
        if (__ballot(clash) == 0) {
            if (u >= 0) acc[u] += s;
            continue;
        }
        const uint64_t sb = __builtin_bit_cast(uint64_t, s);
        const int slo = (int)(uint32_t)sb, shi = (int)(uint32_t)(sb >> 32);
        double sum = 0.0;
        bool leader = true;
#pragma unroll 8
        for (int l = 0; l < 64; ++l) {
            const int ul = __builtin_amdgcn_readlane(u, l);
            const uint64_t bl = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(shi, l) << 32) |
                                (uint32_t)__builtin_amdgcn_readlane(slo, l);
            const bool same = ul == u;
            sum += same ? __builtin_bit_cast(double, bl) : 0.0;
            leader = leader && !(same && l < lane);
        }
        if (leader && u >= 0) acc[u] += sum;  // one leader per u in this group of sources
    }
    for (int u = lane; u < n; u += 64) gW[base + (int64_t)u * n + j] = (T)acc[u];
}

}  // namespace

template <typename T>
hipError_t launch_backward(const T *D, const int32_t *P, const T *G, T *gW, int n, int batch, void *scratch,
                           hipStream_t s) {
    int16_t *U = (int16_t *)scratch;
    double *SV = (double *)((char *)scratch + backward_scratch_split(n, batch));
    const size_t lds = (size_t)n * (sizeof(double) + 2 * sizeof(int16_t));
    hipLaunchKernelGGL((k_backward_tree<T>), dim3((unsigned)n, (unsigned)batch), dim3(NT), lds, s, D, P, G, U, SV,
                       n);
    const int per = (n + 7) / 8;
    hipLaunchKernelGGL((k_backward_columns<T>), dim3((unsigned)(8 * per), (unsigned)batch), dim3(64),
                       (size_t)n * (sizeof(double) + sizeof(int16_t)), s, U, SV, gW, n, per);
    return hipGetLastError();
}

template hipError_t launch_backward<float>(const float *, const int32_t *, const float *, float *, int, int, void *,
                                           hipStream_t);
template hipError_t launch_backward<double>(const double *, const int32_t *, const double *, double *, int, int,
                                            void *, hipStream_t);

}  // namespace fw
