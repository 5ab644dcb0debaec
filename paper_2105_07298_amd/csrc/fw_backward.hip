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
// One workgroup per (graph, source):
//   1. pred_i(j): the last edge of path(i, j) is the last edge of
//      path(P[i][j], j), so follow a <- P[a][j] from a = i while it is >= 0; the
//      vertex reached is pred_i(j).
//   2. depth_i(j) (edges on the path): depth of pred_i(j) plus one, settled
//      level by level.
//   3. subtree sums, deepest level first: every vertex of a level adds its sum
//      to its parent's (LDS atomics, double); a level is complete before the
//      next shallower one starts.
//   4. scatter S(j) into dL/dW[pred_i(j)][j] with global atomics (sources share
//      edges).  The order of the additions is not fixed, so the last bits of
//      the result may differ between runs.
#include "fw_internal.h"

namespace fw {
namespace {

constexpr int NT = 256;

template <typename T> __device__ __forceinline__ T inf_w();
template <> __device__ __forceinline__ float inf_w<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double inf_w<double>() { return __builtin_inf(); }

template <typename T>
__global__ void k_zero(T *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (T)0;
}

// LDS layout (dynamic): S double[n], pred int16[n], depth int16[n].
template <typename T>
__global__ void __launch_bounds__(NT) k_backward(const T *__restrict__ D, const int32_t *__restrict__ P,
                                                const T *__restrict__ G, T *__restrict__ gW, int n) {
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
    // 3. subtree sums from the deepest level up (level-1 vertices hang off i).
    for (int lev = maxd; lev >= 2; --lev) {
        for (int j = threadIdx.x; j < n; j += NT)
            if (depth[j] == lev) atomicAdd(&S[pred[j]], S[j]);
        __syncthreads();
    }
    // 4. scatter into dL/dW.
    T *gWb = gW + base;
    for (int j = threadIdx.x; j < n; j += NT)
        if (depth[j] >= 1) atomicAdd(&gWb[(int64_t)pred[j] * n + j], (T)S[j]);
}

}  // namespace

template <typename T>
hipError_t launch_backward(const T *D, const int32_t *P, const T *G, T *gW, int n, int batch, hipStream_t s) {
    const int64_t total = (int64_t)n * n * batch;
    int64_t gz = (total + NT - 1) / NT;
    hipLaunchKernelGGL((k_zero<T>), dim3((unsigned)(gz < 8192 ? gz : 8192)), dim3(NT), 0, s, gW, total);
    const size_t lds = (size_t)n * (sizeof(double) + 2 * sizeof(int16_t));
    hipLaunchKernelGGL((k_backward<T>), dim3((unsigned)n, (unsigned)batch), dim3(NT), lds, s, D, P, G, gW, n);
    return hipGetLastError();
}

template hipError_t launch_backward<float>(const float *, const int32_t *, const float *, float *, int, int,
                                           hipStream_t);
template hipError_t launch_backward<double>(const double *, const int32_t *, const double *, double *, int, int,
                                            hipStream_t);

}  // namespace fw
