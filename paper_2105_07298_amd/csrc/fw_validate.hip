// fw_validate.hip -- the input contract of the weight matrix, checked on the
// device: the problem statement (paper Sect. 2.2) has 0 on the diagonal and a
// non-negative weight or +infinity off it; NaN and negative weights are outside
// it (with a negative cycle there is no shortest path at all).
#include "fw_internal.h"

namespace fw {
namespace {

constexpr int NT = 256;

// first[0] <- the smallest flat index i*ld + j (i, j < n) whose entry breaks the
// contract, if smaller than its current value (the host sets it to ~0 first).
template <typename T>
__global__ void __launch_bounds__(NT) k_validate(const T *__restrict__ D, int64_t n, unsigned long long *first) {
    const int64_t total = n * n;
    for (int64_t x = (int64_t)blockIdx.x * NT + threadIdx.x; x < total; x += (int64_t)gridDim.x * NT) {
        const T v = D[x];
        const bool diag = x / n == x % n;
        const bool bad = (v != v) || (diag ? !(v == (T)0) : (v < (T)0));
        if (bad) atomicMin(first, (unsigned long long)x);
    }
}

__global__ void k_set_u64(unsigned long long *p, unsigned long long v) { *p = v; }

}  // namespace

template <typename T>
hipError_t launch_validate(const T *D, int64_t n, unsigned long long *first, hipStream_t s) {
    hipLaunchKernelGGL(k_set_u64, dim3(1), dim3(1), 0, s, first, ~0ull);
    const int64_t total = n * n;
    int64_t g = (total + NT - 1) / NT;
    hipLaunchKernelGGL((k_validate<T>), dim3((unsigned)(g < 8192 ? (g < 1 ? 1 : g) : 8192)), dim3(NT), 0, s, D, n,
                       first);
    return hipGetLastError();
}

template hipError_t launch_validate<float>(const float *, int64_t, unsigned long long *, hipStream_t);
template hipError_t launch_validate<double>(const double *, int64_t, unsigned long long *, hipStream_t);
template hipError_t launch_validate<_Float16>(const _Float16 *, int64_t, unsigned long long *, hipStream_t);

}  // namespace fw
