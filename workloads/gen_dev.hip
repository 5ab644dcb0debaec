// gen_dev.hip -- the device twin of gen.c's graph generator (inputs only; no
// shortest-path arithmetic): the same counter-addressed SplitMix64 draws and
// weight laws, so a matrix generated here equals gen_rows_f32/f64's bit for
// bit.  Used where a large input should never exist in host memory.  Built
// with contraction off, so that 1 + 9 * x (W_ONE_TEN) is rounded as on the
// host: a multiply, then an add.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint64_t GOLDEN = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__host__ __device__ inline uint64_t gkey(uint64_t seed, uint64_t stream, uint64_t g) {
    return mix64(mix64(seed * GOLDEN + stream) ^ (g * 0xD1B54A32D192ED03ull));
}

__device__ inline uint64_t draw(uint64_t key, uint64_t i, uint64_t j) {
    return mix64(key + (((i << 32) | j) + 1) * GOLDEN);
}

// the weight laws of gen.c (W_INT, W_UNIT_OPEN, W_ONE_TEN, W_ONE_TWO)
__device__ inline double weight_of(int law, uint64_t h, int64_t wmax, bool is_f64) {
    switch (law) {
    case 0: return (double)(1 + (int64_t)(((h >> 32) * (uint64_t)wmax) >> 32));
    case 1: return is_f64 ? (double)(2 * (h >> 12) + 1) * 0x1p-53 : (double)(2 * (h >> 41) + 1) * 0x1p-24;
    case 2: return 1.0 + 9.0 * ((double)(2 * (h >> 41) + 1) * 0x1p-24);
    case 3: return 1.0 + (double)(h >> 41) * 0x1p-23;
    }
    return __builtin_nan("");
}

template <typename T>
__global__ void k_gen_rows(uint64_t ek, uint64_t wk, int64_t n, int64_t r0, int64_t r1, uint64_t thresh32, int law,
                           int64_t wmax, T *out) {
    const int64_t total = (r1 - r0) * n;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t i = (uint64_t)(r0 + x / n), j = (uint64_t)(x % n);
        T v;
        if (i == j)
            v = (T)0;
        else if (thresh32 < (1ull << 32) && (draw(ek, i, j) >> 32) >= thresh32)
            v = (T)__builtin_inf();
        else
            v = (T)weight_of(law, draw(wk, i, j), wmax, sizeof(T) == 8);
        out[x] = v;
    }
}

}  // namespace

extern "C" {

// Rows [r0, r1) of graph g (as gen_rows_f32 / gen_rows_f64) into device memory
// out (row-major, leading dimension n, out at row r0), on `stream`.  Returns a
// hipError_t code (0 = launched).
int gen_rows_dev(uint64_t seed, uint64_t g, int64_t n, int64_t r0, int64_t r1, uint64_t thresh32, int law,
                 int64_t wmax, int is_f64, void *out, void *stream) {
    const uint64_t ek = gkey(seed, 0, g), wk = gkey(seed, 1, g);
    const int64_t total = (r1 - r0) * n;
    const int64_t blocks = (total + 255) / 256;
    const dim3 grid((unsigned)(blocks < 65536 ? (blocks < 1 ? 1 : blocks) : 65536));
    if (is_f64)
        hipLaunchKernelGGL((k_gen_rows<double>), grid, dim3(256), 0, (hipStream_t)stream, ek, wk, n, r0, r1, thresh32,
                           law, wmax, (double *)out);
    else
        hipLaunchKernelGGL((k_gen_rows<float>), grid, dim3(256), 0, (hipStream_t)stream, ek, wk, n, r0, r1, thresh32,
                           law, wmax, (float *)out);
    return (int)hipGetLastError();
}
}
