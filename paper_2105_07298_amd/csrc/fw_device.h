// fw_device.h -- device helpers shared by the kernel sources: the workgroup
// size, 16-byte vector types, infinity and the element minimum, and the grid
// of the elementwise kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace fw {
namespace {

constexpr int NT = 256;  // threads per workgroup, every kernel

template <typename T> struct V16;
template <> struct V16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int n = 4;
};
template <> struct V16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int n = 2;
};
template <> struct V16<_Float16> {
    typedef _Float16 type __attribute__((ext_vector_type(8)));
    static constexpr int n = 8;
};
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
template <typename T> constexpr bool is_half_v = std::is_same_v<T, _Float16>;

template <typename T> __device__ __forceinline__ T inf_v();
template <> __device__ __forceinline__ float inf_v<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double inf_v<double>() { return __builtin_inf(); }
template <> __device__ __forceinline__ _Float16 inf_v<_Float16>() { return (_Float16)__builtin_inff(); }

__device__ __forceinline__ float vmin(float a, float b) { return __builtin_fminf(a, b); }
// double: the instruction itself.  The library minimum must quiet a signalling
// NaN operand first, and where an accumulator enters a loop iteration the
// compiler cannot tell that it is already quiet, so it re-canonicalised every
// accumulator every iteration (one v_max_f64 per four updates in the last
// phase).  Lengths here are never NaN (input contract), so the plain
// instruction gives the same result.
__device__ __forceinline__ double vmin(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ _Float16 vmin(_Float16 a, _Float16 b) { return __builtin_elementwise_min(a, b); }

inline unsigned grid_for(int64_t n) {
    int64_t g = (n + NT - 1) / NT;
    return (unsigned)(g < 8192 ? (g < 1 ? 1 : g) : 8192);
}

}  // namespace
}  // namespace fw
