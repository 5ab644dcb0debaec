// fw_lex.h -- the lexicographic (length, label) update in its fast form, shared
// by the device kernels that carry the path matrix.  Sect. 2.2 (Algorithm 1):
// a shorter candidate through k replaces the entry and records k as its
// intermediate vertex.  The tie-break is this library's reading, not the
// paper's (the paper never discusses the path matrix under the blocked order):
// equal lengths go to the smaller largest-interior-vertex label, which makes
// the labels independent of the order of the k steps and equal to what the
// classic loop with a strict test stores.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fw {

// The same rule on labels kept offset by one (label + 1: "no interior vertex"
// is 0, and labels compare as unsigned numbers).  For float the pair is one
// 64-bit unsigned key, length bits above label: non-negative floats (+0 to
// +inf) order like their bit patterns, so the lexicographic minimum is the
// minimum of the keys.  Lengths must not be -0.0 (see canon()).
// The key read as an IEEE double orders like the key itself: it is
// non-negative and never NaN (a NaN double would need a float bit pattern
// above +inf), and non-negative doubles order like their bit patterns,
// subnormals included, which these kernels keep (their float mode preserves
// double subnormals).  So one double minimum takes it, with no compare and
// selects.  It is written as the instruction itself: the library minimum would
// first canonicalise both operands against signalling NaNs.
__device__ __forceinline__ void lex_take_u(float &d, uint32_t &p, float s, uint32_t m) {
    const double ks = __builtin_bit_cast(double, ((uint64_t)__float_as_uint(s) << 32) | m);
    const double kd = __builtin_bit_cast(double, ((uint64_t)__float_as_uint(d) << 32) | p);
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(kd), "v"(ks));
    const uint64_t u = __builtin_bit_cast(uint64_t, r);
    d = __uint_as_float((uint32_t)(u >> 32));
    p = (uint32_t)u;
}
// binary16 likewise: its 16 bits above the label make every key a subnormal
// double.
__device__ __forceinline__ void lex_take_u(_Float16 &d, uint32_t &p, _Float16 s, uint32_t m) {
    const double ks = __builtin_bit_cast(double, ((uint64_t)__builtin_bit_cast(uint16_t, s) << 32) | m);
    const double kd = __builtin_bit_cast(double, ((uint64_t)__builtin_bit_cast(uint16_t, d) << 32) | p);
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(kd), "v"(ks));
    const uint64_t u = __builtin_bit_cast(uint64_t, r);
    d = __builtin_bit_cast(_Float16, (uint16_t)(u >> 32));
    p = (uint32_t)u;
}
// double: the key would need 96 bits, so the rule stays two-keyed, written
// without short-circuit logic (which compiles to a branch around every
// update): a tie keeps the smaller label, a shorter candidate takes its own,
// and the length is the double minimum (the same instruction as above).
__device__ __forceinline__ void lex_take_u(double &d, uint32_t &p, double s, uint32_t m) {
    const uint32_t q = (s == d) ? min(p, m) : p;
    p = (s < d) ? m : q;
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(d), "v"(s));
    d = r;
}
// A length as read from memory, with -0.0 turned into +0.0 (equal as numbers,
// but its bit pattern would sort above +inf in lex_take_u's key).
template <typename T>
__device__ __forceinline__ T canon(T x) {
    return x + (T)0;
}

}  // namespace fw
