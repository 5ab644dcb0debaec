// fw_ooc_kernels.hip -- the min-plus products of the out-of-core driver
// (fw_ooc.cpp): the blocked method's panel and bulk updates (paper Sect. 2.2,
// "Blocked FW Algorithm") applied between super-blocks staged from host memory,
// with distances only or with the path labels, and the merge of the labels of
// a diagonal super-block closed in isolation.
#define FW_TILE_FN __host__ __device__ __forceinline__
#include "fw_internal.h"
#include "fw_lex.h"
#include "fw_device.h"

namespace fw {
namespace {

// ---------------------------------------------------------------------------
// General min-plus update C <- min(C, A (x) B) for the out-of-core driver: C is
// M x N, A is M x K, B is K x N, each with its own leading dimension (M, N
// multiples of the tile edges, K of KT).  Same register-blocked tiles as
// k_phase4, but each workgroup walks all of K in chunks of KT, re-staging the
// two panel chunks in LDS, so that its C tile is read and written once per
// product.  Distances only.
template <typename T, int KT, int BM, int BN>
__global__ void __launch_bounds__(NT) k_minplus(T *__restrict__ C, int64_t ldc, const T *__restrict__ A, int64_t lda,
                                               const T *__restrict__ B, int64_t ldb, int64_t K, TileSel sel) {
    constexpr int RM = BM / 16, RN = BN / 16;
    using vec = typename V16<T>::type;
    constexpr int V = V16<T>::n;
    constexpr int TX = BN / RN, TY = NT / TX;
    static_assert(TY * RM == BM && RN % V == 0, "tile shape");
    constexpr int HN = RN / V, CS = BN / HN;
    constexpr int AST = KT + V;
    __shared__ __attribute__((aligned(16))) T As[BM * AST];
    __shared__ __attribute__((aligned(16))) T Bs[KT * BN];

    int bi, bj;
    if (!select_tile<false>(sel, blockIdx.x, bi, bj)) return;
    const int64_t I0 = (int64_t)bi * BM, J0 = (int64_t)bj * BN;
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;

    T acc[RM][RN];
#pragma unroll
    for (int ii = 0; ii < RM; ++ii)
#pragma unroll
        for (int jj = 0; jj < RN; ++jj) acc[ii][jj] = inf_v<T>();

    for (int64_t k0 = 0; k0 < K; k0 += KT) {
        __syncthreads();  // the previous chunk is consumed
        for (int q = tid; q < BM * (KT / V); q += NT) {
            const int row = q / (KT / V), kv = q % (KT / V);
            *(vec *)(As + row * AST + kv * V) = *(const vec *)(A + (I0 + row) * lda + k0 + kv * V);
        }
        for (int q = tid; q < KT * (BN / V); q += NT) {
            const int krow = q / (BN / V), cv = q % (BN / V);
            *(vec *)(Bs + krow * BN + cv * V) = *(const vec *)(B + (k0 + krow) * ldb + J0 + cv * V);
        }
        __syncthreads();
#pragma unroll 2
        for (int kv = 0; kv < KT / V; ++kv) {
            vec a[RM];
#pragma unroll
            for (int ii = 0; ii < RM; ++ii) a[ii] = *(const vec *)(As + (ty + TY * ii) * AST + kv * V);
#pragma unroll
            for (int kk = 0; kk < V; kk += 2) {
                vec b0[HN], b1[HN];
#pragma unroll
                for (int h = 0; h < HN; ++h) {
                    b0[h] = *(const vec *)(Bs + (kv * V + kk) * BN + h * CS + tx * V);
                    b1[h] = *(const vec *)(Bs + (kv * V + kk + 1) * BN + h * CS + tx * V);
                }
#pragma unroll
                for (int ii = 0; ii < RM; ++ii)
#pragma unroll
                    for (int h = 0; h < HN; ++h)
#pragma unroll
                        for (int e = 0; e < V; ++e) {
                            T &x = acc[ii][h * V + e];
                            x = vmin(vmin(x, a[ii][kk] + b0[h][e]), a[ii][kk + 1] + b1[h][e]);
                        }
            }
        }
    }
#pragma unroll
    for (int ii = 0; ii < RM; ++ii)
#pragma unroll
        for (int h = 0; h < HN; ++h) {
            T *cp = C + (I0 + ty + TY * ii) * ldc + J0 + h * CS + tx * V;
            vec nv = *(const vec *)cp;
            bool ch = false;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const T s = acc[ii][h * V + e];
                ch |= s < nv[e];
                nv[e] = vmin(nv[e], s);
            }
            if (ch) *(vec *)cp = nv;
        }
}

// Lexicographic form of the general update, for the out-of-core driver with
// path labels: (C, PC) <- lexmin over k of (A[i][k] + B[k][j],
// max(PA[i][k], kbase + k, PB[k][j])) and the old (C, PC) -- the rule phases 1-3
// apply, with kbase the global index of A's first column.  The tiles of
// k_minplus with the labels beside the lengths: 64 x 64 entries, each thread
// rows ty + 16 ii and a group of V adjacent columns (V = 16 bytes of lengths),
// panel chunks of KT values of k staged in LDS with their labels + 1, and
// every LDS read a 16-byte (lengths) or V-label vector: for float32 one read
// per 4 updates.  The update itself is lex_take_u (one double minimum on the
// packed key for float32).  Written back: the vectors in which an entry changed.
template <typename T, int KT>
__global__ void __launch_bounds__(NT) k_minplus_lex(T *__restrict__ C, int32_t *__restrict__ PC, int64_t ldc,
                                                   const T *__restrict__ A, const int32_t *__restrict__ PA, int64_t lda,
                                                   const T *__restrict__ B, const int32_t *__restrict__ PB, int64_t ldb,
                                                   int64_t K, int32_t kbase, TileSel sel) {
    constexpr int BM = 64, BN = 64;
    using vec = typename V16<T>::type;
    constexpr int V = V16<T>::n;
    typedef uint32_t lvec __attribute__((ext_vector_type(V)));  // V labels + 1
    constexpr int TX = BN / V, TY = NT / TX, RI = BM / TY;
    static_assert(RI * TY == BM && TX * V == BN, "tile shape");
    constexpr int AST = KT + V;  // row stride of the A chunk (16-byte rows, shifted banks)
    __shared__ __attribute__((aligned(16))) T As[BM * AST];
    __shared__ __attribute__((aligned(16))) uint32_t Al[BM * AST];
    __shared__ __attribute__((aligned(16))) T Bs[KT * BN];
    __shared__ __attribute__((aligned(16))) uint32_t Bl[KT * BN];

    int bi, bj;
    if (!select_tile<false>(sel, blockIdx.x, bi, bj)) return;
    const int64_t I0 = (int64_t)bi * BM, J0 = (int64_t)bj * BN;
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;

    T d[RI][V];
    uint32_t p[RI][V];
#pragma unroll
    for (int ii = 0; ii < RI; ++ii) {
        const int64_t g = (I0 + ty + TY * ii) * ldc + J0 + tx * V;
        const vec c = *(const vec *)(C + g);
        const lvec l = *(const lvec *)(PC + g);
#pragma unroll
        for (int e = 0; e < V; ++e) {
            d[ii][e] = canon(c[e]);
            p[ii][e] = l[e] + 1u;
        }
    }

    for (int64_t k0 = 0; k0 < K; k0 += KT) {
        __syncthreads();  // the previous chunk is consumed
        for (int q = tid; q < BM * (KT / V); q += NT) {
            const int row = q / (KT / V), kv = q % (KT / V);
            const int64_t g = (I0 + row) * lda + k0 + kv * V;
            vec a = *(const vec *)(A + g);
            lvec l = *(const lvec *)(PA + g);
#pragma unroll
            for (int e = 0; e < V; ++e) {
                a[e] = canon(a[e]);
                l[e] += 1u;
            }
            *(vec *)(As + row * AST + kv * V) = a;
            *(lvec *)(Al + row * AST + kv * V) = l;
        }
        for (int q = tid; q < KT * (BN / V); q += NT) {
            const int krow = q / (BN / V), cv = q % (BN / V);
            const int64_t g = (k0 + krow) * ldb + J0 + cv * V;
            vec b = *(const vec *)(B + g);
            lvec l = *(const lvec *)(PB + g);
#pragma unroll
            for (int e = 0; e < V; ++e) {
                b[e] = canon(b[e]);
                l[e] += 1u;
            }
            *(vec *)(Bs + krow * BN + cv * V) = b;
            *(lvec *)(Bl + krow * BN + cv * V) = l;
        }
        __syncthreads();
        for (int kv = 0; kv < KT / V; ++kv) {
            vec a[RI];
            lvec la[RI];
#pragma unroll
            for (int ii = 0; ii < RI; ++ii) {
                a[ii] = *(const vec *)(As + (ty + TY * ii) * AST + kv * V);
                la[ii] = *(const lvec *)(Al + (ty + TY * ii) * AST + kv * V);
            }
#pragma unroll
            for (int kk = 0; kk < V; ++kk) {
                const int k = kv * V + kk;
                const vec b = *(const vec *)(Bs + k * BN + tx * V);
                const lvec lb = *(const lvec *)(Bl + k * BN + tx * V);
                const uint32_t kg1 = (uint32_t)(kbase + k0 + k + 1);
#pragma unroll
                for (int ii = 0; ii < RI; ++ii)
#pragma unroll
                    for (int e = 0; e < V; ++e)
                        lex_take_u(d[ii][e], p[ii][e], a[ii][kk] + b[e], max(max(la[ii][kk], lb[e]), kg1));
            }
        }
    }
#pragma unroll
    for (int ii = 0; ii < RI; ++ii) {
        const int64_t g = (I0 + ty + TY * ii) * ldc + J0 + tx * V;
        const vec c = *(const vec *)(C + g);
        const lvec l = *(const lvec *)(PC + g);
        vec nc;
        lvec nl;
        bool ch = false;
#pragma unroll
        for (int e = 0; e < V; ++e) {
            nc[e] = d[ii][e];
            nl[e] = p[ii][e] - 1u;
            ch |= !(d[ii][e] == c[e]) || nl[e] != l[e];
        }
        if (ch) {
            *(vec *)(C + g) = nc;
            *(lvec *)(PC + g) = nl;
        }
    }
}

// Labels of a block closed in isolation (local vertex indices, -1 where the
// entry did not change) turned into global ones: unchanged entries keep their
// old label, changed ones get base + local.
__global__ void k_merge_labels(int32_t *__restrict__ P, const int32_t *__restrict__ Plocal, int64_t count,
                               int32_t base) {
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < count; x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t l = Plocal[x];
        if (l >= 0) P[x] = base + l;
    }
}

}  // namespace

template <typename T>
hipError_t launch_minplus(T *C, int64_t ldc, const T *A, int64_t lda, const T *B, int64_t ldb, int64_t M, int64_t N,
                          int64_t K, hipStream_t s) {
    constexpr int KT = 64, BM = 64, BN = 64;
    if (M % BM || N % BN || K % KT || M <= 0 || N <= 0 || K <= 0) return hipErrorInvalidValue;
    TileSel sel;
    if (!make_tile_sel((int)(M / BM), (int)(N / BN), 0, 0, 0, 1, 0, sel)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_minplus<T, KT, BM, BN>), dim3(8 * sel.per_xcd), dim3(NT), 0, s, C, ldc, A, lda, B, ldb, K,
                       sel);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_minplus_lex(T *C, int32_t *PC, int64_t ldc, const T *A, const int32_t *PA, int64_t lda, const T *B,
                              const int32_t *PB, int64_t ldb, int64_t M, int64_t N, int64_t K, int32_t kbase,
                              hipStream_t s) {
    constexpr int KT = 32;
    if (M % 64 || N % 64 || K % KT || M <= 0 || N <= 0 || K <= 0) return hipErrorInvalidValue;
    TileSel sel;
    if (!make_tile_sel((int)(M / 64), (int)(N / 64), 0, 0, 0, 1, 0, sel)) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_minplus_lex<T, KT>), dim3(8 * sel.per_xcd), dim3(NT), 0, s, C, PC, ldc, A, PA, lda, B, PB,
                       ldb, K, kbase, sel);
    return hipGetLastError();
}

hipError_t launch_merge_labels(int32_t *P, const int32_t *Plocal, int64_t count, int32_t base, hipStream_t s) {
    hipLaunchKernelGGL(k_merge_labels, dim3(grid_for(count)), dim3(NT), 0, s, P, Plocal, count, base);
    return hipGetLastError();
}

template hipError_t launch_minplus_lex<float>(float *, int32_t *, int64_t, const float *, const int32_t *, int64_t,
                                              const float *, const int32_t *, int64_t, int64_t, int64_t, int64_t,
                                              int32_t, hipStream_t);
template hipError_t launch_minplus_lex<double>(double *, int32_t *, int64_t, const double *, const int32_t *, int64_t,
                                               const double *, const int32_t *, int64_t, int64_t, int64_t, int64_t,
                                               int32_t, hipStream_t);
template hipError_t launch_minplus<float>(float *, int64_t, const float *, int64_t, const float *, int64_t, int64_t,
                                          int64_t, int64_t, hipStream_t);
template hipError_t launch_minplus<double>(double *, int64_t, const double *, int64_t, const double *, int64_t,
                                           int64_t, int64_t, int64_t, hipStream_t);

}  // namespace fw
