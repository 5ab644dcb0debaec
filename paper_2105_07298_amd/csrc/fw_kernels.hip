// fw_kernels.hip -- gfx950 kernels of the blocked Floyd-Warshall method.
//
// One round r (k-block K = [r*TB, (r+1)*TB)) is three launches (paper Sect. 2.2,
// "Blocked FW Algorithm"; the GPU split into one kernel for the diagonal block,
// one for both panels and one for the rest follows Sect. 3.2):
//   k_phase1   the diagonal block, TB sequential k-steps in LDS;
//   k_phase23  the row panel D[K, J] and the column panel D[I, K], as min-plus
//              products with the closed diagonal block (no sequential k-steps);
//   k_phase4   every other tile, a register-blocked min-plus product of the final
//              column panel D[I, K] and row panel D[K, J], both staged in LDS.
//
// Path matrix: every candidate through k carries the label
// (length, max(P[i][k], k, P[k][j])); an entry takes a candidate whose label is
// lexicographically smaller.  This reproduces, whatever the block size, what the
// classic loop with a strict test stores (the smallest possible largest interior
// vertex over all shortest paths).  The last phase takes path mode in two
// passes: the k-loop computes only the minimum length S (the same instructions
// as distances-only mode), and the few entries whose S reaches or beats the
// current length are queued and resolved afterwards by scanning the k that
// attain S.
//
// All arithmetic is on the vector ALU: the min-plus product is not a ring
// contraction, so matrix cores do not apply.
#include "fw_internal.h"

#include <limits.h>

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

template <typename T> __device__ __forceinline__ T inf_v();
template <> __device__ __forceinline__ float inf_v<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double inf_v<double>() { return __builtin_inf(); }

__device__ __forceinline__ float vmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double vmin(double a, double b) { return __builtin_fmin(a, b); }

// Lexicographic label update: take (s, m) when it is smaller than (d, p).
template <typename T>
__device__ __forceinline__ void lex_take(T &d, int32_t &p, T s, int32_t m) {
    const bool take = (s < d) || (s == d && m < p);
    d = take ? s : d;
    p = take ? m : p;
}

// ---------------------------------------------------------------------------
// Phase 1: close the diagonal block.  The block and its P stay in LDS; thread
// (ty, tx) owns rows ty + 16*ii and columns tx + 16*jj.  At step k, row k and
// column k of the block are unchanged by the update (D[k][k] = 0, so every
// candidate for them equals the current value with a label that is not
// smaller), hence updating in place while other threads read them is safe; one
// barrier per k orders step k's writes before step k+1's reads.
template <typename T, int TB, bool PATH>
__global__ void __launch_bounds__(NT) k_phase1(T *__restrict__ D, int32_t *__restrict__ P, int64_t ld, int r) {
    constexpr int TS = 16, RM = TB / TS, ST = TB + 1;
    __shared__ T sd[TB * ST];
    __shared__ int32_t sp[PATH ? TB * ST : 1];
    const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
    const int64_t k0 = (int64_t)r * TB;
    T d[RM][RM];
    int32_t p[RM][RM];
#pragma unroll
    for (int ii = 0; ii < RM; ++ii)
#pragma unroll
        for (int jj = 0; jj < RM; ++jj) {
            const int row = ty + TS * ii, col = tx + TS * jj;
            const int64_t g = (k0 + row) * ld + k0 + col;
            d[ii][jj] = D[g];
            sd[row * ST + col] = d[ii][jj];
            if (PATH) {
                p[ii][jj] = P[g];
                sp[row * ST + col] = p[ii][jj];
            }
        }
    __syncthreads();
    for (int k = 0; k < TB; ++k) {
        T a[RM], b[RM];
        int32_t pa[RM], pb[RM];
#pragma unroll
        for (int ii = 0; ii < RM; ++ii) {
            a[ii] = sd[(ty + TS * ii) * ST + k];
            if (PATH) pa[ii] = sp[(ty + TS * ii) * ST + k];
        }
#pragma unroll
        for (int jj = 0; jj < RM; ++jj) {
            b[jj] = sd[k * ST + tx + TS * jj];
            if (PATH) pb[jj] = sp[k * ST + tx + TS * jj];
        }
        const int32_t kg = (int32_t)(k0 + k);
#pragma unroll
        for (int ii = 0; ii < RM; ++ii)
#pragma unroll
            for (int jj = 0; jj < RM; ++jj) {
                const T s = a[ii] + b[jj];
                const int idx = (ty + TS * ii) * ST + tx + TS * jj;
                if (PATH) {
                    const int32_t m = max(max(pa[ii], pb[jj]), kg);
                    if ((s < d[ii][jj]) || (s == d[ii][jj] && m < p[ii][jj])) {
                        d[ii][jj] = s;
                        p[ii][jj] = m;
                        sd[idx] = s;
                        sp[idx] = m;
                    }
                } else if (s < d[ii][jj]) {
                    d[ii][jj] = s;
                    sd[idx] = s;
                }
            }
        __syncthreads();
    }
#pragma unroll
    for (int ii = 0; ii < RM; ++ii)
#pragma unroll
        for (int jj = 0; jj < RM; ++jj) {
            const int64_t g = (k0 + ty + TS * ii) * ld + k0 + tx + TS * jj;
            D[g] = d[ii][jj];
            if (PATH) P[g] = p[ii][jj];
        }
}

// ---------------------------------------------------------------------------
// Phases 2 and 3: the row panel D[K, J] and the column panel D[I, K].  With the
// diagonal block already closed (D*), every path from a vertex of K to j that
// goes through K ends with a closed segment inside K followed by an old entry,
// so the panel update is one min-plus product with the old panel:
//   D[K, J] <- lexmin(D[K, J], D*[K, K] (x) D_old[K, J])
//   D[I, K] <- lexmin(D[I, K], D_old[I, K] (x) D*[K, K]).
// The two kinds of tile are independent and share one launch: workgroups
// [0, nb-1) take the row panel, [nb-1, 2(nb-1)) the column panel.  Each tile is
// read completely (operands into LDS, old values into registers) before it is
// written, and only its own workgroup touches it.
template <typename T, int TB, bool PATH>
__global__ void __launch_bounds__(NT) k_phase23(T *__restrict__ D, int32_t *__restrict__ P, int64_t ld, int r, int nb) {
    constexpr int TS = 16, RM = TB / TS, ST = TB + 1;
    __shared__ T sa[TB * ST];
    __shared__ T sb[TB * ST];
    __shared__ int32_t spa[PATH ? TB * ST : 1];
    __shared__ int32_t spb[PATH ? TB * ST : 1];
    const int w = blockIdx.x;
    const bool rowp = w < nb - 1;
    const int t = rowp ? w : w - (nb - 1);
    const int o = t < r ? t : t + 1;
    const int64_t k0 = (int64_t)r * TB;
    const int64_t I0 = rowp ? k0 : (int64_t)o * TB;
    const int64_t J0 = rowp ? (int64_t)o * TB : k0;
    for (int q = threadIdx.x; q < TB * TB; q += NT) {
        const int rr = q / TB, cc = q % TB;
        const int64_t ga = (I0 + rr) * ld + k0 + cc;  // A = D[I0.., K]
        const int64_t gb = (k0 + rr) * ld + J0 + cc;  // B = D[K, J0..]
        sa[rr * ST + cc] = D[ga];
        sb[rr * ST + cc] = D[gb];
        if (PATH) {
            spa[rr * ST + cc] = P[ga];
            spb[rr * ST + cc] = P[gb];
        }
    }
    const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
    T d[RM][RM];
    int32_t p[RM][RM];
#pragma unroll
    for (int ii = 0; ii < RM; ++ii)
#pragma unroll
        for (int jj = 0; jj < RM; ++jj) {
            const int64_t g = (I0 + ty + TS * ii) * ld + J0 + tx + TS * jj;
            d[ii][jj] = D[g];
            if (PATH) p[ii][jj] = P[g];
        }
    __syncthreads();
    for (int k = 0; k < TB; ++k) {
        T a[RM], b[RM];
        int32_t pa[RM], pb[RM];
#pragma unroll
        for (int ii = 0; ii < RM; ++ii) {
            a[ii] = sa[(ty + TS * ii) * ST + k];
            if (PATH) pa[ii] = spa[(ty + TS * ii) * ST + k];
        }
#pragma unroll
        for (int jj = 0; jj < RM; ++jj) {
            b[jj] = sb[k * ST + tx + TS * jj];
            if (PATH) pb[jj] = spb[k * ST + tx + TS * jj];
        }
        const int32_t kg = (int32_t)(k0 + k);
#pragma unroll
        for (int ii = 0; ii < RM; ++ii)
#pragma unroll
            for (int jj = 0; jj < RM; ++jj) {
                const T s = a[ii] + b[jj];
                if (PATH)
                    lex_take(d[ii][jj], p[ii][jj], s, max(max(pa[ii], pb[jj]), kg));
                else
                    d[ii][jj] = vmin(d[ii][jj], s);
            }
    }
#pragma unroll
    for (int ii = 0; ii < RM; ++ii)
#pragma unroll
        for (int jj = 0; jj < RM; ++jj) {
            const int64_t g = (I0 + ty + TS * ii) * ld + J0 + tx + TS * jj;
            D[g] = d[ii][jj];
            if (PATH) P[g] = p[ii][jj];
        }
}

// ---------------------------------------------------------------------------
// Phase 4: C = D[I0:I0+BM, J0:J0+BN] <- min(C, D[I, K] (x) D[K, J]) for every
// tile outside block row / column r.  The panels are final for the round, so the
// k-loop has no barrier.  Thread layout: TX x TY threads, each owning an RM x RN
// micro-tile in registers: rows ty + TY*ii, columns h*CS + tx*V + e (V
// consecutive elements = one 16-byte vector, HN vectors per thread spread CS
// apart so that a wave's LDS and global accesses are contiguous).
//
// LDS: A panel row-major (row = i, padded by one vector so that the TY rows a
// wave reads start in different banks), B panel row-major (row = k).  A thread
// reads V consecutive k of each of its rows at once (one 16-byte load) and, per
// k, HN vectors of the B row.  Per k and thread: RM + RN values for RM*RN
// updates.
//
// When the tile is wider than the block, the tile that contains block row
// (column) r masks those rows (columns): their A (B) values are +inf, so they
// never change and are never written.  Entries are stored only where they
// changed, so panel entries are never written during this phase.
//
// Tile order: workgroups are spread round-robin over the 8 XCDs; each XCD gets a
// contiguous range of tiles, walked in groups of 8 tile rows so that the
// workgroups resident on one XCD share A and B panels in its L2.
template <typename T, int TB, int BM, int BN, int RM, int RN, bool PATH>
__global__ void __launch_bounds__(NT) k_phase4(T *__restrict__ D, int32_t *__restrict__ P, int64_t ld, int r,
                                              int gm, int gn, int skip, int per_xcd, int ntiles) {
    using vec = typename V16<T>::type;
    constexpr int V = V16<T>::n;
    constexpr int TX = BN / RN, TY = NT / TX;
    static_assert(TY * RM == BM, "tile rows");
    static_assert(RN % V == 0, "micro-tile width");
    constexpr int HN = RN / V, CS = BN / HN;
    constexpr int AST = TB + V;
    constexpr int CAP = 256;  // queued entries per wave and sweep (path mode)
    constexpr int NW = NT / 64;

    __shared__ __attribute__((aligned(16))) T As[BM * AST];
    __shared__ __attribute__((aligned(16))) T Bs[TB * BN];
    __shared__ uint32_t q_rc[PATH ? NW * CAP : 1];
    __shared__ T q_s[PATH ? NW * CAP : 1];

    const int wg = blockIdx.x;
    const int lin = (wg % 8) * per_xcd + wg / 8;
    if (lin >= ntiles) return;
    const int gm_e = gm - (skip >= 0), gn_e = gn - (skip >= 0);
    constexpr int G = 8;
    const int group = lin / (G * gn_e);
    const int first = group * G;
    const int rows_in = min(G, gm_e - first);
    const int idx = lin - group * G * gn_e;
    int bi = first + idx % rows_in, bj = idx / rows_in;
    if (skip >= 0) {
        bi += bi >= skip;
        bj += bj >= skip;
    }
    const int64_t I0 = (int64_t)bi * BM, J0 = (int64_t)bj * BN, k0 = (int64_t)r * TB;
    const bool mask_rows = (I0 <= k0) && (k0 < I0 + BM);
    const bool mask_cols = (J0 <= k0) && (k0 < J0 + BN);

    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;

    // Old C values, requested first so their latency overlaps the panel loads.
    vec c[RM][HN];
#pragma unroll
    for (int ii = 0; ii < RM; ++ii)
#pragma unroll
        for (int h = 0; h < HN; ++h)
            c[ii][h] = *(const vec *)(D + (I0 + ty + TY * ii) * ld + J0 + h * CS + tx * V);

    const vec vinf = inf_v<T>();
    for (int q = tid; q < BM * (TB / V); q += NT) {
        const int row = q / (TB / V), kv = q % (TB / V);
        vec v = *(const vec *)(D + (I0 + row) * ld + k0 + kv * V);
        if (mask_rows && (uint64_t)(I0 + row - k0) < (uint64_t)TB) v = vinf;
        *(vec *)(As + row * AST + kv * V) = v;
    }
    for (int q = tid; q < TB * (BN / V); q += NT) {
        const int krow = q / (BN / V), cv = q % (BN / V);
        vec v = *(const vec *)(D + (k0 + krow) * ld + J0 + cv * V);
        if (mask_cols && (uint64_t)(J0 + cv * V - k0) < (uint64_t)TB) v = vinf;
        *(vec *)(Bs + krow * BN + cv * V) = v;
    }
    __syncthreads();

    T acc[RM][RN];
#pragma unroll
    for (int ii = 0; ii < RM; ++ii)
#pragma unroll
        for (int jj = 0; jj < RN; ++jj) acc[ii][jj] = inf_v<T>();

#pragma unroll 2
    for (int kv = 0; kv < TB / V; ++kv) {
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

    // New distances: store the 16-byte vectors in which some entry decreased.
#pragma unroll
    for (int ii = 0; ii < RM; ++ii)
#pragma unroll
        for (int h = 0; h < HN; ++h) {
            vec nv = c[ii][h];
            bool ch = false;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const T s = acc[ii][h * V + e];
                ch |= s < nv[e];
                nv[e] = s < nv[e] ? s : nv[e];
            }
            if (ch) *(vec *)(D + (I0 + ty + TY * ii) * ld + J0 + h * CS + tx * V) = nv;
        }

    if constexpr (PATH) {
        // Second pass.  An entry needs its path label when S = min_k(A+B) is
        // finite and <= the old length: S < old ("improve") sets P to the
        // smallest label among the k with A+B == S; S == old ("tie") keeps the
        // smaller of that and the old P.  Each wave queues its own entries in
        // LDS (ballot + prefix count, no atomics) and resolves CAP at a time,
        // each lane taking four.  Labels need P of the panels, read from
        // global memory (the panels are not written in this phase).
        const int wave = tid >> 6, lane = tid & 63;
        uint32_t *qrc = q_rc + wave * CAP;
        T *qs = q_s + wave * CAP;
        for (int skip_n = 0;; skip_n += CAP) {
            int cum = 0;
#pragma unroll
            for (int ii = 0; ii < RM; ++ii)
#pragma unroll
                for (int h = 0; h < HN; ++h)
#pragma unroll
                    for (int e = 0; e < V; ++e) {
                        const T s = acc[ii][h * V + e], old = c[ii][h][e];
                        const bool mk = (s <= old) && (s < inf_v<T>());
                        const uint64_t bal = __ballot(mk);
                        if (bal) {
                            const int pos = cum + (int)__builtin_amdgcn_mbcnt_hi(
                                                      (uint32_t)(bal >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                            if (mk && pos >= skip_n && pos < skip_n + CAP) {
                                const uint32_t row = ty + TY * ii, col = h * CS + tx * V + e;
                                qrc[pos - skip_n] = row | (col << 8) | ((uint32_t)(s < old) << 16);
                                qs[pos - skip_n] = s;
                            }
                            cum += __popcll(bal);
                        }
                    }
            const int nq = min(cum - skip_n, CAP);
            if (nq <= 0) break;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

            constexpr int U = CAP / 64;
            uint64_t hits[U];
            uint32_t rc[U];
            int32_t M[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = lane + 64 * u;
                hits[u] = 0;
                rc[u] = 0;
                M[u] = INT_MAX;
                if (t < nq) {
                    rc[u] = qrc[t];
                    const T S = qs[t];
                    const int row = rc[u] & 255, col = (rc[u] >> 8) & 255;
                    const T *arow = As + row * AST;
                    uint64_t hm = 0;
#pragma unroll
                    for (int kv = 0; kv < TB / V; ++kv) {
                        const vec av = *(const vec *)(arow + kv * V);
#pragma unroll
                        for (int e = 0; e < V; ++e) {
                            const T s = av[e] + Bs[(kv * V + e) * BN + col];
                            hm |= (s == S) ? (1ull << (kv * V + e)) : 0ull;
                        }
                    }
                    hits[u] = hm;
                }
            }
            __builtin_amdgcn_wave_barrier();  // queue slots are free for the next sweep from here

            // Old P of each queued entry and the labels of the k that attain S.
            // Every lane issues its loads for all four entries before using any
            // (indices are clamped into the tile when a slot is empty).
            int32_t pold[U];
            bool first = true;
            for (;;) {
                int32_t pa[U], pb[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int row = rc[u] & 255, col = (rc[u] >> 8) & 255;
                    const int k = hits[u] ? __builtin_ctzll(hits[u]) : 0;
                    pa[u] = P[(I0 + row) * ld + k0 + k];
                    pb[u] = P[(k0 + k) * ld + J0 + col];
                    if (first) pold[u] = P[(I0 + row) * ld + J0 + col];
                }
                bool more = false;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (hits[u]) {
                        const int k = __builtin_ctzll(hits[u]);
                        M[u] = min(M[u], max(max(pa[u], pb[u]), (int32_t)(k0 + k)));
                        hits[u] &= hits[u] - 1;
                        more |= hits[u] != 0;
                    }
                }
                first = false;
                if (!__any(more)) break;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (lane + 64 * u < nq) {
                    const int row = rc[u] & 255, col = (rc[u] >> 8) & 255;
                    const bool improve = (rc[u] >> 16) & 1;
                    const int32_t np = improve ? M[u] : min(pold[u], M[u]);
                    if (np != pold[u]) P[(I0 + row) * ld + J0 + col] = np;
                }
            }
            if (cum <= skip_n + CAP) break;
        }
    }
}

// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
__global__ void k_pad_in(const T *__restrict__ src, int64_t n, T *__restrict__ dst, int64_t npad) {
    const int64_t total = npad * npad;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = x / npad, j = x % npad;
        dst[x] = (i < n && j < n) ? src[i * n + j] : (i == j ? (T)0 : inf_v<T>());
    }
}

template <typename T>
__global__ void k_pad_out(const T *__restrict__ src, int64_t npad, T *__restrict__ dst, int64_t n) {
    const int64_t total = n * n;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = x / n, j = x % n;
        dst[x] = src[i * npad + j];
    }
}

inline unsigned grid_for(int64_t n) {
    int64_t g = (n + NT - 1) / NT;
    return (unsigned)(g < 8192 ? (g < 1 ? 1 : g) : 8192);
}

template <typename T, int TB, int TILE>
hipError_t round_impl(T *D, int32_t *P, int64_t ld, int r, hipStream_t s) {
    constexpr int RM4 = (TILE == 128) ? 8 : 4;
    constexpr int RN4 = (sizeof(T) == 8) ? 4 : ((TILE == 128) ? 8 : 4);
    constexpr int BM = TILE, BN = TILE;
    const int nb = (int)(ld / TB);
    const bool path = P != nullptr;
    if (path)
        hipLaunchKernelGGL((k_phase1<T, TB, true>), dim3(1), dim3(NT), 0, s, D, P, ld, r);
    else
        hipLaunchKernelGGL((k_phase1<T, TB, false>), dim3(1), dim3(NT), 0, s, D, P, ld, r);
    if (nb == 1) return hipGetLastError();
    if (path)
        hipLaunchKernelGGL((k_phase23<T, TB, true>), dim3(2 * (nb - 1)), dim3(NT), 0, s, D, P, ld, r, nb);
    else
        hipLaunchKernelGGL((k_phase23<T, TB, false>), dim3(2 * (nb - 1)), dim3(NT), 0, s, D, P, ld, r, nb);
    const int gm = (int)(ld / BM), gn = (int)(ld / BN);
    const int skip = (BM == TB) ? r : -1;
    const int gm_e = gm - (skip >= 0), gn_e = gn - (skip >= 0);
    const int ntiles = gm_e * gn_e;
    if (ntiles > 0) {
        const int per = (ntiles + 7) / 8;
        prof_begin_p4(s);
        if (path)
            hipLaunchKernelGGL((k_phase4<T, TB, BM, BN, RM4, RN4, true>), dim3(8 * per), dim3(NT), 0, s, D, P, ld, r,
                               gm, gn, skip, per, ntiles);
        else
            hipLaunchKernelGGL((k_phase4<T, TB, BM, BN, RM4, RN4, false>), dim3(8 * per), dim3(NT), 0, s, D, P, ld,
                               r, gm, gn, skip, per, ntiles);
        prof_end_p4(s);
    }
    return hipGetLastError();
}

}  // namespace

template <typename T>
bool config_supported(TileCfg c) {
    if (sizeof(T) == 8) return (c.block == 32 || c.block == 64) && c.tile == 64;
    return (c.block == 32 && c.tile == 64) || (c.block == 64 && (c.tile == 64 || c.tile == 128));
}

template <typename T>
hipError_t launch_round(T *D, int32_t *P, int64_t ld, int r, TileCfg c, hipStream_t s) {
    if constexpr (sizeof(T) == 4) {
        if (c.block == 64 && c.tile == 128) return round_impl<T, 64, 128>(D, P, ld, r, s);
        if (c.block == 64 && c.tile == 64) return round_impl<T, 64, 64>(D, P, ld, r, s);
        if (c.block == 32 && c.tile == 64) return round_impl<T, 32, 64>(D, P, ld, r, s);
    } else {
        if (c.block == 64 && c.tile == 64) return round_impl<T, 64, 64>(D, P, ld, r, s);
        if (c.block == 32 && c.tile == 64) return round_impl<T, 32, 64>(D, P, ld, r, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(NT), 0, s, p, n, v);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pad_in(const T *src, int64_t n, T *dst, int64_t npad, hipStream_t s) {
    hipLaunchKernelGGL((k_pad_in<T>), dim3(grid_for(npad * npad)), dim3(NT), 0, s, src, n, dst, npad);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pad_out(const T *src, int64_t npad, T *dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL((k_pad_out<T>), dim3(grid_for(n * n)), dim3(NT), 0, s, src, npad, dst, n);
    return hipGetLastError();
}

template bool config_supported<float>(TileCfg);
template bool config_supported<double>(TileCfg);
template hipError_t launch_round<float>(float *, int32_t *, int64_t, int, TileCfg, hipStream_t);
template hipError_t launch_round<double>(double *, int32_t *, int64_t, int, TileCfg, hipStream_t);
template hipError_t launch_pad_in<float>(const float *, int64_t, float *, int64_t, hipStream_t);
template hipError_t launch_pad_in<double>(const double *, int64_t, double *, int64_t, hipStream_t);
template hipError_t launch_pad_out<float>(const float *, int64_t, float *, int64_t, hipStream_t);
template hipError_t launch_pad_out<double>(const double *, int64_t, double *, int64_t, hipStream_t);
template hipError_t launch_pad_out<int32_t>(const int32_t *, int64_t, int32_t *, int64_t, hipStream_t);

}  // namespace fw
