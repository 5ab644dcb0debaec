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
// 32 or 64 per graph, by size, from the tuning table): the diagonal block is
// closed by TB sequential k-steps; panel and remaining tiles are min-plus
// products of two LDS-resident operand tiles with the old tile held in
// registers.  Every step applies the lexicographic label rule
// (length, max(P[i][k], k, P[k][j])), so D and P equal the single-graph result
// (and the classic loop's, for exact weights) whatever TB is.  Graphs are stored
// unpadded (leading dimension n, any offset), so global accesses are guarded
// element by element: rows and columns beyond n read as isolated padding
// vertices (+inf off the diagonal, 0 on it, label -1) and are never written.
//
// The tile products follow the single-graph last phase: thread (ty, tx) of a
// 16 x 16 layout owns rows ty + 16*ii and a run of VB contiguous columns per
// vector; operand tiles sit in LDS row-major with a row stride of TB + V
// elements, so a thread reads V consecutive k of a row, or VB consecutive
// columns of a k row, with one vector load; without labels two k are folded per
// three-way minimum.  In the last phase the column-panel tile of a block row
// stays staged while the row's tiles are swept.  Labels are held as 16-bit
// label + 1 (n <= 4096), in LDS and, while a graph is solved, in global
// memory too: the first n*n*2 bytes of the graph's P hold them, and a last pass
// widens them in place to the 32-bit labels.
#include "fw_internal.h"
#include "fw_lex.h"

#include <mutex>

namespace fw {
namespace {

constexpr int NT = 256;

template <typename T> __device__ __forceinline__ T inf_b();
template <> __device__ __forceinline__ float inf_b<float>() { return __builtin_inff(); }
template <> __device__ __forceinline__ double inf_b<double>() { return __builtin_inf(); }

__device__ __forceinline__ float bmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double bmin(double a, double b) {  // the instruction: no quieting of NaN (none occur)
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// threadIdx.x hidden from loop-invariant code motion.  Every tile step derives
// its LDS and global offsets from the thread index; left alone, the compiler
// computes all of them once per graph and keeps them live through every phase,
// which took the kernel from about 115 to about 245 registers and made it spill
// at the 168 that three workgroups per CU allow.  Recomputing them per step
// costs a few instructions per tile.
__device__ __forceinline__ int opaque_tid() {
    int v = (int)threadIdx.x;
    asm volatile("" : "+v"(v));
    return v;
}

template <typename T, int W> struct VecT {
    typedef T type __attribute__((ext_vector_type(W)));
};

// One graph and its TB x TB tiles.  Thread (ty, tx) of the 16 x 16 layout owns
// rows ty + 16*ii (RM of them) and, per vector h, the VB contiguous columns from
// h*CS + tx*VB (RN columns in all).
template <typename T, int TB, bool PATH>
struct Graph {
    static constexpr int V = 16 / (int)sizeof(T);  // k per A-operand vector
    static constexpr int RM = TB / 16, RN = TB / 16;
    static constexpr int VB = RN < V ? RN : V;     // columns per B-operand vector
    static constexpr int HN = RN / VB, CS = TB / HN;
    static constexpr int ST = TB + V;              // LDS row stride (elements)
    using vecA = typename VecT<T, V>::type;
    using vecB = typename VecT<T, VB>::type;
    using lvA = typename VecT<uint16_t, V>::type;
    using lvB = typename VecT<uint16_t, VB>::type;

    T *D;
    int32_t *P;
    int n;

    __device__ static int row(int ty, int ii) { return ty + 16 * ii; }
    __device__ static int col(int tx, int h) { return h * CS + tx * VB; }

    // Lengths pass through canon() in path mode (lex_take_u's key needs +0.0);
    // labels are read as label + 1.  A guarded load reads the entry clamped into
    // the graph and then substitutes the padding value, so it has no branch and
    // all loads of a tile are in flight before the first wait.  (Indices within
    // one graph are below 4096^2; byte offsets are formed in 32 bits so that the
    // accesses take the scalar-base + 32-bit vector-offset form.)
    template <typename U> __device__ static U &elem(U *base, uint32_t idx) {
        return *(U *)((char *)base + idx * (uint32_t)sizeof(U));
    }
    __device__ uint32_t at(int i, int j) const { return (uint32_t)(min(i, n - 1) * n + min(j, n - 1)); }
    __device__ T ld_d(int i, int j) const {
        const T v = elem(D, at(i, j));
        const T pad = i == j ? (T)0 : inf_b<T>();
        return (i < n && j < n) ? (PATH ? canon(v) : v) : pad;
    }
    __device__ uint32_t ld_p(int i, int j) const {
        const uint32_t v = elem((uint16_t *)P, at(i, j));
        return (i < n && j < n) ? v : 0u;
    }
    // Tile (I0, J0) into LDS, row-major with stride ST (labels likewise): all
    // global loads first, then the LDS writes.  With kb1 > 0 (the last phase's
    // column-panel tile, whose columns are the round's k) each label + 1 is
    // stored as max(label + 1, kb1 + column), i.e. already combined with k + 1
    // for its column k = J0 + column, so the product does not redo it for every
    // entry of the tile it updates.
    __device__ void stage(T *s, uint16_t *l, int I0, int J0, uint32_t kb1 = 0) const {
        Staged st;
        fetch(st, I0, J0);
        put(st, s, l, I0, J0, kb1);
    }
    // stage() in two halves, so that a tile's loads can be in flight while the
    // previous tile's product runs: fetch issues the loads (the entry clamped
    // into the graph, labels packed two per word), put substitutes the padding
    // values and writes LDS.
    static constexpr int IT = TB * TB / NT;
    struct Staged {
        T v[IT];
        uint32_t w[PATH ? IT / 2 : 1];
    };
    __device__ void fetch(Staged &st, int I0, int J0) const {
        const int tid = opaque_tid();
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int q = tid + it * NT, rr = q / TB, cc = q % TB;
            st.v[it] = elem(D, at(I0 + rr, J0 + cc));
            if (PATH) {
                const uint32_t w = elem((uint16_t *)P, at(I0 + rr, J0 + cc));
                st.w[it / 2] = (it % 2) ? (st.w[it / 2] | (w << 16)) : w;
            }
        }
    }
    __device__ void put(const Staged &st, T *s, uint16_t *l, int I0, int J0, uint32_t kb1 = 0) const {
        const int tid = opaque_tid();
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int q = tid + it * NT, rr = q / TB, cc = q % TB;
            const int i = I0 + rr, j = J0 + cc;
            const bool in = i < n && j < n;
            const T pad = i == j ? (T)0 : inf_b<T>();
            s[rr * ST + cc] = in ? (PATH ? canon(st.v[it]) : st.v[it]) : pad;
            if (PATH) {
                const uint32_t w = in ? ((st.w[it / 2] >> (16 * (it % 2))) & 0xffffu) : 0u;
                l[rr * ST + cc] = (uint16_t)(kb1 ? max(w, kb1 + (uint32_t)cc) : w);
            }
        }
    }
    // The thread's entries of tile (I0, J0): from global memory ...
    __device__ void load(T (&d)[RM][RN], uint32_t (&p)[RM][RN], int I0, int J0, int tx, int ty) const {
#pragma unroll
        for (int ii = 0; ii < RM; ++ii)
#pragma unroll
            for (int h = 0; h < HN; ++h)
#pragma unroll
                for (int e = 0; e < VB; ++e) {
                    const int i = I0 + row(ty, ii), j = J0 + col(tx, h) + e;
                    d[ii][h * VB + e] = ld_d(i, j);
                    if (PATH) p[ii][h * VB + e] = ld_p(i, j);
                }
    }
    // ... lengths only, with label + 1 = 0 (last phase in path mode: every
    // candidate's label + 1 is above k0 >= 0, so an old label, whatever it is,
    // wins every tie with the old length exactly as 0 does, and an entry whose
    // word is still 0 after the product has not changed) ...
    __device__ void load_d0(T (&d)[RM][RN], uint32_t (&p)[RM][RN], int I0, int J0, int tx, int ty) const {
#pragma unroll
        for (int ii = 0; ii < RM; ++ii)
#pragma unroll
            for (int h = 0; h < HN; ++h)
#pragma unroll
                for (int e = 0; e < VB; ++e) {
                    d[ii][h * VB + e] = ld_d(I0 + row(ty, ii), J0 + col(tx, h) + e);
                    p[ii][h * VB + e] = 0u;
                }
    }
    // ... or from a staged copy.
    __device__ static void load_lds(T (&d)[RM][RN], uint32_t (&p)[RM][RN], const T *s, const uint16_t *l, int tx,
                                    int ty) {
#pragma unroll
        for (int ii = 0; ii < RM; ++ii)
#pragma unroll
            for (int h = 0; h < HN; ++h)
#pragma unroll
                for (int e = 0; e < VB; ++e) {
                    const int x = row(ty, ii) * ST + col(tx, h) + e;
                    d[ii][h * VB + e] = s[x];
                    if (PATH) p[ii][h * VB + e] = l[x];
                }
    }
    __device__ void store(const T (&d)[RM][RN], const uint32_t (&p)[RM][RN], int I0, int J0, int tx, int ty) const {
#pragma unroll
        for (int ii = 0; ii < RM; ++ii)
#pragma unroll
            for (int h = 0; h < HN; ++h)
#pragma unroll
                for (int e = 0; e < VB; ++e) {
                    const int i = I0 + row(ty, ii), j = J0 + col(tx, h) + e;
                    if (i < n && j < n) {
                        elem(D, (uint32_t)(i * n + j)) = d[ii][h * VB + e];
                        if (PATH) elem((uint16_t *)P, (uint32_t)(i * n + j)) = (uint16_t)p[ii][h * VB + e];
                    }
                }
    }

    // The entries that a last-phase product (from load_d0) decreased.
    __device__ void store_changed(const T (&d)[RM][RN], const uint32_t (&p)[RM][RN], int I0, int J0, int tx,
                                  int ty) const {
#pragma unroll
        for (int ii = 0; ii < RM; ++ii)
#pragma unroll
            for (int h = 0; h < HN; ++h)
#pragma unroll
                for (int e = 0; e < VB; ++e) {
                    const int i = I0 + row(ty, ii), j = J0 + col(tx, h) + e;
                    if (i < n && j < n && p[ii][h * VB + e] != 0u) {
                        elem(D, (uint32_t)(i * n + j)) = d[ii][h * VB + e];
                        elem((uint16_t *)P, (uint32_t)(i * n + j)) = (uint16_t)p[ii][h * VB + e];
                    }
                }
    }

    // (d, p) <- lexmin over k in the block of (d, p) and the candidates through k:
    // A[i][k] + B[k][j] with label max(LA[i][k], kbase + k, LB[k][j]) (labels +
    // 1; with PREMAX, LA already holds max(LA[i][k], kbase + k + 1), see
    // stage); distances only: d <- min(d, A[i][k] + B[k][j]), two k per v_min3.
    template <bool PREMAX = false>
    __device__ static void product(T (&d)[RM][RN], uint32_t (&p)[RM][RN], const T *A, const uint16_t *LA,
                                   const T *B, const uint16_t *LB, int kbase, int tx, int ty) {
#pragma unroll 2
        for (int kv = 0; kv < TB / V; ++kv) {
            vecA a[RM];
            lvA pa[PATH ? RM : 1];
#pragma unroll
            for (int ii = 0; ii < RM; ++ii) {
                a[ii] = *(const vecA *)(A + row(ty, ii) * ST + kv * V);
                if (PATH) pa[ii] = *(const lvA *)(LA + row(ty, ii) * ST + kv * V);
            }
            if constexpr (PATH) {
#pragma unroll
                for (int kk = 0; kk < V; ++kk) {
                    vecB b[HN];
                    lvB pb[HN];
#pragma unroll
                    for (int h = 0; h < HN; ++h) {
                        b[h] = *(const vecB *)(B + (kv * V + kk) * ST + col(tx, h));
                        pb[h] = *(const lvB *)(LB + (kv * V + kk) * ST + col(tx, h));
                    }
                    const uint32_t kg1 = (uint32_t)(kbase + kv * V + kk + 1);
#pragma unroll
                    for (int ii = 0; ii < RM; ++ii) {
                        const uint32_t mi = PREMAX ? (uint32_t)pa[ii][kk] : max((uint32_t)pa[ii][kk], kg1);
#pragma unroll
                        for (int h = 0; h < HN; ++h)
#pragma unroll
                            for (int e = 0; e < VB; ++e)
                                lex_take_u(d[ii][h * VB + e], p[ii][h * VB + e], a[ii][kk] + b[h][e],
                                           max(mi, (uint32_t)pb[h][e]));
                    }
                }
            } else {
#pragma unroll
                for (int kk = 0; kk < V; kk += 2) {
                    vecB b0[HN], b1[HN];
#pragma unroll
                    for (int h = 0; h < HN; ++h) {
                        b0[h] = *(const vecB *)(B + (kv * V + kk) * ST + col(tx, h));
                        b1[h] = *(const vecB *)(B + (kv * V + kk + 1) * ST + col(tx, h));
                    }
#pragma unroll
                    for (int ii = 0; ii < RM; ++ii)
#pragma unroll
                        for (int h = 0; h < HN; ++h)
#pragma unroll
                            for (int e = 0; e < VB; ++e) {
                                T &x = d[ii][h * VB + e];
                                x = bmin(bmin(x, a[ii][kk] + b0[h][e]), a[ii][kk + 1] + b1[h][e]);
                            }
                }
            }
        }
    }
};

// One graph, whole method, by the calling workgroup.  sa / sb (and la / lb) are
// LDS tiles of TB x ST elements.
template <typename T, int TB, bool PATH>
__device__ void solve_graph(Graph<T, TB, PATH> g, T *sa, T *sb, uint16_t *la, uint16_t *lb) {
    using G = Graph<T, TB, PATH>;
    constexpr int RM = G::RM, RN = G::RN, VB = G::VB, HN = G::HN, ST = G::ST;
    int tx, ty;  // re-derived per step (opaque_tid)
    auto thread_xy = [&]() {
        const int tid = opaque_tid();
        tx = tid % 16;
        ty = tid / 16;
    };
    const int n = g.n;
    if (PATH) {
        for (uint32_t x = threadIdx.x; x < (uint32_t)(n * n); x += NT) G::elem((uint16_t *)g.P, x) = 0;  // no label
    }
    __syncthreads();
    const int R = (n + TB - 1) / TB;
    T d[RM][RN];
    uint32_t p[RM][RN];
    // The tile a step stages into sb / lb (a phase 2/3 panel tile, or a last-phase
    // row-panel tile) is loaded into registers (nb) while the previous step's
    // work runs, and written to LDS after that step's barrier.  Every tile loaded
    // early is final by then: panel tiles change only in their own step, and
    // row-panel tiles are final after phases 2/3, whose steps all end with a
    // barrier.
    typename G::Staged nb;
    for (int r = 0; r < R; ++r) {
        const int k0 = r * TB;
        thread_xy();
        const int T23 = 2 * (R - 1), T4 = (R - 1) * (R - 1);
        auto panel_of = [&](int t, int &I0, int &J0) {
            const bool rowp = t < R - 1;
            const int o0 = rowp ? t : t - (R - 1);
            const int o = o0 < r ? o0 : o0 + 1;
            I0 = rowp ? k0 : o * TB;
            J0 = rowp ? o * TB : k0;
        };
        auto col_of = [&](int t) { const int bj0 = t % (R - 1); return (bj0 < r ? bj0 : bj0 + 1) * TB; };
        // Phase 1: close the diagonal block in LDS.  Row k and column k do not
        // change at step k (D[k][k] = 0: their candidates equal the current
        // value with a label that is not smaller), so updating in place while
        // others read them is safe; one barrier per k orders the steps.
        g.stage(sa, la, k0, k0);
        __syncthreads();
        G::load_lds(d, p, sa, la, tx, ty);
        if (T23 > 0) {  // the first panel tile, under phase 1
            int I0, J0;
            panel_of(0, I0, J0);
            g.fetch(nb, I0, J0);
        }
        for (int k = 0; k < TB; ++k) {
            T a[RM];
            uint32_t pa[RM];
#pragma unroll
            for (int ii = 0; ii < RM; ++ii) {
                a[ii] = sa[G::row(ty, ii) * ST + k];
                if (PATH) pa[ii] = max((uint32_t)la[G::row(ty, ii) * ST + k], (uint32_t)(k0 + k + 1));
            }
#pragma unroll
            for (int h = 0; h < HN; ++h) {
                const typename G::vecB b = *(const typename G::vecB *)(sa + k * ST + G::col(tx, h));
                typename G::lvB pb;
                if (PATH) pb = *(const typename G::lvB *)(la + k * ST + G::col(tx, h));
#pragma unroll
                for (int ii = 0; ii < RM; ++ii)
#pragma unroll
                    for (int e = 0; e < VB; ++e) {
                        T &x = d[ii][h * VB + e];
                        uint32_t &y = p[ii][h * VB + e];
                        const T s = a[ii] + b[e];
                        const int at = G::row(ty, ii) * ST + G::col(tx, h) + e;
                        if (PATH) {
                            const T x0 = x;
                            const uint32_t y0 = y;
                            lex_take_u(x, y, s, max(pa[ii], (uint32_t)pb[e]));
                            if (x != x0 || y != y0) {
                                sa[at] = x;
                                la[at] = (uint16_t)y;
                            }
                        } else if (s < x) {
                            x = s;
                            sa[at] = s;
                        }
                    }
            }
            __syncthreads();
        }
        g.store(d, p, k0, k0, tx, ty);
        // The closed diagonal block stays in sa / la for the panels.
        // Phases 2 and 3: each panel tile is one product with the closed block
        // (the row panel as its right operand, the column panel as its left).
        for (int t = 0; t < T23; ++t) {
            thread_xy();
            const bool rowp = t < R - 1;
            int I0, J0;
            panel_of(t, I0, J0);
            g.put(nb, sb, lb, I0, J0);  // the old panel tile
            __syncthreads();
            G::load_lds(d, p, sb, lb, tx, ty);
            if (t + 1 < T23) {  // the next panel tile, or the first row-panel tile of phase 4
                int I1, J1;
                panel_of(t + 1, I1, J1);
                g.fetch(nb, I1, J1);
            } else {
                g.fetch(nb, k0, col_of(0));
            }
            G::product(d, p, rowp ? sa : sb, rowp ? la : lb, rowp ? sb : sa, rowp ? lb : la, k0, tx, ty);
            g.store(d, p, I0, J0, tx, ty);
            __syncthreads();
        }
        // Phase 4: every other tile, product of its final column-panel tile
        // (staged once per tile row) and row-panel tile; with labels, only the
        // entries that decrease are read back and written.
        for (int t = 0; t < T4; ++t) {
            thread_xy();
            const int bi0 = t / (R - 1), bj0 = t % (R - 1);
            const int bi = bi0 < r ? bi0 : bi0 + 1;
            const int I0 = bi * TB, J0 = col_of(t);
            if (bj0 == 0) g.stage(sa, la, I0, k0, (uint32_t)(k0 + 1));
            g.put(nb, sb, lb, k0, J0);
            if (PATH)
                g.load_d0(d, p, I0, J0, tx, ty);
            else
                g.load(d, p, I0, J0, tx, ty);
            __syncthreads();
            if (t + 1 < T4) g.fetch(nb, k0, col_of(t + 1));
            G::template product<true>(d, p, sa, la, sb, lb, k0, tx, ty);
            if (PATH)
                g.store_changed(d, p, I0, J0, tx, ty);
            else
                g.store(d, p, I0, J0, tx, ty);
            __syncthreads();
        }
    }
    if (PATH) {
        // Every thread's last label stores must be visible before any thread
        // reads them back: with one round (n <= TB) nothing after phase 1's
        // store has a barrier.
        __syncthreads();
        // Widen the 16-bit labels + 1 to 32-bit labels in place, last chunk
        // first.  Chunk [a, a + CH) reads bytes [2a, 2a + 2CH) and writes
        // [4a, 4a + 4CH): the words of lower chunks, not yet read, lie below
        // 2a, and only chunk 0 writes over words of its own, after the barrier
        // that follows its reads.
        constexpr int PER = 8, CH = PER * NT;
        const uint32_t nn = (uint32_t)(n * n);
        for (int c = (int)((nn + CH - 1) / CH) - 1; c >= 0; --c) {
            const uint32_t a = (uint32_t)c * CH;
            uint32_t v[PER];
#pragma unroll
            for (int it = 0; it < PER; ++it) {
                const uint32_t x = a + it * NT + threadIdx.x;
                v[it] = x < nn ? G::elem((uint16_t *)g.P, x) : 0u;
            }
            __syncthreads();
#pragma unroll
            for (int it = 0; it < PER; ++it) {
                const uint32_t x = a + it * NT + threadIdx.x;
                if (x < nn) G::elem(g.P, x) = (int32_t)v[it] - 1;
            }
        }
        __syncthreads();
    }
}

// Workgroups per CU that the LDS of k_batched admits (160 KB per CU): the
// register budget is sized to match.
template <typename T, bool PATH>
constexpr int batched_wgs_per_cu() {
    constexpr int st = 64 + 16 / (int)sizeof(T);
    constexpr int bytes = 2 * 64 * st * ((int)sizeof(T) + (PATH ? 2 : 0));
    constexpr int w = 160 * 1024 / (bytes + 64);
    return w < 1 ? 1 : (w > 4 ? 4 : w);
}

// Persistent batched kernel.  jobs[0] holds the queue counter (0 when the launch
// starts), jobs[1] the number of jobs, and jobs[2 + 2q], jobs[3 + 2q] the offset
// and n of queue slot q.  A graph uses 32 x 32 tiles when n <= small_max_n;
// above, its size class c = (n - 1) / 32 decides: 64 x 64 tiles when c >= 64 or
// bit c of tile64 is set (the tuning table holds the measured choice per class),
// 32 x 32 otherwise.  Both share the LDS arrays, sized for 64.
template <typename T, bool PATH>
__global__ void __launch_bounds__(NT, (batched_wgs_per_cu<T, PATH>())) k_batched(T *__restrict__ dist, int32_t *__restrict__ path,
                                               int64_t *__restrict__ jobs, int small_max_n, uint64_t tile64) {
    constexpr int ST = Graph<T, 64, PATH>::ST;
    __shared__ __attribute__((aligned(16))) T sa[64 * ST];
    __shared__ __attribute__((aligned(16))) T sb[64 * ST];
    __shared__ __attribute__((aligned(16))) uint16_t la[PATH ? 64 * ST : 8];  // labels + 1
    __shared__ __attribute__((aligned(16))) uint16_t lb[PATH ? 64 * ST : 8];
    __shared__ int s_job;
    unsigned long long *counter = (unsigned long long *)jobs;
    const int njobs = __builtin_amdgcn_readfirstlane((int)jobs[1]);
    for (;;) {
        if (threadIdx.x == 0) s_job = (int)atomicAdd(counter, 1ull);
        __syncthreads();
        const int q = __builtin_amdgcn_readfirstlane(s_job);  // uniform: graph bases in scalar registers
        __syncthreads();
        if (q >= njobs) return;
        const int64_t off0 = jobs[2 + 2 * q];
        const int64_t off = ((int64_t)__builtin_amdgcn_readfirstlane((int)(off0 >> 32)) << 32) |
                            (uint32_t)__builtin_amdgcn_readfirstlane((int)off0);
        const int n = __builtin_amdgcn_readfirstlane((int)jobs[3 + 2 * q]);
        const int c = (n - 1) >> 5;
        const bool small = (n <= small_max_n) || (c < 64 && !((tile64 >> c) & 1));
        if (small) {
            Graph<T, 32, PATH> g{dist + off, PATH ? path + off : nullptr, n};
            solve_graph<T, 32, PATH>(g, sa, sb, la, lb);
        } else {
            Graph<T, 64, PATH> g{dist + off, PATH ? path + off : nullptr, n};
            solve_graph<T, 64, PATH>(g, sa, sb, la, lb);
        }
    }
}

// Job table from device arrays of vertex counts nv[batch] and element offsets
// off[batch], in the layout k_batched reads: [0] the queue counter (set to 0),
// [1] the number of jobs, then (offset, n) per queue slot in order of
// decreasing n (longest job first).  A graph whose n is outside [1, BJ_MAXN] or
// whose offset is negative gets no slot (it is not solved and not touched).
// One workgroup, a counting sort on n: a histogram in LDS, its exclusive scan
// from the largest n down, then every graph takes the next slot of its n (the
// order among graphs of equal n is arbitrary; each is solved independently).
constexpr int BJ_NT = 1024, BJ_MAXN = 4096, BJ_PER = BJ_MAXN / BJ_NT;
__global__ void __launch_bounds__(BJ_NT) k_build_jobs(const int32_t *__restrict__ nv, const int64_t *__restrict__ off,
                                                     int batch, int64_t *__restrict__ jobs) {
    __shared__ int cnt[BJ_MAXN + 1];
    __shared__ int part[BJ_NT];
    const int t = threadIdx.x;
    for (int x = t; x <= BJ_MAXN; x += BJ_NT) cnt[x] = 0;
    __syncthreads();
    for (int b = t; b < batch; b += BJ_NT) {
        const int n = nv[b];
        if (n >= 1 && n <= BJ_MAXN && off[b] >= 0) atomicAdd(&cnt[n], 1);
    }
    __syncthreads();
    // Thread t owns bins n = BJ_MAXN - BJ_PER t - q, q < BJ_PER (n = 1 .. BJ_MAXN
    // from thread BJ_NT - 1 up to thread 0); an inclusive scan of the per-thread
    // sums (Hillis-Steele in LDS) gives each thread the count of larger n.
    int local[BJ_PER], sum = 0;
#pragma unroll
    for (int q = 0; q < BJ_PER; ++q) {
        local[q] = cnt[BJ_MAXN - BJ_PER * t - q];
        sum += local[q];
    }
    part[t] = sum;
    __syncthreads();
    for (int d = 1; d < BJ_NT; d <<= 1) {
        const int v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - sum;
#pragma unroll
    for (int q = 0; q < BJ_PER; ++q) {
        cnt[BJ_MAXN - BJ_PER * t - q] = run;  // first slot of this n
        run += local[q];
    }
    if (t == BJ_NT - 1) {
        jobs[0] = 0;
        jobs[1] = part[t];
    }
    __syncthreads();
    for (int b = t; b < batch; b += BJ_NT) {
        const int n = nv[b];
        const int64_t o = off[b];
        if (n >= 1 && n <= BJ_MAXN && o >= 0) {
            const int slot = atomicAdd(&cnt[n], 1);
            jobs[2 + 2 * slot] = o;
            jobs[3 + 2 * slot] = n;
        }
    }
}

// The job table of fw_apsp_batched_device_noalloc, for callers that cannot
// allocate: one per GPU, held until the process ends.  Host code never passes
// the array's name to a kernel: each device's address comes from
// hipGetSymbolAddress (noalloc_jobs below).
static __device__ __align__(256) int64_t scratch[2 + 2 * (size_t)kNoAllocMaxBatch];

}  // namespace

template <typename T>
hipError_t launch_batched(T *dist, int32_t *path, int64_t *jobs, BatchedTiles tiles, int grid, hipStream_t s) {
    if (path)
        hipLaunchKernelGGL((k_batched<T, true>), dim3(grid), dim3(NT), 0, s, dist, path, jobs, tiles.small_max_n,
                           tiles.tile64);
    else
        hipLaunchKernelGGL((k_batched<T, false>), dim3(grid), dim3(NT), 0, s, dist, path, jobs, tiles.small_max_n,
                           tiles.tile64);
    return hipGetLastError();
}

hipError_t launch_build_jobs(const int32_t *nv, const int64_t *off, int batch, int64_t *jobs, hipStream_t s) {
    hipLaunchKernelGGL(k_build_jobs, dim3(1), dim3(BJ_NT), 0, s, nv, off, batch, jobs);
    return hipGetLastError();
}

// Device address of `scratch` on the current device, looked up once per device
// (with that device current) and kept; later calls only read the table.
hipError_t noalloc_jobs(int dev, int64_t **out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static int64_t *addr[kMaxDevices] = {};
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = (int64_t *)p;
    }
    *out = addr[dev];
    return hipSuccess;
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
template hipError_t launch_batched<float>(float *, int32_t *, int64_t *, BatchedTiles, int, hipStream_t);
template hipError_t launch_batched<double>(double *, int32_t *, int64_t *, BatchedTiles, int, hipStream_t);

}  // namespace fw
