// fw_kernels.hip -- gfx950 kernels of the blocked Floyd-Warshall method.
//
// One round r (k-block K = [r*TB, (r+1)*TB)) is three launches (paper Sect. 2.2,
// "Blocked FW Algorithm"; the GPU split into one kernel for the diagonal block,
// one for both panels and one for the rest follows Sect. 3.2):
//   k_phase1   the diagonal block, TB sequential k-steps in LDS;
//   k_phase23  the row panel D[K, J] and the column panel D[I, K], as min-plus
//              products with the closed diagonal block (no sequential k-steps);
//   k_phase4   every other tile, a register-blocked min-plus product of the final
//              column panel D[I, K] and row panel D[K, J], both staged in LDS;
//   k_phase4w  the same product with one row of the column panel per wave and
//              k, read into scalar registers, and only the row panel in LDS.
// Every kernel is written for float32 and float64; phases 1-3, k_phase4 and the
// label resolution also exist for binary16 (_Float16), where k_phase4 works on
// pairs of columns with packed half-precision instructions.
//
// Path matrix: every candidate through k carries the label
// (length, max(P[i][k], k, P[k][j])); an entry takes a candidate whose label is
// lexicographically smaller.  This reproduces, whatever the block size, what the
// classic loop with a strict test stores (the smallest possible largest interior
// vertex over all shortest paths).  Phases 1-3 apply that rule directly.  The
// last phase defers it: an entry that strictly improves in round r is only
// marked "pending from round r" in a separate array L (L = r + 1; 0 means the
// label in P is current), and k_resolve computes all pending labels in one pass
// after the last round (see there for why the final distances suffice).  While
// an entry is pending, P still holds an older label; every label set before
// round r is below the round's first vertex k0, and so is the pending one, so
// phases 1-3 of later rounds treat the stale value exactly as they would treat
// the true label: it never wins a max() against k and never makes a tie win.
// Phases 1-3 clear L for every entry whose (length, label) they change.
//
// All arithmetic is on the vector ALU: the min-plus product is not a ring
// contraction, so matrix cores do not apply.
// The tile selections run on the device too (defined before fw_internal.h
// includes them).
#define FW_TILE_FN __host__ __device__ __forceinline__
#include "fw_internal.h"
#include "fw_lex.h"
#include "fw_device.h"

#include <limits.h>
#include <type_traits>

namespace fw {
namespace {

// ---------------------------------------------------------------------------
// Phase 1: close the diagonal block.  The block and its P stay in LDS; thread
// (ty, tx) owns rows ty + 16*ii and columns tx + 16*jj.  At step k, row k and
// column k of the block are unchanged by the update (D[k][k] = 0, so every
// candidate for them equals the current value with a label that is not
// smaller), hence updating in place while other threads read them is safe; one
// barrier per k orders step k's writes before step k+1's reads.  The k-steps
// are a dependent chain on one CU; the block runs with TS x TS threads: 1024
// (few entries each, every SIMD busy within a step) or 256 (one wave per SIMD).
// The 256-thread form is the one that fits on a CU beside the last phase's
// workgroups when it runs concurrently with them (the lookahead schedules):
// 1024 threads need four waves on every SIMD of one CU, i.e. a CU that two or
// more last-phase workgroups have left, which seldom happens while the
// last-phase launch is still placing workgroups.  It is used for 64-deep
// float32 and float64 blocks, whose fused last-phase launches run beside
// phases 1-3 of the next pair (measured at n = 16384, float32 with P: phase 1
// waited 522 us for a CU beside a launch of six workgroups per CU, and took
// 69 us in the 256-thread form).  binary16 and 32-deep blocks keep 1024 threads:
// their last-phase launches are short, and phase 1's own duration counts.
template <typename T, int TB> constexpr int p1_ts() { return (sizeof(T) == 8 || (sizeof(T) == 4 && TB == 64)) ? 16 : 32; }
template <typename T, int TB, bool PATH, int TS>
__global__ void __launch_bounds__(TS *TS) k_phase1(T *__restrict__ D, int32_t *__restrict__ P,
                                                  uint16_t *__restrict__ L, int64_t ld, int r) {
    constexpr int RM = TB / TS, ST = TB + 1;
    static_assert(RM * TS == TB, "phase 1 thread layout");
    __shared__ T sd[TB * ST];
    __shared__ uint32_t sp[PATH ? TB * ST : 1];  // labels + 1
    const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
    const int64_t k0 = (int64_t)r * TB;
    static_assert(RM * RM <= 32, "phase 1 change mask");
    T d[RM][RM];
    uint32_t p[RM][RM];
    uint32_t changed = 0;  // bit ii * RM + jj: entry (ii, jj) changed
#pragma unroll
    for (int ii = 0; ii < RM; ++ii)
#pragma unroll
        for (int jj = 0; jj < RM; ++jj) {
            const int row = ty + TS * ii, col = tx + TS * jj;
            const int64_t g = (k0 + row) * ld + k0 + col;
            d[ii][jj] = PATH ? canon(D[g]) : D[g];
            sd[row * ST + col] = d[ii][jj];
            if (PATH) {
                p[ii][jj] = (uint32_t)(P[g] + 1);
                sp[row * ST + col] = p[ii][jj];
            }
        }
    __syncthreads();
    for (int k = 0; k < TB; ++k) {
        T a[RM], b[RM];
        uint32_t pa[RM], pb[RM];
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
        const uint32_t kg1 = (uint32_t)(k0 + k + 1);
#pragma unroll
        for (int ii = 0; ii < RM; ++ii)
#pragma unroll
            for (int jj = 0; jj < RM; ++jj) {
                const T s = a[ii] + b[jj];
                const int idx = (ty + TS * ii) * ST + tx + TS * jj;
                if (PATH) {
                    const T d0 = d[ii][jj];
                    const uint32_t p0 = p[ii][jj];
                    lex_take_u(d[ii][jj], p[ii][jj], s, max(max(pa[ii], pb[jj]), kg1));
                    if (p[ii][jj] != p0 || d[ii][jj] != d0) {
                        sd[idx] = d[ii][jj];
                        sp[idx] = p[ii][jj];
                        changed |= 1u << (ii * RM + jj);
                    }
                } else if (s < d[ii][jj]) {
                    d[ii][jj] = s;
                    sd[idx] = s;
                    changed |= 1u << (ii * RM + jj);
                }
            }
        __syncthreads();
    }
#pragma unroll
    for (int ii = 0; ii < RM; ++ii)
#pragma unroll
        for (int jj = 0; jj < RM; ++jj) {
            if (!((changed >> (ii * RM + jj)) & 1)) continue;
            const int64_t g = (k0 + ty + TS * ii) * ld + k0 + tx + TS * jj;
            D[g] = d[ii][jj];
            if (PATH) {
                P[g] = (int32_t)p[ii][jj] - 1;
                L[g] = 0;
            }
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
__global__ void __launch_bounds__(NT) k_phase23(T *__restrict__ D, int32_t *__restrict__ P, uint16_t *__restrict__ L,
                                               int64_t ld, int r, int nb) {
    // The operands are staged KC = 32 values of k at a time (33.5 KB of LDS with
    // labels for TB = 64 instead of 66.6 KB), so that a workgroup of this kernel
    // fits on a CU beside three of the last phase's when the two run
    // concurrently (pairs-with-lookahead schedule).
    constexpr int TS = 16, RM = TB / TS, KC = TB < 32 ? TB : 32, SA = KC + 1, SB = TB + 1;
    __shared__ T sa[TB * SA];  // A chunk: rows x KC
    __shared__ T sb[KC * SB];  // B chunk: KC x columns
    __shared__ uint32_t spa[PATH ? TB * SA : 1];  // labels + 1
    __shared__ uint32_t spb[PATH ? KC * SB : 1];
    const int w = blockIdx.x;
    const bool rowp = w < nb - 1;
    const int t = rowp ? w : w - (nb - 1);
    const int o = t < r ? t : t + 1;
    const int64_t k0 = (int64_t)r * TB;
    const int64_t I0 = rowp ? k0 : (int64_t)o * TB;
    const int64_t J0 = rowp ? (int64_t)o * TB : k0;
    // A = D[I0.., K] and B = D[K, J0..]: for a row panel A is the closed diagonal
    // block and B the old tile, for a column panel the other way round.
    const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
    T d[RM][RM];
    uint32_t p[RM][RM];
#pragma unroll
    for (int ii = 0; ii < RM; ++ii)
#pragma unroll
        for (int jj = 0; jj < RM; ++jj) {
            const int64_t g = (I0 + ty + TS * ii) * ld + J0 + tx + TS * jj;
            d[ii][jj] = PATH ? canon(D[g]) : D[g];
            if (PATH) p[ii][jj] = (uint32_t)(P[g] + 1);
        }
    for (int kc = 0; kc < TB; kc += KC) {
        if (kc) __syncthreads();  // every thread is done with the previous chunk
        for (int q = threadIdx.x; q < TB * KC; q += NT) {
            const int rr = q / KC, cc = q % KC;
            const int64_t g = (I0 + rr) * ld + k0 + kc + cc;
            sa[rr * SA + cc] = PATH ? canon(D[g]) : D[g];
            if (PATH) spa[rr * SA + cc] = (uint32_t)(P[g] + 1);
        }
        for (int q = threadIdx.x; q < KC * TB; q += NT) {
            const int rr = q / TB, cc = q % TB;
            const int64_t g = (k0 + kc + rr) * ld + J0 + cc;
            sb[rr * SB + cc] = PATH ? canon(D[g]) : D[g];
            if (PATH) spb[rr * SB + cc] = (uint32_t)(P[g] + 1);
        }
        __syncthreads();
        for (int k = 0; k < KC; ++k) {
            T a[RM], b[RM];
            uint32_t pa[RM], pb[RM];
#pragma unroll
            for (int ii = 0; ii < RM; ++ii) {
                a[ii] = sa[(ty + TS * ii) * SA + k];
                if (PATH) pa[ii] = spa[(ty + TS * ii) * SA + k];
            }
#pragma unroll
            for (int jj = 0; jj < RM; ++jj) {
                b[jj] = sb[k * SB + tx + TS * jj];
                if (PATH) pb[jj] = spb[k * SB + tx + TS * jj];
            }
            const uint32_t kg1 = (uint32_t)(k0 + kc + k + 1);
#pragma unroll
            for (int ii = 0; ii < RM; ++ii)
#pragma unroll
                for (int jj = 0; jj < RM; ++jj) {
                    const T s = a[ii] + b[jj];
                    if (PATH)
                        lex_take_u(d[ii][jj], p[ii][jj], s, max(max(pa[ii], pb[jj]), kg1));
                    else
                        d[ii][jj] = vmin(d[ii][jj], s);
                }
        }
    }
    // Store the entries that changed.  The old values are read again rather
    // than kept in registers through the k-loop (which would cost the kernel
    // its fit beside the last phase's workgroups): nothing else writes the tile
    // while this workgroup runs, so they are still in memory.
#pragma unroll
    for (int ii = 0; ii < RM; ++ii)
#pragma unroll
        for (int jj = 0; jj < RM; ++jj) {
            const int64_t g = (I0 + ty + TS * ii) * ld + J0 + tx + TS * jj;
            const T d0 = PATH ? canon(D[g]) : D[g];
            if (d[ii][jj] == d0 && (!PATH || p[ii][jj] == (uint32_t)(P[g] + 1))) continue;
            D[g] = d[ii][jj];
            if (PATH) {
                P[g] = (int32_t)p[ii][jj] - 1;
                L[g] = 0;
            }
        }
}

// Last-phase LDS panels are filled by direct global-to-LDS loads: one wave
// instruction moves 64 16-byte vectors and lands lane l's vector at the wave's
// LDS address + 16 l, so each panel is laid out in whole 64-vector slots.  A
// rows are padded by one vector (its slot is filled with a harmless reload) so
// that the rows a wave reads start in different banks.
template <typename T>
constexpr int p4_slots_a(int BM, int kc) { return (BM * (kc / (16 / (int)sizeof(T)) + 1) + 63) / 64 * 64; }
template <typename T>
constexpr int p4_slots_b(int BN, int kc) { return (kc * (BN / (16 / (int)sizeof(T))) + 63) / 64 * 64; }

// Panel buffers: with two, chunk c + 1 of k loads while chunk c is swept; with
// one, each chunk's loads are all issued at once and waited for before its
// sweep.  float32 and float64 use one: at six (float32) or four (float64)
// workgroups per CU the other workgroups hide a chunk's load, and one buffer
// allows chunks twice as deep for the same LDS, i.e. half the barriers
// (measured at n = 16384, two buffers of 16-deep chunks -> one of 32: float32
// with P 173.3 -> 172.1 ms, distances 145.0 -> 143.5 ms, float64 unchanged).
// binary16 keeps two.
template <typename T>
constexpr int p4_buffers() { return is_half_v<T> ? 2 : 1; }

// k per staged chunk of the last phase's panels: the whole block, halved while
// the buffers take more than the LDS share of the workgroups per CU that the
// kernel's registers allow: 40 KB (four of the 160 KB), and 32 KB (five or more)
// for the float32 64 x 64 tile.
template <typename T>
constexpr int p4_kchunk(int TB, int BM, int BN) {
    int kc = TB;
    const int v = 16 / (int)sizeof(T);
    const int cap = (sizeof(T) == 4 && BM == 64 && BN == 64) ? 32 * 1024 : 40 * 1024;
    while (kc > 2 * v && p4_buffers<T>() * (p4_slots_a<T>(BM, kc) + p4_slots_b<T>(BN, kc)) * 16 > cap) kc /= 2;
    return kc;
}

// One 16-byte direct load from global memory into LDS for this lane.  lds must
// be the same for every lane of the wave (it becomes the wave's base address);
// the vector lands at lds + 16 * lane.  Completion is counted by vmcnt.
__device__ __forceinline__ void lds_load16(const void *g, void *lds) {
    __builtin_amdgcn_global_load_lds((__attribute__((address_space(1))) void *)g,
                                     (__attribute__((address_space(3))) void *)lds, 16, 0, 0);
}
// The value itself, in a register the compiler cannot see through: a 32-bit
// offset stays 32 bits at its use, so the load takes the scalar-base plus
// 32-bit-offset form instead of a hoisted 64-bit address per lane.
__device__ __forceinline__ uint32_t opaque(uint32_t x) {
    asm volatile("" : "+v"(x));
    return x;
}
// Wait until this wave's direct loads (every vector memory load) have landed:
// s_waitcnt with vmcnt 0 (bits 3:0 and 15:14) and the other counters at their
// maxima (expcnt 7 in bits 6:4, lgkmcnt 15 in bits 11:8), i.e. no wait on them.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// ---------------------------------------------------------------------------
// Phase 4: C = D[I0:I0+BM, J0:J0+BN] <- min(C, D[I, K] (x) D[K, J]) for every
// tile outside block row / column r.  The panels are final for the round, so the
// k-loop has no barrier (beyond one per staged chunk of KC values of k, see
// p4_kchunk).  Thread layout: TX x TY threads, each owning an RM x RN
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
// Path mode: before this round every label of a phase-4 entry is below
// k0 = r*TB (its paths use interior vertices of earlier blocks only), and every
// candidate through block r has a label of at least k0.  So a candidate that
// merely ties the old length never changes the label, and an entry that strictly
// improves gets a label decided entirely by this round's candidates: it is
// marked pending (L = r + 1) and resolved by k_resolve.  Each such mark is
// written on its own (a 2-byte store under the entry's own condition), so this
// phase never reads L.
template <typename T, int TB, int BM, int BN, bool PATH, bool BAND, bool FUSE = false>
__global__ void __launch_bounds__(NT) k_phase4(T *__restrict__ D, uint16_t *__restrict__ L, int64_t ld, int r,
                                              TileSel sel) {
    constexpr int RM = BM / 16, RN = BN / 16;  // 16 x 16 threads
    using vec = typename V16<T>::type;
    constexpr int V = V16<T>::n;
    constexpr int TX = BN / RN, TY = NT / TX;
    static_assert(TY * RM == BM, "tile rows");
    static_assert(RN % V == 0, "micro-tile width");
    constexpr int HN = RN / V, CS = BN / HN;
    // The panels of a round are staged KC values of k at a time in one or two
    // buffers (p4_buffers; KC = TB unless the buffers would take more than the
    // LDS share in p4_kchunk).
    constexpr int KC = p4_kchunk<T>(TB, BM, BN);
    static_assert(TB % KC == 0 && KC % V == 0, "k chunk");
    constexpr int AST = KC + V;
    constexpr int KV = KC / V;  // vectors of k per A row
    constexpr int SA = p4_slots_a<T>(BM, KC), SB = p4_slots_b<T>(BN, KC);
    constexpr int CPR = TB / KC, NCH = (FUSE ? 2 : 1) * CPR;  // chunks per round, per launch
    // Old C values are requested before the panel loads (binary16, up to 128
    // bytes per thread) or after the k-loop.  float32 and float64 load them
    // after: the registers a prefetch holds through the k-loop cost a workgroup
    // per CU (float32 64 x 64 tile: 100 VGPRs, four workgroups, with it; 76 and
    // six without), and the extra workgroups hide more latency (measured at
    // n = 16384 with the direct-load staging: float32 with P 178.8 -> 174.4 ms,
    // distances 146.3 -> 144.7 ms).
    constexpr bool PREFETCH_C = is_half_v<T> && RM * RN * (int)sizeof(T) <= 128;
    // float64 sweeps one vector of k per loop iteration: unrolled twice, the
    // compiler's schedule took the fused launch from four waves per SIMD to three.
    constexpr int SWEEP_UNROLL = sizeof(T) == 8 ? 1 : 2;

    // Two buffers as distinct LDS objects, each named statically where it is
    // used: the compiler can then tell the next chunk's direct loads from the
    // current chunk's reads and does not wait for the former before the latter.
    constexpr int NBUF = p4_buffers<T>();
    __shared__ __attribute__((aligned(16))) T As0[SA * V], As1[NBUF == 2 ? SA * V : 1];
    __shared__ __attribute__((aligned(16))) T Bs0[SB * V], Bs1[NBUF == 2 ? SB * V : 1];

    int bi, bj;
    if (!select_tile<BAND>(sel, blockIdx.x, bi, bj)) return;
    const int64_t I0 = (int64_t)bi * BM, J0 = (int64_t)bj * BN, k0 = (int64_t)r * TB;

    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    const int64_t toff = (I0 + ty) * ld + J0 + tx * V;  // this thread's first entry of the tile
    auto c_ptr = [&](int ii, int h) { return D + toff + (int64_t)(TY * ii) * ld + h * CS; };

    auto l_ptr = [&](int ii, int h) { return L + toff + (int64_t)(TY * ii) * ld + h * CS; };
    vec c[RM][HN];
    if constexpr (PREFETCH_C) {
        // Old C values, requested first so their latency overlaps the panel
        // loads.
#pragma unroll
        for (int ii = 0; ii < RM; ++ii)
#pragma unroll
            for (int h = 0; h < HN; ++h) c[ii][h] = *(const vec *)c_ptr(ii, h);
    }

    // Start loading columns kb + kc .. kb + kc + KC - 1 of the column panel
    // D[I, K] and the same rows of the row panel D[K, J] into buffers nA, nB:
    // wave w issues slot groups w, w + 4, ...  A lane's byte offset from the
    // chunk's first element is the same for every chunk (below 2^32: fewer
    // than 128 rows of ld <= 2^20 elements of at most 8 bytes, the host's limit
    // on n); a padding or overflow slot reloads the chunk's first vector.
    const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
    const uint32_t lane = (uint32_t)tid % 64;
    constexpr int WPG = NT / 64, GA = SA / 64, GB = SB / 64;
    constexpr int MA = (GA + WPG - 1) / WPG, MB = (GB + WPG - 1) / WPG;
    uint32_t offa[MA], offb[MB];
#pragma unroll
    for (int t = 0; t < MA; ++t) {
        const uint32_t q = (uint32_t)(wave + t * WPG) * 64 + lane, row = q / (KV + 1), kv = q % (KV + 1);
        offa[t] = (q < (uint32_t)(BM * (KV + 1)) && kv < (uint32_t)KV) ? (uint32_t)((row * ld + kv * V) * sizeof(T)) : 0u;
    }
#pragma unroll
    for (int t = 0; t < MB; ++t) {
        const uint32_t q = (uint32_t)(wave + t * WPG) * 64 + lane, krow = q / (BN / V), cv = q % (BN / V);
        offb[t] = q < (uint32_t)(KC * (BN / V)) ? (uint32_t)((krow * ld + cv * V) * sizeof(T)) : 0u;
    }
    auto issue = [&](T *nA, T *nB, int64_t kb, int kc) {
        const char *ga = (const char *)(D + I0 * ld + kb + kc);
#pragma unroll
        for (int t = 0; t < MA; ++t)
            if (wave + t * WPG < GA) lds_load16(ga + opaque(offa[t]), nA + (wave + t * WPG) * 64 * V);
        const char *gb = (const char *)(D + (kb + kc) * ld + J0);
#pragma unroll
        for (int t = 0; t < MB; ++t)
            if (wave + t * WPG < GB) lds_load16(gb + opaque(offb[t]), nB + (wave + t * WPG) * 64 * V);
    };
    // After a chunk has landed: in a tile wider than the block, the block's own
    // rows (columns) of the staged panels become +inf.  A tile no wider than the
    // block never needs it (every selection then skips the block's tile rows and
    // columns: nsr, nsc >= 1), and the test is left out of the code.
    auto mask = [&](T *A, T *B, int64_t kb) {
        const bool mask_rows = BM > TB && sel.nsr == 0 && (I0 <= kb) && (kb < I0 + BM);
        const bool mask_cols = BN > TB && sel.nsc == 0 && (J0 <= kb) && (kb < J0 + BN);
        if (!mask_rows && !mask_cols) return;
        const vec vinf = inf_v<T>();
        if (mask_rows)
            for (int q = tid; q < TB * KV; q += NT)
                *(vec *)(A + (kb - I0 + q / KV) * AST + (q % KV) * V) = vinf;
        if (mask_cols)
            for (int q = tid; q < KC * (TB / V); q += NT)
                *(vec *)(B + (q / (TB / V)) * BN + kb - J0 + (q % (TB / V)) * V) = vinf;
        __syncthreads();
    };

    // acc <- min over the staged block of A[i][k] + B[k][j].  binary16 keeps
    // two adjacent columns per register (AW = 2): per pair of k, two packed
    // adds (the A value reaches both halves through the operand-select bits)
    // and one packed three-way minimum update two entries for two k each.  The
    // IEEE minimum (v_pk_minimum3_f16) differs from min only for NaN and the
    // order of -0 and +0, neither of which occurs in lengths >= +0.
    constexpr int AW = is_half_v<T> ? 2 : 1;
    using AccV = std::conditional_t<is_half_v<T>, half2_t, T>;
    AccV acc[RM][RN / AW];
    auto sweep = [&](const T *As_, const T *Bs_) {
#pragma unroll SWEEP_UNROLL
        for (int kv = 0; kv < KC / V; ++kv) {
            vec a[RM];
#pragma unroll
            for (int ii = 0; ii < RM; ++ii) a[ii] = *(const vec *)(As_ + (ty + TY * ii) * AST + kv * V);
#pragma unroll
            for (int kk = 0; kk < V; kk += 2) {
                vec b0[HN], b1[HN];
#pragma unroll
                for (int h = 0; h < HN; ++h) {
                    b0[h] = *(const vec *)(Bs_ + (kv * V + kk) * BN + h * CS + tx * V);
                    b1[h] = *(const vec *)(Bs_ + (kv * V + kk + 1) * BN + h * CS + tx * V);
                }
#pragma unroll
                for (int ii = 0; ii < RM; ++ii)
#pragma unroll
                    for (int h = 0; h < HN; ++h) {
                        if constexpr (is_half_v<T>) {
                            const half2_t a0 = {a[ii][kk], a[ii][kk]}, a1 = {a[ii][kk + 1], a[ii][kk + 1]};
#pragma unroll
                            for (int e = 0; e < V; e += 2) {
                                half2_t &x = acc[ii][(h * V + e) / 2];
                                const half2_t s0 = a0 + half2_t{b0[h][e], b0[h][e + 1]};
                                const half2_t s1 = a1 + half2_t{b1[h][e], b1[h][e + 1]};
                                x = __builtin_elementwise_minimum(__builtin_elementwise_minimum(x, s0), s1);
                            }
                        } else {
#pragma unroll
                            for (int e = 0; e < V; ++e) {
                                T &x = acc[ii][h * V + e];
                                x = vmin(vmin(x, a[ii][kk] + b0[h][e]), a[ii][kk + 1] + b1[h][e]);
                            }
                        }
                    }
            }
        }
    };
    auto acc_at = [&](const AccV (&src)[RM][RN / AW], int ii, int jj) -> T {
        if constexpr (is_half_v<T>)
            return src[ii][jj / 2][jj % 2];
        else
            return src[ii][jj];
    };

    // acc <- min over round r's block of the staged products; for a fused pair
    // (rounds r and r + 1, tiles outside both blocks) acc0 keeps round r's
    // minimum and acc takes round r + 1's, whose panels are final by now.
    // Chunk c covers k = k0 + (c / CPR) TB + (c % CPR) KC onwards.
    AccV acc0[RM][RN / AW];
    auto reset = [&]() {
#pragma unroll
        for (int ii = 0; ii < RM; ++ii)
#pragma unroll
            for (int jj = 0; jj < RN / AW; ++jj) acc[ii][jj] = inf_v<T>();
    };
    auto chunk_kb = [&](int c) { return k0 + (int64_t)(c / CPR) * TB; };
    // Chunk ch: with two buffers, start loading chunk ch + 1 into the other one
    // (it was last read in chunk ch - 1, which every wave has finished); sweep
    // this one; with one buffer, load chunk ch + 1 into it once every wave is
    // done; then wait for chunk ch + 1 and the barrier that makes it visible.
    auto step = [&](T *cA, T *cB, T *nA, T *nB, int ch) {
        if (NBUF == 2 && ch + 1 < NCH) issue(nA, nB, chunk_kb(ch + 1), ((ch + 1) % CPR) * KC);
        sweep(cA, cB);
        if constexpr (FUSE) {
            if (ch == CPR - 1) {
#pragma unroll
                for (int ii = 0; ii < RM; ++ii)
#pragma unroll
                    for (int jj = 0; jj < RN / AW; ++jj) acc0[ii][jj] = acc[ii][jj];
                reset();
            }
        }
        if (ch + 1 < NCH) {
            if (NBUF == 1) {
                __syncthreads();  // every wave is done with the buffer
                issue(cA, cB, chunk_kb(ch + 1), ((ch + 1) % CPR) * KC);
            }
            wait_vmem();
            __syncthreads();  // chunk ch + 1 has landed for every wave
            mask(NBUF == 2 ? nA : cA, NBUF == 2 ? nB : cB, chunk_kb(ch + 1));
        }
    };
    reset();
    issue(As0, Bs0, k0, 0);
    wait_vmem();
    __syncthreads();
    mask(As0, Bs0, k0);
    if constexpr (NBUF == 2) {
        for (int c = 0; c < NCH; c += 2) {
            step(As0, Bs0, As1, Bs1, c);
            if (c + 1 < NCH) step(As1, Bs1, As0, Bs0, c + 1);
        }
    } else {
        for (int c = 0; c < NCH; ++c) step(As0, Bs0, As0, Bs0, c);
    }

    if constexpr (!PREFETCH_C) {
#pragma unroll
        for (int ii = 0; ii < RM; ++ii)
#pragma unroll
            for (int h = 0; h < HN; ++h) c[ii][h] = *(const vec *)c_ptr(ii, h);
    }

    // New distances: store the 16-byte vectors in which some entry decreased;
    // in path mode mark each decreased entry pending from the last round in
    // which it decreased (r, or r + 1 for a fused pair).
    // The entry's decrease flags (lt0: in round r, lt1: in round r + 1 of a
    // fused pair) select the store and the mark directly.
    const uint16_t pend = (uint16_t)(r + 1), pend1 = (uint16_t)(r + 2);
#pragma unroll
    for (int ii = 0; ii < RM; ++ii)
#pragma unroll
        for (int h = 0; h < HN; ++h) {
            vec nv = c[ii][h];
            bool lt0[V], lt1[V];
            bool ch = false;
#pragma unroll
            for (int e = 0; e < V; ++e) {
                const T s = acc_at(acc, ii, h * V + e);
                if constexpr (FUSE) {
                    const T s0 = acc_at(acc0, ii, h * V + e);
                    lt0[e] = s0 < nv[e];
                    const T c1 = lt0[e] ? s0 : nv[e];
                    lt1[e] = s < c1;
                    nv[e] = lt1[e] ? s : c1;
                } else {
                    lt0[e] = s < nv[e];
                    lt1[e] = false;
                    nv[e] = lt0[e] ? s : nv[e];
                }
                ch |= lt0[e] || lt1[e];
            }
            if (ch) {
                *(vec *)c_ptr(ii, h) = nv;
                if constexpr (PATH) {
                    uint16_t *lp = l_ptr(ii, h);
#pragma unroll
                    for (int e = 0; e < V; ++e)
                        if (lt0[e] || lt1[e]) lp[e] = lt1[e] ? pend1 : pend;
                }
            }
        }
}

// ---------------------------------------------------------------------------
// Phase 4, wave-row form.  Same tiles, same result and the same path-mode
// marks as k_phase4; only the data movement differs.  Wave w of the workgroup
// owns RM consecutive rows of a BM x BN tile (BM = 4 * RM, which divides TB, so
// whole tile rows of block row K are skipped), lane l the RN consecutive
// columns from l * RN (BN = 64 * RN; a tile containing block column K masks it
// in the staged panel, as k_phase4 does).  For a given row i and k, the
// column-panel value D[i][k] is the same for all 64 lanes of the wave, so it is
// read with scalar loads (the column panel lies in block column K, which this
// launch never writes) and enters each addition as a scalar operand.  Only the
// row panel D[K, J] is staged in LDS; per k each lane reads its RN entries of
// it, 4 / RM bytes of LDS traffic per update for float (k_phase4's 4 x 4
// register tiles need 2 bytes, which is all the LDS delivers at the VALU's
// update rate).
template <typename T, int TB, int RM, int RN, bool PATH, bool BAND>
__global__ void __launch_bounds__(NT) k_phase4w(T *__restrict__ D, uint16_t *__restrict__ L, int64_t ld, int r,
                                               TileSel sel) {
    constexpr int BM = (NT / 64) * RM, BN = 64 * RN;
    static_assert(TB % BM == 0, "wave-row tiles must divide the block");
    using vec = typename V16<T>::type;
    constexpr int V = V16<T>::n;
    static_assert(BN % V == 0, "row panel width");
    typedef T cvec __attribute__((ext_vector_type(RN)));
    typedef const T __attribute__((address_space(4))) CT;  // scalar (constant) loads
    __shared__ __attribute__((aligned(16))) T Bs[TB * BN];

    int bi, bj;
    if (!select_tile<BAND>(sel, blockIdx.x, bi, bj)) return;
    const int64_t I0 = (int64_t)bi * BM, J0 = (int64_t)bj * BN, k0 = (int64_t)r * TB;
    const bool mask_cols = sel.nsc == 0 && (J0 <= k0) && (k0 < J0 + BN);

    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int64_t i0 = I0 + (int64_t)wave * RM;
    T *crow = D + i0 * ld + J0 + lane * RN;
    uint16_t *lrow = L + (crow - D);

    // Old C values first, so their latency overlaps the staging.
    cvec c[RM];
#pragma unroll
    for (int ii = 0; ii < RM; ++ii) c[ii] = *(const cvec *)(crow + ii * ld);
    const vec vinf = inf_v<T>();
    for (int q = threadIdx.x; q < TB * (BN / V); q += NT) {
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
        for (int e = 0; e < RN; ++e) acc[ii][e] = inf_v<T>();
    CT *A = (CT *)(D + i0 * ld + k0);
    constexpr int KC = 16 / (int)sizeof(T);  // k per 16-byte scalar load of a row
#pragma unroll 2
    for (int kc = 0; kc < TB; kc += KC) {
        T a[RM][KC];
#pragma unroll
        for (int ii = 0; ii < RM; ++ii)
#pragma unroll
            for (int kk = 0; kk < KC; ++kk) a[ii][kk] = A[ii * ld + kc + kk];
#pragma unroll
        for (int kk = 0; kk < KC; kk += 2) {
            const cvec b0 = *(const cvec *)(Bs + (kc + kk) * BN + lane * RN);
            const cvec b1 = *(const cvec *)(Bs + (kc + kk + 1) * BN + lane * RN);
#pragma unroll
            for (int ii = 0; ii < RM; ++ii)
#pragma unroll
                for (int e = 0; e < RN; ++e)
                    acc[ii][e] = vmin(vmin(acc[ii][e], a[ii][kk] + b0[e]), a[ii][kk + 1] + b1[e]);
        }
    }

    // Store the rows of a lane in which some entry decreased; in path mode mark
    // each decreased entry pending from this round.
    const uint16_t pend = (uint16_t)(r + 1);
#pragma unroll
    for (int ii = 0; ii < RM; ++ii) {
        cvec nv = c[ii];
        bool ch = false, lt[RN];
#pragma unroll
        for (int e = 0; e < RN; ++e) {
            lt[e] = acc[ii][e] < nv[e];
            ch |= lt[e];
            nv[e] = lt[e] ? acc[ii][e] : nv[e];
        }
        if (ch) {
            *(cvec *)(crow + ii * ld) = nv;
            if constexpr (PATH) {
#pragma unroll
                for (int e = 0; e < RN; ++e)
                    if (lt[e]) lrow[ii * ld + e] = pend;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Label resolution (path mode, after the last round).  Entry (i, j) pending
// from round r (L = r + 1) last decreased in the last phase of round r, to
// S = min over k in K_r of A[i][k] + B[k][j].  For every k that attains S, the
// entries (i, k) and (k, j) were already final then: a later decrease of either
// would give (i, j) a strictly shorter path, contradicting that S is final.  So
// the k that attain S are found from the final matrix -- those with
// D[i][k] + D[k][j] == D[i][j], the same float addition -- and the label is
// min over them of max(P[i][k], k, P[k][j]).  Any k that attains D[i][j] only
// with final values (because D[i][k] or D[k][j] decreased later) has a label
// from a later round, larger than every label of round r, so it never changes
// the minimum -- and such a k is recognisable: one of its two entries
// decreased after round r, so if that entry is still pending, it is pending
// from a round later than r; such k are skipped.  Otherwise (i, k) and (k, j)
// carry either their final label or, if pending from a round before r, a label
// below k0 (P holds an older one, also below k0, until that entry is resolved),
// which does not change max(., k, .).  Entries are therefore resolved
// independently, in one launch, updating P in place.  Column segments come from
// a transposed copy DT (DT[j][k] = D[k][j]) so that both segments are
// contiguous.  With non-integer weights, rounding can break the exact equality
// (a sub-path decreased later by less than the sum's rounding step); then the k
// with the smallest sum is taken and the label is k itself, which still encodes
// a path of length D[i][j] up to rounding.
// For ld <= 65535 each entry's label + 1 and mark are packed in one word
// (W = mark << 16 | label + 1, k_pack_marks), so that a candidate k costs one
// gathered word of (k, j) instead of a label and a mark.  A word read here is
// either still pending (its mark and the label it had when marked) or already
// resolved (its mark and its final label): the argument above gives the same
// minimum either way.  A resolved word keeps its mark, so whether a neighbour
// entry counts as decreased after round r never depends on whether another
// thread has resolved it yet, and the result does not depend on timing.
// The resolve itself.  A wave takes the pending entries among its 64
// consecutive columns of row i, four at a time, with 16 lanes per entry and
// TB / 16 consecutive candidates k per lane: every load instruction then reads
// whole segments of four entries, where one thread per entry made each load
// touch 64 different cache lines.  The lanes that find an exact hit gather its
// words (in parallel), the group's minimum label is reduced across its 16 lanes
// (one DPP row), and the group's first lane writes the entry.  An entry without
// a usable hit (rare: rounding) gets the first strict minimum, from the group's
// first lane.  Each entry's mark and length are read once, coalesced, by the
// lane of its column and listed in LDS (pending entries only, in column order);
// a group takes EPG entries per pass, their loads all in flight together; the
// results go through LDS to one coalesced store per wave.  PACKED: marks and
// labels in W (above); else marks in L and labels in P, for ld > 65535.  Labels
// are handled as label + 1 (unsigned).
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_min(uint32_t v) {
    return min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, 0xF, 0xF, false));
}
template <typename T, int TB, bool PACKED, int EPG>
__global__ void __launch_bounds__(NT) k_resolve(const T *__restrict__ D, const T *__restrict__ DT,
                                               uint32_t *__restrict__ W, const uint16_t *__restrict__ L,
                                               int32_t *__restrict__ P, int64_t ld) {
    constexpr int CPL = TB / 16;  // candidates per lane
    static_assert(CPL * 16 == TB, "resolve group");
    typedef T cvec __attribute__((ext_vector_type(CPL)));
    __shared__ uint32_t res[NT];                 // results by column, for one coalesced store per wave
    __shared__ uint32_t s_col[NT], s_mark[NT];   // each wave's pending entries, compacted
    __shared__ T s_len[NT];
    const int lane = threadIdx.x & 63, g = lane >> 4, p = lane & 15, wbase = threadIdx.x & ~63;
    const int64_t jb = (int64_t)blockIdx.x * NT + wbase;  // the wave's first column
    auto mark_of = [&](int64_t x) -> uint32_t { return PACKED ? W[x] >> 16 : (uint32_t)L[x]; };
    auto label1_of = [&](int64_t x) -> uint32_t { return PACKED ? W[x] & 0xffffu : (uint32_t)(P[x] + 1); };
    for (int64_t i = blockIdx.y; i < ld; i += gridDim.y) {  // grid y is capped at 65535 rows
        const int64_t j = jb + lane;
        const uint32_t mk = j < ld ? mark_of(i * ld + j) : 0u;
        const T dj = j < ld ? D[i * ld + j] : T(0);
        const uint64_t pending = __ballot(mk != 0);  // the same in every lane
        const int npend = __builtin_popcountll(pending);
        if (mk != 0) {
            const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(pending >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)pending, 0));
            s_col[wbase + rank] = lane;
            s_mark[wbase + rank] = mk;
            s_len[wbase + rank] = dj;
        }
        __syncthreads();  // the lists are written
        // Passes of 4 * EPG entries: group g takes list slots base + 4 m + g.
        for (int base = 0; base < npend; base += 4 * EPG) {
            int col[EPG];
            uint32_t lv[EPG];
            T d[EPG];
            cvec a[EPG], b[EPG];
#pragma unroll
            for (int m = 0; m < EPG; ++m) {
                const int sl = base + 4 * m + g;
                const bool ok = sl < npend;
                col[m] = ok ? (int)s_col[wbase + sl] : -1;
                lv[m] = ok ? s_mark[wbase + sl] : 1u;
                d[m] = ok ? s_len[wbase + sl] : T(0);
                const int64_t je = jb + (ok ? col[m] : 0), kl = (int64_t)(lv[m] - 1) * TB + p * CPL;
                a[m] = *(const cvec *)(D + i * ld + kl);
                b[m] = *(const cvec *)(DT + je * ld + kl);
            }
#pragma unroll
            for (int m = 0; m < EPG; ++m) {
                const int64_t je = jb + (col[m] >= 0 ? col[m] : 0);
                const int64_t k0 = (int64_t)(lv[m] - 1) * TB, kl = k0 + p * CPL;
                uint32_t hm = 0;
#pragma unroll
                for (int c = 0; c < CPL; ++c) hm |= (a[m][c] + b[m][c] == d[m]) ? (1u << c) : 0u;
                if (col[m] < 0) hm = 0;
                uint32_t M = 0xffffffffu;
                while (hm) {  // this lane's exact hits: their two words each
                    const int64_t kg = kl + __builtin_ctz(hm);
                    hm &= hm - 1;
                    if (mark_of(i * ld + kg) <= lv[m] && mark_of(kg * ld + je) <= lv[m])  // else decreased after round lv - 1
                        M = min(M, max(max(label1_of(i * ld + kg), label1_of(kg * ld + je)), (uint32_t)(kg + 1)));
                }
                M = dpp_min<0xB1>(M);   // quad_perm [1, 0, 3, 2]
                M = dpp_min<0x4E>(M);   // quad_perm [2, 3, 0, 1]
                M = dpp_min<0x141>(M);  // row_half_mirror
                M = dpp_min<0x140>(M);  // row_mirror: the minimum of all 16 lanes
                if (p == 0 && col[m] >= 0) {
                    if (M == 0xffffffffu) {
                        T best = inf_v<T>();
                        int kbest = 0;
                        for (int k = 0; k < TB; ++k) {
                            const T sk = D[i * ld + k0 + k] + DT[je * ld + k0 + k];
                            kbest = (sk < best) ? k : kbest;
                            best = vmin(best, sk);
                        }
                        M = (uint32_t)(k0 + kbest + 1);
                    }
                    res[wbase + col[m]] = M;
                }
            }
        }
        __syncthreads();  // every group's result is in res
        if (mk != 0) {
            if constexpr (PACKED)
                W[i * ld + j] = (mk << 16) | res[threadIdx.x];
            else
                P[i * ld + j] = (int32_t)res[threadIdx.x] - 1;
        }
        __syncthreads();  // res and the lists are free for the next row
    }
}

// P (labels, -1 = none) and L (marks) -> W = mark << 16 | label + 1, in P's
// storage; and back to labels after the resolve.
__global__ void __launch_bounds__(NT) k_pack_marks(int32_t *__restrict__ P, const uint16_t *__restrict__ L,
                                                   int64_t count) {
    for (int64_t x = (int64_t)blockIdx.x * NT + threadIdx.x; x < count; x += (int64_t)gridDim.x * NT)
        P[x] = (int32_t)(((uint32_t)L[x] << 16) | (uint32_t)(P[x] + 1));
}
__global__ void __launch_bounds__(NT) k_unpack_labels(int32_t *__restrict__ P, int64_t count) {
    for (int64_t x = (int64_t)blockIdx.x * NT + threadIdx.x; x < count; x += (int64_t)gridDim.x * NT)
        P[x] = (int32_t)((uint32_t)P[x] & 0xffffu) - 1;
}

// Tiled transpose: DT[j][i] = D[i][j] (ld x ld, ld a multiple of 64).
template <typename T>
__global__ void __launch_bounds__(NT) k_transpose(const T *__restrict__ D, T *__restrict__ DT, int64_t ld) {
    __shared__ T t[64][65];
    const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x % 64, ty = threadIdx.x / 64;
    for (int rr = ty; rr < 64; rr += NT / 64) t[rr][tx] = D[(i0 + rr) * ld + j0 + tx];
    __syncthreads();
    for (int rr = ty; rr < 64; rr += NT / 64) DT[(j0 + rr) * ld + i0 + tx] = t[tx][rr];
}

// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// rows x cols block with leading dimension ld: +inf, and 0 where row == col if
// zero_diag.
template <typename T>
__global__ void k_fill_blank(T *__restrict__ p, int64_t ld, int64_t rows, int64_t cols, int zero_diag) {
    const int64_t total = rows * cols;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = x / cols, j = x % cols;
        p[i * ld + j] = (zero_diag && i == j) ? (T)0 : inf_v<T>();
    }
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


template <typename T, int TB>
void launch_p123(T *D, int32_t *P, uint16_t *L, int64_t ld, int r, hipStream_t s) {
    const int nb = (int)(ld / TB);
    const bool path = P != nullptr;
    constexpr int TS = TB < p1_ts<T, TB>() ? TB : p1_ts<T, TB>();
    if (path)
        hipLaunchKernelGGL((k_phase1<T, TB, true, TS>), dim3(1), dim3(TS * TS), 0, s, D, P, L, ld, r);
    else
        hipLaunchKernelGGL((k_phase1<T, TB, false, TS>), dim3(1), dim3(TS * TS), 0, s, D, P, L, ld, r);
    if (nb == 1) return;
    if (path)
        hipLaunchKernelGGL((k_phase23<T, TB, true>), dim3(2 * (nb - 1)), dim3(NT), 0, s, D, P, L, ld, r, nb);
    else
        hipLaunchKernelGGL((k_phase23<T, TB, false>), dim3(2 * (nb - 1)), dim3(NT), 0, s, D, P, L, ld, r, nb);
}

// One last-phase launch (any P4Mode, see
// P4Mode) with the LDS-panel kernel (WAVE = false) or the wave-row kernel
// (BM = 4 * RM).  r is the round applied (the first of the two for a pair).
template <typename T, int TB, int BM, int BN, bool WAVE>
hipError_t p4_impl(T *D, uint16_t *L, bool path, int64_t ld, int r, P4Mode mode, hipStream_t s) {
    const int rb = BM <= TB ? TB / BM : 0;  // tile rows per block; 0: the block row is masked
    const int cb = BN == TB ? 1 : 0;        // likewise for columns
    const int nb = (int)(ld / TB);
    TileSel sel;
    bool band = false, fuse = false;
    if (!p4_select((int)(ld / BM), (int)(ld / BN), rb, cb, r, nb, mode, sel, band, fuse)) return hipErrorInvalidValue;
    if (fuse && (WAVE || BM != TB || BN != TB)) return hipErrorInvalidValue;
    if (sel.ntiles == 0) return hipSuccess;
    // Algorithmic min-plus updates of the bulk launches (timed by the profiling
    // hooks): every tile outside the skipped blocks, times the rounds applied.
    int64_t upd = 0;
    if (mode == P4Mode::all) upd = (ld - TB) * (ld - TB) * TB;
    if (mode == P4Mode::rest) upd = (ld - 2 * TB) * (ld - 2 * TB) * TB;
    if (mode == P4Mode::pair) upd = 2 * (ld - 2 * TB) * (ld - 2 * TB) * TB;
    if (mode == P4Mode::pair_rest) {
        const int64_t w = nb - r < 4 ? nb - r : 4;
        upd = 2 * (ld - w * TB) * (ld - w * TB) * TB;
    }
    const dim3 grid(8 * sel.per_xcd);
    constexpr int RM = BM / (NT / 64), RN = BN / 64;
#define FW_P4_LAUNCH(PATHV, BANDV, FUSEV)                                                                           \
    do {                                                                                                         \
        if constexpr (WAVE) {                                                                                    \
            if constexpr (!FUSEV)                                                                                \
                hipLaunchKernelGGL((k_phase4w<T, TB, RM, RN, PATHV, BANDV>), grid, dim3(NT), 0, s, D, L, ld, r,    \
                                   sel);                                                                         \
        } else if constexpr (!FUSEV || (BM == TB && BN == TB)) {                                                 \
            hipLaunchKernelGGL((k_phase4<T, TB, BM, BN, PATHV, BANDV, FUSEV>), grid, dim3(NT), 0, s, D, L, ld, r,  \
                               sel);                                                                             \
        }                                                                                                        \
    } while (0)
    const bool timed = upd > 0;
    if (timed) prof_begin_p4(s);
    if (path) {
        if (band && fuse)
            FW_P4_LAUNCH(true, true, true);
        else if (band)
            FW_P4_LAUNCH(true, true, false);
        else if (fuse)
            FW_P4_LAUNCH(true, false, true);
        else
            FW_P4_LAUNCH(true, false, false);
    } else {
        if (band && fuse)
            FW_P4_LAUNCH(false, true, true);
        else if (band)
            FW_P4_LAUNCH(false, true, false);
        else if (fuse)
            FW_P4_LAUNCH(false, false, true);
        else
            FW_P4_LAUNCH(false, false, false);
    }
    if (timed) prof_end_p4(s, upd);
#undef FW_P4_LAUNCH
    return hipGetLastError();
}

}  // namespace

// Compiled (block, tile_m, tile_n) combinations: LDS-panel last phase ...
#define FW_P4_CONFIGS_F32(X)                                                                           \
    X(32, 64, 64) X(32, 128, 64) X(32, 64, 128) X(32, 128, 128) X(64, 64, 64) X(64, 128, 64) X(64, 64, 128) \
    X(64, 128, 128)
#define FW_P4_CONFIGS_F64(X) \
    X(32, 64, 64) X(32, 128, 64) X(32, 64, 128) X(32, 128, 128) X(64, 64, 64) X(64, 128, 64) X(64, 64, 128)
// ... and wave-row last phase (tile_m = 4 x rows per wave, tile_n = 64 x columns per lane).
#define FW_P4W_CONFIGS_F32(X)                                                                               \
    X(32, 16, 256) X(32, 32, 128) X(32, 32, 256) X(64, 16, 256) X(64, 32, 128) X(64, 32, 256) X(64, 64, 128) \
    X(64, 64, 256)
#define FW_P4W_CONFIGS_F64(X) X(32, 16, 128) X(32, 32, 64) X(32, 32, 128) X(64, 32, 64) X(64, 32, 128) X(64, 64, 128)
// binary16: LDS-panel last phase only; a 16-byte vector holds 8 columns, so
// tiles are at least 128 wide (8 columns per thread, 16 threads across).
#define FW_P4_CONFIGS_F16(X) X(32, 64, 128) X(32, 128, 128) X(64, 32, 128) X(64, 64, 128) X(64, 128, 128) X(64, 64, 256)
#define FW_P4W_CONFIGS_F16(X)

// FW_FOR_DTYPE(T, PANELS, WAVE, X): expand X over the panel (PANELS true) or
// wave-row configurations compiled for element type T.
#define FW_FOR_DTYPE(T, PANELS, X)                       \
    do {                                                 \
        if constexpr (std::is_same_v<T, float>) {        \
            if constexpr (PANELS) {                      \
                FW_P4_CONFIGS_F32(X)                     \
            } else {                                     \
                FW_P4W_CONFIGS_F32(X)                    \
            }                                            \
        } else if constexpr (std::is_same_v<T, double>) { \
            if constexpr (PANELS) {                      \
                FW_P4_CONFIGS_F64(X)                     \
            } else {                                     \
                FW_P4W_CONFIGS_F64(X)                    \
            }                                            \
        } else {                                         \
            if constexpr (PANELS) {                      \
                FW_P4_CONFIGS_F16(X)                     \
            } else {                                     \
                FW_P4W_CONFIGS_F16(X)                    \
            }                                            \
        }                                                \
    } while (0)

template <typename T>
bool config_supported(TileCfg c) {
#define FW_MATCH(B, M, N) if (c.block == B && c.tile_m == M && c.tile_n == N) return true;
    if (c.variant == FW_VARIANT_PANELS) FW_FOR_DTYPE(T, true, FW_MATCH);
    else if (c.variant == FW_VARIANT_WAVEROWS) FW_FOR_DTYPE(T, false, FW_MATCH);
#undef FW_MATCH
    return false;
}

template <typename T>
int list_configs(TileCfg *out, int cap) {
    int k = 0;
#define FW_PUT(B, M, N, VAR)                              \
    {                                                     \
        if (out && k < cap) out[k] = TileCfg{B, M, N, VAR, 0}; \
        ++k;                                              \
    }
#define FW_PUT_P(B, M, N) FW_PUT(B, M, N, FW_VARIANT_PANELS)
#define FW_PUT_W(B, M, N) FW_PUT(B, M, N, FW_VARIANT_WAVEROWS)
    FW_FOR_DTYPE(T, true, FW_PUT_P);
    FW_FOR_DTYPE(T, false, FW_PUT_W);
#undef FW_PUT
#undef FW_PUT_P
#undef FW_PUT_W
    return k;
}

template <typename T>
hipError_t launch_phase123(T *D, int32_t *P, uint16_t *L, int64_t ld, int r, int block, hipStream_t s) {
    if (block == 64)
        launch_p123<T, 64>(D, P, L, ld, r, s);
    else if (block == 32)
        launch_p123<T, 32>(D, P, L, ld, r, s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <typename T>
hipError_t launch_phase4(T *D, uint16_t *L, bool path, int64_t ld, int r, TileCfg c, P4Mode mode, hipStream_t s) {
#define FW_DISPATCH(B, M, N) \
    if (c.block == B && c.tile_m == M && c.tile_n == N) return p4_impl<T, B, M, N, false>(D, L, path, ld, r, mode, s);
#define FW_DISPATCH_W(B, M, N) \
    if (c.block == B && c.tile_m == M && c.tile_n == N) return p4_impl<T, B, M, N, true>(D, L, path, ld, r, mode, s);
    if (c.variant == FW_VARIANT_PANELS) FW_FOR_DTYPE(T, true, FW_DISPATCH);
    else if (c.variant == FW_VARIANT_WAVEROWS) FW_FOR_DTYPE(T, false, FW_DISPATCH_W);
#undef FW_DISPATCH
#undef FW_DISPATCH_W
    return hipErrorInvalidValue;
}

bool lookahead_supported(TileCfg c) { return c.tile_n == c.block && c.tile_m <= c.block; }

bool pairs_supported(TileCfg c) {
    return c.variant == FW_VARIANT_PANELS && c.tile_m == c.block && c.tile_n == c.block;
}

constexpr int kResolveEPG = 2;  // entries per 16-lane group and pass in k_resolve

template <typename T>
hipError_t launch_resolve(const T *D, T *DT, const uint16_t *L, int32_t *P, int64_t ld, int block, hipStream_t s) {
    hipLaunchKernelGGL((k_transpose<T>), dim3((unsigned)(ld / 64), (unsigned)(ld / 64)), dim3(NT), 0, s, D, DT, ld);
    const dim3 grid((unsigned)((ld + NT - 1) / NT), (unsigned)(ld < 65535 ? ld : 65535));
    if (block != 64 && block != 32) return hipErrorInvalidValue;
    if (ld <= 65535) {  // label + 1 and the mark fit one word
        uint32_t *W = (uint32_t *)P;
        hipLaunchKernelGGL(k_pack_marks, dim3(grid_for(ld * ld)), dim3(NT), 0, s, P, L, ld * ld);
        if (block == 64)
            hipLaunchKernelGGL((k_resolve<T, 64, true, kResolveEPG>), grid, dim3(NT), 0, s, D, DT, W, L, P, ld);
        else
            hipLaunchKernelGGL((k_resolve<T, 32, true, kResolveEPG>), grid, dim3(NT), 0, s, D, DT, W, L, P, ld);
        hipLaunchKernelGGL(k_unpack_labels, dim3(grid_for(ld * ld)), dim3(NT), 0, s, P, ld * ld);
        return hipGetLastError();
    }
    if (block == 64)
        hipLaunchKernelGGL((k_resolve<T, 64, false, kResolveEPG>), grid, dim3(NT), 0, s, D, DT, nullptr, L, P, ld);
    else
        hipLaunchKernelGGL((k_resolve<T, 32, false, kResolveEPG>), grid, dim3(NT), 0, s, D, DT, nullptr, L, P, ld);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill_blank(T *p, int64_t ld, int64_t rows, int64_t cols, bool zero_diag, hipStream_t s) {
    hipLaunchKernelGGL((k_fill_blank<T>), dim3(grid_for(rows * cols)), dim3(NT), 0, s, p, ld, rows, cols,
                       zero_diag ? 1 : 0);
    return hipGetLastError();
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
template int list_configs<float>(TileCfg *, int);
template hipError_t launch_fill_blank<float>(float *, int64_t, int64_t, int64_t, bool, hipStream_t);
template hipError_t launch_fill_blank<double>(double *, int64_t, int64_t, int64_t, bool, hipStream_t);
template int list_configs<double>(TileCfg *, int);
template hipError_t launch_phase123<float>(float *, int32_t *, uint16_t *, int64_t, int, int, hipStream_t);
template hipError_t launch_phase123<double>(double *, int32_t *, uint16_t *, int64_t, int, int, hipStream_t);
template hipError_t launch_phase4<float>(float *, uint16_t *, bool, int64_t, int, TileCfg, P4Mode, hipStream_t);
template hipError_t launch_phase4<double>(double *, uint16_t *, bool, int64_t, int, TileCfg, P4Mode, hipStream_t);
template hipError_t launch_resolve<float>(const float *, float *, const uint16_t *, int32_t *, int64_t, int, hipStream_t);
template hipError_t launch_resolve<double>(const double *, double *, const uint16_t *, int32_t *, int64_t, int, hipStream_t);
template hipError_t launch_pad_in<float>(const float *, int64_t, float *, int64_t, hipStream_t);
template hipError_t launch_pad_in<double>(const double *, int64_t, double *, int64_t, hipStream_t);
template hipError_t launch_pad_out<float>(const float *, int64_t, float *, int64_t, hipStream_t);
template hipError_t launch_pad_out<double>(const double *, int64_t, double *, int64_t, hipStream_t);
template hipError_t launch_pad_out<int32_t>(const int32_t *, int64_t, int32_t *, int64_t, hipStream_t);
template bool config_supported<_Float16>(TileCfg);
template int list_configs<_Float16>(TileCfg *, int);
template hipError_t launch_phase123<_Float16>(_Float16 *, int32_t *, uint16_t *, int64_t, int, int, hipStream_t);
template hipError_t launch_phase4<_Float16>(_Float16 *, uint16_t *, bool, int64_t, int, TileCfg, P4Mode, hipStream_t);
template hipError_t launch_resolve<_Float16>(const _Float16 *, _Float16 *, const uint16_t *, int32_t *, int64_t, int,
                                             hipStream_t);
template hipError_t launch_pad_in<_Float16>(const _Float16 *, int64_t, _Float16 *, int64_t, hipStream_t);
template hipError_t launch_pad_out<_Float16>(const _Float16 *, int64_t, _Float16 *, int64_t, hipStream_t);

}  // namespace fw
