// fw_ooc.cpp -- shortest distances for a matrix held in host memory (out of
// core): the blocked method with super-blocks of edge S sized to a device
// memory budget.  Super-round R, with K the vertices of super-block R:
//   1. the diagonal super-block D[K,K] is closed in device memory by the
//      in-core blocked sweep (fw_apsp);
//   2. the row band D[K,:] becomes min(D[K,J], D*[K,K] (x) D_old[K,J]) per
//      super-column J (one min-plus product each, as phases 2 of the blocked
//      method with the closed diagonal block);
//   3. the column band D[:,K] likewise, min(D[I,K], D_old[I,K] (x) D*[K,K]);
//   4. every other super-tile is updated, D[I,J] <- min(D[I,J], D[I,K] (x) D[K,J]):
//      first super-row and super-column R + 1, straight into a second set of
//      band buffers where super-round R + 1 finds its bands (and its diagonal
//      block) without a round trip through host memory; then the rest, each
//      streamed through the device once, with its upload, product and download
//      on three streams and two device buffers, so that transfers in both
//      directions overlap the products.
// With the path matrix, every block carries its labels and the products apply
// the lexicographic rule (length, largest interior vertex) of phases 1-3 with
// global vertex indices.  The diagonal closure runs on the block alone, whose
// labels are local and -1 where an entry did not change: those entries keep
// their earlier label (below K's first vertex, so it loses no tie), the others
// get K's first vertex plus the local label.
// Edges that do not fill a super-block are padded with +inf and label -1
// (isolated vertices), so every product runs on full S x S blocks.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <utility>

#include "../../include/fw_apsp.h"
#include "fw_internal.h"

namespace fw {

size_t ooc_working_bytes(int64_t n, int64_t S, size_t es, bool path) {
    const int64_t NS = (n + S - 1) / S, NP = NS * S;
    // diagonal, temp, 2 tile buffers; two sets of row and column bands (this
    // super-round's and the next one's)
    const size_t blocks = (size_t)(4 * S * S + 4 * S * NP);
    return blocks * es + (path ? blocks * sizeof(int32_t) + (size_t)(S * S) * sizeof(int32_t) : 0);
}

namespace {

struct Streams {
    hipStream_t cs = nullptr, h2d = nullptr, d2h = nullptr;
    hipEvent_t loaded[2] = {nullptr, nullptr}, computed[2] = {nullptr, nullptr}, stored[2] = {nullptr, nullptr};
    hipEvent_t start = nullptr, bands = nullptr, rows_done = nullptr, cols_done = nullptr, ahead = nullptr;
    ~Streams() {
        for (hipEvent_t e : {loaded[0], loaded[1], computed[0], computed[1], stored[0], stored[1], start, bands,
                             rows_done, cols_done, ahead})
            if (e) (void)hipEventDestroy(e);
        for (hipStream_t s : {cs, h2d, d2h})
            if (s) (void)hipStreamDestroy(s);
    }
    hipError_t create() {
        hipError_t e;
        for (hipStream_t *s : {&cs, &h2d, &d2h})
            if ((e = hipStreamCreateWithFlags(s, hipStreamNonBlocking)) != hipSuccess) return e;
        for (hipEvent_t *ev : {&loaded[0], &loaded[1], &computed[0], &computed[1], &stored[0], &stored[1], &start,
                               &bands, &rows_done, &cols_done, &ahead})
            if ((e = hipEventCreateWithFlags(ev, hipEventDisableTiming)) != hipSuccess) return e;
        return hipSuccess;
    }
};

struct DeviceBuffer {
    void *p = nullptr;
    ~DeviceBuffer() {
        if (p) (void)hipFree(p);
    }
};

#define FW_TRY(x)                                \
    do {                                         \
        hipError_t e_ = (x);                     \
        if (e_ != hipSuccess) {                  \
            *what = #x;                          \
            return e_;                           \
        }                                        \
    } while (0)

}  // namespace

template <typename T>
hipError_t run_ooc(int64_t n, T *H, int32_t *HP, int64_t S, hipStream_t user, const char **what) {
    const int64_t NS = (n + S - 1) / S, NP = NS * S;
    const size_t es = sizeof(T), is = sizeof(int32_t);
    const bool path = HP != nullptr;
    Streams st;
    FW_TRY(st.create());
    DeviceBuffer buf;
    FW_TRY(hipMalloc(&buf.p, ooc_working_bytes(n, S, es, path)));
    T *Dd = (T *)buf.p, *TMP = Dd + S * S, *Cb[2] = {TMP + S * S, TMP + 2 * S * S};
    // Band sets: RBs[b] is S x NP (leading dimension NP), CBs[b] NP x S (leading
    // dimension S); super-round R reads set R % 2 and fills set (R + 1) % 2.
    T *RBs[2], *CBs[2];
    RBs[0] = Cb[1] + S * S;
    CBs[0] = RBs[0] + S * NP;
    RBs[1] = CBs[0] + NP * S;
    CBs[1] = RBs[1] + S * NP;
    // Labels, same shapes (path mode), plus the diagonal block's local labels.
    int32_t *Pd = path ? (int32_t *)(CBs[1] + NP * S) : nullptr, *TMPP = path ? Pd + S * S : nullptr;
    int32_t *CbP[2] = {path ? TMPP + S * S : nullptr, path ? TMPP + 2 * S * S : nullptr};
    int32_t *RBPs[2] = {nullptr, nullptr}, *CBPs[2] = {nullptr, nullptr};
    if (path) {
        RBPs[0] = CbP[1] + S * S;
        CBPs[0] = RBPs[0] + S * NP;
        RBPs[1] = CBPs[0] + NP * S;
        CBPs[1] = RBPs[1] + S * NP;
    }
    int32_t *Ploc = path ? CBPs[1] + NP * S : nullptr;
    const hipStream_t cs = st.cs;
    // P starts as "no interior vertex" (-1).  The host array is output only:
    // super-round 0 reads every tile once, and its labels are then the -1 the
    // device buffers are filled with, not an upload; every tile is written
    // back by the end of super-round 1 (super-round 0 alone when NS = 1).
    // Order after the caller's earlier work on its stream.
    FW_TRY(hipEventRecord(st.start, user));
    FW_TRY(hipStreamWaitEvent(cs, st.start, 0));
    // Tile buffers and the first band set start blank (padding rows and columns:
    // +inf, label -1); uploads into them wait for that.
    FW_TRY(launch_fill_blank<T>(Cb[0], S, S, S, false, cs));
    FW_TRY(launch_fill_blank<T>(Cb[1], S, S, S, false, cs));
    FW_TRY(launch_fill_blank<T>(RBs[0], NP, S, NP, false, cs));
    FW_TRY(launch_fill_blank<T>(CBs[0], S, NP, S, false, cs));
    if (path) {
        FW_TRY(launch_fill_i32(CbP[0], S * S, -1, cs));
        FW_TRY(launch_fill_i32(CbP[1], S * S, -1, cs));
        FW_TRY(launch_fill_i32(RBPs[0], S * NP, -1, cs));
        FW_TRY(launch_fill_i32(CBPs[0], NP * S, -1, cs));
    }
    FW_TRY(hipEventRecord(st.start, cs));
    FW_TRY(hipStreamWaitEvent(st.h2d, st.start, 0));
    auto edge = [&](int64_t b) { return std::min(S, n - b * S); };
    const hipMemcpyKind H2D = hipMemcpyHostToDevice, D2H = hipMemcpyDeviceToHost, D2D = hipMemcpyDeviceToDevice;
    const fw_dtype_t dt = sizeof(T) == 4 ? FW_F32 : FW_F64;
    // A band's copy between host and device, without the diagonal super-block's
    // part (columns [K0, K0 + SK) of the row band, rows of the column band): that
    // part of a band buffer is never read, and leaving it out keeps the band's
    // transfers apart from the diagonal block's, so they can run on other streams
    // while the block is closed.
    auto row_band_copy = [&](void *dev, int64_t ldd, void *host, size_t e, int64_t K0, int64_t SK,
                             hipMemcpyKind kind, hipStream_t s) -> hipError_t {
        for (auto [c0, c1] : {std::pair<int64_t, int64_t>{0, K0}, {K0 + SK, n}}) {
            if (c1 <= c0) continue;
            char *d = (char *)dev + c0 * e, *h = (char *)host + (K0 * n + c0) * e;
            hipError_t err = kind == hipMemcpyHostToDevice
                                 ? hipMemcpy2DAsync(d, ldd * e, h, n * e, (c1 - c0) * e, SK, kind, s)
                                 : hipMemcpy2DAsync(h, n * e, d, ldd * e, (c1 - c0) * e, SK, kind, s);
            if (err != hipSuccess) return err;
        }
        return hipSuccess;
    };
    auto col_band_copy = [&](void *dev, void *host, size_t e, int64_t K0, int64_t SK, hipMemcpyKind kind,
                             hipStream_t s) -> hipError_t {
        for (auto [r0, r1] : {std::pair<int64_t, int64_t>{0, K0}, {K0 + SK, n}}) {
            if (r1 <= r0) continue;
            char *d = (char *)dev + r0 * S * e, *h = (char *)host + (r0 * n + K0) * e;
            hipError_t err = kind == hipMemcpyHostToDevice
                                 ? hipMemcpy2DAsync(d, S * e, h, n * e, SK * e, r1 - r0, kind, s)
                                 : hipMemcpy2DAsync(h, n * e, d, S * e, SK * e, r1 - r0, kind, s);
            if (err != hipSuccess) return err;
        }
        return hipSuccess;
    };
    for (int64_t R = 0; R < NS; ++R) {
        const int64_t K0 = R * S, SK = edge(R);
        const int cur = (int)(R & 1), nxt = cur ^ 1;
        T *RB = RBs[cur], *CB = CBs[cur];
        int32_t *RBP = RBPs[cur], *CBP = CBPs[cur];
        // 0. The bands.  Super-round 0 uploads them (on the upload stream, while
        // the diagonal block is closed); a later one finds them in its band set,
        // computed there by the previous super-round's first products, except the
        // two tiles that were in that super-round's own bands: (R, R - 1) from its
        // column band and (R - 1, R) from its row band.
        if (NS > 1 && R == 0) {
            FW_TRY(row_band_copy(RB, NP, H, es, K0, SK, H2D, st.h2d));
            FW_TRY(col_band_copy(CB, H, es, K0, SK, H2D, st.h2d));
            FW_TRY(hipEventRecord(st.bands, st.h2d));
        } else if (R > 0) {
            const int64_t Q = R - 1;
            FW_TRY(hipMemcpy2DAsync(RB + Q * S, NP * es, CBs[nxt] + R * S * S, S * es, S * es, S, D2D, cs));
            FW_TRY(hipMemcpy2DAsync(CB + Q * S * S, S * es, RBs[nxt] + R * S, NP * es, S * es, S, D2D, cs));
            if (path) {
                FW_TRY(hipMemcpy2DAsync(RBP + Q * S, NP * is, CBPs[nxt] + R * S * S, S * is, S * is, S, D2D, cs));
                FW_TRY(hipMemcpy2DAsync(CBP + Q * S * S, S * is, RBPs[nxt] + R * S, NP * is, S * is, S, D2D, cs));
            }
            FW_TRY(hipEventRecord(st.bands, cs));  // the other set is free after these copies
        }
        // 1. diagonal super-block, closed in core: from the host in super-round 0,
        // else from the row band (its tile (R, R), computed by the previous
        // super-round)
        FW_TRY(launch_fill_blank<T>(Dd, S, S, S, true, cs));  // padding vertices are isolated
        if (path) FW_TRY(launch_fill_i32(Pd, S * S, -1, cs));
        if (R == 0) {
            FW_TRY(hipMemcpy2DAsync(Dd, S * es, H + K0 * n + K0, n * es, SK * es, SK, H2D, cs));
        } else {
            FW_TRY(hipMemcpy2DAsync(Dd, S * es, RB + K0, NP * es, SK * es, SK, D2D, cs));
            if (path) FW_TRY(hipMemcpy2DAsync(Pd, S * is, RBP + K0, NP * is, SK * is, SK, D2D, cs));
        }
        if (fw_apsp(dt, S, Dd, Ploc, cs) != FW_OK) {
            *what = "in-core closure of the diagonal super-block";
            return hipErrorUnknown;
        }
        FW_TRY(hipMemcpy2DAsync(H + K0 * n + K0, n * es, Dd, S * es, SK * es, SK, D2H, cs));
        if (path) {
            FW_TRY(launch_merge_labels(Pd, Ploc, S * S, (int32_t)K0, cs));
            FW_TRY(hipMemcpy2DAsync(HP + K0 * n + K0, n * is, Pd, S * is, SK * is, SK, D2H, cs));
        }
        if (NS == 1) break;
        if (R == 0) FW_TRY(hipStreamWaitEvent(cs, st.bands, 0));
        // 2. row band; its download overlaps the column band's products
        for (int64_t J = 0; J < NS; ++J) {
            if (J == R) continue;
            FW_TRY(hipMemcpy2DAsync(TMP, S * es, RB + J * S, NP * es, S * es, S, D2D, cs));
            if (path) {
                FW_TRY(hipMemcpy2DAsync(TMPP, S * is, RBP + J * S, NP * is, S * is, S, D2D, cs));
                FW_TRY(launch_minplus_lex<T>(RB + J * S, RBP + J * S, NP, Dd, Pd, S, TMP, TMPP, S, S, S, S,
                                             (int32_t)K0, cs));
            } else {
                FW_TRY(launch_minplus<T>(RB + J * S, NP, Dd, S, TMP, S, S, S, S, cs));
            }
        }
        FW_TRY(hipEventRecord(st.rows_done, cs));
        FW_TRY(hipStreamWaitEvent(st.d2h, st.rows_done, 0));
        FW_TRY(row_band_copy(RB, NP, H, es, K0, SK, D2H, st.d2h));
        if (path) FW_TRY(row_band_copy(RBP, NP, HP, is, K0, SK, D2H, st.d2h));
        // 3. column band; its download overlaps the other super-tiles' products
        for (int64_t I = 0; I < NS; ++I) {
            if (I == R) continue;
            FW_TRY(hipMemcpyAsync(TMP, CB + I * S * S, (size_t)(S * S) * es, D2D, cs));
            if (path) {
                FW_TRY(hipMemcpyAsync(TMPP, CBP + I * S * S, (size_t)(S * S) * is, D2D, cs));
                FW_TRY(launch_minplus_lex<T>(CB + I * S * S, CBP + I * S * S, S, TMP, TMPP, S, Dd, Pd, S, S, S, S,
                                             (int32_t)K0, cs));
            } else {
                FW_TRY(launch_minplus<T>(CB + I * S * S, S, TMP, S, Dd, S, S, S, S, cs));
            }
        }
        FW_TRY(hipEventRecord(st.cols_done, cs));
        FW_TRY(hipStreamWaitEvent(st.d2h, st.cols_done, 0));
        FW_TRY(col_band_copy(CB, H, es, K0, SK, D2H, st.d2h));
        if (path) FW_TRY(col_band_copy(CBP, HP, is, K0, SK, D2H, st.d2h));
        // 4a. Lookahead: super-row and super-column R + 1 of this super-round's
        // update go straight into the next band set, where super-round R + 1
        // reads them as its bands; they are neither downloaded now nor uploaded
        // then (their host copies are stale until super-round R + 1 writes its
        // bands back, and nothing reads them before).  The set is blanked first:
        // its padding rows and columns must read +inf, and the set last held
        // super-round R - 1's bands.
        const int64_t L = R + 1;
        const bool ahead = L < NS;
        if (ahead) {
            T *RN = RBs[nxt], *CN = CBs[nxt];
            int32_t *RNP = RBPs[nxt], *CNP = CBPs[nxt];
            FW_TRY(hipStreamWaitEvent(st.h2d, st.bands, 0));
            FW_TRY(launch_fill_blank<T>(RN, NP, S, NP, false, st.h2d));
            FW_TRY(launch_fill_blank<T>(CN, S, NP, S, false, st.h2d));
            if (path) {
                FW_TRY(launch_fill_i32(RNP, S * NP, -1, st.h2d));
                FW_TRY(launch_fill_i32(CNP, NP * S, -1, st.h2d));
            }
            const int64_t SL = edge(L);
            for (int64_t J = 0; J < NS; ++J) {  // tiles (L, J), the diagonal one included
                if (J == R) continue;
                FW_TRY(hipMemcpy2DAsync(RN + J * S, NP * es, H + L * S * n + J * S, n * es, edge(J) * es, SL, H2D,
                                        st.h2d));
                if (path && R > 0)
                    FW_TRY(hipMemcpy2DAsync(RNP + J * S, NP * is, HP + L * S * n + J * S, n * is, edge(J) * is, SL,
                                            H2D, st.h2d));
            }
            for (int64_t I = 0; I < NS; ++I) {  // tiles (I, L)
                if (I == R || I == L) continue;
                FW_TRY(hipMemcpy2DAsync(CN + I * S * S, S * es, H + I * S * n + L * S, n * es, SL * es, edge(I), H2D,
                                        st.h2d));
                if (path && R > 0)
                    FW_TRY(hipMemcpy2DAsync(CNP + I * S * S, S * is, HP + I * S * n + L * S, n * is, SL * is, edge(I),
                                            H2D, st.h2d));
            }
            FW_TRY(hipEventRecord(st.ahead, st.h2d));
            FW_TRY(hipStreamWaitEvent(cs, st.ahead, 0));
            for (int64_t J = 0; J < NS; ++J) {
                if (J == R) continue;
                if (path)
                    FW_TRY(launch_minplus_lex<T>(RN + J * S, RNP + J * S, NP, CB + L * S * S, CBP + L * S * S, S,
                                                 RB + J * S, RBP + J * S, NP, S, S, S, (int32_t)K0, cs));
                else
                    FW_TRY(launch_minplus<T>(RN + J * S, NP, CB + L * S * S, S, RB + J * S, NP, S, S, S, cs));
            }
            for (int64_t I = 0; I < NS; ++I) {
                if (I == R || I == L) continue;
                if (path)
                    FW_TRY(launch_minplus_lex<T>(CN + I * S * S, CNP + I * S * S, S, CB + I * S * S, CBP + I * S * S, S,
                                                 RB + L * S, RBP + L * S, NP, S, S, S, (int32_t)K0, cs));
                else
                    FW_TRY(launch_minplus<T>(CN + I * S * S, S, CB + I * S * S, S, RB + L * S, NP, S, S, S, cs));
            }
        }
        // 4b. the other super-tiles: upload (h2d) -> product (cs) -> download (d2h).
        // Uploads may start during steps 1-3 (after the bands' and the lookahead
        // tiles' on the same stream): those tiles are disjoint from the blocks and
        // bands written back there.
        int64_t t = 0;
        for (int64_t I = 0; I < NS; ++I) {
            if (I == R || (ahead && I == L)) continue;
            for (int64_t J = 0; J < NS; ++J) {
                if (J == R || (ahead && J == L)) continue;
                const int b = (int)(t & 1);
                const int64_t SI = edge(I), SJ = edge(J);
                T *h = H + I * S * n + J * S;
                int32_t *hp = path ? HP + I * S * n + J * S : nullptr;
                if (t >= 2) FW_TRY(hipStreamWaitEvent(st.h2d, st.stored[b], 0));  // buffer b is free again
                FW_TRY(hipMemcpy2DAsync(Cb[b], S * es, h, n * es, SJ * es, SI, H2D, st.h2d));
                if (path && R > 0) FW_TRY(hipMemcpy2DAsync(CbP[b], S * is, hp, n * is, SJ * is, SI, H2D, st.h2d));
                if (path && R == 0) FW_TRY(launch_fill_i32(CbP[b], S * S, -1, st.h2d));
                FW_TRY(hipEventRecord(st.loaded[b], st.h2d));
                FW_TRY(hipStreamWaitEvent(cs, st.loaded[b], 0));
                if (path)
                    FW_TRY(launch_minplus_lex<T>(Cb[b], CbP[b], S, CB + I * S * S, CBP + I * S * S, S, RB + J * S,
                                                 RBP + J * S, NP, S, S, S, (int32_t)K0, cs));
                else
                    FW_TRY(launch_minplus<T>(Cb[b], S, CB + I * S * S, S, RB + J * S, NP, S, S, S, cs));
                FW_TRY(hipEventRecord(st.computed[b], cs));
                FW_TRY(hipStreamWaitEvent(st.d2h, st.computed[b], 0));
                FW_TRY(hipMemcpy2DAsync(h, n * es, Cb[b], S * es, SJ * es, SI, D2H, st.d2h));
                if (path) FW_TRY(hipMemcpy2DAsync(hp, n * is, CbP[b], S * is, SJ * is, SI, D2H, st.d2h));
                FW_TRY(hipEventRecord(st.stored[b], st.d2h));
                ++t;
            }
        }
        // The next super-round reads what this one wrote back: drain all streams.
        FW_TRY(hipStreamSynchronize(st.d2h));
        FW_TRY(hipStreamSynchronize(st.h2d));
        FW_TRY(hipStreamSynchronize(cs));
    }
    FW_TRY(hipStreamSynchronize(cs));
    return hipSuccess;
}

template hipError_t run_ooc<float>(int64_t, float *, int32_t *, int64_t, hipStream_t, const char **);
template hipError_t run_ooc<double>(int64_t, double *, int32_t *, int64_t, hipStream_t, const char **);

}  // namespace fw
