/*
 * fw_oracle.c -- plain CPU oracle for all-pairs shortest paths.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or call
 * this file; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * library: it is written from the paper's definitions, deliberately slow and
 * obviously correct.
 *
 * What it computes (paper, Sect. 2.2 "FW Algorithm", Algorithm 1): for a dense
 * N x N distance matrix D (D[i][j] = weight of edge i->j, +infinity when there
 * is no edge, 0 on the diagonal), N outer iterations k = 0..N-1; iteration k
 * tries every pair (i, j) through the intermediate vertex k and, when that is
 * shorter, stores the new length in D[i][j] and k in the path matrix P[i][j].
 *
 * Readings where the paper is silent or ambiguous (all listed in the design doc):
 *   - the update test is strict (a + b < D[i][j]).  Algorithm 1 prints a
 *     non-strict test; with it D is the same but P[i][j] gets overwritten by i
 *     or j (because D[i][i] = 0) and by n-1 for unreachable pairs, so P would no
 *     longer encode paths.
 *   - P starts as -1 everywhere ("no intermediate vertex": the direct edge, or
 *     no path at all).
 *   - infinity is IEEE +inf for real weights; for integer weights the int64
 *     variant uses the sentinel ORACLE_I64_INF and never adds it.
 *
 * Floating point: real weights are computed in double (float inputs widen
 * exactly).  Integer-valued weights use int64, which is exact.
 *
 * Parallelism: the i loop of one k iteration is split over OpenMP threads.  At
 * iteration k row k and column k do not change (D[k][k] = 0 and weights are
 * non-negative), so every thread reads the same values a serial run would and
 * the result is bit-identical to the serial loop.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define ORACLE_I64_INF INT64_MAX

static int pick_threads(int threads) { return threads > 0 ? threads : omp_get_max_threads(); }

/* Classic Floyd-Warshall, double.  D (n*n, row-major) holds W on entry and the
 * shortest distances on exit; P (n*n) receives the intermediate vertex, -1 for
 * "none".  Paper Sect. 2.2, Algorithm 1 (strict test, see header). */
void oracle_fw_f64_steps(int64_t n, double *D, int32_t *P, int64_t k_begin, int64_t k_end, int threads);

void oracle_fw_f64(int64_t n, double *D, int32_t *P, int threads)
{
    for (int64_t x = 0; x < n * n; ++x) P[x] = -1;
    oracle_fw_f64_steps(n, D, P, 0, n, threads);
}

/* Outer iterations k_begin <= k < k_end of the loop above (P already set up).
 * oracle_fw_f64 runs all of them; a prefix of them times the loop on a bounded
 * sample of a large input. */
void oracle_fw_f64_steps(int64_t n, double *D, int32_t *P, int64_t k_begin, int64_t k_end, int threads)
{
    for (int64_t k = k_begin; k < k_end; ++k) {
        const double *rowk = D + k * n;
#pragma omp parallel for schedule(static) num_threads(pick_threads(threads))
        for (int64_t i = 0; i < n; ++i) {
            double a = D[i * n + k];
            if (a == INFINITY) continue;
            double *rowi = D + i * n;
            int32_t *prow = P + i * n;
            for (int64_t j = 0; j < n; ++j) {
                double b = rowk[j];
                double s = a + b;
                if (s < rowi[j]) {          /* ORACLE_UPDATE_TEST */
                    rowi[j] = s;
                    prow[j] = (int32_t)k;   /* ORACLE_PATH_STORE */
                }
            }
        }
    }
}

/* Classic Floyd-Warshall, int64 with an explicit "no edge" sentinel.  Same loop
 * as oracle_fw_f64; a sentinel operand is skipped instead of added. */
void oracle_fw_i64(int64_t n, int64_t *D, int32_t *P, int threads)
{
    for (int64_t x = 0; x < n * n; ++x) P[x] = -1;
    for (int64_t k = 0; k < n; ++k) {
        const int64_t *rowk = D + k * n;
#pragma omp parallel for schedule(static) num_threads(pick_threads(threads))
        for (int64_t i = 0; i < n; ++i) {
            int64_t a = D[i * n + k];
            if (a == ORACLE_I64_INF) continue;
            int64_t *rowi = D + i * n;
            int32_t *prow = P + i * n;
            for (int64_t j = 0; j < n; ++j) {
                int64_t b = rowk[j];
                if (b == ORACLE_I64_INF) continue;
                int64_t s = a + b;
                if (s < rowi[j]) {
                    rowi[j] = s;
                    prow[j] = (int32_t)k;
                }
            }
        }
    }
}

/*
 * Single-source shortest paths by Dijkstra's algorithm on the dense weight
 * matrix (array scan, no heap: O(n^2) per source), with a lexicographic label
 * (length, largest interior vertex) so that the second component reproduces the
 * canonical path-matrix row P[src][*] (the smallest possible "largest interior
 * vertex" over all shortest paths, which is what the strict classic loop
 * stores).  Extending a path by an edge u->v turns the label (d, m) into
 * (d + w, max(m, u)) for u != src and (w, -1) for u == src; with positive exact
 * weights this is strictly increasing and order-preserving, so Dijkstra's
 * argument holds for the pair.  Requires weights > 0 off the diagonal.
 *
 * Independent of Floyd-Warshall: it pins rows of D and P at sizes the cubic
 * oracle cannot reach.  int64 variant for integer weights (exact).
 */
void oracle_dijkstra_i64(int64_t n, const int64_t *W, int64_t src, int64_t *dist, int32_t *pmax)
{
    unsigned char *done = (unsigned char *)calloc((size_t)n, 1);
    for (int64_t v = 0; v < n; ++v) { dist[v] = ORACLE_I64_INF; pmax[v] = -1; }
    dist[src] = 0;
    for (;;) {
        int64_t u = -1;
        for (int64_t v = 0; v < n; ++v) {
            if (done[v] || dist[v] == ORACLE_I64_INF) continue;
            if (u < 0 || dist[v] < dist[u] || (dist[v] == dist[u] && pmax[v] < pmax[u])) u = v;
        }
        if (u < 0) break;
        done[u] = 1;
        int32_t mu = (u == src) ? -1 : (pmax[u] > (int32_t)u ? pmax[u] : (int32_t)u);
        const int64_t *wu = W + u * n;
        for (int64_t v = 0; v < n; ++v) {
            if (done[v] || v == u || wu[v] == ORACLE_I64_INF) continue;
            int64_t s = dist[u] + wu[v];
            if (s < dist[v] || (s == dist[v] && mu < pmax[v])) { dist[v] = s; pmax[v] = mu; }
        }
    }
    free(done);
}

/* Same as oracle_dijkstra_i64 in double (IEEE +inf = no edge).  With real
 * weights only the distance row is meaningful as a pin (rounding can reorder
 * near-ties), which is how the tests use it. */
void oracle_dijkstra_f64(int64_t n, const double *W, int64_t src, double *dist, int32_t *pmax)
{
    unsigned char *done = (unsigned char *)calloc((size_t)n, 1);
    for (int64_t v = 0; v < n; ++v) { dist[v] = INFINITY; pmax[v] = -1; }
    dist[src] = 0.0;
    for (;;) {
        int64_t u = -1;
        for (int64_t v = 0; v < n; ++v) {
            if (done[v] || dist[v] == INFINITY) continue;
            if (u < 0 || dist[v] < dist[u] || (dist[v] == dist[u] && pmax[v] < pmax[u])) u = v;
        }
        if (u < 0) break;
        done[u] = 1;
        int32_t mu = (u == src) ? -1 : (pmax[u] > (int32_t)u ? pmax[u] : (int32_t)u);
        const double *wu = W + u * n;
        for (int64_t v = 0; v < n; ++v) {
            if (done[v] || v == u || wu[v] == INFINITY) continue;
            double s = dist[u] + wu[v];
            if (s < dist[v] || (s == dist[v] && mu < pmax[v])) { dist[v] = s; pmax[v] = mu; }
        }
    }
    free(done);
}

/* oracle_dijkstra_i64 for integer-valued weights stored as float (is_f64 = 0) or
 * double (is_f64 = 1): every finite weight is converted exactly to int64 when
 * it is read, +inf is "no edge".  Avoids an int64 copy of a very large matrix. */
static void dijkstra_floatint(int64_t n, const void *Wv, int is_f64, int64_t src, int64_t *dist, int32_t *pmax)
{
    unsigned char *done = (unsigned char *)calloc((size_t)n, 1);
    for (int64_t v = 0; v < n; ++v) { dist[v] = ORACLE_I64_INF; pmax[v] = -1; }
    dist[src] = 0;
    for (;;) {
        int64_t u = -1;
        for (int64_t v = 0; v < n; ++v) {
            if (done[v] || dist[v] == ORACLE_I64_INF) continue;
            if (u < 0 || dist[v] < dist[u] || (dist[v] == dist[u] && pmax[v] < pmax[u])) u = v;
        }
        if (u < 0) break;
        done[u] = 1;
        int32_t mu = (u == src) ? -1 : (pmax[u] > (int32_t)u ? pmax[u] : (int32_t)u);
        for (int64_t v = 0; v < n; ++v) {
            double w = is_f64 ? ((const double *)Wv)[u * n + v] : (double)((const float *)Wv)[u * n + v];
            if (done[v] || v == u || w == INFINITY) continue;
            int64_t s = dist[u] + (int64_t)w;
            if (s < dist[v] || (s == dist[v] && mu < pmax[v])) { dist[v] = s; pmax[v] = mu; }
        }
    }
    free(done);
}

void oracle_dijkstra_rows_floatint(int64_t n, const void *W, int is_f64, int64_t nsrc, const int64_t *srcs,
                                   int64_t *dist, int32_t *pmax, int threads)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(pick_threads(threads))
    for (int64_t s = 0; s < nsrc; ++s)
        dijkstra_floatint(n, W, is_f64, srcs[s], dist + s * n, pmax + s * n);
}

/*
 * The same lexicographic single-source labels for positive integer weights
 * (1 <= w <= wmax, held as float or double, +inf = no edge), by Dial's form of
 * Dijkstra's algorithm: vertices wait in buckets indexed by tentative distance;
 * since every edge is at least 1, all of bucket d is final when the scan reaches
 * it, and relaxing it only fills buckets d+1 .. d+wmax, so a ring of wmax+1
 * buckets suffices.  Within a bucket the order of relaxation does not matter
 * (each target keeps the smallest label it is offered).  No minimum scan: one
 * pass over the row of each reached vertex.  Doubly linked lists move a vertex
 * to a lower bucket when its distance drops.
 */
/* A row source for graphs too large to hold in host memory: rowfn(ctx, u, out)
 * writes row u of the weight matrix (n doubles, +inf = no edge) to out. */
typedef void (*oracle_row_fn)(const void *ctx, int64_t u, double *out);

static void dial_one(int64_t n, const void *Wv, int is_f64, oracle_row_fn rowfn, const void *ctx, int64_t wmax,
                     int64_t src, int64_t *dist, int32_t *pmax)
{
    double *rowbuf = rowfn ? (double *)malloc(sizeof(double) * (size_t)n) : NULL;
    const int64_t nb = wmax + 1;
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * (size_t)nb);
    int64_t *nxt = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *prv = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    double *dd = (double *)malloc(sizeof(double) * (size_t)n); /* distances; integers, exact in double */
    unsigned char *queued_v = (unsigned char *)calloc((size_t)n, 1);
    for (int64_t b = 0; b < nb; ++b) head[b] = -1;
    for (int64_t v = 0; v < n; ++v) { dd[v] = INFINITY; pmax[v] = -1; }
#define DIAL_PUSH(v)  do { int64_t b_ = (int64_t)dd[v] % nb; prv[v] = -1; nxt[v] = head[b_]; \
                           if (head[b_] >= 0) prv[head[b_]] = (v); \
                           head[b_] = (v); queued_v[v] = 1; } while (0)
#define DIAL_UNLINK(v) do { int64_t b_ = (int64_t)dd[v] % nb; \
                            if (prv[v] >= 0) nxt[prv[v]] = nxt[v]; else head[b_] = nxt[v]; \
                            if (nxt[v] >= 0) prv[nxt[v]] = prv[v]; \
                            queued_v[v] = 0; } while (0)
    dd[src] = 0.0;
    DIAL_PUSH(src);
    int64_t queued = 1;
    for (int64_t d = 0; queued > 0; ++d) {
        const int64_t b = d % nb;
        const double df = (double)d;
        while (head[b] >= 0) {
            const int64_t u = head[b];
            DIAL_UNLINK(u);
            --queued;
            const int32_t mu = (u == src) ? -1 : (pmax[u] > (int32_t)u ? pmax[u] : (int32_t)u);
            const float *rf = rowfn ? NULL : (const float *)Wv + u * n;
            const double *rd = rowfn ? rowbuf : (const double *)Wv + u * n;
            if (rowfn) rowfn(ctx, u, rowbuf);
            /* A vertex already taken has a distance <= d < d + w, and a missing edge
             * gives +inf, so neither passes the tests below. */
            for (int64_t v = 0; v < n; ++v) {
                const double w = (rowfn || is_f64) ? rd[v] : (double)rf[v];
                const double sv = df + w;
                if (sv < dd[v]) {
                    if (queued_v[v]) DIAL_UNLINK(v); else ++queued;
                    dd[v] = sv;
                    pmax[v] = mu;
                    DIAL_PUSH(v);
                } else if (sv == dd[v] && mu < pmax[v] && v != u) {
                    pmax[v] = mu;
                }
            }
        }
    }
#undef DIAL_PUSH
#undef DIAL_UNLINK
    for (int64_t v = 0; v < n; ++v) dist[v] = (dd[v] == INFINITY) ? ORACLE_I64_INF : (int64_t)dd[v];
    free(head); free(nxt); free(prv); free(dd); free(queued_v); free(rowbuf);
}

void oracle_dial_rows(int64_t n, const void *W, int is_f64, int64_t wmax, int64_t nsrc, const int64_t *srcs,
                      int64_t *dist, int32_t *pmax, int threads)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(pick_threads(threads))
    for (int64_t s = 0; s < nsrc; ++s)
        dial_one(n, W, is_f64, NULL, NULL, wmax, srcs[s], dist + s * n, pmax + s * n);
}

/* The same with every row read through rowfn when its vertex is settled (the
 * matrix itself never exists in host memory; each source reads each reached row
 * once).  rowfn must be safe to call from several threads at once. */
void oracle_dial_rows_fn(int64_t n, oracle_row_fn rowfn, const void *ctx, int64_t wmax, int64_t nsrc,
                         const int64_t *srcs, int64_t *dist, int32_t *pmax, int threads)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(pick_threads(threads))
    for (int64_t s = 0; s < nsrc; ++s)
        dial_one(n, NULL, 1, rowfn, ctx, wmax, srcs[s], dist + s * n, pmax + s * n);
}

/* Many sources at once, one source per thread (for sampled-row verification of
 * large graphs).  dist/pmax are nsrc x n. */
void oracle_dijkstra_rows_i64(int64_t n, const int64_t *W, int64_t nsrc, const int64_t *srcs,
                              int64_t *dist, int32_t *pmax, int threads)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(pick_threads(threads))
    for (int64_t s = 0; s < nsrc; ++s)
        oracle_dijkstra_i64(n, W, srcs[s], dist + s * n, pmax + s * n);
}

void oracle_dijkstra_rows_f64(int64_t n, const double *W, int64_t nsrc, const int64_t *srcs,
                              double *dist, int32_t *pmax, int threads)
{
#pragma omp parallel for schedule(dynamic, 1) num_threads(pick_threads(threads))
    for (int64_t s = 0; s < nsrc; ++s)
        oracle_dijkstra_f64(n, W, srcs[s], dist + s * n, pmax + s * n);
}

/*
 * Gradient of L(D(W)) with respect to W, by walking every shortest path.
 *
 * D[i][j] is the sum of the edge weights on the path that P encodes, so
 * dD[i][j]/dW[u][v] is 1 when edge u->v lies on that path and 0 otherwise
 * (D is piecewise linear in W; at ties this is the subgradient along the
 * encoded path).  Hence dL/dW[u][v] = sum over pairs (i, j) whose path uses
 * u->v of G[i][j].  The path of (i, j) is the edge i->j when P[i][j] = -1, and
 * otherwise the path of (i, P[i][j]) followed by the path of (P[i][j], j).
 * Pairs with i == j or D[i][j] = +inf contribute nothing.  Accumulates in
 * double.  O(sum of path lengths).  Not parallel: the scatter is plain.
 */
int oracle_backward_pathwalk_f64(int64_t n, const double *D, const int32_t *P, const double *G, double *gW)
{
    memset(gW, 0, sizeof(double) * (size_t)(n * n));
    int64_t cap = 64, top;
    int64_t *stk = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)cap);
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            if (i == j || D[i * n + j] == INFINITY) continue;
            double g = G[i * n + j];
            top = 0;
            stk[0] = i; stk[1] = j; top = 1;
            while (top > 0) {
                --top;
                int64_t a = stk[2 * top], b = stk[2 * top + 1];
                int32_t m = P[a * n + b];
                if (m < 0) { gW[a * n + b] += g; continue; }
                if (m == a || m == b || m >= n) { free(stk); return -1; } /* not a path encoding */
                if (top + 2 > cap) {
                    if (cap > 2 * n + 4) { free(stk); return -1; }             /* cyclic encoding */
                    cap *= 2;
                    stk = (int64_t *)realloc(stk, sizeof(int64_t) * 2 * (size_t)cap);
                }
                stk[2 * top] = m; stk[2 * top + 1] = b; ++top;
                stk[2 * top] = a; stk[2 * top + 1] = m; ++top;
            }
        }
    }
    free(stk);
    return 0;
}

/* Reconstruct path (i -> j) from P into out[] (vertex list, including i and j).
 * Returns the number of vertices, 0 if unreachable/none, or -1 if the encoding
 * is invalid or longer than cap.  Used by the invariant checks. */
int64_t oracle_reconstruct(int64_t n, const int32_t *P, int64_t i, int64_t j, int64_t *out, int64_t cap)
{
    if (i == j) { if (cap < 1) return -1; out[0] = i; return 1; }
    int64_t len = 0;
    int64_t scap = 2 * n + 4, top = 0;
    int64_t *stk = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)scap);
    stk[0] = i; stk[1] = j; top = 1;
    if (len >= cap) { free(stk); return -1; }
    out[len++] = i;
    while (top > 0) {
        --top;
        int64_t a = stk[2 * top], b = stk[2 * top + 1];
        int32_t m = P[a * n + b];
        if (m < 0) {
            if (len >= cap) { free(stk); return -1; }
            out[len++] = b;
            continue;
        }
        if (m == a || m == b || m >= n || top + 2 > scap) { free(stk); return -1; }
        stk[2 * top] = m; stk[2 * top + 1] = b; ++top;
        stk[2 * top] = a; stk[2 * top + 1] = m; ++top;
    }
    free(stk);
    return len;
}

/*
 * Walk the encoded paths of rows rows[0..nrows) of P and add up their weights
 * (the checker of a path matrix; what P must encode follows from Sect. 2.2,
 * Algorithm 1: P[i][j] = k names an intermediate vertex, so the path of (i, j) is
 * the path of (i, k) followed by the path of (k, j), and -1 means the edge i->j
 * itself).
 *
 * For source i = rows[q] and every j != i: S[q][j] = sum of W over the edges of
 * the encoded path, summed in path order in double (+inf when it uses a missing
 * edge), and H[q][j] = its number of edges.  H[q][j] = -1 marks an encoding that
 * is no path: a label equal to an endpoint or outside [-1, n), a walk that would
 * need more than n - 1 edges, or a recursion deeper than 2n (a cyclic encoding).
 * j == i gets S = 0, H = 0.  Parallel over the rows (pairs are independent).
 */
void oracle_path_sums_rows_f64(int64_t n, const double *W, const int32_t *P, int64_t nrows, const int64_t *rows,
                               double *S, int64_t *H, int threads)
{
#pragma omp parallel num_threads(pick_threads(threads))
    {
        int64_t scap = 2 * n + 4;
        int64_t *stk = (int64_t *)malloc(sizeof(int64_t) * 2 * (size_t)scap);
#pragma omp for schedule(dynamic, 4)
        for (int64_t q = 0; q < nrows; ++q) {
            const int64_t i = rows[q];
            for (int64_t j = 0; j < n; ++j) {
                if (i == j) { S[q * n + j] = 0.0; H[q * n + j] = 0; continue; }
                double sum = 0.0;
                int64_t edges = 0, top = 1, bad = 0;
                stk[0] = i; stk[1] = j;
                while (top > 0) {
                    --top;
                    int64_t a = stk[2 * top], b = stk[2 * top + 1];
                    int32_t m = P[a * n + b];
                    if (m == -1) {
                        if (++edges > n - 1) { bad = 1; break; }
                        sum += W[a * n + b];
                        continue;
                    }
                    if (m < -1 || m >= n || m == a || m == b || top + 2 > scap) { bad = 1; break; }
                    stk[2 * top] = m; stk[2 * top + 1] = b; ++top;
                    stk[2 * top] = a; stk[2 * top + 1] = m; ++top;
                }
                S[q * n + j] = bad ? NAN : sum;
                H[q * n + j] = bad ? -1 : edges;
            }
        }
        free(stk);
    }
}

/*
 * Triangle inequality D[i][j] <= (D[i][k] + D[k][j]) (1 + rtol) for every i in
 * rows[0..nrows), every j and every k in ks[0..nk) (shortest distances satisfy
 * it for every k).  Returns the number of violating (i, j, k); +inf sums never
 * violate.
 */
int64_t oracle_triangle_violations_rows(int64_t n, const double *D, int64_t nrows, const int64_t *rows,
                                        const int64_t *ks, int64_t nk, double rtol, int threads)
{
    int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad) num_threads(pick_threads(threads))
    for (int64_t q = 0; q < nrows; ++q) {
        const double *rowi = D + rows[q] * n;
        for (int64_t t = 0; t < nk; ++t) {
            const int64_t k = ks[t];
            const double a = rowi[k];
            if (a == INFINITY) continue;
            const double *rowk = D + k * n;
            for (int64_t j = 0; j < n; ++j) {
                const double via = a + rowk[j];
                if (via != INFINITY && rowi[j] > via + rtol * via) ++bad;
            }
        }
    }
    return bad;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
