/*
 * gen.c -- seeded synthetic graph generator (inputs only; no shortest-path
 * arithmetic).  Both the HIP library's tests/benchmark and the CPU oracle take
 * their inputs from here, so the two sides always see the same weight bits.
 *
 * Every random draw is one output of SplitMix64 (Steele, Lea & Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014): the generator state
 * advances by the golden-ratio increment 0x9E3779B97F4A7C15 and each output is
 * the state passed through the mix64 finaliser below.  A draw is addressed by a
 * counter, so any entry (or row) can be regenerated on its own:
 *
 *   base(seed, stream)      = mix64(seed * GOLDEN + stream)
 *   gkey(seed, stream, g)   = mix64(base ^ (g * 0xD1B54A32D192ED03))
 *   draw(seed,stream,g,i,j) = mix64(gkey + (idx + 1) * GOLDEN),  idx = i * 2^32 + j
 *
 * i.e. draw is output number idx of the SplitMix64 sequence started at gkey.
 * Streams: 0 edge presence, 1 weight, 2 upstream gradient, 3 per-graph vertex
 * count, 4 per-graph density.
 */
#include <stdint.h>
#include <math.h>
#include <omp.h>

#define GOLDEN 0x9E3779B97F4A7C15ull

static inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t gen_gkey(uint64_t seed, uint64_t stream, uint64_t g)
{
    uint64_t base = mix64(seed * GOLDEN + stream);
    return mix64(base ^ (g * 0xD1B54A32D192ED03ull));
}

static inline uint64_t draw(uint64_t gkey, uint64_t i, uint64_t j)
{
    uint64_t idx = (i << 32) | j;
    return mix64(gkey + (idx + 1) * GOLDEN);
}

uint64_t gen_draw(uint64_t seed, uint64_t stream, uint64_t g, uint64_t i, uint64_t j)
{
    return draw(gen_gkey(seed, stream, g), i, j);
}

/* Weight laws (the value for one present edge from one 64-bit draw h). */
enum {
    W_INT = 0,        /* 1 + floor(u32 * wmax / 2^32), u32 = h >> 32: integer in [1, wmax]   */
    W_UNIT_OPEN = 1,  /* (2b + 1) * 2^-(B+1), b = top B bits: exact, inside (0, 1)            */
    W_ONE_TEN = 2,    /* 1 + 9 * (2b + 1) * 2^-24 (b = top 23 bits), in double, then to float  */
    W_ONE_TWO = 3     /* 1 + b * 2^-23 (b = top 23 bits): exact float in [1, 2)              */
};

static inline double weight_of(int law, uint64_t h, int64_t wmax, int is_f64)
{
    switch (law) {
    case W_INT:
        return (double)(1 + (int64_t)(((h >> 32) * (uint64_t)wmax) >> 32));
    case W_UNIT_OPEN:
        if (is_f64) return (double)(2 * (h >> 12) + 1) * 0x1p-53;
        return (double)(2 * (h >> 41) + 1) * 0x1p-24;
    case W_ONE_TEN:
        return 1.0 + 9.0 * ((double)(2 * (h >> 41) + 1) * 0x1p-24);
    case W_ONE_TWO:
        return 1.0 + (double)(h >> 41) * 0x1p-23;
    }
    return NAN;
}

/* Edge i->j (i != j) is present when the stream-0 draw's top 32 bits fall below
 * thresh32 = floor(p * 2^32) (thresh32 >= 2^32 means "always"). */
static inline int present(uint64_t ekey, uint64_t i, uint64_t j, uint64_t thresh32)
{
    if (thresh32 >= (1ull << 32)) return 1;
    return (draw(ekey, i, j) >> 32) < thresh32;
}

/* Rows [r0, r1) of graph g (n vertices) into out (row-major, leading dim n,
 * out points at row r0).  Diagonal 0, missing edges +inf. */
void gen_rows_f32(uint64_t seed, uint64_t g, int64_t n, int64_t r0, int64_t r1, uint64_t thresh32,
                  int law, int64_t wmax, float *out)
{
    uint64_t ek = gen_gkey(seed, 0, g), wk = gen_gkey(seed, 1, g);
#pragma omp parallel for schedule(static)
    for (int64_t i = r0; i < r1; ++i) {
        float *row = out + (i - r0) * n;
        for (int64_t j = 0; j < n; ++j) {
            if (i == j) { row[j] = 0.0f; continue; }
            if (!present(ek, (uint64_t)i, (uint64_t)j, thresh32)) { row[j] = INFINITY; continue; }
            row[j] = (float)weight_of(law, draw(wk, (uint64_t)i, (uint64_t)j), wmax, 0);
        }
    }
}

void gen_rows_f64(uint64_t seed, uint64_t g, int64_t n, int64_t r0, int64_t r1, uint64_t thresh32,
                  int law, int64_t wmax, double *out)
{
    uint64_t ek = gen_gkey(seed, 0, g), wk = gen_gkey(seed, 1, g);
#pragma omp parallel for schedule(static)
    for (int64_t i = r0; i < r1; ++i) {
        double *row = out + (i - r0) * n;
        for (int64_t j = 0; j < n; ++j) {
            if (i == j) { row[j] = 0.0; continue; }
            if (!present(ek, (uint64_t)i, (uint64_t)j, thresh32)) { row[j] = INFINITY; continue; }
            row[j] = weight_of(law, draw(wk, (uint64_t)i, (uint64_t)j), wmax, 1);
        }
    }
}

/* One row of a graph, serially, for callers that regenerate rows on demand (a
 * search over a matrix too large to keep in host memory): the graph is described
 * by ctx, row i is written to out as n doubles, with the value gen_rows_f32 or
 * gen_rows_f64 gives that entry (so float rows are rounded to float first).
 * Safe to call from several threads at once. */
typedef struct {
    uint64_t seed, g;
    int64_t n;
    uint64_t thresh32;
    int32_t law, is_f64;
    int64_t wmax;
} gen_graph_t;

void gen_row_cb(const void *ctx, int64_t i, double *out)
{
    const gen_graph_t *G = (const gen_graph_t *)ctx;
    const uint64_t ek = gen_gkey(G->seed, 0, G->g), wk = gen_gkey(G->seed, 1, G->g);
    for (int64_t j = 0; j < G->n; ++j) {
        if (i == j) { out[j] = 0.0; continue; }
        if (!present(ek, (uint64_t)i, (uint64_t)j, G->thresh32)) { out[j] = INFINITY; continue; }
        const double w = weight_of(G->law, draw(wk, (uint64_t)i, (uint64_t)j), G->wmax, G->is_f64);
        out[j] = G->is_f64 ? w : (double)(float)w;
    }
}

/* Standard normal draws (Box-Muller on two stream-2 uniforms), n x n, float32.
 * u1 = (top53(h1) + 1) * 2^-53 in (0, 1], u2 = top53(h2) * 2^-53 in [0, 1),
 * h1 = draw(i, 2j), h2 = draw(i, 2j + 1); z = sqrt(-2 ln u1) cos(2 pi u2). */
void gen_normal_f32(uint64_t seed, uint64_t g, int64_t n, float *out)
{
    uint64_t key = gen_gkey(seed, 2, g);
    const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double u1 = (double)((draw(key, (uint64_t)i, (uint64_t)(2 * j)) >> 11) + 1) * 0x1p-53;
            double u2 = (double)(draw(key, (uint64_t)i, (uint64_t)(2 * j + 1)) >> 11) * 0x1p-53;
            out[i * n + j] = (float)(sqrt(-2.0 * log(u1)) * cos(two_pi * u2));
        }
    }
}

/* Per-graph vertex count, uniform integer in [lo, hi]: lo + floor(u32 * (hi-lo+1) / 2^32). */
int64_t gen_graph_n(uint64_t seed, uint64_t g, int64_t lo, int64_t hi)
{
    uint64_t h = gen_draw(seed, 3, g, 0, 0);
    return lo + (int64_t)(((h >> 32) * (uint64_t)(hi - lo + 1)) >> 32);
}

/* Per-graph edge density, uniform real in [lo, hi): lo + (hi - lo) * top53(h) * 2^-53. */
double gen_graph_density(uint64_t seed, uint64_t g, double lo, double hi)
{
    uint64_t h = gen_draw(seed, 4, g, 0, 0);
    return lo + (hi - lo) * ((double)(h >> 11) * 0x1p-53);
}

int gen_max_threads(void) { return omp_get_max_threads(); }
