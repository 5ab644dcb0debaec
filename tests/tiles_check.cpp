// Host-only check of the last-phase tile selections in fw_tiles.h: for grids of
// every tile shape the library compiles and every round, the workgroups of a
// launch visit each selected tile exactly once, a normal launch selects every
// tile outside block row and column r, and with lookahead the cross and rest
// launches split that set into block row / column r + 1 and the remainder.
#include <cstdio>
#include <set>
#include <utility>
#include <algorithm>
#include <vector>

#include "../paper_2105_07298_amd/csrc/fw_tiles.h"

using Tile = std::pair<int, int>;
static int failures = 0;
#define CHECK(cond, ...)                     \
    do {                                     \
        if (!(cond)) {                       \
            if (failures++ < 20) {           \
                std::printf(__VA_ARGS__);    \
                std::printf("\n");           \
            }                                \
        }                                    \
    } while (0)

static bool visit(const fw::TileSel &s, bool cross, std::set<Tile> &out) {
    bool once = true;
    for (int wg = 0; wg < 8 * s.per_xcd; ++wg) {
        int bi = -1, bj = -1;
        const bool ok = cross ? fw::select_tile<true>(s, wg, bi, bj) : fw::select_tile<false>(s, wg, bi, bj);
        if (!ok) continue;
        if (bi < 0 || bi >= s.gm || bj < 0 || bj >= s.gn) return false;
        once &= out.insert({bi, bj}).second;
    }
    return once;
}

int main() {
    long cases = 0;
    for (int TB : {32, 64})
        for (int BM : {16, 32, 64, 128})
            for (int BN : {64, 128, 256}) {
                if (BN < TB) continue;
                const int unit = std::max(TB, std::max(BM, BN));
                for (int ld = unit; ld <= 24 * 64; ld += unit) {
                    const int nb = ld / TB, gm = ld / BM, gn = ld / BN;
                    const int rb = BM <= TB ? TB / BM : 0, cb = BN == TB ? 1 : 0;
                    for (int r = 0; r < nb; ++r) {
                        ++cases;
                        auto row_in = [&](int bi, int blk) { return rb && bi / rb == blk; };
                        auto col_in = [&](int bj, int blk) { return cb && bj == blk; };
                        std::set<Tile> want;
                        for (int bi = 0; bi < gm; ++bi)
                            for (int bj = 0; bj < gn; ++bj)
                                if (!row_in(bi, r) && !col_in(bj, r)) want.insert({bi, bj});
                        fw::TileSel all;
                        CHECK(fw::make_tile_sel(gm, gn, rb, cb, r, nb, 0, all), "all rejected TB=%d BM=%d BN=%d ld=%d", TB, BM, BN, ld);
                        std::set<Tile> got;
                        CHECK(visit(all, false, got), "all: tile twice or out of range TB=%d BM=%d BN=%d ld=%d r=%d", TB, BM, BN, ld, r);
                        CHECK(got == want, "all: wrong set TB=%d BM=%d BN=%d ld=%d r=%d (%zu vs %zu)", TB, BM, BN, ld, r, got.size(), want.size());
                        fw::TileSel cr, rest;
                        const bool la = rb > 0 && cb == 1 && r + 1 < nb;
                        const bool okc = fw::make_tile_sel(gm, gn, rb, cb, r, nb, 1, cr);
                        const bool okr = fw::make_tile_sel(gm, gn, rb, cb, r, nb, 2, rest);
                        fw::TileSel tmp;
                        const bool okp = fw::make_tile_sel(gm, gn, rb, cb, r, nb, 3, tmp);
                        CHECK(okc == la && okr == la && okp == la, "lookahead applicability TB=%d BM=%d BN=%d ld=%d r=%d", TB, BM, BN, ld, r);
                        if (!la) continue;
                        std::set<Tile> gc, gr;
                        CHECK(visit(cr, true, gc), "cross: tile twice or out of range TB=%d BM=%d ld=%d r=%d", TB, BM, ld, r);
                        CHECK(visit(rest, false, gr), "rest: tile twice or out of range TB=%d BM=%d ld=%d r=%d", TB, BM, ld, r);
                        std::set<Tile> wc, wr;
                        for (const Tile &t : want)
                            (row_in(t.first, r + 1) || col_in(t.second, r + 1) ? wc : wr).insert(t);
                        CHECK(gc == wc, "cross: wrong set TB=%d BM=%d ld=%d r=%d (%zu vs %zu)", TB, BM, ld, r, gc.size(), wc.size());
                        CHECK(gr == wr, "rest: wrong set TB=%d BM=%d ld=%d r=%d (%zu vs %zu)", TB, BM, ld, r, gr.size(), wr.size());
                        // Pairs: round r + 1 on block r (skipping block r + 1) plus the same
                        // rest selection covers every tile outside block row / column r + 1.
                        fw::TileSel cp;
                        CHECK(fw::make_tile_sel(gm, gn, rb, cb, r, nb, 3, cp), "cross-prev rejected ld=%d r=%d", ld, r);
                        std::set<Tile> gp;
                        CHECK(visit(cp, true, gp), "cross-prev: tile twice or out of range TB=%d BM=%d ld=%d r=%d", TB, BM, ld, r);
                        std::set<Tile> want1, wp;
                        for (int bi = 0; bi < gm; ++bi)
                            for (int bj = 0; bj < gn; ++bj)
                                if (!row_in(bi, r + 1) && !col_in(bj, r + 1)) want1.insert({bi, bj});
                        for (const Tile &t : want1)
                            if (row_in(t.first, r) || col_in(t.second, r)) wp.insert(t);
                        CHECK(gp == wp, "cross-prev: wrong set TB=%d BM=%d ld=%d r=%d (%zu vs %zu)", TB, BM, ld, r, gp.size(), wp.size());
                        std::set<Tile> uni = gp;
                        uni.insert(gr.begin(), gr.end());
                        CHECK(uni == want1 && uni.size() == gp.size() + gr.size(), "pair cover TB=%d BM=%d ld=%d r=%d", TB, BM, ld, r);
                    }
                }
            }
    std::printf("%ld cases, %d failures\n", cases, failures);
    return failures ? 1 : 0;
}
