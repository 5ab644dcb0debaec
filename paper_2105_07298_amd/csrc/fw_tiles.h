// fw_tiles.h -- which output tiles one last-phase launch updates, and which
// workgroup takes which tile.  Plain C++ shared by the kernels (FW_TILE_FN set
// to a host/device inline), by the host runtime and by a host-only test of the
// selections and round schedules.
#pragma once
#include <stdint.h>

#ifndef FW_TILE_FN
#define FW_TILE_FN inline
#endif

namespace fw {

// Last-phase launch modes.  r is the round applied (the first of the two for a
// fused pair), R the number of blocks:
//   all             every tile outside block row and column r;
//   cross           block row and column r + 1, outside block r: what phases 1-3
//                   of round r + 1 read and write;
//   rest            every tile outside block rows and columns r and r + 1;
//   crossprev       block row and column r - 1, outside block r (round r applied
//                   to the block before it);
//   pair            rounds r and r + 1 in one pass over the rest tiles;
//   pair_band       rounds r and r + 1 on block rows and columns r + 2 and r + 3
//                   (those below R), outside blocks r and r + 1;
//   pair_rest       rounds r and r + 1 on every tile outside blocks r .. r + 3;
//   crossprev_band  round r on the tiles (r - 1, j) and (j, r - 1) with j in
//                   r + 1 .. r + 2;
//   crossprev_rest  round r on the rest of block row and column r - 1: outside
//                   blocks r .. r + 2.
// pair_band + pair_rest = pair, and crossprev_band + crossprev_rest = crossprev
// (on the same r), which is how the pairs-with-lookahead schedule splits a pair
// of rounds between two streams.
enum class P4Mode { all, cross, rest, crossprev, pair, pair_band, pair_rest, crossprev_band, crossprev_rest };

// Tiles of one last-phase launch over a gm x gn grid of BM x BN tiles.
//   Normal selection: every tile outside tile rows [sr, sr + nsr) and tile
//   columns [sc, sc + nsc).  A block row (column) of the round that is narrower
//   than a tile is not skipped (nsr or nsc = 0) but masked inside its tile.
//   Band selection (tiles one block wide, rb tile rows per block): the tiles of
//   block rows and block columns [cross, cross + bw), except those in block
//   rows / columns [xs, xs + wx) (the two ranges disjoint).  bw = wx = 1 with
//   xs = cross - 1 is round cross - 1's cross launch; xs = cross + 1 round
//   cross + 1's cross-previous launch.
//   List selection (nl > 0): the nl tiles (li[k], lj[k]).
struct TileSel {
    int gm, gn;
    int sr, nsr, sc, nsc;
    int cross, xs, rb, bw, wx;
    int nl, li[4], lj[4];
    int per_xcd, ntiles;
};

FW_TILE_FN void tile_sel_init(int gm, int gn, int rb, TileSel &sel) {
    sel.gm = gm;
    sel.gn = gn;
    sel.sr = gm;
    sel.nsr = 0;
    sel.sc = gn;
    sel.nsc = 0;
    sel.cross = -1;
    sel.xs = -1;
    sel.rb = rb;
    sel.bw = 0;
    sel.wx = 0;
    sel.nl = 0;
    for (int k = 0; k < 4; ++k) sel.li[k] = sel.lj[k] = 0;
    sel.per_xcd = 0;
    sel.ntiles = 0;
}

FW_TILE_FN bool tile_sel_count(int64_t ntiles, TileSel &sel) {
    if (ntiles < 0 || ntiles > (int64_t)1 << 30) return false;
    sel.ntiles = (int)ntiles;
    sel.per_xcd = (int)((ntiles + 7) / 8);
    return true;
}

// Band selection; needs rb >= 1 tile rows per block, tiles one block wide, both
// ranges inside [0, nblocks) and disjoint.
FW_TILE_FN bool make_band_sel(int gm, int gn, int rb, int cb, int c, int bw, int xs, int wx, int nblocks,
                              TileSel &sel) {
    tile_sel_init(gm, gn, rb, sel);
    if (rb == 0 || cb != 1 || bw < 1 || wx < 1 || c < 0 || xs < 0 || c + bw > nblocks || xs + wx > nblocks)
        return false;
    if (!(c + bw <= xs || xs + wx <= c)) return false;
    sel.cross = c;
    sel.bw = bw;
    sel.xs = xs;
    sel.wx = wx;
    sel.nsr = rb;  // tiles never straddle a block: nothing to mask
    sel.nsc = 1;
    return tile_sel_count((int64_t)bw * rb * (gn - wx) + (int64_t)bw * (gm - (int64_t)(bw + wx) * rb), sel);
}

// Every tile outside block rows and columns [r, r + w).
FW_TILE_FN bool make_rest_sel(int gm, int gn, int rb, int cb, int r, int w, int nblocks, TileSel &sel) {
    tile_sel_init(gm, gn, rb, sel);
    if (rb == 0 || cb != 1 || w < 1 || r < 0 || r + w > nblocks) return false;
    sel.sr = r * rb;
    sel.nsr = w * rb;
    sel.sc = r;
    sel.nsc = w;
    return tile_sel_count((int64_t)(gm - sel.nsr) * (gn - sel.nsc), sel);
}

// Launch modes all, cross, rest, crossprev (and pair, which selects like rest):
// rb / cb are the tile rows / columns per block (0 when a tile is wider than the
// block).  Fills sel for round r of nblocks; false if the mode does not apply.
FW_TILE_FN bool make_tile_sel(int gm, int gn, int rb, int cb, int r, int nblocks, int mode, TileSel &sel) {
    if (mode == 1) return make_band_sel(gm, gn, rb, cb, r + 1, 1, r, 1, nblocks, sel);
    if (mode == 3) return make_band_sel(gm, gn, rb, cb, r, 1, r + 1, 1, nblocks, sel);
    if (mode == 2) return make_rest_sel(gm, gn, rb, cb, r, 2, nblocks, sel);
    tile_sel_init(gm, gn, rb, sel);
    if (rb) {
        sel.sr = r * rb;
        sel.nsr = rb;
    }
    if (cb) {
        sel.sc = r * cb;
        sel.nsc = cb;
    }
    return tile_sel_count((int64_t)(gm - sel.nsr) * (gn - sel.nsc), sel);
}

// The selection of one launch of mode `mode` applying round r (tiles one block
// square for the pair_* and *_band / *_rest modes).  band = true when the
// kernel must take tiles from the band / list form, fuse = true when the launch
// applies rounds r and r + 1.
FW_TILE_FN bool p4_select(int gm, int gn, int rb, int cb, int r, int nblocks, P4Mode mode, TileSel &sel, bool &band,
                          bool &fuse) {
    band = mode == P4Mode::cross || mode == P4Mode::crossprev || mode == P4Mode::pair_band ||
           mode == P4Mode::crossprev_band || mode == P4Mode::crossprev_rest;
    fuse = mode == P4Mode::pair || mode == P4Mode::pair_band || mode == P4Mode::pair_rest;
    if (fuse && r + 2 > nblocks) return false;
    switch (mode) {
    case P4Mode::all: return make_tile_sel(gm, gn, rb, cb, r, nblocks, 0, sel);
    case P4Mode::cross: return make_tile_sel(gm, gn, rb, cb, r, nblocks, 1, sel);
    case P4Mode::rest:
    case P4Mode::pair: return make_tile_sel(gm, gn, rb, cb, r, nblocks, 2, sel);
    case P4Mode::crossprev: return r >= 1 && make_tile_sel(gm, gn, rb, cb, r - 1, nblocks, 3, sel);
    case P4Mode::pair_band: {
        const int bw = nblocks - (r + 2) < 2 ? nblocks - (r + 2) : 2;
        return bw >= 1 && make_band_sel(gm, gn, rb, cb, r + 2, bw, r, 2, nblocks, sel);
    }
    case P4Mode::pair_rest: {
        const int w = nblocks - r < 4 ? nblocks - r : 4;
        return make_rest_sel(gm, gn, rb, cb, r, w, nblocks, sel);
    }
    case P4Mode::crossprev_band: {
        const int b = r - 1, bw = nblocks - (b + 2) < 2 ? nblocks - (b + 2) : 2;
        tile_sel_init(gm, gn, rb, sel);
        if (b < 0 || bw < 1 || rb != 1 || cb != 1) return false;
        sel.nsr = rb;
        sel.nsc = 1;
        for (int k = 0; k < bw; ++k) {
            sel.li[2 * k] = b;
            sel.lj[2 * k] = b + 2 + k;
            sel.li[2 * k + 1] = b + 2 + k;
            sel.lj[2 * k + 1] = b;
        }
        sel.nl = 2 * bw;
        return tile_sel_count(sel.nl, sel);
    }
    case P4Mode::crossprev_rest: {
        const int b = r - 1, wx = nblocks - (b + 1) < 3 ? nblocks - (b + 1) : 3;
        return b >= 0 && wx >= 1 && make_band_sel(gm, gn, rb, cb, b, 1, b + 1, wx, nblocks, sel);
    }
    }
    return false;
}

// Tile (bi, bj) of workgroup wg of a launch with 8 * per_xcd workgroups; false
// for the workgroups that pad the grid.  Workgroups go round-robin over the 8
// XCDs and each XCD takes a contiguous range of the tile sequence, walked in
// groups of 8 tile rows so that the workgroups resident on one XCD share
// panels in its L2.  BAND selects the band / list forms.
template <bool BAND>
FW_TILE_FN bool select_tile(const TileSel &t, int wg, int &bi, int &bj) {
    const int lin = (wg % 8) * t.per_xcd + wg / 8;
    if (lin >= t.ntiles) return false;
    if (BAND) {
        if (t.nl) {
            bi = t.li[lin];
            bj = t.lj[lin];
            return true;
        }
        const int c = t.cross, xs = t.xs, bw = t.bw, wx = t.wx, rb = t.rb;
        const int nrow = bw * rb * (t.gn - wx);
        if (lin < nrow) {  // the band's tile rows, every column outside the skip range
            bi = c * rb + lin % (bw * rb);
            const int jj = lin / (bw * rb);
            bj = jj < xs ? jj : jj + wx;
        } else {  // the band's columns, every tile row outside the band and the skip range
            const int ii = lin - nrow;
            bj = c + ii % bw;
            const bool band_first = c < xs;
            const int lo = band_first ? c : xs, wlo = band_first ? bw : wx;
            const int hi = band_first ? xs : c, whi = band_first ? wx : bw;
            int i = ii / bw;
            if (i >= lo * rb) i += wlo * rb;
            if (i >= hi * rb) i += whi * rb;
            bi = i;
        }
        return true;
    }
    const int gm_e = t.gm - t.nsr, gn_e = t.gn - t.nsc;
    const int G = 8;
    const int group = lin / (G * gn_e);
    const int first = group * G;
    const int rows_in = (gm_e - first) < G ? (gm_e - first) : G;
    const int idx = lin - group * G * gn_e;
    bi = first + idx % rows_in;
    bj = idx / rows_in;
    bi += (bi >= t.sr) ? t.nsr : 0;
    bj += (bj >= t.sc) ? t.nsc : 0;
    return true;
}

}  // namespace fw
