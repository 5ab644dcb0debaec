// fw_tiles.h -- which output tiles one last-phase launch updates, and which
// workgroup takes which tile.  Plain C++ shared by the kernels (FW_TILE_FN set
// to a host/device inline) and by a host-only test of the selections.
#pragma once
#include <stdint.h>

#ifndef FW_TILE_FN
#define FW_TILE_FN inline
#endif

namespace fw {

// Tiles of one last-phase launch over a gm x gn grid of BM x BN tiles.
//   Normal selection: every tile outside tile rows [sr, sr + nsr) and tile
//   columns [sc, sc + nsc).  A block row (column) of the round that is narrower
//   than a tile is not skipped (nsr or nsc = 0) but masked inside its tile.
//   Cross selection (tiles one block wide, rb tile rows per block): the tiles
//   of block row and block column c = cross, except those in block row /
//   column xs = c - 1 or c + 1.  With xs = c - 1 (round c - 1, lookahead) and a
//   normal selection that skips block rows and columns c - 1 and c, it covers
//   round c - 1; with xs = c + 1 (round c + 1 applied to block c) and the same
//   normal selection, it covers round c + 1.
struct TileSel {
    int gm, gn;
    int sr, nsr, sc, nsc;
    int cross, xs, rb;
    int per_xcd, ntiles;
};

// Launch modes (the values of P4Mode): 0 all, 1 cross (block r + 1, skipping
// r), 2 rest (skipping blocks r and r + 1), 3 cross of block r skipping r + 1.
// rb / cb: tile rows / columns per block (0 when a tile is wider than the
// block).  Fills sel for round r of nblocks; false if the mode does not apply.
FW_TILE_FN bool make_tile_sel(int gm, int gn, int rb, int cb, int r, int nblocks, int mode, TileSel &sel) {
    sel.gm = gm;
    sel.gn = gn;
    sel.sr = gm;
    sel.nsr = 0;
    sel.sc = gn;
    sel.nsc = 0;
    sel.cross = -1;
    sel.xs = -1;
    sel.rb = rb;
    int64_t ntiles;
    if (mode == 1 || mode == 3) {
        if (rb == 0 || cb != 1 || r + 1 >= nblocks) return false;
        sel.cross = mode == 1 ? r + 1 : r;
        sel.xs = mode == 1 ? r : r + 1;
        sel.nsr = rb;
        sel.nsc = 1;
        ntiles = (int64_t)rb * (gn - 1) + (gm - 2 * rb);
    } else {
        const int w = mode == 2 ? 2 : 1;
        if (w == 2 && (rb == 0 || cb != 1 || r + 1 >= nblocks)) return false;
        if (rb) {
            sel.sr = r * rb;
            sel.nsr = w * rb;
        }
        if (cb) {
            sel.sc = r * cb;
            sel.nsc = w * cb;
        }
        ntiles = (int64_t)(gm - sel.nsr) * (gn - sel.nsc);
    }
    if (ntiles < 0 || ntiles > (int64_t)1 << 30) return false;
    sel.ntiles = (int)ntiles;
    sel.per_xcd = (int)((ntiles + 7) / 8);
    return true;
}

// Tile (bi, bj) of workgroup wg of a launch with 8 * per_xcd workgroups; false
// for the workgroups that pad the grid.  Workgroups go round-robin over the 8
// XCDs and each XCD takes a contiguous range of the tile sequence, walked in
// groups of 8 tile rows so that the workgroups resident on one XCD share
// panels in its L2.
template <bool CROSS>
FW_TILE_FN bool select_tile(const TileSel &t, int wg, int &bi, int &bj) {
    const int lin = (wg % 8) * t.per_xcd + wg / 8;
    if (lin >= t.ntiles) return false;
    if (CROSS) {
        const int c = t.cross, xs = t.xs, lo = c < xs ? c : xs, nrow = t.rb * (t.gn - 1);
        if (lin < nrow) {
            bi = c * t.rb + lin % t.rb;
            const int jj = lin / t.rb;
            bj = jj < xs ? jj : jj + 1;
        } else {
            const int ii = lin - nrow;
            bi = ii < lo * t.rb ? ii : ii + 2 * t.rb;  // blocks c and xs are adjacent
            bj = c;
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
