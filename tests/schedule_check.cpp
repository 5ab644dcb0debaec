// Host-only expansion of the pairs-with-lookahead plan (csrc/fw_plan.h, the
// code the runtime enqueues) into explicit operations: for R = 1 .. 40 blocks
// (tiles one block square), every phase 1-3 launch and every last-phase launch
// with the tiles its selection visits (csrc/fw_tiles.h), plus the event records
// and waits.  tests/test_schedule.py checks the ordering and runs the result.
//   R <R>
//   P123 <stream> <r>
//   P4 <stream> <r> <fused 0/1> <ntiles> <bi> <bj> ...
//   REC <stream> <event> / WAIT <stream> <event>
//   ERROR <text>
#include <cstdio>
#include <set>
#include <utility>
#include <vector>

#include "../paper_2105_07298_amd/csrc/fw_plan.h"

int main() {
    for (int R = 1; R <= 40; ++R) {
        std::printf("R %d\n", R);
        fw::plan_pairs_lookahead(R, [&](const fw::PlanOp &op) {
            switch (op.kind) {
            case fw::PlanKind::p123: std::printf("P123 %d %d\n", op.stream, op.r); break;
            case fw::PlanKind::record: std::printf("REC %d %d\n", op.stream, op.ev); break;
            case fw::PlanKind::wait: std::printf("WAIT %d %d\n", op.stream, op.ev); break;
            case fw::PlanKind::p4: {
                fw::TileSel sel;
                bool band = false, fuse = false;
                if (!fw::p4_select(R, R, 1, 1, op.r, R, op.mode, sel, band, fuse)) {
                    std::printf("ERROR mode %d rejected for r=%d R=%d\n", (int)op.mode, op.r, R);
                    return;
                }
                std::vector<std::pair<int, int>> tiles;
                std::set<std::pair<int, int>> seen;
                for (int wg = 0; wg < 8 * sel.per_xcd; ++wg) {
                    int bi = -1, bj = -1;
                    const bool ok = band ? fw::select_tile<true>(sel, wg, bi, bj) : fw::select_tile<false>(sel, wg, bi, bj);
                    if (!ok) continue;
                    if (bi < 0 || bi >= R || bj < 0 || bj >= R || !seen.insert({bi, bj}).second)
                        std::printf("ERROR tile (%d, %d) out of range or twice, mode %d r=%d R=%d\n", bi, bj,
                                    (int)op.mode, op.r, R);
                    tiles.push_back({bi, bj});
                }
                std::printf("P4 %d %d %d %zu", op.stream, op.r, fuse ? 1 : 0, tiles.size());
                for (auto &t : tiles) std::printf(" %d %d", t.first, t.second);
                std::printf("\n");
                break;
            }
            }
        });
    }
    return 0;
}
