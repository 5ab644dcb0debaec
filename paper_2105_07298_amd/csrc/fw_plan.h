// fw_plan.h -- the launch plan of the pairs-with-lookahead round schedule, as a
// sequence of operations on two streams.  Plain C++: the runtime enqueues the
// plan, and a host-only test replays it to check that every two operations
// touching a common tile (one of them writing it) are ordered by stream order
// or events, and that the plan computes the blocked method's result.
#pragma once
#include "fw_tiles.h"

namespace fw {

enum class PlanKind { p123, p4, record, wait };

struct PlanOp {
    int stream;  // 0: the caller's stream, 1: the auxiliary stream
    PlanKind kind;
    int r;        // round (p123, p4)
    P4Mode mode;  // p4
    int ev;       // event (record, wait)
};

// Events of the plan: ready(q) = aux has finished phases 1-3 (and the cross
// launch) of pair q; main_done(q) = the caller's stream has finished its part of
// pair q; band_done(q) = aux has finished pair q's band tiles.  Each alternates
// between two events, so a wait never sees a record of a later pair.
constexpr int kPlanEvents = 7;
FW_TILE_FN int ev_ready(int q) { return q & 1; }
FW_TILE_FN int ev_main_done(int q) { return 2 + (q & 1); }
FW_TILE_FN int ev_band_done(int q) { return 4 + (q & 1); }
constexpr int kEvStart = 6;

// Rounds go in pairs (r, r + 1), r = 2q, as in the pairs schedule: round r's
// last phase on block r + 1, phases 1-3 of round r + 1, both rounds' last phase
// on every other tile outside blocks r and r + 1, then round r + 1's last phase
// on block r.  Here the auxiliary stream also prepares pair q + 1 while the
// caller's stream runs the bulk of pair q.  It first takes, from the bulk, the
// tiles of the next pair's block rows and columns (pair_band), and from the
// last step the four tiles that join block r to them (crossprev_band).  Then it
// runs phases 1-3 of rounds r + 2 and r + 3 and round r + 2's cross launch.
// The caller's stream keeps the remaining tiles (pair_rest, crossprev_rest).
// Its crossprev_rest waits for pair_band, whose tiles read block r as round
// r's panels; aux's next pair_band waits for crossprev_rest, which finishes
// the tiles that pair_band reads.  R >= 2.
template <typename Emit>
FW_TILE_FN void plan_pairs_lookahead(int R, Emit emit) {
    const int sm = 0, sa = 1;  // the caller's stream, the auxiliary stream
    auto p123 = [&](int st, int r) { emit(PlanOp{st, PlanKind::p123, r, P4Mode::all, -1}); };
    auto p4 = [&](int st, int r, P4Mode m) { emit(PlanOp{st, PlanKind::p4, r, m, -1}); };
    auto rec = [&](int st, int ev) { emit(PlanOp{st, PlanKind::record, -1, P4Mode::all, ev}); };
    auto wait = [&](int st, int ev) { emit(PlanOp{st, PlanKind::wait, -1, P4Mode::all, ev}); };
    rec(sm, kEvStart);
    wait(sa, kEvStart);
    p123(sa, 0);
    if (R > 1) {
        p4(sa, 0, P4Mode::cross);
        p123(sa, 1);
    }
    rec(sa, ev_ready(0));
    for (int q = 0; 2 * q < R; ++q) {
        const int r = 2 * q;
        if (r + 1 == R) {  // a last round on its own
            wait(sm, ev_ready(q));
            p4(sm, r, P4Mode::all);
            break;
        }
        const bool next = r + 2 < R;
        if (next) {
            if (q > 0) wait(sa, ev_main_done(q - 1));
            p4(sa, r, P4Mode::pair_band);
            rec(sa, ev_band_done(q));
        }
        wait(sm, ev_ready(q));
        p4(sm, r, P4Mode::pair_rest);
        if (next) wait(sm, ev_band_done(q));
        p4(sm, r + 1, P4Mode::crossprev_rest);
        rec(sm, ev_main_done(q));
        if (next) {
            p4(sa, r + 1, P4Mode::crossprev_band);
            p123(sa, r + 2);
            if (r + 3 < R) {
                p4(sa, r + 2, P4Mode::cross);
                p123(sa, r + 3);
            }
            rec(sa, ev_ready(q + 1));
        }
    }
}

}  // namespace fw
