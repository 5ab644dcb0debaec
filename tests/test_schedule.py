"""The pairs-with-lookahead round schedule (csrc/fw_plan.h, the plan the runtime
enqueues on two streams), checked on the host.

tests/schedule_check.cpp expands the plan for 1 to 40 blocks into its launches,
each last-phase launch with the exact tiles its selection visits.  Then:
  * every two operations that touch a common tile, one of them writing it, are
    ordered by stream order and event record/wait edges as in the enqueue
    order, so any execution the two streams allow equals the sequential one;
  * executed in enqueue order on the NumPy model of the library's path-mode
    method (deferred last-phase labels, one resolution pass), the plan gives the
    classic loop's D and canonical P, ties included;
  * for every block count the launches cover each round's last phase exactly:
    every tile outside block r gets round r exactly once.
"""
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads
from conftest import ROOT
from test_blocked_emulation import blocked_model_deferred


@pytest.fixture(scope="module")
def plans(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sched") / "schedule_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror", "-o", exe,
                    os.path.join(ROOT, "tests", "schedule_check.cpp")], check=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120, check=True).stdout
    assert "ERROR" not in out, [l for l in out.splitlines() if l.startswith("ERROR")][:5]
    plans, cur = {}, None
    for line in out.splitlines():
        f = line.split()
        if f[0] == "R":
            cur = plans.setdefault(int(f[1]), [])
        elif f[0] == "P123":
            cur.append(("p123", int(f[1]), int(f[2])))
        elif f[0] == "P4":
            st, r, fused, nt = int(f[1]), int(f[2]), int(f[3]), int(f[4])
            xs = list(map(int, f[5:]))
            assert len(xs) == 2 * nt
            cur.append(("p4", st, r, bool(fused), [(xs[2 * k], xs[2 * k + 1]) for k in range(nt)]))
        elif f[0] in ("REC", "WAIT"):
            cur.append((f[0].lower(), int(f[1]), int(f[2])))
    return plans


def access(op, R):
    """(reads, writes) as sets of (block row, block column)."""
    if op[0] == "p123":
        r = op[2]
        w = {(r, j) for j in range(R)} | {(i, r) for i in range(R)}
        return w, w
    _, _, r, fused, tiles = op
    w = set(tiles)
    rd = set(w)
    for rr in ((r, r + 1) if fused else (r,)):
        rd |= {(i, rr) for i, _ in tiles} | {(rr, j) for _, j in tiles}
    return rd, w


def test_every_conflict_is_ordered(plans):
    for R, ops in plans.items():
        before = {0: set(), 1: set()}
        events, preds, acc = {}, {}, {}
        work = []
        for k, op in enumerate(ops):
            if op[0] == "rec":
                events[op[2]] = set(before[op[1]])
            elif op[0] == "wait":
                assert op[2] in events, f"R={R}: wait on event {op[2]} before any record"
                before[op[1]] |= events[op[2]]
            else:
                st = op[1]
                preds[k] = set(before[st])
                before[st] |= {k}
                acc[k] = access(op, R)
                work.append(k)
        # the caller's stream ends after every operation of the auxiliary stream
        assert set(work) <= before[0] | ({max(work)} if work else set()), f"R={R}: aux work not joined"
        for x in range(len(work)):
            a = work[x]
            ra, wa = acc[a]
            for b in work[x + 1:]:
                rb, wb = acc[b]
                if wa & (rb | wb) or wb & ra:
                    assert a in preds[b], f"R={R}: {ops[a][:3]} and {ops[b][:3]} conflict but are not ordered"


def test_each_round_covers_its_last_phase_once(plans):
    for R, ops in plans.items():
        got = {}
        for op in ops:
            if op[0] != "p4":
                continue
            _, _, r, fused, tiles = op
            for rr in ((r, r + 1) if fused else (r,)):
                for t in tiles:
                    got.setdefault(rr, []).append(t)
        for r in range(R):
            want = sorted((i, j) for i in range(R) for j in range(R) if i != r and j != r)
            assert sorted(got.get(r, [])) == want, f"R={R}: round {r} covers the wrong tiles"
        p123 = [op[2] for op in ops if op[0] == "p123"]
        assert p123 == list(range(R)), f"R={R}: phases 1-3 out of order"


@pytest.mark.parametrize("TB", [1, 2, 3])
@pytest.mark.parametrize("seed", range(5))
def test_plan_equals_classic(plans, TB, seed):
    rng = np.random.default_rng(seed + 310)
    n = int(rng.integers(4, 40))
    W = workloads.int_graph(n=n, p=float(rng.uniform(0.05, 0.6)), wmax=int(rng.integers(1, 4)), seed=seed + 410)
    R = -(-n // TB)
    ops = [("p123", op[2]) if op[0] == "p123" else ("p4", op[2], op[3], op[4])
           for op in plans[R] if op[0] in ("p123", "p4")]
    D, P = oracle.fw(W)
    Dm, Pm = blocked_model_deferred(W.astype(np.float64), TB, schedule="ops", ops=ops)
    np.testing.assert_array_equal(Dm, D)
    np.testing.assert_array_equal(Pm, P)


def test_swapping_the_band_wait_breaks_ordering(plans):
    """The check is not vacuous: without the wait for the band tiles before the
    caller's crossprev_rest, the crossprev_rest writes of block r race with the
    band launch's reads of them."""
    R = 8
    ops = [op for op in plans[R]]
    # drop the caller's waits on band_done events (4 and 5)
    ops = [op for op in ops if not (op[0] == "wait" and op[1] == 0 and op[2] in (4, 5))]
    before = {0: set(), 1: set()}
    events, preds, acc, work = {}, {}, {}, []
    for k, op in enumerate(ops):
        if op[0] == "rec":
            events[op[2]] = set(before[op[1]])
        elif op[0] == "wait":
            before[op[1]] |= events[op[2]]
        else:
            preds[k] = set(before[op[1]])
            before[op[1]] |= {k}
            acc[k] = access(op, R)
            work.append(k)
    unordered = 0
    for x in range(len(work)):
        a = work[x]
        ra, wa = acc[a]
        for b in work[x + 1:]:
            rb, wb = acc[b]
            if (wa & (rb | wb) or wb & ra) and a not in preds[b]:
                unordered += 1
    assert unordered > 0
