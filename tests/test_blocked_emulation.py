"""A slow NumPy model of the blocked method the HIP kernels implement (test code,
not the oracle), checked against the oracle.

Model (paper Sect. 2.2, "Blocked FW Algorithm"): D is cut into TB x TB blocks;
round r takes the k-block K = [r*TB, (r+1)*TB) through
  phase 1  the diagonal block, sequential k-steps (classic loop inside K),
  phase 2  the row panel D[K, J]   <- lexmin(D[K, J], D*[K, K] (x) D_old[K, J]),
  phase 3  the column panel D[I, K] <- lexmin(D[I, K], D_old[I, K] (x) D*[K, K]),
  phase 4  every other block D[I, J] <- lexmin(D[I, J], D[I, K] (x) D[K, J]),
where (x) is the min-plus product and every candidate through k carries the
label (length, max(P[i][k], k, P[k][j])).  Phase 4 is taken in two passes
(minimum length first, then the smallest label among the k that reach it),
exactly as the GPU kernel does.  For integer weights the result must equal the
classic loop bit for bit, whatever TB and the padding are.
"""
import numpy as np
import pytest

import oracle
import workloads


def lex_update(d, p, s, m):
    better = (s < d) | ((s == d) & (m < p))
    return np.where(better, s, d), np.where(better, m, p)


def product_lex(DA, PA, DB, PB, k_ids, Dc, Pc):
    """lexmin over k of (DA[:,k] + DB[k,:], max(PA[:,k], k, PB[k,:])) folded into (Dc, Pc)."""
    for t, k in enumerate(k_ids):
        s = DA[:, t:t + 1] + DB[t:t + 1, :]
        m = np.maximum(np.maximum(PA[:, t:t + 1], k), PB[t:t + 1, :])
        Dc, Pc = lex_update(Dc, Pc, s, m)
    return Dc, Pc


def product_two_pass(DA, PA, DB, PB, k_ids, Dc, Pc):
    S = np.full(Dc.shape, np.inf)
    for t in range(len(k_ids)):
        S = np.minimum(S, DA[:, t:t + 1] + DB[t:t + 1, :])
    marked = (S <= Dc) & np.isfinite(S)
    BIG = np.iinfo(np.int64).max
    M = np.full(Dc.shape, BIG, dtype=np.int64)
    for t, k in enumerate(k_ids):
        s = DA[:, t:t + 1] + DB[t:t + 1, :]
        m = np.maximum(np.maximum(PA[:, t:t + 1], k), PB[t:t + 1, :])
        M = np.where(marked & (s == S), np.minimum(M, m), M)
    improve = marked & (S < Dc)
    tie = marked & (S == Dc)
    Pn = np.where(improve, M, np.where(tie, np.minimum(Pc, M), Pc))
    return np.where(improve, S, Dc), Pn


def product_sentinel(DA, PA, DB, PB, k_ids, Dc, Pc, sentinel=-1):
    """The batched kernel's last phase: the tile starts with its old lengths and the
    label `sentinel` (-1, "no interior vertex": below every candidate's label, which
    is at least k >= the round's first vertex), takes the lexicographic product, and
    writes back only the entries whose label left the sentinel (those that
    decreased); the others keep their old length and label."""
    Dn, Pn = product_lex(DA, PA, DB, PB, k_ids, Dc, np.full(Pc.shape, sentinel, dtype=np.int64))
    changed = Pn != sentinel
    return np.where(changed, Dn, Dc), np.where(changed, Pn, Pc)


def blocked_model(W, TB, two_pass=True, phase4=None):
    n = W.shape[0]
    npad = -(-n // TB) * TB
    D = np.full((npad, npad), np.inf)
    np.fill_diagonal(D, 0.0)
    D[:n, :n] = W
    P = np.full((npad, npad), -1, dtype=np.int64)
    R = npad // TB
    for r in range(R):
        K = np.arange(r * TB, (r + 1) * TB)
        ks = slice(r * TB, (r + 1) * TB)
        # phase 1: sequential closure of the diagonal block
        for k in K:
            s = D[ks, k:k + 1] + D[k:k + 1, ks]
            m = np.maximum(np.maximum(P[ks, k:k + 1], k), P[k:k + 1, ks])
            D[ks, ks], P[ks, ks] = lex_update(D[ks, ks], P[ks, ks], s, m)
        Dkk, Pkk = D[ks, ks].copy(), P[ks, ks].copy()
        others = [b for b in range(R) if b != r]
        # phases 2 and 3 read the old panels and the closed diagonal block
        for b in others:
            js = slice(b * TB, (b + 1) * TB)
            D[ks, js], P[ks, js] = product_lex(Dkk, Pkk, D[ks, js].copy(), P[ks, js].copy(), K,
                                               D[ks, js], P[ks, js])
            D[js, ks], P[js, ks] = product_lex(D[js, ks].copy(), P[js, ks].copy(), Dkk, Pkk, K,
                                               D[js, ks], P[js, ks])
        # phase 4 reads the final panels of this round
        for bi in others:
            for bj in others:
                is_, js = slice(bi * TB, (bi + 1) * TB), slice(bj * TB, (bj + 1) * TB)
                f = phase4 or (product_two_pass if two_pass else product_lex)
                D[is_, js], P[is_, js] = f(D[is_, ks], P[is_, ks], D[ks, js], P[ks, js], K,
                                           D[is_, js], P[is_, js])
    return D[:n, :n], P[:n, :n].astype(np.int32)


@pytest.mark.parametrize("TB", [1, 2, 3, 4, 8, 16])
@pytest.mark.parametrize("seed", range(4))
def test_model_equals_classic_tie_heavy(TB, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 40))
    W = workloads.int_graph(n=n, p=float(rng.uniform(0.05, 0.6)), wmax=int(rng.integers(1, 4)), seed=seed + 70)
    D, P = oracle.fw(W)
    Dm, Pm = blocked_model(W.astype(np.float64), TB)
    np.testing.assert_array_equal(Dm, D)
    np.testing.assert_array_equal(Pm, P)


@pytest.mark.parametrize("two_pass", [True, False])
def test_model_c1_like(two_pass):
    W = workloads.int_graph(n=96, p=0.5, wmax=1000, seed=1)
    D, P = oracle.fw(W)
    Dm, Pm = blocked_model(W.astype(np.float64), 16, two_pass=two_pass)
    np.testing.assert_array_equal(Dm, D)
    np.testing.assert_array_equal(Pm, P)


@pytest.mark.parametrize("TB", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("seed", range(4))
def test_sentinel_last_phase_equals_classic(TB, seed):
    """The batched kernel's last phase (old labels not read, only decreased entries
    written) gives the classic loop's D and P on tie-heavy graphs."""
    rng = np.random.default_rng(seed + 20)
    n = int(rng.integers(5, 40))
    W = workloads.int_graph(n=n, p=float(rng.uniform(0.05, 0.6)), wmax=int(rng.integers(1, 4)), seed=seed + 90)
    D, P = oracle.fw(W)
    Dm, Pm = blocked_model(W.astype(np.float64), TB, phase4=product_sentinel)
    np.testing.assert_array_equal(Dm, D)
    np.testing.assert_array_equal(Pm, P)


def test_sentinel_must_sort_below_candidates():
    """Control: a sentinel above every label lets a tie with the old length replace
    the old label, and P then differs from the classic loop's."""
    W = workloads.int_graph(n=40, p=0.3, wmax=2, seed=3).astype(np.float64)
    D, P = oracle.fw(W)
    high = lambda *a: product_sentinel(*a, sentinel=1 << 40)
    Dm, Pm = blocked_model(W, 4, phase4=high)
    np.testing.assert_array_equal(Dm, D)
    assert not np.array_equal(Pm, P)


def test_naive_p_rule_differs():
    """Storing k on strict improvement (no lexicographic label) is tile dependent: the
    model with that rule disagrees with the classic P on a tie-heavy graph."""
    W = workloads.int_graph(n=40, p=0.3, wmax=2, seed=3).astype(np.float64)
    D, P = oracle.fw(W)

    def naive_update(d, p, s, m):
        better = s < d
        return np.where(better, s, d), np.where(better, m, p)

    global lex_update
    saved = lex_update
    try:
        lex_update = naive_update
        Dm, Pm = blocked_model(W, 4, two_pass=False)
    finally:
        lex_update = saved
    np.testing.assert_array_equal(Dm, D)
    assert not np.array_equal(Pm, P)


def test_model_real_weights_tolerance():
    W = workloads.unit_complete(64, dtype=np.float64, seed=2)
    D, _ = oracle.fw(W)
    Dm, Pm = blocked_model(W, 8)
    np.testing.assert_allclose(Dm, D, rtol=1e-14)
    oracle.check_invariants(W, Dm, Pm, exact=False, rtol=1e-12)


def blocked_model_deferred(W, TB, schedule="serial", ops=None):
    """The GPU's path-mode schedule: phases 1-3 apply the lexicographic rule to P
    (which holds an older label while an entry is pending) and clear the entry's
    mark L when they change it; the last phase only marks strict improvements
    (L = r + 1); one pass after the last round resolves every pending label from
    the final D, in place, skipping the k whose entries are pending from a later
    round.

    schedule "pairs" runs rounds two at a time as the library's pairs schedule
    does: round r's last phase on block row / column r + 1, phases 1-3 of round
    r + 1, then both rounds' last phase in one pass over the tiles outside blocks
    r and r + 1 (round r's minimum kept apart, the mark naming the last round in
    which the entry decreased), and only then round r + 1's last phase on block
    row / column r.

    schedule "ops" runs an explicit operation list instead, in order: ("p123", r),
    ("p4", r, fused, tiles) with tiles a list of (block row, block column)."""
    n = W.shape[0]
    npad = -(-n // TB) * TB
    D = np.full((npad, npad), np.inf)
    np.fill_diagonal(D, 0.0)
    D[:n, :n] = W
    P = np.full((npad, npad), -1, dtype=np.int64)
    L = np.zeros((npad, npad), dtype=np.int64)
    R = npad // TB
    blk = lambda b: slice(b * TB, (b + 1) * TB)

    def phases123(r):
        K = np.arange(r * TB, (r + 1) * TB)
        ks = blk(r)
        D0, P0 = D[ks, ks].copy(), P[ks, ks].copy()
        for k in K:
            s = D[ks, k:k + 1] + D[k:k + 1, ks]
            m = np.maximum(np.maximum(P[ks, k:k + 1], k), P[k:k + 1, ks])
            D[ks, ks], P[ks, ks] = lex_update(D[ks, ks], P[ks, ks], s, m)
        L[ks, ks] = np.where((D[ks, ks] != D0) | (P[ks, ks] != P0), 0, L[ks, ks])
        Dkk, Pkk = D[ks, ks].copy(), P[ks, ks].copy()
        for b in [b for b in range(R) if b != r]:
            js = blk(b)
            for (rs, cs, A, PA, B, PB) in ((ks, js, Dkk, Pkk, None, None), (js, ks, None, None, Dkk, Pkk)):
                Dold, Pold = D[rs, cs].copy(), P[rs, cs].copy()
                if A is not None:
                    Dn, Pn = product_lex(A, PA, Dold, Pold, K, Dold, Pold)
                else:
                    Dn, Pn = product_lex(Dold, Pold, B, PB, K, Dold, Pold)
                D[rs, cs], P[rs, cs] = Dn, Pn
                L[rs, cs] = np.where((Dn != Dold) | (Pn != Pold), 0, L[rs, cs])

    def block_min(r, bi, bj):
        S = np.full((TB, TB), np.inf)
        for t in range(TB):
            S = np.minimum(S, D[blk(bi), r * TB + t:r * TB + t + 1] + D[r * TB + t:r * TB + t + 1, blk(bj)])
        return S

    def last_phase(r, tiles):
        for bi, bj in tiles:
            S = block_min(r, bi, bj)
            imp = S < D[blk(bi), blk(bj)]
            D[blk(bi), blk(bj)] = np.where(imp, S, D[blk(bi), blk(bj)])
            L[blk(bi), blk(bj)] = np.where(imp, r + 1, L[blk(bi), blk(bj)])

    def fused_pair(r, tiles):
        for bi, bj in tiles:
            S0 = block_min(r, bi, bj)
            S1 = block_min(r + 1, bi, bj)
            C = D[blk(bi), blk(bj)]
            lt0 = S0 < C
            C1 = np.where(lt0, S0, C)
            lt1 = S1 < C1
            D[blk(bi), blk(bj)] = np.where(lt1, S1, C1)
            L[blk(bi), blk(bj)] = np.where(lt1, r + 2, np.where(lt0, r + 1, L[blk(bi), blk(bj)]))

    def outside(*bs):
        return [(bi, bj) for bi in range(R) for bj in range(R) if bi not in bs and bj not in bs]

    if schedule == "ops":
        for op in ops:
            if op[0] == "p123":
                phases123(op[1])
            elif op[2]:
                fused_pair(op[1], op[3])
            else:
                last_phase(op[1], op[3])
    elif schedule == "serial":
        for r in range(R):
            phases123(r)
            last_phase(r, outside(r))
    else:
        for r in range(0, R, 2):
            phases123(r)
            if r + 1 == R:
                last_phase(r, outside(r))
                break
            last_phase(r, [t for t in outside(r) if t[0] == r + 1 or t[1] == r + 1])
            phases123(r + 1)
            fused_pair(r, outside(r, r + 1))
            last_phase(r + 1, [t for t in outside(r + 1) if t[0] == r or t[1] == r])
    # resolution, in place, entries in an arbitrary order
    order = np.argwhere(L > 0)
    np.random.default_rng(0).shuffle(order)
    for i, j in order:
        lv = L[i, j]
        ks = np.arange((lv - 1) * TB, lv * TB)
        sums = D[i, ks] + D[ks, j]
        labels = [max(P[i, k], k, P[k, j]) for k in ks[sums == D[i, j]]
                  if L[i, k] <= lv and L[k, j] <= lv]
        assert labels
        P[i, j] = min(labels)
    return D[:n, :n], P[:n, :n].astype(np.int32)


@pytest.mark.parametrize("TB", [1, 2, 3, 4, 8, 16])
@pytest.mark.parametrize("seed", range(4))
def test_deferred_labels_equal_classic(TB, seed):
    rng = np.random.default_rng(seed + 40)
    n = int(rng.integers(5, 48))
    W = workloads.int_graph(n=n, p=float(rng.uniform(0.05, 0.6)), wmax=int(rng.integers(1, 4)), seed=seed + 170)
    D, P = oracle.fw(W)
    Dm, Pm = blocked_model_deferred(W.astype(np.float64), TB)
    np.testing.assert_array_equal(Dm, D)
    np.testing.assert_array_equal(Pm, P)


def test_deferred_labels_c1_like():
    W = workloads.int_graph(n=128, p=0.5, wmax=1000, seed=1)
    D, P = oracle.fw(W)
    Dm, Pm = blocked_model_deferred(W.astype(np.float64), 16)
    np.testing.assert_array_equal(Dm, D)
    np.testing.assert_array_equal(Pm, P)


@pytest.mark.parametrize("TB", [1, 2, 3, 4, 8])
@pytest.mark.parametrize("seed", range(6))
def test_pairs_schedule_equals_classic(TB, seed):
    """The pairs schedule (two rounds' last phase fused on the tiles outside both
    blocks) gives the classic loop's D and canonical P, ties included, for odd and
    even round counts."""
    rng = np.random.default_rng(seed + 90)
    n = int(rng.integers(5, 48))
    W = workloads.int_graph(n=n, p=float(rng.uniform(0.05, 0.6)), wmax=int(rng.integers(1, 4)), seed=seed + 270)
    D, P = oracle.fw(W)
    Dm, Pm = blocked_model_deferred(W.astype(np.float64), TB, schedule="pairs")
    np.testing.assert_array_equal(Dm, D)
    np.testing.assert_array_equal(Pm, P)
