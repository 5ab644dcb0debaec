"""Pins of the checker itself: oracle.check_invariants must reject a (D, P) that
is wrong in any single entry, in both its exact (integer) and real-weight modes,
at the tolerances and sample sizes the GPU tests use.

What a correct (D, P) is comes from Sect. 2.2 (Algorithm 1) with readings R1-R2:
D[i][j] the length of a shortest path, P[i][j] an intermediate vertex of one
(the largest interior vertex of the canonical path), -1 for the direct edge or no
path.  Each corruption below breaks that in one entry; the checker is given the
oracle's own (D, P) with that one change and must raise.  The same corruptions
are run against mutated copies of the checker in test_oracle_mutants.py, which
must let at least one of them through."""
import numpy as np
import pytest

import oracle
import workloads

# (rtol, nsample) pairs the GPU tests call the checker with; nsample 0 shows the
# all-pairs checks alone catch every corruption.
REAL_SETTINGS = [(1e-5, 3000), (1e-5, 1000), (1e-6, 200), (1e-12, 0), (1e-5, 0)]


def int_case():
    """Integer weights in [1, 9], density 0.08: multi-hop shortest paths, ties and
    unreachable pairs (vertex 0 has no in-edges)."""
    W = workloads.int_graph(n=60, p=0.08, wmax=9, seed=21)
    W[1:, 0] = np.inf
    D, P = oracle.fw(W)
    assert (P >= 0).sum() > 200 and np.isinf(D).any()
    return W, D, P


def real_case():
    """Real weights in (0, 1), density 0.1, with unreachable pairs."""
    W = workloads.graph(22, 60, 0.1, workloads.W_UNIT_OPEN, 0, np.float64)
    W[1:, 0] = np.inf
    D, P = oracle.fw(W, exact=False)
    assert (P >= 0).sum() > 200 and np.isinf(D).any()
    return W, D, P


def _pick(mask, seed=0):
    I, J = np.nonzero(mask)
    assert I.size, "no entry to corrupt"
    q = np.random.default_rng(seed).integers(I.size)
    return int(I[q]), int(J[q])


def corrupt(kind, W, D, P):
    """A copy of (D, P) with one entry made wrong in the way `kind` names."""
    D, P = D.copy(), P.copy()
    n = W.shape[0]
    off = ~np.eye(n, dtype=bool)
    multi = (P >= 0)
    if kind == "p_is_source":            # P[i][j] <- i
        i, j = _pick(multi)
        P[i, j] = i
    elif kind == "p_is_target":          # P[i][j] <- j
        i, j = _pick(multi)
        P[i, j] = j
    elif kind == "p_off_path":           # P[i][j] <- a vertex on no shortest i->j path
        for i, j in zip(*np.nonzero(multi)):
            via = D[i, :] + D[:, j]
            cand = np.nonzero(np.isfinite(via) & (via > D[i, j] * 1.01 + 1e-9))[0]
            cand = cand[(cand != i) & (cand != j)]
            if cand.size:
                P[i, j] = int(cand[0])
                return D, P
        raise AssertionError("no off-path vertex found")
    elif kind == "label_unreachable":    # a label on an unreachable pair
        i, j = _pick(np.isinf(D) & off)
        # a k that the other checks would not object to: i reaches k, and (i, k)
        # is labelled below k
        ks = [k for k in range(n) if k not in (i, j) and np.isfinite(D[i, k]) and P[i, k] < k]
        P[i, j] = ks[0] if ks else next(k for k in range(n) if k not in (i, j))
    elif kind == "direct_not_shortest":  # P[i][j] <- -1 where a multi-hop path is strictly shorter
        i, j = _pick(multi & (W > D))
        P[i, j] = -1
    elif kind == "d_raised":             # D[i][j] raised above the two-hop sum through P[i][j], still <= W
        i, j = _pick(multi & (W >= D * 1.2 + 1))
        D[i, j] = D[i, j] + 1.0 if oracle.is_integer_valued(W) else D[i, j] * 1.1
    elif kind == "d_lowered":            # D[i][j] below every path
        i, j = _pick(multi)
        D[i, j] = D[i, j] - 1.0 if oracle.is_integer_valued(W) else D[i, j] * 0.9
    elif kind == "cycle":                # labels that make the reconstruction loop
        i, j = _pick(multi)
        k = int(P[i, j])
        P[i, k] = j                      # path(i, j) -> path(i, k) -> path(i, j) ...
    elif kind == "wrong_tie_label":      # another vertex of a shortest path than the canonical one
        for i, j in zip(*np.nonzero(multi)):
            via = D[i, :] + D[:, j]
            cand = np.nonzero(via == D[i, j])[0]
            cand = cand[(cand != i) & (cand != j) & (cand != P[i, j])]
            if cand.size:
                P[i, j] = int(cand[0])
                return D, P
        raise AssertionError("no tie found")
    else:
        raise ValueError(kind)
    return D, P


KINDS = ["p_is_source", "p_is_target", "p_off_path", "label_unreachable", "direct_not_shortest",
         "d_raised", "d_lowered", "cycle"]


def escaped(check, cases=None):
    """Corruptions (kind, mode) that `check` (a check_invariants) accepts; [] when it
    rejects all of them.  Also fails when it rejects a correct (D, P)."""
    out = []
    int_c, real_c = cases or (int_case(), real_case())

    def accepts(W, D, P, exact, rtol, nsample):
        try:
            check(W, D, P, exact=exact, rtol=rtol, nsample=nsample)
            return True
        except AssertionError:
            return False

    for W, D, P in (int_c, real_c):
        assert accepts(W, D, P, False, 1e-5, 0), "a correct (D, P) was rejected"
    W, D, P = int_c
    assert accepts(W, D, P, True, 0.0, 0), "a correct (D, P) was rejected"
    for kind in KINDS + ["wrong_tie_label"]:
        Dc, Pc = corrupt(kind, W, D, P)
        for nsample in (2000, 0):
            if accepts(W, Dc, Pc, True, 0.0, nsample):
                out.append((kind, "exact", nsample))
    for W, D, P in (int_c, real_c):
        for kind in KINDS:
            Dc, Pc = corrupt(kind, W, D, P)
            for rtol, nsample in REAL_SETTINGS:
                if accepts(W, Dc, Pc, False, rtol, nsample):
                    out.append((kind, "real", rtol, nsample))
    return out


def test_correct_results_pass():
    W, D, P = int_case()
    oracle.check_invariants(W, D, P, exact=True)
    oracle.check_invariants(W, D, P, exact=False, rtol=1e-12)
    W, D, P = real_case()
    oracle.check_invariants(W, D, P, exact=False, rtol=1e-12)


def test_float32_rounded_result_passes_real_mode():
    """A float32 computation of the same graph (D rounded along its own paths) is
    accepted at the float32 tolerance: the checker's tolerances are not too tight
    for what the GPU tests feed it."""
    W, D, P = real_case()
    W32 = W.astype(np.float32)
    D32 = D.astype(np.float32).astype(np.float64)
    oracle.check_invariants(W32, D32, P, exact=False, rtol=1e-5, nsample=500)


@pytest.mark.parametrize("kind", KINDS + ["wrong_tie_label"])
@pytest.mark.parametrize("nsample", [2000, 0])
def test_exact_mode_rejects(kind, nsample):
    W, D, P = int_case()
    Dc, Pc = corrupt(kind, W, D, P)
    with pytest.raises(AssertionError):
        oracle.check_invariants(W, Dc, Pc, exact=True, nsample=nsample)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("rtol,nsample", REAL_SETTINGS)
@pytest.mark.parametrize("case", ["int", "real"])
def test_real_mode_rejects(kind, rtol, nsample, case):
    W, D, P = int_case() if case == "int" else real_case()
    Dc, Pc = corrupt(kind, W, D, P)
    with pytest.raises(AssertionError):
        oracle.check_invariants(W, Dc, Pc, exact=False, rtol=rtol, nsample=nsample)


def test_single_wrong_label_in_large_matrix_is_found():
    """One wrong label among the 1024^2 pairs of a complete graph: a sampled check would
    almost surely miss it; the all-pairs pass must not."""
    W = workloads.graph(23, 1024, 1.0, workloads.W_UNIT_OPEN, 0, np.float32).astype(np.float64)
    D, P = oracle.fw(W, exact=False)
    Dc, Pc = corrupt("p_off_path", W, D, P)
    with pytest.raises(AssertionError):
        oracle.check_invariants(W, Dc, Pc, exact=False, rtol=1e-5, nsample=1000)


def test_path_sums_on_hand_built_encodings():
    """path_sums on a 4-vertex chain 0->1->2->3 (weights 1, 2, 4): hand-derived sums
    and edge counts, and -1 for a cyclic and an endpoint encoding."""
    inf = np.inf
    W = np.array([[0, 1, inf, inf], [inf, 0, 2, inf], [inf, inf, 0, 4], [inf, inf, inf, 0]])
    P = -np.ones((4, 4), dtype=np.int32)
    P[0, 2], P[1, 3], P[0, 3] = 1, 2, 2
    S, H = oracle.path_sums(W, P)
    assert S[0, 3] == 7 and H[0, 3] == 3
    assert S[0, 2] == 3 and H[0, 2] == 2
    assert S[1, 3] == 6 and H[1, 3] == 2
    assert np.isinf(S[3, 0]) and H[3, 0] == 1   # the missing direct edge
    Pc = P.copy()
    Pc[0, 2] = 3                                 # 0->3 via 2, 0->2 via 3: a cycle
    assert oracle.path_sums(W, Pc)[1][0, 3] == -1
    Pc = P.copy()
    Pc[0, 3] = 0                                 # endpoint label
    assert oracle.path_sums(W, Pc)[1][0, 3] == -1


def test_triangle_violations_counts():
    D = np.array([[0.0, 1.0, 5.0], [np.inf, 0.0, 1.0], [np.inf, np.inf, 0.0]])
    assert oracle.triangle_violations(D, [0, 1, 2]) == 1   # D[0][2] = 5 > 1 + 1 through k = 1
    D[0, 2] = 2.0
    assert oracle.triangle_violations(D, [0, 1, 2]) == 0


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("case", ["int", "real"])
def test_rows_mode_rejects(kind, case):
    """Restricted to a few source rows (as at n >= 8192, where the GPU tests check 64
    sampled rows), a corruption in one of those rows is still caught."""
    W, D, P = int_case() if case == "int" else real_case()
    Dc, Pc = corrupt(kind, W, D, P)
    bad = np.unique(np.nonzero((Dc != D) | (Pc != P))[0])
    assert bad.size == 1
    rows = np.array(sorted({int(bad[0]), 3, 17, 40}))
    oracle.check_invariants(W, D, P, exact=False, rtol=1e-5, nsample=0, rows=rows)
    with pytest.raises(AssertionError):
        oracle.check_invariants(W, Dc, Pc, exact=False, rtol=1e-5, nsample=0, rows=rows)
