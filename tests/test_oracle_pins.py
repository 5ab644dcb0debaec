"""Pins for the CPU oracle: each check fixes it against something other than itself.

brute force (the definition, n <= 8), closed forms, a hand-worked golden example,
scipy/networkx library routines, an independent algorithm (Dijkstra), and
invariants.  All CPU-only.
"""
import numpy as np
import pytest

import oracle
import workloads
from conftest import load_golden


def rand_graph(rng, n, p, wmax=None):
    W = np.full((n, n), np.inf)
    mask = rng.random((n, n)) < p
    if wmax is None:
        w = rng.random((n, n)) + 0.01
    else:
        w = rng.integers(1, wmax + 1, size=(n, n)).astype(np.float64)
    W[mask] = w[mask]
    np.fill_diagonal(W, 0.0)
    return W


# ---------------------------------------------------------------- brute force

@pytest.mark.parametrize("seed", range(40))
def test_brute_force_integer_ties(seed):
    """Tie-heavy integer weights: D and the canonical P equal exhaustive search exactly."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 9))
    W = rand_graph(rng, n, p=float(rng.uniform(0.2, 0.9)), wmax=int(rng.integers(1, 4)))
    D, P = oracle.fw(W)
    Db, Pb = oracle.brute_force(W)
    np.testing.assert_array_equal(D, Db)
    np.testing.assert_array_equal(P, Pb)


@pytest.mark.parametrize("seed", range(15))
def test_brute_force_real(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 9))
    W = rand_graph(rng, n, p=0.6)
    D, P = oracle.fw(W)
    Db, Pb = oracle.brute_force(W)
    fin = np.isfinite(Db)
    np.testing.assert_array_equal(np.isfinite(D), fin)
    np.testing.assert_allclose(D[fin], Db[fin], rtol=1e-14)
    np.testing.assert_array_equal(P, Pb)  # distinct random doubles: unique shortest paths


def test_golden_hand_example():
    g = load_golden("tie_example_5.txt")
    D, P = oracle.fw(g["W"])
    np.testing.assert_array_equal(D, g["D"])
    np.testing.assert_array_equal(P, g["P"].astype(np.int32))
    Db, Pb = oracle.brute_force(g["W"])
    np.testing.assert_array_equal(Db, g["D"])
    np.testing.assert_array_equal(Pb, g["P"].astype(np.int32))


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [2, 5, 64, 300])
def test_directed_path_graph(n):
    """0->1->...->n-1: D[i][j] = sum of w[i..j-1] for i < j, inf for i > j; P[i][j] = j-1 when j >= i+2."""
    rng = np.random.default_rng(n)
    w = rng.integers(1, 50, size=n - 1).astype(np.float64)
    W = np.full((n, n), np.inf)
    np.fill_diagonal(W, 0)
    W[np.arange(n - 1), np.arange(1, n)] = w
    D, P = oracle.fw(W)
    pre = np.concatenate([[0.0], np.cumsum(w)])
    for i in range(n):
        for j in range(n):
            if i <= j:
                assert D[i, j] == pre[j] - pre[i]
                assert P[i, j] == (j - 1 if j >= i + 2 else -1)
            else:
                assert D[i, j] == np.inf and P[i, j] == -1


@pytest.mark.parametrize("n", [3, 50, 200])
def test_complete_one_two(n):
    """Complete graph with weights in [1, 2): every 2-hop path is >= 2 > any edge, so D = W, P = -1."""
    W, _ = workloads.grad_graph(n=n, seed=9)
    D, P = oracle.fw(W)
    np.testing.assert_array_equal(D, W.astype(np.float64))
    assert np.all(P == -1)


def test_star_graph():
    """Edges only to and from hub h: leaves i != j have D = W[i][h] + W[h][j], P = h."""
    n, h = 9, 4
    rng = np.random.default_rng(3)
    W = np.full((n, n), np.inf)
    np.fill_diagonal(W, 0)
    W[:, h] = rng.integers(1, 9, n)
    W[h, :] = rng.integers(1, 9, n)
    W[h, h] = 0
    D, P = oracle.fw(W)
    for i in range(n):
        for j in range(n):
            if i == j or h in (i, j):
                assert P[i, j] == -1
                continue
            assert D[i, j] == W[i, h] + W[h, j]
            assert P[i, j] == h


def test_disconnected_components():
    rng = np.random.default_rng(5)
    A = rand_graph(rng, 20, 0.4, wmax=9)
    B = rand_graph(rng, 15, 0.4, wmax=9)
    W = np.full((35, 35), np.inf)
    W[:20, :20] = A
    W[20:, 20:] = B
    D, P = oracle.fw(W)
    Da, Pa = oracle.fw(A)
    Db, Pb = oracle.fw(B)
    assert np.all(np.isinf(D[:20, 20:])) and np.all(np.isinf(D[20:, :20]))
    assert np.all(P[:20, 20:] == -1) and np.all(P[20:, :20] == -1)
    np.testing.assert_array_equal(D[:20, :20], Da)
    np.testing.assert_array_equal(P[:20, :20], Pa)
    np.testing.assert_array_equal(D[20:, 20:], Db)
    np.testing.assert_array_equal(P[20:, 20:], Pb + (Pb >= 0) * 20)


def test_uniform_complete_graph():
    """All edges of equal weight c: D = W (c <= 2c), P = -1."""
    n = 40
    W = np.full((n, n), 3.0)
    np.fill_diagonal(W, 0)
    D, P = oracle.fw(W)
    np.testing.assert_array_equal(D, W)
    assert np.all(P == -1)


# ---------------------------------------------------------------- library routines

@pytest.mark.parametrize("kind", ["int", "real"])
def test_scipy_shortest_path(kind):
    from scipy.sparse.csgraph import shortest_path
    rng = np.random.default_rng(7)
    n = 300
    W = rand_graph(rng, n, 0.05, wmax=20 if kind == "int" else None)
    D, P = oracle.fw(W)
    Wz = np.where(np.isfinite(W), W, 0.0)  # scipy dense: 0 = no edge off the diagonal
    for method in ("D", "FW"):
        Ds = shortest_path(Wz, method=method, directed=True)
        fin = np.isfinite(Ds)
        np.testing.assert_array_equal(np.isfinite(D), fin)
        if kind == "int":
            np.testing.assert_array_equal(D[fin], Ds[fin])
        else:
            np.testing.assert_allclose(D[fin], Ds[fin], rtol=1e-13)


def test_networkx_shortest_path_lengths():
    import networkx as nx
    rng = np.random.default_rng(8)
    n = 120
    W = rand_graph(rng, n, 0.08, wmax=15)
    D, _ = oracle.fw(W)
    G = nx.DiGraph()
    G.add_nodes_from(range(n))
    for i, j in zip(*np.nonzero(np.isfinite(W) & ~np.eye(n, dtype=bool))):
        G.add_edge(int(i), int(j), weight=float(W[i, j]))
    lengths = dict(nx.all_pairs_dijkstra_path_length(G))
    for i in range(n):
        for j in range(n):
            assert D[i, j] == lengths[i].get(j, np.inf)


# ---------------------------------------------------------------- independent algorithm

def test_dijkstra_rows_match_fw_integer():
    W = workloads.int_graph(n=512, p=0.5, wmax=1000, seed=1)
    D, P = oracle.fw(W)
    srcs = workloads.sample_sources(512, 64)
    Dr, Pr = oracle.dijkstra_rows(W, srcs)
    np.testing.assert_array_equal(Dr, D[srcs])
    np.testing.assert_array_equal(Pr, P[srcs])


def test_dijkstra_rows_tie_heavy():
    """Weights in [1, 3] at low density: many ties, P still canonical on both sides."""
    W = workloads.int_graph(n=256, p=0.05, wmax=3, seed=12)
    D, P = oracle.fw(W)
    srcs = np.arange(256)
    Dr, Pr = oracle.dijkstra_rows(W, srcs)
    np.testing.assert_array_equal(Dr, D)
    np.testing.assert_array_equal(Pr, P)


def test_dijkstra_rows_real():
    W = workloads.unit_complete(384, dtype=np.float64, seed=2)
    D, P = oracle.fw(W)
    srcs = workloads.sample_sources(384, 32)
    Dr, _ = oracle.dijkstra_rows(W, srcs)
    np.testing.assert_allclose(Dr, D[srcs], rtol=1e-13)


# ---------------------------------------------------------------- invariants

def test_invariants_c1_shape():
    W = workloads.int_graph(n=512, p=0.5, wmax=1000, seed=1)
    D, P = oracle.fw(W)
    oracle.check_invariants(W, D, P, exact=True)


def test_invariants_real():
    W = workloads.unit_complete(256, dtype=np.float64, seed=2)
    D, P = oracle.fw(W)
    oracle.check_invariants(W, D, P, exact=False, rtol=1e-13)


def test_threads_bit_identical():
    W = workloads.unit_complete(300, dtype=np.float64, seed=21)
    D1, P1 = oracle.fw(W, threads=1)
    D8, P8 = oracle.fw(W, threads=8)
    np.testing.assert_array_equal(D1, D8)
    np.testing.assert_array_equal(P1, P8)


def test_float32_input_widened_exactly():
    """float32 weights enter the double loop unchanged (widening is exact)."""
    W32 = workloads.unit_complete(128, dtype=np.float32, seed=2)
    D_a, P_a = oracle.fw(W32)
    D_b, P_b = oracle.fw(W32.astype(np.float64))
    np.testing.assert_array_equal(D_a, D_b)
    np.testing.assert_array_equal(P_a, P_b)


def test_input_contract_rejected():
    W = np.zeros((3, 3))
    W[1, 1] = 1.0
    with pytest.raises(ValueError):
        oracle.fw(W)
    W = np.zeros((3, 3))
    W[0, 1] = np.nan
    with pytest.raises(ValueError):
        oracle.fw(W)


def test_step_ranges_compose():
    """Running the outer iterations in two ranges gives the full loop's result."""
    W = workloads.unit_complete(200, dtype=np.float64, seed=13)
    D, P = oracle.fw(W)
    D2 = W.copy()
    P2 = np.full((200, 200), -1, dtype=np.int32)
    oracle.fw_steps(D2, P2, 0, 77)
    oracle.fw_steps(D2, P2, 77, 200)
    np.testing.assert_array_equal(D2, D)
    np.testing.assert_array_equal(P2, P)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_dijkstra_integer_float_input_matches_int64(dtype):
    """The float-input Dijkstra (exact conversion on read) equals the int64 one and FW."""
    W = workloads.int_graph(n=300, p=0.1, wmax=100, seed=31, dtype=dtype)
    srcs = workloads.sample_sources(300, 40)
    D1, P1 = oracle.dijkstra_rows_integer_float(W, srcs)
    D2, P2 = oracle.dijkstra_rows(W, srcs, exact=True)
    np.testing.assert_array_equal(D1, D2)
    np.testing.assert_array_equal(P1, P2)
    D, P = oracle.fw(W)
    np.testing.assert_array_equal(D1, D[srcs])
    np.testing.assert_array_equal(P1, P[srcs])


@pytest.mark.parametrize("wmax,p", [(1, 0.05), (3, 0.03), (100, 0.1), (7, 0.6)])
def test_dial_matches_fw_and_dijkstra(wmax, p):
    """Dial's bucket queue gives the classic loop's rows of D and canonical P."""
    n = 400
    W = workloads.int_graph(n=n, p=p, wmax=wmax, seed=32 + wmax)
    D, P = oracle.fw(W)
    srcs = np.arange(0, n, 7)
    Dd, Pd = oracle.dial_rows(W, srcs, wmax)
    np.testing.assert_array_equal(Dd, D[srcs])
    np.testing.assert_array_equal(Pd, P[srcs])
    Dd64, Pd64 = oracle.dial_rows(W.astype(np.float64), srcs, wmax)
    np.testing.assert_array_equal(Dd64, Dd)
    np.testing.assert_array_equal(Pd64, Pd)


def test_dial_with_generated_rows_equals_dial_on_the_matrix():
    """The on-demand-row form of the Dial search (used where the matrix never exists
    in host memory) gives the same rows of D and P as the search over the matrix,
    in both element types."""
    for dtype in (np.float32, np.float64):
        n = 700
        W = workloads.int_graph(n=n, p=0.05, wmax=20, seed=3, dtype=dtype)
        srcs = workloads.sample_sources(n, 12)
        Dm, Pm = oracle.dial_rows(W, srcs, 20)
        spec = workloads.graph_spec(3, n, 0.05, workloads.W_INT, 20, dtype)
        Dg, Pg = oracle.dial_rows_generated(spec, workloads.row_fn(), srcs, 20)
        assert np.array_equal(Dm, Dg) and np.array_equal(Pm, Pg)
        Do, Po = oracle.fw(W)
        assert np.array_equal(Dg, Do[srcs]) and np.array_equal(Pg, Po[srcs])
