"""Pins for the oracle's gradient (path walk): closed forms, a library routine
(networkx edge betweenness), Euler homogeneity, and float64 central differences."""
import numpy as np
import pytest

import oracle
import workloads


def loss_and_grad(W, G):
    D, P = oracle.fw(W, exact=False)
    fin = np.isfinite(D)
    L = float(np.sum(G[fin] * D[fin]))
    return L, oracle.backward_pathwalk(D, P, G), D, P


def test_complete_one_two_closed_form():
    """D = W on the complete [1,2) graph, so dL/dW = G off the diagonal and 0 on it."""
    W, G = workloads.grad_graph(n=96, seed=5)
    _, gW, _, _ = loss_and_grad(W.astype(np.float64), G.astype(np.float64))
    expect = G.astype(np.float64).copy()
    np.fill_diagonal(expect, 0.0)
    np.testing.assert_array_equal(gW, expect)


def test_path_graph_closed_form():
    """On 0->1->..->n-1, edge (t, t+1) carries every pair i <= t < j: gW = sum of those G[i][j]."""
    n = 30
    rng = np.random.default_rng(1)
    W = np.full((n, n), np.inf)
    np.fill_diagonal(W, 0)
    W[np.arange(n - 1), np.arange(1, n)] = rng.uniform(1, 2, n - 1)
    G = rng.standard_normal((n, n))
    _, gW, _, _ = loss_and_grad(W, G)
    for t in range(n - 1):
        expect = sum(G[i, j] for i in range(t + 1) for j in range(t + 1, n))
        assert abs(gW[t, t + 1] - expect) < 1e-12
    mask = np.ones((n, n), dtype=bool)
    mask[np.arange(n - 1), np.arange(1, n)] = False
    assert np.all(gW[mask] == 0)


def test_networkx_edge_betweenness():
    """With G = 1 and unique shortest paths, dL/dW[u][v] counts the pairs routed over u->v."""
    import networkx as nx
    rng = np.random.default_rng(2)
    n = 60
    W = np.full((n, n), np.inf)
    mask = rng.random((n, n)) < 0.15
    W[mask] = rng.uniform(0.1, 1.0, size=mask.sum())
    np.fill_diagonal(W, 0)
    G = np.ones((n, n))
    _, gW, _, _ = loss_and_grad(W, G)
    g = nx.DiGraph()
    g.add_nodes_from(range(n))
    for i, j in zip(*np.nonzero(np.isfinite(W) & ~np.eye(n, dtype=bool))):
        g.add_edge(int(i), int(j), weight=float(W[i, j]))
    eb = nx.edge_betweenness_centrality(g, normalized=False, weight="weight")
    for (u, v), val in eb.items():
        assert abs(gW[u, v] - val) < 1e-9, (u, v, gW[u, v], val)


def test_euler_homogeneity():
    """D(c W) = c D(W), so sum(W * dL/dW) = sum(G * D) (finite entries)."""
    W = workloads.unit_complete(128, dtype=np.float64, seed=2)
    rng = np.random.default_rng(3)
    G = rng.standard_normal(W.shape)
    L, gW, _, _ = loss_and_grad(W, G)
    fin = np.isfinite(W)
    assert abs(float(np.sum(W[fin] * gW[fin])) - L) < 1e-9 * max(1.0, abs(L))


@pytest.mark.parametrize("case", ["unit_dense", "sparse_one_two"])
def test_central_differences(case):
    """float64 central differences (eps = 1e-4) on 60 random edges; kink guard skips edges
    whose forward and backward one-sided differences disagree."""
    rng = np.random.default_rng(11)
    if case == "unit_dense":
        n = 48
        W = workloads.unit_complete(n, dtype=np.float64, seed=33)
    else:
        n = 64
        W = workloads.graph(34, n, 0.08, workloads.W_ONE_TWO, 0, np.float64)
    G = rng.standard_normal((n, n))
    _, gW, _, _ = loss_and_grad(W, G)
    E = np.argwhere(np.isfinite(W) & ~np.eye(n, dtype=bool))
    pick = E[rng.choice(len(E), size=min(60, len(E)), replace=False)]
    eps = 1e-4
    checked = 0
    for u, v in pick:
        def L_at(delta):
            Wp = W.copy()
            Wp[u, v] += delta
            D, _ = oracle.fw(Wp, exact=False)
            fin = np.isfinite(D)
            return float(np.sum(G[fin] * D[fin]))
        L0, Lp, Lm = L_at(0.0), L_at(eps), L_at(-eps)
        fwd, bwd = (Lp - L0) / eps, (L0 - Lm) / eps
        if abs(fwd - bwd) > 1e-6 * max(1.0, abs(fwd)):
            continue  # kink: the path set changes inside [-eps, eps]
        fd = (Lp - Lm) / (2 * eps)
        assert abs(fd - gW[u, v]) < 1e-6 * max(1.0, abs(fd)), (u, v, fd, gW[u, v])
        checked += 1
    assert checked >= 40
    # the non-degenerate case must exercise multi-hop paths
    _, P = oracle.fw(W, exact=False)
    assert np.any(P >= 0)
