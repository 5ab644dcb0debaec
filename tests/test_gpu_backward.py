"""GPU backward (fw_apsp_backward, subtree sums over shortest-path trees) against
the oracle's path walk, closed forms, float64 central differences and the
autograd wiring."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    import paper_2105_07298_amd as fw
    fw.lib()
    return torch.device("cuda:0")


def gpu_forward_backward(W, G, dev, case=""):
    import torch
    import paper_2105_07298_amd as fw
    print(f"[gpu] fwd+bwd {case} shape={W.shape} dtype={W.dtype}", flush=True)
    Wt = torch.from_numpy(np.ascontiguousarray(W)).to(dev).requires_grad_(True)
    D, P = fw.apsp_autograd(Wt)
    D.backward(torch.from_numpy(np.ascontiguousarray(G)).to(dev))
    torch.cuda.synchronize()
    return D.detach().cpu().numpy(), P.cpu().numpy(), Wt.grad.cpu().numpy()


@pytest.mark.parametrize("dtype,tol", [(np.float32, 1e-5), (np.float64, 1e-12)])
def test_integer_graph_matches_path_walk(dev, dtype, tol):
    """Tie-heavy integer weights: P is the oracle's, so the gradient is the oracle path walk."""
    W = workloads.int_graph(n=300, p=0.03, wmax=3, seed=61).astype(dtype)
    G = np.random.default_rng(1).standard_normal(W.shape).astype(dtype)
    D, P, gW = gpu_forward_backward(W, G, dev, "int")
    Do, Po = oracle.fw(W)
    np.testing.assert_array_equal(P, Po)
    ref = oracle.backward_pathwalk(Do, Po, G.astype(np.float64))
    np.testing.assert_allclose(gW, ref, rtol=tol, atol=tol * np.abs(ref).max())


@pytest.mark.parametrize("n", [64, 256])
def test_nondegenerate_real_weights(dev, n):
    """Uniform (0,1) complete graph: multi-hop paths; gradient vs the oracle path walk."""
    W = workloads.unit_complete(n, dtype=np.float64, seed=62)
    G = np.random.default_rng(2).standard_normal(W.shape)
    D, P, gW = gpu_forward_backward(W, G, dev, "unit")
    Do, Po = oracle.fw(W)
    assert (Po >= 0).mean() > 0.5
    np.testing.assert_array_equal(P, Po)
    ref = oracle.backward_pathwalk(Do, Po, G)
    np.testing.assert_allclose(gW, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def test_sparse_one_two_central_differences(dev):
    """Weights in [1, 2) at density 0.05 (multi-hop, generically unique paths): float64
    central differences of L = sum(G * D) with the oracle's forward, eps = 1e-4, on
    60 edges; edges where the one-sided differences disagree (a kink) are skipped."""
    n = 200
    W = workloads.graph(34, n, 0.05, workloads.W_ONE_TWO, 0, np.float64)
    G = np.random.default_rng(3).standard_normal((n, n))
    _, _, gW = gpu_forward_backward(W, G, dev, "sparse[1,2)")
    rng = np.random.default_rng(4)
    E = np.argwhere(np.isfinite(W) & ~np.eye(n, dtype=bool))
    checked = 0
    for u, v in E[rng.choice(len(E), 60, replace=False)]:
        def L(delta):
            Wp = W.copy()
            Wp[u, v] += delta
            D, _ = oracle.fw(Wp, exact=False)
            fin = np.isfinite(D)
            return float(np.sum(G[fin] * D[fin]))
        L0, Lp, Lm = L(0.0), L(1e-4), L(-1e-4)
        if abs((Lp - L0) - (L0 - Lm)) > 1e-10 * max(1.0, abs(L0)):
            continue
        fd = (Lp - Lm) / 2e-4
        assert abs(fd - gW[u, v]) <= 1e-6 * max(1.0, abs(fd)), (u, v, fd, gW[u, v])
        checked += 1
    assert checked >= 40


def test_c5_closed_form_and_fd(dev):
    """n = 2048 complete graph, weights in [1, 2) (float32), G ~ N(0,1): D = W, so
    dL/dW = G off the diagonal and 0 on it; float64 central differences (GPU float64
    forward) on 200 seeded edges agree."""
    import torch
    import paper_2105_07298_amd as fw
    W, G = workloads.grad_graph(n=2048, seed=5)
    D, P, gW = gpu_forward_backward(W, G, dev, "C5")
    np.testing.assert_array_equal(D, W)
    assert np.all(P == -1)
    expect = G.copy()
    np.fill_diagonal(expect, 0)
    np.testing.assert_array_equal(gW, expect)
    W64 = torch.from_numpy(W.astype(np.float64)).to(dev)
    G64 = torch.from_numpy(G.astype(np.float64)).to(dev)
    rng = np.random.default_rng(5)
    off = np.argwhere(~np.eye(2048, dtype=bool))
    for u, v in off[rng.choice(len(off), 200, replace=False)]:
        vals = []
        for delta in (1e-4, -1e-4):
            Wp = W64.clone()
            Wp[u, v] += delta
            Dp, _ = fw.apsp(Wp, path=False)
            vals.append(float((G64 * Dp).sum()))
        fd = (vals[0] - vals[1]) / 2e-4
        assert abs(fd - float(gW[u, v])) <= 1e-6 * max(1.0, abs(fd)), (u, v, fd, gW[u, v])


def test_batched_forward_backward(dev):
    """A batch of 256 graphs at n = 128 with integer weights in [1, 20] at density 0.1
    (multi-hop paths, exact in float32, so both sides share the canonical P): every
    sampled graph's gradient equals the oracle path walk of the oracle's forward."""
    B, n = 256, 128
    Ws = np.stack([workloads.graph(70, n, 0.1, workloads.W_INT, 20, np.float32, g=b) for b in range(B)])
    G = np.random.default_rng(6).standard_normal(Ws.shape).astype(np.float32)
    D, P, gW = gpu_forward_backward(Ws, G, dev, "batch")
    for b in range(0, B, 17):
        Do, Po = oracle.fw(Ws[b])
        np.testing.assert_array_equal(P[b], Po)
        ref = oracle.backward_pathwalk(Do, Po, G[b].astype(np.float64))
        np.testing.assert_allclose(gW[b], ref, rtol=1e-5, atol=1e-5 * np.abs(ref).max())


def test_batched_real_weights_vs_path_walk(dev):
    """A batch of 64 graphs at n = 128, float32 weights in [1, 2) at density 0.1
    (multi-hop paths, real weights): each graph's GPU (D, P) passes the checker, and
    its gradient equals the oracle path walk over the GPU's own (D, P) -- the
    subgradient along the paths that P encodes, whichever of two near-equal paths
    rounding made the GPU pick."""
    B, n = 64, 128
    Ws = np.stack([workloads.graph(71, n, 0.1, workloads.W_ONE_TWO, 0, np.float32, g=b) for b in range(B)])
    G = np.random.default_rng(7).standard_normal(Ws.shape).astype(np.float32)
    D, P, gW = gpu_forward_backward(Ws, G, dev, "batch-real")
    hops = 0
    for b in range(B):
        Do, _ = oracle.fw(Ws[b], exact=False)
        fin = np.isfinite(Do)
        assert np.array_equal(np.isfinite(D[b]), fin)
        assert np.max(np.abs(D[b][fin] - Do[fin]) / np.maximum(Do[fin], 1e-30)) <= 1e-5
        oracle.check_invariants(Ws[b], D[b], P[b], exact=False, rtol=1e-5, nsample=50, seed=b)
        hops += int((P[b] >= 0).sum())
        ref = oracle.backward_pathwalk(D[b].astype(np.float64), P[b], G[b].astype(np.float64))
        np.testing.assert_allclose(gW[b], ref, rtol=1e-5, atol=1e-5 * np.abs(ref).max())
    assert hops > B * n * 10  # multi-hop paths throughout


def test_c5_batch_closed_form(dev):
    """The 256 x 128 complete-graph batch with weights in [1, 2): D = W and dL/dW = G
    off the diagonal for every graph."""
    B, n = 256, 128
    Ws = np.stack([workloads.grad_graph(n=n, seed=5, g=b)[0] for b in range(B)])
    G = np.stack([workloads.grad_graph(n=n, seed=5, g=b)[1] for b in range(B)])
    D, P, gW = gpu_forward_backward(Ws, G, dev, "C5-batch")
    np.testing.assert_array_equal(D, Ws)
    assert np.all(P == -1)
    expect = G.copy()
    expect[:, np.arange(n), np.arange(n)] = 0
    np.testing.assert_array_equal(gW, expect)


def test_backward_is_deterministic(dev):
    """The same (D, P, G) gives the same gradient bit for bit on repeated calls
    (float32 and float64), and it equals the oracle path walk over those (D, P)."""
    import torch
    import paper_2105_07298_amd as fw
    for dtype, tol in ((np.float32, 1e-5), (np.float64, 1e-12)):
        W = workloads.unit_complete(384, dtype=dtype, seed=63)
        G = np.random.default_rng(8).standard_normal(W.shape).astype(dtype)
        print(f"[gpu] backward determinism {np.dtype(dtype).name}", flush=True)
        D, P = fw.apsp(torch.from_numpy(W).to(dev))
        Gt = torch.from_numpy(G).to(dev)
        outs = [fw.apsp_backward(D, P, Gt) for _ in range(3)]
        torch.cuda.synchronize()
        outs = [o.cpu().numpy() for o in outs]
        for o in outs[1:]:
            assert np.array_equal(o, outs[0])
        ref = oracle.backward_pathwalk(D.cpu().numpy().astype(np.float64), P.cpu().numpy(), G.astype(np.float64))
        np.testing.assert_allclose(outs[0], ref, rtol=tol, atol=tol * np.abs(ref).max())


def test_backward_bad_labels_count_as_unreachable(dev):
    """Labels outside [-1, n) in a caller's path matrix are never followed: the pair
    (and the subtree below it in that source's tree) contributes nothing."""
    import torch
    import paper_2105_07298_amd as fw
    n = 96
    W = np.full((n, n), np.inf, dtype=np.float32)
    np.fill_diagonal(W, 0)
    W[np.arange(n - 1), np.arange(1, n)] = 1.0 + np.arange(n - 1, dtype=np.float32) / 128
    Do, Po = oracle.fw(W)
    G = np.random.default_rng(9).standard_normal((n, n))
    Pbad = Po.copy()
    Pbad[0, 40] = n + 5        # out of range: source 0 loses vertex 40 and everything after it
    Pbad[3, 70] = -7           # negative non-sentinel: source 3 loses 70 onwards
    Gm = G.copy()
    Gm[0, 40:] = 0
    Gm[3, 70:] = 0
    expect = oracle.backward_pathwalk(Do, Po, Gm)
    print("[gpu] backward with out-of-range labels", flush=True)
    gW = fw.apsp_backward(torch.from_numpy(Do.astype(np.float32)).to(dev), torch.from_numpy(Pbad).to(dev),
                          torch.from_numpy(G.astype(np.float32)).to(dev))
    torch.cuda.synchronize()
    np.testing.assert_allclose(gW.cpu().numpy(), expect, rtol=1e-5, atol=1e-5 * np.abs(expect).max())


def test_backward_rejects_bad_arguments(dev):
    import paper_2105_07298_amd as fw
    L = fw.lib()
    assert L.fw_apsp_backward(0, 5000, 1, 4096, 4096, 4096, 4096, None) == fw.FW_EINVAL
    assert L.fw_apsp_backward(0, 16, 1, 4096, None, 4096, 4096, None) == fw.FW_EINVAL
    assert L.fw_apsp_backward(0, 16, 0, 4096, 4096, 4096, 4096, None) == fw.FW_EINVAL
