"""GPU parity of fw_apsp_batched (one persistent launch over many graphs) against
the CPU oracle, graph by graph, and against fw_apsp on each graph."""
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


def ragged(graphs, dtype):
    ns = np.array([g.shape[0] for g in graphs], dtype=np.int32)
    off = np.zeros(len(graphs) + 1, dtype=np.int64)
    off[1:] = np.cumsum(ns.astype(np.int64) ** 2)
    W = np.concatenate([g.astype(dtype).ravel() for g in graphs])
    return ns, off, W


def run_batched(ns, off, W, dev, path=True, case="", route=0):
    import torch
    import paper_2105_07298_amd as fw
    print(f"[gpu] fw_apsp_batched {case} batch={ns.size} dtype={W.dtype} path={path} route={route}", flush=True)
    D, P = fw.apsp_batched(torch.from_numpy(W).to(dev), ns, off[:-1], path=path, route=route)
    torch.cuda.synchronize()
    return D.cpu().numpy(), (P.cpu().numpy() if P is not None else None)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("path", [True, False])
@pytest.mark.parametrize("route", [0, -1])
def test_batched_integer_exact(dev, dtype, path, route):
    """Uneven sizes (1 .. 300, including non-multiples of the tile), tie-heavy integer
    weights: every graph's D and P equal the oracle bit for bit, with the largest
    graphs routed to fw_apsp (route 0: the n = 300 graph holds far more than its share)
    and with every graph in the persistent launch (route -1)."""
    rng = np.random.default_rng(5)
    sizes = [1, 2, 5, 17, 63, 64, 65, 100, 128, 129, 200, 300] + list(rng.integers(1, 260, 28))
    graphs = [workloads.int_graph(n=int(n), p=float(rng.uniform(0.02, 0.5)), wmax=3, seed=300 + i)
              for i, n in enumerate(sizes)]
    ns, off, W = ragged(graphs, dtype)
    D, P = run_batched(ns, off, W, dev, path=path, case="integer", route=route)
    for b, g in enumerate(graphs):
        n = g.shape[0]
        Do, Po = oracle.fw(g)
        np.testing.assert_array_equal(D[off[b]:off[b + 1]].reshape(n, n).astype(np.float64), Do)
        if path:
            np.testing.assert_array_equal(P[off[b]:off[b + 1]].reshape(n, n), Po)


def test_batched_equals_single_graph(dev):
    """Each graph's batched result equals the oracle's, and fw_apsp's on the same graph."""
    import torch
    import paper_2105_07298_amd as fw
    rng = np.random.default_rng(6)
    graphs = [workloads.int_graph(n=int(n), p=0.2, wmax=20, seed=400 + i)
              for i, n in enumerate(rng.integers(16, 400, 12))]
    ns, off, W = ragged(graphs, np.float32)
    D, P = run_batched(ns, off, W, dev, case="vs-single")
    for b, g in enumerate(graphs):
        n = g.shape[0]
        Db, Pb = D[off[b]:off[b + 1]].reshape(n, n), P[off[b]:off[b + 1]].reshape(n, n)
        Do, Po = oracle.fw(g)
        np.testing.assert_array_equal(Db.astype(np.float64), Do)
        np.testing.assert_array_equal(Pb, Po)
        Ds, Ps = fw.apsp(torch.from_numpy(g).to(dev))
        np.testing.assert_array_equal(Db, Ds.cpu().numpy())
        np.testing.assert_array_equal(Pb, Ps.cpu().numpy())


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_batched_one_round_graphs(dev, dtype):
    """3,000 graphs with n in [2, 32] (one round of 32-tiles: phase 1 only, whose
    label stores the widening pass then reads back) and tie-heavy integer weights,
    with the path matrix: D and P equal the oracle's graph by graph."""
    rng = np.random.default_rng(12)
    sizes = rng.integers(2, 33, 3000)
    graphs = [workloads.int_graph(n=int(n), p=float(rng.uniform(0.1, 0.6)), wmax=3, seed=900 + i)
              for i, n in enumerate(sizes)]
    ns, off, W = ragged(graphs, dtype)
    D, P = run_batched(ns, off, W, dev, case="one-round")
    print("[cpu] oracle on 3,000 graphs", flush=True)
    for b, g in enumerate(graphs):
        n = g.shape[0]
        Do, Po = oracle.fw(g, threads=1)
        np.testing.assert_array_equal(D[off[b]:off[b + 1]].reshape(n, n).astype(np.float64), Do, err_msg=str(b))
        np.testing.assert_array_equal(P[off[b]:off[b + 1]].reshape(n, n), Po, err_msg=str(b))


def test_batched_gaps_and_order(dev):
    """Graphs at arbitrary (unaligned, non-contiguous) offsets; bytes between graphs untouched."""
    rng = np.random.default_rng(7)
    graphs = [workloads.int_graph(n=int(n), p=0.3, wmax=9, seed=500 + i)
              for i, n in enumerate([70, 3, 129, 1, 40])]
    ns = np.array([g.shape[0] for g in graphs], dtype=np.int32)
    gaps = [5, 1, 3, 7, 2]
    offs, pos = [], 0
    for g, gap in zip(graphs, gaps):
        pos += gap
        offs.append(pos)
        pos += g.size
    W = np.full(pos + 3, -7.0, dtype=np.float32)
    for g, o in zip(graphs, offs):
        W[o:o + g.size] = g.ravel()
    offs = np.array(offs + [pos], dtype=np.int64)
    D, P = run_batched(ns, offs, W, dev, case="gaps")
    mask = np.ones(W.size, dtype=bool)
    for b, g in enumerate(graphs):
        n = g.shape[0]
        o = offs[b]
        mask[o:o + g.size] = False
        Do, Po = oracle.fw(g)
        np.testing.assert_array_equal(D[o:o + g.size].reshape(n, n).astype(np.float64), Do)
        np.testing.assert_array_equal(P[o:o + g.size].reshape(n, n), Po)
    assert np.all(D[mask] == -7.0)


@pytest.mark.timeout(900)
def test_batched_c4_full(dev):
    """The benchmark batch: 10,000 graphs, n uniform in [16, 512], density uniform in
    [0.1, 1.0), weights uniform real in [1, 10] (float32), path matrices.  Every graph
    within 1e-5 relative of the float64 oracle, and every graph's path matrix through
    the checker (all pairs: encoded paths exist, split at their label and sum to D)."""
    ns, off, W = workloads.batch_graphs(batch=10000, seed=4)
    D, P = run_batched(ns, off, W, dev, case="C4")
    print("[cpu] oracle on 10,000 graphs", flush=True)
    worst = 0.0
    rng = np.random.default_rng(8)
    for b in range(ns.size):
        n = int(ns[b])
        Wg = W[off[b]:off[b + 1]].reshape(n, n)
        Dg = D[off[b]:off[b + 1]].reshape(n, n)
        Do, _ = oracle.fw(Wg, exact=False)
        fin = np.isfinite(Do)
        assert np.array_equal(np.isfinite(Dg), fin), b
        nz = fin & (Do > 0)
        worst = max(worst, float(np.max(np.abs(Dg[nz] - Do[nz]) / Do[nz])) if nz.any() else 0.0)
        Pg = P[off[b]:off[b + 1]].reshape(n, n)
        oracle.check_invariants(Wg, Dg, Pg, exact=False, rtol=1e-5, nsample=10 if b % 100 else 200, seed=b)
    print(f"max relative error over the batch {worst:.3e}", flush=True)
    assert worst <= 1e-5


@pytest.mark.parametrize("route", [0, -1, 100])
def test_batched_routing(dev, route):
    """One graph of n = 700 among small ones: routed to fw_apsp by the automatic rule
    (route 0) or by size (route 100, which also routes the n = 130 graph), or kept in
    the persistent launch (route -1); D and P equal the oracle's in every case."""
    rng = np.random.default_rng(10)
    sizes = [700, 130, 65, 33, 7] + list(rng.integers(2, 60, 11))
    graphs = [workloads.int_graph(n=int(n), p=0.05 if n > 300 else 0.2, wmax=4, seed=700 + i)
              for i, n in enumerate(sizes)]
    ns, off, W = ragged(graphs, np.float32)
    D, P = run_batched(ns, off, W, dev, case="routing", route=route)
    for b, g in enumerate(graphs):
        n = g.shape[0]
        Do, Po = oracle.fw(g)
        np.testing.assert_array_equal(D[off[b]:off[b + 1]].reshape(n, n).astype(np.float64), Do)
        np.testing.assert_array_equal(P[off[b]:off[b + 1]].reshape(n, n), Po)


def test_batched_large_graph_in_launch(dev):
    """n = 2048 (32 rounds of 64-tiles, labels up to 2047 in the 16-bit in-solve
    form) kept in the persistent launch, beside small graphs: D and P equal the
    oracle's bit for bit (tie-heavy integer weights), and fw_apsp's."""
    import torch
    import paper_2105_07298_amd as fw
    graphs = [workloads.int_graph(n=2048, p=0.01, wmax=3, seed=800)] + \
             [workloads.int_graph(n=int(n), p=0.2, wmax=3, seed=801 + i) for i, n in enumerate([5, 63, 130])]
    ns, off, W = ragged(graphs, np.float32)
    D, P = run_batched(ns, off, W, dev, case="large in launch", route=-1)
    for b, g in enumerate(graphs):
        n = g.shape[0]
        Db, Pb = D[off[b]:off[b + 1]].reshape(n, n), P[off[b]:off[b + 1]].reshape(n, n)
        print(f"[cpu] oracle n={n}", flush=True)
        Do, Po = oracle.fw(g)
        np.testing.assert_array_equal(Db.astype(np.float64), Do)
        np.testing.assert_array_equal(Pb, Po)
        assert n < 2048 or (Po >= 1024).any()  # labels beyond 10 bits occur
        Ds, Ps = fw.apsp(torch.from_numpy(g).to(dev))
        np.testing.assert_array_equal(Db, Ds.cpu().numpy())
        np.testing.assert_array_equal(Pb, Ps.cpu().numpy())


def test_batched_rejects_bad_arguments(dev):
    import ctypes
    import paper_2105_07298_amd as fw
    from paper_2105_07298_amd._lib import FwBatchedConfig
    L = fw.lib()
    ns = np.array([4, 0], dtype=np.int32)
    offs = np.array([0, 16], dtype=np.int64)
    st = L.fw_apsp_batched(0, 2, ns.ctypes.data, offs.ctypes.data, 4096, None, None)
    assert st == fw.FW_EINVAL
    ns = np.array([4097], dtype=np.int32)
    st = L.fw_apsp_batched(0, 1, ns.ctypes.data, offs.ctypes.data, 4096, None, None)
    assert st == fw.FW_EINVAL
    ns = np.array([4], dtype=np.int32)
    for bad in (FwBatchedConfig(-1, -2, 0, 0), FwBatchedConfig(-1, 0, 1, 0), FwBatchedConfig(-1, 0, 0, 1)):
        st = L.fw_apsp_batched_config(0, 1, ns.ctypes.data, offs.ctypes.data, 4096, None, ctypes.byref(bad), None)
        assert st == fw.FW_EINVAL


@pytest.mark.parametrize("small_max_n", [0, 96, 1 << 20])
def test_batched_tile_choice_invariance(dev, small_max_n):
    """Whatever graphs are processed in 32 x 32 or 64 x 64 tiles, D and P are the oracle's."""
    import torch
    import paper_2105_07298_amd as fw
    rng = np.random.default_rng(9)
    graphs = [workloads.int_graph(n=int(n), p=0.1, wmax=3, seed=600 + i)
              for i, n in enumerate(rng.integers(1, 200, 24))]
    ns, off, W = ragged(graphs, np.float32)
    print(f"[gpu] fw_apsp_batched_config small_max_n={small_max_n}", flush=True)
    D, P = fw.apsp_batched(torch.from_numpy(W).to(dev), ns, off[:-1], path=True, small_max_n=small_max_n)
    torch.cuda.synchronize()
    D, P = D.cpu().numpy(), P.cpu().numpy()
    for b, g in enumerate(graphs):
        n = g.shape[0]
        Do, Po = oracle.fw(g)
        np.testing.assert_array_equal(D[off[b]:off[b + 1]].reshape(n, n).astype(np.float64), Do)
        np.testing.assert_array_equal(P[off[b]:off[b + 1]].reshape(n, n), Po)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_batched_device_arrays(dev, dtype):
    """fw_apsp_batched_device: counts and offsets in device memory, the queue built on
    the device.  Every valid graph equals the oracle bit for bit (tie-heavy integer
    weights, n from 1 to 300); graphs with n = 0, n = 5000 or a negative offset are
    skipped and their bytes left untouched."""
    import torch
    import paper_2105_07298_amd as fw
    rng = np.random.default_rng(13)
    sizes = [1, 2, 31, 32, 33, 64, 65, 300] + list(rng.integers(1, 200, 40))
    graphs = [workloads.int_graph(n=int(n), p=float(rng.uniform(0.02, 0.4)), wmax=3, seed=1100 + i)
              for i, n in enumerate(sizes)]
    ns, off, W = ragged(graphs, dtype)
    # three invalid entries pointing at a sentinel region after the graphs
    tail = W.size
    W = np.concatenate([W, np.full(64, -3.0, dtype=dtype)])
    ns_d = np.concatenate([ns, np.array([0, 5000, 4], dtype=np.int32)])
    off_d = np.concatenate([off[:-1], np.array([tail, tail, -16], dtype=np.int64)])
    Wt = torch.from_numpy(W).to(dev)
    P = torch.full(Wt.shape, -9, dtype=torch.int32, device=dev)
    print(f"[gpu] fw_apsp_batched_device batch={ns_d.size} dtype={W.dtype}", flush=True)
    fw.apsp_batched_device_(Wt, torch.from_numpy(ns_d).to(dev), torch.from_numpy(off_d).to(dev), P)
    torch.cuda.synchronize()
    D, P = Wt.cpu().numpy(), P.cpu().numpy()
    for b, g in enumerate(graphs):
        n = g.shape[0]
        Do, Po = oracle.fw(g)
        np.testing.assert_array_equal(D[off[b]:off[b + 1]].reshape(n, n).astype(np.float64), Do)
        np.testing.assert_array_equal(P[off[b]:off[b + 1]].reshape(n, n), Po)
    assert np.all(D[tail:] == -3.0) and np.all(P[tail:] == -9)
