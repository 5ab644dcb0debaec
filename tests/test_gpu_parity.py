"""GPU parity: fw_apsp (through the C ABI) against the CPU oracle on the same
seeded inputs.

Integer-valued weights: distances and path matrix bit-exact (every sum is an
integer below 2^24, so float32 is exact and the lexicographic path rule gives the
canonical P whatever the block size).  Real weights: max relative error 1e-5
(float32) / 1e-12 (float64) against the float64 oracle on the same weight bits,
identical +inf pattern, and the path matrix checked by its invariants.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu



def compiled_configs(dtype, n):
    """Every compiled configuration, once per round schedule that applies to it at size n."""
    import paper_2105_07298_amd as fw
    out = []
    for b, tm, tn, var in fw.fw_list_configs(fw.FW_F32 if dtype == np.float32 else fw.FW_F64):
        out.append((b, tm, tn, var, fw.FW_SCHED_SERIAL))
        if fw.lookahead_applies(b, tm, tn, n):
            out.append((b, tm, tn, var, fw.FW_SCHED_LOOKAHEAD))
        if fw.pairs_applies(b, tm, tn, var, n):
            out.append((b, tm, tn, var, fw.FW_SCHED_PAIRS))
        if fw.pairs_lookahead_applies(b, tm, tn, var, n):
            out.append((b, tm, tn, var, fw.FW_SCHED_PAIRS_LOOKAHEAD))
    return out


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_2105_07298_amd as fw
    fw.lib()
    return torch.device("cuda:0")


def run_gpu(W, dev, path=True, block=0, tile=(0, 0), variant=0, schedule=0, case=""):
    import torch
    import paper_2105_07298_amd as fw
    print(f"[gpu] fw_apsp {case} n={W.shape[0]} dtype={W.dtype} path={path} block={block} tile={tile} "
          f"variant={variant} schedule={schedule}", flush=True)
    D, P = fw.apsp(torch.from_numpy(np.ascontiguousarray(W)).to(dev), path=path, block=block,
                   tile_m=tile[0], tile_n=tile[1], variant=variant, schedule=schedule)
    torch.cuda.synchronize()
    return D.cpu().numpy(), (P.cpu().numpy() if P is not None else None)


def assert_exact(W, Dg, Pg, Do=None, Po=None):
    if Do is None:
        Do, Po = oracle.fw(W)
    np.testing.assert_array_equal(Dg.astype(np.float64), Do)
    if Pg is not None:
        np.testing.assert_array_equal(Pg, Po)


def rel_err(Dg, Do):
    fin = np.isfinite(Do)
    assert np.array_equal(np.isfinite(Dg), fin), "+inf pattern differs"
    d = Dg[fin].astype(np.float64)
    o = Do[fin]
    nz = o != 0
    assert np.all(d[~nz] == 0), "zero distance mismatch"
    return float(np.max(np.abs(d[nz] - o[nz]) / o[nz])) if nz.any() else 0.0


# ------------------------------------------------------------------ integer weights: bit-exact

@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("path", [True, False])
def test_c1_bit_exact(dev, dtype, path):
    """n = 512, edge probability 0.5, integer weights in [1, 1000]."""
    W = workloads.int_graph(n=512, p=0.5, wmax=1000, seed=1, dtype=dtype)
    Dg, Pg = run_gpu(W, dev, path=path, case="C1")
    assert_exact(W, Dg, Pg)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_block_and_tile_invariance_tie_heavy(dev, dtype):
    """Weights in [1, 3] at low density: many equal-length paths.  Every compiled
    (block, tile) gives the oracle's D and canonical P exactly."""
    W = workloads.int_graph(n=448, p=0.02, wmax=3, seed=21, dtype=dtype)
    Do, Po = oracle.fw(W)
    assert (Po >= 0).mean() > 0.5
    for block, tm, tn, var, sch in compiled_configs(dtype, W.shape[0]):
        Dg, Pg = run_gpu(W, dev, block=block, tile=(tm, tn), variant=var, schedule=sch, case="tie-heavy")
        assert_exact(W, Dg, Pg, Do, Po)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n", [1, 2, 3, 5, 31, 63, 64, 65, 127, 129, 200, 333])
def test_ragged_sizes(dev, dtype, n):
    W = workloads.int_graph(n=n, p=0.3, wmax=50, seed=100 + n, dtype=dtype)
    Dg, Pg = run_gpu(W, dev, case="ragged")
    assert_exact(W, Dg, Pg)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_no_edges(dev, dtype):
    n = 130
    W = np.full((n, n), np.inf, dtype=dtype)
    np.fill_diagonal(W, 0)
    Dg, Pg = run_gpu(W, dev, case="no-edges")
    np.testing.assert_array_equal(Dg, W)
    assert np.all(Pg == -1)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_complete_one_two_is_fixed_point(dev, dtype):
    """Weights in [1, 2): every two-hop path is >= 2 > any edge, so D = W and P = -1."""
    W, _ = workloads.grad_graph(n=320, seed=5)
    W = W.astype(dtype)
    Dg, Pg = run_gpu(W, dev, case="complete[1,2)")
    np.testing.assert_array_equal(Dg, W)
    assert np.all(Pg == -1)


def test_directed_path_graph(dev):
    n = 300
    rng = np.random.default_rng(3)
    W = np.full((n, n), np.inf, dtype=np.float32)
    np.fill_diagonal(W, 0)
    W[np.arange(n - 1), np.arange(1, n)] = rng.integers(1, 20, n - 1)
    Dg, Pg = run_gpu(W, dev, case="path-graph")
    assert_exact(W, Dg, Pg)
    j = np.arange(n)
    assert np.all(Pg[0, 2:] == j[2:] - 1)


def test_disconnected_blocks(dev):
    A = workloads.int_graph(n=150, p=0.1, wmax=9, seed=41)
    B = workloads.int_graph(n=170, p=0.1, wmax=9, seed=42)
    W = np.full((320, 320), np.inf, dtype=np.float32)
    W[:150, :150] = A
    W[150:, 150:] = B
    Dg, Pg = run_gpu(W, dev, case="disconnected")
    assert_exact(W, Dg, Pg)
    assert np.all(np.isinf(Dg[:150, 150:])) and np.all(Pg[:150, 150:] == -1)


def test_distance_only_matches_path_mode(dev):
    W = workloads.unit_complete(640, dtype=np.float32, seed=2)
    D1, _ = run_gpu(W, dev, path=False, case="dist-only")
    D2, _ = run_gpu(W, dev, path=True, case="path")
    np.testing.assert_array_equal(D1, D2)


def test_misaligned_and_nondefault_stream(dev):
    """A tensor view that is not 16-byte aligned goes through the padded copy; the call
    runs on the caller's current (non-default) stream."""
    import torch
    import paper_2105_07298_amd as fw
    n = 256
    W = workloads.int_graph(n=n, p=0.2, wmax=100, seed=7)
    buf = torch.empty(n * n + 1, dtype=torch.float32, device=dev)
    D = buf[1:].view(n, n)
    assert D.data_ptr() % 16 != 0
    D.copy_(torch.from_numpy(W))
    P = torch.empty((n, n), dtype=torch.int32, device=dev)
    s = torch.cuda.Stream(dev)
    with torch.cuda.stream(s):
        print("[gpu] fw_apsp misaligned view on a side stream", flush=True)
        fw.apsp_(D, P)
    s.synchronize()
    assert_exact(W, D.cpu().numpy(), P.cpu().numpy())


# ------------------------------------------------------------------ real weights: tolerance

@pytest.mark.parametrize("dtype,tol", [(np.float32, 1e-5), (np.float64, 1e-12)])
def test_c2_4096_full_matrix(dev, dtype, tol):
    """Complete graph, weights strictly inside (0, 1), n = 4096: every entry vs the
    float64 oracle on the same weight bits."""
    W = workloads.unit_complete(4096, dtype=dtype, seed=2)
    Dg, Pg = run_gpu(W, dev, case="C2")
    print("[cpu] oracle n=4096", flush=True)
    Do, _ = oracle.fw(W, exact=False)
    err = rel_err(Dg, Do)
    print(f"max relative error {err:.3e}", flush=True)
    assert err <= tol
    oracle.check_invariants(W, Dg, Pg, exact=False, rtol=max(tol, 1e-7), nsample=3000)


@pytest.mark.parametrize("dtype,tol", [(np.float32, 1e-5), (np.float64, 1e-12)])
def test_configs_real_weights(dev, dtype, tol):
    """Complete graph, weights in (0, 1), n = 700 (pads to several tiles of every
    shape, with a ragged last block): every compiled configuration is within the
    tolerance of the float64 oracle, and those that share a block size agree bit
    for bit (for each entry they form the minimum of the same float sums; only
    the tile shape or the last-phase kernel differs)."""
    W = workloads.unit_complete(700, dtype=dtype, seed=9)
    Do, _ = oracle.fw(W, exact=False)
    first = {}
    for block, tm, tn, var, sch in compiled_configs(dtype, W.shape[0]):
        Dg, Pg = run_gpu(W, dev, block=block, tile=(tm, tn), variant=var, schedule=sch, case="real-weights")
        assert rel_err(Dg, Do) <= tol
        if block not in first:
            first[block] = (Dg, Pg)
            oracle.check_invariants(W, Dg, Pg, exact=False, rtol=max(tol, 1e-7), nsample=1000)
        else:
            np.testing.assert_array_equal(Dg, first[block][0])
            np.testing.assert_array_equal(Pg, first[block][1])


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype,tol", [(np.float32, 1e-5), (np.float64, 1e-12)])
@pytest.mark.parametrize("n", [8192, 16384])
def test_c2_large_dijkstra_rows(dev, n, dtype, tol):
    """n = 8192 and 16384 (the benchmark size; the tuned schedule changes at 8192):
    64 seeded source rows vs float64 Dijkstra, and the path matrix on those rows
    through the checker (every encoded path exists, splits at its label and sums to
    D within the tolerance)."""
    W = workloads.unit_complete(n, dtype=dtype, seed=2)
    Dg, Pg = run_gpu(W, dev, case=f"C2-{n}")
    srcs = workloads.sample_sources(n, 64)
    print("[cpu] dijkstra 64 rows", flush=True)
    Dr, _ = oracle.dijkstra_rows(W, srcs, exact=False)
    err = rel_err(Dg[srcs], Dr)
    print(f"max relative error {err:.3e}", flush=True)
    assert err <= tol
    print("[cpu] checker on the 64 rows", flush=True)
    oracle.check_invariants(W, Dg, Pg, exact=False, rtol=max(tol, 1e-7), nsample=200, rows=srcs)


def test_lookahead_16384_matches_serial(dev):
    """n = 16384 float32 with the path matrix, 64 x 64 tiles: the lookahead (two
    streams), pairs (two rounds fused) and pairs-with-lookahead schedules give bit
    for bit the serial schedule's D and P, and the sampled rows match the float64
    Dijkstra oracle within the float32 tolerance."""
    import paper_2105_07298_amd as fw
    n = 16384
    W = workloads.unit_complete(n, dtype=np.float32, seed=2)
    res = {}
    for sch in (fw.FW_SCHED_SERIAL, fw.FW_SCHED_LOOKAHEAD, fw.FW_SCHED_PAIRS, fw.FW_SCHED_PAIRS_LOOKAHEAD):
        res[sch] = run_gpu(W, dev, block=64, tile=(64, 64), variant=fw.FW_P4_PANELS, schedule=sch,
                           case="schedules")
    for sch in (2, 3, 4):
        np.testing.assert_array_equal(res[1][0], res[sch][0])
        np.testing.assert_array_equal(res[1][1], res[sch][1])
    srcs = workloads.sample_sources(n, 16)
    print("[cpu] dijkstra 16 rows", flush=True)
    Dr, _ = oracle.dijkstra_rows(W, srcs, exact=False)
    assert rel_err(res[2][0][srcs], Dr) <= 1e-5
