"""GPU parity of the half-width variant (FW_F16): fw_apsp on binary16 distances
against the integer oracle.

Binary16 represents every integer up to 2048 exactly.  With integer weights and
every finite shortest distance below 2048, each length that can be a final
distance or tie with one is an exact sum, so D and the canonical P must equal the
int64 oracle bit for bit; every test checks that precondition on the oracle's D
before comparing.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    import paper_2105_07298_amd as fw
    fw.lib()
    return torch.device("cuda:0")


def f16_configs(n):
    import paper_2105_07298_amd as fw
    out = []
    for b, tm, tn, var in fw.fw_list_configs(fw.FW_F16):
        out.append((b, tm, tn, var, fw.FW_SCHED_SERIAL))
        if fw.lookahead_applies(b, tm, tn, n):
            out.append((b, tm, tn, var, fw.FW_SCHED_LOOKAHEAD))
        if fw.pairs_applies(b, tm, tn, var, n):
            out.append((b, tm, tn, var, fw.FW_SCHED_PAIRS))
        if fw.pairs_lookahead_applies(b, tm, tn, var, n):
            out.append((b, tm, tn, var, fw.FW_SCHED_PAIRS_LOOKAHEAD))
    return out


def run_f16(W32, dev, path=True, block=0, tile=(0, 0), variant=0, schedule=0, case=""):
    """W32: integer-valued float32 weights (+inf = no edge); run in binary16."""
    import torch
    import paper_2105_07298_amd as fw
    W16 = W32.astype(np.float16)
    assert np.array_equal(W16.astype(np.float32), W32), "weights not exact in binary16"
    print(f"[gpu] fw_apsp f16 {case} n={W32.shape[0]} path={path} block={block} tile={tile} variant={variant} "
          f"schedule={schedule}", flush=True)
    D, P = fw.apsp(torch.from_numpy(W16).to(dev), path=path, block=block, tile_m=tile[0], tile_n=tile[1],
                   variant=variant, schedule=schedule)
    torch.cuda.synchronize()
    assert D.dtype == torch.float16
    return D.cpu().numpy().astype(np.float64), (P.cpu().numpy() if P is not None else None)


def oracle_exact(W32):
    Do, Po = oracle.fw(W32, exact=True)
    fin = np.isfinite(Do)
    assert Do[fin].max(initial=0) < 2048, "workload outside the exact binary16 range"
    return Do, Po


@pytest.mark.parametrize("path", [True, False])
def test_f16_c1_bit_exact(dev, path):
    """n = 512, edge probability 0.5, integer weights in [1, 1000]."""
    W = workloads.int_graph(n=512, p=0.5, wmax=1000, seed=1)
    Do, Po = oracle_exact(W)
    Dg, Pg = run_f16(W, dev, path=path, case="C1")
    np.testing.assert_array_equal(Dg, Do)
    if path:
        np.testing.assert_array_equal(Pg, Po)


def test_f16_every_config_tie_heavy(dev):
    """Weights in [1, 3] at low density (many equal-length paths): every compiled
    binary16 configuration gives the oracle's D and canonical P exactly."""
    W = workloads.int_graph(n=448, p=0.02, wmax=3, seed=21)
    Do, Po = oracle_exact(W)
    assert (Po >= 0).mean() > 0.5
    cfgs = f16_configs(W.shape[0])
    assert len(cfgs) >= 4
    for block, tm, tn, var, sch in cfgs:
        Dg, Pg = run_f16(W, dev, block=block, tile=(tm, tn), variant=var, schedule=sch, case="tie-heavy")
        np.testing.assert_array_equal(Dg, Do)
        np.testing.assert_array_equal(Pg, Po)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 63, 65, 127, 129, 200, 333])
def test_f16_ragged_sizes(dev, n):
    W = workloads.int_graph(n=n, p=0.3, wmax=50, seed=100 + n)
    Do, Po = oracle_exact(W)
    Dg, Pg = run_f16(W, dev, case="ragged")
    np.testing.assert_array_equal(Dg, Do)
    np.testing.assert_array_equal(Pg, Po)


def test_f16_path_graph_to_2047(dev):
    """Directed path 0 -> 1 -> ... -> n-1 whose total length is 2047, the largest
    odd integer binary16 holds: D[i][j] is the sum of the weights between i and j
    (closed form), P[i][j] = j - 1 for j >= i + 2, and nothing reaches backwards.
    The sums above 2048 that this graph cannot produce are exactly the ones the
    contract excludes."""
    n = 342
    w = np.full(n - 1, 6.0)  # 341 edges of weight 6 sum to 2046 ...
    w[170] = 7.0             # ... and one of weight 7 makes it 2047
    assert w.sum() == 2047
    W = np.full((n, n), np.inf, dtype=np.float32)
    np.fill_diagonal(W, 0)
    W[np.arange(n - 1), np.arange(1, n)] = w
    Dg, Pg = run_f16(W, dev, case="path-2047")
    csum = np.concatenate([[0.0], np.cumsum(w)])
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    Dc = np.where(j >= i, csum[j] - csum[np.minimum(i, j)], np.inf)
    Pc = np.where(j >= i + 2, j - 1, -1)
    np.testing.assert_array_equal(Dg, Dc)
    np.testing.assert_array_equal(Pg, Pc)
    assert Dg[0, n - 1] == 2047


def test_f16_matches_f32(dev):
    """Same integer graph in binary16 and float32: identical D and P (float32 is
    exact there too), distances only and with the path matrix."""
    import torch
    import paper_2105_07298_amd as fw
    W = workloads.int_graph(n=700, p=0.05, wmax=20, seed=33)
    oracle_exact(W)
    D32, P32 = fw.apsp(torch.from_numpy(W).to(dev), path=True)
    Dg, Pg = run_f16(W, dev, case="vs-f32")
    Dd, _ = run_f16(W, dev, path=False, case="vs-f32 dist")
    np.testing.assert_array_equal(Dg, D32.cpu().numpy().astype(np.float64))
    np.testing.assert_array_equal(Pg, P32.cpu().numpy())
    np.testing.assert_array_equal(Dd, Dg)


def test_f16_16384_sampled_rows(dev):
    """The binary16 bench workload at full size: complete graph, n = 16384,
    integer weights in [1, 1000] (every distance <= 1000): 32 rows bit-exact
    against the oracle's lexicographic Dial rows, D and P."""
    import torch
    import paper_2105_07298_amd as fw
    n = 16384
    print(f"[cpu] generating n={n}", flush=True)
    W = workloads.int_graph(n=n, p=1.0, wmax=1000, seed=2)
    srcs = workloads.sample_sources(n, 32)
    print("[gpu] fw_apsp f16 with path matrix", flush=True)
    D = torch.from_numpy(W.astype(np.float16)).to(dev)
    P = torch.empty((n, n), dtype=torch.int32, device=dev)
    fw.apsp_(D, P)
    idx = torch.from_numpy(srcs).to(dev)
    Dg = D.index_select(0, idx).cpu().numpy().astype(np.float64)
    Pg = P.index_select(0, idx).cpu().numpy()
    del D, P
    torch.cuda.empty_cache()
    print("[cpu] oracle Dial, 32 sources", flush=True)
    Dr, Pr = oracle.dial_rows(W, srcs, 1000)
    assert Dr.max() <= 1000
    np.testing.assert_array_equal(Dg, Dr)
    np.testing.assert_array_equal(Pg, Pr)


def test_f16_rejected_where_unsupported(dev):
    """The batched, backward and out-of-core entry points have no binary16 form:
    FW_EINVAL, nothing launched."""
    import torch
    import paper_2105_07298_amd as fw
    W = torch.zeros(64 * 64, dtype=torch.float16, device=dev)
    with pytest.raises(fw.FwError) as e:
        fw.apsp_batched_(W, [64], [0])
    assert e.value.status == fw.FW_EINVAL
    Wc = torch.zeros((64, 64), dtype=torch.float16)
    with pytest.raises(fw.FwError) as e:
        fw.apsp_ooc_(Wc)
    assert e.value.status == fw.FW_EINVAL
