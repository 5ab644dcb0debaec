"""Out-of-core distances (fw_apsp_ooc): the matrix stays in pinned host memory and
streams through a device working set sized so that several super-rounds run,
with a ragged last super-block.  Integer weights: bit-exact against the oracle;
real weights: within the float32 / float64 tolerance of the float64 oracle."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def run_ooc(W, S_want):
    import torch
    import paper_2105_07298_amd as fw
    fw.lib()
    dt = fw.FW_F32 if W.dtype == np.float32 else fw.FW_F64
    n = W.shape[0]
    es = W.itemsize
    nb = -(-n // S_want)
    budget = (4 * S_want * S_want + 2 * S_want * nb * S_want) * es
    S = fw.fw_ooc_superblock(dt, n, budget)
    assert S == S_want, (S, S_want)
    H = torch.empty((n, n), dtype=torch.float32 if dt == fw.FW_F32 else torch.float64, pin_memory=True)
    H.copy_(torch.from_numpy(W))
    print(f"[gpu] fw_apsp_ooc n={n} dtype={W.dtype} S={S} budget={budget}", flush=True)
    fw.apsp_ooc_(H, budget)
    return H.numpy().astype(np.float64)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n,S", [(3000, 1024), (1000, 1024), (777, 256)])
def test_ooc_integer_bit_exact(dtype, n, S):
    W = workloads.int_graph(n=n, p=0.3, wmax=100, seed=31 + n, dtype=dtype)
    Dg = run_ooc(W, S)
    Do, _ = oracle.fw(W)
    np.testing.assert_array_equal(Dg, Do)


@pytest.mark.parametrize("dtype,tol", [(np.float32, 1e-5), (np.float64, 1e-12)])
def test_ooc_real_weights(dtype, tol):
    n = 2048
    W = workloads.unit_complete(n, dtype=dtype, seed=5)
    Dg = run_ooc(W, 512)
    Do, _ = oracle.fw(W, exact=False)
    fin = np.isfinite(Do)
    assert np.array_equal(np.isfinite(Dg), fin)
    assert np.max(np.abs(Dg[fin] - Do[fin]) / np.maximum(Do[fin], 1e-300)) <= tol
