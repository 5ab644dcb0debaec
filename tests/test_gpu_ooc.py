"""Out-of-core APSP (fw_apsp_ooc): the matrix stays in pinned host memory and
streams through a device working set sized so that 1, 2, 3 or 4 super-rounds run
(with two, the next super-round's bands are the lookahead's diagonal tile plus the
two tiles copied over on the device), with a ragged last super-block.  The host
path array is left uninitialised: it is output only.  Integer weights: D and P
bit-exact against the oracle; real weights: D within the float32 / float64
tolerance of the float64 oracle, and P satisfies the oracle's invariants."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def run_ooc(W, S_want, path):
    import torch
    import paper_2105_07298_amd as fw
    fw.lib()
    dt = fw.FW_F32 if W.dtype == np.float32 else fw.FW_F64
    n = W.shape[0]
    es = W.itemsize
    nb = -(-n // S_want)
    blocks = 4 * S_want * S_want + 4 * S_want * nb * S_want
    budget = blocks * es + ((blocks + S_want * S_want) * 4 if path else 0)
    S = fw.fw_ooc_superblock(dt, n, path, budget)
    assert S == S_want, (S, S_want)
    H = torch.empty((n, n), dtype=torch.float32 if dt == fw.FW_F32 else torch.float64, pin_memory=True)
    H.copy_(torch.from_numpy(W))
    HP = torch.empty((n, n), dtype=torch.int32, pin_memory=True) if path else None
    print(f"[gpu] fw_apsp_ooc n={n} dtype={W.dtype} path={path} S={S} budget={budget}", flush=True)
    fw.apsp_ooc_(H, HP, budget)
    return H.numpy().astype(np.float64), (HP.numpy().copy() if path else None)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n,S", [(3000, 1024), (1500, 1024), (1000, 1024), (777, 256)])
@pytest.mark.parametrize("path", [False, True])
def test_ooc_integer_bit_exact(dtype, n, S, path):
    W = workloads.int_graph(n=n, p=0.3, wmax=100, seed=31 + n, dtype=dtype)
    Dg, Pg = run_ooc(W, S, path)
    Do, Po = oracle.fw(W)
    np.testing.assert_array_equal(Dg, Do)
    if path:
        np.testing.assert_array_equal(Pg, Po)


def test_ooc_tie_heavy_path():
    """Weights in [1, 3] at low density: many equal-length paths, so P depends on
    the tie rule in every product."""
    W = workloads.int_graph(n=1300, p=0.02, wmax=3, seed=21, dtype=np.float32)
    Dg, Pg = run_ooc(W, 512, True)
    Do, Po = oracle.fw(W)
    assert (Po >= 0).mean() > 0.5
    np.testing.assert_array_equal(Dg, Do)
    np.testing.assert_array_equal(Pg, Po)


@pytest.mark.parametrize("dtype,tol", [(np.float32, 1e-5), (np.float64, 1e-12)])
def test_ooc_real_weights(dtype, tol):
    n = 2048
    W = workloads.unit_complete(n, dtype=dtype, seed=5)
    Dg, Pg = run_ooc(W, 512, True)
    Do, _ = oracle.fw(W, exact=False)
    fin = np.isfinite(Do)
    assert np.array_equal(np.isfinite(Dg), fin)
    assert np.max(np.abs(Dg[fin] - Do[fin]) / np.maximum(Do[fin], 1e-300)) <= tol
    oracle.check_invariants(W, Dg, Pg, exact=False, rtol=max(tol, 1e-7), nsample=1000)
