"""Error paths of the C ABI on the GPU: a call that fails after allocating its
stream-ordered scratch frees it and leaves its stream usable.  The failure is
injected on the host (fw_debug_fail_next): the call returns before launching
anything, so no kernel or device fault is involved."""
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


def test_injected_failure_single_graph(dev):
    """fw_apsp on a ragged n (padded scratch plus path-mode scratch, about 130 MB a
    call): ten injected failures return FW_EHIP and leave no device memory behind;
    the next call on the same stream computes the oracle's D and P."""
    import torch
    import paper_2105_07298_amd as fw
    n = 3000
    W = workloads.int_graph(n=n, p=0.01, wmax=50, seed=31)
    s = torch.cuda.Stream(dev)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(dev)[0]
    with torch.cuda.stream(s):
        for _ in range(10):
            fw.lib().fw_debug_fail_next(1)
            print("[gpu] fw_apsp with an injected failure", flush=True)
            with pytest.raises(fw.FwError) as ei:
                fw.apsp(torch.from_numpy(W).to(dev), path=True)
            assert ei.value.status == fw.FW_EHIP and "injected" in str(ei.value)
        s.synchronize()
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info(dev)[0]
        assert free1 > free0 - (600 << 20), (free0, free1)  # ten leaked calls would hold 1.3 GB
        print("[gpu] fw_apsp after the failures, same stream", flush=True)
        D, P = fw.apsp(torch.from_numpy(W).to(dev), path=True)
    s.synchronize()
    Do, Po = oracle.fw(W)
    np.testing.assert_array_equal(D.cpu().numpy().astype(np.float64), Do)
    np.testing.assert_array_equal(P.cpu().numpy(), Po)


def test_injected_failure_batched(dev):
    """fw_apsp_batched fails after its job table allocation; the next batched call
    on the same stream is correct."""
    import torch
    import paper_2105_07298_amd as fw
    rng = np.random.default_rng(32)
    graphs = [workloads.int_graph(n=int(n), p=0.2, wmax=5, seed=1000 + i) for i, n in enumerate(rng.integers(2, 90, 50))]
    ns = np.array([g.shape[0] for g in graphs], dtype=np.int32)
    off = np.zeros(len(graphs) + 1, dtype=np.int64)
    off[1:] = np.cumsum(ns.astype(np.int64) ** 2)
    W = np.concatenate([g.ravel() for g in graphs])
    s = torch.cuda.Stream(dev)
    with torch.cuda.stream(s):
        fw.lib().fw_debug_fail_next(2)
        print("[gpu] fw_apsp_batched with an injected failure", flush=True)
        with pytest.raises(fw.FwError) as ei:
            fw.apsp_batched(torch.from_numpy(W).to(dev), ns, off[:-1], path=True)
        assert ei.value.status == fw.FW_EHIP
        print("[gpu] fw_apsp_batched after the failure, same stream", flush=True)
        D, P = fw.apsp_batched(torch.from_numpy(W).to(dev), ns, off[:-1], path=True)
    s.synchronize()
    D, P = D.cpu().numpy(), P.cpu().numpy()
    for b, g in enumerate(graphs):
        n = g.shape[0]
        Do, Po = oracle.fw(g)
        np.testing.assert_array_equal(D[off[b]:off[b + 1]].reshape(n, n).astype(np.float64), Do)
        np.testing.assert_array_equal(P[off[b]:off[b + 1]].reshape(n, n), Po)


def test_fail_next_cleared_by_zero(dev):
    import torch
    import paper_2105_07298_amd as fw
    fw.lib().fw_debug_fail_next(1)
    fw.lib().fw_debug_fail_next(0)
    W = workloads.int_graph(n=70, p=0.3, wmax=9, seed=33)
    D, P = fw.apsp(torch.from_numpy(W).to(dev), path=True)
    torch.cuda.synchronize()
    Do, Po = oracle.fw(W)
    np.testing.assert_array_equal(D.cpu().numpy().astype(np.float64), Do)
    np.testing.assert_array_equal(P.cpu().numpy(), Po)


@pytest.mark.parametrize("dtype", [np.float32, np.float64, np.float16])
def test_validate_input(dev, dtype):
    """fw_validate_input accepts a matrix inside the contract (including +inf and -0.0
    off the diagonal) and names the first entry of one that is not: a non-zero
    diagonal entry, a NaN, a negative weight."""
    import torch
    import paper_2105_07298_amd as fw
    n = 300
    W = workloads.int_graph(n=n, p=0.3, wmax=9, seed=34).astype(dtype)
    W[5, 7] = -0.0
    print(f"[gpu] fw_validate_input {np.dtype(dtype).name}", flush=True)
    fw.validate(torch.from_numpy(W).to(dev))
    for (i, j, v, what) in ((17, 17, 1.0, "diagonal"), (200, 3, np.nan, "NaN"), (41, 250, -2.0, "negative")):
        Wb = W.copy()
        Wb[i, j] = v
        Wb[290, 1] = -5.0  # a later offence: the first one in row-major order is reported
        with pytest.raises(fw.FwError) as ei:
            fw.validate(torch.from_numpy(Wb).to(dev))
        assert ei.value.status == fw.FW_EINPUT
        assert f"({i}, {j})" in str(ei.value) and what in str(ei.value), str(ei.value)
