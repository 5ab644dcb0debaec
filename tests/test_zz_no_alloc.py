"""fw_apsp_batched_device_noalloc (the entry point for callers that cannot
allocate) against fw_apsp_batched_device, through the C ABI: two calls in a row
on one stream, the second with a smaller batch, each equal bit for bit to the
allocating entry point's result and to the oracle."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _batch(seed, count, nmax):
    rng = np.random.default_rng(seed)
    graphs = [workloads.int_graph(n=int(n), p=float(rng.uniform(0.05, 0.5)), wmax=4, seed=seed * 1000 + i)
              for i, n in enumerate(rng.integers(1, nmax, count))]
    ns = np.array([g.shape[0] for g in graphs], dtype=np.int32)
    off = np.zeros(len(graphs) + 1, dtype=np.int64)
    off[1:] = np.cumsum(ns.astype(np.int64) ** 2)
    return graphs, ns, off, np.concatenate([g.ravel() for g in graphs])


def test_noalloc_matches_allocating_entry_point():
    import torch
    import paper_2105_07298_amd as fw
    assert torch.cuda.is_available()
    L = fw.lib()
    dev = torch.device("cuda:0")
    s = torch.cuda.Stream(dev)
    for call, (seed, count, nmax) in enumerate([(41, 120, 260), (42, 30, 100)]):
        graphs, ns, off, W = _batch(seed, count, nmax)
        with torch.cuda.stream(s):
            n_d = torch.from_numpy(ns).to(dev)
            o_d = torch.from_numpy(off).to(dev)
            results = []
            for name in ("fw_apsp_batched_device_noalloc", "fw_apsp_batched_device"):
                D = torch.from_numpy(W).to(dev)
                P = torch.empty(D.shape, dtype=torch.int32, device=dev)
                print(f"[gpu] call {call}: {name} batch={ns.size}", flush=True)
                st = getattr(L, name)(fw.FW_F32, int(ns.size), n_d.data_ptr(), o_d.data_ptr(), D.data_ptr(),
                                      P.data_ptr(), s.cuda_stream)
                assert st == fw.FW_OK, fw.fw_last_error()
                results.append((D, P))
        s.synchronize()
        (D0, P0), (D1, P1) = [(d.cpu().numpy(), p.cpu().numpy()) for d, p in results]
        np.testing.assert_array_equal(D0, D1)
        np.testing.assert_array_equal(P0, P1)
        for b, g in enumerate(graphs):
            n = g.shape[0]
            Do, Po = oracle.fw(g)
            np.testing.assert_array_equal(D0[off[b]:off[b + 1]].reshape(n, n).astype(np.float64), Do)
            np.testing.assert_array_equal(P0[off[b]:off[b + 1]].reshape(n, n), Po)


def test_noalloc_rejects_batch_above_the_table():
    import paper_2105_07298_amd as fw
    L = fw.lib()
    st = L.fw_apsp_batched_device_noalloc(fw.FW_F32, 262145, 4096, 4096, 4096, None, None)
    assert st == fw.FW_EINVAL and "262144" in fw.fw_last_error()
