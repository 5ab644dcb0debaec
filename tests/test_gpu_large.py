"""Large single graph at its full size: n = 65536, edge probability 0.1, integer
weights in [1, 100] (every sum below 2^24, so float32 is exact).  The GPU result
(distances and path matrix) must equal, bit for bit, 64 rows computed by the
oracle's lexicographic Dial (bucket-queue Dijkstra) from seeded sources.  About 17 GB (float32) /
34 GB (float64) of distances on the device, plus the path matrix."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_c3_n65536_sampled_rows_bit_exact(dtype):
    import torch
    import paper_2105_07298_amd as fw
    fw.lib()
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    n = 65536
    print(f"[cpu] generating n={n} {np.dtype(dtype).name}", flush=True)
    W = workloads.int_graph(n=n, p=0.1, wmax=100, seed=3, dtype=dtype)
    srcs = workloads.sample_sources(n, 64)
    print("[gpu] fw_apsp with path matrix", flush=True)
    D = torch.from_numpy(W).to(dev)
    P = torch.empty((n, n), dtype=torch.int32, device=dev)
    fw.apsp_(D, P)
    idx = torch.from_numpy(srcs).to(dev)
    Dg = D.index_select(0, idx).cpu().numpy().astype(np.float64)
    Pg = P.index_select(0, idx).cpu().numpy()
    del D, P
    torch.cuda.empty_cache()
    print("[cpu] oracle Dial, 64 sources", flush=True)
    Dr, Pr = oracle.dial_rows(W, srcs, 100)
    np.testing.assert_array_equal(Dg, Dr)
    np.testing.assert_array_equal(Pg, Pr)
    assert np.isfinite(Dr).mean() > 0.99 and (Pr >= 0).mean() > 0.5
