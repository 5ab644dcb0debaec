"""Large single graph at its full size: n = 65536, edge probability 0.1, integer
weights in [1, 100] (every sum below 2^24, so float32 is exact).  The GPU result
(distances and path matrix) must equal, bit for bit, 64 rows computed by the
oracle's lexicographic Dial (bucket-queue Dijkstra) from seeded sources.  About
17 GB (float32) / 34 GB (float64) of distances on the device, plus the path
matrix.  The matrix never exists in host memory: the device twin of the input
generator writes it straight into device memory, and the oracle regenerates each
row it needs with the host generator (the two produce the same bits; see
tests/test_gpu_workloads.py)."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_c3_n65536_sampled_rows_bit_exact(dtype):
    import torch
    import paper_2105_07298_amd as fw
    fw.lib()
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    n = 65536
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    print(f"[gpu] generating n={n} {np.dtype(dtype).name} on the device", flush=True)
    D = torch.empty((n, n), dtype=tdt, device=dev)
    workloads.rows_dev(3, n, 0, n, 0.1, workloads.W_INT, 100, D)
    srcs = workloads.sample_sources(n, 64)
    print("[gpu] fw_apsp with path matrix", flush=True)
    P = torch.empty((n, n), dtype=torch.int32, device=dev)
    fw.apsp_(D, P)
    idx = torch.from_numpy(srcs).to(dev)
    Dg = D.index_select(0, idx).cpu().numpy().astype(np.float64)
    Pg = P.index_select(0, idx).cpu().numpy()
    del D, P
    torch.cuda.empty_cache()
    print("[cpu] oracle Dial, 64 sources, rows regenerated on demand", flush=True)
    spec = workloads.graph_spec(3, n, 0.1, workloads.W_INT, 100, dtype)
    Dr, Pr = oracle.dial_rows_generated(spec, workloads.row_fn(), srcs, 100)
    np.testing.assert_array_equal(Dg, Dr)
    np.testing.assert_array_equal(Pg, Pr)
    assert np.isfinite(Dr).mean() > 0.99 and (Pr >= 0).mean() > 0.5
