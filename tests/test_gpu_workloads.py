"""The device twin of the input generator (workloads/gen_dev.hip) against the host
generator (workloads/gen.c): the same bits for every weight law and element type,
on row ranges that do not start at 0 and on sizes that are not multiples of
anything."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("law,wmax,p", [(workloads.W_INT, 100, 0.1), (workloads.W_INT, 1000, 0.5),
                                        (workloads.W_UNIT_OPEN, 0, 1.0), (workloads.W_ONE_TEN, 0, 0.37),
                                        (workloads.W_ONE_TWO, 0, 0.05)])
def test_device_generator_matches_host(dtype, law, wmax, p):
    import torch
    dev = torch.device("cuda:0")
    n, r0, r1 = 1037, 13, 700
    host = workloads.rows(9, n, r0, r1, p, law, wmax, dtype, g=4)
    out = torch.empty((r1 - r0) * n, dtype=torch.float32 if dtype == np.float32 else torch.float64, device=dev)
    print(f"[gpu] gen_rows_dev law={law} dtype={np.dtype(dtype).name}", flush=True)
    workloads.rows_dev(9, n, r0, r1, p, law, wmax, out, g=4)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(r1 - r0, n)
    assert np.array_equal(got.view(np.uint8), host.view(np.uint8))
