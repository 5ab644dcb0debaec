"""The synthetic input generator: definition, determinism, laws and row regeneration."""
import numpy as np

import workloads

M64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def mix64(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def py_draw(seed, stream, g, i, j):
    base = mix64((seed * GOLDEN + stream) & M64)
    gkey = mix64(base ^ ((g * 0xD1B54A32D192ED03) & M64))
    idx = (i << 32) | j
    return mix64((gkey + (idx + 1) * GOLDEN) & M64)


def test_splitmix64_reference_value():
    # first output of SplitMix64 seeded with 0 (published test value of the generator)
    assert mix64(GOLDEN) == 0xE220A8397B1DCDAF


def test_draw_matches_python_definition():
    rng = np.random.default_rng(0)
    for _ in range(200):
        s, st, g, i, j = (int(x) for x in rng.integers(0, 2**31, 5))
        assert workloads.draw(s, st % 6, g, i, j) == py_draw(s, st % 6, g, i, j)


def test_int_graph_law():
    W = workloads.int_graph(n=512, p=0.5, wmax=1000, seed=1)
    assert W.dtype == np.float32 and W.shape == (512, 512)
    assert np.all(np.diagonal(W) == 0)
    off = ~np.eye(512, dtype=bool)
    fin = np.isfinite(W) & off
    v = W[fin]
    assert v.min() >= 1 and v.max() <= 1000 and np.all(v == np.floor(v))
    assert abs(fin.sum() / off.sum() - 0.5) < 0.01
    # entry-level definition
    for (i, j) in [(0, 1), (3, 400), (511, 0)]:
        h_e = py_draw(1, 0, 0, i, j)
        present = (h_e >> 32) < (1 << 31)
        if present:
            h_w = py_draw(1, 1, 0, i, j)
            assert W[i, j] == 1 + (((h_w >> 32) * 1000) >> 32)
        else:
            assert np.isinf(W[i, j])


def test_unit_open_law_exact():
    for dt, bits in ((np.float32, 23), (np.float64, 52)):
        W = workloads.unit_complete(256, dtype=dt, seed=2)
        off = ~np.eye(256, dtype=bool)
        v = W[off].astype(np.float64)
        assert np.all(v > 0) and np.all(v < 1)
        # every value is (2b + 1) * 2^-(bits+1): odd multiple of the half-ulp grid
        scaled = v * 2.0 ** (bits + 1)
        assert np.all(scaled == np.floor(scaled)) and np.all(scaled % 2 == 1)
        assert v.min() >= 2.0 ** -(bits + 1)


def test_rows_regenerate_slices():
    W = workloads.int_graph(n=300, p=0.1, wmax=100, seed=3)
    part = workloads.rows(3, 300, 100, 137, 0.1, workloads.W_INT, 100)
    np.testing.assert_array_equal(part, W[100:137])


def test_deterministic_and_seed_sensitive():
    a = workloads.unit_complete(64, seed=2)
    b = workloads.unit_complete(64, seed=2)
    c = workloads.unit_complete(64, seed=3)
    np.testing.assert_array_equal(a, b)
    assert not np.array_equal(a, c)


def test_batch_graphs_small():
    ns, off, W = workloads.batch_graphs(batch=50, seed=4)
    assert ns.min() >= 16 and ns.max() <= 512
    assert off[0] == 0 and np.all(np.diff(off) == ns.astype(np.int64) ** 2)
    dens = workloads.batch_densities(50, seed=4)
    assert dens.min() >= 0.1 and dens.max() < 1.0
    g = 7
    Wg = W[off[g]:off[g + 1]].reshape(ns[g], ns[g])
    assert np.all(np.diagonal(Wg) == 0)
    v = Wg[np.isfinite(Wg) & ~np.eye(ns[g], dtype=bool)]
    assert v.min() >= 1 and v.max() <= 10


def test_batch_size_distribution():
    ns = workloads.batch_sizes(10000, seed=4)
    assert ns.min() == 16 and ns.max() == 512
    assert abs(ns.mean() - 264) < 5


def test_grad_graph_law():
    W, G = workloads.grad_graph(n=128, seed=5)
    off = ~np.eye(128, dtype=bool)
    v = W[off]
    assert v.min() >= 1 and v.max() < 2
    assert np.all((v.astype(np.float64) - 1) * 2**23 == np.floor((v.astype(np.float64) - 1) * 2**23))
    assert abs(G.mean()) < 0.05 and abs(G.std() - 1) < 0.05


def test_row_callback_matches_rows():
    """gen_row_cb (the row source of the oracle's on-demand searches) gives the rows
    gen_rows_f32 / gen_rows_f64 give, widened to double."""
    import ctypes
    for dtype in (np.float32, np.float64):
        for law, wmax, p in ((workloads.W_INT, 100, 0.1), (workloads.W_UNIT_OPEN, 0, 1.0),
                             (workloads.W_ONE_TEN, 0, 0.4)):
            n = 301
            W = workloads.rows(7, n, 0, n, p, law, wmax, dtype, g=2)
            spec = workloads.graph_spec(7, n, p, law, wmax, dtype, g=2)
            out = np.empty(n, dtype=np.float64)
            for i in (0, 5, 300):
                workloads._load().gen_row_cb(ctypes.byref(spec), i, out.ctypes.data_as(ctypes.c_void_p))
                assert np.array_equal(out, W[i].astype(np.float64))
