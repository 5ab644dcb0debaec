"""Seeded synthetic inputs for the shortest-path workloads.

Holds no shortest-path arithmetic: it only draws weight matrices (and upstream
gradients) from a counter-based SplitMix64 generator (see gen.c for the exact
definition), so the CPU oracle and the GPU library always receive the same bits.

Workloads (sizes and laws of the paper-shaped runs, Sect. 4.1: dense N x N
matrices, N in {4096 .. 65536}, float and double):
  int_graph     directed graph, edge i->j present with probability p, integer
                weight uniform in [1, wmax] (exact in float32 while sums < 2^24)
  unit_complete complete graph, weights uniform real strictly inside (0, 1)
  batch_graphs  many graphs of uneven size and density, weights in [1, 10]
  grad_graph    complete graph with weights in [1, 2) plus N(0,1) upstream dL/dD
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libfwgen.so")
_lib = None

W_INT, W_UNIT_OPEN, W_ONE_TEN, W_ONE_TWO = 0, 1, 2, 3


_DEV_SRC = os.path.join(_HERE, "gen_dev.hip")
_DEV_LIB = os.path.join(_HERE, "libfwgen_dev.so")
_dev_lib = None


class GraphSpec(ctypes.Structure):
    """The graph description gen_row_cb reads (gen.c's gen_graph_t)."""
    _fields_ = [("seed", ctypes.c_uint64), ("g", ctypes.c_uint64), ("n", ctypes.c_int64),
                ("thresh32", ctypes.c_uint64), ("law", ctypes.c_int32), ("is_f64", ctypes.c_int32),
                ("wmax", ctypes.c_int64)]


def build(out: str = _LIB) -> str:
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall",
                    "-o", out, _SRC, "-lm"], check=True)
    return out


def build_dev(out: str = _DEV_LIB) -> str:
    """The device twin (hipcc, gfx950), contraction off so weights round as on the host."""
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-o", out, _DEV_SRC], check=True)
    return out


def _load_dev():
    global _dev_lib
    if _dev_lib is None:
        if not os.path.exists(_DEV_LIB):
            raise ImportError(f"{_DEV_LIB} is missing: build it with workloads.build_dev()")
        lib = ctypes.CDLL(_DEV_LIB)
        lib.gen_rows_dev.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_uint64, ctypes.c_int, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                     ctypes.c_void_p]
        lib.gen_rows_dev.restype = ctypes.c_int
        _dev_lib = lib
    return _dev_lib


def rows_dev(seed: int, n: int, r0: int, r1: int, p: float, law: int, wmax: int, out, g: int = 0,
             stream: int | None = None):
    """rows() generated on the GPU straight into the device tensor out ((r1 - r0) * n
    float32/float64 elements, contiguous), on the given stream (default: the current one)."""
    import torch
    assert out.is_cuda and out.is_contiguous() and out.numel() == (r1 - r0) * n
    assert out.dtype in (torch.float32, torch.float64)
    if stream is None:
        stream = torch.cuda.current_stream(out.device).cuda_stream
    rc = _load_dev().gen_rows_dev(seed, g, n, r0, r1, threshold(p), law, wmax, int(out.dtype == torch.float64),
                                  out.data_ptr(), stream)
    if rc != 0:
        raise RuntimeError(f"gen_rows_dev launch failed ({rc})")
    return out


def graph_spec(seed, n, p, law, wmax=0, dtype=np.float32, g=0) -> GraphSpec:
    """The description of graph(seed, n, p, law, wmax, dtype, g) that gen_row_cb
    regenerates rows from."""
    return GraphSpec(seed, g, n, threshold(p), law, int(np.dtype(dtype) == np.float64), wmax)


def row_fn():
    """Address of gen_row_cb (for C code that reads rows on demand)."""
    return ctypes.cast(_load().gen_row_cb, ctypes.c_void_p).value


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    u64, i64, vp = ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p
    lib.gen_gkey.argtypes = [u64, u64, u64]
    lib.gen_gkey.restype = u64
    lib.gen_draw.argtypes = [u64, u64, u64, u64, u64]
    lib.gen_draw.restype = u64
    lib.gen_rows_f32.argtypes = [u64, u64, i64, i64, i64, u64, ctypes.c_int, i64, vp]
    lib.gen_rows_f64.argtypes = [u64, u64, i64, i64, i64, u64, ctypes.c_int, i64, vp]
    lib.gen_normal_f32.argtypes = [u64, u64, i64, vp]
    lib.gen_graph_n.argtypes = [u64, u64, i64, i64]
    lib.gen_graph_n.restype = i64
    lib.gen_graph_density.argtypes = [u64, u64, ctypes.c_double, ctypes.c_double]
    lib.gen_graph_density.restype = ctypes.c_double
    lib.gen_row_cb.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    lib.gen_row_cb.restype = None
    _lib = lib
    return lib


def threshold(p: float) -> int:
    """Edge-presence threshold floor(p * 2^32) (2^32 = always present)."""
    return min(int(np.floor(p * 2.0**32)), 2**32)


def draw(seed, stream, g, i, j) -> int:
    return int(_load().gen_draw(seed, stream, g, i, j))


def rows(seed: int, n: int, r0: int, r1: int, p: float, law: int, wmax: int = 0,
         dtype=np.float32, g: int = 0, out: np.ndarray | None = None) -> np.ndarray:
    """Rows [r0, r1) of graph g: (r1 - r0) x n, diagonal 0, missing edges +inf."""
    lib = _load()
    dtype = np.dtype(dtype)
    if out is None:
        out = np.empty((r1 - r0, n), dtype=dtype)
    assert out.dtype == dtype and out.flags["C_CONTIGUOUS"] and out.size == (r1 - r0) * n
    fn = lib.gen_rows_f32 if dtype == np.float32 else lib.gen_rows_f64
    fn(seed, g, n, r0, r1, threshold(p), law, wmax, out.ctypes.data_as(ctypes.c_void_p))
    return out


def graph(seed, n, p, law, wmax=0, dtype=np.float32, g=0, out=None):
    return rows(seed, n, 0, n, p, law, wmax, dtype, g, out)


# ---- named workloads -------------------------------------------------------

def int_graph(n=512, p=0.5, wmax=1000, seed=1, dtype=np.float32, g=0):
    """Directed graph, edges with probability p, integer weights in [1, wmax]."""
    return graph(seed, n, p, W_INT, wmax, dtype, g)


def unit_complete(n, dtype=np.float32, seed=2, g=0):
    """Complete directed graph, weights (2b+1)*2^-(B+1) strictly inside (0, 1)."""
    return graph(seed, n, 1.0, W_UNIT_OPEN, 0, dtype, g)


def batch_sizes(batch=10000, lo=16, hi=512, seed=4):
    lib = _load()
    return np.array([lib.gen_graph_n(seed, g, lo, hi) for g in range(batch)], dtype=np.int32)


def batch_densities(batch=10000, lo=0.1, hi=1.0, seed=4):
    lib = _load()
    return np.array([lib.gen_graph_density(seed, g, lo, hi) for g in range(batch)], dtype=np.float64)


def batch_graphs(batch=10000, lo=16, hi=512, seed=4, dtype=np.float32):
    """Ragged batch: (n[batch] int32, offset[batch+1] int64, W concatenated row-major).

    Graph g has n_g ~ U{lo..hi} vertices, density ~ U[0.1, 1.0), weights
    1 + 9 u (u strictly inside (0,1)) rounded once to float32.
    """
    ns = batch_sizes(batch, lo, hi, seed)
    dens = batch_densities(batch, 0.1, 1.0, seed)
    off = np.zeros(batch + 1, dtype=np.int64)
    off[1:] = np.cumsum(ns.astype(np.int64) ** 2)
    W = np.empty(int(off[-1]), dtype=dtype)
    for g in range(batch):
        n = int(ns[g])
        rows(seed, n, 0, n, float(dens[g]), W_ONE_TEN, 0, dtype, g,
             out=W[off[g]:off[g + 1]].reshape(n, n))
    return ns, off, W


def grad_graph(n=2048, seed=5, g=0, p=1.0):
    """Graph with weights in [1, 2) (exact float32) and N(0,1) upstream gradient G."""
    W = graph(seed, n, p, W_ONE_TWO, 0, np.float32, g)
    G = np.empty((n, n), dtype=np.float32)
    _load().gen_normal_f32(seed, g, n, G.ctypes.data_as(ctypes.c_void_p))
    return W, G


def sample_sources(n, count=64, seed=64):
    """count distinct source vertices, seeded."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(count, n), replace=False)).astype(np.int64)
