"""CPU oracle for all-pairs shortest paths -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The HIP library never imports, links or
calls it, and it imports nothing from the HIP library: the two share no code.

Contents
  fw(W)                 classic Floyd-Warshall (paper Sect. 2.2, Algorithm 1,
                        strict update test), int64 when every finite weight is an
                        integer, else float64.  Returns (D, P).
  dijkstra_rows(W, src) per-source Dijkstra with lexicographic labels
                        (length, largest interior vertex): rows of D and of the
                        canonical P without the cubic loop.
  dial_rows(W, src, C)  the same labels by Dial's bucket queue, for integer
                        weights in [1, C] (large sparse-ish graphs);
                        dial_rows_generated reads each row through a callback
                        instead (the matrix never exists in host memory).
  brute_force(W)        enumeration of every simple path, n <= 8: the definition
                        of (D, P) written out.
  backward_pathwalk     dL/dW from dL/dD by walking each pair's shortest path.
  reconstruct(P, i, j)  vertex list of the path P encodes.
  path_sums(W, P)       every pair's encoded path walked and summed (the checker's
                        all-pairs pass).
  check_invariants      D[i][i] = 0, D <= W, triangle inequality, P never names
                        an endpoint, and on every pair the encoded path exists,
                        splits at P[i][j] and sums to D (exactly and canonically
                        for integer weights, within rtol for real weights).

Parity status of each function and the pins that fix it are listed in the design doc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

I64_INF = np.iinfo(np.int64).max


def build(src: str = _SRC, out: str = _LIB) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall", "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


def load(path: str = _LIB):
    """Load a compiled oracle library (default: the in-tree one, building it if absent)."""
    global _lib
    if path == _LIB and _lib is not None:
        return _lib
    if not os.path.exists(path):
        if path != _LIB:
            raise FileNotFoundError(path)
        build()
    lib = ctypes.CDLL(path)
    i64, i32p, vp = ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.c_void_p
    lib.oracle_fw_f64.argtypes = [i64, vp, vp, ctypes.c_int]
    lib.oracle_fw_i64.argtypes = [i64, vp, vp, ctypes.c_int]
    lib.oracle_fw_f64_steps.argtypes = [i64, vp, vp, i64, i64, ctypes.c_int]
    lib.oracle_dijkstra_rows_f64.argtypes = [i64, vp, i64, vp, vp, vp, ctypes.c_int]
    lib.oracle_dijkstra_rows_i64.argtypes = [i64, vp, i64, vp, vp, vp, ctypes.c_int]
    lib.oracle_dijkstra_rows_floatint.argtypes = [i64, vp, ctypes.c_int, i64, vp, vp, vp, ctypes.c_int]
    lib.oracle_dial_rows.argtypes = [i64, vp, ctypes.c_int, i64, i64, vp, vp, vp, ctypes.c_int]
    lib.oracle_dial_rows_fn.argtypes = [i64, vp, vp, i64, i64, vp, vp, vp, ctypes.c_int]
    lib.oracle_backward_pathwalk_f64.argtypes = [i64, vp, vp, vp, vp]
    lib.oracle_backward_pathwalk_f64.restype = ctypes.c_int
    lib.oracle_reconstruct.argtypes = [i64, vp, i64, i64, vp, i64]
    lib.oracle_reconstruct.restype = i64
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_path_sums_rows_f64.argtypes = [i64, vp, vp, i64, vp, vp, vp, ctypes.c_int]
    lib.oracle_triangle_violations_rows.argtypes = [i64, vp, i64, vp, vp, i64, ctypes.c_double, ctypes.c_int]
    lib.oracle_triangle_violations_rows.restype = i64
    if path == _LIB:
        _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def is_integer_valued(W: np.ndarray) -> bool:
    """True when every finite entry of W is an integer small enough for int64 sums."""
    W = np.asarray(W)
    if W.dtype.kind in "iu":
        return True
    fin = np.isfinite(W)
    v = W[fin]
    return bool(np.all(v == np.floor(v)) and (v.size == 0 or np.abs(v).max() < 2.0**52))


def to_i64(W: np.ndarray) -> np.ndarray:
    """Integer-valued weights (+inf = no edge) -> int64 with the oracle's sentinel."""
    W = np.asarray(W)
    if W.dtype.kind in "iu":
        return np.ascontiguousarray(W, dtype=np.int64)
    out = np.full(W.shape, I64_INF, dtype=np.int64)
    fin = np.isfinite(W)
    out[fin] = W[fin].astype(np.int64)
    return out


def from_i64(D: np.ndarray) -> np.ndarray:
    """int64 distances (sentinel = unreachable) -> float64 with +inf."""
    out = D.astype(np.float64)
    out[D == I64_INF] = np.inf
    return out


def _check_input(W: np.ndarray):
    W = np.asarray(W)
    if W.ndim != 2 or W.shape[0] != W.shape[1]:
        raise ValueError("W must be square")
    if W.dtype.kind == "f" and np.isnan(W).any():
        raise ValueError("W contains NaN")
    d = np.diagonal(W)
    if not np.all(d == 0):
        raise ValueError("oracle input contract: W[i][i] must be 0")


def fw(W: np.ndarray, exact: bool | None = None, threads: int = 0):
    """Classic Floyd-Warshall of W -> (D, P).

    exact=True forces the int64 loop (W must be integer-valued), exact=False the
    float64 loop; None picks int64 when W is integer-valued.  D comes back as
    float64 with +inf for unreachable pairs in both cases; P as int32 (-1 = none).
    """
    _check_input(W)
    lib = load()
    n = W.shape[0]
    if exact is None:
        exact = is_integer_valued(W)
    P = np.empty((n, n), dtype=np.int32)
    if exact:
        D = to_i64(W).copy()
        lib.oracle_fw_i64(n, _ptr(D), _ptr(P), threads)
        return from_i64(D), P
    D = np.ascontiguousarray(W, dtype=np.float64).copy()
    lib.oracle_fw_f64(n, _ptr(D), _ptr(P), threads)
    return D, P


def fw_steps(D: np.ndarray, P: np.ndarray, k_begin: int, k_end: int, threads: int = 0):
    """Run outer iterations [k_begin, k_end) of the float64 classic loop in place
    (D float64, P int32, both C-contiguous; P set to -1 before the first call)."""
    lib = load()
    assert D.dtype == np.float64 and P.dtype == np.int32
    lib.oracle_fw_f64_steps(D.shape[0], _ptr(D), _ptr(P), k_begin, k_end, threads)


def max_threads() -> int:
    return int(load().oracle_max_threads())


def dijkstra_rows(W: np.ndarray, srcs, exact: bool | None = None, threads: int = 0):
    """Rows srcs of (D, P) by lexicographic Dijkstra. Returns (Drows float64, Prows int32)."""
    _check_input(W)
    lib = load()
    n = W.shape[0]
    srcs = np.ascontiguousarray(np.asarray(srcs, dtype=np.int64))
    if exact is None:
        exact = is_integer_valued(W)
    P = np.empty((srcs.size, n), dtype=np.int32)
    if exact:
        Wi = to_i64(W)
        D = np.empty((srcs.size, n), dtype=np.int64)
        lib.oracle_dijkstra_rows_i64(n, _ptr(Wi), srcs.size, _ptr(srcs), _ptr(D), _ptr(P), threads)
        return from_i64(D), P
    Wd = np.ascontiguousarray(W, dtype=np.float64)
    D = np.empty((srcs.size, n), dtype=np.float64)
    lib.oracle_dijkstra_rows_f64(n, _ptr(Wd), srcs.size, _ptr(srcs), _ptr(D), _ptr(P), threads)
    return D, P


def dijkstra_rows_integer_float(W: np.ndarray, srcs, threads: int = 0):
    """dijkstra_rows for integer-valued weights held as float32/float64 (+inf = no
    edge), converting each weight exactly to int64 as it is read (no int64 copy of W;
    the caller guarantees W is integer-valued, diagonal 0).  Returns (Drows float64,
    Prows int32)."""
    lib = load()
    W = np.ascontiguousarray(W)
    assert W.dtype in (np.float32, np.float64) and W.ndim == 2 and W.shape[0] == W.shape[1]
    n = W.shape[0]
    srcs = np.ascontiguousarray(np.asarray(srcs, dtype=np.int64))
    D = np.empty((srcs.size, n), dtype=np.int64)
    P = np.empty((srcs.size, n), dtype=np.int32)
    lib.oracle_dijkstra_rows_floatint(n, _ptr(W), int(W.dtype == np.float64), srcs.size, _ptr(srcs),
                                      _ptr(D), _ptr(P), threads)
    return from_i64(D), P


def dial_rows(W: np.ndarray, srcs, wmax: int, threads: int = 0):
    """Rows srcs of (D, P) for positive integer weights in [1, wmax] held as
    float32/float64 (+inf = no edge), by Dial's bucket-queue Dijkstra with the same
    lexicographic labels.  Returns (Drows float64, Prows int32)."""
    lib = load()
    W = np.ascontiguousarray(W)
    assert W.dtype in (np.float32, np.float64) and W.ndim == 2 and W.shape[0] == W.shape[1]
    n = W.shape[0]
    srcs = np.ascontiguousarray(np.asarray(srcs, dtype=np.int64))
    D = np.empty((srcs.size, n), dtype=np.int64)
    P = np.empty((srcs.size, n), dtype=np.int32)
    lib.oracle_dial_rows(n, _ptr(W), int(W.dtype == np.float64), int(wmax), srcs.size, _ptr(srcs), _ptr(D),
                         _ptr(P), threads)
    return from_i64(D), P


def dial_rows_generated(spec, rowfn: int, srcs, wmax: int, threads: int = 0):
    """dial_rows for a graph whose weight matrix is never held in host memory: rows
    are regenerated on demand by the C function at address rowfn, called as
    rowfn(&spec, u, out) to fill row u (n doubles, +inf = no edge); spec is a
    ctypes structure the function understands (the input generator's graph
    description).  Integer weights in [1, wmax].  Returns (Drows float64, Prows int32)."""
    lib = load()
    n = int(spec.n)
    srcs = np.ascontiguousarray(np.asarray(srcs, dtype=np.int64))
    D = np.empty((srcs.size, n), dtype=np.int64)
    P = np.empty((srcs.size, n), dtype=np.int32)
    lib.oracle_dial_rows_fn(n, ctypes.c_void_p(rowfn), ctypes.byref(spec), int(wmax), srcs.size, _ptr(srcs),
                            _ptr(D), _ptr(P), threads)
    return from_i64(D), P


def backward_pathwalk(D: np.ndarray, P: np.ndarray, G: np.ndarray) -> np.ndarray:
    """dL/dW (float64) given forward (D, P) and G = dL/dD, by walking every encoded path."""
    lib = load()
    n = D.shape[0]
    Dd = np.ascontiguousarray(D, dtype=np.float64)
    Pc = np.ascontiguousarray(P, dtype=np.int32)
    Gd = np.ascontiguousarray(G, dtype=np.float64)
    gW = np.empty((n, n), dtype=np.float64)
    rc = lib.oracle_backward_pathwalk_f64(n, _ptr(Dd), _ptr(Pc), _ptr(Gd), _ptr(gW))
    if rc != 0:
        raise ValueError("P is not a valid path encoding")
    return gW


def reconstruct(P: np.ndarray, i: int, j: int):
    """Vertex list i .. j of the path P encodes (None if the encoding is invalid)."""
    lib = load()
    n = P.shape[0]
    Pc = np.ascontiguousarray(P, dtype=np.int32)
    out = np.empty(n + 1, dtype=np.int64)
    m = lib.oracle_reconstruct(n, _ptr(Pc), i, j, _ptr(out), n + 1)
    if m < 0:
        return None
    return out[:m].tolist()


def brute_force(W: np.ndarray):
    """Definition of (D, P) by exhaustive search over simple paths (n <= 8).

    D[i][j] = smallest total weight over all simple i->j paths (0 for i == j,
    +inf if none); P[i][j] = smallest "largest interior vertex" among the paths
    that attain D[i][j], -1 when i == j, when there is no path, or when the
    direct edge attains it (a path with no interior vertex).  Path length is
    summed left to right in float64 (exact for integer weights).
    """
    W = np.asarray(W, dtype=np.float64)
    n = W.shape[0]
    if n > 8:
        raise ValueError("brute force is limited to n <= 8")
    D = np.full((n, n), np.inf)
    P = np.full((n, n), -1, dtype=np.int32)
    for i in range(n):
        D[i, i] = 0.0
        best = {}
        stack = [(i, 0.0, -1, (i,))]
        while stack:
            v, length, maxint, path = stack.pop()
            for w in range(n):
                if w in path or not np.isfinite(W[v, w]):
                    continue
                L = length + W[v, w]
                key = (L, maxint)  # interior vertices of path+w are path[1:]
                if w not in best or key < best[w]:
                    best[w] = key
                stack.append((w, L, max(maxint, w), path + (w,)))
        for j, (L, m) in best.items():
            if j != i:
                D[i, j] = L
                P[i, j] = m
    return D, P


def path_sums(W: np.ndarray, P: np.ndarray, rows=None, threads: int = 0):
    """Walk the encoded paths of the given source rows (default: all): (S, H) with
    S[q][j] the sum of W along the path of (rows[q], j) (float64, path order) and
    H[q][j] its edge count, H = -1 where P encodes no path (endpoint or
    out-of-range label, cycle, more than n - 1 edges)."""
    lib = load()
    n = W.shape[0]
    Wd = np.ascontiguousarray(W, dtype=np.float64)
    Pc = np.ascontiguousarray(P, dtype=np.int32)
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    S = np.empty((rows.size, n), dtype=np.float64)
    H = np.empty((rows.size, n), dtype=np.int64)
    lib.oracle_path_sums_rows_f64(n, _ptr(Wd), _ptr(Pc), rows.size, _ptr(rows), _ptr(S), _ptr(H), threads)
    return S, H


def triangle_violations(D: np.ndarray, ks, rtol: float = 0.0, rows=None, threads: int = 0) -> int:
    """Number of (i, j, k), i in rows (default all), k in ks, with
    D[i][j] > (D[i][k] + D[k][j]) (1 + rtol)."""
    lib = load()
    Dd = np.ascontiguousarray(D, dtype=np.float64)
    n = Dd.shape[0]
    ks = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    return int(lib.oracle_triangle_violations_rows(n, _ptr(Dd), rows.size, _ptr(rows), _ptr(ks), ks.size,
                                                   float(rtol), threads))


def check_invariants(W, D, P, exact: bool, sample=None, rtol: float = 0.0, nsample: int = 2000,
                     seed: int = 0, rows=None):
    """Assert the properties every correct (D, P) has; raises AssertionError on the first failure.

    What (D, P) must be follows from Sect. 2.2 (Algorithm 1): D[i][j] the length
    of a shortest i->j path, P[i][j] an intermediate vertex of one, -1 for the
    direct edge or no path (readings R1-R2).

    Checked on every pair (i, j) with i in `rows` (default: every row): D[i][i] =
    0, P[i][i] = -1, D <= W, the triangle inequality D[i][j] <= D[i][k] + D[k][j]
    (every k for n <= 2048, else 64 sampled k), P in [-1, n), P[i][j] never i or j,
    P = -1 on unreachable pairs, and the path P encodes for (i, j) exists (no
    cycle, at most n - 1 edges, only existing edges) and its weights add up to
    D[i][j].

    exact (integer weights): that sum equals D[i][j] exactly; P[i][j] = -1 means
    D[i][j] = W[i][j], and P[i][j] = k >= 0 means D[i][j] = D[i][k] + D[k][j] with
    P[i][k] < k and P[k][j] < k.  By induction on k these make P the canonical
    path matrix (its k is the largest interior vertex of the encoded path).

    real weights (exact=False): the same relations within rtol: |D - W| <= rtol D
    where P = -1, |D[i][k] + D[k][j] - D[i][j]| <= rtol D[i][j] at k = P[i][j] >= 0
    (finite pairs), and |sum - D[i][j]| <= rtol D[i][j] h for an encoded path of
    h edges.

    Both: sampled pairs are also reconstructed vertex by vertex (no repeated
    vertex; with exact weights the largest interior vertex is P[i][j]).
    """
    W = np.asarray(W)
    D = np.asarray(D)
    P = np.asarray(P)
    n = W.shape[0]
    assert D.shape == (n, n) and P.shape == (n, n), "shape"
    rows = np.arange(n, dtype=np.int64) if rows is None else np.asarray(rows, dtype=np.int64)
    Wr = W[rows].astype(np.float64)
    Dr = D[rows].astype(np.float64)
    Pr = P[rows]
    R = np.arange(rows.size)
    assert not np.isnan(Dr).any(), "D holds NaN"
    assert np.all(Dr[R, rows] == 0), "D[i][i] != 0"
    assert np.all(Pr[R, rows] == -1), "P[i][i] != -1"
    assert np.all(Dr <= Wr), "D exceeds W"
    finD = np.isfinite(Dr)
    ks = np.arange(n) if n <= 2048 else np.random.default_rng(seed).choice(n, 64, replace=False)
    assert triangle_violations(D, ks, rtol, rows=rows) == 0, "triangle inequality broken"
    assert np.all((Pr >= -1) & (Pr < n)), "P out of range"
    off = rows[:, None] != np.arange(n)[None, :]
    assert not np.any((Pr == rows[:, None]) & off), "P[i][j] == i"
    assert not np.any((Pr == np.arange(n)[None, :]) & off), "P[i][j] == j"
    assert np.all(Pr[~finD] == -1), "P set on an unreachable pair"
    direct = (Pr == -1) & finD & off

    def dval(a, b):  # D[a][b] as float64, elementwise
        return np.asarray(D[a, b], dtype=np.float64)

    if exact:
        assert np.all(Dr[direct] == Wr[direct]), "P = -1 but D differs from the direct edge"
        Q, J = np.nonzero(Pr >= 0)
        I, K = rows[Q], Pr[Q, J].astype(np.int64)
        assert np.all(dval(I, K) + dval(K, J) == Dr[Q, J]), "D[i][j] != D[i][k] + D[k][j] for k = P[i][j]"
        assert np.all(P[I, K] < K), "P[i][P[i][j]] >= P[i][j] (not canonical)"
        assert np.all(P[K, J] < K), "P[P[i][j]][j] >= P[i][j] (not canonical)"
    else:
        dd = Dr[direct]
        assert np.all(np.abs(dd - Wr[direct]) <= rtol * dd), "P = -1 but D differs from the direct edge"
        Q, J = np.nonzero((Pr >= 0) & finD)
        I, K = rows[Q], Pr[Q, J].astype(np.int64)
        dij = Dr[Q, J]
        assert np.all(np.abs(dval(I, K) + dval(K, J) - dij) <= rtol * dij), \
            "D[i][k] + D[k][j] differs from D[i][j] at k = P[i][j]"
    S, H = path_sums(W, P, rows=rows)
    assert np.all(H[finD] >= 0), "P encodes no path (cycle, endpoint label or too long) for some pair"
    if exact:
        assert np.array_equal(S[finD], Dr[finD]), "an encoded path does not sum to D"
    else:
        df = Dr[finD]
        assert np.all(np.abs(S[finD] - df) <= rtol * df * np.maximum(H[finD], 1)), \
            "an encoded path does not sum to D within rtol"
    if sample is None:
        rng = np.random.default_rng(seed)
        Q, J = np.nonzero(finD & off)
        if Q.size > nsample:
            pick = rng.choice(Q.size, nsample, replace=False)
            Q, J = Q[pick], J[pick]
        sample = list(zip(rows[Q].tolist(), J.tolist()))
    for (i, j) in sample:
        dij = float(D[i, j])
        if not np.isfinite(dij):
            continue
        path = reconstruct(P, i, j)
        assert path is not None, f"invalid path encoding at ({i},{j})"
        assert path[0] == i and path[-1] == j
        assert len(set(path)) == len(path), f"path for ({i},{j}) repeats a vertex"
        s = 0.0
        for a, b in zip(path[:-1], path[1:]):
            w = float(W[a, b])
            assert np.isfinite(w), f"path ({i},{j}) uses a missing edge {a}->{b}"
            s += w
        if exact:
            assert s == dij, f"path ({i},{j}) sums to {s} != D {dij}"
            if len(path) > 2:
                assert max(path[1:-1]) == P[i, j], "P is not the largest interior vertex"
        else:
            assert abs(s - dij) <= rtol * max(abs(dij), 1e-30) * len(path), \
                f"path ({i},{j}) sums to {s} vs D {dij}"
