"""Pin sensitivity: plant plausible mistakes in a copy of the C oracle (on the CPU),
compile it, and check that the pins reject every mutant while accepting the
unmodified copy.  Needs gcc."""
import os
import shutil
import subprocess
import tempfile
import types

import numpy as np
import pytest

import oracle
import workloads
from conftest import load_golden
from test_checker_pins import escaped

SRC = os.path.join(os.path.dirname(oracle.__file__), "fw_oracle.c")

MUTANTS = {
    "non_strict_test": [("if (s < rowi[j])", "if (s <= rowi[j])")],
    "store_i_not_k": [("prow[j] = (int32_t)k;", "prow[j] = (int32_t)i;")],
    "transposed_operand": [("double b = rowk[j];", "double b = D[j * n + k];"),
                           ("int64_t b = rowk[j];", "int64_t b = D[j * n + k];")],
    "dropped_term": [("double s = a + b;", "double s = b;"),
                     ("int64_t s = a + b;", "int64_t s = b;")],
    "p_init_zero": [("P[x] = -1;", "P[x] = 0;")],
    "last_k_skipped": [("for (int64_t k = 0; k < n; ++k)", "for (int64_t k = 0; k < n - 1; ++k)")],
    "dijkstra_no_tiebreak": [("(s == dist[v] && mu < pmax[v])", "(0)")],
    "dijkstra_pmax_u": [("int32_t mu = (u == src) ? -1 : (pmax[u] > (int32_t)u ? pmax[u] : (int32_t)u);",
                         "int32_t mu = (u == src) ? -1 : (int32_t)u;")],
    "backward_transposed": [("gW[a * n + b] += g;", "gW[b * n + a] += g;")],
    "backward_split_swapped": [("stk[2 * top] = m; stk[2 * top + 1] = b; ++top;\n                stk[2 * top] = a;",
                                "stk[2 * top] = b; stk[2 * top + 1] = m; ++top;\n                stk[2 * top] = a;")],
}


def run_pins():
    """Return the names of the pins that fail with the currently loaded oracle library."""
    failed = []

    def pin(name, fn):
        try:
            fn()
        except (AssertionError, ValueError):
            failed.append(name)

    def brute():
        for seed in range(12):
            rng = np.random.default_rng(seed)
            n = int(rng.integers(3, 8))
            W = np.full((n, n), np.inf)
            m = rng.random((n, n)) < 0.6
            W[m] = rng.integers(1, 4, size=m.sum())
            np.fill_diagonal(W, 0)
            D, P = oracle.fw(W)
            Db, Pb = oracle.brute_force(W)
            assert np.array_equal(D, Db) and np.array_equal(P, Pb)
        for seed in range(6):
            rng = np.random.default_rng(50 + seed)
            n = 7
            W = np.where(rng.random((n, n)) < 0.6, rng.random((n, n)) + 0.01, np.inf)
            np.fill_diagonal(W, 0)
            D, P = oracle.fw(W)
            Db, Pb = oracle.brute_force(W)
            fin = np.isfinite(Db)
            assert np.array_equal(np.isfinite(D), fin) and np.allclose(D[fin], Db[fin], rtol=1e-14)
            assert np.array_equal(P, Pb)

    def golden():
        g = load_golden("tie_example_5.txt")
        D, P = oracle.fw(g["W"])
        assert np.array_equal(D, g["D"]) and np.array_equal(P, g["P"])

    def dijkstra():
        W = workloads.int_graph(n=128, p=0.06, wmax=3, seed=12)
        Dr, Pr = oracle.dijkstra_rows(W, np.arange(128))
        Db = [oracle.brute_force(W[:8, :8])]  # keeps the brute-force path exercised
        D, P = oracle.fw(W)
        assert np.array_equal(Dr, D) and np.array_equal(Pr, P)
        assert Db

    def backward():
        n = 30
        rng = np.random.default_rng(1)
        W = np.full((n, n), np.inf)
        np.fill_diagonal(W, 0)
        W[np.arange(n - 1), np.arange(1, n)] = rng.uniform(1, 2, n - 1)
        W[0, 5] = 100.0  # a long direct edge that no shortest path uses
        G = rng.standard_normal((n, n))
        D, P = oracle.fw(W)
        gW = oracle.backward_pathwalk(D, P, G)
        for t in range(n - 1):
            e = sum(G[i, j] for i in range(t + 1) for j in range(t + 1, n))
            assert abs(gW[t, t + 1] - e) < 1e-12
        assert gW[0, 5] == 0.0 and gW[5, 0] == 0.0

    def invariants():
        W = workloads.int_graph(n=200, p=0.1, wmax=20, seed=4)
        D, P = oracle.fw(W)
        oracle.check_invariants(W, D, P, exact=True)

    pin("brute", brute)
    pin("golden", golden)
    pin("dijkstra", dijkstra)
    pin("backward", backward)
    def checker():
        assert escaped(oracle.check_invariants) == []

    pin("invariants", invariants)
    pin("checker", checker)
    return failed


@pytest.fixture(scope="module")
def workdir():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    d = tempfile.mkdtemp(prefix="oracle_mutants_")
    yield d
    shutil.rmtree(d, ignore_errors=True)


def build_variant(workdir, name, edits):
    src = open(SRC).read()
    for old, new in edits:
        assert old in src, f"mutation anchor missing: {old!r}"
        src = src.replace(old, new)
    cpath = os.path.join(workdir, f"{name}.c")
    with open(cpath, "w") as f:
        f.write(src)
    return oracle.build(src=cpath, out=os.path.join(workdir, f"lib{name}.so"))


def test_unmodified_copy_passes(workdir, monkeypatch):
    lib = oracle.load(build_variant(workdir, "clean", []))
    monkeypatch.setattr(oracle, "_lib", lib)
    assert run_pins() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(workdir, monkeypatch, name):
    lib = oracle.load(build_variant(workdir, name, MUTANTS[name]))
    monkeypatch.setattr(oracle, "_lib", lib)
    failed = run_pins()
    assert failed, f"no pin rejects mutant {name}"


# Mutants of the checker itself (oracle.check_invariants, Python): each must let
# at least one corrupted (D, P) of test_checker_pins through, i.e. the checker's
# pins notice when the checker is weakened.
ORACLE_PY = os.path.join(os.path.dirname(oracle.__file__), "__init__.py")
CHECKER_MUTANTS = {
    "accept_all": [('    assert D.shape == (n, n) and P.shape == (n, n), "shape"', "    return")],
    # the sampled reconstruction emptied, and the all-pairs walk and split check dropped
    "pair_checks_emptied": [("        sample = list(zip(rows[Q].tolist(), J.tolist()))", "        sample = []"),
                            ("    S, H = path_sums(W, P, rows=rows)", "    S, H = Dr.copy(), np.ones(Dr.shape, dtype=np.int64)"),
                            ("        assert np.all(np.abs(dval(I, K) + dval(K, J) - dij) <= rtol * dij), \\",
                             "        assert True, \\")],
    "canonical_dropped": [('        assert np.all(P[I, K] < K), "P[i][P[i][j]] >= P[i][j] (not canonical)"', ""),
                          ('        assert np.all(P[K, J] < K), "P[P[i][j]][j] >= P[i][j] (not canonical)"', ""),
                          ("                assert max(path[1:-1]) == P[i, j], \"P is not the largest interior vertex\"",
                           "                pass")],
    "unreachable_label_allowed": [('    assert np.all(Pr[~finD] == -1), "P set on an unreachable pair"', "")],
}


def mutated_oracle(edits):
    src = open(ORACLE_PY).read()
    for old, new in edits:
        assert old in src, f"mutation anchor missing: {old!r}"
        src = src.replace(old, new)
    mod = types.ModuleType("oracle_checker_mutant")
    mod.__file__ = ORACLE_PY
    exec(compile(src, ORACLE_PY, "exec"), mod.__dict__)
    return mod


def test_checker_unmodified_copy_passes():
    assert escaped(mutated_oracle([]).check_invariants) == []


@pytest.mark.parametrize("name", sorted(CHECKER_MUTANTS))
def test_checker_mutant_is_caught(name):
    got = escaped(mutated_oracle(CHECKER_MUTANTS[name]).check_invariants)
    assert got, f"no corruption gets past checker mutant {name}"
