"""The batched routing rule (csrc/fw_route.h), checked on the host: which graphs
fw_apsp_batched hands to fw_apsp instead of its persistent launch, in which one
workgroup solves one graph (768 resident workgroups on the MI355X with labels)."""
import os
import subprocess

import numpy as np
import pytest

import workloads
from conftest import ROOT

SLOTS = 768


@pytest.fixture(scope="module")
def route(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("route") / "route_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror", "-o", exe,
                    os.path.join(ROOT, "tests", "route_check.cpp")], check=True)

    def run(ns, route=0, slots=SLOTS):
        line = f"{slots} {route} " + " ".join(str(int(n)) for n in ns) + "\n"
        out = subprocess.run([exe], input=line, capture_output=True, text=True, timeout=60, check=True).stdout
        count, flags = out.split()
        assert int(count) == flags.count("1")
        return [c == "1" for c in flags]
    return run


def test_benchmark_batch_routes_nothing(route):
    ns, _, _ = workloads.batch_graphs(batch=10000, seed=4)
    assert not any(route(ns))


def test_one_large_graph_among_small_ones(route):
    ns = [2048] + [100] * 1000 + [37]
    assert route(ns) == [True] + [False] * 1001


def test_equal_graphs_that_fill_the_launch_stay(route):
    # each holds exactly its share of the work: none is the batch's tail
    assert not any(route([512] * SLOTS))
    # a lone graph of n >= 256 is far above its share; below 256 it never moves
    assert route([256]) == [True]
    assert route([255]) == [False]


def test_threshold(route):
    # n^3 against 4 * sum(n^3) / slots: with the n = 600 graph alone among graphs of
    # n = 300, it is routed once it holds more than 4/768 of the batch's work
    # routed while SLOTS * 600^3 > 4 * (600^3 + k * 300^3), strictly
    k_max = ((SLOTS - 4) * 600 ** 3 - 1) // (4 * 300 ** 3)
    assert route([600] + [300] * k_max)[0]
    assert not route([600] + [300] * (k_max + 1))[0]


def test_explicit_settings(route):
    ns = [4096, 300, 256, 255, 10]
    assert route(ns, route=-1) == [False] * 5
    assert route(ns, route=256) == [True, True, True, False, False]
    assert route(ns, route=11) == [True, True, True, True, False]
