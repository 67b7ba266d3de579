"""The community split that writes the block-model (3,4) golden values
(tests/golden/make_golden.py) equals Alg. Peeling on the whole graph, and
refuses graphs where a 4-clique spans two communities."""

import importlib.util
import os
import sys

import numpy as np
import pytest

import oracle
from synth import RawGraph, sbm

_spec = importlib.util.spec_from_file_location(
    "make_golden", os.path.join(os.path.dirname(__file__), "golden", "make_golden.py"))
mg = importlib.util.module_from_spec(_spec)
sys.modules["make_golden"] = mg  # the process pool pickles its worker by name
_spec.loader.exec_module(mg)


@pytest.mark.parametrize("seed", [41, 42, 43])
def test_split_equals_whole_graph_peeling(seed):
    raw, labels = sbm(n_comm=12, size_lo=8, size_hi=20, p_in=0.6, p_out=0.003,
                      seed=seed, with_communities=True)
    want = oracle.Graph.from_raw(raw).peel(3, 4)
    got = mg.kappa_by_community(raw, labels, threads=2)
    assert want.max() >= 2
    assert np.array_equal(got, want)


def test_split_refuses_spanning_cliques():
    # two K5 communities joined by a K4 that takes two vertices of each
    src, dst = [], []
    for base in (0, 5):
        for a in range(5):
            for b in range(a + 1, 5):
                src.append(base + a)
                dst.append(base + b)
    for a, b in ((0, 5), (0, 6), (1, 5), (1, 6)):
        src.append(a)
        dst.append(b)
    raw = RawGraph(10, np.array(src, np.int32), np.array(dst, np.int32), "k5k5")
    labels = np.array([0] * 5 + [1] * 5, np.int32)
    with pytest.raises(RuntimeError):
        mg.kappa_by_community(raw, labels, threads=2)
