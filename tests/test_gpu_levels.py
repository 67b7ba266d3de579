"""Degree levels (Defn. 4) on the GPU (nd_levels) against the oracle's: the
same level for every r-clique and the same number of levels, for every kind;
the printed levels of the paper's k-core example; and the convergence
theorem checked on the GPU's own SND iterates (level-i r-cliques are exact
from sweep i on, so SND needs at most as many sweeps as there are
levels)."""

import json
import os

import numpy as np
import pytest
import torch

import oracle
from synth import RawGraph, chung_lu, erdos_renyi, sbm

pytestmark = pytest.mark.gpu

KINDS = {"core": (1, 2), "truss": (2, 3), "nucleus34": (3, 4), "nucleus13": (1, 3),
         "nucleus24": (2, 4)}


@pytest.fixture(scope="module")
def ctx(nd):
    return nd.Context(0)


def make(nd, ctx, raw):
    return nd.Graph.from_edges(ctx, raw.n, torch.from_numpy(raw.src),
                               torch.from_numpy(raw.dst))


def graphs():
    yield chung_lu(3000, 2.1, 12.0, seed=71)
    yield sbm(n_comm=25, size_lo=8, size_hi=30, p_in=0.4, p_out=0.003, seed=72)
    yield erdos_renyi(500, 0.03, seed=73)
    pairs = [(i, i + 1) for i in range(299)]  # a path: many levels
    yield RawGraph(300, np.array([a for a, b in pairs], np.int32),
                   np.array([b for a, b in pairs], np.int32), "path")


@pytest.mark.parametrize("kind", list(KINDS))
@pytest.mark.parametrize("big", [None, "1", "40"])
def test_levels_equal_oracle(nd, ctx, kind, big, monkeypatch):
    """big: levels with at least this many candidates run as grid-wide
    kernels (1: every level; 40: a mix; None: the default, mostly one
    workgroup at these sizes)."""
    if big is not None:
        monkeypatch.setenv("ND_LEVELS_BIG", big)
    r, s = KINDS[kind]
    for raw in graphs():
        og = oracle.Graph.from_raw(raw)
        want, want_n = og.levels(r, s)
        g = make(nd, ctx, raw)
        lv, n = g.levels(kind)
        assert n == want_n, raw.name
        assert np.array_equal(lv.cpu().numpy(), want), raw.name
        # convergence theorem on the GPU iterates
        if want.size:
            its = []
            kappa, res = g.decompose(kind, "snd", keep_iterates=its)
            assert res["sweeps"] <= n + 1
            lvn = lv.cpu().numpy()
            kap = kappa.cpu().numpy()
            for t, (_, tau) in enumerate(its, start=1):
                done = lvn < t
                assert np.array_equal(tau.cpu().numpy()[done], kap[done]), t


def test_levels_paper_core_example(nd, ctx):
    spec = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "paper_examples.json")))["core_example"]
    names = spec["vertices"]
    ix = {v: i for i, v in enumerate(names)}
    src = np.array([ix[a] for a, b in spec["edges"]], np.int32)
    dst = np.array([ix[b] for a, b in spec["edges"]], np.int32)
    g = make(nd, ctx, RawGraph(len(names), src, dst, "core_example"))
    lv, n = g.levels("core")
    for v, l in spec["printed"]["levels"].items():
        assert int(lv[ix[v]]) == l
    assert n == 4


def test_levels_edge_cases(nd, ctx):
    empty = RawGraph(7, np.zeros(0, np.int32), np.zeros(0, np.int32), "empty")
    g = make(nd, ctx, empty)
    lv, n = g.levels("core")
    assert n == 1 and (lv.cpu().numpy() == 0).all()  # all of degree 0
    lv, n = g.levels("truss")
    assert n == 0 and lv.numel() == 0
