"""The two ways the triangle list is built give the same list, and every
kind built on either is exact.  Prepared first for (3,4), a graph lists its
triangles from the per-vertex bit rows (vertices of degree <= 256; the edges
below larger ones by intersection); prepared first for (1,3), by edge
intersection alone, after which (3,4) builds its rows in its own count pass.
The book graph has spine vertices of degree > 256, so both halves of the
bit-row path run."""

import numpy as np
import pytest
import torch

import oracle
from synth import books, chung_lu, sbm

pytestmark = pytest.mark.gpu

GRAPHS = [
    ("cl4k", lambda: chung_lu(4096, 2.1, 16.0, seed=7)),
    ("sbm40", lambda: sbm(n_comm=40, size_lo=10, size_hi=40, p_in=0.3,
                          p_out=0.002, seed=9)),
    ("books", lambda: books(pages=(400, 800, 1600), page_degree=8.0, seed=5)),
]


@pytest.fixture(scope="module")
def ctx(nd):
    return nd.Context(0)


@pytest.mark.parametrize("name,make", GRAPHS, ids=[x[0] for x in GRAPHS])
def test_triangle_paths_agree(nd, ctx, name, make):
    raw = make()
    og = oracle.Graph.from_raw(raw)
    tri = og.rcliques(3)

    def graph():
        return nd.Graph.from_edges(ctx, raw.n, torch.from_numpy(raw.src),
                                   torch.from_numpy(raw.dst))

    rows_first = graph()  # (3,4) first: triangles from the bit rows
    k34a, _ = rows_first.decompose("nucleus34", "snd", use_frontier=True)
    assert np.array_equal(rows_first.rcliques("nucleus34").cpu().numpy(), tri)
    for kind, (r, s) in (("nucleus13", (1, 3)), ("nucleus24", (2, 4))):
        k, _ = rows_first.decompose(kind, "snd", use_frontier=True)
        assert np.array_equal(k.cpu().numpy(), og.peel(r, s)), kind
    isect_first = graph()  # (1,3) first: triangles by intersection
    k13, _ = isect_first.decompose("nucleus13", "and")
    assert np.array_equal(k13.cpu().numpy(), og.peel(1, 3))
    k34b, _ = isect_first.decompose("nucleus34", "snd", use_frontier=True)
    assert np.array_equal(isect_first.rcliques("nucleus34").cpu().numpy(), tri)
    want = og.peel(3, 4)
    assert np.array_equal(k34a.cpu().numpy(), want)
    assert np.array_equal(k34b.cpu().numpy(), want)
    assert np.array_equal(rows_first.sdegree("nucleus34").cpu().numpy(),
                          og.sdeg(3, 4))
    assert np.array_equal(isect_first.sdegree("nucleus34").cpu().numpy(),
                          og.sdeg(3, 4))
    rows_first.close()
    isect_first.close()


@pytest.mark.parametrize("name,make", GRAPHS, ids=[x[0] for x in GRAPHS])
def test_n34_without_kept_rows(nd, ctx, name, make, monkeypatch):
    """The (3,4) builder's path without kept bit rows (tight budgets):
    triangles by intersection, rows rebuilt by the count and the fill pass.
    Its incidence lists (as sets), S-degrees and kappa equal the path's with
    rows and the oracle's."""
    raw = make()
    og = oracle.Graph.from_raw(raw)
    want = og.peel(3, 4)
    canon = []
    for env in ({}, {"ND_N34_NO_ROWS": "1"}):
        with monkeypatch.context() as m:
            for k, v in env.items():
                m.setenv(k, v)
            g = nd.Graph.from_edges(ctx, raw.n, torch.from_numpy(raw.src),
                                    torch.from_numpy(raw.dst))
            g.prepare("nucleus34")
        assert np.array_equal(g.rcliques("nucleus34").cpu().numpy(), og.rcliques(3))
        assert np.array_equal(g.sdegree("nucleus34").cpu().numpy(), og.sdeg(3, 4))
        off, ids = g.incidence("nucleus34")
        nr = off.numel() - 1
        rid = torch.repeat_interleave(torch.arange(nr, device=off.device),
                                      off[1:] - off[:-1]).long()
        srt = torch.sort(ids.long(), dim=1).values
        key = ((rid * nr + srt[:, 0]) * nr + srt[:, 1]) * nr + srt[:, 2]
        canon.append(torch.sort(key).values)
        for mode in ("snd", "and"):
            kappa, res = g.decompose("nucleus34", mode, use_frontier=True)
            assert res["converged"] == 1
            assert np.array_equal(kappa.cpu().numpy(), want), (env, mode)
        g.close()
    assert torch.equal(canon[0], canon[1])
