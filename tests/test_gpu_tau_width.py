"""The tau widths of the one-graph sweeps.  tau is stored in 8 bits when
every S-degree is below 256, in 16 below 32768, else in 32; the iterates
and results must not depend on it.  For every kind, one graph whose largest
S-degree is exactly 255 (8-bit path) and one where it is 256 (16-bit path):
an Erdos-Renyi graph (n = 2000, p = 0.005, every S-degree far below 255)
with, on vertices of their own, a gadget that gives one r-clique exactly
D s-cliques:
  (1,2) a star of D leaves;          (1,3) a vertex with D disjoint rim
  (2,3) an edge with D pages;              edges (D triangles);
  (3,4) a triangle with D apexes;    (2,4) an edge with D joined page pairs
                                           (D 4-cliques).
Each graph's SND iterates (frontier off and on), AND and one application
of U on an arbitrary tau are compared with the oracle, and the reported
width with the largest S-degree.
"""

import numpy as np
import pytest
import torch

import oracle
from synth import RawGraph, erdos_renyi

pytestmark = pytest.mark.gpu

KINDS = {"core": (1, 2), "truss": (2, 3), "nucleus34": (3, 4), "nucleus13": (1, 3),
         "nucleus24": (2, 4)}


def gadget_graph(kind, d):
    base = erdos_renyi(2000, 0.005, seed=81)
    n0 = base.n
    src, dst = [base.src], [base.dst]

    def join(a, b):
        src.append(np.asarray(a, np.int32).ravel())
        dst.append(np.asarray(b, np.int32).ravel())

    hub = np.arange(n0, n0 + 3, dtype=np.int32)     # up to three hub vertices
    extra = np.arange(n0 + 3, n0 + 3 + 2 * d, dtype=np.int32)
    u, v, w = hub
    if kind == "core":
        join(np.full(d, u), extra[:d])
    elif kind == "truss":
        join([u], [v])
        join(np.full(d, u), extra[:d])
        join(np.full(d, v), extra[:d])
    elif kind == "nucleus34":
        join([u, u, v], [v, w, w])
        for x in hub:
            join(np.full(d, x), extra[:d])
    elif kind == "nucleus13":
        p, q = extra[0::2], extra[1::2]
        join(p, q)
        join(np.full(d, u), p)
        join(np.full(d, u), q)
    else:  # nucleus24
        p, q = extra[0::2], extra[1::2]
        join([u], [v])
        join(p, q)
        for x in (u, v):
            join(np.full(d, x), p)
            join(np.full(d, x), q)
    return RawGraph(n0 + 3 + 2 * d, np.concatenate(src), np.concatenate(dst),
                    f"er2000+{kind}{d}")


@pytest.fixture(scope="module")
def ctx(nd):
    return nd.Context(0)


@pytest.mark.parametrize("d,width", [(255, 1), (256, 2)])
@pytest.mark.parametrize("kind", list(KINDS))
def test_tau_width_boundary(nd, ctx, kind, d, width):
    r, s = KINDS[kind]
    raw = gadget_graph(kind, d)
    og = oracle.Graph.from_raw(raw)
    ds = og.sdeg(r, s)
    assert int(ds.max()) == d, "the gadget must set the largest S-degree"
    seq = og.snd(r, s)
    kref = og.peel(r, s)
    assert np.array_equal(seq[-1], kref)
    g = nd.Graph.from_edges(ctx, raw.n, torch.from_numpy(raw.src),
                            torch.from_numpy(raw.dst))
    for fr in (False, True):
        its = []
        kappa, res = g.decompose(kind, "snd", use_frontier=fr, keep_iterates=its)
        assert res["tau_bytes"] == width and res["max_sdegree"] == d
        assert res["sweeps"] == len(seq) - 1 == len(its)
        for t, (changed, tau) in enumerate(its, start=1):
            assert np.array_equal(tau.cpu().numpy(), seq[t]), (fr, t)
            assert changed == int((seq[t] != seq[t - 1]).sum())
        assert np.array_equal(kappa.cpu().numpy(), kref)
        ka, ra = g.decompose(kind, "and", use_frontier=fr)
        assert ra["tau_bytes"] == width and ra["converged"] == 1
        assert np.array_equal(ka.cpu().numpy(), kref), ("and", fr)
    rng = np.random.default_rng(d)
    tau = np.minimum((rng.random(ds.size) * (ds + 1)).astype(np.int32), ds)
    tau[np.argmax(ds)] = d  # the gadget's r-clique at the top of the range
    assert np.array_equal(g.update(kind, torch.from_numpy(tau)).cpu().numpy(),
                          og.update(r, s, tau))
    g.close()
