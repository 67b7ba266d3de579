"""The 32-bit tau path.  When some S-degree reaches 32768 the library stores
tau in 32 bits, which instantiates every sweep, batch, PartialAND and
ego-estimate kernel with int32 values instead of uint16.  One graph takes
every kind there, and each entry point is compared with the oracle.

The graph: a triangle {a, b, c} whose three vertices have 33,000 common
neighbours (the pages), the pages joined in pairs, a and b also joined to
150 vertices of a Chung-Lu graph on 3,000 vertices (so that the iteration
has work to do in both parts).  Then
  * vertex a has degree > 33,000 (k-core) and lies in > 82,000 triangles
    (1,3),
  * edge ab lies in 33,001+ triangles (k-truss) and in 49,500 4-cliques
    (2,4),
  * triangle abc lies in 33,000 4-cliques (3,4).
(Pages joined in one long path instead would make (1,2) and (1,3) take about
16,500 sweeps, one step along the path per sweep.)
"""

import numpy as np
import pytest
import torch

import oracle
from synth import RawGraph, chung_lu

pytestmark = pytest.mark.gpu

KINDS = {"core": (1, 2), "truss": (2, 3), "nucleus34": (3, 4), "nucleus13": (1, 3),
         "nucleus24": (2, 4)}
PAGES = 33000


def hub_graph():
    cl = chung_lu(3000, 2.1, 14.0, seed=71)
    n0 = cl.n
    a, b, c = n0, n0 + 1, n0 + 2
    pages = np.arange(n0 + 3, n0 + 3 + PAGES, dtype=np.int32)
    src = [cl.src, np.array([a, a, b], np.int32)]
    dst = [cl.dst, np.array([b, c, c], np.int32)]
    for x in (a, b, c):
        src.append(np.full(PAGES, x, np.int32))
        dst.append(pages)
    src.append(pages[0::2])
    dst.append(pages[1::2])
    hooks = np.arange(0, 3000, 20, dtype=np.int32)
    for x in (a, b):
        src.append(np.full(hooks.size, x, np.int32))
        dst.append(hooks)
    return RawGraph(n0 + 3 + PAGES, np.concatenate(src), np.concatenate(dst),
                    "hub33000")


@pytest.fixture(scope="module")
def ctx(nd):
    return nd.Context(0)


@pytest.fixture(scope="module")
def raw():
    return hub_graph()


@pytest.fixture(scope="module")
def og(raw):
    return oracle.Graph.from_raw(raw)


def make(nd, ctx, raw):
    return nd.Graph.from_edges(ctx, raw.n, torch.from_numpy(raw.src),
                               torch.from_numpy(raw.dst))


@pytest.mark.parametrize("kind", list(KINDS))
def test_int32_snd_iterates_and_and(nd, ctx, raw, og, kind):
    r, s = KINDS[kind]
    g = make(nd, ctx, raw)
    ds = og.sdeg(r, s)
    assert int(ds.max()) >= 32768, "the case must take the 32-bit tau path"
    seq = og.snd(r, s)
    kref = og.peel(r, s)
    assert np.array_equal(seq[-1], kref)
    for fr in (False, True):
        its = []
        kappa, res = g.decompose(kind, "snd", use_frontier=fr, keep_iterates=its)
        assert res["tau_bytes"] == 4 and res["max_sdegree"] == int(ds.max())
        assert res["sweeps"] == len(seq) - 1 == len(its)
        for t, (changed, tau) in enumerate(its, start=1):
            assert np.array_equal(tau.cpu().numpy(), seq[t]), (fr, t)
            assert changed == int((seq[t] != seq[t - 1]).sum())
        assert np.array_equal(kappa.cpu().numpy(), kref)
        ka, ra = g.decompose(kind, "and", use_frontier=fr)
        assert ra["tau_bytes"] == 4 and ra["converged"] == 1
        assert np.array_equal(ka.cpu().numpy(), kref), ("and", fr)
    # one application of U on arbitrary tau <= d_s
    rng = np.random.default_rng(5)
    tau = np.minimum((rng.random(ds.size) * (ds + 1)).astype(np.int32), ds)
    tau[np.argmax(ds)] = ds.max() - 7  # the hub: the coarse-then-fine search
    assert np.array_equal(g.update(kind, torch.from_numpy(tau)).cpu().numpy(),
                          og.update(r, s, tau))


@pytest.mark.parametrize("kind", ["core", "truss", "nucleus34"])
def test_int32_active_counts(nd, ctx, raw, og, kind):
    """The active-ratio counts on the 32-bit path equal the rule's."""
    from test_gpu_parity import expected_active
    r, s = KINDS[kind]
    g = make(nd, ctx, raw)
    seq = og.snd(r, s)
    want = expected_active(og, r, s, seq)
    st = []
    g.decompose(kind, "snd", use_frontier=True, count_active=True, keep_stats=st)
    assert [x["active_next"] for x in st] == want


@pytest.mark.parametrize("kind", list(KINDS))
def test_int32_batch_and_server(nd, ctx, raw, og, kind):
    """Batched with a graph whose tau fits 16 bits, the 32-bit graph is swept
    in 32 bits and the other in 16 (two combined lists); served requests
    too.  Every result equals the oracle's."""
    r, s = KINDS[kind]
    small = chung_lu(2000, 2.2, 10.0, seed=72)
    want = [og.peel(r, s), oracle.Graph.from_raw(small).peel(r, s)]
    for mode in ("snd", "and"):
        gs = [make(nd, ctx, raw), make(nd, ctx, small)]
        for fr in (False, True):
            kappas, results = nd.batch_decompose(ctx, gs, kind, mode,
                                                 use_frontier=fr)
            for k, rs, w, tb in zip(kappas, results, want, (4, 2)):
                assert rs["tau_bytes"] == tb and rs["converged"] == 1
                assert np.array_equal(k.cpu().numpy(), w), (mode, fr)
    srv = nd.Server(ctx, max_slots=4)
    ts = [srv.submit(make(nd, ctx, x), kind, m, use_frontier=fr)
          for x, m, fr in ((raw, "snd", True), (small, "and", False),
                           (raw, "and", False))]
    for t, w in zip(ts, (want[0], want[1], want[0])):
        kappa, res, info = srv.wait(t)
        assert res["converged"] == 1
        assert np.array_equal(kappa.numpy(), w)
    srv.close()


@pytest.mark.parametrize("kind", ["core", "truss", "nucleus34"])
def test_int32_partial_and_ego(nd, ctx, raw, og, kind):
    """PartialAND on sets holding the hub r-clique, and ego-network
    estimates of the hub (its ego network exceeds the one-workgroup table,
    so it runs as PartialAND) and of ordinary r-cliques."""
    r, s = KINDS[kind]
    g = make(nd, ctx, raw)
    ds = og.sdeg(r, s)
    hub = int(np.argmax(ds))
    rng = np.random.default_rng(9)
    ids = np.unique(np.concatenate([[hub], rng.integers(0, ds.size, 400)])).astype(np.int32)
    got, res = g.partial_and(kind, torch.from_numpy(ids))
    tau, sweeps, ok = og.partial_and(r, s, ids)
    assert ok and np.array_equal(got.cpu().numpy(), tau[ids])
    qs = np.concatenate([[hub], rng.choice(np.nonzero(ds)[0], 40)]).astype(np.int32)
    est, sw = g.ego_estimate(kind, torch.from_numpy(qs))
    west, wsw = og.ego_estimate(r, s, qs)
    assert np.array_equal(est.cpu().numpy(), west)
