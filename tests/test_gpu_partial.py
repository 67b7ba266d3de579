"""PartialAND (nd_partial_and) and ego-network estimates (nd_ego_estimate)
on the GPU against the oracle's PartialAND: equal values on every listed
r-clique, for every kind, on random sets, ego networks, hub queries whose
ego network exceeds one workgroup's table, and the edge cases."""

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
    yield chung_lu(3000, 2.1, 12.0, seed=61)
    yield sbm(n_comm=25, size_lo=8, size_hi=30, p_in=0.4, p_out=0.003, seed=62)
    yield erdos_renyi(400, 0.04, seed=63)


@pytest.mark.parametrize("kind", list(KINDS))
def test_partial_and_equals_oracle(nd, ctx, kind):
    r, s = KINDS[kind]
    rng = np.random.default_rng(64)
    for raw in graphs():
        og = oracle.Graph.from_raw(raw)
        nr = og.num_rcliques(r)
        if nr == 0:
            continue
        g = make(nd, ctx, raw)
        sets = [rng.choice(nr, size=min(nr, m), replace=False)
                for m in (1, 7, 100, nr // 3 + 1)]
        sets.append(np.concatenate([sets[1], sets[1]]))  # repeats
        for P in sets:
            want, _, conv = og.partial_and(r, s, P)
            got, res = g.partial_and(kind, P)
            assert conv and res["converged"] == 1
            assert np.array_equal(got.cpu().numpy(), want[P]), (raw.name, len(P))
        # the whole set is AND itself: kappa
        got, _ = g.partial_and(kind, np.arange(nr))
        assert np.array_equal(got.cpu().numpy(), og.peel(r, s)), raw.name


@pytest.mark.parametrize("kind", list(KINDS))
def test_ego_estimates_equal_oracle(nd, ctx, kind):
    r, s = KINDS[kind]
    rng = np.random.default_rng(65)
    for raw in graphs():
        og = oracle.Graph.from_raw(raw)
        nr = og.num_rcliques(r)
        if nr == 0:
            continue
        g = make(nd, ctx, raw)
        qs = rng.integers(0, nr, size=min(nr, 60))
        want, want_sw = og.ego_estimate(r, s, qs)
        est, sw = g.ego_estimate(kind, qs)
        assert np.array_equal(est.cpu().numpy(), want), raw.name
        assert (sw.cpu().numpy() >= 1).all()
        again, _ = g.ego_estimate(kind, qs)
        assert torch.equal(again, est)
        # each estimate also equals nd_partial_and on the same ego set
        for q in qs[:5]:
            P = og.ego_set(r, s, int(q))
            got, _ = g.partial_and(kind, P)
            assert int(got[int(np.searchsorted(P, q))]) == int(est[list(qs).index(q)])


def test_ego_estimates_hub_queries_fallback(nd, ctx):
    """Ego networks beyond the 4096-entry workgroup table: a vertex of degree
    5000 (k-core) and an edge in 3000 triangles (k-truss, 6001 members),
    mixed with small queries in one call."""
    from synth import RawGraph
    hub = [(0, 1 + i) for i in range(5000)] + [(1 + i, 2 + i) for i in range(0, 4999, 2)]
    book = [(0, 1)] + [(x, 2 + i) for i in range(3000) for x in (0, 1)]
    for kind, pairs, qlist in (("core", hub, [0, 1, 2, 17, 4000]),
                               ("truss", book, [0, 1, 2, 5, 6000])):
        n = max(max(p) for p in pairs) + 1
        raw = RawGraph(n, np.array([a for a, b in pairs], np.int32),
                       np.array([b for a, b in pairs], np.int32), kind + "_hub")
        r, s = KINDS[kind]
        og = oracle.Graph.from_raw(raw)
        qs = np.array([q for q in qlist if q < og.num_rcliques(r)])
        want, _ = og.ego_estimate(r, s, qs)
        g = make(nd, ctx, raw)
        est, sw = g.ego_estimate(kind, qs)
        assert np.array_equal(est.cpu().numpy(), want), kind
        assert (sw.cpu().numpy() >= 1).all()


def test_partial_and_edge_cases(nd, ctx):
    raw = chung_lu(1500, 2.2, 10.0, seed=66)
    og = oracle.Graph.from_raw(raw)
    g = make(nd, ctx, raw)
    nr = og.num_rcliques(2)
    # empty set
    got, res = g.partial_and("truss", np.zeros(0, np.int32))
    assert got.numel() == 0 and res["converged"] == 1
    # an id out of range
    with pytest.raises(nd.NdError) as e:
        g.partial_and("truss", [0, nr])
    assert e.value.name == "invalid"
    with pytest.raises(nd.NdError) as e:
        g.ego_estimate("truss", [-1])
    assert e.value.name == "invalid"
    # max_iters stops a set that needs more sweeps: an upper bound remains
    P = np.arange(nr)
    want, sweeps, _ = og.partial_and(2, 3, P)
    if sweeps > 2:
        got, res = g.partial_and("truss", P, max_iters=1,
                                 allow_not_converged=True)
        assert res["converged"] == 0
        assert (got.cpu().numpy() >= want).all()
        with pytest.raises(nd.NdError) as e:
            g.partial_and("truss", P, max_iters=1)
        assert e.value.name == "not_converged"
    # ego estimates with no queries
    est, sw = g.ego_estimate("truss", np.zeros(0, np.int32))
    assert est.numel() == 0
    # a graph without triangles: every estimate is 0
    path = RawGraph(50, np.arange(49, dtype=np.int32),
                    np.arange(1, 50, dtype=np.int32), "path")
    gp = make(nd, ctx, path)
    est, sw = gp.ego_estimate("truss", np.arange(49))
    assert (est.cpu().numpy() == 0).all()
