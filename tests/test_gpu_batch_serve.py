"""Batched and served decomposition: every result equals the graph's lone
nd_decompose result and the oracle, whatever else shares the launches."""

import time

import numpy as np
import pytest
import torch

import oracle
from synth import books, chung_lu, erdos_renyi, sbm

pytestmark = pytest.mark.gpu

KINDS = {"core": (1, 2), "truss": (2, 3), "nucleus34": (3, 4), "nucleus13": (1, 3),
         "nucleus24": (2, 4)}


@pytest.fixture(scope="module")
def ctx(nd):
    return nd.Context(0)


def mixed_graphs():
    out = [
        erdos_renyi(600, 0.02, seed=31),
        chung_lu(3000, 2.1, 12.0, seed=32),
        chung_lu(800, 2.4, 8.0, seed=33),
        sbm(n_comm=20, size_lo=10, size_hi=30, p_in=0.35, p_out=0.004, seed=34),
        chung_lu(20000, 2.2, 16.0, seed=35),
        books(pages=(400, 800, 1600), page_degree=8.0, seed=36),
    ]
    # a graph with an edge in 3000 triangles and a triangle in 3000 4-cliques
    pairs = [(0, 1), (0, 2), (1, 2)] + [(x, 3 + i) for i in range(3000)
                                        for x in (0, 1, 2)]
    src = np.array([a for a, b in pairs], np.int32)
    dst = np.array([b for a, b in pairs], np.int32)
    from synth import RawGraph
    out.append(RawGraph(3003, src, dst, "book"))
    out.append(RawGraph(5, np.zeros(0, np.int32), np.zeros(0, np.int32), "empty"))
    return out


def make(nd, ctx, raw):
    return nd.Graph.from_edges(ctx, raw.n, torch.from_numpy(raw.src),
                               torch.from_numpy(raw.dst))


@pytest.mark.parametrize("kind", list(KINDS))
@pytest.mark.parametrize("mode", ["snd", "and"])
@pytest.mark.parametrize("frontier", [False, True])
def test_batch_equals_solo_and_oracle(nd, ctx, kind, mode, frontier):
    raws = mixed_graphs()
    r, s = KINDS[kind]
    gs = [make(nd, ctx, raw) for raw in raws]
    solo = [g.decompose(kind, mode) for g in gs]
    kappas, results = nd.batch_decompose(ctx, gs, kind, mode,
                                         use_frontier=frontier)
    for raw, (ks, rs), kb, rb in zip(raws, solo, kappas, results):
        assert torch.equal(kb, ks), raw.name
        assert rb["converged"] == 1
        if mode == "snd":
            assert rb["sweeps"] == rs["sweeps"], raw.name
        want = oracle.Graph.from_raw(raw).peel(r, s)
        assert np.array_equal(kb.cpu().numpy(), want), raw.name


@pytest.mark.parametrize("kind", list(KINDS))
def test_batch_prepares_while_sweeping(nd, ctx, kind):
    """Graphs handed to the batch unprepared are prepared on the library's
    threads while the prepared ones are swept, each joining when ready; the
    results equal the oracle's, whichever graphs were prepared beforehand."""
    raws = mixed_graphs() + [chung_lu(int(n), 2.2, 12.0, seed=600 + i)
                             for i, n in enumerate((900, 7000, 2500, 15000))]
    r, s = KINDS[kind]
    gs = [make(nd, ctx, raw) for raw in raws]
    if r <= 2:  # |R| is read off the graph, nothing is built
        for g, raw in zip(gs, raws):
            og = oracle.Graph.from_raw(raw)
            assert g.rclique_count(kind) == og.num_rcliques(r)
    for g in gs[::3]:
        g.prepare(kind)
    kappas, results = nd.batch_decompose(ctx, gs + gs[:2], kind, "snd",
                                         use_frontier=True)
    for i, (k, rb) in enumerate(zip(kappas, results)):
        raw = raws[i % len(raws)]
        assert rb["converged"] == 1
        want = oracle.Graph.from_raw(raw).peel(r, s)
        assert np.array_equal(k.cpu().numpy(), want), (raw.name, i)
        assert rb["sweeps"] == len(oracle.Graph.from_raw(raw).snd(r, s)) - 1 \
            or want.size == 0, raw.name


def test_graphs_from_edges(nd, ctx):
    """Graphs built together equal graphs built one at a time (CSR and
    decomposition); an invalid edge list fails the whole call."""
    raws = mixed_graphs()
    gs = nd.graphs_from_edges(ctx, [(r.n, torch.from_numpy(r.src), torch.from_numpy(r.dst))
                                    for r in raws])
    for g, raw in zip(gs, raws):
        one = make(nd, ctx, raw)
        ro1, c1 = one.csr()
        ro2, c2 = g.csr()
        assert torch.equal(ro1, ro2) and torch.equal(c1, c2), raw.name
        assert np.array_equal(g.decompose("truss")[0].cpu().numpy(),
                              oracle.Graph.from_raw(raw).peel(2, 3))
    bad = [(raws[0].n, torch.from_numpy(raws[0].src), torch.from_numpy(raws[0].dst)),
           (3, torch.tensor([0, 1], dtype=torch.int32), torch.tensor([1, 7], dtype=torch.int32))]
    with pytest.raises(nd.NdError) as e:
        nd.graphs_from_edges(ctx, bad)
    assert e.value.name == "invalid"
    assert nd.graphs_from_edges(ctx, []) == []


def test_prepare_many(nd, ctx):
    raws = mixed_graphs()
    gs = [make(nd, ctx, raw) for raw in raws]
    gs[1].prepare("nucleus34")
    nd.prepare_many(ctx, gs + [gs[0]], "nucleus34")
    for g, raw in zip(gs, raws):
        og = oracle.Graph.from_raw(raw)
        nr, P, _ = g.sizes("nucleus34")
        assert nr == og.num_rcliques(3)
        assert np.array_equal(g.decompose("nucleus34")[0].cpu().numpy(),
                              og.peel(3, 4))


def test_batch_replays_with_eager_work_between(nd, ctx):
    """Repeated batches (the epoch loop replays a captured HIP graph) with
    eager decompositions and synchronisations in between: every replay
    matches the eager result."""
    raws = [chung_lu(2000 + 500 * i, 2.2, 10.0, seed=50 + i) for i in range(12)]
    gs = [make(nd, ctx, raw) for raw in raws]
    eager = [g.decompose("truss", "snd")[0] for g in gs]
    for rep in range(4):
        kappas, results = nd.batch_decompose(ctx, gs, "truss", "snd")
        torch.cuda.synchronize()
        for e, k in zip(eager, kappas):
            assert torch.equal(e, k), rep
        # eager work between replays
        again = gs[rep].decompose("truss", "and")[0]
        assert torch.equal(again, eager[rep])
        torch.cuda.synchronize()


@pytest.mark.parametrize("frontier", [False, True])
def test_batch_many_small_graphs(nd, ctx, frontier):
    raws = [chung_lu(int(n), 2.0 + 0.05 * (i % 10), 8.0 + i % 20, seed=100 + i)
            for i, n in enumerate(np.linspace(200, 4000, 64))]
    gs = [make(nd, ctx, raw) for raw in raws]
    kappas, results = nd.batch_decompose(ctx, gs, "core", "snd",
                                         use_frontier=frontier)
    for raw, g, k, rb in zip(raws, gs, kappas, results):
        want, rs = g.decompose("core", "snd")
        assert torch.equal(k, want), raw.name
        # frontier SND computes the same iterates, so the same sweep count
        assert rb["sweeps"] == rs["sweeps"], raw.name


def test_batch_frontier_stamps_wrap(nd, ctx):
    """More sweeps than the frontier stamps repeat after (510): on a path the
    k-core iteration lowers one vertex per end per sweep, so SND takes about
    n/2 sweeps; the frontier results, alone and batched, equal the plain one
    and the sweep counts agree."""
    from synth import RawGraph
    n = 1400
    raw = RawGraph(n, np.arange(n - 1, dtype=np.int32),
                   np.arange(1, n, dtype=np.int32), "path")
    g = make(nd, ctx, raw)
    want, rs = g.decompose("core", "snd")
    assert rs["sweeps"] == len(oracle.Graph.from_raw(raw).snd(1, 2)) - 1 > 600
    k1, r1 = g.decompose("core", "snd", use_frontier=True)
    assert torch.equal(k1, want) and r1["sweeps"] == rs["sweeps"]
    kb, rb = nd.batch_decompose(ctx, [g], "core", "snd", use_frontier=True)
    assert torch.equal(kb[0], want) and rb[0]["sweeps"] == rs["sweeps"]
    for mode in ("and",):
        k2, _ = g.decompose("core", mode, use_frontier=True)
        kb2, _ = nd.batch_decompose(ctx, [g], "core", mode, use_frontier=True)
        assert torch.equal(k2, want) and torch.equal(kb2[0], want)
    assert np.array_equal(want.cpu().numpy(), np.ones(n, np.int32))


def test_batch_max_iters(nd, ctx):
    raw = chung_lu(4096, 2.1, 16.0, seed=7)
    og = oracle.Graph.from_raw(raw)
    seq = og.snd(2, 3)
    g = make(nd, ctx, raw)
    with pytest.raises(nd.NdError) as e:
        nd.batch_decompose(ctx, [g], "truss", "snd", max_iters=2)
    assert e.value.name == "not_converged"


# -------------------------------------------------------------- serving


def test_server_results_equal_oracle_and_solo(nd, ctx):
    """Every served result equals the oracle's kappa (Alg. Peeling) and the
    graph's lone decomposition, whatever it shared launches with."""
    raws = mixed_graphs() + [chung_lu(int(n), 2.3, 10.0, seed=200 + i)
                             for i, n in enumerate(np.linspace(500, 30000, 20))]
    kinds = ["truss", "core", "nucleus13", "nucleus34", "nucleus24", "truss", "core",
             "nucleus34"]
    kinds += ["truss" if i % 2 else "core" for i in range(20)]
    modes = ["snd" if i % 3 else "and" for i in range(len(raws))]
    solo = [make(nd, ctx, raw).decompose(k, m)[0].cpu()
            for raw, k, m in zip(raws, kinds, modes)]
    srv = nd.Server(ctx, max_slots=8)
    tickets = []
    for i, (raw, k, m) in enumerate(zip(raws, kinds, modes)):
        tickets.append(srv.submit(make(nd, ctx, raw), k, m,
                                  use_frontier=i % 2 == 0))
        time.sleep(0.002)  # staggered arrivals: later ones join a running mix
    for t, want, raw, k in zip(tickets, solo, raws, kinds):
        kappa, res, info = srv.wait(t)
        assert torch.equal(kappa, want), raw.name
        r, s = KINDS[k]
        assert np.array_equal(kappa.numpy(), oracle.Graph.from_raw(raw).peel(r, s)), \
            (raw.name, k)
        assert res["converged"] == 1 and info["latency_ms"] > 0
        assert info["epoch_done"] >= info["epoch_joined"]
    srv.close()


def test_server_requests_overlap_on_the_device(nd, ctx):
    """Continuous batching: requests submitted while another is being swept
    join its batch (their epochs overlap, the batch sweeps them together),
    and the sweeps go on while a large newcomer is being prepared."""
    from synth import RawGraph
    n = 100000  # a path: k-core SND takes about n/2 sweeps
    path = RawGraph(n, np.arange(n - 1, dtype=np.int32),
                    np.arange(1, n, dtype=np.int32), "path")
    others = [chung_lu(3000 + 1000 * i, 2.2, 10.0, seed=500 + i) for i in range(4)]
    big = chung_lu(60000, 2.1, 24.0, seed=510)
    srv = nd.Server(ctx, max_slots=16)
    t_long = srv.submit(make(nd, ctx, path), "core", "snd")
    time.sleep(0.2)
    t_others = []
    for raw in others:
        t_others.append(srv.submit(make(nd, ctx, raw), "core", "snd"))
        time.sleep(0.01)
    t_big = srv.submit(make(nd, ctx, big), "truss", "snd")
    k_long, r_long, i_long = srv.wait(t_long)
    assert int(k_long.min()) == 1 and int(k_long.max()) == 1  # kappa of a path
    # on a path t* = floor((n-1)/2) (pinned in the oracle's tests); one more
    # sweep observes no change
    assert r_long["sweeps"] == (n - 1) // 2 + 1
    joined = 0
    for t, raw in zip(t_others, others):
        kappa, res, info = srv.wait(t)
        assert np.array_equal(kappa.numpy(), oracle.Graph.from_raw(raw).peel(1, 2))
        if info["joined_running"]:
            joined += 1
            # it joined the long request's batch while that one was running
            assert i_long["epoch_joined"] < info["epoch_joined"] < i_long["epoch_done"]
            assert info["peak_members"] >= 2
    assert joined >= 1
    assert i_long["peak_members"] >= 2
    kb, rb, ib = srv.wait(t_big)
    assert rb["converged"] == 1
    assert np.array_equal(kb.numpy(), oracle.Graph.from_raw(big).peel(2, 3))
    # the long request kept sweeping while the newcomer was being prepared
    assert ib["epochs_during_prep"] > 0 and ib["prep_ms"] > 0
    srv.close()


def test_server_beside_caller_work_on_the_legacy_stream(nd, ctx):
    """While a long request keeps the worker replaying its epoch graphs, the
    caller builds graphs and runs torch work on the legacy default stream;
    every request's result equals the oracle's."""
    from synth import RawGraph
    n = 12000
    path = RawGraph(n, np.arange(n - 1, dtype=np.int32),
                    np.arange(1, n, dtype=np.int32), "path")
    srv = nd.Server(ctx, max_slots=32)
    t_long = srv.submit(make(nd, ctx, path), "core", "snd")
    raws = [chung_lu(1500 + 100 * i, 2.2, 10.0, seed=700 + i) for i in range(24)]
    ts = []
    for raw in raws:
        x = torch.ones(1 << 16, device="cuda")
        torch.cuda.default_stream().synchronize()
        ts.append(srv.submit(make(nd, ctx, raw), "truss", "snd"))
        assert float(x.sum()) == float(1 << 16)
    for t, raw in zip(ts, raws):
        kappa, res, info = srv.wait(t)
        assert np.array_equal(kappa.numpy(), oracle.Graph.from_raw(raw).peel(2, 3))
    k_long, r_long, _ = srv.wait(t_long)
    assert r_long["sweeps"] == (n - 1) // 2 + 1 and int(k_long.max()) == 1
    srv.close()


def test_server_budget_admission_and_oom(nd):
    # a budget that holds about one graph at a time: requests wait for memory
    ctx = nd.Context(0, hbm_budget_bytes=96 << 20)
    raws = [chung_lu(30000, 2.2, 16.0, seed=300 + i) for i in range(6)]
    solo_ctx = nd.Context(0)
    solo = [make(nd, solo_ctx, raw).decompose("truss")[0].cpu() for raw in raws]
    srv = nd.Server(ctx, max_slots=4)
    ts = [srv.submit(make(nd, ctx, raw), "truss") for raw in raws]
    for t, want in zip(ts, solo):
        kappa, res, info = srv.wait(t)
        assert torch.equal(kappa, want)
    # a graph too large for the whole budget fails with OOM, alone
    big = chung_lu(300000, 2.1, 32.0, seed=399)
    try:
        g = make(nd, ctx, big)
    except nd.NdError as e:
        assert e.name == "oom"
    else:
        t = srv.submit(g, "truss")
        with pytest.raises(nd.NdError) as e:
            srv.wait(t)
        assert e.value.name == "oom"
    srv.close()


def test_server_cancel_and_busy(nd, ctx):
    srv = nd.Server(ctx, max_slots=1, max_queue=3)
    raws = [chung_lu(20000, 2.1, 24.0, seed=400 + i) for i in range(3)]
    ts = [srv.submit(make(nd, ctx, raw), "truss") for raw in raws]
    with pytest.raises(nd.NdError) as e:
        for i in range(4):
            srv.submit(make(nd, ctx, raws[0]), "truss")
    assert e.value.name == "busy"
    srv.cancel(ts[2])
    got = srv.wait(ts[0])
    assert got is not None
    with pytest.raises(nd.NdError) as e:
        srv.wait(ts[2])
    assert e.value.name == "cancelled"
    srv.close()
