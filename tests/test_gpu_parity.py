"""Parity of the HIP library (through the C ABI) with the CPU oracle.

Every comparison is bit-exact: canonical CSR, r-clique lists, S-degrees,
incidence lists (as sets), one application of U on arbitrary inputs, every
SND iterate, and the converged kappa of SND and AND.
"""

import math

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


def gpu_graph(nd, ctx, raw):
    return nd.Graph.from_edges(ctx, raw.n, torch.from_numpy(raw.src),
                               torch.from_numpy(raw.dst))


def canon_incidence(off, ids):
    """Per r-clique, the multiset of s-cliques (each a sorted id tuple), in a
    canonical order: returns (R index per row, sorted rows)."""
    off = np.asarray(off, np.int64)
    ids = np.sort(np.asarray(ids), axis=1)
    rid = np.repeat(np.arange(off.size - 1), np.diff(off))
    keys = [ids[:, j] for j in range(ids.shape[1] - 1, -1, -1)] + [rid]
    order = np.lexsort(keys)
    return rid[order], ids[order]


def oracle_incidence(og, r, s):
    nr = og.num_rcliques(r)
    rows, off = [], [0]
    for R in range(nr):
        m = og.members(r, s, R)
        rows.append(m)
        off.append(off[-1] + m.shape[0])
    k = math.comb(s, r) - 1
    ids = np.concatenate(rows) if rows else np.zeros((0, k), np.int32)
    return np.array(off), ids.reshape(-1, k)


SMALL = [
    ("er2000", lambda: erdos_renyi(2000, 0.005, seed=1)),
    ("cl4k", lambda: chung_lu(4096, 2.1, 16.0, seed=7)),
    ("sbm40", lambda: sbm(n_comm=40, size_lo=10, size_hi=40, p_in=0.3,
                          p_out=0.002, seed=9)),
    # spine edges (and vertices) with S-degree 400 / 800 / 1600: one r-clique
    # in each of the 8-, 16- and 32-values-per-lane bins of the sweep
    ("books", lambda: books(pages=(400, 800, 1600), page_degree=8.0, seed=5)),
]


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
def test_canonical_csr(nd, ctx, name, make):
    raw = make()
    # add loops and reversed repeats to exercise canonicalisation
    src = np.concatenate([raw.src, raw.src[:50], np.arange(20, dtype=np.int32)])
    dst = np.concatenate([raw.dst, raw.dst[:50], np.arange(20, dtype=np.int32)])
    src[-70:-20], dst[-70:-20] = raw.dst[:50], raw.src[:50]
    g = nd.Graph.from_edges(ctx, raw.n, torch.from_numpy(src),
                            torch.from_numpy(dst))
    og = oracle.Graph(raw.n, src, dst)
    ro, col = g.csr()
    oro, ocol = og.csr()
    assert np.array_equal(ro.cpu().numpy(), oro)
    assert np.array_equal(col.cpu().numpy(), ocol)


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
@pytest.mark.parametrize("kind", list(KINDS))
def test_rcliques_sdeg_incidence(nd, ctx, name, make, kind):
    raw = make()
    r, s = KINDS[kind]
    g = gpu_graph(nd, ctx, raw)
    og = oracle.Graph.from_raw(raw)
    rc = g.rcliques(kind).cpu().numpy()
    assert np.array_equal(rc, og.rcliques(r))
    ds = g.sdegree(kind).cpu().numpy()
    assert np.array_equal(ds, og.sdeg(r, s))
    off, ids = g.incidence(kind)
    goff, gids = off.cpu().numpy(), ids.cpu().numpy()
    assert np.array_equal(np.diff(goff), ds)
    ooff, oids = oracle_incidence(og, r, s)
    a = canon_incidence(goff, gids)
    b = canon_incidence(ooff, oids)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
@pytest.mark.parametrize("kind", list(KINDS))
def test_update_arbitrary_tau(nd, ctx, name, make, kind):
    raw = make()
    r, s = KINDS[kind]
    g = gpu_graph(nd, ctx, raw)
    og = oracle.Graph.from_raw(raw)
    ds = og.sdeg(r, s)
    rng = np.random.default_rng(17)
    for trial in range(3):
        tau = (rng.random(ds.size) * (ds + 1)).astype(np.int32)
        tau = np.minimum(tau, ds)
        got = g.update(kind, torch.from_numpy(tau)).cpu().numpy()
        assert np.array_equal(got, og.update(r, s, tau)), trial


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
@pytest.mark.parametrize("kind", list(KINDS))
@pytest.mark.parametrize("frontier", [False, True], ids=["full", "frontier"])
def test_snd_every_iterate_and_kappa(nd, ctx, name, make, kind, frontier):
    """Every SND iterate equals the oracle's; with the notification frontier
    (Section 4.3) the iterates are the same, only fewer r-cliques are
    recomputed."""
    raw = make()
    r, s = KINDS[kind]
    g = gpu_graph(nd, ctx, raw)
    og = oracle.Graph.from_raw(raw)
    seq = og.snd(r, s)  # tau_0 .. tau_T, tau_T == tau_{T-1}
    its = []
    kappa, res = g.decompose(kind, "snd", keep_iterates=its,
                             use_frontier=frontier)
    kappa = kappa.cpu().numpy()
    assert res["converged"] == 1
    if og.num_rcliques(r) == 0:
        assert res["sweeps"] == 0
        return
    assert res["sweeps"] == len(seq) - 1 == len(its)
    for t, (changed, tau) in enumerate(its, start=1):
        want = seq[t]
        assert np.array_equal(tau.cpu().numpy(), want), f"iterate {t}"
        assert changed == int((seq[t] != seq[t - 1]).sum())
    assert np.array_equal(kappa, og.peel(r, s))


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
@pytest.mark.parametrize("kind", list(KINDS))
@pytest.mark.parametrize("frontier", [False, True], ids=["full", "frontier"])
def test_and_converges_to_kappa(nd, ctx, name, make, kind, frontier):
    raw = make()
    r, s = KINDS[kind]
    g = gpu_graph(nd, ctx, raw)
    og = oracle.Graph.from_raw(raw)
    if og.num_rcliques(r) == 0:
        pytest.skip("no r-cliques")
    seq = og.snd(r, s)
    kref = og.peel(r, s)
    its = []
    kappa, res = g.decompose(kind, "and", keep_iterates=its,
                             use_frontier=frontier)
    assert np.array_equal(kappa.cpu().numpy(), kref)
    assert res["converged"] == 1
    # never more sweeps than SND; every AND iterate between kappa and SND's
    assert res["sweeps"] <= len(seq) - 1
    for t, (_, tau) in enumerate(its, start=1):
        a = tau.cpu().numpy()
        assert (a >= kref).all() and (a <= seq[min(t, len(seq) - 1)]).all()


def test_snd_deterministic_and_chunked(nd, ctx):
    raw = chung_lu(8192, 2.1, 24.0, seed=23)
    g = gpu_graph(nd, ctx, raw)
    k1, r1 = g.decompose("truss", "snd")
    k2, r2 = g.decompose("truss", "snd")
    its = []
    k3, r3 = g.decompose("truss", "snd", keep_iterates=its)
    assert torch.equal(k1, k2) and torch.equal(k1, k3)
    assert r1["sweeps"] == r2["sweeps"] == r3["sweeps"]
    k4, _ = g.decompose("truss", "and")
    assert torch.equal(k1, k4)
    k5, r5 = g.decompose("truss", "snd", use_frontier=True)
    assert torch.equal(k1, k5) and r5["sweeps"] == r1["sweeps"]
    assert r5["updates"] < r1["updates"]  # the frontier skips idle r-cliques


def test_max_iters_returns_iterate(nd, ctx):
    raw = chung_lu(4096, 2.1, 16.0, seed=7)
    g = gpu_graph(nd, ctx, raw)
    og = oracle.Graph.from_raw(raw)
    seq = og.snd(2, 3)
    assert len(seq) > 3
    tau, res = g.decompose("truss", "snd", max_iters=2,
                           allow_not_converged=True)
    assert res["converged"] == 0 and res["sweeps"] == 2
    assert np.array_equal(tau.cpu().numpy(), seq[2])
    with pytest.raises(nd.NdError) as e:
        g.decompose("truss", "snd", max_iters=2)
    assert e.value.name == "not_converged"


def expected_active(og, r, s, seq):
    """Active r-cliques after each SND sweep t = 1, 2, ... (Section 4.3):
    those the library's notifications flag for sweep t+1 -- every r-clique
    that changed at sweep t, and every member R' of an s-clique of a changed
    R with h < tau_{t-1}(R') <= tau_{t-1}(R) and tau_{t-1}(Q) >= tau_{t-1}(R')
    for the other members Q (the rule checked against the oracle's iterates
    in test_notify_rule)."""
    from test_notify_rule import marked, pairs
    R, O = pairs(og, r, s)
    s64 = [x.astype(np.int64) for x in seq]
    return [int((marked(R, O, s64[t - 1], s64[t], False)
                 | (s64[t] != s64[t - 1])).sum()) for t in range(1, len(s64))]


@pytest.mark.parametrize("kind", ["core", "truss", "nucleus34"])
def test_active_counts_and_stop_ratio(nd, ctx, kind):
    """The active-ratio indicator (Section 5.1.4): each sweep's count of
    active r-cliques equals the notification rule's on the oracle's
    iterates, with and without the frontier (with it, exactly the next
    sweep's evaluated count); stop_active_ratio stops after the first sweep
    whose active / |R| falls below the ratio, returning that iterate."""
    raw = chung_lu(4096, 2.1, 16.0, seed=7)
    r, s = KINDS[kind]
    g = gpu_graph(nd, ctx, raw)
    og = oracle.Graph.from_raw(raw)
    seq = og.snd(r, s)
    nr = seq[0].size
    active = expected_active(og, r, s, seq)
    assert active[-1] == 0
    for fr in (False, True):
        st = []
        kappa, res = g.decompose(kind, "snd", use_frontier=fr, count_active=True,
                                 keep_stats=st)
        assert np.array_equal(kappa.cpu().numpy(), seq[-1])
        assert [x["active_next"] for x in st] == active, fr
        assert [x["changed"] for x in st] == \
            [int((seq[t] != seq[t - 1]).sum()) for t in range(1, len(seq))]
        if fr:
            assert [x["evaluated"] for x in st[1:]] == active[:-1]
    st = []
    g.decompose(kind, "snd", keep_stats=st)  # not counted unless asked
    assert all(x["active_next"] == -1 for x in st)
    for ratio in (0.4, 0.1, 0.01):
        want_t = next(i + 1 for i, a in enumerate(active) if a < ratio * nr)
        for fr in (False, True):
            tau, res = g.decompose(kind, "snd", stop_active_ratio=ratio,
                                   use_frontier=fr)
            assert res["sweeps"] == want_t, (ratio, fr)
            assert np.array_equal(tau.cpu().numpy(), seq[want_t])


@pytest.mark.parametrize("kind", ["core", "truss", "nucleus34"])
def test_and_active_counts(nd, ctx, kind):
    """AND with the frontier: the active count after a sweep is exactly what
    the next sweep recomputes, and the result is kappa."""
    raw = chung_lu(4096, 2.1, 16.0, seed=8)
    r, s = KINDS[kind]
    g = gpu_graph(nd, ctx, raw)
    kref = oracle.Graph.from_raw(raw).peel(r, s)
    st = []
    kappa, res = g.decompose(kind, "and", use_frontier=True, count_active=True,
                             keep_stats=st)
    assert np.array_equal(kappa.cpu().numpy(), kref)
    assert [x["evaluated"] for x in st[1:]] == [x["active_next"] for x in st[:-1]]
    assert st[-1]["active_next"] == 0


# ----------------------------------------------------------- edge cases


def edges_graph(nd, ctx, n, pairs):
    src = np.array([a for a, b in pairs], np.int32)
    dst = np.array([b for a, b in pairs], np.int32)
    return (nd.Graph.from_edges(ctx, n, torch.from_numpy(src),
                                torch.from_numpy(dst)),
            oracle.Graph(n, src, dst))


EDGE_CASES = {
    "empty": (0, []),
    "isolated": (7, []),
    "single_edge": (2, [(0, 1)]),
    "loops_only": (3, [(0, 0), (1, 1), (2, 2)]),
    "k6": (6, [(a, b) for a in range(6) for b in range(a + 1, 6)]),
    "k40": (40, [(a, b) for a in range(40) for b in range(a + 1, 40)]),
    # hub of degree 20000 > 16384 bins: coarse-then-fine histogram path
    "star20000": (20001, [(0, i) for i in range(1, 20001)]),
    # hub of degree 40000 >= 32768: k-core tau stored in 32 bits
    "star40000": (40001, [(0, i) for i in range(1, 40001)]),
    # K_{40,20000} plus a 60-clique joined to vertex 0, whose degree
    # 20060 takes the coarse path with a large H
    "bipartite_hub": (20100, [(a, 100 + b) for a in range(40) for b in range(20000)]
                      + [(40 + a, 40 + b) for a in range(60) for b in range(a + 1, 60)]
                      + [(0, 40 + a) for a in range(60)]),
    # an edge in 3000 triangles, a triangle in 3000 4-cliques (workgroup bins)
    "book3000": (3003, [(0, 1), (0, 2), (1, 2)] + [(x, 3 + i) for i in range(3000)
                                                    for x in (0, 1, 2)]),
}


@pytest.mark.parametrize("case", list(EDGE_CASES))
@pytest.mark.parametrize("kind", list(KINDS))
def test_edge_cases(nd, ctx, case, kind):
    n, pairs = EDGE_CASES[case]
    r, s = KINDS[kind]
    g, og = edges_graph(nd, ctx, n, pairs)
    nr = og.num_rcliques(r)
    want = og.peel(r, s)
    for mode in ("snd", "and"):
        for fr in (False, True):
            kappa, res = g.decompose(kind, mode, use_frontier=fr)
            assert res["converged"] == 1
            assert np.array_equal(kappa.cpu().numpy(), want), (mode, fr)
    assert g.sizes(kind)[0] == nr
    if nr:
        ds = og.sdeg(r, s)
        tau = np.minimum(np.arange(nr, dtype=np.int32) % 7, ds).astype(np.int32)
        assert np.array_equal(g.update(kind, torch.from_numpy(tau)).cpu().numpy(),
                              og.update(r, s, tau))


def test_invalid_inputs(nd, ctx):
    with pytest.raises(nd.NdError) as e:
        nd.Graph.from_edges(ctx, 3, torch.tensor([0, 5]), torch.tensor([1, 2]))
    assert e.value.name == "invalid"
    ro = torch.tensor([0, 1, 3, 4], dtype=torch.int64)
    col = torch.tensor([1, 0, 2, 1], dtype=torch.int32)
    g = nd.Graph.from_csr(ctx, 3, ro, col)
    assert g.dims() == (3, 4)
    bad = {
        "unsorted": ([0, 1, 3, 4], [1, 2, 0, 1]),
        "asymmetric": ([0, 1, 2, 3], [1, 2, 1]),
        "self_loop": ([0, 2, 3, 4], [0, 1, 0, 1]),
        "out_of_range": ([0, 1, 3, 4], [1, 0, 7, 1]),
        "bad_offsets": ([0, 3, 1, 4], [1, 0, 2, 1]),
        "duplicate": ([0, 2, 4, 4], [1, 1, 0, 0]),
    }
    for name, (r, c) in bad.items():
        with pytest.raises(nd.NdError) as e:
            nd.Graph.from_csr(ctx, 3, torch.tensor(r, dtype=torch.int64),
                              torch.tensor(c, dtype=torch.int32))
        assert e.value.name == "invalid", name
    g2 = nd.Graph.from_edges(ctx, 4, torch.tensor([0, 1]), torch.tensor([1, 2]))
    with pytest.raises(nd.NdError):
        g2.update("core", torch.tensor([5, 0, 0, 0]))  # above d_s


def test_truss_builder_paths_agree(nd, ctx, monkeypatch):
    """The k-truss builder's three paths give every edge the same triangles:
    the default one (the 64-lane bin intersected per source with out(u) in
    LDS, its (u,w) sides counted and placed in LDS), the one without the
    LDS copy, and the one that intersects twice instead of recording the
    triangles.  The graph has about 9.3e4 oriented edges in the 64-lane
    bin; kappa and one application of U equal the oracle's."""
    raw = chung_lu(30000, 2.0, 40.0, seed=61)
    og = oracle.Graph.from_raw(raw)
    want = og.peel(2, 3)
    ne = og.num_rcliques(2)
    ds = og.sdeg(2, 3)
    canon = []
    for env in ({}, {"ND_TRUSS_NO_LDS": "1"}, {"ND_TRUSS_NO_TRIBUF": "1"}):
        with monkeypatch.context() as m:
            for k, v in env.items():
                m.setenv(k, v)
            g = gpu_graph(nd, ctx, raw)
            g.prepare("truss")
        off, ids = g.incidence("truss")
        rid = torch.repeat_interleave(torch.arange(ne, device=off.device),
                                      off[1:] - off[:-1])
        lo = torch.minimum(ids[:, 0], ids[:, 1]).long()
        hi = torch.maximum(ids[:, 0], ids[:, 1]).long()
        canon.append(torch.sort((rid * ne + lo) * ne + hi).values)
        kappa, res = g.decompose("truss", "snd", use_frontier=True)
        assert res["converged"] == 1
        assert np.array_equal(kappa.cpu().numpy(), want), env
        if not env:
            tau = np.minimum(np.arange(ne, dtype=np.int32) % 11, ds).astype(np.int32)
            assert np.array_equal(g.update("truss", torch.from_numpy(tau)).cpu().numpy(),
                                  og.update(2, 3, tau))
        g.close()
    assert canon[0].numel() == int(ds.sum())
    assert all(torch.equal(canon[0], c) for c in canon[1:])
