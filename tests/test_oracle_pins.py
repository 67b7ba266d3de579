"""Pins for the CPU oracle: the paper's printed examples, closed forms,
library special cases and brute force.  CPU only."""

import itertools
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_examples.json")))


def named_graph(spec):
    names = spec["vertices"]
    ix = {v: i for i, v in enumerate(names)}
    src = [ix[a] for a, b in spec["edges"]]
    dst = [ix[b] for a, b in spec["edges"]]
    return names, ix, oracle.Graph(len(names), src, dst), src, dst


# ------------------------------------------------------------------ H


@pytest.mark.parametrize("case", GOLD["hindex_printed"],
                         ids=lambda c: str(c["K"]))
def test_hindex_printed_values(case):
    assert oracle.hindex(case["K"]) == case["H"]


def test_hindex_definition_random():
    rng = np.random.default_rng(0)
    for _ in range(2000):
        n = int(rng.integers(0, 25))
        K = rng.integers(0, 30, size=n)
        assert oracle.hindex(K) == brute.hindex_def(K)


def test_hindex_special_cases():
    assert oracle.hindex([]) == 0
    assert oracle.hindex([0, 0, 0]) == 0
    assert oracle.hindex([7] * 7) == 7
    assert oracle.hindex([100] * 5) == 5          # bounded by |K|
    assert oracle.hindex(list(range(1, 11))) == 5  # 5 values >= 5, not 6 >= 6


# ------------------------------------------------- k-core worked example


def test_core_example_snd():
    spec = GOLD["core_example"]
    pr = spec["printed"]
    names, ix, g, _, _ = named_graph(spec)
    seq = g.snd(1, 2)
    tau0, tau1, tau2 = seq[0], seq[1], seq[2]
    for v, d in pr["tau0_of_neighbours_of_a"].items():
        assert tau0[ix[v]] == d
    for v, t in pr["snd_tau1"].items():
        assert tau1[ix[v]] == t
    changed = sorted(names[i] for i in np.nonzero(tau1 != tau0)[0])
    assert changed == sorted(pr["snd_updated_in_iteration_1"])
    for v, t in pr["snd_tau2"].items():
        assert tau2[ix[v]] == t
    # tau_2 is the first iterate equal to kappa; tau_3 repeats it.
    t_star = pr["snd_iterations_to_converge"]
    assert len(seq) == t_star + 2
    assert np.array_equal(seq[t_star], seq[t_star + 1])
    assert np.array_equal(seq[t_star], g.peel(1, 2))


def test_core_example_levels():
    spec = GOLD["core_example"]
    names, ix, g, _, _ = named_graph(spec)
    lv, nl = g.levels(1, 2)
    for v, l in spec["printed"]["levels"].items():
        assert lv[ix[v]] == l
    assert nl == 4


@pytest.mark.parametrize("which", ["level", "natural"])
def test_core_example_and_orders(which):
    spec = GOLD["core_example"]
    pr = spec["printed"]
    names, ix, g, _, _ = named_graph(spec)
    order = [ix[v] for v in pr[f"and_{which}_order"]]
    kappa = g.peel(1, 2)
    tau, sweeps, seq = g.and_run(1, 2, order=order)
    assert np.array_equal(tau, kappa)
    t_star = pr[f"and_{which}_order_iterations"]
    # converged after t_star sweeps; one more sweep sees no change
    assert sweeps == t_star + 1
    assert np.array_equal(seq[t_star], kappa)
    assert not np.array_equal(seq[t_star - 1], kappa)
    if which == "level":
        assert seq[1][ix["a"]] == pr["and_level_order_tau1_a"]
    else:
        upd = sorted(names[i] for i in np.nonzero(seq[2] != seq[1])[0])
        assert upd == pr["and_natural_only_update_in_iteration_2"]


def test_core_example_notifications():
    """Section 4.3's example: Alg. AND with notifications in the order
    a..f takes 9 tau computations in 3 iterations, only `a` being active
    after the first; the result is kappa."""
    spec = GOLD["core_example"]
    pr = spec["printed"]
    names, ix, g, _, _ = named_graph(spec)
    order = [ix[v] for v in pr["and_natural_order"]]
    tau, iters, comps, active = g.and_notify(1, 2, order=order)
    assert sum(comps) == pr["notification_tau_computations"]
    assert iters == pr["notification_iterations"]
    assert comps == [6, 1, 2] and active[0] == 1
    assert np.array_equal(tau, g.peel(1, 2))
    # with the listing's self-activation the printed counts do not hold
    _, iters_sa, comps_sa, _ = g.and_notify(1, 2, order=order,
                                           self_activate=True)
    assert sum(comps_sa) != pr["notification_tau_computations"]


# ------------------------------------------------ k-truss worked example


def test_truss_example():
    spec = GOLD["truss_example"]
    pr = spec["printed"]
    names, ix, g, _, _ = named_graph(spec)
    E = g.rcliques(2)
    eix = {names[a] + names[b]: i for i, (a, b) in enumerate(E)}
    seq = g.snd(2, 3)
    for e, t in pr["tau0"].items():
        assert seq[0][eix["".join(sorted(e))]] == t
    for e, t in pr["tau1"].items():
        assert seq[1][eix[e]] == t
    # the rho multisets printed for bc and ae
    for e, key in (("bc", "rho_bc"), ("ae", "rho_ae")):
        mem = g.members(2, 3, eix[e])
        rho = sorted((min(seq[0][m] for m in row) for row in mem), reverse=True)
        assert rho == sorted(pr[key], reverse=True)
    t_star = pr["snd_iterations_to_converge"]
    assert len(seq) == t_star + 2
    assert np.array_equal(seq[t_star], g.peel(2, 3))


# -------------------------------------------------------- closed forms


def complete(n):
    a, b = zip(*itertools.combinations(range(n), 2)) if n > 1 else ((), ())
    return oracle.Graph(n, list(a), list(b))


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7])
def test_complete_graph(n):
    g = complete(n)
    for (r, s), val in (((1, 2), n - 1), ((2, 3), n - 2), ((3, 4), n - 3)):
        if g.num_rcliques(r) == 0:
            continue
        kappa = g.peel(r, s)
        assert (kappa == val).all(), (r, s)
        # K_n is S-degree-regular: SND never changes anything
        assert len(g.snd(r, s)) == 2


@pytest.mark.parametrize("n", [4, 5, 9, 16])
def test_cycle(n):
    src = list(range(n))
    dst = [(i + 1) % n for i in range(n)]
    g = oracle.Graph(n, src, dst)
    assert (g.peel(1, 2) == 2).all()
    assert (g.peel(2, 3) == 0).all()


def test_triangle_is_k3():
    g = oracle.Graph(3, [0, 1, 2], [1, 2, 0])
    assert (g.peel(2, 3) == 1).all()
    assert g.num_rcliques(3) == 1 and (g.peel(3, 4) == 0).all()


@pytest.mark.parametrize("a,b", [(1, 1), (2, 3), (3, 3), (4, 7)])
def test_complete_bipartite(a, b):
    src, dst = zip(*[(i, a + j) for i in range(a) for j in range(b)])
    g = oracle.Graph(a + b, src, dst)
    assert (g.peel(1, 2) == min(a, b)).all()
    assert (g.peel(2, 3) == 0).all()


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7, 8, 11, 20])
def test_path_kappa_and_iterations(n):
    """P_n: core number 1 everywhere.  The value 1 enters at the two ends
    and moves one vertex inward per SND iteration, so the vertex farthest from
    both ends, at distance floor((n-1)/2), is exact first at that iteration."""
    g = oracle.Graph(n, list(range(n - 1)), list(range(1, n)))
    seq = g.snd(1, 2)
    kappa = g.peel(1, 2)
    assert (kappa == 1).all()
    t_star = (n - 1) // 2
    assert np.array_equal(seq[t_star], kappa)
    if t_star > 0:
        assert not np.array_equal(seq[t_star - 1], kappa)
    assert len(seq) == t_star + 2


def test_petersen_regular_triangle_free():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    src, dst = zip(*(outer + spokes + inner))
    g = oracle.Graph(10, src, dst)
    assert (g.peel(1, 2) == 3).all()
    assert len(g.snd(1, 2)) == 2         # d-regular: tau_0 = kappa
    assert (g.peel(2, 3) == 0).all()      # no triangles
    assert len(g.snd(2, 3)) == 2


def test_star():
    g = oracle.Graph(9, [0] * 8, list(range(1, 9)))
    assert (g.peel(1, 2) == 1).all()


def test_empty_and_isolated():
    g = oracle.Graph(0, [], [])
    assert g.num_rcliques(1) == 0 and g.peel(1, 2).size == 0
    g = oracle.Graph(5, [], [])
    assert (g.peel(1, 2) == 0).all()
    assert g.num_rcliques(2) == 0


# ---------------------------------------------------- canonicalisation


def test_canonical_csr_matches_set_construction():
    rng = np.random.default_rng(3)
    n, m = 60, 400
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    src[:10] = dst[:10]  # some self-loops
    src = np.concatenate([src, dst[:30]])  # some reversed repeats
    dst = np.concatenate([dst, src[:30]])
    g = oracle.Graph(n, src, dst)
    row_off, col = g.csr()
    E = brute.simple_edges(n, src, dst)
    adj = {v: sorted([b for a, b in E if a == v] + [a for a, b in E if b == v])
           for v in range(n)}
    assert row_off[0] == 0 and row_off[-1] == 2 * len(E)
    for v in range(n):
        assert list(col[row_off[v]:row_off[v + 1]]) == adj[v]


def test_invalid_ids_rejected():
    with pytest.raises(ValueError):
        oracle.Graph(3, [0, 5], [1, 2])
    with pytest.raises(ValueError):
        oracle.Graph(3, [-1], [1])


# ---------------------------------------------------------- networkx


def _random_graph(n, p, seed):
    rng = np.random.default_rng(seed)
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < p
    return iu[keep], ju[keep]


@pytest.mark.parametrize("seed", range(6))
def test_core_numbers_match_networkx(seed):
    nx = pytest.importorskip("networkx")
    n = 120
    src, dst = _random_graph(n, 0.06 + 0.02 * seed, seed)
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from(zip(src.tolist(), dst.tolist()))
    ref = nx.core_number(G)
    g = oracle.Graph(n, src, dst)
    kappa = g.peel(1, 2)
    assert [ref[v] for v in range(n)] == kappa.tolist()
    assert np.array_equal(g.snd(1, 2)[-1], kappa)


@pytest.mark.parametrize("seed", range(4))
def test_truss_numbers_match_networkx(seed):
    """networkx.k_truss(G, k) is the maximal subgraph whose edges lie in at
    least k-2 triangles (Cohen's convention); the paper counts triangles
    directly (Section 2.1), so kappa_3(e) = max{k : e in k_truss(G, k+2)}."""
    nx = pytest.importorskip("networkx")
    n = 45
    src, dst = _random_graph(n, 0.25 + 0.05 * seed, 100 + seed)
    G = nx.Graph()
    G.add_edges_from(zip(src.tolist(), dst.tolist()))
    g = oracle.Graph(n, src, dst)
    E = g.rcliques(2)
    kappa = g.peel(2, 3)
    ref = np.zeros(len(E), np.int64)
    k = 0
    while True:
        T = nx.k_truss(G, k + 2)
        if T.number_of_edges() == 0:
            break
        for i, (a, b) in enumerate(E):
            if T.has_edge(int(a), int(b)):
                ref[i] = k
        k += 1
    assert ref.tolist() == kappa.tolist()


# --------------------------------------------------------- brute force


def _tiny_cases(r, max_r, count, seed):
    rng = np.random.default_rng(seed)
    got = 0
    while got < count:
        n = int(rng.integers(3, 8))
        p = float(rng.uniform(0.3, 0.95))
        src, dst = _random_graph(n, p, int(rng.integers(1 << 30)))
        g = oracle.Graph(n, src, dst)
        nr = g.num_rcliques(r)
        if 1 <= nr <= max_r:
            got += 1
            yield n, src, dst, g


@pytest.mark.parametrize("r,s", [(1, 2), (2, 3), (3, 4), (1, 3), (2, 4)])
def test_peeling_equals_lemma1_bruteforce(r, s):
    for n, src, dst, g in _tiny_cases(r, 13, 25, seed=10 * r + s):
        Rs, best = brute.kappa_bruteforce(n, src, dst, r, s)
        assert [tuple(x) for x in g.rcliques(r)] == Rs
        assert g.peel(r, s).tolist() == best
        assert g.snd(r, s)[-1].tolist() == best


@pytest.mark.parametrize("r,s", [(1, 2), (2, 3), (3, 4)])
def test_update_equals_definition_bruteforce(r, s):
    rng = np.random.default_rng(7 + r)
    for n, src, dst, g in _tiny_cases(r, 30, 20, seed=100 + r):
        nr = g.num_rcliques(r)
        tau = rng.integers(0, 6, nr).astype(np.int32)
        assert g.update(r, s, tau).tolist() == brute.update_def(n, src, dst,
                                                                r, s, tau)


@pytest.mark.parametrize("r,s", [(1, 2), (2, 3), (3, 4)])
def test_sdeg_and_members_bruteforce(r, s):
    for n, src, dst, g in _tiny_cases(r, 40, 15, seed=200 + r):
        E = brute.simple_edges(n, src, dst)
        Rs = brute.cliques(n, E, r)
        Ss = brute.cliques(n, E, s)
        idx = {R: i for i, R in enumerate(Rs)}
        ds = g.sdeg(r, s)
        for i, R in enumerate(Rs):
            want = sorted(
                tuple(idx[sub] for sub in itertools.combinations(S, r)
                      if sub != R)
                for S in Ss if set(R) <= set(S))
            got = sorted(tuple(row) for row in g.members(r, s, i))
            assert got == want
            assert ds[i] == len(want)
