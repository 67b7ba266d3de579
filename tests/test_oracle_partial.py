"""PartialAND (Section 4.3, end) and its ego-network estimates (Section 5.3
application) in the oracle, pinned against what the definitions fix.  CPU
only.

* P = every r-clique: PartialAND is AND itself, whose limit is kappa
  (Section 4.2); compared with Alg. Peeling.
* P = {R}: the other r-cliques keep tau_0 = d_s, so the result is one
  application of U to d_s at R, by the brute-force definition of U.
* Tiny sets: the result is the largest fixed point of U restricted to P
  below d_s, found by enumerating every tau on P between 0 and d_s.
* kappa <= estimate <= d_s, and a larger set never gives a larger value.
"""

import itertools

import numpy as np
import pytest

import oracle
from oracle.brute import update_def
from synth import RawGraph, chung_lu, erdos_renyi, sbm

KINDS = [(1, 2), (2, 3), (3, 4)]


def small_graphs():
    yield "er", erdos_renyi(60, 0.15, seed=21)
    yield "cl", chung_lu(300, 2.1, 9.0, seed=22)
    yield "sbm", sbm(n_comm=8, size_lo=5, size_hi=10, p_in=0.7, p_out=0.02,
                     seed=23)


@pytest.mark.parametrize("name,raw", list(small_graphs()),
                         ids=lambda x: x if isinstance(x, str) else "")
@pytest.mark.parametrize("r,s", KINDS)
def test_full_set_is_kappa(name, raw, r, s):
    g = oracle.Graph.from_raw(raw)
    nr = g.num_rcliques(r)
    tau, sweeps, conv = g.partial_and(r, s, np.arange(nr))
    assert conv
    assert np.array_equal(tau, g.peel(r, s))


@pytest.mark.parametrize("r,s", KINDS)
def test_single_rclique_is_one_update(r, s):
    raw = erdos_renyi(14, 0.55, seed=24)
    g = oracle.Graph.from_raw(raw)
    nr = g.num_rcliques(r)
    ds = g.sdeg(r, s)
    want = update_def(raw.n, raw.src, raw.dst, r, s, list(ds))
    for R in range(0, nr, max(1, nr // 12)):
        tau, sweeps, conv = g.partial_and(r, s, [R])
        assert conv and tau[R] == want[R]
        others = np.ones(nr, bool)
        others[R] = False
        assert np.array_equal(tau[others], ds[others])


def greatest_fixed_point(raw, r, s, P, ds):
    """Enumerate every tau on P with 0 <= tau <= d_s (others at d_s); keep
    those fixed by U on P; return their componentwise maximum."""
    fixed = []
    for vals in itertools.product(*[range(ds[p] + 1) for p in P]):
        tau = list(ds)
        for p, v in zip(P, vals):
            tau[p] = v
        u = update_def(raw.n, raw.src, raw.dst, r, s, tau)
        if all(u[p] == tau[p] for p in P):
            fixed.append(vals)
    top = tuple(max(v[i] for v in fixed) for i in range(len(P)))
    assert top in fixed  # the fixed points form a lattice
    return top


@pytest.mark.parametrize("r,s", [(1, 2), (2, 3)])
def test_tiny_sets_match_enumeration(r, s):
    # two triangles sharing an edge plus a pendant path: small d_s everywhere
    pairs = [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3), (3, 4), (4, 5), (2, 5)]
    raw = RawGraph(6, np.array([a for a, b in pairs], np.int32),
                   np.array([b for a, b in pairs], np.int32), "tiny")
    g = oracle.Graph.from_raw(raw)
    ds = g.sdeg(r, s)
    nr = g.num_rcliques(r)
    rng = np.random.default_rng(25)
    for size in (2, 3, 4):
        for _ in range(3):
            P = sorted(rng.choice(nr, size=min(size, nr), replace=False).tolist())
            tau, _, conv = g.partial_and(r, s, P)
            assert conv
            assert tuple(int(tau[p]) for p in P) == \
                greatest_fixed_point(raw, r, s, P, list(ds))


@pytest.mark.parametrize("r,s", KINDS)
def test_ego_estimates_bounded_and_monotone(r, s):
    raw = chung_lu(500, 2.2, 10.0, seed=26)
    g = oracle.Graph.from_raw(raw)
    nr = g.num_rcliques(r)
    kappa = g.peel(r, s)
    ds = g.sdeg(r, s)
    qs = np.random.default_rng(27).integers(0, nr, size=25)
    est, _ = g.ego_estimate(r, s, qs)
    assert (est >= kappa[qs]).all() and (est <= ds[qs]).all()
    for q in qs[:8]:
        P1 = g.ego_set(r, s, int(q))
        # a superset: the ego sets of q's ego set
        P2 = np.unique(np.concatenate([g.ego_set(r, s, int(x)) for x in P1]))
        t1, _, _ = g.partial_and(r, s, P1)
        t2, _, _ = g.partial_and(r, s, P2)
        assert (t2[P1] <= t1[P1]).all()
        assert (t2[P1] >= kappa[P1]).all()


def test_ego_set_is_neighbourhood():
    raw = erdos_renyi(40, 0.2, seed=28)
    g = oracle.Graph.from_raw(raw)
    # r = 1: the vertex and its neighbours
    off, col = g.csr()
    for u in range(0, 40, 7):
        want = np.unique(np.concatenate([[u], col[off[u]:off[u + 1]]]))
        assert np.array_equal(g.ego_set(1, 2, u), want)
