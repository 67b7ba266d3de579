"""The paper's theorems as invariants of the oracle's iterates.  CPU only.

Theorem 1 (monotonicity, lower bound), Theorem 2 (kappa non-decreasing over
degree levels), Theorem 3 (level i exact from iteration i on), Lemma 2
(convergence within the last level index), and the asynchronous variant's
guarantees of Section 4.2 (never more iterations than SND; every sweep's
values lie between kappa and the synchronous iterate).
"""

import numpy as np
import pytest

import oracle
from synth import chung_lu, erdos_renyi, sbm

KINDS = [(1, 2), (2, 3), (3, 4)]


def graphs():
    yield "er", erdos_renyi(150, 0.08, seed=11)
    yield "cl", chung_lu(400, 2.1, 10.0, seed=12)
    yield "sbm", sbm(n_comm=12, size_lo=6, size_hi=14, p_in=0.6, p_out=0.01,
                     seed=13)


@pytest.mark.parametrize("name,raw", list(graphs()), ids=lambda x: x if
                         isinstance(x, str) else "")
@pytest.mark.parametrize("r,s", KINDS)
def test_theorems(name, raw, r, s):
    g = oracle.Graph.from_raw(raw)
    if g.num_rcliques(r) == 0:
        pytest.skip("no r-cliques")
    kappa = g.peel(r, s)
    seq = g.snd(r, s)
    ds = seq[0]
    assert np.array_equal(seq[-1], kappa)
    # Theorem 1: tau_{t+1} <= tau_t and tau_t >= kappa
    for a, b in zip(seq, seq[1:]):
        assert (b <= a).all()
    for t in seq:
        assert (t >= kappa).all()
    # fixed point: U kappa = kappa
    assert np.array_equal(g.update(r, s, kappa), kappa)
    # Theorem 2 and Theorem 3 with the degree levels
    lv, nl = g.levels(r, s)
    order = np.lexsort((np.arange(lv.size), lv))
    assert (np.diff(kappa[order]) >= 0).all()
    for t, tau in enumerate(seq):
        sel = lv <= t
        assert np.array_equal(tau[sel], kappa[sel])
    # Lemma 2: the first exact iterate comes no later than the last level
    t_star = next(t for t, tau in enumerate(seq) if np.array_equal(tau, kappa))
    assert t_star <= nl - 1
    # level-0 r-cliques have minimum degree and are exact at tau_0
    assert (ds[lv == 0] == ds.min()).all()
    # Section 4.2: AND in natural order
    tau_and, sweeps, aseq = g.and_run(r, s)
    assert np.array_equal(tau_and, kappa)
    assert sweeps <= len(seq) - 1
    for t, at in enumerate(aseq):
        st = seq[min(t, len(seq) - 1)]
        assert (at >= kappa).all() and (at <= st).all()


@pytest.mark.parametrize("r,s", KINDS)
def test_and_random_orders(r, s):
    raw = chung_lu(300, 2.2, 12.0, seed=21)
    g = oracle.Graph.from_raw(raw)
    kappa = g.peel(r, s)
    snd_sweeps = len(g.snd(r, s)) - 1
    rng = np.random.default_rng(5)
    for _ in range(4):
        order = rng.permutation(kappa.size)
        tau, sweeps, _ = g.and_run(r, s, order=order)
        assert np.array_equal(tau, kappa)
        assert sweeps <= snd_sweeps


@pytest.mark.parametrize("r,s", KINDS)
def test_resume_from_iterate(r, s):
    """Restarting SND from any iterate tau_t reproduces the rest bit for bit
    (the iteration is a function of the current iterate only)."""
    raw = erdos_renyi(120, 0.12, seed=31)
    g = oracle.Graph.from_raw(raw)
    seq = g.snd(r, s)
    for t in range(len(seq) - 1):
        assert np.array_equal(g.update(r, s, seq[t]), seq[t + 1])


def test_update_range_and_threads_agree():
    raw = chung_lu(500, 2.1, 12.0, seed=41)
    g = oracle.Graph.from_raw(raw)
    tau = g.sdeg(2, 3)
    full1 = g.update(2, 3, tau, threads=1)
    full8 = g.update(2, 3, tau, threads=8)
    assert np.array_equal(full1, full8)
    part = g.update(2, 3, tau, lo=100, hi=400)
    assert np.array_equal(part[100:400], full1[100:400])
    assert np.array_equal(part[:100], tau[:100])


@pytest.mark.parametrize("name,raw", list(graphs()), ids=lambda x: x if
                         isinstance(x, str) else "")
@pytest.mark.parametrize("r,s", KINDS)
def test_and_with_notifications(name, raw, r, s):
    """Alg. AND with notifications (Section 4.3) reaches kappa, with no more
    computations than the same sweeps would take without notifications, and
    every computation after the first iteration is of an r-clique a
    neighbour's change made active; in id order its iterations bound the
    plain in-place sweeps'."""
    g = oracle.Graph.from_raw(raw)
    nr = g.num_rcliques(r)
    if nr == 0:
        pytest.skip("no r-cliques")
    kappa = g.peel(r, s)
    tau, iters, comps, active = g.and_notify(r, s)
    assert np.array_equal(tau, kappa)
    assert comps[0] == nr and all(c <= nr for c in comps)
    # the work of iteration i+1 is exactly what was active after iteration i
    assert comps[1:] == active[:-1]
    assert active[-1] == 0 or iters == len(comps)
    _, sweeps, _ = g.and_run(r, s)
    assert sum(comps) <= sweeps * nr
    # a reversed visiting order reaches the same kappa
    tau_rev, _, _, _ = g.and_notify(r, s, order=np.arange(nr)[::-1])
    assert np.array_equal(tau_rev, kappa)
