"""The notification rules of the frontier (Section 4.3) against the oracle's
SND iterates.  CPU only.

The library's synchronous sweeps with the frontier recompute, at sweep t+1,
every r-clique that changed at sweep t (self-activation) and every neighbour
R' that a changed R marks through an s-clique S with
    h < tau_t(R') <= tau_t(R)  and  tau_t(Q) >= tau_t(R') for the other Q of S
(h = tau_{t+1}(R)); in-place sweeps use the looser test h < tau(R') and
h <= tau(Q).  For the iterates to be exact, every r-clique whose value
changes at sweep t+1 has to be among those recomputed.  This checks that on
the oracle's iterates and incidence lists, for every kind, that the rules do
skip work (the frontier is not vacuous), and that the SND rule marks exactly
the members holding their s-clique's minimum rho when h < rho <= tau_t(R),
the form the device evaluates from the values it gathered.
"""

import numpy as np
import pytest

import oracle
from synth import chung_lu, erdos_renyi, sbm

KINDS = [(1, 2), (2, 3), (3, 4)]


def graphs():
    yield "er", erdos_renyi(150, 0.08, seed=21)
    yield "cl", chung_lu(600, 2.1, 12.0, seed=22)
    yield "sbm", sbm(n_comm=10, size_lo=8, size_hi=16, p_in=0.6, p_out=0.02,
                     seed=23)


def pairs(g, r, s):
    """(R, others) per incidence: R repeated, the k other r-cliques of S."""
    nr = g.num_rcliques(r)
    own, oth = [], []
    for R in range(nr):
        m = g.members(r, s, R)
        own.append(np.full(len(m), R, np.int64))
        oth.append(m.astype(np.int64))
    k = oth[0].shape[1] if oth else 0
    if not own:
        return np.zeros(0, np.int64), np.zeros((0, k), np.int64)
    return np.concatenate(own), np.concatenate(oth)


def marked(R, O, prev, cur, loose):
    """Flags set by the changed r-cliques of one sweep (prev -> cur)."""
    flags = np.zeros(prev.size, bool)
    ch = cur[R] != prev[R]
    h, told = cur[R], prev[R]
    k = O.shape[1]
    for x in range(k):
        v = prev[O[:, x]]
        ok = ch & (h < v)
        if not loose:
            ok &= v <= told
        for y in range(k):
            if y != x:
                ok &= (h <= prev[O[:, y]]) if loose else (prev[O[:, y]] >= v)
        flags[O[ok, x]] = True
    return flags


def marked_by_minimum(R, O, prev, cur):
    """The SND rule as the device evaluates it from its own gathers: the
    members holding the minimum rho of the s-clique, when h < rho <= told."""
    flags = np.zeros(prev.size, bool)
    ch = cur[R] != prev[R]
    vals = prev[O]
    rho = vals.min(axis=1)
    ok = ch & (cur[R] < rho) & (rho <= prev[R])
    for x in range(O.shape[1]):
        flags[O[ok & (vals[:, x] == rho), x]] = True
    return flags


@pytest.mark.parametrize("name,raw", list(graphs()), ids=lambda x: x if
                         isinstance(x, str) else "")
@pytest.mark.parametrize("r,s", KINDS)
def test_frontier_rules_cover_every_change(name, raw, r, s):
    g = oracle.Graph.from_raw(raw)
    if g.num_rcliques(r) == 0:
        pytest.skip("no r-cliques")
    R, O = pairs(g, r, s)
    seq = [t.astype(np.int64) for t in g.snd(r, s)]
    skipped = {False: 0, True: 0}
    for t in range(1, len(seq) - 1):
        prev, cur, nxt = seq[t - 1], seq[t], seq[t + 1]
        changed = cur != prev
        need = nxt != cur
        assert np.array_equal(marked(R, O, prev, cur, False),
                              marked_by_minimum(R, O, prev, cur))
        for loose in (False, True):
            act = marked(R, O, prev, cur, loose) | changed
            assert not np.any(need & ~act), (name, r, s, t, loose)
            skipped[loose] += int((~act).sum())
    # the tight rule never marks more than the loose one, and both skip work
    # on the graphs that take more than a couple of sweeps
    if len(seq) > 4:
        assert skipped[False] >= skipped[True] > 0


def test_tight_rule_marks_fewer():
    """On a power-law graph the tight rule marks strictly fewer r-cliques."""
    g = oracle.Graph.from_raw(chung_lu(2000, 2.1, 16.0, seed=24))
    R, O = pairs(g, 2, 3)
    seq = [t.astype(np.int64) for t in g.snd(2, 3)]
    tight = loose = 0
    for t in range(1, len(seq) - 1):
        tight += int(marked(R, O, seq[t - 1], seq[t], False).sum())
        loose += int(marked(R, O, seq[t - 1], seq[t], True).sum())
    assert tight < loose
