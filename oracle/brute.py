"""Brute-force definitions for tiny graphs (test infrastructure only).

Independent of ``oracle.c``: cliques are found by checking every vertex
subset, and kappa_s comes from the characterisation of Lemma 1 rather than
from any iteration or peeling.

Lemma 1 (Section 2.1) states kappa_s(R) = max over subgraphs G' containing R
of delta_{r,s}(G'), the minimum S-degree inside G'.  We take "subgraph" in the
sense the paper uses for degree levels (Section 3.1): a set T of r-cliques,
where an s-clique is present exactly when all of its r-cliques are in T.  So

    kappa_s(R) = max_{T containing R}  min_{R' in T} |{S : R' < S, all
                                                        r-subsets of S in T}|

For r = 1, 2 this coincides with the vertex/edge-induced subgraph reading.
"""

from __future__ import annotations

import itertools


def simple_edges(n, src, dst):
    """Set of unordered pairs (a, b), a < b, of the simple graph."""
    e = set()
    for a, b in zip(src, dst):
        a, b = int(a), int(b)
        if a != b:
            e.add((min(a, b), max(a, b)))
    return e


def cliques(n, edges, k):
    """All k-cliques as sorted tuples, in lexicographic order."""
    adj = {v: set() for v in range(n)}
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    out = []
    for t in itertools.combinations(range(n), k):
        if all(t[j] in adj[t[i]] for i in range(k) for j in range(i + 1, k)):
            out.append(t)
    return out


def hindex_def(values):
    """Largest k such that at least k of the values are >= k (Section 2.2)."""
    vals = list(values)
    best = 0
    for k in range(0, len(vals) + 1):
        if sum(1 for x in vals if x >= k) >= k:
            best = k
    return best


def kappa_bruteforce(n, src, dst, r, s, max_r=16):
    """kappa_s of every r-clique by maximising over all r-clique subsets."""
    edges = simple_edges(n, src, dst)
    Rs = cliques(n, edges, r)
    Ss = cliques(n, edges, s)
    nr = len(Rs)
    if nr > max_r:
        raise ValueError(f"{nr} r-cliques: too many for brute force")
    idx = {R: i for i, R in enumerate(Rs)}
    # each s-clique as the bitmask of its r-subsets
    smask = []
    for S in Ss:
        m = 0
        for sub in itertools.combinations(S, r):
            m |= 1 << idx[sub]
        smask.append(m)
    best = [0] * nr
    for T in range(1, 1 << nr):
        present = [m for m in smask if m & ~T == 0]
        delta = None
        for i in range(nr):
            if T >> i & 1:
                d = sum(1 for m in present if m >> i & 1)
                delta = d if delta is None else min(delta, d)
        for i in range(nr):
            if T >> i & 1 and delta > best[i]:
                best[i] = delta
    return Rs, best


def update_def(n, src, dst, r, s, tau):
    """U tau by the definition (Section 3), with cliques found by brute force.

    rho(S,R) = min of tau over the other r-cliques of S; U tau(R) = H of the
    rho values over all S containing R.
    """
    edges = simple_edges(n, src, dst)
    Rs = cliques(n, edges, r)
    Ss = cliques(n, edges, s)
    idx = {R: i for i, R in enumerate(Rs)}
    out = []
    for R in Rs:
        rhos = []
        for S in Ss:
            if set(R) <= set(S):
                others = [idx[sub] for sub in itertools.combinations(S, r)
                          if sub != R]
                rhos.append(min(tau[i] for i in others))
        out.append(hindex_def(rhos))
    return out
