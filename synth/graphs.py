"""Seeded generators for the synthetic workloads.

Every generator returns a ``RawGraph``: a vertex count and two int32 endpoint
arrays.  The edge list is *raw*: ball-dropping generators leave self-loops and
repeated pairs in it on purpose, because turning a raw list into a simple
undirected graph (the paper's setting, Section 2) is the first step of the
decomposition and is done independently by both consumers.

Randomness comes from numpy's ``default_rng`` (PCG64), seeded explicitly, so
the same seed gives the same bytes on every machine running this image.

Workload recipes (stand-ins for the paper's real graphs of Table 2, which are
power-law social/web networks; the SBM stands in for clustered graphs where
(3,4)-nuclei are non-trivial):

* ``er2000``   Erdos-Renyi G(n=2000, p=0.005), one Bernoulli draw per pair.
* ``cl20``     Chung-Lu, n=2^20, degree exponent 2.1, mean degree 32.
* ``cl23``     Chung-Lu, n=2^23, degree exponent 2.3, mean degree 32.
* ``sbm``      stochastic block model, 5000 communities of U{50..400}
               vertices, p_in=0.3, p_out=2e-6.
* ``stream``   4096 Chung-Lu graphs, n ~ U{1000..200000}, mean ~ U[8,64],
               exponent ~ U[2.0,2.5], Poisson arrivals.

Chung-Lu reading: weights w_i = w_min * (n/(i+1))^(1/(beta-1)), capped at
sqrt(n * mean) (the structural cutoff, so that w_i w_j / W <= 1), with w_min
bisected so that the mean capped weight equals the target mean degree.
n*mean/2 endpoint pairs are then drawn with probability proportional to w
("ball dropping"), and vertex ids are relabelled by a seeded random
permutation so that hubs are not clustered at low ids.
"""

from __future__ import annotations

import dataclasses
import math
import os

import numpy as np


@dataclasses.dataclass
class RawGraph:
    """A raw undirected edge list: ``src[i] -- dst[i]`` for each i."""

    n: int
    src: np.ndarray  # int32[m]
    dst: np.ndarray  # int32[m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(np.random.PCG64(int(seed)))


def erdos_renyi(n: int, p: float, seed: int = 1) -> RawGraph:
    """G(n, p) with one independent Bernoulli(p) draw per unordered pair.

    Pairs are visited in lexicographic order (i < j); the result is already
    simple (no loops, no repeats).
    """
    rng = _rng(seed)
    src_parts, dst_parts = [], []
    # Row by row keeps memory at O(n) per step and the draw order fixed.
    for i in range(n - 1):
        cnt = n - 1 - i
        hit = np.nonzero(rng.random(cnt) < p)[0]
        if hit.size:
            src_parts.append(np.full(hit.size, i, dtype=np.int32))
            dst_parts.append((hit + i + 1).astype(np.int32))
    if src_parts:
        src = np.concatenate(src_parts)
        dst = np.concatenate(dst_parts)
    else:
        src = np.zeros(0, np.int32)
        dst = np.zeros(0, np.int32)
    return RawGraph(n, src, dst, f"er(n={n},p={p},seed={seed})")


def books(pages=(400, 800, 1600), page_degree: float = 8.0,
          seed: int = 1) -> RawGraph:
    """Disjoint "books": a spine edge (a, b) and p page vertices, each joined
    to both a and b, with a G(p, page_degree / p) graph among the pages.

    The spine edge lies in exactly p triangles and its endpoints have p + 1
    neighbours, so the pages counts choose the S-degree of single r-cliques
    (for example one per range of a sweep's lane mapping), while the random
    page graph keeps the iterates non-trivial.
    """
    rng = _rng(seed)
    src_parts, dst_parts = [], []
    base = 0
    for p in pages:
        a, b = base, base + 1
        x = np.arange(base + 2, base + 2 + p, dtype=np.int64)
        src_parts += [np.array([a]), np.full(p, a), np.full(p, b)]
        dst_parts += [np.array([b]), x, x]
        q = page_degree / max(p, 1)
        for i in range(p - 1):
            hit = np.nonzero(rng.random(p - 1 - i) < q)[0]
            if hit.size:
                src_parts.append(np.full(hit.size, x[i]))
                dst_parts.append(x[i + 1 + hit])
        base += 2 + p
    src = np.concatenate(src_parts).astype(np.int32)
    dst = np.concatenate(dst_parts).astype(np.int32)
    return RawGraph(base, src, dst,
                    f"books(pages={tuple(pages)},deg={page_degree},seed={seed})")


def _searchsorted_threads(cdf: np.ndarray, keys: np.ndarray) -> np.ndarray:
    """np.searchsorted(cdf, keys, side="right"), over chunks of keys on a
    thread pool (numpy releases the GIL inside the search)."""
    if keys.size < (1 << 20):
        return np.searchsorted(cdf, keys, side="right")
    from concurrent.futures import ThreadPoolExecutor
    out = np.empty(keys.size, dtype=np.int64)
    bounds = np.linspace(0, keys.size, 65).astype(np.int64)

    def run(i):
        a, b = bounds[i], bounds[i + 1]
        out[a:b] = np.searchsorted(cdf, keys[a:b], side="right")

    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(run, range(64)))
    return out


def chung_lu_weights(n: int, beta: float, mean: float) -> np.ndarray:
    """Capped power-law weights with the requested mean (see module doc)."""
    cap = math.sqrt(n * mean)
    base = (n / (np.arange(n, dtype=np.float64) + 1.0)) ** (1.0 / (beta - 1.0))

    def mean_for(wmin: float) -> float:
        return float(np.minimum(wmin * base, cap).mean())

    lo, hi = 0.0, mean
    while mean_for(hi) < mean:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mean_for(mid) < mean:
            lo = mid
        else:
            hi = mid
    return np.minimum(hi * base, cap)


def chung_lu(n: int, beta: float, mean: float, seed: int) -> RawGraph:
    """Chung-Lu by ball dropping; the raw list keeps loops and repeats."""
    rng = _rng(seed)
    w = chung_lu_weights(n, beta, mean)
    cdf = np.cumsum(w)
    m = int(round(n * mean / 2.0))
    # Endpoints drawn with probability proportional to w, by inverting the CDF
    # (the searches run in chunks on a few threads; the result is the same).
    draws = rng.random(2 * m) * cdf[-1]
    ends = _searchsorted_threads(cdf, draws)
    np.minimum(ends, n - 1, out=ends)
    perm = rng.permutation(n).astype(np.int32)
    src = perm[ends[:m]]
    dst = perm[ends[m:]]
    return RawGraph(n, src.astype(np.int32), dst.astype(np.int32),
                    f"chung_lu(n={n},beta={beta},mean={mean},seed={seed})")


def sbm(n_comm: int = 5000, size_lo: int = 50, size_hi: int = 400,
        p_in: float = 0.3, p_out: float = 2e-6, seed: int = 4,
        with_communities: bool = False):
    """Stochastic block model with uniform community sizes.

    Intra-community pairs get one Bernoulli(p_in) draw each.  The number of
    inter-community edges is drawn as Binomial(#inter pairs, p_out) and that
    many uniformly random cross-community pairs are sampled (a repeated pair,
    which is vanishingly rare at these densities, is left in the raw list).
    With ``with_communities`` the result is ``(graph, labels)``, labels[v]
    being the community of (relabelled) vertex v; the graph is the same.
    """
    rng = _rng(seed)
    sizes = rng.integers(size_lo, size_hi + 1, size=n_comm)
    starts = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    n = int(sizes.sum())
    src_parts, dst_parts = [], []
    for c in range(n_comm):
        s = int(sizes[c])
        iu, ju = np.triu_indices(s, 1)
        hit = rng.random(iu.size) < p_in
        src_parts.append((iu[hit] + starts[c]).astype(np.int32))
        dst_parts.append((ju[hit] + starts[c]).astype(np.int32))
    intra_pairs = int((sizes * (sizes - 1) // 2).sum())
    inter_pairs = n * (n - 1) // 2 - intra_pairs
    m_out = int(rng.binomial(inter_pairs, p_out))
    comm = np.repeat(np.arange(n_comm), sizes)
    got_u, got_v, have = [], [], 0
    while have < m_out:
        need = m_out - have
        u = rng.integers(0, n, size=2 * need + 16)
        v = rng.integers(0, n, size=2 * need + 16)
        keep = comm[u] != comm[v]
        u, v = u[keep][:need], v[keep][:need]
        got_u.append(u.astype(np.int32))
        got_v.append(v.astype(np.int32))
        have += u.size
    src_parts.extend(got_u)
    dst_parts.extend(got_v)
    src = np.concatenate(src_parts).astype(np.int32)
    dst = np.concatenate(dst_parts).astype(np.int32)
    perm = rng.permutation(n).astype(np.int32)
    g = RawGraph(n, perm[src], perm[dst],
                 f"sbm(c={n_comm},sizes={size_lo}..{size_hi},p_in={p_in},"
                 f"p_out={p_out},seed={seed})")
    if not with_communities:
        return g
    labels = np.empty(n, np.int32)
    labels[perm] = comm
    return g, labels


def request_stream(count: int = 4096, n_lo: int = 1000, n_hi: int = 200000,
                   mean_lo: float = 8.0, mean_hi: float = 64.0,
                   beta_lo: float = 2.0, beta_hi: float = 2.5,
                   rate_per_s: float = 100.0, seed: int = 5):
    """Specs and Poisson arrival times for a stream of Chung-Lu graphs.

    Returns a list of dicts ``{"n", "mean", "beta", "seed", "arrival_s"}``;
    graph i uses seed ``seed + i`` and is generated on demand with
    ``chung_lu``.  Inter-arrival gaps are exponential with the given rate.
    """
    rng = _rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    means = rng.uniform(mean_lo, mean_hi, size=count)
    betas = rng.uniform(beta_lo, beta_hi, size=count)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    return [dict(n=int(ns[i]), mean=float(means[i]), beta=float(betas[i]),
                 seed=int(seed + i), arrival_s=float(arrivals[i]))
            for i in range(count)]


WORKLOADS = {
    "er2000": dict(kind="core", make=lambda: erdos_renyi(2000, 0.005, seed=1)),
    "cl20": dict(kind="truss", make=lambda: chung_lu(1 << 20, 2.1, 32.0, seed=2)),
    "cl23": dict(kind="core", make=lambda: chung_lu(1 << 23, 2.3, 32.0, seed=3)),
    "sbm": dict(kind="nucleus34", make=lambda: sbm(seed=4)),
}


def workload(name: str) -> RawGraph:
    """Build one of the named full-size workloads (see module doc)."""
    g = WORKLOADS[name]["make"]()
    g.name = name + ":" + g.name
    return g
