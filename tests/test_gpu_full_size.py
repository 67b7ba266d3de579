"""Full-size parity on the single-GPU workloads: k-truss on Chung-Lu n=2^20
(beta 2.1, mean 32), k-core on Chung-Lu n=2^23 (beta 2.3, mean 32) and the
(3,4)-nucleus on the stochastic block model (5000 communities of U{50..400}
vertices, p_in 0.3, p_out 2e-6; 4.2*10^8 triangles, whose golden values come
from the oracle run community by community, an exact split that the golden
script checks).

* kappa: the GPU's result, from SND and AND, with and without the
  notification frontier, equals the oracle's Alg. Peeling result, compared by
  the SHA-256 digest of its little-endian int32 bytes in r-clique id order.
  The digests are in tests/golden/full_size.json, written by
  tests/golden/make_golden.py, which runs the oracle only.
* iterates: sampled r-clique ranges of several SND iterates tau_t equal the
  oracle's update operator (Section 3, Defn. of U) applied to tau_{t-1} on
  the same ranges, one r-clique at a time.
"""

import hashlib
import json
import os

import numpy as np
import pytest
import torch

import oracle
from synth import WORKLOADS, workload

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                     "full_size.json")))


def digest(kappa: torch.Tensor) -> str:
    a = kappa.cpu().numpy().astype("<i4")
    return hashlib.sha256(a.tobytes()).hexdigest()


def histogram(kappa: torch.Tensor) -> dict:
    vals, counts = np.unique(kappa.cpu().numpy(), return_counts=True)
    return {str(int(v)): int(c) for v, c in zip(vals, counts)}


_cache = {}


def graph(nd, name):
    if name not in _cache:
        _cache.clear()  # one full-size graph resident at a time
        raw = workload(name)
        ctx = nd.Context(0)
        g = nd.Graph.from_edges(ctx, raw.n, torch.from_numpy(raw.src).cuda(),
                                torch.from_numpy(raw.dst).cuda())
        _cache[name] = (raw, ctx, g)
    return _cache[name]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("name", ["cl20", "cl23", "sbm"])
def test_full_size_kappa_equals_oracle(nd, name):
    want = GOLDEN[name]
    kind = WORKLOADS[name]["kind"]
    raw, ctx, g = graph(nd, name)
    assert raw.name.endswith(want["generator"].split(":", 1)[1])
    for mode in ("snd", "and"):
        for frontier in (False, True):
            kappa, res = g.decompose(kind, mode, use_frontier=frontier)
            assert res["converged"] == 1
            assert kappa.numel() == want["n_rcliques"]
            got = digest(kappa)
            if got != want["kappa_sha256"]:
                assert histogram(kappa) == want["kappa_histogram"], (mode, frontier)
            assert got == want["kappa_sha256"], (mode, frontier)
            assert int(kappa.max()) == want["kappa_max"]
            assert int(kappa.to(torch.int64).sum()) == want["kappa_sum"]


@pytest.mark.timeout(900)
def test_full_size_sampled_iterates_equal_update_operator(nd):
    """k-truss on the n=2^20 workload: for sweeps 1, 2, 3, 10 and the last,
    U(tau_{t-1}) from the oracle on three random ranges of 4096 edges equals
    the GPU's tau_t there."""
    raw, ctx, g = graph(nd, "cl20")
    its = []
    kappa, res = g.decompose("truss", "snd", keep_iterates=its)
    T = res["sweeps"]
    assert len(its) == T
    og = oracle.Graph.from_raw(raw)
    nr = og.num_rcliques(2)
    tau0 = g.sdegree("truss").cpu().numpy()
    rng = np.random.default_rng(11)
    for t in sorted({1, 2, 3, 10, T}):
        prev = tau0 if t == 1 else its[t - 2][1].cpu().numpy()
        cur = its[t - 1][1].cpu().numpy()
        for lo in rng.integers(0, nr - 4096, size=3):
            lo = int(lo)
            want = og.update(2, 3, prev, lo=lo, hi=lo + 4096)
            assert np.array_equal(cur[lo:lo + 4096], want[lo:lo + 4096]), (t, lo)
    assert torch.equal(its[-1][1], kappa)


@pytest.mark.timeout(900)
def test_full_size_core_sampled_iterates(nd):
    """k-core on the n=2^23 workload: for sweeps 1, 2, 5, 20 and the last,
    U(tau_{t-1}) from the oracle on three random ranges of 20000 vertices
    equals the GPU's tau_t there."""
    raw, ctx, g = graph(nd, "cl23")
    its = []
    kappa, res = g.decompose("core", "snd", keep_iterates=its)
    T = res["sweeps"]
    og = oracle.Graph.from_raw(raw)
    nr = og.num_rcliques(1)
    tau0 = g.sdegree("core").cpu().numpy()
    rng = np.random.default_rng(12)
    for t in sorted({1, 2, 5, 20, T}):
        prev = tau0 if t == 1 else its[t - 2][1].cpu().numpy()
        cur = its[t - 1][1].cpu().numpy()
        for lo in rng.integers(0, nr - 20000, size=3):
            lo = int(lo)
            want = og.update(1, 2, prev, lo=lo, hi=lo + 20000)
            assert np.array_equal(cur[lo:lo + 20000], want[lo:lo + 20000]), (t, lo)
    assert torch.equal(its[-1][1], kappa)


@pytest.mark.timeout(900)
def test_full_size_nucleus34_iterates_per_community(nd):
    """(3,4) on the block model: every SND iterate of the whole graph,
    restricted to the triangles of five communities, equals the oracle's
    SND iterates (Alg. 2) on each community's induced subgraph.  The
    restriction is exact when no 4-clique leaves a community, and the test
    checks that through the S-degrees, which would differ otherwise."""
    from synth import sbm

    raw, ctx, g = graph(nd, "sbm")
    raw2, labels = sbm(seed=4, with_communities=True)
    assert np.array_equal(raw2.src, raw.src) and np.array_equal(raw2.dst, raw.dst)
    tri = g.rcliques("nucleus34")  # (nt, 3) device tensor, lexicographic
    lab = torch.from_numpy(labels).cuda().long()
    l0, l1, l2 = lab[tri[:, 0].long()], lab[tri[:, 1].long()], lab[tri[:, 2].long()]
    comms = [int(c) for c in np.random.default_rng(21).choice(labels.max() + 1, 5,
                                                              replace=False)]
    idx = [torch.nonzero((l0 == c) & (l1 == c) & (l2 == c)).flatten()
           for c in comms]
    del tri, l0, l1, l2
    allidx = torch.cat(idx)
    its = []
    kappa, res = g.decompose("nucleus34", "snd", keep_iterates=its,
                             keep_index=allidx)
    T = res["sweeps"]
    ds = g.sdegree("nucleus34")[allidx].cpu().numpy()
    at = 0
    for c, ix in zip(comms, idx):
        verts = np.sort(np.nonzero(labels == c)[0]).astype(np.int32)
        keep = (labels[raw.src] == c) & (labels[raw.dst] == c)
        og = oracle.Graph(verts.size, np.searchsorted(verts, raw.src[keep]),
                          np.searchsorted(verts, raw.dst[keep]))
        n = ix.numel()
        assert og.num_rcliques(3) == n
        assert np.array_equal(ds[at:at + n], og.sdeg(3, 4))
        seq = og.snd(3, 4)  # tau_0 .. tau_Tc, the last two equal
        for t in range(1, T + 1):
            got = its[t - 1][1][at:at + n].cpu().numpy()
            assert np.array_equal(got, seq[min(t, len(seq) - 1)]), (c, t)
        at += n
