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
