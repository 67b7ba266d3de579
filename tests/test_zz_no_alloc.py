"""nd_decompose_noalloc (the entry point for callers that cannot allocate)
against nd_decompose on the same prepared graphs, through the C ABI.

Results must be identical bit for bit (kappa, sweeps, updates), on calls in a
row that reuse the one static workspace with a smaller input second, for
SND/AND with and without the frontier, host and device output, per-sweep
snapshots, and the errors the entry point owns (graph not prepared, workspace
too small).  The allocating path is checked against the oracle as well.
"""

import ctypes

import numpy as np
import pytest
import torch

import oracle
from synth import chung_lu, books

pytestmark = pytest.mark.gpu

KINDS = {"core": (1, 2), "truss": (2, 3), "nucleus34": (3, 4)}


@pytest.fixture(scope="module")
def ctx(nd):
    return nd.Context(0)


def prepared(nd, ctx, raw, kind):
    g = nd.Graph.from_edges(ctx, raw.n, torch.from_numpy(raw.src),
                            torch.from_numpy(raw.dst))
    g.prepare(kind)
    return g


def run_noalloc(nd, g, kind, nr, **kw):
    out = torch.full((max(nr, 1),), -7, dtype=torch.int32, device="cuda")
    before = g.ctx.bytes_in_use()
    kappa, res = g.decompose(kind, out=out, noalloc=True, **kw)
    torch.cuda.synchronize()
    # the context's allocator was not touched (nothing allocated or cached)
    assert g.ctx.bytes_in_use() == before
    return kappa.cpu().numpy().copy(), res


@pytest.mark.parametrize("kind", list(KINDS))
@pytest.mark.parametrize("mode,frontier", [("snd", False), ("snd", True),
                                           ("and", False), ("and", True)])
def test_noalloc_equals_decompose_twice(nd, ctx, kind, mode, frontier):
    r, s = KINDS[kind]
    # the second graph is smaller: the workspace keeps the first call's
    # contents, which must not leak into the second result
    for raw in (chung_lu(6000, 2.1, 14.0, seed=31), chung_lu(2500, 2.3, 10.0, seed=32)):
        g = prepared(nd, ctx, raw, kind)
        nr = g.sizes(kind)[0]
        want, rw = g.decompose(kind, mode, use_frontier=frontier)
        want = want.cpu().numpy()
        got, rg = run_noalloc(nd, g, kind, nr, mode=mode, use_frontier=frontier)
        assert np.array_equal(got[:nr], want)
        assert np.array_equal(want, oracle.Graph.from_raw(raw).peel(r, s))
        assert rg["converged"] == 1 and rg["n_rcliques"] == nr
        if mode == "snd":  # deterministic iterates: same sweeps and work
            assert rg["sweeps"] == rw["sweeps"] and rg["updates"] == rw["updates"]


def test_noalloc_snapshots_and_active_counts(nd, ctx):
    raw = books(pages=(300, 700), page_degree=6.0, seed=3)
    kind = "truss"
    for n_call in range(2):
        g = prepared(nd, ctx, raw if n_call == 0 else chung_lu(1500, 2.2, 8.0, seed=5),
                     kind)
        nr = g.sizes(kind)[0]
        sa, sb = [], []
        g.decompose(kind, "snd", use_frontier=True, count_active=True,
                    keep_stats=sa)
        got, _ = run_noalloc(nd, g, kind, nr, mode="snd", use_frontier=True,
                             count_active=True, keep_stats=sb)
        assert [(x["changed"], x["evaluated"], x["active_next"]) for x in sa] == \
               [(x["changed"], x["evaluated"], x["active_next"]) for x in sb]


def test_noalloc_host_output_raw_abi(nd, ctx):
    """Host kappa through the raw C entry point (staged in the workspace)."""
    lib = nd._lib
    raw = chung_lu(3000, 2.1, 12.0, seed=41)
    for kind in ("truss", "core"):
        g = prepared(nd, ctx, raw, kind)
        nr = g.sizes(kind)[0]
        want = g.decompose(kind, "snd")[0].cpu().numpy()
        host = np.full(nr, -1, np.int32)
        o = nd.nd_opts()
        lib.nd_opts_init(ctypes.byref(o))
        res = nd.nd_result()
        st = lib.nd_decompose_noalloc(g._h, nd.KIND[kind], ctypes.byref(o),
                                      host.ctypes.data_as(ctypes.c_void_p), 0,
                                      None, ctypes.byref(res))
        assert st == 0, lib.nd_last_error()
        assert np.array_equal(host, want)


def test_noalloc_errors(nd, ctx):
    lib = nd._lib
    raw = chung_lu(2000, 2.1, 10.0, seed=43)
    g = nd.Graph.from_edges(ctx, raw.n, torch.from_numpy(raw.src),
                            torch.from_numpy(raw.dst))
    out = torch.zeros(max(raw.n, 1) * 8, dtype=torch.int32, device="cuda")
    o = nd.nd_opts()
    lib.nd_opts_init(ctypes.byref(o))
    res = nd.nd_result()
    # not prepared for the kind: refused, nothing prepared behind the back
    st = lib.nd_decompose_noalloc(g._h, nd.KIND["truss"], ctypes.byref(o),
                                  ctypes.c_void_p(out.data_ptr()), 1, None,
                                  ctypes.byref(res))
    assert st == 1 and b"nd_prepare" in lib.nd_last_error()
    # 48M isolated vertices (every d_s 0: 8-bit tau): SND needs 2 x 48 MiB
    # of tau (fits the 128 MiB workspace); with the frontier's flags
    # (+96 MiB) it does not
    n = 48 << 20
    e = torch.zeros(0, dtype=torch.int32)
    gb = nd.Graph.from_edges(ctx, n, e, e)
    gb.prepare("core")
    big = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    kappa, r = gb.decompose("core", out=big, noalloc=True)
    assert int(kappa.abs().max()) == 0 and r["converged"] == 1
    with pytest.raises(nd.NdError) as ei:
        gb.decompose("core", use_frontier=True, out=big, noalloc=True)
    assert ei.value.status == 2 and "workspace" in str(ei.value)
