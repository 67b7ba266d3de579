"""Python binding of ``libnd.so`` (include/nd.h): argument marshalling only.

Every computation runs in the HIP library; this module converts torch
tensors and streams to the C ABI's pointers, sizes and status codes.  It
raises ``ImportError`` when the library has not been built: there is no CPU
fallback.

Kinds (Section 5 of Sariyuce, Seshadhri, Pinar): ``"core"`` = (1,2),
``"truss"`` = (2,3) with truss numbers counted in triangles, ``"nucleus34"`` =
(3,4), and the generic variants ``"nucleus13"`` = (1,3) and ``"nucleus24"`` =
(2,4).  Modes: ``"snd"`` (Alg. 2) and ``"and"`` (Alg. 3).
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Callable, Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python "
        "paper_1704_00386_amd/build.py` (there is no fallback path)")

_lib = ctypes.CDLL(LIB_PATH)
# The HIP runtime the library links; used only to copy per-sweep snapshots
# out of the device pointer handed to the iteration callback.
_hip = ctypes.CDLL("libamdhip64.so")
_hip.hipMemcpy.restype = ctypes.c_int
_hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                           ctypes.c_int]
_HIP_D2D = 3

KIND = {"core": 0, "truss": 1, "nucleus34": 2, "nucleus13": 3, "nucleus24": 4}
RS = {"core": (1, 2), "truss": (2, 3), "nucleus34": (3, 4), "nucleus13": (1, 3),
      "nucleus24": (2, 4)}
MODE = {"snd": 0, "and": 1}

STATUS = {0: "ok", 1: "invalid", 2: "oom", 3: "device", 4: "unsupported",
          5: "not_converged", 6: "busy", 7: "cancelled", 8: "timeout"}


class NdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class nd_iter_info(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int32), ("evaluated", ctypes.c_int64),
                ("changed", ctypes.c_int64), ("active_next", ctypes.c_int64),
                ("tau_dev", ctypes.c_void_p), ("ms", ctypes.c_double)]


ITER_CB = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p,
                           ctypes.POINTER(nd_iter_info))


class nd_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("max_iters", ctypes.c_int32),
                ("use_frontier", ctypes.c_int32),
                ("stop_active_ratio", ctypes.c_double),
                ("snapshot_every", ctypes.c_int32),
                ("count_active", ctypes.c_int32),
                ("on_iter", ITER_CB), ("user", ctypes.c_void_p)]


class nd_result(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("n_rcliques", ctypes.c_int64),
                ("n_incidence", ctypes.c_int64), ("updates", ctypes.c_int64),
                ("ms_prep", ctypes.c_double), ("ms_iterate", ctypes.c_double),
                ("max_sdegree", ctypes.c_int32), ("tau_bytes", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class nd_serve_info(ctypes.Structure):
    _fields_ = [("latency_ms", ctypes.c_double), ("prep_ms", ctypes.c_double),
                ("epochs_during_prep", ctypes.c_int64),
                ("epoch_joined", ctypes.c_int64), ("epoch_done", ctypes.c_int64),
                ("joined_running", ctypes.c_int32),
                ("peak_members", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("nd_status_str", ctypes.c_char_p, ctypes.c_int)
_sig("nd_last_error", ctypes.c_char_p)
_sig("nd_opts_init", None, ctypes.POINTER(nd_opts))
_sig("nd_ctx_create", ctypes.c_int, ctypes.c_int, ctypes.c_size_t,
     ctypes.POINTER(_P))
_sig("nd_ctx_destroy", None, _P)
_sig("nd_ctx_bytes_in_use", ctypes.c_size_t, _P)
_sig("nd_graph_from_edges", ctypes.c_int, _P, _I32, _I64, _P, _P, ctypes.c_int,
     _P, ctypes.POINTER(_P))
_sig("nd_graphs_from_edges", ctypes.c_int, _P, _I32, ctypes.POINTER(_I32),
     ctypes.POINTER(_I64), ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.c_int,
     _P, ctypes.POINTER(_P))
_sig("nd_graph_from_csr", ctypes.c_int, _P, _I32, _I64, _P, _P, ctypes.c_int,
     _P, ctypes.POINTER(_P))
_sig("nd_graph_destroy", None, _P)
_sig("nd_graph_dims", ctypes.c_int, _P, ctypes.POINTER(_I32),
     ctypes.POINTER(_I64))
_sig("nd_graph_csr", ctypes.c_int, _P, _P, _P, ctypes.c_int, _P)
_sig("nd_prepare", ctypes.c_int, _P, ctypes.c_int, _P)
_sig("nd_sizes", ctypes.c_int, _P, ctypes.c_int, ctypes.POINTER(_I64),
     ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_size_t))
_sig("nd_rcliques", ctypes.c_int, _P, ctypes.c_int, _P, ctypes.c_int, _P)
_sig("nd_incidence", ctypes.c_int, _P, ctypes.c_int, _P, _P, ctypes.c_int, _P)
_sig("nd_sdegree", ctypes.c_int, _P, ctypes.c_int, _P, ctypes.c_int, _P)
_sig("nd_decompose", ctypes.c_int, _P, ctypes.c_int, ctypes.POINTER(nd_opts),
     _P, ctypes.c_int, _P, ctypes.POINTER(nd_result))
_sig("nd_decompose_noalloc", ctypes.c_int, _P, ctypes.c_int,
     ctypes.POINTER(nd_opts), _P, ctypes.c_int, _P, ctypes.POINTER(nd_result))
_sig("nd_update", ctypes.c_int, _P, ctypes.c_int, _P, _P, ctypes.c_int, _P)
_sig("nd_levels", ctypes.c_int, _P, ctypes.c_int, _P,
     ctypes.POINTER(ctypes.c_int32), ctypes.c_int, _P)
_sig("nd_partial_and", ctypes.c_int, _P, ctypes.c_int, _P, ctypes.c_int64,
     ctypes.POINTER(nd_opts), _P, ctypes.c_int, _P, ctypes.POINTER(nd_result))
_sig("nd_ego_estimate", ctypes.c_int, _P, ctypes.c_int, _P, ctypes.c_int64,
     _I32, _P, _P, ctypes.c_int, _P)
_sig("nd_prepare_many", ctypes.c_int, _P, _I32, ctypes.POINTER(_P),
     ctypes.c_int, _P)
_sig("nd_batch_decompose", ctypes.c_int, _P, _I32, ctypes.POINTER(_P),
     ctypes.c_int, ctypes.POINTER(nd_opts), ctypes.POINTER(_P), ctypes.c_int,
     _P, ctypes.POINTER(nd_result))
_sig("nd_server_create", ctypes.c_int, _P, _I32, _I32, ctypes.POINTER(_P))
_sig("nd_server_submit", ctypes.c_int, _P, _P, ctypes.c_int,
     ctypes.POINTER(nd_opts), ctypes.POINTER(ctypes.c_uint64))
_sig("nd_server_wait", ctypes.c_int, _P, ctypes.c_uint64, _I64,
     ctypes.POINTER(nd_result), ctypes.POINTER(nd_serve_info))
_sig("nd_server_result", ctypes.c_int, _P, ctypes.c_uint64, _P, _I64)
_sig("nd_server_cancel", ctypes.c_int, _P, ctypes.c_uint64)
_sig("nd_server_destroy", None, _P)


def _check(status: int, what: str = ""):
    if status != 0:
        msg = _lib.nd_last_error().decode(errors="replace")
        raise NdError(status, f"{what}: {msg}" if what else msg)


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_i32(t: torch.Tensor, device) -> torch.Tensor:
    t = torch.as_tensor(t)
    return t.to(device=device, dtype=torch.int32).contiguous()


def _make_opts(mode="snd", max_iters=-1, use_frontier=False,
               stop_active_ratio=0.0, on_iter=None, count_active=False,
               snapshot_every=1):
    o = nd_opts()
    _lib.nd_opts_init(ctypes.byref(o))
    o.mode = MODE[mode]
    o.max_iters = int(max_iters)
    o.use_frontier = int(bool(use_frontier))
    o.stop_active_ratio = float(stop_active_ratio)
    o.count_active = int(bool(count_active))
    o.snapshot_every = int(snapshot_every)
    keep = None
    if on_iter is not None:
        def _cb(_user, info_p):
            info = info_p.contents
            return int(bool(on_iter(info)))
        keep = ITER_CB(_cb)
        o.on_iter = keep
    return o, keep


class Context:
    """A device context (nd_ctx): the device and its memory budget."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = _P()
        _check(_lib.nd_ctx_create(int(device), int(hbm_budget_bytes),
                                  ctypes.byref(h)), "nd_ctx_create")
        self._h = h
        self.device = torch.device("cuda", device)

    def bytes_in_use(self) -> int:
        return int(_lib.nd_ctx_bytes_in_use(self._h))

    def close(self):
        if getattr(self, "_h", None):
            _lib.nd_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A simple undirected graph held on the device (nd_graph)."""

    def __init__(self, ctx: Context, handle):
        self.ctx = ctx
        self._h = handle

    @classmethod
    def from_edges(cls, ctx: Context, n: int, src, dst, stream=None) -> "Graph":
        """Raw undirected pairs; loops and repeats are removed on the device."""
        s = _dev_i32(src, ctx.device)
        d = _dev_i32(dst, ctx.device)
        if s.numel() != d.numel():
            raise ValueError("src and dst differ in length")
        h = _P()
        _check(_lib.nd_graph_from_edges(ctx._h, int(n), int(s.numel()),
                                        _P(s.data_ptr()), _P(d.data_ptr()), 1,
                                        _stream(stream), ctypes.byref(h)),
               "nd_graph_from_edges")
        return cls(ctx, h)

    @classmethod
    def from_csr(cls, ctx: Context, n: int, row_off, col, stream=None) -> "Graph":
        ro = torch.as_tensor(row_off).to(ctx.device, torch.int64).contiguous()
        c = _dev_i32(col, ctx.device)
        h = _P()
        _check(_lib.nd_graph_from_csr(ctx._h, int(n), int(c.numel()),
                                      _P(ro.data_ptr()), _P(c.data_ptr()), 1,
                                      _stream(stream), ctypes.byref(h)),
               "nd_graph_from_csr")
        return cls(ctx, h)

    def close(self):
        if getattr(self, "_h", None):
            _lib.nd_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def detach(self):
        """Give up ownership (the server takes graphs over)."""
        h, self._h = self._h, None
        return h

    def dims(self):
        n = _I32()
        nnz = _I64()
        _check(_lib.nd_graph_dims(self._h, ctypes.byref(n), ctypes.byref(nnz)))
        return int(n.value), int(nnz.value)

    def csr(self, stream=None):
        n, nnz = self.dims()
        ro = torch.empty(n + 1, dtype=torch.int64, device=self.ctx.device)
        col = torch.empty(max(nnz, 1), dtype=torch.int32, device=self.ctx.device)
        _check(_lib.nd_graph_csr(self._h, _P(ro.data_ptr()),
                                 _P(col.data_ptr()), 1, _stream(stream)),
               "nd_graph_csr")
        return ro, col[:nnz]

    def prepare(self, kind: str, stream=None):
        _check(_lib.nd_prepare(self._h, KIND[kind], _stream(stream)),
               "nd_prepare")

    def sizes(self, kind: str):
        nr, P = _I64(), _I64()
        b = ctypes.c_size_t()
        _check(_lib.nd_sizes(self._h, KIND[kind], ctypes.byref(nr),
                             ctypes.byref(P), ctypes.byref(b)), "nd_sizes")
        return int(nr.value), int(P.value), int(b.value)

    def rclique_count(self, kind: str) -> int:
        """|R| for `kind`; for r <= 2 read off the graph without preparing."""
        nr = _I64()
        _check(_lib.nd_sizes(self._h, KIND[kind], ctypes.byref(nr), None, None),
               "nd_sizes")
        return int(nr.value)

    def rcliques(self, kind: str, stream=None) -> torch.Tensor:
        nr, _, _ = self.sizes(kind)
        r = RS[kind][0]
        out = torch.empty(max(nr * r, 1), dtype=torch.int32,
                          device=self.ctx.device)
        _check(_lib.nd_rcliques(self._h, KIND[kind], _P(out.data_ptr()), 1,
                                _stream(stream)), "nd_rcliques")
        return out[: nr * r].view(nr, r)

    def incidence(self, kind: str, stream=None):
        nr, P, _ = self.sizes(kind)
        r, s = RS[kind]
        from math import comb
        k = comb(s, r) - 1
        off = torch.empty(nr + 1, dtype=torch.int64, device=self.ctx.device)
        ids = torch.empty(max(P * k, 1), dtype=torch.int32,
                          device=self.ctx.device)
        _check(_lib.nd_incidence(self._h, KIND[kind], _P(off.data_ptr()),
                                 _P(ids.data_ptr()), 1, _stream(stream)),
               "nd_incidence")
        return off, ids[: P * k].view(P, k)

    def sdegree(self, kind: str, stream=None) -> torch.Tensor:
        nr, _, _ = self.sizes(kind)
        ds = torch.empty(max(nr, 1), dtype=torch.int32, device=self.ctx.device)
        _check(_lib.nd_sdegree(self._h, KIND[kind], _P(ds.data_ptr()), 1,
                               _stream(stream)), "nd_sdegree")
        return ds[:nr]

    def update(self, kind: str, tau, stream=None) -> torch.Tensor:
        """U tau (one application of the update operator)."""
        t = _dev_i32(tau, self.ctx.device)
        out = torch.empty_like(t)
        _check(_lib.nd_update(self._h, KIND[kind], _P(t.data_ptr()),
                              _P(out.data_ptr()), 1, _stream(stream)),
               "nd_update")
        return out

    def levels(self, kind: str, stream=None):
        """Degree levels (nd_levels): (level per r-clique as an int32 tensor
        on the device, number of levels)."""
        nr, _, _ = self.sizes(kind)
        out = torch.empty(max(nr, 1), dtype=torch.int32, device=self.ctx.device)
        nl = ctypes.c_int32()
        _check(_lib.nd_levels(self._h, KIND[kind], _P(out.data_ptr()),
                              ctypes.byref(nl), 1, _stream(stream)),
               "nd_levels")
        return out[:nr], int(nl.value)

    def partial_and(self, kind: str, ids, max_iters: int = -1, stream=None,
                    allow_not_converged: bool = False):
        """PartialAND on the r-cliques `ids` (nd_partial_and): their final
        values (int32 tensor on the device, one per id) and the result dict."""
        t = _dev_i32(ids, self.ctx.device)
        out = torch.empty(max(t.numel(), 1), dtype=torch.int32,
                          device=self.ctx.device)
        o, keep = _make_opts("and", max_iters)
        res = nd_result()
        st = _lib.nd_partial_and(self._h, KIND[kind], _P(t.data_ptr()),
                                 t.numel(), ctypes.byref(o),
                                 _P(out.data_ptr()), 1, _stream(stream),
                                 ctypes.byref(res))
        del keep
        if not (st == 0 or (st == 5 and allow_not_converged)):
            _check(st, "nd_partial_and")
        return out[:t.numel()], res.as_dict()

    def ego_estimate(self, kind: str, queries, max_iters: int = -1,
                     stream=None):
        """PartialAND estimates on the queries' ego networks
        (nd_ego_estimate): (estimates, sweeps), int32 tensors on the
        device."""
        q = _dev_i32(queries, self.ctx.device)
        n = q.numel()
        est = torch.empty(max(n, 1), dtype=torch.int32, device=self.ctx.device)
        sw = torch.empty(max(n, 1), dtype=torch.int32, device=self.ctx.device)
        _check(_lib.nd_ego_estimate(self._h, KIND[kind], _P(q.data_ptr()), n,
                                    int(max_iters), _P(est.data_ptr()),
                                    _P(sw.data_ptr()), 1, _stream(stream)),
               "nd_ego_estimate")
        return est[:n], sw[:n]

    def decompose(self, kind: str, mode: str = "snd", max_iters: int = -1,
                  use_frontier: bool = False, stop_active_ratio: float = 0.0,
                  on_iter: Optional[Callable] = None, out=None, stream=None,
                  allow_not_converged: bool = False,
                  keep_iterates: Optional[list] = None,
                  keep_index: Optional[torch.Tensor] = None,
                  count_active: bool = False, snapshot_every: int = 1,
                  keep_stats: Optional[list] = None, noalloc: bool = False):
        """kappa for every r-clique (int32 tensor on the device) and the
        nd_result statistics as a dict.  With keep_iterates=[] the list
        receives (changed, tau_t) for every sweep t = 1, 2, ...; with
        keep_index (r-clique ids, a device tensor) only tau_t[keep_index]
        is kept, so that big graphs can keep many sweeps.  keep_stats=[]
        receives a dict of nd_iter_info's counts for every sweep the callback
        sees.  noalloc=True calls nd_decompose_noalloc: the graph must be
        prepared and `out` (int32, device, at least |R| long) receives kappa;
        nothing is prepared or allocated here."""
        if noalloc:
            if out is None:
                raise ValueError("noalloc needs the caller's kappa buffer `out`")
            if keep_iterates is not None:
                raise ValueError("keep_iterates allocates; not with noalloc")
            kappa, nr = out, None
        else:
            nr, _, _ = self.sizes(kind)
            kappa = out if out is not None else torch.empty(
                max(nr, 1), dtype=torch.int32, device=self.ctx.device)
        if keep_stats is not None:
            stats_cb = on_iter

            def on_iter(info):
                keep_stats.append({"iter": int(info.iter),
                                   "evaluated": int(info.evaluated),
                                   "changed": int(info.changed),
                                   "active_next": int(info.active_next),
                                   "ms": float(info.ms)})
                return stats_cb(info) if stats_cb else 0
        if keep_iterates is not None:
            user_cb = on_iter
            dev = self.ctx.device
            full = None if keep_index is None else torch.empty(
                max(nr, 1), dtype=torch.int32, device=dev)

            def on_iter(info):
                snap = full if full is not None else torch.empty(
                    max(nr, 1), dtype=torch.int32, device=dev)
                rc = _hip.hipMemcpy(snap.data_ptr(), info.tau_dev, 4 * nr,
                                    _HIP_D2D)
                if rc != 0:
                    raise RuntimeError(f"hipMemcpy failed ({rc})")
                if keep_index is None:
                    kept = snap[:nr]
                else:
                    kept = snap[keep_index]
                    torch.cuda.synchronize()  # before the next sweep's copy
                keep_iterates.append((int(info.changed), kept))
                return user_cb(info) if user_cb else 0
        o, keep = _make_opts(mode, max_iters, use_frontier, stop_active_ratio,
                             on_iter, count_active, snapshot_every)
        res = nd_result()
        fn = _lib.nd_decompose_noalloc if noalloc else _lib.nd_decompose
        st = fn(self._h, KIND[kind], ctypes.byref(o), _P(kappa.data_ptr()), 1,
                _stream(stream), ctypes.byref(res))
        del keep
        if not (st == 0 or (st == 5 and allow_not_converged)):
            _check(st, "nd_decompose_noalloc" if noalloc else "nd_decompose")
        if nr is None:
            nr = int(res.n_rcliques)
        return kappa[:nr], res.as_dict()


def graphs_from_edges(ctx: Context, edge_lists, stream=None):
    """nd_graphs_from_edges: [Graph] from [(n, src, dst)], built together."""
    count = len(edge_lists)
    ns = (_I32 * max(count, 1))()
    ms = (_I64 * max(count, 1))()
    ss = (_P * max(count, 1))()
    ds = (_P * max(count, 1))()
    keep = []
    for i, (n, src, dst) in enumerate(edge_lists):
        s = _dev_i32(src, ctx.device)
        d = _dev_i32(dst, ctx.device)
        if s.numel() != d.numel():
            raise ValueError(f"graph {i}: src and dst differ in length")
        keep += [s, d]
        ns[i], ms[i] = int(n), int(s.numel())
        ss[i], ds[i] = s.data_ptr(), d.data_ptr()
    out = (_P * max(count, 1))()
    _check(_lib.nd_graphs_from_edges(ctx._h, count, ns, ms, ss, ds, 1,
                                     _stream(stream), out), "nd_graphs_from_edges")
    del keep
    return [Graph(ctx, _P(out[i])) for i in range(count)]


def prepare_many(ctx: Context, graphs: Sequence[Graph], kind: str,
                 stream=None):
    """nd_prepare_many: prepare several graphs with overlapping builds."""
    hs = (_P * max(len(graphs), 1))()
    for i, g in enumerate(graphs):
        hs[i] = g._h
    _check(_lib.nd_prepare_many(ctx._h, len(graphs), hs, KIND[kind],
                                _stream(stream)), "nd_prepare_many")


def batch_decompose(ctx: Context, graphs: Sequence[Graph], kind: str,
                    mode: str = "snd", max_iters: int = -1,
                    use_frontier: bool = False, stream=None):
    """Decompose several graphs in one combined sweep; returns ([kappa],
    [result dict])."""
    count = len(graphs)
    outs, ptrs = [], (_P * max(count, 1))()
    hs = (_P * max(count, 1))()
    for i, g in enumerate(graphs):
        hs[i] = g._h
    if RS[kind][0] > 2:  # |R| is known only once the graphs are prepared
        _check(_lib.nd_prepare_many(ctx._h, count, hs, KIND[kind],
                                    _stream(stream)), "nd_prepare_many")
    for i, g in enumerate(graphs):
        nr = g.rclique_count(kind)
        k = torch.empty(max(nr, 1), dtype=torch.int32, device=ctx.device)
        outs.append(k[:nr])
        ptrs[i] = k.data_ptr()
    o, keep = _make_opts(mode, max_iters, use_frontier)
    res = (nd_result * max(count, 1))()
    _check(_lib.nd_batch_decompose(ctx._h, count, hs, KIND[kind],
                                   ctypes.byref(o), ptrs, 1, _stream(stream),
                                   res), "nd_batch_decompose")
    del keep
    return outs, [res[i].as_dict() for i in range(count)]


class Server:
    """Continuous-batching request loop (nd_server).  Submitted graphs are
    owned by the server; results come back in host memory."""

    def __init__(self, ctx: Context, max_slots: int = 64,
                 max_queue: int = 1 << 16):
        h = _P()
        _check(_lib.nd_server_create(ctx._h, int(max_slots), int(max_queue),
                                     ctypes.byref(h)), "nd_server_create")
        self._h = h
        self.ctx = ctx

    def submit(self, graph: Graph, kind: str, mode: str = "snd",
               max_iters: int = -1, use_frontier: bool = False) -> int:
        o, keep = _make_opts(mode, max_iters, use_frontier)
        t = ctypes.c_uint64()
        _check(_lib.nd_server_submit(self._h, graph._h, KIND[kind],
                                     ctypes.byref(o), ctypes.byref(t)),
               "nd_server_submit")
        graph.detach()
        return int(t.value)

    def wait(self, ticket: int, timeout_us: int = -1,
             allow_not_converged: bool = False):
        """(kappa as a host int32 tensor, result dict, serve-info dict), or
        None on timeout.  Raises NdError for a failed or cancelled request
        (and for one that stopped at max_iters unless allow_not_converged)."""
        res = nd_result()
        info = nd_serve_info()
        st = _lib.nd_server_wait(self._h, ctypes.c_uint64(ticket),
                                 int(timeout_us), ctypes.byref(res),
                                 ctypes.byref(info))
        if st == 8:
            return None
        if st in (0, 5):
            n = int(res.n_rcliques)
            buf = torch.empty(max(n, 1), dtype=torch.int32)
            _check(_lib.nd_server_result(self._h, ctypes.c_uint64(ticket),
                                         _P(buf.data_ptr()), n),
                   "nd_server_result")
            if st == 5 and not allow_not_converged:
                _check(st, "nd_server_wait")
            return buf[:n], res.as_dict(), info.as_dict()
        _check(st, "nd_server_wait")

    def cancel(self, ticket: int):
        _check(_lib.nd_server_cancel(self._h, ctypes.c_uint64(ticket)),
               "nd_server_cancel")

    def close(self):
        if getattr(self, "_h", None):
            _lib.nd_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
