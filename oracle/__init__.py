"""Python access to the CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports
this package, and this package never imports the product library.

The oracle follows the paper's definitions directly (Sariyuce, Seshadhri,
Pinar, "Local Algorithms for Hierarchical Dense Subgraph Discovery"):

* ``peel``        kappa_s by Alg. Peeling (Section 2.1, Alg. 1);
* ``update``      one application of the update operator U (Section 3);
* ``snd``         the synchronous iteration tau_{t+1} = U tau_t from
                  tau_0 = d_s (Section 4.1, Alg. SND), every iterate kept;
* ``and_sweep``   one in-place asynchronous sweep (Section 4.2, Alg. AND);
* ``and_notify``  Alg. AND with its notification lines (Section 4.3), with
                  the per-iteration counts of computations and of active
                  r-cliques (the indicator of Section 5.1.4);
* ``levels``      degree levels (Section 3.1);
* ``hindex``      H of a multiset (Section 2.2).

Pinned by ``tests/test_oracle_*.py`` against the paper's worked examples,
closed forms, brute force and networkx.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

KINDS = {"core": (1, 2), "truss": (2, 3), "nucleus34": (3, 4), "nucleus13": (1, 3),
         "nucleus24": (2, 4)}


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (fast; done on demand when missing)."""
    if force or not os.path.exists(_SO) or (
            os.path.getmtime(_SO) < os.path.getmtime(_SRC)):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-pthread",
               _SRC, "-o", _SO]
        subprocess.run(cmd, check=True)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_SO)
    P = ctypes.c_void_p
    i32p = ctypes.POINTER(ctypes.c_int32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.og_new.restype = P
    lib.og_new.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p]
    lib.og_free.argtypes = [P]
    lib.og_last_error.restype = ctypes.c_char_p
    lib.og_n.restype = ctypes.c_int32
    lib.og_n.argtypes = [P]
    lib.og_nnz.restype = ctypes.c_int64
    lib.og_nnz.argtypes = [P]
    lib.og_csr.argtypes = [P, i64p, i32p]
    lib.og_num_rcliques.restype = ctypes.c_int64
    lib.og_num_rcliques.argtypes = [P, ctypes.c_int]
    lib.og_rcliques.restype = ctypes.c_int
    lib.og_rcliques.argtypes = [P, ctypes.c_int, i32p]
    lib.og_hindex.restype = ctypes.c_int32
    lib.og_hindex.argtypes = [i32p, ctypes.c_int64]
    lib.og_sdeg.restype = ctypes.c_int
    lib.og_sdeg.argtypes = [P, ctypes.c_int, ctypes.c_int, i32p, ctypes.c_int]
    lib.og_members.restype = ctypes.c_int64
    lib.og_members.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int64,
                               i32p, ctypes.c_int64]
    lib.og_peel.restype = ctypes.c_int
    lib.og_peel.argtypes = [P, ctypes.c_int, ctypes.c_int, i32p, ctypes.c_int]
    lib.og_update.restype = ctypes.c_int
    lib.og_update.argtypes = [P, ctypes.c_int, ctypes.c_int, i32p, i32p,
                              ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
    lib.og_update_set.restype = ctypes.c_int
    lib.og_update_set.argtypes = [P, ctypes.c_int, ctypes.c_int, i32p, i32p,
                                  i32p, ctypes.c_int64, ctypes.c_int]
    lib.og_and_sweep.restype = ctypes.c_int64
    lib.og_and_sweep.argtypes = [P, ctypes.c_int, ctypes.c_int, i32p, i64p]
    lib.og_levels.restype = ctypes.c_int32
    lib.og_levels.argtypes = [P, ctypes.c_int, ctypes.c_int, i32p]
    _lib = lib
    return lib


def _i32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _i64(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


class Graph:
    """A simple undirected graph held by the oracle."""

    def __init__(self, n: int, src, dst):
        lib = _load()
        src = np.ascontiguousarray(src, dtype=np.int32)
        dst = np.ascontiguousarray(dst, dtype=np.int32)
        if src.shape != dst.shape:
            raise ValueError("src and dst differ in length")
        h = lib.og_new(int(n), int(src.size), _i32(src), _i32(dst))
        if not h:
            raise ValueError(lib.og_last_error().decode())
        self._h = h
        self._lib = lib

    @classmethod
    def from_raw(cls, raw) -> "Graph":
        return cls(raw.n, raw.src, raw.dst)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.og_free(h)
            self._h = None

    def _check(self, rc):
        if rc < 0:
            raise RuntimeError(self._lib.og_last_error().decode())
        return rc

    @property
    def n(self) -> int:
        return int(self._lib.og_n(self._h))

    def csr(self):
        """Canonical CSR (row_off int64[n+1], col int32[2|E|])."""
        n, nnz = self.n, int(self._lib.og_nnz(self._h))
        row_off = np.zeros(n + 1, np.int64)
        col = np.zeros(max(nnz, 1), np.int32)
        self._lib.og_csr(self._h, _i64(row_off), _i32(col))
        return row_off, col[:nnz]

    def num_rcliques(self, r: int) -> int:
        return self._check(int(self._lib.og_num_rcliques(self._h, r)))

    def rcliques(self, r: int) -> np.ndarray:
        nr = self.num_rcliques(r)
        out = np.zeros((max(nr, 1), r), np.int32)
        self._check(self._lib.og_rcliques(self._h, r, _i32(out)))
        return out[:nr]

    def sdeg(self, r: int, s: int, threads: int | None = None) -> np.ndarray:
        nr = self.num_rcliques(r)
        ds = np.zeros(max(nr, 1), np.int32)
        self._check(self._lib.og_sdeg(self._h, r, s, _i32(ds),
                                      threads or default_threads()))
        return ds[:nr]

    def members(self, r: int, s: int, R: int) -> np.ndarray:
        """Other r-clique ids of each s-clique containing R, shape (d_s, k)."""
        from math import comb
        k = comb(s, r) - 1
        d = self._check(int(self._lib.og_members(self._h, r, s, R, None, 0)))
        out = np.zeros(max(d * k, 1), np.int32)
        self._check(int(self._lib.og_members(self._h, r, s, R, _i32(out),
                                             d * k)))
        return out[: d * k].reshape(d, k)

    def peel(self, r: int, s: int, threads: int | None = None) -> np.ndarray:
        nr = self.num_rcliques(r)
        kappa = np.zeros(max(nr, 1), np.int32)
        self._check(self._lib.og_peel(self._h, r, s, _i32(kappa),
                                      threads or default_threads()))
        return kappa[:nr]

    def update(self, r: int, s: int, tau, lo: int = 0, hi: int | None = None,
               threads: int | None = None, out=None) -> np.ndarray:
        """U tau on ids [lo, hi); other entries of the result copy tau."""
        nr = self.num_rcliques(r)
        tau = np.ascontiguousarray(tau, dtype=np.int32)
        if tau.size != nr:
            raise ValueError("tau has the wrong length")
        res = tau.copy() if out is None else out
        hi = nr if hi is None else hi
        if nr:
            self._check(self._lib.og_update(self._h, r, s, _i32(tau), _i32(res),
                                            lo, hi,
                                            threads or default_threads()))
        return res

    def snd(self, r: int, s: int, max_iters: int = 1 << 30,
            threads: int | None = None):
        """Alg. SND: returns the list [tau_0, tau_1, ..., tau_T] where
        tau_0 = d_s and tau_T is the first iterate equal to its predecessor
        (so tau_T = tau_{T-1} = kappa).  With no r-cliques: [empty]."""
        tau = self.sdeg(r, s, threads)
        seq = [tau]
        for _ in range(max_iters):
            nxt = self.update(r, s, tau, threads=threads)
            seq.append(nxt)
            if np.array_equal(nxt, tau):
                break
            tau = nxt
        return seq

    def update_set(self, r: int, s: int, tau, ids,
                   threads: int | None = None) -> np.ndarray:
        """U tau on the listed ids only; other entries copy tau."""
        nr = self.num_rcliques(r)
        tau = np.ascontiguousarray(tau, dtype=np.int32)
        if tau.size != nr:
            raise ValueError("tau has the wrong length")
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        res = tau.copy()
        if ids.size:
            self._check(self._lib.og_update_set(self._h, r, s, _i32(tau),
                                                _i32(res), _i32(ids), ids.size,
                                                threads or default_threads()))
        return res

    def partial_and(self, r: int, s: int, ids, max_iters: int = 1 << 30,
                    threads: int | None = None):
        """PartialAND (Section 4.3, end): the update operator applied only to
        the r-cliques in the set P = ids until none of them changes; every
        other r-clique keeps tau_0 = d_s.  Returns (tau, sweeps, converged)
        with tau over all r-cliques.

        Taken here as synchronous sweeps over P.  U restricted to P is
        monotone and tau_0 is above its image, so synchronous and in-place
        sweeps (in any order) descend to the same limit: the largest fixed
        point of the restricted operator below tau_0."""
        tau = self.sdeg(r, s, threads)
        P = np.unique(np.asarray(ids, dtype=np.int32))
        sweeps = 0
        while sweeps < max_iters:
            nxt = self.update_set(r, s, tau, P, threads)
            sweeps += 1
            if np.array_equal(nxt[P], tau[P]):
                return nxt, sweeps, True
            tau = nxt
        return tau, sweeps, P.size == 0

    def ego_set(self, r: int, s: int, q: int) -> np.ndarray:
        """The ego network of r-clique q used for its PartialAND estimate
        (the application of Section 5.3): q and every r-clique sharing an s-clique
        with q (its neighbours for r = 1, the edges of its triangles for
        r = 2, ...), sorted."""
        m = self.members(r, s, q).reshape(-1)
        return np.unique(np.concatenate([np.array([q], np.int32), m]))

    def ego_estimate(self, r: int, s: int, queries, threads: int | None = None):
        """PartialAND on each query's ego network; the estimate is the
        query's own resulting tau.  Returns (estimates, sweeps)."""
        est, sw = [], []
        for q in np.asarray(queries, dtype=np.int64):
            tau, n, _ = self.partial_and(r, s, self.ego_set(r, s, int(q)),
                                         threads=threads)
            est.append(int(tau[q]))
            sw.append(n)
        return np.array(est, np.int32), np.array(sw, np.int32)

    def and_sweep(self, r: int, s: int, tau, order=None) -> int:
        """One in-place Alg. AND sweep over tau (modified); returns #changed."""
        assert tau.dtype == np.int32 and tau.flags.c_contiguous
        o = None
        if order is not None:
            order = np.ascontiguousarray(order, dtype=np.int64)
            o = _i64(order)
        return self._check(int(self._lib.og_and_sweep(self._h, r, s, _i32(tau),
                                                      o)))

    def and_run(self, r: int, s: int, order=None, max_sweeps: int = 1 << 30):
        """Alg. AND until a sweep changes nothing; returns (tau, sweeps, seq)
        where seq holds tau after each sweep."""
        tau = self.sdeg(r, s).copy()
        seq = [tau.copy()]
        sweeps = 0
        while sweeps < max_sweeps:
            ch = self.and_sweep(r, s, tau, order)
            sweeps += 1
            seq.append(tau.copy())
            if ch == 0:
                break
        return tau, sweeps, seq

    def and_notify(self, r: int, s: int, order=None,
                   self_activate: bool = False, max_iters: int = 1 << 30):
        """Alg. AND with the notification mechanism (Section 4.3), sequential
        and in place, visiting r-cliques in `order` (default: id order, the
        natural order).  Every r-clique starts active.  An iteration visits
        the r-cliques that are active when it begins, marking each idle as
        it is visited; when R's value changes to h, every R' sharing an
        s-clique with R whose current value is at least h is marked active.
        The loop ends after the first iteration that changes nothing.

        Two readings are forced by the worked example of Section 4.3 (order
        a..f: only `a` active after the first iteration, `a` alone processed
        in the second, `b` and `e` in the third; 9 computations in 3
        iterations):
          * the work of an iteration is the active set at its start -- the
            parallel loop's view: `b` and `e`, notified by `a` in the second
            iteration, are recomputed in the third, though they come after
            `a` in the order; a notification that reaches an r-clique before
            its visit in the same iteration is cleared by that visit (`f` in
            the first);
          * no self-activation: the listing marks R itself active when it
            changes, which would keep `b` and `e` active after the first
            iteration (`self_activate` turns it on).
        Small graphs only (pure Python).

        Returns (tau, iterations, computations per iteration, active
        r-cliques after each iteration)."""
        nr = self.num_rcliques(r)
        tau = self.sdeg(r, s).astype(np.int64)
        mem = [self.members(r, s, R) for R in range(nr)]
        nbr = [np.unique(m.reshape(-1)) for m in mem]
        visit = range(nr) if order is None else [int(x) for x in order]
        active = np.ones(nr, bool)
        comps, act_after = [], []
        iters, changed_any = 0, True
        while changed_any and iters < max_iters:
            changed_any = False
            iters += 1
            n = 0
            for R in [R for R in visit if active[R]]:
                active[R] = False
                n += 1
                m = mem[R]
                rho = tau[m].min(axis=1) if m.size else np.zeros(0, np.int64)
                h = hindex(rho)
                if tau[R] != h:
                    changed_any = True
                    if self_activate:
                        active[R] = True
                    for Rp in nbr[R]:
                        if h <= tau[Rp]:
                            active[Rp] = True
                tau[R] = h
            comps.append(n)
            act_after.append(int(active.sum()))
        return tau.astype(np.int32), iters, comps, act_after

    def levels(self, r: int, s: int):
        """(level per r-clique, number of levels)."""
        nr = self.num_rcliques(r)
        lv = np.zeros(max(nr, 1), np.int32)
        nl = self._check(int(self._lib.og_levels(self._h, r, s, _i32(lv))))
        return lv[:nr], nl


def hindex(values) -> int:
    """H of a multiset of non-negative integers (Section 2.2)."""
    lib = _load()
    a = np.ascontiguousarray(values, dtype=np.int32)
    return int(lib.og_hindex(_i32(a), int(a.size)))
