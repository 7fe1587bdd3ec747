"""CPU oracle for the multi-scale LFK growth sweep (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never uses it.

The arithmetic lives in ``lcd_oracle.c`` (plain single-threaded C, built with
gcc, contraction off).  This module builds it, loads it with ctypes and
marshals numpy arrays; it computes nothing of the method itself.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lcd_oracle.c")
LIB = os.path.join(HERE, "liblcd_oracle.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (always, unless ``force`` is False and a
    library newer than the source already exists)."""
    if (not force and os.path.exists(LIB)
            and os.path.getmtime(LIB) >= os.path.getmtime(SRC)):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


class TraceRec(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int64), ("V", ctypes.c_int64),
                ("Kp", ctypes.c_int64), ("Vp", ctypes.c_int64),
                ("alpha", ctypes.c_double), ("t", ctypes.c_double),
                ("kind", ctypes.c_int32), ("result", ctypes.c_int32),
                ("node", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("mask", ctypes.c_uint64)]


class Trace(ctypes.Structure):
    _fields_ = [("rec", ctypes.POINTER(TraceRec)), ("cap", ctypes.c_int64),
                ("count", ctypes.c_int64)]


_lib = None


def lib():
    """The loaded oracle.  ``LCDO_LIB`` in the environment selects another
    build of the same source (used by the mutation test)."""
    global _lib
    if _lib is None:
        path = os.environ.get("LCDO_LIB")
        if not path:
            build(force=False)
            path = LIB
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        L.lcdo_log.restype = ctypes.c_double
        L.lcdo_log.argtypes = [ctypes.c_uint64]
        L.lcdo_rank.restype = ctypes.c_double
        L.lcdo_rank.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_double]
        L.lcdo_improves_export.restype = ctypes.c_int
        L.lcdo_improves_export.argtypes = [ctypes.c_int64] * 4 + [
            ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
        L.lcdo_log_many.restype = None
        L.lcdo_log_many.argtypes = [P, P, ctypes.c_int64]
        L.lcdo_ctx_new.restype = P
        L.lcdo_ctx_new.argtypes = [ctypes.c_int32, P, P, P]
        L.lcdo_ctx_free.restype = None
        L.lcdo_ctx_free.argtypes = [P]
        L.lcdo_degrees.restype = P
        L.lcdo_degrees.argtypes = [P]
        L.lcdo_run_set.restype = ctypes.c_int
        L.lcdo_run_set.argtypes = [P, P, ctypes.c_int32, P, ctypes.c_int32,
                                   ctypes.c_uint32, P, ctypes.c_int64, P, P, P, P,
                                   P, ctypes.POINTER(Trace)]
        L.lcdo_run_merge.restype = ctypes.c_int
        L.lcdo_run_merge.argtypes = [P, P, P, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_uint32,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_int64), P, P, P, P, P, P, P, P]
        L.lcdo_seeds.restype = ctypes.c_int64
        L.lcdo_seeds.argtypes = [P, P, ctypes.c_int, P]
        L.lcdo_run_sets.restype = ctypes.c_int
        L.lcdo_run_sets.argtypes = [P, P, P, ctypes.c_int32, P, ctypes.c_int32,
                                    ctypes.c_uint32, P, ctypes.c_int64, P, P, P, P,
                                    P, P, P]
        L.lcdo_nmi.restype = ctypes.c_double
        L.lcdo_nmi.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_int32, P, P]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def log(x) -> np.ndarray:
    x = np.ascontiguousarray(np.asarray(x, dtype=np.uint64))
    out = np.empty(x.shape, dtype=np.float64)
    lib().lcdo_log_many(_ptr(x), _ptr(out), x.size)
    return out


def improves(Kp: int, Vp: int, K: int, V: int, alpha: float):
    t = ctypes.c_double()
    r = lib().lcdo_improves_export(Kp, Vp, K, V, alpha, ctypes.byref(t))
    return bool(r), t.value


def rank(d: int, k: int, alpha: float) -> float:
    return lib().lcdo_rank(d, k, alpha)


def _cover_csr(cover):
    """A cover as (int64 offsets, int32 members): a list of node-id arrays,
    or an (offsets, members) pair already in that form."""
    if isinstance(cover, tuple):
        ptr, mem = cover
        return (np.ascontiguousarray(ptr, dtype=np.int64), np.ascontiguousarray(mem, dtype=np.int32))
    sizes = [len(c) for c in cover]
    ptr = np.zeros(len(cover) + 1, np.int64)
    np.cumsum(sizes, out=ptr[1:])
    mem = (np.concatenate([np.asarray(c, np.int32) for c in cover]) if cover and ptr[-1] > 0
           else np.zeros(1, np.int32))
    return ptr, np.ascontiguousarray(mem, dtype=np.int32)


def nmi(n: int, cover_x, cover_y) -> float:
    """Normalised mutual information of two covers of n nodes (the
    overlapping-community definition the paper uses in Sec. 4; readings N1-N4
    in lcd_oracle.c).  A cover is a list of node-id arrays (each without
    repeats) or an (offsets, members) pair."""
    px, mx = _cover_csr(cover_x)
    py, my = _cover_csr(cover_y)
    v = lib().lcdo_nmi(int(n), px.size - 1, _ptr(px), _ptr(mx), py.size - 1, _ptr(py), _ptr(my))
    if v < -1.0:
        raise MemoryError("lcdo_nmi")
    return v


def nmi_successive(n: int, covers, p: int) -> np.ndarray:
    """Sec. 4's NMI averaged over p successive scales: for every window of
    p consecutive covers starting at scale s, the mean of the NMI of its
    p - 1 consecutive pairs (reading N5); len(covers) - p + 1 values."""
    if p < 2 or p > len(covers):
        raise ValueError("p must be in [2, number of scales]")
    pair = [nmi(n, covers[t], covers[t + 1]) for t in range(len(covers) - 1)]
    out = []
    for s in range(len(covers) - p + 1):
        acc = 0.0
        for t in range(s, s + p - 1):
            acc += pair[t]
        out.append(acc / (p - 1))
    return np.array(out, dtype=np.float64)


class Oracle:
    """The oracle bound to one graph (arrays are kept alive here)."""

    def __init__(self, n: int, row_ptr, col, w=None):
        self.n = int(n)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.w = None if w is None else np.ascontiguousarray(w, dtype=np.uint8)
        self._ctx = lib().lcdo_ctx_new(self.n, _ptr(self.row_ptr), _ptr(self.col),
                                       _ptr(self.w))
        if not self._ctx:
            raise MemoryError("oracle context")

    @classmethod
    def from_graph(cls, g):
        return cls(g.n, g.row_ptr, g.col, g.w)

    def close(self):
        if self._ctx:
            lib().lcdo_ctx_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run_merge(self, seed_ptr, seed_nodes, scales, k_prune: int = 0, eta=(1, 2),
                  max_rounds: int = 100000) -> dict:
        """Algorithm 2 with its check-and-merge phase; records laid out like
        run_sets(), plus into[R] (-1 live, else the live id merged into) and
        rounds[S]."""
        sp = np.ascontiguousarray(seed_ptr, dtype=np.int32)
        sn = np.ascontiguousarray(seed_nodes, dtype=np.int32)
        sc = np.ascontiguousarray(scales, dtype=np.float64)
        ns, S = sp.size - 1, sc.size
        R = ns * S
        off = np.zeros(max(R, 1), np.int64)
        cnt = np.zeros(max(R, 1), np.int32)
        K = np.zeros(max(R, 1), np.int64)
        V = np.zeros(max(R, 1), np.int64)
        f = np.zeros(max(R, 1), np.float64)
        ctr = np.zeros(max(R, 1) * 4, np.uint64)
        into = np.zeros(max(R, 1), np.int32)
        rounds = np.zeros(max(S, 1), np.int32)
        needed = ctypes.c_int64()
        cap = max(1024, 4 * self.n)
        for _ in range(4):
            members = np.empty(cap, np.int32)
            rc = lib().lcdo_run_merge(self._ctx, _ptr(sp), _ptr(sn), ns, _ptr(sc), S, k_prune,
                                      int(eta[0]), int(eta[1]), max_rounds, _ptr(members), cap,
                                      ctypes.byref(needed), _ptr(off), _ptr(cnt), _ptr(K), _ptr(V),
                                      _ptr(f), _ptr(ctr), _ptr(into), _ptr(rounds))
            if rc == -1:
                cap = needed.value
                continue
            if rc != 0:
                raise RuntimeError("lcdo_run_merge failed (%d)" % rc)
            return dict(members=members[:needed.value].copy(), off=off[:R], cnt=cnt[:R], K=K[:R], V=V[:R],
                        f=f[:R], ctr=ctr[:R * 4].reshape(R, 4), into=into[:R], rounds=rounds[:S],
                        n_sets=ns, n_scales=S)
        raise RuntimeError("lcdo_run_merge: member buffer did not converge")

    def seeds(self, perm, rule: int = 1) -> np.ndarray:
        """Seed selection of Algorithm 2 (rule 1 or 2) visiting nodes in the
        order perm; the seeds in order of selection."""
        perm = np.ascontiguousarray(perm, dtype=np.int32)
        out = np.empty(max(self.n, 1), dtype=np.int32)
        k = lib().lcdo_seeds(self._ctx, _ptr(perm), rule, _ptr(out))
        if k < 0:
            raise ValueError("perm is not a permutation of the nodes, or rule is not 1 or 2")
        return out[:k].copy()

    def degrees(self) -> np.ndarray:
        p = lib().lcdo_degrees(self._ctx)
        return np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(ctypes.c_int64)),
                                     shape=(self.n,)).copy()

    def run_sets(self, seed_ptr, seed_nodes, scales, k_prune: int = 0,
                 members_cap: Optional[int] = None) -> dict:
        """Grow every seed set through every scale.  Record r = j*S + s."""
        seed_ptr = np.ascontiguousarray(seed_ptr, dtype=np.int32)
        seed_nodes = np.ascontiguousarray(seed_nodes, dtype=np.int32)
        scales = np.ascontiguousarray(scales, dtype=np.float64)
        ns = seed_ptr.size - 1
        S = scales.size
        R = ns * S
        cap = members_cap if members_cap is not None else max(1024, R * 64)
        while True:
            members = np.empty(cap, dtype=np.int32)
            off = np.empty(R, dtype=np.int64)
            cnt = np.empty(R, dtype=np.int32)
            K = np.empty(R, dtype=np.int64)
            V = np.empty(R, dtype=np.int64)
            f = np.empty(R, dtype=np.float64)
            ctr = np.empty(R * 4, dtype=np.uint64)
            needed = ctypes.c_int64()
            rc = lib().lcdo_run_sets(self._ctx, _ptr(seed_ptr), _ptr(seed_nodes), ns,
                                     _ptr(scales), S, k_prune, _ptr(members), cap,
                                     ctypes.byref(needed), _ptr(off), _ptr(cnt), _ptr(K),
                                     _ptr(V), _ptr(f), _ptr(ctr))
            if rc == 0:
                break
            if rc != -1:
                raise RuntimeError("oracle failed (%d)" % rc)
            cap = int(needed.value)
        return dict(members=members[:needed.value], off=off, cnt=cnt, K=K, V=V, f=f,
                    ctr=ctr.reshape(R, 4), n_sets=ns, n_scales=S)

    def run_set(self, seeds, scales, k_prune: int = 0, trace_cap: int = 0):
        """One seed set; returns (list of member arrays per scale, K, V, f,
        counters [S,4], trace records list)."""
        seeds = np.ascontiguousarray(seeds, dtype=np.int32)
        scales = np.ascontiguousarray(scales, dtype=np.float64)
        S = scales.size
        cap = max(1024, self.n * S)
        members = np.empty(cap, dtype=np.int32)
        off = np.empty(S + 1, dtype=np.int64)
        K = np.empty(S, dtype=np.int64)
        V = np.empty(S, dtype=np.int64)
        f = np.empty(S, dtype=np.float64)
        ctr = np.empty(S * 4, dtype=np.uint64)
        tr = None
        recs = None
        if trace_cap:
            recs = (TraceRec * trace_cap)()
            tr = Trace(ctypes.cast(recs, ctypes.POINTER(TraceRec)), trace_cap, 0)
        rc = lib().lcdo_run_set(self._ctx, _ptr(seeds), seeds.size, _ptr(scales), S,
                                k_prune, _ptr(members), cap, _ptr(off), _ptr(K), _ptr(V),
                                _ptr(f), _ptr(ctr), ctypes.byref(tr) if tr else None)
        if rc != 0:
            raise RuntimeError("oracle member buffer too small")
        per = [members[off[s]:off[s + 1]].copy() for s in range(S)]
        trace = []
        if tr is not None:
            if tr.count > trace_cap:
                raise RuntimeError("trace capacity %d < %d" % (trace_cap, tr.count))
            for i in range(tr.count):
                r = recs[i]
                trace.append(dict(kind=r.kind, K=r.K, V=r.V, Kp=r.Kp, Vp=r.Vp, alpha=r.alpha,
                                  t=r.t, result=r.result, node=r.node, mask=r.mask))
        return per, K, V, f, ctr.reshape(S, 4), trace


def records_to_sets(res: dict, j: int, s: int) -> np.ndarray:
    r = j * res["n_scales"] + s
    o = res["off"][r]
    return res["members"][o:o + res["cnt"][r]]
