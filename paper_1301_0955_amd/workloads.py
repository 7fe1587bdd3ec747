"""Seeded synthetic inputs for the multi-scale local community sweep.

This module only *makes inputs*: graphs, seed sets, scale lists and query
streams.  It holds none of the method's arithmetic (no fitness, no ranking,
no growth), so both the CPU oracle and the HIP path can be fed from it
without sharing any of the computation they are compared on.

Shapes follow the paper's experimental set-up (Sec. 4): networks with
communities nested at two or three levels whose members send a fraction
``mu`` of their edges out of the community, generated in the spirit of the
Lancichinetti--Fortunato hierarchical benchmark.  That generator is not
reproduced here; the procedure below is our own (power-law degrees and
community sizes, per-level stub matching inside buckets, duplicate and
self-loop removal).

Every generator takes an explicit integer ``seed`` and uses numpy's PCG64
stream, so a (generator, parameters, seed) triple always yields the same
bytes.  Streams: graph = seed, seed permutation = seed + 1, edge weights =
seed + 2, query stream = seed + 3.
"""
from __future__ import annotations

import ctypes
import dataclasses
import hashlib
import math
import os
import subprocess
from typing import Optional

import numpy as np

_GEN_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gen")
_GEN_SRC = os.path.join(_GEN_DIR, "lfr_gen.c")
_GEN_LIB = os.path.join(_GEN_DIR, "liblfr_gen.so")
_gen = None


def build_generator(force: bool = True) -> str:
    """Compile the C part of the input generator (gen/lfr_gen.c) with gcc."""
    if (not force and os.path.exists(_GEN_LIB)
            and os.path.getmtime(_GEN_LIB) >= os.path.getmtime(_GEN_SRC)):
        return _GEN_LIB
    tmp = _GEN_LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", _GEN_SRC, "-o", tmp],
                   check=True)
    os.replace(tmp, _GEN_LIB)
    return _GEN_LIB


def _genlib():
    global _gen
    if _gen is None:
        L = ctypes.CDLL(build_generator(force=False))
        P = ctypes.c_void_p
        L.lfrgen_match.restype = ctypes.c_int64
        L.lfrgen_match.argtypes = [ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_int32,
                                   ctypes.c_uint64, P, P, ctypes.c_int64]
        L.lfrgen_csr.restype = ctypes.c_int
        L.lfrgen_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, ctypes.c_int32,
                                 ctypes.c_uint64, P, P, P]
        L.lfrgen_seed_rule1.restype = ctypes.c_int64
        L.lfrgen_seed_rule1.argtypes = [ctypes.c_int64, P, P, P, P]
        L.lfrgen_assign.restype = ctypes.c_int
        L.lfrgen_assign.argtypes = [ctypes.c_int64, P, P, ctypes.c_int64, P, ctypes.c_uint64, P]
        _gen = L
    return _gen


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


@dataclasses.dataclass
class Graph:
    """Undirected graph in symmetric CSR form.

    ``row_ptr`` int32[n+1], ``col`` int32[nnz] with every row sorted
    ascending, no self-loops and no duplicate neighbours; ``w`` is uint8[nnz]
    (the same weight on both directions of an edge) or ``None`` for an
    unweighted graph (every weight 1).
    """

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    w: Optional[np.ndarray]
    meta: dict

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def degree(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr).tobytes())
        h.update(np.ascontiguousarray(self.col).tobytes())
        if self.w is not None:
            h.update(np.ascontiguousarray(self.w).tobytes())
        return h.hexdigest()

    def csr_bytes(self) -> int:
        b = self.row_ptr.nbytes + self.col.nbytes
        if self.w is not None:
            b += self.w.nbytes
        return b


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray,
                   w: Optional[np.ndarray], meta: Optional[dict] = None) -> Graph:
    """Symmetric CSR from an undirected edge list.

    Self-loops are dropped; a pair listed more than once keeps its first
    weight.  Rows come out sorted by neighbour id.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    if w is not None:
        w = np.asarray(w, dtype=np.uint8)[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = lo * np.int64(n) + hi
    key_u, first = np.unique(key, return_index=True)
    lo = key_u // n
    hi = key_u % n
    if w is not None:
        w = w[first]
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    order = np.lexsort((dst, src))
    src = src[order]
    dst = dst[order]
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    ww = None
    if w is not None:
        ww = np.concatenate([w, w])[order].astype(np.uint8)
    return Graph(n=int(n), row_ptr=row_ptr.astype(np.int32),
                 col=dst.astype(np.int32), w=ww, meta=dict(meta or {}))


# ---------------------------------------------------------------------------
# Two-level planted partition (the small case)
# ---------------------------------------------------------------------------

def planted_partition(n: int = 1000, group: int = 250, sub: int = 50,
                      p_sub: float = 0.3, p_group: float = 0.03,
                      p_out: float = 0.002, seed: int = 1) -> Graph:
    """Node i belongs to group i // group and sub-community i // sub; each
    pair i < j is an edge with probability p_sub (same sub-community),
    p_group (same group, other sub-community) or p_out (otherwise).
    Unweighted."""
    rng = _rng(seed)
    iu, ju = np.triu_indices(n, 1)
    same_sub = (iu // sub) == (ju // sub)
    same_grp = (iu // group) == (ju // group)
    p = np.where(same_sub, p_sub, np.where(same_grp, p_group, p_out))
    pick = rng.random(iu.shape[0]) < p
    meta = dict(kind="planted_partition", n=n, group=group, sub=sub,
                p_sub=p_sub, p_group=p_group, p_out=p_out, seed=seed)
    return csr_from_edges(n, iu[pick], ju[pick], None, meta)


# ---------------------------------------------------------------------------
# Hierarchical LFR-style generator (medium / large cases)
# ---------------------------------------------------------------------------

def _powerlaw_pmf(lo: int, hi: int, tau: float) -> tuple[np.ndarray, np.ndarray]:
    ks = np.arange(lo, hi + 1, dtype=np.float64)
    p = ks ** (-tau)
    return ks, p / p.sum()


def _sample_discrete(rng, ks, p, size):
    cdf = np.cumsum(p)
    cdf[-1] = 1.0
    idx = np.searchsorted(cdf, rng.random(size), side="right")
    return ks[np.minimum(idx, len(ks) - 1)].astype(np.int64)


def powerlaw_degrees(rng, n: int, tau: float, mean: float, kmax: int) -> np.ndarray:
    """Discrete power law P(k) ~ k^-tau on [kmin, kmax].  The integer kmin
    that brackets the target mean is mixed with kmin + 1 so the expected
    mean equals ``mean``."""
    means = {}
    for a in range(1, kmax):
        ks, p = _powerlaw_pmf(a, kmax, tau)
        means[a] = float((ks * p).sum())
    a = max(k for k, m in means.items() if m <= mean) if any(
        m <= mean for m in means.values()) else 1
    if a + 1 >= kmax:
        ks, p = _powerlaw_pmf(a, kmax, tau)
        return _sample_discrete(rng, ks, p, n)
    m0, m1 = means[a], means[a + 1]
    q = 1.0 if m1 == m0 else (m1 - mean) / (m1 - m0)
    q = min(max(q, 0.0), 1.0)
    ks0, p0 = _powerlaw_pmf(a, kmax, tau)
    ks1, p1 = _powerlaw_pmf(a + 1, kmax, tau)
    d0 = _sample_discrete(rng, ks0, p0, n)
    d1 = _sample_discrete(rng, ks1, p1, n)
    return np.where(rng.random(n) < q, d0, d1)


def community_sizes(rng, n: int, tau: float, smin: int, smax: int) -> np.ndarray:
    ks, p = _powerlaw_pmf(smin, smax, tau)
    mean = float((ks * p).sum())
    out = []
    total = 0
    while total < n:
        batch = _sample_discrete(rng, ks, p, max(16, int(1.2 * (n - total) / mean) + 16))
        for s in batch:
            out.append(int(s))
            total += int(s)
            if total >= n:
                break
    sizes = np.array(out, dtype=np.int64)
    excess = int(sizes.sum() - n)
    sizes[-1] -= excess
    if sizes[-1] < smin and len(sizes) > 1:
        sizes[-2] += sizes[-1]
        sizes = sizes[:-1]
    return sizes


def _match_stubs(rng, nodes: np.ndarray, bucket: np.ndarray):
    """Random perfect matching of stubs inside each bucket (one stub left
    over in odd buckets).  Returns two endpoint arrays."""
    if nodes.size == 0:
        return nodes[:0], nodes[:0]
    key = rng.random(nodes.size)
    order = np.lexsort((key, bucket))
    nodes = nodes[order]
    bucket = bucket[order]
    starts = np.flatnonzero(np.r_[True, bucket[1:] != bucket[:-1]])
    sizes = np.diff(np.r_[starts, bucket.size])
    start_of = np.repeat(starts, sizes)
    pos = np.arange(bucket.size) - start_of
    size_of = np.repeat(sizes, sizes)
    first = (pos % 2 == 0) & (pos + 1 < size_of)
    i = np.flatnonzero(first)
    return nodes[i], nodes[i + 1]


def lfr_hierarchical(n: int, tau_deg: float, mean_deg: float, max_deg: int,
                     tau_comm: float = 1.5, cmin: int = 20, cmax: int = 200,
                     mu: float = 0.3, levels: int = 2, fan: int = 10,
                     weighted: bool = False, wmax: int = 16,
                     seed: int = 1, rematch_rounds: int = 6) -> Graph:
    """Power-law graph with communities nested ``levels`` deep.

    level 1: communities (sizes ~ s^-tau_comm on [cmin, cmax]);
    level 2: groups of ``fan`` communities; level 3: groups of ``fan`` groups.
    A node sends a fraction 1 - mu of its stubs inside its community; the
    remaining mu is halved at each further level (mu/2 inside the group and
    mu/2 outside for two levels; mu/2, mu/4 and mu/4 for three levels).
    Stubs are matched uniformly at random inside each bucket; a pair that is
    a self-loop or repeats an existing edge is undone and its stubs are
    matched again (``rematch_rounds`` times), so realised degrees can fall a
    little below the drawn ones (the achieved values are in ``meta``).
    Node ids are a random permutation of the community layout.
    """
    if levels not in (2, 3):
        raise ValueError("levels must be 2 or 3")
    rng = _rng(seed)
    deg = powerlaw_degrees(rng, n, tau_deg, mean_deg, max_deg)
    sizes = community_sizes(rng, n, tau_comm, cmin, cmax)
    perm = rng.permutation(n)
    comm_of = np.empty(n, dtype=np.int64)
    comm_of[perm] = np.repeat(np.arange(sizes.size), sizes)
    csize = sizes[comm_of]
    grp_of = comm_of // fan
    sup_of = grp_of // fan
    if levels == 2:
        fracs = [1.0 - mu, mu / 2.0, mu / 2.0]
        buckets = [comm_of, grp_of, np.zeros(n, dtype=np.int64)]
    else:
        fracs = [1.0 - mu, mu / 2.0, mu / 4.0, mu / 4.0]
        buckets = [comm_of, grp_of, sup_of, np.zeros(n, dtype=np.int64)]
    stubs = []
    rem = deg.copy()
    for li, f in enumerate(fracs[:-1]):
        s = np.floor(f * deg + rng.random(n)).astype(np.int64)
        if li == 0:
            s = np.minimum(s, csize - 1)
        s = np.minimum(s, rem)
        stubs.append(s)
        rem = rem - s
    stubs.append(rem)
    us, vs = [], []
    have = np.zeros(0, dtype=np.int64)          # sorted keys of accepted pairs
    for s, b in zip(stubs, buckets):
        pool = np.repeat(np.arange(n, dtype=np.int64), s)
        for _ in range(rematch_rounds):
            if pool.size < 2:
                break
            a, c = _match_stubs(rng, pool, b[pool])
            paired = np.zeros(pool.size, dtype=bool)
            # stubs left unpaired in odd buckets go back to the pool
            lo = np.minimum(a, c)
            hi = np.maximum(a, c)
            key = lo * np.int64(n) + hi
            ok = a != c
            _, first = np.unique(key, return_index=True)
            firstmask = np.zeros(key.size, dtype=bool)
            firstmask[first] = True
            ok &= firstmask
            if have.size:
                pos = np.searchsorted(have, key)
                pos = np.minimum(pos, have.size - 1)
                ok &= have[pos] != key
            us.append(a[ok])
            vs.append(c[ok])
            have = np.union1d(have, key[ok])
            # rebuild the pool from rejected pairs and the odd stubs
            used = np.concatenate([a[ok], c[ok]])
            cnt_pool = np.bincount(pool, minlength=n)
            cnt_used = np.bincount(used, minlength=n)
            left = cnt_pool - cnt_used
            pool = np.repeat(np.arange(n, dtype=np.int64), left)
            del paired
            if pool.size < 0.002 * s.sum() + 2:
                break
    u = np.concatenate(us)
    v = np.concatenate(vs)
    w = None
    # weights are drawn per undirected edge after de-duplication below
    g = csr_from_edges(n, u, v, None)
    if weighted:
        wr = _rng(seed + 2)
        src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_ptr))
        dst = g.col.astype(np.int64)
        upper = src < dst
        m = int(upper.sum())
        wu = wr.integers(1, wmax + 1, size=m, dtype=np.int64).astype(np.uint8)
        # the same weight on both directions: index every edge by its
        # position in the upper-triangle enumeration
        key_all = np.minimum(src, dst) * np.int64(n) + np.maximum(src, dst)
        key_up = key_all[upper]
        pos = np.searchsorted(key_up, key_all)
        w = wu[pos]
        g.w = w
    # achieved structure
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.row_ptr))
    dst = g.col.astype(np.int64)
    same_c = comm_of[src] == comm_of[dst]
    same_g = grp_of[src] == grp_of[dst]
    meta = dict(kind="lfr_hierarchical", n=n, tau_deg=tau_deg, mean_deg=mean_deg,
                max_deg=max_deg, tau_comm=tau_comm, cmin=cmin, cmax=cmax, mu=mu,
                levels=levels, fan=fan, weighted=weighted, wmax=wmax, seed=seed,
                n_comms=int(sizes.size),
                achieved_mean_deg=float(g.nnz / n),
                achieved_max_deg=int(np.diff(g.row_ptr).max()),
                achieved_mu_comm=float(1.0 - same_c.mean()) if g.nnz else 0.0,
                achieved_mu_group=float(1.0 - same_g.mean()) if g.nnz else 0.0)
    g.meta = meta
    g.meta["_comm_of"] = comm_of
    return g


def lfr_hierarchical_fast(n: int, tau_deg: float, mean_deg: float, max_deg: int,
                          tau_comm: float = 1.5, cmin: int = 20, cmax: int = 200,
                          mu: float = 0.3, levels: int = 3, fan: int = 10,
                          weighted: bool = True, wmax: int = 16, seed: int = 1,
                          rematch_rounds: int = 6) -> Graph:
    """The construction of ``lfr_hierarchical`` for graphs of 10^7 nodes.
    Degrees, community sizes and the stubs per level are drawn with numpy
    as there.  Nodes are not placed in communities by a plain permutation:
    as in the Lancichinetti-Fortunato construction, a node goes to a
    community that can hold its internal stubs (size above (1 - mu) times
    its degree), drawn at random among those with room, largest needs first
    (gen/lfr_gen.c), so that hubs do not leak their edges out of small
    communities; community ids are then shuffled before they are grouped
    ``fan`` at a time.  The stub matching (shuffle inside each bucket, pair
    in order, undo self-loops and repeated pairs and match their stubs
    again) and the CSR assembly run in C on splitmix64 streams.  Weights
    are uniform in 1..wmax per undirected edge."""
    if levels not in (2, 3):
        raise ValueError("levels must be 2 or 3")
    L = _genlib()
    rng = _rng(seed)
    deg = powerlaw_degrees(rng, n, tau_deg, mean_deg, max_deg)
    sizes = community_sizes(rng, n, tau_comm, cmin, cmax)
    by_size = np.argsort(-sizes, kind="stable")
    need = np.minimum(np.ceil((1.0 - mu) * deg).astype(np.int64) + 1, int(sizes.max()))
    order = np.lexsort((rng.random(n), -need)).astype(np.int64)
    slot = np.empty(n, np.int64)
    need = np.ascontiguousarray(need, dtype=np.int64)
    sorted_sizes = np.ascontiguousarray(sizes[by_size], dtype=np.int64)   # held across the call
    if L.lfrgen_assign(n, need.ctypes.data, order.ctypes.data, sizes.size,
                       sorted_sizes.ctypes.data, int(seed), slot.ctypes.data) != 0:
        raise MemoryError("lfrgen_assign failed")
    relabel = rng.permutation(sizes.size)          # random ids before grouping
    comm_of = relabel[by_size[slot]]
    csize = np.bincount(comm_of, minlength=sizes.size)[comm_of]
    grp_of = comm_of // fan
    sup_of = grp_of // fan
    if levels == 2:
        fracs = [1.0 - mu, mu / 2.0, mu / 2.0]
        buckets = [comm_of, grp_of, np.zeros(n, dtype=np.int64)]
    else:
        fracs = [1.0 - mu, mu / 2.0, mu / 4.0, mu / 4.0]
        buckets = [comm_of, grp_of, sup_of, np.zeros(n, dtype=np.int64)]
    stubs = []
    rem = deg.copy()
    for li, f in enumerate(fracs[:-1]):
        s = np.floor(f * deg + rng.random(n)).astype(np.int64)
        if li == 0:
            s = np.minimum(s, csize - 1)
        s = np.minimum(s, rem)
        stubs.append(s)
        rem = rem - s
    stubs.append(rem)
    st = np.ascontiguousarray(np.stack(stubs), dtype=np.int64)
    bk = np.ascontiguousarray(np.stack(buckets), dtype=np.int64)
    cap = int(st.sum() // 2 + 16)
    u = np.empty(cap, np.int32)
    v = np.empty(cap, np.int32)
    m = L.lfrgen_match(n, len(fracs), st.ctypes.data, bk.ctypes.data, rematch_rounds,
                       int(seed), u.ctypes.data, v.ctypes.data, cap)
    if m < 0:
        raise MemoryError("lfrgen_match failed (%d)" % m)
    del st, bk
    if 2 * m >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    row_ptr = np.empty(n + 1, np.int32)
    col = np.empty(2 * m, np.int32)
    w = np.empty(2 * m, np.uint8) if weighted else None
    if L.lfrgen_csr(n, m, u.ctypes.data, v.ctypes.data, wmax if weighted else 0,
                    int(seed) + 2, row_ptr.ctypes.data, col.ctypes.data,
                    w.ctypes.data if weighted else None) != 0:
        raise MemoryError("lfrgen_csr failed")
    del u, v
    g = Graph(n=int(n), row_ptr=row_ptr, col=col, w=w, meta={})
    src = np.repeat(np.arange(n, dtype=np.int32), np.diff(row_ptr))
    same_c = comm_of[src] == comm_of[col]
    same_g = grp_of[src] == grp_of[col]
    g.meta = dict(kind="lfr_hierarchical_fast", n=n, tau_deg=tau_deg, mean_deg=mean_deg,
                  max_deg=max_deg, tau_comm=tau_comm, cmin=cmin, cmax=cmax, mu=mu,
                  levels=levels, fan=fan, weighted=weighted, wmax=wmax, seed=seed,
                  n_comms=int(sizes.size),
                  achieved_mean_deg=float(g.nnz / n),
                  achieved_max_deg=int(np.diff(row_ptr).max()),
                  achieved_mu_comm=float(1.0 - same_c.mean()) if g.nnz else 0.0,
                  achieved_mu_group=float(1.0 - same_g.mean()) if g.nnz else 0.0)
    g.meta["_comm_of"] = comm_of
    return g


# ---------------------------------------------------------------------------
# Block graphs with communities of tens of thousands of nodes
# ---------------------------------------------------------------------------

def block_graph(n_blocks: int, size: int, deg_in: int, deg_out: int, weighted: bool, seed: int,
                wmax: int = 16) -> Graph:
    """n_blocks blocks of `size` consecutive node ids; every node draws
    deg_in partners uniformly inside its block and deg_out uniformly over the
    whole graph (duplicates and self-pairs dropped).  Sparse, so blocks of
    tens of thousands of nodes cost O(n) memory: a community that grows over
    a block holds tens of thousands of table entries."""
    rng = _rng(seed)
    n = n_blocks * size
    node = np.arange(n, dtype=np.int64)
    base = (node // size) * size
    u_in = np.repeat(node, deg_in)
    v_in = np.repeat(base, deg_in) + rng.integers(0, size, size=u_in.size)
    u_out = np.repeat(node, deg_out)
    v_out = rng.integers(0, n, size=u_out.size)
    u = np.concatenate([u_in, u_out])
    v = np.concatenate([v_in, v_out])
    w = rng.integers(1, wmax + 1, size=u.size).astype(np.uint8) if weighted else None
    return csr_from_edges(n, u, v, w, dict(kind="blocks", n_blocks=n_blocks, size=size, deg_in=deg_in,
                                           deg_out=deg_out, weighted=weighted, seed=seed))


# ---------------------------------------------------------------------------
# Tiny random graphs for exhaustive checks
# ---------------------------------------------------------------------------

def random_graph(n: int, p: float, weighted: bool, seed: int, wmax: int = 5) -> Graph:
    rng = _rng(seed)
    iu, ju = np.triu_indices(n, 1)
    pick = rng.random(iu.shape[0]) < p
    u, v = iu[pick], ju[pick]
    w = rng.integers(1, wmax + 1, size=u.size).astype(np.uint8) if weighted else None
    return csr_from_edges(n, u, v, w, dict(kind="random", n=n, p=p, seed=seed))


# ---------------------------------------------------------------------------
# Scales, seeds, queries
# ---------------------------------------------------------------------------

def log_scales(X: int, vmin: float = 0.5, vmax: float = 1.0) -> np.ndarray:
    """X scale values from vmax down to vmin, dense near vmin.

    The paper's sampling formula (Sec. 4) is garbled in print; the reading
    used here is alpha_i = vmin + (vmax - vmin) * (1 - ln i / ln X) for
    i = 1..X, which stays inside [vmin, vmax], clusters values near vmin and
    comes out in order of increasing coarseness (decreasing alpha).
    """
    if X < 1:
        raise ValueError("X >= 1")
    if X == 1:
        return np.array([vmax], dtype=np.float64)
    i = np.arange(1, X + 1, dtype=np.float64)
    return vmin + (vmax - vmin) * (1.0 - np.log(i) / np.log(float(X)))


def singleton_seeds(n: int) -> tuple[np.ndarray, np.ndarray]:
    return (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32))


def seed_permutation(g: Graph, seed: int) -> np.ndarray:
    """The random visiting order of the seed rules (node ids, int32)."""
    return _rng(seed + 1).permutation(g.n).astype(np.int32)


def seed_rule1(g: Graph, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """The paper's first seed rule (Sec. 3, seed initialisation of
    Algorithm 2): candidates are the nodes with at least two neighbours;
    repeatedly pick a candidate at random, make it a seed and drop it and its
    neighbours from the candidates.  "At random" is a seeded permutation
    scanned in order; seed sets are singletons in order of selection."""
    perm = _rng(seed + 1).permutation(g.n)
    deg = np.diff(g.row_ptr)
    cand = (deg >= 2)
    rp = g.row_ptr
    col = g.col
    out = []
    cand_l = cand  # numpy bool array; slice assignment clears neighbours
    for v in perm.tolist():
        if cand_l[v]:
            out.append(v)
            cand_l[v] = False
            cand_l[col[rp[v]:rp[v + 1]]] = False
    nodes = np.array(out, dtype=np.int32)
    return np.arange(nodes.size + 1, dtype=np.int32), nodes


def seed_rule1_fast(g: Graph, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """``seed_rule1`` with the scan in C (same permutation, same seeds)."""
    perm = _rng(seed + 1).permutation(g.n).astype(np.int32)
    out = np.empty(max(g.n, 1), np.int32)
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)    # held across the call
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    k = _genlib().lfrgen_seed_rule1(g.n, rp.ctypes.data, col.ctypes.data, perm.ctypes.data,
                                    out.ctypes.data)
    if k < 0:
        raise MemoryError("lfrgen_seed_rule1 failed")
    nodes = out[:k].copy()
    return np.arange(nodes.size + 1, dtype=np.int32), nodes


def subsample_sets(seed_ptr: np.ndarray, seed_nodes: np.ndarray, stride: int,
                   offset: int = 0) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Every ``stride``-th seed set.  Returns (ptr, nodes, picked set ids)."""
    ids = np.arange(offset, seed_ptr.size - 1, stride)
    sizes = seed_ptr[ids + 1] - seed_ptr[ids]
    ptr = np.zeros(ids.size + 1, dtype=np.int32)
    np.cumsum(sizes, out=ptr[1:])
    nodes = np.concatenate([seed_nodes[seed_ptr[i]:seed_ptr[i + 1]] for i in ids]) \
        if ids.size else np.zeros(0, dtype=np.int32)
    return ptr, nodes.astype(np.int32), ids


def bfs_prefix(g: Graph, root: int, size: int) -> np.ndarray:
    """First ``size`` nodes reached by a breadth-first search from ``root``
    (neighbours visited in ascending id order)."""
    seen = {root}
    order = [root]
    head = 0
    while head < len(order) and len(order) < size:
        u = order[head]
        head += 1
        for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]].tolist():
            if v not in seen:
                seen.add(v)
                order.append(v)
                if len(order) >= size:
                    break
    return np.array(sorted(order), dtype=np.int32)


def query_stream(g: Graph, n_queries: int, qps: float, max_size: int = 256,
                 alpha_lo: float = 0.5, alpha_hi: float = 1.0, seed: int = 1):
    """Open-loop Poisson stream of local-community queries: arrival times
    (seconds), seed sets of size floor(exp(U ln(max_size+1))) in [1, max_size]
    taken as BFS prefixes from a uniform root, and alpha log-uniform on
    [alpha_lo, alpha_hi]."""
    rng = _rng(seed + 3)
    gaps = rng.exponential(1.0 / qps, size=n_queries)
    t = np.cumsum(gaps)
    sizes = np.floor(np.exp(rng.random(n_queries) * math.log(max_size + 1))).astype(np.int64)
    sizes = np.clip(sizes, 1, max_size)
    roots = rng.integers(0, g.n, size=n_queries)
    alphas = np.exp(rng.uniform(math.log(alpha_lo), math.log(alpha_hi), size=n_queries))
    sets = [bfs_prefix(g, int(r), int(s)) for r, s in zip(roots, sizes)]
    return t, sets, alphas


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def workload_small(seed: int = 1):
    """1,000-node two-level planted partition, every node a singleton seed,
    10 scales on [0.5, 1]."""
    g = planted_partition(seed=seed)
    sp, sn = singleton_seeds(g.n)
    return g, sp, sn, log_scales(10)


def workload_medium(seed: int = 1):
    """100k-node two-level LFR-style graph (degree exponent 2.5, mean 20,
    max 100; community sizes exponent 1.5 on [20, 200]; mixing 0.3;
    unweighted), rule-1 seeds, 32 scales on [0.5, 1]."""
    g = lfr_hierarchical(100_000, 2.5, 20.0, 100, 1.5, 20, 200, mu=0.3,
                         levels=2, weighted=False, seed=seed)
    sp, sn = seed_rule1(g, seed)
    return g, sp, sn, log_scales(32)


def workload_large(seed: int = 1):
    """1M-node three-level LFR-style graph (mean degree 15, max 200, mixing
    0.25, weights uniform in 1..16), rule-1 seeds, 64 scales on [0.5, 1]."""
    g = lfr_hierarchical(1_000_000, 2.5, 15.0, 200, 1.5, 20, 200, mu=0.25,
                         levels=3, weighted=True, seed=seed)
    sp, sn = seed_rule1(g, seed)
    return g, sp, sn, log_scales(64)


def workload_xl(seed: int = 1):
    """10M-node, ~10^8-edge three-level power-law graph (degree exponent
    2.2, mean 20, max 5,000; community sizes exponent 1.5 on [20, 5,000],
    so that a hub's internal edges fit its community;
    mixing 0.3 halving per level; weights uniform in 1..16), rule-1 seeds,
    32 scales on [0.5, 1]."""
    g = lfr_hierarchical_fast(10_000_000, 2.2, 20.0, 5000, 1.5, 20, 5000, mu=0.3,
                              levels=3, weighted=True, wmax=16, seed=seed)
    sp, sn = seed_rule1_fast(g, seed)
    return g, sp, sn, log_scales(32)


def workload_multigraph(n_graphs: int = 64, nmin: int = 1000, nmax: int = 200_000, seed: int = 1):
    """Independent graphs for one batched sweep: node counts log-uniform in
    [nmin, nmax], each generated like the 100k workload (two levels, degree
    exponent 2.5, mean 20, max 100, mixing 0.3) with weights 1..16; rule-1
    seeds per graph (local ids); 32 scales on [0.5, 1].  Returns (graphs,
    seed_ptr, seed_nodes, seed_graph, scales)."""
    rng = _rng(seed + 7)
    sizes = np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=n_graphs)).astype(np.int64)
    graphs, ptr, nodes, which = [], [np.zeros(1, np.int32)], [], []
    total = 0
    for i, n in enumerate(sizes.tolist()):
        g = lfr_hierarchical(int(n), 2.5, 20.0, 100, 1.5, 20, 200, mu=0.3, levels=2,
                             weighted=True, wmax=16, seed=seed * 1000 + i)
        sp, sn = seed_rule1(g, seed * 1000 + i)
        graphs.append(g)
        ptr.append(sp[1:].astype(np.int64) + total)
        nodes.append(sn)
        which.append(np.full(sp.size - 1, i, np.int32))
        total += int(sn.size)
    seed_ptr = np.concatenate(ptr).astype(np.int32)
    return (graphs, seed_ptr, np.concatenate(nodes).astype(np.int32),
            np.concatenate(which).astype(np.int32), log_scales(32))
