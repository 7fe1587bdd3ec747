"""Exhaustive pins for the oracle on graphs of at most 12 nodes.

* Every set the oracle visits, and every candidate set it tests, has K and V
  equal to the values of a table built by enumerating the edges of all 2^n
  subsets (Eq. 1 with R1: K counts internal edges from both ends, V is the
  member-degree sum).  Any slip in the incremental bookkeeping (a dropped
  factor 2, a stale d_in, a wrong sign on removal) fails this.
* Invariants of every reported community: K even, K <= V, k_out = V - K
  equals the weight leaving the set counted edge by edge.
* The reported criterion f = K / V^alpha matches a 40-digit decimal value.
* Every result is 1-flip locally optimal in exact arithmetic: no single
  node joins or leaves to raise f by more than the decision margin
  (additions always; removals for singleton starts, whose first growth call
  always ends with removal passes, and because decreasing alpha only makes
  removal less attractive).
"""
import decimal
import itertools

import numpy as np
import pytest

from paper_1301_0955_amd import workloads as W

decimal.getcontext().prec = 40
EPS = 2.0 ** -40
SCALES = np.array([1.4, 1.0, 0.8, 0.62, 0.45, 0.3])


def _tables(g):
    n = g.n
    masks = np.arange(1 << n, dtype=np.int64)
    bit = lambda u: (masks >> u) & 1
    K = np.zeros(1 << n, dtype=np.int64)
    V = np.zeros(1 << n, dtype=np.int64)
    OUT = np.zeros(1 << n, dtype=np.int64)
    k = np.zeros(n, dtype=np.int64)
    for u in range(n):
        for j in range(g.row_ptr[u], g.row_ptr[u + 1]):
            v = int(g.col[j])
            wt = 1 if g.w is None else int(g.w[j])
            k[u] += wt
            both = bit(u) & bit(v)
            K += wt * both                       # each direction once -> 2x
            OUT += wt * (bit(u) & (1 - bit(v)))
    for u in range(n):
        V += k[u] * bit(u)
    return K, V, OUT, k


def _mask(nodes):
    m = 0
    for u in nodes:
        m |= 1 << int(u)
    return m


def _t_exact(Kp, Vp, K, V, alpha):
    D = decimal.Decimal
    return (D(Kp) / D(K)).ln() - D(repr(alpha)) * (D(Vp) / D(V)).ln()


GRAPHS = [(n, p, wt, s) for n in (5, 8, 10, 12) for p in (0.3, 0.55)
          for wt in (False, True) for s in (1, 2)]


@pytest.mark.parametrize("n,p,weighted,seed", GRAPHS)
def test_bruteforce_trajectory_and_optimality(oracle_mod, n, p, weighted, seed):
    g = W.random_graph(n, p, weighted, seed)
    Kt, Vt, OUTt, k = _tables(g)
    o = oracle_mod.Oracle.from_graph(g)
    assert np.array_equal(o.degrees(), k)
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    starts = [[u] for u in range(n)]
    for _ in range(4):
        sz = int(rng.integers(2, max(3, n // 2)))
        starts.append(sorted(rng.choice(n, size=sz, replace=False).tolist()))
    for seeds in starts:
        per, K, V, f, ctr, trace = o.run_set(seeds, SCALES, trace_cap=200000)
        cur = _mask(seeds)
        for r in trace:
            assert r["K"] == Kt[cur] and r["V"] == Vt[cur]
            nxt = cur ^ (1 << r["node"])
            if r["kind"] == 0:
                assert not (cur >> r["node"]) & 1
            else:
                assert (cur >> r["node"]) & 1
            assert r["Kp"] == Kt[nxt] and r["Vp"] == Vt[nxt]
            if r["result"]:
                cur = nxt
                assert r["mask"] == cur
        for s, alpha in enumerate(SCALES):
            m = _mask(per[s])
            assert list(per[s]) == sorted(per[s])
            assert K[s] == Kt[m] and V[s] == Vt[m]
            assert K[s] % 2 == 0 and K[s] <= V[s]
            assert V[s] - K[s] == OUTt[m]
            if K[s] > 0:
                ref = decimal.Decimal(int(K[s])) / decimal.Decimal(int(V[s])) ** decimal.Decimal(repr(float(alpha)))
                assert abs(decimal.Decimal(f[s]) - ref) <= abs(ref) * decimal.Decimal("1e-12")
            # 1-flip local optimality in exact arithmetic
            if K[s] == 0:
                # only possible when the start has no neighbour at all
                assert all(k[u] == 0 for u in per[s])
                continue
            for u in range(n):
                inside = (m >> u) & 1
                if inside and len(seeds) > 1:
                    continue
                nm = m ^ (1 << u)
                if Kt[nm] == 0:
                    continue
                t = _t_exact(int(Kt[nm]), int(Vt[nm]), int(K[s]), int(V[s]), float(alpha))
                assert t <= decimal.Decimal(EPS) + decimal.Decimal("1e-12"), (seeds, s, u, t)


def test_counter_definitions_small(oracle_mod):
    """G counts pops and removal visits, R rank computations, M moves and C
    growth calls: on a triangle with a pendant node, grown from one triangle
    node at alpha = 1, the counts follow by hand."""
    # 0-1, 0-2, 1-2 triangle; 2-3 pendant.  k = [2, 2, 3, 1]
    g = W.csr_from_edges(4, np.array([0, 0, 1, 2]), np.array([1, 2, 2, 3]), None)
    o = oracle_mod.Oracle.from_graph(g)
    per, K, V, f, ctr, _ = o.run_set([0], [1.0])
    # From {0}: K = 0, so the first pop always joins.  Ranks at alpha=1:
    # node 1: ln(2*1) - ln 2 = 0; node 2: ln 2 - ln 3 < 0 -> pop 1 (G=1) and add.
    # Queue update: neighbour 2 (R+1).  State {0,1}: K=2, V=4.  Pop 2 (G=2):
    # K'=2+4=6, V'=7: 6/7 > 2/4 -> add; neighbour 3 queued (R+1).  State
    # {0,1,2}: K=6, V=7.  Pop 3 (G=3): K'=8, V'=8: 1 > 6/7 -> add (M=3),
    # no non-member neighbours.  Removal pass over [0,1,2,3] (G=7): removing 0
    # gives K'=4, V'=6 (< 1), 1 likewise, 2 gives K'=2,V'=5... none removed.
    # Second growth call: queue empty, nothing moves (C=2).
    assert per[0].tolist() == [0, 1, 2, 3]
    assert (K[0], V[0]) == (8, 8)
    G, R, M, C = ctr[0].tolist()
    assert (M, C) == (3, 2)
    assert R == 2 + 1 + 1       # queue built from {1, 2}; then 2 and 3 updated
    assert G == 3 + 4           # three pops, one removal pass over 4 members
