"""Definition-level replay of the growth sweep, used to pin the oracle.

Independent of ``oracle/``: plain Python, no incremental bookkeeping.  At
every step d_in of every node, K and V are recomputed from the member set by
scanning the edge list, and the queue is the set of live nodes whose current
rank is evaluated afresh at each pop (Sec. 2, Algorithm 1; Eq. 1 and 2).
Only the member set and the live set are carried from step to step.

The natural log follows the same fully specified integer-log definition as
the oracle (so ranks that tie in exact arithmetic tie the same way); it is
checked separately against a 40-digit ``decimal`` logarithm.
"""
from __future__ import annotations

import numpy as np

EPS = 2.0 ** -40
_SQRT2 = float.fromhex("0x1.6a09e667f3bcdp+0")
_LN2_HI = 6.93147180369123816490e-01
_LN2_LO = 1.90821492927058770002e-10
_C = [1.0 / (2 * j + 1) for j in range(12)]


def spec_log(x: int) -> float:
    """Natural log of a positive integer x < 2**53: x = m 2^e with m in
    (sqrt(2)/2, sqrt(2)], ln m = 2 atanh((m-1)/(m+1)) by its series to the
    z^11 term, ln 2 split in a high and a low part."""
    x = int(x)
    e = x.bit_length() - 1
    m = float(x) * (2.0 ** -e)
    if m > _SQRT2:
        m = m * 0.5
        e += 1
    s = (m - 1.0) / (m + 1.0)
    z = s * s
    p = _C[11]
    for j in range(10, -1, -1):
        p = p * z
        p = p + _C[j]
    h = s * p
    lnm = h + h
    de = float(e)
    return de * _LN2_HI + (de * _LN2_LO + lnm)


class Graph:
    def __init__(self, n, row_ptr, col, w=None):
        self.n = int(n)
        self.adj = []
        for u in range(self.n):
            lo, hi = int(row_ptr[u]), int(row_ptr[u + 1])
            nb = col[lo:hi].tolist()
            ws = [1] * len(nb) if w is None else [int(x) for x in w[lo:hi]]
            self.adj.append(dict(zip(nb, ws)))
        self.k = [sum(a.values()) for a in self.adj]


def d_in(g: Graph, c: set, u: int) -> int:
    return sum(wt for v, wt in g.adj[u].items() if v in c)


def KV(g: Graph, c: set):
    K = sum(wt for u in c for v, wt in g.adj[u].items() if v in c)
    V = sum(g.k[u] for u in c)
    return K, V


def improves(Kp, Vp, K, V, alpha):
    if Kp == 0:
        return False
    if K == 0:
        return True
    a = spec_log(Kp) - spec_log(K)
    b = spec_log(Vp) - spec_log(V)
    return (a - alpha * b) > EPS


def rank(d, k, alpha):
    return spec_log(2 * d) - alpha * spec_log(k)


def grow(g: Graph, c: set, alpha: float, k_prune: int, ctr: list) -> int:
    moves = 0
    added = False
    live = {u for u in range(g.n) if u not in c and d_in(g, c, u) > 0}
    ctr[1] += len(live)
    while live:
        best = None
        for u in live:
            key = (rank(d_in(g, c, u), g.k[u], alpha), -u)
            if best is None or key > best[0]:
                best = (key, u)
        n = best[1]
        live.discard(n)
        ctr[0] += 1
        K, V = KV(g, c)
        d = d_in(g, c, n)
        if improves(K + 2 * d, V + g.k[n], K, V, alpha):
            c.add(n)
            moves += 1
            added = True
            ctr[2] += 1
            for v in g.adj[n]:
                if v not in c:
                    live.add(v)
                    ctr[1] += 1
    if added:
        p = 0
        while k_prune == 0 or p < k_prune:
            p += 1
            removed = False
            for n in sorted(c):
                ctr[0] += 1
                K, V = KV(g, c)
                d = d_in(g, c, n)
                if improves(K - 2 * d, V - g.k[n], K, V, alpha):
                    c.discard(n)
                    moves += 1
                    removed = True
                    ctr[2] += 1
            if not removed:
                break
    return moves


def sweep(g: Graph, seeds, scales, k_prune: int = 0):
    """Returns per scale: (sorted members, K, V, [G, R, M, C])."""
    c = set(int(s) for s in seeds)
    out = []
    for alpha in scales:
        ctr = [0, 0, 0, 0]
        while True:
            ctr[3] += 1
            if grow(g, c, float(alpha), k_prune, ctr) == 0:
                break
        K, V = KV(g, c)
        out.append((sorted(c), K, V, ctr))
    return out
