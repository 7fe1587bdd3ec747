"""Definition-level replay of the multi-scale loop with its check-and-merge
phase (Sec. 3, Algorithm 2 with the overlap pre-test of Algorithm 3), used to
pin the oracle's ``lcdo_run_merge``.

Independent of ``oracle/``: plain Python sets and dictionaries, no
incremental bookkeeping.  Each growth call is the from-scratch replay of
Algorithm 1 in ``_replay.grow`` (every d_in, K, V and rank recomputed from
the member set at each step).  The round structure follows Algorithm 2 as
printed: in every round each live community that is not held back by the
pre-test gets one call of the growth function; then the check pairs the
communities that overlap enough, and the pairs merge; the round repeats
while anything changed.  Readings of the points the paper leaves open:

* memberships are rebuilt from the member sets at the start of a round and
  again after its growth;
* the partner of c is the first community i != c, walking c's members in
  ascending order and, for each, the communities holding it in ascending
  order, whose running count x of shared nodes reaches
  x * eta_den >= eta_num * min(|c|, |i|);
* a community is grown in a round when it has no partner under the round's
  first memberships and it needs a call: at the start of a scale, after a
  call that changed it, after a merge it survived;
* the check takes each community that was held back or changed, in
  ascending order, with its partner under the post-growth memberships, as
  the pair (lower, higher); the pairs, sorted and without repeats, merge in
  passes: a pass takes, in order, the pairs that share no community with a
  pair taken before it in the pass, and merges each into its lower id (union
  of the member sets; the higher id dies); dead ids are renamed to their
  survivor in the pairs left, and passes repeat until none is left.
"""
from __future__ import annotations

from _replay import KV, grow


def _memberships(mem, alive):
    where = {}
    for j, m in enumerate(mem):
        if alive[j]:
            for v in m:
                where.setdefault(v, []).append(j)
    return where          # ids ascending: communities are visited in order


def _partner(c, mem, where, eta):
    num, den = eta
    count = {}
    for v in sorted(mem[c]):
        for i in where.get(v, []):
            if i == c:
                continue
            count[i] = count.get(i, 0) + 1
            if count[i] * den >= num * min(len(mem[c]), len(mem[i])):
                return i
    return None


def merge_sweep(g, seed_sets, scales, eta=(1, 2), k_prune=0, max_rounds=100000, calls_per_round=1):
    """Per scale s and set j: (members, K, V, [G, R, M, C], into) where into
    is -1 for a live community, else the live id it went into.

    ``calls_per_round`` is 1 for the reading above; ``None`` grows each
    community to its fixpoint inside a round instead (the other reading,
    used by the tests to show that a case tells the two apart)."""
    ns = len(seed_sets)
    mem = [set(int(u) for u in s) for s in seed_sets]
    alive = [True] * ns
    into = [-1] * ns
    K = [0] * ns
    V = [0] * ns
    out = []
    for alpha in scales:
        alpha = float(alpha)
        acc = [[0, 0, 0, 0] for _ in range(ns)]
        need = list(alive)
        for _ in range(max_rounds):
            where = _memberships(mem, alive)
            held = [alive[j] and _partner(j, mem, where, eta) is not None for j in range(ns)]
            changed = [False] * ns
            for j in range(ns):
                if not (alive[j] and need[j] and not held[j]):
                    continue
                c = set(mem[j])
                ctr = [0, 0, 0, 1]
                if calls_per_round == 1:
                    grow(g, c, alpha, k_prune, ctr)
                else:
                    while grow(g, c, alpha, k_prune, ctr):
                        ctr[3] += 1
                changed[j] = c != mem[j]
                mem[j] = c
                K[j], V[j] = KV(g, c)
                acc[j] = [a + b for a, b in zip(acc[j], ctr)]
                need[j] = changed[j] if calls_per_round == 1 else False
            where = _memberships(mem, alive)
            pairs = set()
            for j in range(ns):
                if alive[j] and (held[j] or changed[j]):
                    i = _partner(j, mem, where, eta)
                    if i is not None:
                        pairs.add((min(i, j), max(i, j)))
            merged = bool(pairs)
            pairs = sorted(pairs)
            while pairs:
                used = set()
                rest = []
                ren = {}
                for a, b in pairs:
                    if a in used or b in used:
                        rest.append((a, b))
                        continue
                    used.update((a, b))
                    mem[a] = mem[a] | mem[b]
                    mem[b] = set()
                    alive[b] = False
                    into[b] = a
                    need[a] = True
                    ren[b] = a
                nxt = set()
                for a, b in rest:
                    a, b = ren.get(a, a), ren.get(b, b)
                    if a != b:
                        nxt.add((min(a, b), max(a, b)))
                pairs = sorted(nxt)
            if not any(changed) and not merged:
                break
        else:
            raise RuntimeError("scale did not settle")
        rec = []
        for j in range(ns):
            to = j
            while not alive[to]:
                to = into[to]
            if alive[j]:
                rec.append((sorted(mem[j]), K[j], V[j], acc[j], -1))
            else:
                rec.append(([], 0, 0, acc[j], to))
        out.append(rec)
    return out
