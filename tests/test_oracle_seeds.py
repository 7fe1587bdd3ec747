"""Pins for the oracle's seed selection (Sec. 3, initialisation of
Algorithm 2).

Visiting nodes in a given order and keeping every node that is still a
candidate, while dropping its neighbours (rule 1) or everything within two
hops (rule 2), yields the unique set I with: a candidate v (at least two
neighbours) is in I exactly when no earlier-visited member of I lies within
that distance of v.  The tests check that characterisation by brute force
(distances from adjacency-matrix powers), the visiting order of the result,
and agreement of rule 1 with the input generator's own implementation."""
import numpy as np
import pytest

from paper_1301_0955_amd import workloads as W


def _dist_le(g, r):
    n = g.n
    A = np.zeros((n, n), dtype=np.int64)
    for u in range(n):
        A[u, g.col[g.row_ptr[u]:g.row_ptr[u + 1]]] = 1
    R = A.copy()
    if r == 2:
        R = ((A + A @ A) > 0).astype(np.int64)
    np.fill_diagonal(R, 0)
    return R > 0


@pytest.mark.parametrize("n,p,seed", [(12, 0.2, 1), (25, 0.12, 2), (40, 0.08, 3), (60, 0.05, 4),
                                      (30, 0.3, 5)])
@pytest.mark.parametrize("rule", [1, 2])
def test_seeds_are_the_order_first_independent_set(oracle_mod, n, p, seed, rule):
    g = W.random_graph(n, p, weighted=False, seed=seed)
    perm = np.random.Generator(np.random.PCG64(seed + 100)).permutation(n)
    pos = np.empty(n, dtype=np.int64)
    pos[perm] = np.arange(n)
    seeds = oracle_mod.Oracle.from_graph(g).seeds(perm, rule)
    # in visiting order, distinct
    assert np.all(np.diff(pos[seeds]) > 0)
    near = _dist_le(g, rule)
    cand = np.diff(g.row_ptr) >= 2
    inI = np.zeros(n, dtype=bool)
    inI[seeds] = True
    for v in range(n):
        blocked = bool(np.any(inI & near[v] & (pos < pos[v])))
        assert inI[v] == (bool(cand[v]) and not blocked), (v, rule)


def test_rule1_matches_input_generator(oracle_mod):
    for g, s in ((W.workload_small()[0], 1), (W.lfr_hierarchical(5000, 2.5, 12.0, 60, 1.5, 20, 120, mu=0.3,
                                                                  levels=2, weighted=False, seed=3), 3)):
        sp, sn = W.seed_rule1(g, s)
        got = oracle_mod.Oracle.from_graph(g).seeds(W.seed_permutation(g, s), 1)
        assert np.array_equal(got, sn)


def test_rule2_is_a_subset_order_of_magnitude(oracle_mod):
    g = W.workload_small()[0]
    perm = W.seed_permutation(g, 1)
    o = oracle_mod.Oracle.from_graph(g)
    s1, s2 = o.seeds(perm, 1), o.seeds(perm, 2)
    assert 0 < s2.size < s1.size
    assert s1[0] == s2[0]                       # the first candidate is a seed under both rules


def test_seeds_reject_bad_input(oracle_mod):
    g = W.workload_small()[0]
    o = oracle_mod.Oracle.from_graph(g)
    with pytest.raises(ValueError):
        o.seeds(np.zeros(g.n, np.int32), 1)     # not a permutation
    with pytest.raises(ValueError):
        o.seeds(np.arange(g.n), 3)
