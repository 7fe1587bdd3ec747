"""The multi-scale relevance analysis on the device (lcd_cover_nmi,
lcd_result_nmi, lcd_result_nmi_successive, lcd_result_nmi_cover) against the
oracle's NMI: within 1e-12 (the per-community terms use the same specified
log on both sides; only the order of the final sums differs)."""
import numpy as np
import pytest

import oracle
from paper_1301_0955_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1301_0955_amd import lcd
    lcd.library()
    return lcd


def _cover(rng, n, k, pmax=0.4):
    out = []
    for _ in range(k):
        m = rng.random(n) < rng.uniform(0.02, pmax)
        out.append(np.flatnonzero(m).astype(np.int32))      # may be empty
    return out


@pytest.mark.parametrize("seed", range(5))
def test_random_covers(L, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(20, 3000))
    X = _cover(rng, n, int(rng.integers(1, 60)))
    Y = _cover(rng, n, int(rng.integers(1, 60)))
    for a, b in ((X, Y), (X, X), (Y, X)):
        ref = oracle.nmi(n, a, b)
        got = L.lcd_cover_nmi(n, a, b)
        assert abs(got - ref) <= TOL * max(1.0, abs(ref)), (got, ref)


def test_crossing_halves_and_empty(L):
    n = 1000
    idx = np.arange(n, dtype=np.int32)
    assert L.lcd_cover_nmi(n, [idx[:500], idx[500:]], [idx[::2], idx[1::2]]) == 0.0
    assert L.lcd_cover_nmi(n, [], []) == 1.0
    assert L.lcd_cover_nmi(n, [idx[:10]], []) == 0.0


def test_malformed_cover_rejected(L):
    with pytest.raises(L.LcdError):
        L.lcd_cover_nmi(10, [np.array([3, 2], np.int32)], [np.array([1], np.int32)])   # not ascending
    with pytest.raises(L.LcdError):
        L.lcd_cover_nmi(10, [np.array([1, 12], np.int32)], [np.array([1], np.int32)])  # id out of range


def _oracle_covers(ref, S):
    ns = ref["n_sets"]
    covers = []
    for s in range(S):
        c = []
        for j in range(ns):
            r = j * S + s
            if ref["cnt"][r] > 0:
                c.append(ref["members"][ref["off"][r]:ref["off"][r] + ref["cnt"][r]])
        covers.append(c)
    return covers


def test_merge_result_successive_and_planted(L):
    g, sp, sn, sc = W.workload_small()
    G = L.Graph.from_workload(g)
    res = L.lcd_sweep_merge(G, sc, sp, sn)
    ref = oracle.Oracle.from_graph(g).run_merge(sp, sn, sc)
    S = sc.size
    covers = _oracle_covers(ref, S)
    for s in range(S - 1):
        a, b = res.nmi(s, s + 1), oracle.nmi(g.n, covers[s], covers[s + 1])
        assert abs(a - b) <= TOL * max(1.0, abs(b)), s
    for p in (3, 5):
        a, b = res.nmi_successive(p), oracle.nmi_successive(g.n, covers, p)
        assert a.shape == b.shape and np.all(np.abs(a - b) <= TOL), p
    subs = [np.arange(50 * k, 50 * k + 50, dtype=np.int32) for k in range(20)]
    groups = [np.arange(250 * k, 250 * k + 250, dtype=np.int32) for k in range(4)]
    for s in (0, S - 1):
        for planted in (subs, groups):
            a, b = res.nmi_cover(s, planted), oracle.nmi(g.n, covers[s], planted)
            assert abs(a - b) <= TOL * max(1.0, abs(b))
    # the method finds the planted levels: sub-communities at the finest
    # scale, the groups at the coarsest
    assert res.nmi_cover(0, subs) > 0.9 and res.nmi_cover(S - 1, groups) > 0.99
    res.free()


def test_sweep_result_scales(L):
    g = W.lfr_hierarchical(2000, 2.5, 10.0, 40, 1.5, 20, 60, mu=0.3, levels=2, weighted=True, seed=5)
    sp, sn = W.seed_rule1(g, 5)
    sc = W.log_scales(6)
    G = L.Graph.from_workload(g)
    res = L.lcd_sweep(G, sc, sp, sn)
    ref = oracle.Oracle.from_graph(g).run_sets(sp, sn, sc)
    covers = _oracle_covers(ref, sc.size)
    for s1, s2 in ((0, 1), (2, 5), (4, 4)):
        a, b = res.nmi(s1, s2), oracle.nmi(g.n, covers[s1], covers[s2])
        assert abs(a - b) <= TOL * max(1.0, abs(b)), (s1, s2)
    res.free()
