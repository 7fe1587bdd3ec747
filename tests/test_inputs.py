"""Host-side input preparation: graph generators, seed rule, scale list."""
import numpy as np
import pytest

from paper_1301_0955_amd import workloads as W


def _check_csr(g):
    rp, col = g.row_ptr.astype(np.int64), g.col.astype(np.int64)
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == col.size
    src = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(col >= 0) and np.all(col < g.n)
    assert not np.any(src == col)
    key = src * g.n + col
    assert np.all(np.diff(key) > 0)                # sorted rows, no duplicates
    rkey = np.sort(col * g.n + src)
    assert np.array_equal(key, rkey)               # symmetric
    if g.w is not None:
        order = np.argsort(col * g.n + src)
        assert np.array_equal(g.w, g.w[order])     # same weight both ways
        assert g.w.min() >= 1


def test_planted_partition_shape():
    g = W.planted_partition(seed=1)
    _check_csr(g)
    assert g.n == 1000
    # expected 11,100 undirected edges (7,350 + 3,000 + 750)
    assert abs(g.nnz / 2 - 11100) < 400
    assert W.planted_partition(seed=1).sha256() == g.sha256()
    assert W.planted_partition(seed=2).sha256() != g.sha256()


@pytest.mark.parametrize("levels,weighted", [(2, False), (3, True)])
def test_lfr_style_shape(levels, weighted):
    g = W.lfr_hierarchical(20000, 2.5, 15.0, 100, 1.5, 20, 200, mu=0.25,
                           levels=levels, weighted=weighted, seed=4)
    _check_csr(g)
    m = g.meta
    assert 13.0 < m["achieved_mean_deg"] <= 15.5
    assert m["achieved_max_deg"] <= 100
    assert 0.2 < m["achieved_mu_comm"] < 0.35
    assert m["achieved_mu_group"] < m["achieved_mu_comm"]
    if weighted:
        assert g.w.max() <= 16


def test_scale_list_reading():
    # alpha_i = 0.5 + 0.5 (1 - ln i / ln 10), i = 1..10
    want = [1.0, 0.8495, 0.7614, 0.6990, 0.6505, 0.6109, 0.5775, 0.5485, 0.5229, 0.5]
    got = W.log_scales(10)
    assert np.allclose(got, want, atol=5e-5)
    assert np.all(np.diff(got) < 0)
    s = W.log_scales(64)
    assert s[0] == 1.0 and s[-1] == 0.5 and np.all(np.diff(s) < 0)
    # dense near the low end
    assert (s[-2] - s[-1]) < (s[0] - s[1])


def test_seed_rule1_properties():
    g = W.lfr_hierarchical(5000, 2.5, 10.0, 60, 1.5, 20, 100, mu=0.3, levels=2, seed=9)
    ptr, seeds = W.seed_rule1(g, 9)
    assert np.array_equal(ptr, np.arange(seeds.size + 1))
    deg = np.diff(g.row_ptr)
    assert np.all(deg[seeds] >= 2)
    is_seed = np.zeros(g.n, bool)
    is_seed[seeds] = True
    # seeds are pairwise non-adjacent
    for s in seeds[:500]:
        assert not is_seed[g.col[g.row_ptr[s]:g.row_ptr[s + 1]]].any()
    # maximal: every candidate is a seed or adjacent to one
    covered = is_seed.copy()
    for s in seeds:
        covered[g.col[g.row_ptr[s]:g.row_ptr[s + 1]]] = True
    assert np.all(covered[deg >= 2])
    # selection order = scan order of the seeded permutation
    perm = np.random.Generator(np.random.PCG64(10)).permutation(g.n)
    pos = np.empty(g.n, np.int64)
    pos[perm] = np.arange(g.n)
    assert np.all(np.diff(pos[seeds]) > 0)
    ptr2, seeds2 = W.seed_rule1(g, 9)
    assert np.array_equal(seeds, seeds2)


def test_query_stream_shape():
    g = W.lfr_hierarchical(3000, 2.5, 10.0, 50, 1.5, 20, 100, mu=0.3, levels=2, seed=2)
    t, sets, alphas = W.query_stream(g, 500, 2000.0, seed=1)
    assert np.all(np.diff(t) > 0)
    assert 0.15 < t[-1] < 0.35
    sizes = np.array([s.size for s in sets])
    assert sizes.min() >= 1 and sizes.max() <= 256
    assert np.all((alphas >= 0.5) & (alphas <= 1.0))
    for s in sets[:50]:
        assert np.all(np.diff(s) > 0)


def test_multigraph_shape():
    gs, sp, sn, sg, sc = W.workload_multigraph(5, 300, 2000, seed=3)
    assert len(gs) == 5 and sc.size == 32
    assert sp[0] == 0 and sp[-1] == sn.size and np.all(np.diff(sp) >= 1)
    assert sg.size == sp.size - 1 and np.all(np.diff(sg) >= 0)
    for j in range(sg.size):
        assert np.all(sn[sp[j]:sp[j + 1]] < gs[sg[j]].n)
    for g in gs:
        assert 300 <= g.n <= 2000 and g.w is not None
