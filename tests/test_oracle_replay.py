"""Pin the oracle's trajectory against the definition-level replay
(tests/_replay.py): same member sets at every scale and the same work
counters G, R, M, C, on random weighted and unweighted graphs, on seed sets
of one or several nodes, with unbounded and bounded removal passes, and on a
sample of the 1,000-node planted-partition workload."""
import numpy as np
import pytest

import _replay as RP
from paper_1301_0955_amd import workloads as W

SCALES = W.log_scales(6, 0.35, 1.2)


def _compare(o, rg, seeds, scales, k_prune):
    per, K, V, f, ctr, _ = o.run_set(seeds, scales, k_prune=k_prune)
    ref = RP.sweep(rg, seeds, scales, k_prune)
    for s in range(len(scales)):
        members, Kr, Vr, cr = ref[s]
        assert per[s].tolist() == members, (seeds, s)
        assert (int(K[s]), int(V[s])) == (Kr, Vr)
        assert ctr[s].tolist() == cr, (seeds, s, ctr[s].tolist(), cr)


@pytest.mark.parametrize("n,p,weighted,seed", [(20, 0.2, False, 1), (24, 0.15, True, 2),
                                                (30, 0.12, True, 3), (16, 0.4, False, 4),
                                                (40, 0.08, False, 5)])
@pytest.mark.parametrize("k_prune", [0, 1])
def test_replay_random(oracle_mod, n, p, weighted, seed, k_prune):
    g = W.random_graph(n, p, weighted, seed)
    o = oracle_mod.Oracle.from_graph(g)
    rg = RP.Graph(g.n, g.row_ptr, g.col, g.w)
    rng = np.random.Generator(np.random.PCG64(seed))
    starts = [[u] for u in range(0, n, 3)]
    starts += [sorted(rng.choice(n, size=3, replace=False).tolist()) for _ in range(3)]
    for seeds in starts:
        _compare(o, rg, seeds, SCALES, k_prune)


def test_replay_planted_partition_sample(oracle_mod):
    g, sp, sn, scales = W.workload_small()
    o = oracle_mod.Oracle.from_graph(g)
    rg = RP.Graph(g.n, g.row_ptr, g.col, g.w)
    for u in (0, 137, 599):
        _compare(o, rg, [u], scales[:4], 0)


def test_replay_lfr_sample(oracle_mod):
    g = W.lfr_hierarchical(600, 2.5, 8.0, 30, 1.5, 10, 40, mu=0.3, levels=2,
                           weighted=True, seed=3)
    o = oracle_mod.Oracle.from_graph(g)
    rg = RP.Graph(g.n, g.row_ptr, g.col, g.w)
    for u in (5, 211):
        _compare(o, rg, [u], W.log_scales(4), 0)
