"""The multi-scale loop with its check-and-merge phase (lcd_sweep_merge):
every record (members, K, V, counters, f) and every merged-into id equals the
oracle's run of the same reading of Algorithm 2."""
import time

import numpy as np
import pytest

import oracle
from _gpu_common import compare_results
from paper_1301_0955_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1301_0955_amd import lcd
    lcd.library()
    return lcd


def _run(L, g, sp, sn, sc, eta=(1, 2), **kw):
    G = L.Graph.from_workload(g)
    t0 = time.perf_counter()
    res = L.lcd_sweep_merge(G, sc, sp, sn, eta=eta, **kw)
    dt = time.perf_counter() - t0
    got = L.sweep_to_numpy(res)
    into = L.merged_into(res)
    with pytest.raises(L.LcdError):
        res.rerun()                   # refused on the host: nothing to replay
    res.free()
    ref = oracle.Oracle.from_graph(g).run_merge(sp, sn, sc, eta=eta)
    compare_results(got, ref, label="merge")
    assert np.array_equal(into, ref["into"])
    return ref, dt


def test_merge_planted_partition(L):
    g, sp, sn, sc = W.workload_small()
    ref, dt = _run(L, g, sp, sn, sc)
    S = sc.size
    print("planted: %.2f s, live at finest / coarsest scale %d / %d, rounds %s"
          % (dt, (ref["into"][0::S] == -1).sum(), (ref["into"][S - 1::S] == -1).sum(), ref["rounds"].tolist()))


@pytest.mark.parametrize("eta,kw", [((1, 2), dict(lds_capacity=128)), ((2, 3), dict())])
def test_merge_weighted_lfr(L, eta, kw):
    g = W.lfr_hierarchical(3000, 2.5, 12.0, 60, 1.5, 20, 120, mu=0.25, levels=3, weighted=True,
                           wmax=16, seed=5)
    sp, sn = W.seed_rule1(g, 5)
    _run(L, g, sp, sn, W.log_scales(8), eta=eta, **kw)


def test_merge_rejects_bad_eta(L):
    g, sp, sn, sc = W.workload_small()
    with pytest.raises(L.LcdError):
        L.lcd_sweep_merge(L.Graph.from_workload(g), sc, sp, sn, eta=(0, 1))
