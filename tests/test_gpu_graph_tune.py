"""hipGraph replay of the persistent sweep and the autotuner.

The captured sweep is replayed several times with other (eager) sweeps and
synchronisations in between; every replay must reproduce the oracle's
records bit for bit.  The autotuner only changes launch sizing, so a sweep
with the tuned sizing must give the same records as well."""
import sys

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


@pytest.fixture(scope="module")
def small():
    g, sp, sn, scales = W.workload_small()
    ref = oracle.Oracle.from_graph(g).run_sets(sp, sn, scales)
    return g, sp, sn, scales, ref


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("kw", [dict(), dict(lds_capacity=64, team_capacity=128),
                                dict(lds_capacity=64, spill_mode=1)])
def test_graph_replays_match_oracle(L, small, kw):
    import torch
    g, sp, sn, scales, ref = small
    G = L.Graph.from_workload(g)
    res = L.lcd_sweep(G, scales, sp, sn, use_graph=1, **kw)
    compare_results(L.sweep_to_numpy(res), ref, label="graph first launch")
    for i in range(3):
        # eager work of the program between replays
        other = L.lcd_sweep(G, scales[:3], sp[:50], sn[:sp[49]], k_prune=1, **kw)
        other.free()
        torch.cuda.synchronize()
        res.rerun()
        st = res.stats()
        assert st["launches"] >= 3
        compare_results(L.sweep_to_numpy(res), ref, label="graph replay %d" % i)
    _say("graph %s: %.2f ms per replay" % (kw, st["ms_total"]))
    res.free()


def test_graph_recaptures_after_pool_growth(L, small):
    g, sp, sn, scales, ref = small
    G = L.Graph.from_workload(g)
    res = L.lcd_sweep(G, scales, sp, sn, use_graph=1, pool_hint=1024)
    st = res.stats()
    assert st["reruns"] >= 1
    compare_results(L.sweep_to_numpy(res), ref, label="after pool growth")
    res.rerun()
    compare_results(L.sweep_to_numpy(res), ref, label="replay after pool growth")
    res.free()


def test_tuner_sizing_keeps_results(L, small):
    g, sp, sn, scales, ref = small
    G = L.Graph.from_workload(g)
    rep = L.lcd_tune(G, scales, sp, sn)
    _say("tuned %s in %d candidates" % (rep["best"], len(rep["tried"])))
    assert len(rep["tried"]) >= 8 and rep["ms_best"] > 0
    res = L.lcd_sweep(G, scales, sp, sn)
    st = res.stats()
    assert st["lds_capacity"] == rep["best"]["lds_capacity"]
    compare_results(L.sweep_to_numpy(res), ref, label="tuned sizing")
    res.free()
    # explicit sizing is never overridden, and untune restores the defaults
    res = L.lcd_sweep(G, scales, sp, sn, lds_capacity=128)
    assert res.stats()["lds_capacity"] == 128
    res.free()
    G.untune()
    res = L.lcd_sweep(G, scales, sp, sn)
    assert res.stats()["lds_capacity"] == 512
    res.free()
