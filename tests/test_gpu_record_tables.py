"""Communities of tens of thousands of nodes on an 80,000-node block graph:
they outgrow the 16,384-entry global tier and finish in the tables that
hold every node (131,072 entries), which use the record layout, the record
kernel, hash slots holding the node id, and removal searches over an
id-bucketed member list.  Every record must equal the oracle's (members, K,
V and the counters bit for bit, f within 1e-12), in full and in delta
output, in one launch group and in the per-scale loop."""
import numpy as np
import pytest

import oracle
from _gpu_common import compare_results
from paper_1301_0955_amd import workloads as W

pytestmark = pytest.mark.gpu

RECORD_MIN_ENTRIES = 65536


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1301_0955_amd import lcd
    lcd.library()
    return lcd


@pytest.fixture(scope="module")
def blocks():
    g = W.block_graph(4, 20000, 8, 1, True, seed=3)
    sc = W.log_scales(4)
    rng = np.random.default_rng(5)
    sn = rng.choice(g.n, 6, replace=False).astype(np.int32)
    sp = np.arange(7, dtype=np.int32)
    ref = oracle.Oracle.from_graph(g).run_sets(sp, sn, sc)
    # the oracle's communities cover whole blocks at most scales
    assert int(ref["cnt"].max()) > 16384
    return g, sp, sn, sc, ref


@pytest.mark.parametrize("label,kw", [
    ("default tiers", dict()),
    ("delta output", dict(output_mode=1)),
    ("per-scale loop", dict(mode=1)),
    ("bucketed queue and id-bucketed removal from the smallest tables", dict(queue_min_entries=64)),
])
def test_record_tables_match_oracle(L, blocks, label, kw):
    g, sp, sn, sc, ref = blocks
    G = L.Graph.from_workload(g)
    res = L.lcd_sweep(G, sc, sp, sn, **kw)
    st = res.stats()
    compare_results(L.sweep_to_numpy(res), ref, label=label)
    nt = st["tiers"]
    caps = st["tier_capacity"][:nt]
    finished = [t["sets_finished"] for t in st["tier"][:nt]]
    # the sets finished in record-layout tables
    assert any(c >= RECORD_MIN_ENTRIES and f > 0 for c, f in zip(caps, finished)), (caps, finished)
    res.free()
    G.free()
