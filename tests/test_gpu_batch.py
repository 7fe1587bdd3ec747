"""Batches of independent graphs in one sweep (lcd_graph_upload_batch +
lcd_sweep_batch): every record equals the oracle run on its own member graph
(member ids mapped back from batch ids)."""
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


def _check_graphs(L, gs, sp, sn, sg, sc, got, node_off):
    """Records of seed sets with batch ids against the oracle on each
    member graph (ids mapped back to local ones)."""
    S = sc.size
    for i, g in enumerate(gs):
        ids = np.nonzero(sg == i)[0]
        sp_i = np.concatenate([[0], np.cumsum(sp[ids + 1] - sp[ids])]).astype(np.int32)
        sn_i = np.concatenate([sn[sp[j]:sp[j + 1]] for j in ids]).astype(np.int32) - int(node_off[i])
        ref = oracle.Oracle.from_graph(g).run_sets(sp_i, sn_i, sc)
        sub = dict(K=np.concatenate([got["K"][j * S:(j + 1) * S] for j in ids]),
                   V=np.concatenate([got["V"][j * S:(j + 1) * S] for j in ids]),
                   f=np.concatenate([got["f"][j * S:(j + 1) * S] for j in ids]),
                   ctr=np.concatenate([got["ctr"][j * S:(j + 1) * S] for j in ids]))
        mem, off, cnt = [], [], []
        pos = 0
        for j in ids:
            for s in range(S):
                r = j * S + s
                m = got["members"][got["off"][r]:got["off"][r] + got["cnt"][r]] - node_off[i]
                assert m.size == 0 or (m.min() >= 0 and m.max() < g.n)
                mem.append(m)
                off.append(pos)
                cnt.append(m.size)
                pos += m.size
        sub.update(members=np.concatenate(mem).astype(np.int32), off=np.array(off, np.int64),
                   cnt=np.array(cnt, np.int32), n_sets=ids.size, n_scales=S)
        compare_results(sub, ref, label="graph %d" % i)


def test_full_size_batch_sampled(L):
    """The benchmark's batch: 64 graphs of 1k-200k nodes in one launch; two
    seed sets of every graph through the oracle on its own graph."""
    gs, sp, sn, sg, sc = W.workload_multigraph()
    G = L.Graph.batch(gs)
    node_off = G.batch_info()
    res = L.lcd_sweep_batch(G, sc, sp, sn, sg)
    ids_all = np.concatenate([np.nonzero(sg == i)[0][np.linspace(0, (sg == i).sum() - 1, min(2, (sg == i).sum()))
                                                     .astype(np.int64)] for i in range(len(gs))])
    got_sel = res.sets_to_numpy(ids_all.astype(np.int32))
    res.free()
    # the selected sets, in selection order, with batch ids
    sp_sel = np.zeros(ids_all.size + 1, np.int32)
    np.cumsum(sp[ids_all + 1] - sp[ids_all], out=sp_sel[1:])
    sn_sel = np.concatenate([sn[sp[j]:sp[j + 1]] + int(node_off[sg[j]]) for j in ids_all]).astype(np.int32)
    sg_sel = sg[ids_all]
    _check_graphs(L, gs, sp_sel, sn_sel, sg_sel, sc, got_sel, node_off)


def test_batch_of_graphs_matches_oracle_per_graph(L):
    gs, sp, sn, sg, sc = W.workload_multigraph(6, 300, 3000, seed=2)
    G = L.Graph.batch(gs)
    node_off = G.batch_info()
    assert node_off.size == len(gs) + 1 and node_off[-1] == sum(g.n for g in gs)
    res = L.lcd_sweep_batch(G, sc, sp, sn, sg)
    got = L.sweep_to_numpy(res)
    res.free()
    S = sc.size
    for i, g in enumerate(gs):
        ids = np.nonzero(sg == i)[0]
        sp_i = np.concatenate([[0], np.cumsum(sp[ids + 1] - sp[ids])]).astype(np.int32)
        sn_i = np.concatenate([sn[sp[j]:sp[j + 1]] for j in ids]).astype(np.int32)
        ref = oracle.Oracle.from_graph(g).run_sets(sp_i, sn_i, sc)
        # this graph's records, member ids back to local ids
        sub = dict(K=np.concatenate([got["K"][j * S:(j + 1) * S] for j in ids]),
                   V=np.concatenate([got["V"][j * S:(j + 1) * S] for j in ids]),
                   f=np.concatenate([got["f"][j * S:(j + 1) * S] for j in ids]),
                   ctr=np.concatenate([got["ctr"][j * S:(j + 1) * S] for j in ids]))
        mem, off, cnt = [], [], []
        pos = 0
        for j in ids:
            for s in range(S):
                r = j * S + s
                m = got["members"][got["off"][r]:got["off"][r] + got["cnt"][r]] - node_off[i]
                assert m.size == 0 or (m.min() >= 0 and m.max() < g.n)
                mem.append(m)
                off.append(pos)
                cnt.append(m.size)
                pos += m.size
        sub.update(members=np.concatenate(mem).astype(np.int32), off=np.array(off, np.int64),
                   cnt=np.array(cnt, np.int32), n_sets=ids.size, n_scales=S)
        compare_results(sub, ref, label="graph %d" % i)


def test_batch_sweep_rejects_foreign_seeds(L):
    gs, sp, sn, sg, sc = W.workload_multigraph(3, 300, 1000, seed=4)
    G = L.Graph.batch(gs)
    bad = sn.copy()
    bad[0] = gs[sg[0]].n          # one past the end of its own graph
    with pytest.raises(L.LcdError) as e:
        L.lcd_sweep_batch(G, sc, sp, bad, sg)
    assert e.value.status == L.LCD_EINVAL
    with pytest.raises(L.LcdError):
        L.lcd_sweep_batch(G, sc, sp, sn, np.full(sg.size, len(gs), np.int32))
