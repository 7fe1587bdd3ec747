"""lcd_sweep_into (no allocation inside the library) against lcd_sweep.

Two calls in a row through the C ABI, the second on a smaller input (fewer
seed sets, fewer scales), each compared record by record with lcd_sweep on
the same input: member lists and counters bit for bit, K and V exactly, f
within 1e-12 relative.  A members buffer that is too small is reported with
the size needed."""
import numpy as np
import pytest

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


def _records(o, ns, S):
    off = o["rec_off"][:ns * S].cpu().numpy()
    cnt = o["rec_cnt"][:ns * S].cpu().numpy()
    mem = o["members"][:max(o["members_used"], 1)].cpu().numpy()
    lists = [mem[off[r]:off[r] + cnt[r]] for r in range(ns * S)]
    return (lists, o["rec_k"][:ns * S].cpu().numpy(), o["rec_v"][:ns * S].cpu().numpy(),
            o["rec_f"][:ns * S].cpu().numpy(), o["rec_ctr"][:4 * ns * S].cpu().numpy().reshape(-1, 4))


def _compare(L, G, sc, sp, sn, got, kw):
    ref = L.sweep_to_numpy(L.lcd_sweep(G, sc, sp, sn, **kw))
    ns, S = sp.size - 1, sc.size
    lists, K, V, f, ctr = _records(got, ns, S)
    for r in range(ns * S):
        a = ref["members"][ref["off"][r]:ref["off"][r] + ref["cnt"][r]]
        assert np.array_equal(lists[r], a), r
    assert np.array_equal(K, ref["K"]) and np.array_equal(V, ref["V"])
    assert np.array_equal(ctr.astype(np.uint64), ref["ctr"].astype(np.uint64))
    assert np.all(np.abs(f - ref["f"]) <= 1e-12 * np.abs(ref["f"]))


def test_sweep_into_matches_sweep_twice(L):
    g = W.lfr_hierarchical(3000, 2.5, 12.0, 60, 1.5, 20, 300, mu=0.25, levels=3, weighted=True,
                           wmax=16, seed=5)
    sp, sn = W.seed_rule1(g, 5)
    sc = W.log_scales(8)
    G = L.Graph.from_workload(g)
    # small LDS tables, so that sets also run in the workgroup tiers
    kw = dict(lds_capacity=128, team_capacity=512)
    out = L.lcd_sweep_into(G, sc, sp, sn, members_cap=4_000_000, **kw)
    _compare(L, G, sc, sp, sn, out, kw)
    used_first = out["members_used"]
    # second call, smaller input, into the same buffers
    sp2, sn2, _ = W.subsample_sets(sp, sn, 3)
    sc2 = sc[:5]
    out2 = L.lcd_sweep_into(G, sc2, sp2, sn2, members_cap=4_000_000, out=out, **kw)
    assert out2["members_used"] < used_first
    _compare(L, G, sc2, sp2, sn2, out2, kw)


def test_sweep_into_reports_small_buffer(L):
    g, sp, sn, sc = W.workload_small()
    G = L.Graph.from_workload(g)
    with pytest.raises(L.LcdError) as e:
        L.lcd_sweep_into(G, sc, sp, sn, members_cap=100)
    assert e.value.status == 5                 # LCD_ECAPACITY
    out = L.lcd_sweep_into(G, sc, sp, sn, members_cap=2_000_000)
    _compare(L, G, sc, sp, sn, out, {})


def test_sweep_into_rejects_bad_inputs(L):
    g, sp, sn, sc = W.workload_small()
    G = L.Graph.from_workload(g)
    bad = sn.copy()
    bad[3] = g.n + 5                           # a seed id out of range
    with pytest.raises(L.LcdError) as e:
        L.lcd_sweep_into(G, sc, sp, bad, members_cap=2_000_000)
    assert e.value.status == 1                 # LCD_EINVAL
    with pytest.raises(L.LcdError):
        L.lcd_sweep_into(G, sc[::-1].copy(), sp, sn, members_cap=2_000_000)   # increasing scales
