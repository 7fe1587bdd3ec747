"""Parity of the HIP sweep with the CPU oracle, through the C ABI.

Memberships bit-exact, K and V exact, work counters G/R/M/C exact, reported
f within 1e-12 relative (each side evaluates pow() itself)."""
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


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_both(L, g, sp, sn, scales, k_prune=0, **kw):
    G = L.Graph.from_workload(g)
    res = L.lcd_sweep(G, scales, sp, sn, k_prune=k_prune, **kw)
    got = L.sweep_to_numpy(res)
    st = res.stats()
    o = oracle.Oracle.from_graph(g)
    ref = o.run_sets(sp, sn, scales, k_prune=k_prune)
    res.free()
    G.free()
    return got, ref, st


def test_device_info(L):
    info = L.lcd_device_info()
    _say("device %s" % info)
    assert info["arch"].startswith("gfx950")


def test_device_log_bitwise(L):
    import torch
    rng = np.random.Generator(np.random.PCG64(3))
    xs = np.concatenate([
        np.arange(1, 1 << 20, dtype=np.int64),
        rng.integers(1, 2**53, size=1 << 20, dtype=np.int64),
        np.exp(rng.uniform(0, np.log(2.0**53 - 2), 1 << 20)).astype(np.int64) + 1,
        np.array([2**e + d for e in range(1, 53) for d in (-1, 0, 1)], dtype=np.int64),
    ])
    xs = xs[(xs >= 1) & (xs < 2**53)]
    dev = L.lcd_log_device(torch.from_numpy(xs)).cpu().numpy()
    ref = oracle.log(xs.astype(np.uint64))
    diff = np.flatnonzero(dev.view(np.int64) != ref.view(np.int64))
    assert diff.size == 0, (xs[diff[:5]], dev[diff[:5]], ref[diff[:5]])


def test_device_log_bitwise_1e8(L):
    """10^8 integers in ten chunks (uniform on [1, 2^53), log-uniform, and
    every integer below 10^7): the device log equals the oracle's bit for
    bit on each."""
    import torch
    rng = np.random.Generator(np.random.PCG64(11))
    for c in range(10):
        if c < 4:
            xs = rng.integers(1, 2**53, size=10_000_000, dtype=np.int64)
        elif c < 9:
            xs = np.exp(rng.uniform(0, np.log(2.0**53 - 2), 10_000_000)).astype(np.int64) + 1
        else:
            xs = np.arange(1, 10_000_001, dtype=np.int64)
        xs = xs[(xs >= 1) & (xs < 2**53)]
        dev = L.lcd_log_device(torch.from_numpy(xs)).cpu().numpy()
        ref = oracle.log(xs.astype(np.uint64))
        diff = np.flatnonzero(dev.view(np.int64) != ref.view(np.int64))
        assert diff.size == 0, (c, xs[diff[:5]], dev[diff[:5]], ref[diff[:5]])
        print("log chunk %d: %d values equal" % (c, xs.size), flush=True)


def test_small_workload_full(L):
    _say("small workload: 1000 sets x 10 scales")
    g, sp, sn, scales = W.workload_small()
    got, ref, st = run_both(L, g, sp, sn, scales)
    compare_results(got, ref, label="small")
    _say("stats %s" % st)


@pytest.mark.parametrize("kw", [dict(), dict(lds_capacity=64, team_capacity=128)])
def test_small_workload_per_scale_loop(L, kw):
    # one launch group per scale, each resuming from the records of the scale
    # before; with small tables the spilled sets also resume in later tiers
    g, sp, sn, scales = W.workload_small()
    got, ref, st = run_both(L, g, sp, sn, scales, mode=1, **kw)
    compare_results(got, ref, label="per-scale loop %s" % kw)
    assert st["launches"] >= scales.size


@pytest.mark.parametrize("label,kw", [
    ("workgroup tiers: 4096-entry LDS table", dict(lds_capacity=64)),
    ("workgroup tiers: global tables", dict(lds_capacity=64, team_capacity=128)),
    ("workgroup tiers: one wave per workgroup", dict(lds_capacity=64, team_capacity=128, team_waves=1)),
    ("workgroup tiers: three waves", dict(lds_capacity=128, team_capacity=256, team_waves=3)),
    ("one-wave global tiers", dict(lds_capacity=64, spill_mode=1)),
    ("one-wave global tier, then workgroups", dict(lds_capacity=64, spill_mode=2)),
    ("global tables, rank-bucketed queue in every call", dict(lds_capacity=64, team_capacity=128,
                                                             queue_min_entries=1)),
    ("global tables, queue bucketed from 160 entries on", dict(lds_capacity=64, team_capacity=128,
                                                              queue_min_entries=160)),
])
def test_small_workload_spill_tiers(L, label, kw):
    # a 64-entry tier-0 table sends nearly every community to the later tiers
    g, sp, sn, scales = W.workload_small()
    _say("spill: %s" % label)
    got, ref, st = run_both(L, g, sp, sn, scales, **kw)
    assert st["n_spilled"] > 900
    compare_results(got, ref, label=label)
    _say("  tiers %d, sets finished per tier %s, %.2f ms"
         % (st["tiers"], [t["sets_finished"] for t in st["tier"]], st["ms_total"]))


def test_small_workload_k_prune_1(L):
    g, sp, sn, scales = W.workload_small()
    got, ref, _ = run_both(L, g, sp, sn, scales, k_prune=1)
    compare_results(got, ref, label="k_prune=1")


@pytest.mark.parametrize("n,p,weighted,seed", [(30, 0.15, False, 1), (50, 0.1, True, 2),
                                                (80, 0.05, True, 3), (120, 0.04, False, 4),
                                                (200, 0.03, True, 5), (64, 0.5, True, 6)])
def test_random_graphs(L, n, p, weighted, seed):
    g = W.random_graph(n, p, weighted, seed, wmax=16)
    rng = np.random.Generator(np.random.PCG64(seed))
    sets = [[u] for u in range(n)]
    for _ in range(20):
        sz = int(rng.integers(2, 9))
        sets.append(sorted(rng.choice(n, size=sz, replace=False).tolist()))
    sp = np.zeros(len(sets) + 1, np.int32)
    sp[1:] = np.cumsum([len(s) for s in sets])
    sn = np.concatenate([np.array(s, np.int32) for s in sets])
    scales = np.array([3.0, 1.3, 1.0, 0.8, 0.6, 0.45, 0.3, 0.1, 0.0])
    got, ref, _ = run_both(L, g, sp, sn, scales)
    compare_results(got, ref, label="random n=%d" % n)


def test_edge_cases(L):
    # isolated node, a pair, a path, and a star; singleton and whole-graph seeds
    edges = [(1, 2), (3, 4), (4, 5), (5, 6), (7, 8), (7, 9), (7, 10), (7, 11)]
    u = np.array([a for a, b in edges])
    v = np.array([b for a, b in edges])
    g = W.csr_from_edges(12, u, v, None)
    sets = [[0], [1], [3], [6], [7], [8], [3, 4, 5, 6], [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11]]
    sp = np.zeros(len(sets) + 1, np.int32)
    sp[1:] = np.cumsum([len(s) for s in sets])
    sn = np.concatenate([np.array(s, np.int32) for s in sets])
    for scales in (np.array([1.0]), np.array([64.0, 1.0, 0.5, 0.0])):
        got, ref, _ = run_both(L, g, sp, sn, scales)
        compare_results(got, ref, label="edge cases")


def test_no_sets(L):
    g, _, _, scales = W.workload_small()
    G = L.Graph.from_workload(g)
    res = L.lcd_sweep(G, scales, np.zeros(1, np.int32), np.zeros(0, np.int32))
    assert res.n_sets == 0
    assert res.counters() == [0, 0, 0, 0]
    assert res.sizes(0) == 0


def test_sweep_validation(L):
    g, sp, sn, scales = W.workload_small()
    G = L.Graph.from_workload(g)
    with pytest.raises(L.LcdError) as e:
        L.lcd_sweep(G, scales[::-1].copy(), sp, sn)
    assert e.value.status == L.LCD_EINVAL
    with pytest.raises(L.LcdError) as e:
        L.lcd_sweep(G, scales, np.array([0, 2], np.int32), np.array([5, 5], np.int32))
    assert e.value.status == L.LCD_EINVAL
    with pytest.raises(L.LcdError) as e:
        L.lcd_sweep(G, scales, np.array([0, 1], np.int32), np.array([1000], np.int32))
    assert e.value.status == L.LCD_EINVAL


def test_overlap_readout(L):
    # the node -> sets map against the inversion of the oracle's member sets
    g, sp, sn, scales = W.workload_small()
    G = L.Graph.from_workload(g)
    res = L.lcd_sweep(G, scales, sp, sn)
    ref = oracle.Oracle.from_graph(g).run_sets(sp, sn, scales)
    S = scales.size
    for s in (0, 4, 9):
        npt, nst = res.overlap(s)
        npt = npt.cpu().numpy()
        nst = nst.cpu().numpy()
        want = [[] for _ in range(g.n)]
        for j in range(res.n_sets):
            r = j * S + s
            for u in ref["members"][ref["off"][r]:ref["off"][r] + ref["cnt"][r]]:
                want[u].append(j)
        ptr = np.zeros(g.n + 1, np.int64)
        ptr[1:] = np.cumsum([len(x) for x in want])
        assert np.array_equal(npt, ptr)
        assert np.array_equal(nst, np.concatenate([np.array(x, np.int32) for x in want]))


def test_watchdog_turns_runaway_into_error(L):
    """With a zero time budget every seed set stops at its first watchdog
    check: the sweep must come back as an error (and every kernel exit)."""
    g, sp, sn, scales = W.workload_small()
    G = L.Graph.from_workload(g)
    with pytest.raises(L.LcdError) as e:
        L.lcd_sweep(G, scales, sp, sn, watchdog_ms=-1)
    assert e.value.status == L.LCD_EDEVICE
    assert "watchdog" in str(e.value)
    # the library stays usable afterwards
    res = L.lcd_sweep(G, scales, sp[:11], sn[:10])
    assert res.n_sets == 10
