"""The query server (lcd_server_*): each query (S, alpha) grows S at the one
scale alpha until nothing changes (Sec. 2 and Algorithm 1 at a single
scale).  Every result must equal the oracle's growth of the same seed set
at that scale (members, K, V, G, R, M, C exactly, f within 1e-12), and be
the same when the query runs alone as when it runs in a mix of batches that
overlap on the device."""
import sys

import numpy as np
import pytest

import oracle
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
def graph():
    # weighted 3-level graph; large seed sets at small alpha outgrow the LDS
    # tables, so the global-memory tiers serve some queries too
    return W.lfr_hierarchical(20_000, 2.5, 15.0, 100, 1.5, 20, 200, mu=0.25, levels=3,
                              weighted=True, wmax=16, seed=5)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _same(a, b, where):
    assert np.array_equal(a["members"], b["members"]), where
    assert a["K"] == b["K"] and a["V"] == b["V"], where
    assert np.array_equal(np.asarray(a["ctr"], np.uint64), np.asarray(b["ctr"], np.uint64)), where


def _oracle_one(o, seeds, alpha):
    per, K, V, f, ctr, _ = o.run_set(seeds, np.array([alpha]))
    return dict(members=per[0], K=int(K[0]), V=int(V[0]), f=float(f[0]), ctr=ctr[0])


def test_server_mix_equals_alone_and_oracle(L, graph):
    g = graph
    G = L.Graph.from_workload(g)
    _, sets, alphas = W.query_stream(g, 240, 2000.0, max_size=256, seed=11)
    # a few heavy queries first (large seed sets at the coarsest scale), so
    # the batches that follow start while those still run
    heavy = [(W.bfs_prefix(g, r, 256), 0.5) for r in (7, 911, 4242)]
    queries = heavy + list(zip(sets, alphas))
    o = oracle.Oracle.from_graph(g)
    # every lane layout: one stage per tier on eight lanes (10 or more
    # hardware queues) or six (8 or 9), and tier 0 then the rest on four
    # lanes (fewer queues); the server reads the queue count when it is
    # created
    import os
    for queues, cap in (("12", 1024), ("12", 256), ("8", 1024), ("4", 1024)):
        old_q = os.environ.get("GPU_MAX_HW_QUEUES")
        os.environ["GPU_MAX_HW_QUEUES"] = queues
        try:
            srv = L.Server(G, max_slots=512, lds_capacity=cap)
        finally:
            if old_q is None:
                del os.environ["GPU_MAX_HW_QUEUES"]
            else:
                os.environ["GPU_MAX_HW_QUEUES"] = old_q
        with srv:
            assert srv.stats()["lanes"] == {"12": 8, "8": 6, "4": 4}[queues]
            tickets = [srv.submit(s, a) for s, a in queries]
            mix = [srv.result(t, 120_000) for t in tickets]
            st = srv.stats()
            _say("queues %s cap %d: %d queries, %d batches (%d after stage 0), largest %d, lanes busy at "
                 "once %d, forwarded %d, routed %d, requeued %d"
                 % (queues, cap, st["completed"], st["batches"], st["spill_batches"], st["max_batch"],
                    st["max_lanes_busy"], st["forwarded"], st["routed"], st["requeued"]))
            if cap == 256:
                # 256-seed queries hold more than 256 table entries from the
                # start: they are queued straight to a later stage
                assert st["routed"] > 0
            assert st["completed"] == len(queries) and st["failed"] == 0
            assert st["max_lanes_busy"] >= 2        # batches overlapped on the device
            assert st["forwarded"] > 0              # some queries outgrew tier 0
            for i, ((s, a), got) in enumerate(zip(queries, mix)):
                ref = _oracle_one(o, s, a)
                _same(got, ref, ("oracle", cap, i))
                assert abs(got["f"] - ref["f"]) <= 1e-12 * abs(ref["f"]), (cap, i)
                assert got["t_submit_ns"] <= got["t_start_ns"] <= got["t_done_ns"]
            # the same queries one at a time
            for i in range(0, len(queries), 6):
                s, a = queries[i]
                alone = srv.result(srv.submit(s, a), 120_000)
                assert alone["batch_size"] == 1
                _same(alone, mix[i], ("alone", cap, i))
                assert alone["f"] == mix[i]["f"]


def test_server_errors_and_capacity(L, graph):
    import ctypes
    g = graph
    G = L.Graph.from_workload(g)
    with L.Server(G) as srv:
        with pytest.raises(L.LcdError) as e:
            srv.submit([1, 1], 0.7)
        assert e.value.status == L.LCD_EINVAL
        with pytest.raises(L.LcdError):
            srv.submit([g.n], 0.7)
        with pytest.raises(L.LcdError):
            srv.submit([3], float("nan"))
        with pytest.raises(L.LcdError):
            srv.submit([], 0.7)
        with pytest.raises(L.LcdError) as e:
            srv.poll(987654321)
        assert e.value.status == L.LCD_EINVAL
        # a buffer that is too small keeps the ticket; a large one retires it
        t = srv.submit(W.bfs_prefix(g, 17, 40), 0.6)
        assert srv.wait(t, 60_000)
        lib = L.library()
        info = L.lcd_query_info()
        buf = np.zeros(1, np.int32)
        s = lib.lcd_server_poll(srv._h, t, buf.ctypes.data_as(ctypes.c_void_p), 1, ctypes.byref(info))
        assert s == L.LCD_ECAPACITY and info.n_members > 1
        r = srv.poll(t)
        assert r["members"].size == info.n_members
        with pytest.raises(L.LcdError):
            srv.poll(t)                               # retired
    # a zero watchdog budget turns every query into an error, and a server
    # created afterwards answers normally
    with L.Server(G, watchdog_ms=-1) as bad:
        ts = [bad.submit([u], 0.8) for u in (1, 2, 3)]
        for t in ts:
            bad.wait(t, 60_000)
            with pytest.raises(L.LcdError) as e:
                bad.poll(t)
            assert e.value.status == L.LCD_EDEVICE and "watchdog" in str(e.value)
    with L.Server(G) as srv:
        r = srv.result(srv.submit([5], 0.8), 60_000)
        ref = _oracle_one(oracle.Oracle.from_graph(g), [5], 0.8)
        _same(r, ref, "after watchdog")


def test_server_small_budget_and_cancel(L, graph):
    """Admission under a forced small memory budget (the smallest the lanes
    accept: one table of each global tier per lane that runs it), with every
    result still equal to the oracle's; a budget below it is refused; and
    cancellation: a withdrawn query ends LCD_ECANCELED whether it was still
    waiting or already on the device, the rest are answered exactly."""
    import re
    g = graph
    G = L.Graph.from_workload(g)
    with pytest.raises(L.LcdError) as e:
        L.Server(G, mem_budget=1 << 20)
    assert e.value.status == L.LCD_ENOMEM
    need = int(re.search(r"below the (\d+) bytes", str(e.value)).group(1))
    o = oracle.Oracle.from_graph(g)
    _, sets, alphas = W.query_stream(g, 160, 2000.0, max_size=256, seed=23)
    heavy = [(W.bfs_prefix(g, r, 256), 0.5) for r in (3, 1201)]
    queries = heavy + list(zip(sets, alphas))
    with L.Server(G, mem_budget=need + (1 << 20)) as srv:
        st = srv.stats()
        assert all(x <= 1 for x in st["spill_tables"]), st
        tickets = [srv.submit(s, a) for s, a in queries]
        # withdraw every fifth query at once (most are still waiting), and
        # the first heavy one after it has started
        cut = set(range(2, len(queries), 5))
        withdrawn = {i for i in cut if srv.cancel(tickets[i])}
        assert withdrawn
        if srv.cancel(tickets[0]):
            withdrawn.add(0)
        for i, t in enumerate(tickets):
            assert srv.wait(t, 120_000)
            if i in withdrawn:
                with pytest.raises(L.LcdError) as e:
                    srv.poll(t)
                assert e.value.status == L.LCD_ECANCELED
                continue
            _same(srv.poll(t), _oracle_one(o, *queries[i]), "small budget, query %d" % i)
        st = srv.stats()
        assert st["cancelled"] == len(withdrawn)
        assert st["completed"] == len(queries) - len(withdrawn)
        _say("small budget %d B: tables %s, %d withdrawn, stats %s" % (need, st["spill_tables"], len(withdrawn), st))
        # a completed query can no longer be withdrawn
        t = srv.submit([5], 0.8)
        srv.wait(t, 60_000)
        assert not srv.cancel(t)
        _same(srv.poll(t), _oracle_one(o, [5], 0.8), "after cancel")
