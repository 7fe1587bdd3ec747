#!/usr/bin/env python3
"""Benchmark of the multi-scale local community sweep on one MI355X.

One step = one lcd_sweep() call: every seed set of the workload grown
through every scale (queue-emulated additions, removal passes, fixpoint per
scale, chained scales), with sorted member lists, K, V, f and the work
counters written for every (seed set, scale).  Inputs (graph, seeds,
scales) are resident on the device before the timed region.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# The query server's launch lanes are HIP streams, which HIP spreads over
# GPU_MAX_HW_QUEUES hardware queues (4 by default); with 8 or more the server
# runs one stage per tier on six lanes, none sharing a queue.  This has to be
# set before the HIP runtime starts.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "0") or 0) < 12:
    os.environ["GPU_MAX_HW_QUEUES"] = "12"

METRIC = ("candidate-node gains/s + full multi-scale sweep time; "
          "p50/p99 seed-query latency")
HBM_PEAK_GBS = 8000.0
RECORD_BYTES = 8 + 4 + 8 + 8 + 8 + 32   # off, cnt, K, V, f, four counters
KERNEL_OF_KIND = {0: "sweep_lds_kernel", 1: "sweep_global_kernel", 2: "sweep_team_lds_kernel",
                  3: "sweep_team_global_kernel"}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def workload(name: str):
    from paper_1301_0955_amd import workloads as W
    if name == "small":
        g, sp, sn, sc = W.workload_small()
        desc = "planted-partition-1k: 1,000 nodes (4 groups x 5 sub-communities), every node a seed, 10 scales on [0.5,1]"
    elif name == "medium":
        g, sp, sn, sc = W.workload_medium()
        desc = ("lfr2-100k: 100,000-node 2-level LFR-style graph (degree exp 2.5, mean 20, max 100; "
                "community sizes exp 1.5 on [20,200]; mixing 0.3; unweighted), rule-1 seeds, 32 scales on [0.5,1]")
    elif name == "large":
        g, sp, sn, sc = W.workload_large()
        desc = ("lfr3-1M: 1,000,000-node 3-level LFR-style graph (mean degree 15, max 200, mixing 0.25, "
                "weights 1..16), rule-1 seeds, 64 scales on [0.5,1]")
    else:
        raise SystemExit("unknown workload %s" % name)
    return g, sp, sn, sc, desc


def algorithmic_bytes(t: dict, weighted: bool, seed_nodes: int, n_records: int) -> int:
    """HBM bytes the method itself must move for the work one tier finished:
    per gathered CSR row its two offsets and its entries (id, plus weight),
    one degree read per table entry created, the seed ids, and the output
    (member ids and one record per (set, scale))."""
    wb = 1 if weighted else 0
    return (8 * t["rows_gathered"] + (4 + wb) * t["row_entries"] + 4 * t["entries_created"]
            + 4 * seed_nodes + 4 * t["members_written"] + RECORD_BYTES * n_records)


def cpu_baseline(g, sp, sn, sc, stride, got_res):
    """The oracle on every stride-th seed set, single thread, on this host."""
    import oracle
    from paper_1301_0955_amd import workloads as W
    sp2, sn2, ids = W.subsample_sets(sp, sn, stride)
    o = oracle.Oracle.from_graph(g)
    t0 = time.perf_counter()
    ref = o.run_sets(sp2, sn2, sc)
    dt = time.perf_counter() - t0
    G = int(ref["ctr"][:, 0].sum())
    parity = None
    if got_res is not None:
        S = sc.size
        ok = True
        for j, q in enumerate(ids.tolist()):
            for s in range(S):
                r, rq = j * S + s, q * S + s
                a = got_res["members"][got_res["off"][rq]:got_res["off"][rq] + got_res["cnt"][rq]]
                b = ref["members"][ref["off"][r]:ref["off"][r] + ref["cnt"][r]]
                if (not np.array_equal(a, b) or got_res["K"][rq] != ref["K"][r]
                        or not np.array_equal(got_res["ctr"][rq], ref["ctr"][r])):
                    ok = False
                    break
            if not ok:
                break
        parity = "bit-exact" if ok else "MISMATCH"
    return dict(value=G / dt, unit="gains/s", cores=1, kind="oracle",
                sample="every %dth seed set (%d of %d), all %d scales; %.1f s, %d gains"
                       % (stride, ids.size, sp.size - 1, sc.size, dt, G),
                seconds=dt, parity_on_sample=parity)


def profiled_traffic(kernel: str, tier_caps, workload_name: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on this workload, tier layout and kernel source;
    else None."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "sweep_lfr2-100k_kernels.md")
    if workload_name != "medium" or not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"^kernels_sha256: ([0-9a-f]{64})", text, re.M)
    m_tr = re.search(r"^traffic_bytes_per_launch: (\{.*\})", text, re.M)
    m_caps = re.search(r"^profiled_tier_capacities: (\[.*\])", text, re.M)
    if not (m_sha and m_tr and m_caps):
        return None
    src = os.path.join(ROOT, "paper_1301_0955_amd", "csrc", "lcd_kernels.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m_sha.group(1):
        return None
    if json.loads(m_caps.group(1)) != list(tier_caps):
        return None
    return json.loads(m_tr.group(1)).get(kernel)


def profiled_utilisation(kernel: str, workload_name: str):
    """VALU-issue and FP64 fractions of `kernel` from the committed counter
    summary of this kernel source on this workload; else None."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "sweep_lfr2-100k_utilisation.md")
    if workload_name != "medium" or not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"kernels_sha256 ([0-9a-f]{64})", text)
    m_u = re.search(r"^utilisation: (\{.*\})", text, re.M)
    if not (m_sha and m_u):
        return None
    src = os.path.join(ROOT, "paper_1301_0955_amd", "csrc", "lcd_kernels.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != m_sha.group(1):
        return None
    u = json.loads(m_u.group(1)).get(kernel)
    if u is None:
        return None
    return dict(valu_issue_frac=u["valu_issue_frac"], fp64_frac_upper=u["fp64_frac_upper"],
                source="profiles/sweep_lfr2-100k_utilisation.md")


def W_seed_perm(g):
    from paper_1301_0955_amd import workloads as W
    return W.seed_permutation(g, 1)


def percentiles(x):
    x = np.asarray(x, dtype=np.float64)
    if x.size == 0:
        return {}
    p = np.percentile(x, [50, 90, 99, 99.9])
    return dict(p50=round(float(p[0]), 4), p90=round(float(p[1]), 4), p99=round(float(p[2]), 4),
                p999=round(float(p[3]), 4), mean=round(float(x.mean()), 4), max=round(float(x.max()), 4))


# device memory the query server may hold: the global-table tiers buy as
# many tables as it allows (a table of the whole-graph tier is 32 MiB on the
# 1M-node graph)
SERVE_MEM_BUDGET = 16 << 30


def serve_bench(lcd, G, g, qps, seconds, warmup_s, oracle_sample, seed=1):
    """Open-loop Poisson stream of (seed set, alpha) queries against the
    query server; latency = completion stamp - scheduled arrival."""
    import oracle
    from paper_1301_0955_amd import workloads as W
    n = int(round(qps * (warmup_s + seconds)))
    t_arr, sets, alphas = W.query_stream(g, n, qps, max_size=256, seed=seed)
    srv = lcd.Server(G, mem_budget=SERVE_MEM_BUDGET, max_slots=8192)
    for i in range(8):                      # first launches of the query kernels
        srv.result(srv.submit(sets[i], alphas[i]))
    st0 = srv.stats()
    sched = np.zeros(n, np.int64)
    tickets = []
    base = time.monotonic_ns() + 20_000_000
    next_log = 2.0
    for i in range(n):
        target = base + int(t_arr[i] * 1e9)
        while True:
            now = time.monotonic_ns()
            if now >= target:
                break
            if target - now > 2_000_000:
                time.sleep(0.001)
        sched[i] = target
        tickets.append(srv.submit(sets[i], alphas[i]))
        if t_arr[i] >= next_log:
            log("serving: %.0f s of %.0f submitted (%d queries)" % (t_arr[i], warmup_s + seconds, i + 1))
            next_log += 2.0
    res = []
    for t in tickets:
        res.append(srv.result(t, 120_000))
    st = srv.stats()
    srv.close()
    meas = np.nonzero(t_arr >= warmup_s)[0]
    lat_ms = np.array([(res[i]["t_done_ns"] - sched[i]) * 1e-6 for i in meas])
    queue_ms = np.array([(res[i]["t_start_ns"] - sched[i]) * 1e-6 for i in meas])
    first = sched[meas[0]]
    last = max(res[i]["t_done_ns"] for i in meas)
    batches = st["batches"] - st0["batches"]
    out = dict(
        workload="lfr3-1M resident; Poisson arrivals at %g queries/s; seed sets = BFS prefixes of "
                 "log-uniform size in [1, 256]; alpha log-uniform on [0.5, 1]; one fixpoint growth per "
                 "query" % qps,
        offered_qps=qps, seconds=seconds, warmup_s=warmup_s, queries=int(meas.size),
        achieved_qps=round(meas.size / ((last - first) * 1e-9), 1),
        latency_ms=percentiles(lat_ms), queue_ms=percentiles(queue_ms),
        mean_seed_size=round(float(np.mean([len(sets[i]) for i in meas])), 2),
        mean_members=round(float(np.mean([res[i]["members"].size for i in meas])), 2),
        batches=int(batches), mean_batch=round((st["completed"] - st0["completed"]) / max(batches, 1), 2),
        max_batch=st["max_batch"], max_lanes_busy=st["max_lanes_busy"], lanes=st["lanes"],
        stage_lanes=st["spill_lanes"], forwarded=st["forwarded"] - st0["forwarded"],
        later_stage_batches=st["spill_batches"] - st0["spill_batches"],
        requeued=st["requeued"], failed=st["failed"], server_mem_bytes=st["mem_held"],
        spill_tables=list(st["spill_tables"]))
    # latency by the lane that answered (lane k serves stage min(k, stages - 1))
    by_lane = {}
    for k in sorted(set(int(res[i]["lane"]) for i in meas)):
        sel = np.array([(res[i]["t_done_ns"] - sched[i]) * 1e-6 for i in meas if res[i]["lane"] == k])
        by_lane[str(k)] = dict(queries=int(sel.size), share=round(sel.size / meas.size, 4),
                               p50=round(float(np.percentile(sel, 50)), 3),
                               p99=round(float(np.percentile(sel, 99)), 3))
    out["latency_by_lane_ms"] = by_lane
    # the oracle on a sample of the same queries: per-query CPU latency and parity
    if oracle_sample > 0:
        o = oracle.Oracle.from_graph(g)
        pick = meas[np.linspace(0, meas.size - 1, min(oracle_sample, meas.size)).astype(np.int64)]
        cpu_ms = []
        ok = True
        for i in pick.tolist():
            t0 = time.perf_counter()
            per, K, V, f, ctr, _ = o.run_set(sets[i], np.array([alphas[i]]))
            cpu_ms.append((time.perf_counter() - t0) * 1e3)
            r = res[i]
            if (not np.array_equal(per[0], r["members"]) or int(K[0]) != r["K"] or int(V[0]) != r["V"]
                    or not np.array_equal(ctr[0], r["ctr"])):
                ok = False
        out["cpu_oracle"] = dict(kind="oracle", cores=1, queries=int(pick.size),
                                 latency_ms=percentiles(cpu_ms),
                                 note="service time of one query on one host core, no queueing")
        out["parity_on_sample"] = "bit-exact" if ok else "MISMATCH"
    return out


def merge_bench(lcd, G, g, sp, sn, sc, with_oracle):
    """The multi-scale loop with the check-and-merge phase (lcd_sweep_merge):
    on a 20k-node weighted hierarchy beside the oracle (every record and
    merged-into id compared), and on the main workload (device only)."""
    import oracle
    from paper_1301_0955_amd import workloads as W
    gm = W.lfr_hierarchical(20_000, 2.5, 15.0, 100, 1.5, 20, 200, mu=0.25, levels=3, weighted=True,
                            wmax=16, seed=5)
    msp, msn = W.seed_rule1(gm, 5)
    msc = W.log_scales(16)
    GM = lcd.Graph.from_workload(gm)
    walls = []
    for _ in range(2):
        t0 = time.perf_counter()
        r = lcd.lcd_sweep_merge(GM, msc, msp, msn)
        walls.append(time.perf_counter() - t0)
        got = lcd.sweep_to_numpy(r)
        into = lcd.merged_into(r)
        r.free()
    S = msc.size
    small = dict(workload="20,000-node 3-level weighted LFR-style graph (mean degree 15, max 100, mixing "
                          "0.25, weights 1..16), rule-1 seeds (%d), 16 scales, eta 1/2" % (msp.size - 1),
                 seconds_gpu=round(min(walls), 4),
                 live_finest=int((into[0::S] == -1).sum()), live_coarsest=int((into[S - 1::S] == -1).sum()))
    if with_oracle:
        t0 = time.perf_counter()
        ref = oracle.Oracle.from_graph(gm).run_merge(msp, msn, msc)
        small["seconds_oracle_1core"] = round(time.perf_counter() - t0, 4)
        small["rounds"] = int(ref["rounds"].sum())
        same = np.array_equal(into, ref["into"]) and np.array_equal(got["cnt"], ref["cnt"])
        same = same and np.array_equal(got["K"], ref["K"]) and np.array_equal(got["V"], ref["V"])
        same = same and np.array_equal(got["ctr"], np.asarray(ref["ctr"], np.uint64))
        if same:   # member lists record by record (the two lay records out differently)
            for rr in range(int(ref["cnt"].size)):
                c = int(ref["cnt"][rr])
                a, b = int(got["off"][rr]), int(ref["off"][rr])
                if c and not np.array_equal(got["members"][a:a + c], ref["members"][b:b + c]):
                    same = False
                    break
        small["identical"] = bool(same)
    GM.free()
    t0 = time.perf_counter()
    r = lcd.lcd_sweep_merge(G, sc, sp, sn)
    wall = time.perf_counter() - t0
    into = lcd.merged_into(r)
    r.free()
    S = sc.size
    main = dict(seconds_gpu=round(wall, 4), live_finest=int((into[0::S] == -1).sum()),
                live_coarsest=int((into[S - 1::S] == -1).sum()))
    log("merge: lfr-20k %.3f s (oracle %s s), main workload %.3f s"
        % (small["seconds_gpu"], small.get("seconds_oracle_1core"), main["seconds_gpu"]))
    return dict(lfr_20k=small, main_workload=main)


def sweep_compare(lcd, G, g, sp, sn, sc, steps, prm):
    """Persistent all-scales launch vs the per-scale launch loop on one
    workload (device time of each, identical results required)."""
    import torch
    t0 = time.perf_counter()
    tuned = lcd.lcd_tune(G, sc, sp, sn)
    log("lfr3-1M autotuned in %.1f s: %s" % (time.perf_counter() - t0, tuned["best"]))
    d_sc = torch.as_tensor(sc, dtype=torch.float64, device="cuda")
    d_sp = torch.as_tensor(sp, dtype=torch.int32, device="cuda")
    d_sn = torch.as_tensor(sn, dtype=torch.int32, device="cuda")
    r = lcd.lcd_sweep(G, d_sc, d_sp, d_sn, **prm)
    r.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rs = [lcd.lcd_sweep(G, d_sc, d_sp, d_sn, **prm) for _ in range(steps)]
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    sts = [x.stats() for x in rs]
    tot = rs[0].counters()
    ids = np.arange(0, sp.size - 1, 997, dtype=np.int32)
    a = rs[0].sets_to_numpy(ids)
    for x in rs:
        x.free()
    rl = lcd.lcd_sweep(G, d_sc, d_sp, d_sn, mode=lcd.LCD_PER_SCALE_LOOP, **prm)
    lst = rl.stats()
    b = rl.sets_to_numpy(ids)
    tot_l = rl.counters()
    rl.free()
    same = (tot == tot_l and np.array_equal(a["members"], b["members"]) and np.array_equal(a["K"], b["K"])
            and np.array_equal(a["ctr"], b["ctr"]))
    ms = float(np.mean([x["ms_total"] for x in sts]))
    return dict(ms_per_sweep_wall=round(wall * 1e3, 3), sweep_ms_device=round(ms, 3),
                ms_tier=[round(float(np.mean([x["ms_tier"][k] for x in sts])), 3)
                         for k in range(sts[0]["tiers"])],
                tier_kernels=[KERNEL_OF_KIND[k] for k in sts[0]["tier_kind"][:sts[0]["tiers"]]],
                tuned=tuned["best"],
                gains=int(tot[0]), gains_per_s=tot[0] / (wall), spilled_sets=sts[0]["n_spilled"],
                lds_capacity=sts[0]["lds_capacity"],
                per_scale_loop_ms_device=round(lst["ms_total"], 3), per_scale_loop_launches=lst["launches"],
                persistent_speedup=round(lst["ms_total"] / ms, 3), identical_results=bool(same))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="medium", choices=["small", "medium", "large"])
    ap.add_argument("--lds-capacity", type=int, default=0)
    ap.add_argument("--waves-per-block", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--cpu-stride", type=int, default=0,
                    help="oracle sample stride (0 = sized for ~15 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-loop-compare", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (static sizing)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 4 times (a plain copy kernel of known "
                         "size, to scale HBM byte counters) and exit")
    ap.add_argument("--no-large", action="store_true", help="skip the 1M-node sweep comparison")
    ap.add_argument("--no-serve", action="store_true", help="skip the query-serving run")
    ap.add_argument("--no-merge", action="store_true", help="skip the check-and-merge runs")
    ap.add_argument("--multigraph", action="store_true",
                    help="also sweep 64 independent graphs (1k-200k nodes) in one batched launch")
    ap.add_argument("--serve-qps", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--serve-warmup", type=float, default=2.0)
    ap.add_argument("--serve-oracle", type=int, default=300,
                    help="queries the oracle re-runs for CPU latency and parity")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(asked for --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = args.calibrate_copy << 18            # int32 elements
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied %d MiB x 4" % args.calibrate_copy)
        return
    from paper_1301_0955_amd import lcd

    t0 = time.perf_counter()
    g, sp, sn, sc, desc = workload(args.workload)
    log("workload %s ready in %.1f s: n=%d nnz=%d sets=%d scales=%d"
        % (args.workload, time.perf_counter() - t0, g.n, g.nnz, sp.size - 1, sc.size))
    G = lcd.Graph.from_workload(g)
    d_sc = torch.as_tensor(sc, dtype=torch.float64, device="cuda")
    d_sp = torch.as_tensor(sp, dtype=torch.int32, device="cuda")
    d_sn = torch.as_tensor(sn, dtype=torch.int32, device="cuda")
    prm = dict(lds_capacity=args.lds_capacity, waves_per_block=args.waves_per_block,
               blocks_per_cu=args.blocks_per_cu)
    tuned = None
    if not any(prm.values()) and not args.no_tune:
        t0 = time.perf_counter()
        tuned = lcd.lcd_tune(G, sc, sp, sn)
        log("autotuned in %.1f s: %s (sample of every %d-th set)"
            % (time.perf_counter() - t0, tuned["best"], tuned["sample_stride"]))
    torch.cuda.synchronize()

    # one result object; every step re-runs the whole sweep into it (inputs
    # and outputs stay on the device; the first call allocates)
    res = lcd.lcd_sweep(G, d_sc, d_sp, d_sn, **prm)
    for i in range(args.warmup):
        st = res.rerun().stats()
        log("warmup %d: device %.2f ms, tiers %s ms, spilled %d, reruns %d"
            % (i, st["ms_total"], [round(x, 2) for x in st["ms_tier"][:st["tiers"]]],
               st["n_spilled"], st["reruns"]))
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        stats.append(res.rerun().stats())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / max(args.steps, 1)
    totals = res.counters()
    log("timed %d steps: %.2f ms/step wall" % (args.steps, ms_step))
    got = lcd.sweep_to_numpy(res)
    res.free()

    # the same sweep captured in a hipGraph and replayed
    rg = lcd.lcd_sweep(G, d_sc, d_sp, d_sn, use_graph=1, **prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        rg.rerun()
    torch.cuda.synchronize()
    graph_ms = 1e3 * (time.perf_counter() - t0) / max(args.steps, 1)
    graph_same = bool(np.array_equal(rg.counters(), totals))
    rg.free()
    # a fresh call each step (allocation, seed upload, launch, statistics)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(2):
        lcd.lcd_sweep(G, d_sc, d_sp, d_sn, **prm).free()
    fresh_ms = 1e3 * (time.perf_counter() - t0) / 2
    log("hipGraph replay %.2f ms/step, fresh call %.2f ms" % (graph_ms, fresh_ms))

    gains = totals[0]
    ms_dev = float(np.mean([s["ms_total"] for s in stats]))
    st0 = stats[0]
    S = sc.size
    weighted = g.w is not None
    nt = st0["tiers"]
    ms_tier = [float(np.mean([s["ms_tier"][k] for s in stats])) for k in range(nt)]
    k_dom = int(np.argmax(ms_tier))
    t_dom = st0["tier"][k_dom]
    kbytes = algorithmic_bytes(t_dom, weighted, int(sn.size) if k_dom == 0 else 0,
                               t_dom["sets_finished"] * S)
    kname = KERNEL_OF_KIND[st0["tier_kind"][k_dom]]
    kms = ms_tier[k_dom]
    achieved = kbytes / (kms * 1e-3) / 1e9
    traffic = profiled_traffic(kname, st0["tier_capacity"][:nt], args.workload)
    roofline = dict(bound="hbm", kernel=kname, tier=k_dom, achieved=round(achieved, 3), peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 7), traffic=traffic,
                    traffic_GBs=None if traffic is None else round(traffic / (kms * 1e-3) / 1e9, 2),
                    algorithmic_bytes=int(kbytes), kernel_ms=round(kms, 4),
                    secondary=profiled_utilisation(kname, args.workload),
                    tiers=[dict(kernel=KERNEL_OF_KIND[st0["tier_kind"][k]],
                                table_entries=st0["tier_capacity"][k], ms=round(ms_tier[k], 3),
                                sets_finished=st0["tier"][k]["sets_finished"],
                                algorithmic_bytes=int(algorithmic_bytes(
                                    st0["tier"][k], weighted, int(sn.size) if k == 0 else 0,
                                    st0["tier"][k]["sets_finished"] * S)))
                           for k in range(nt)])

    loop = None
    if not args.no_loop_compare:
        r = lcd.lcd_sweep(G, d_sc, d_sp, d_sn, mode=lcd.LCD_PER_SCALE_LOOP, **prm)
        lst = r.stats()
        same = lcd.sweep_to_numpy(r)
        r.free()
        identical = (np.array_equal(same["K"], got["K"]) and np.array_equal(same["ctr"], got["ctr"])
                     and np.array_equal(same["cnt"], got["cnt"]))
        loop = dict(device_ms=round(lst["ms_total"], 3), launches=lst["launches"],
                    persistent_speedup=round(lst["ms_total"] / ms_dev, 3),
                    identical_results=bool(identical))
        log("per-scale loop: %.2f ms device (%d launches)" % (lst["ms_total"], lst["launches"]))

    cpu = None
    if not args.no_cpu_baseline:
        stride = args.cpu_stride or {"small": 1, "medium": 16, "large": 1024}[args.workload]
        log("cpu baseline: oracle on every %dth seed set" % stride)
        cpu = cpu_baseline(g, sp, sn, sc, stride, got)
        log("cpu baseline: %s" % cpu["sample"])

    # seed selection (initialisation of Algorithm 2) on the device vs the oracle
    seeds_info = {}
    perm = W_seed_perm(g)
    for rule in (1, 2):
        t0 = time.perf_counter()
        dev = lcd.lcd_seeds(G, perm, rule)
        t_dev = time.perf_counter() - t0
        entry = dict(seeds=int(dev.size), ms_device_call=round(t_dev * 1e3, 3))
        if not args.no_cpu_baseline:
            import oracle
            t0 = time.perf_counter()
            ref = oracle.Oracle.from_graph(g).seeds(perm, rule)
            entry["ms_oracle_1core"] = round((time.perf_counter() - t0) * 1e3, 3)
            entry["identical"] = bool(np.array_equal(dev, ref))
        seeds_info["rule%d" % rule] = entry
    log("seed selection: %s" % seeds_info)

    merge = None if args.no_merge else merge_bench(lcd, G, g, sp, sn, sc, not args.no_cpu_baseline)

    large = serving = None
    if not (args.no_large and args.no_serve) and args.workload != "large":
        t0 = time.perf_counter()
        from paper_1301_0955_amd import workloads as W
        gl, spl, snl, scl = W.workload_large()
        log("lfr3-1M ready in %.1f s: n=%d nnz=%d sets=%d scales=%d"
            % (time.perf_counter() - t0, gl.n, gl.nnz, spl.size - 1, scl.size))
        GL = lcd.Graph.from_workload(gl)
        if not args.no_large:
            large = sweep_compare(lcd, GL, gl, spl, snl, scl, 2, {})
            large["workload"] = ("lfr3-1M: 1,000,000-node 3-level LFR-style graph (mean degree 15, "
                                 "max 200, mixing 0.25, weights 1..16), rule-1 seeds (%d), 64 scales "
                                 "on [0.5,1]" % (spl.size - 1))
            log("lfr3-1M sweep: %.1f ms device, per-scale loop %.1f ms"
                % (large["sweep_ms_device"], large["per_scale_loop_ms_device"]))
        if not args.no_serve:
            serving = serve_bench(lcd, GL, gl, args.serve_qps, args.serve_seconds, args.serve_warmup,
                                  args.serve_oracle)
            log("serving: p50 %.3f ms, p99 %.3f ms at %.0f offered, %.0f achieved queries/s"
                % (serving["latency_ms"]["p50"], serving["latency_ms"]["p99"], serving["offered_qps"],
                   serving["achieved_qps"]))
        GL.free()

    multi = None
    if args.multigraph:
        from paper_1301_0955_amd import workloads as W
        t0 = time.perf_counter()
        gs, msp, msn, msg, msc = W.workload_multigraph()
        log("multigraph ready in %.1f s: %d graphs, %d nodes, %d seed sets"
            % (time.perf_counter() - t0, len(gs), sum(x.n for x in gs), msp.size - 1))
        GB = lcd.Graph.batch(gs)
        r = lcd.lcd_sweep_batch(GB, msc, msp, msn, msg)
        tot = r.counters()
        r.free()
        walls = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = lcd.lcd_sweep_batch(GB, msc, msp, msn, msg)
            walls.append(time.perf_counter() - t0)
            mst = r.stats()
            r.free()
        multi = dict(workload="64 independent LFR-style graphs, node counts log-uniform in [1k, 200k] "
                              "(%d nodes in all), weights 1..16, rule-1 seeds per graph, 32 scales, one "
                              "batched launch" % sum(x.n for x in gs),
                     graphs=len(gs), nodes=int(sum(x.n for x in gs)), seed_sets=int(msp.size - 1),
                     sweep_ms_device=round(mst["ms_total"], 3), ms_per_call_wall=round(1e3 * min(walls), 3),
                     gains=int(tot[0]), gains_per_s=tot[0] / min(walls))
        log("multigraph: %.1f ms device per sweep" % mst["ms_total"])
        GB.free()

    out = {
        "metric": METRIC,
        "value": gains / (ms_step * 1e-3),
        "unit": "gains/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n": g.n, "nnz": g.nnz, "seed_sets": int(sp.size - 1),
                   "scales": int(S), "graph_sha256": g.sha256()[:16],
                   "lds_capacity": st0["lds_capacity"], "waves_per_block": st0["waves_per_block"],
                   "grid_blocks": st0["grid_blocks"], "tiers": nt,
                   "tuned": tuned["best"] if tuned else None},
        "hipgraph_ms_per_step": round(graph_ms, 4),
        "hipgraph_identical_counters": graph_same,
        "fresh_call_ms": round(fresh_ms, 3),
        "sweep_ms_device": round(ms_dev, 4),
        "gains_per_step": int(gains),
        "counters": {"G": totals[0], "R": totals[1], "M": totals[2], "C": totals[3]},
        "gains_per_s_device": gains / (ms_dev * 1e-3),
        "spilled_sets": st0["n_spilled"],
        "roofline": roofline,
        "per_scale_loop": loop,
        "cpu_baseline": cpu,
        "seed_selection": seeds_info,
        "merge": merge,
        "large_sweep": large,
        "serving": serving,
        "multigraph": multi,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
