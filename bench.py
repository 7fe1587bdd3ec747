#!/usr/bin/env python3
"""Benchmark of the multi-scale local community sweep on one MI355X.

One step = one sweep (lcd_result_rerun of an lcd_sweep result): every seed
set of the workload grown through every scale (queue-emulated additions,
removal passes, fixpoint per scale, chained scales), with sorted member
lists, K, V, f and the work counters written for every (seed set, scale).
Inputs (graph, seeds, scales) are resident on the device before the timed
region.

The headline workload is the 10M-node graph of the largest configuration
with one GPU's share of its rule-1 seed sets (every --xl-stride-th set in
selection order: the sweep shards over seed sets with no exchange, so a
share at the full graph shape is what one GPU of a multi-GPU run does).

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
SUMMARY_BYTES = 24        # per (set, scale): K, V, f (the algorithmic output unit)
XL_STRIDE = 64            # default seed share of the 10M-node workload
KERNEL_OF_KIND = {0: "sweep_lds_kernel", 1: "sweep_global_kernel", 2: "sweep_team_lds_kernel",
                  3: "sweep_team_global_kernel"}
RECORD_MIN_ENTRIES = 65536   # workgroup tables this large run the record-layout kernel


def kernel_of(kind: int, cap: int) -> str:
    """Name of the kernel that runs a tier of this kind and table size."""
    if kind == 3 and cap >= RECORD_MIN_ENTRIES:
        return "sweep_team_global_rec_kernel"
    return KERNEL_OF_KIND[kind]


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
    elif name.startswith("xl"):
        stride = int(name[2:] or XL_STRIDE)
        g, sp_all, sn_all, sc = W.workload_xl()
        sp, sn, _ = W.subsample_sets(sp_all, sn_all, stride)
        m = g.meta
        desc = ("lfr3-10M: 10,000,000-node 3-level power-law graph (degree exponent 2.2, mean 20, max 5,000; "
                "achieved mean %.1f, max %d, %d directed entries; communities 20..5,000 nodes; mixing 0.3 "
                "(achieved %.3f); weights 1..16), every %dth of its %d rule-1 seed sets (%d sets: one GPU's "
                "share), 32 scales on [0.5,1]"
                % (m["achieved_mean_deg"], m["achieved_max_deg"], g.nnz, m["achieved_mu_comm"], stride,
                   sp_all.size - 1, sp.size - 1))
    else:
        raise SystemExit("unknown workload %s" % name)
    return g, sp, sn, sc, desc


def gather_bytes(t: dict, weighted: bool) -> int:
    """Algorithmic input bytes of one tier (the measurement rules):
    per CSR row that a move or a seed-set member gathers, its two offsets and
    its entries (id, plus weight); one degree read per table entry created
    for a committed scale.  Rows that a set resumed from a record gathers
    again, and work of a scale that overflowed and was redone in the next
    tier, are not counted."""
    wb = 1 if weighted else 0
    rows = t["move_rows"] + t["seed_rows"]
    ents = t["move_row_entries"] + t["seed_row_entries"]
    return 8 * rows + (4 + wb) * ents + 4 * t["entries_committed"]


def output_bytes(moves: int, seed_nodes: int, n_records: int) -> int:
    """Algorithmic output: 4 B per member change between consecutive scales
    (at most the seed set plus one per move) and a 24-byte summary (K, V, f)
    per (set, scale)."""
    return 4 * (moves + seed_nodes) + SUMMARY_BYTES * n_records


_CPU_JOB = None   # (graph, seed_ptr, seed_nodes, scales) inherited by forked oracle workers


def _oracle_chunk(ids):
    """Oracle run of the seed sets `ids` (a worker of the CPU baseline)."""
    import oracle
    g, sp, sn, sc = _CPU_JOB
    sizes = sp[ids + 1] - sp[ids]
    ptr = np.zeros(ids.size + 1, np.int32)
    np.cumsum(sizes, out=ptr[1:])
    nodes = np.concatenate([sn[sp[i]:sp[i + 1]] for i in ids]) if ids.size else np.zeros(0, np.int32)
    o = oracle.Oracle.from_graph(g)
    t0 = time.perf_counter()
    ref = o.run_sets(ptr, nodes, sc)
    dt = time.perf_counter() - t0
    return ids, ref, dt


class CpuBaseline:
    """The oracle on a bounded sample of the benchmarked seed sets, sharded
    over the host cores as independent processes (seed sets are independent
    in the sweep).  The worker pool is forked before the process touches the
    GPU; the runs start after the GPU's timed steps."""

    def __init__(self, g, sp, sn, sc, n_sample: int, cores: int):
        global _CPU_JOB
        import multiprocessing as mp
        ns = sp.size - 1
        self.ids = np.unique(np.linspace(0, max(ns - 1, 0), min(n_sample, ns)).astype(np.int64))
        self.cores = max(1, min(cores, self.ids.size))
        self.ns, self.S = ns, sc.size
        _CPU_JOB = (g, sp, sn, sc)
        self.pool = mp.get_context("fork").Pool(self.cores)

    def run(self, got_sets):
        """got_sets(ids) -> the GPU's records of those sets (lcd sets_to_numpy
        layout).  Returns the cpu_baseline object of the bench line."""
        chunks = [self.ids[k::self.cores] for k in range(self.cores)]
        t0 = time.perf_counter()
        outs = self.pool.map(_oracle_chunk, chunks)
        wall = time.perf_counter() - t0
        self.pool.close()
        self.pool.join()
        G = sum(int(ref["ctr"][:, 0].sum()) for _, ref, _ in outs)
        busy = sum(dt for _, _, dt in outs)
        ok = True
        S = self.S
        for ids, ref, _ in outs:
            got = got_sets(ids.astype(np.int32))
            for q in range(ids.size):
                for s in range(S):
                    r = q * S + s
                    a = got["members"][got["off"][r]:got["off"][r] + got["cnt"][r]]
                    b = ref["members"][ref["off"][r]:ref["off"][r] + ref["cnt"][r]]
                    fa, fb = float(got["f"][r]), float(ref["f"][r])
                    if (not np.array_equal(a, b) or got["K"][r] != ref["K"][r] or got["V"][r] != ref["V"][r]
                            or abs(fa - fb) > 1e-12 * abs(fb)
                            or not np.array_equal(np.asarray(got["ctr"][r], np.uint64),
                                                  np.asarray(ref["ctr"][r], np.uint64))):
                        ok = False
        return dict(value=G / wall, unit="gains/s", cores=self.cores, kind="oracle",
                    sample="%d of the %d benchmarked seed sets (evenly spaced), all %d scales, sharded over %d "
                           "processes: %.1f s wall, %.1f core-s, %d gains"
                           % (self.ids.size, self.ns, S, self.cores, wall, busy, G),
                    seconds=round(wall, 3), core_seconds=round(busy, 3), gains=G,
                    single_core_gains_per_s=G / busy if busy > 0 else None,
                    parity_on_sample=("bit-exact members, K, V, counters; f within 1e-12" if ok else "MISMATCH"))


# committed rocprofv3 summaries, per workload (a summary is used only while
# the kernel source, the workload and the tier layout match the run)
PROFILE_OF = {"medium": "sweep_lfr2-100k", "xl64": "sweep_lfr3-10M-share64"}


def _profile_text(workload_name: str, kind: str):
    import hashlib
    import re
    name = PROFILE_OF.get(workload_name)
    if name is None:
        return None
    path = os.path.join(ROOT, "profiles", "%s_%s.md" % (name, kind))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m_sha = re.search(r"kernels_sha256:? ([0-9a-f]{64})", text)
    src = os.path.join(ROOT, "paper_1301_0955_amd", "csrc", "lcd_kernels.hip")
    if not m_sha or hashlib.sha256(open(src, "rb").read()).hexdigest() != m_sha.group(1):
        return None
    return text


def profiled_traffic(kernel: str, tier_caps, workload_name: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on this workload, tier layout and kernel source;
    else None."""
    import re
    text = _profile_text(workload_name, "kernels")
    if text is None:
        return None
    m_tr = re.search(r"^traffic_bytes_per_launch: (\{.*\})", text, re.M)
    m_caps = re.search(r"^profiled_tier_capacities: (\[.*\])", text, re.M)
    if not (m_tr and m_caps) or json.loads(m_caps.group(1)) != list(tier_caps):
        return None
    return json.loads(m_tr.group(1)).get(kernel)


def profiled_utilisation(kernel: str, workload_name: str):
    """VALU-issue and FP64 fractions of `kernel` from the committed counter
    summary of this kernel source on this workload; else None."""
    import re
    text = _profile_text(workload_name, "utilisation")
    if text is None:
        return None
    m_u = re.search(r"^utilisation: (\{.*\})", text, re.M)
    if not m_u:
        return None
    u = json.loads(m_u.group(1)).get(kernel)
    if u is None:
        return None
    return dict(valu_issue_frac=u["valu_issue_frac"], fp64_frac_upper=u["fp64_frac_upper"],
                source="profiles/%s_utilisation.md" % PROFILE_OF[workload_name])


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
        routed=st["routed"] - st0["routed"],
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
                tier_kernels=[kernel_of(k, c) for k, c in zip(sts[0]["tier_kind"][:sts[0]["tiers"]],
                                                              sts[0]["tier_capacity"])],
                tuned=tuned["best"],
                gains=int(tot[0]), gains_per_s=tot[0] / (wall), spilled_sets=sts[0]["n_spilled"],
                lds_capacity=sts[0]["lds_capacity"],
                per_scale_loop_ms_device=round(lst["ms_total"], 3), per_scale_loop_launches=lst["launches"],
                persistent_speedup=round(lst["ms_total"] / ms, 3), identical_results=bool(same))


CPU_SETS_PER_CORE = {"small": 100, "medium": 300, "large": 40, "xl": 12}


def seeds_bench(lcd, G, g, with_oracle: bool) -> dict:
    """Seed selection (initialisation of Algorithm 2), rules 1 and 2, on the
    device (whole call, two runs, the second timed) vs the oracle's scan on
    one host core (its graph built beforehand, two runs, the second timed);
    the seeds must be identical."""
    perm = W_seed_perm(g)
    info = {}
    orc = None
    if with_oracle:
        import oracle
        orc = oracle.Oracle.from_graph(g)   # the graph resident on both sides before the timed calls
    for rule in (1, 2):
        lcd.lcd_seeds(G, perm, rule)
        t0 = time.perf_counter()
        dev = lcd.lcd_seeds(G, perm, rule)
        t_dev = time.perf_counter() - t0
        entry = dict(seeds=int(dev.size), ms_device_call=round(t_dev * 1e3, 3))
        if orc is not None:
            orc.seeds(perm, rule)
            t0 = time.perf_counter()
            ref = orc.seeds(perm, rule)
            entry["ms_oracle_1core"] = round((time.perf_counter() - t0) * 1e3, 3)
            entry["identical"] = bool(np.array_equal(dev, ref))
        info["rule%d" % rule] = entry
    return info


def medium_compare(lcd, steps, with_seeds=False, with_oracle=True):
    """The 100k-node workload: autotuned persistent sweep vs the per-scale
    launch loop (device time of each; identical counters and records), and
    optionally seed selection on its graph."""
    from paper_1301_0955_amd import workloads as W
    g, sp, sn, sc = W.workload_medium()
    G = lcd.Graph.from_workload(g)
    out = sweep_compare(lcd, G, g, sp, sn, sc, steps, {})
    out["workload"] = ("lfr2-100k: 100,000-node 2-level LFR-style graph (degree exp 2.5, mean 20, max 100; "
                       "community sizes exp 1.5 on [20,200]; mixing 0.3; unweighted), rule-1 seeds (%d), "
                       "32 scales on [0.5,1]" % (sp.size - 1))
    if with_seeds:
        out["seed_selection"] = seeds_bench(lcd, G, g, with_oracle)
    G.free()
    return out


def nmi_bench(lcd):
    """Sec. 4's multi-scale relevance analysis on the device: the NMI of
    successive community sets (averaged over 3 and 5 scales) and with the
    planted levels, for the check-and-merge run of the planted-partition
    graph, against the oracle's NMI of the oracle's own run."""
    import oracle
    from paper_1301_0955_amd import workloads as W
    g, sp, sn, sc = W.workload_small()
    G = lcd.Graph.from_workload(g)
    res = lcd.lcd_sweep_merge(G, sc, sp, sn)
    t0 = time.perf_counter()
    w3 = res.nmi_successive(3)
    w5 = res.nmi_successive(5)
    subs = [np.arange(50 * k, 50 * k + 50, dtype=np.int32) for k in range(20)]
    groups = [np.arange(250 * k, 250 * k + 250, dtype=np.int32) for k in range(4)]
    vs_sub = [res.nmi_cover(s, subs) for s in range(sc.size)]
    vs_grp = [res.nmi_cover(s, groups) for s in range(sc.size)]
    dt = time.perf_counter() - t0
    res.free()
    G.free()
    ref = oracle.Oracle.from_graph(g).run_merge(sp, sn, sc)
    S = sc.size
    covers = [[ref["members"][ref["off"][j * S + s]:ref["off"][j * S + s] + ref["cnt"][j * S + s]]
               for j in range(sp.size - 1) if ref["cnt"][j * S + s] > 0] for s in range(S)]
    err = max(float(np.max(np.abs(w3 - oracle.nmi_successive(g.n, covers, 3)))),
              float(np.max(np.abs(w5 - oracle.nmi_successive(g.n, covers, 5)))),
              max(abs(vs_sub[s] - oracle.nmi(g.n, covers[s], subs)) for s in range(S)),
              max(abs(vs_grp[s] - oracle.nmi(g.n, covers[s], groups)) for s in range(S)))
    return dict(workload="planted-partition-1k with the check-and-merge phase, 10 scales",
                nmi_successive_3=[round(x, 6) for x in w3.tolist()],
                nmi_successive_5=[round(x, 6) for x in w5.tolist()],
                nmi_vs_planted_sub=[round(x, 6) for x in vs_sub], nmi_vs_planted_groups=[round(x, 6) for x in vs_grp],
                seconds_device_calls=round(dt, 4), max_abs_diff_vs_oracle=err)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="xl",
                    help="small | medium | large | xl[STRIDE] (the 10M-node graph with every STRIDE-th seed set, "
                         "default %d)" % XL_STRIDE)
    ap.add_argument("--lds-capacity", type=int, default=0)
    ap.add_argument("--output", choices=("delta", "full"), default="delta",
                    help="member pool layout of the timed sweep")
    ap.add_argument("--waves-per-block", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--cpu-sets", type=int, default=0, help="oracle sample size (0 = sized per workload)")
    ap.add_argument("--cpu-cores", type=int, default=0, help="oracle processes (0 = min(16, host cores))")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-loop-compare", action="store_true")
    ap.add_argument("--tune", action="store_true", help="autotune the headline workload (default: xl not tuned)")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (static sizing)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 4 times (a plain copy kernel of known "
                         "size, to scale HBM byte counters) and exit")
    ap.add_argument("--no-large", action="store_true", help="skip the 1M-node sweep comparison")
    ap.add_argument("--no-medium", action="store_true", help="skip the 100k-node sweep comparison")
    ap.add_argument("--no-serve", action="store_true", help="skip the query-serving run")
    ap.add_argument("--no-merge", action="store_true", help="skip the check-and-merge runs")
    ap.add_argument("--no-nmi", action="store_true", help="skip the NMI analysis leg")
    ap.add_argument("--no-multigraph", action="store_true", help="skip the 64-graph batched sweep")
    ap.add_argument("--no-hipgraph", action="store_true", help="skip the hipGraph replay of the timed sweep")
    ap.add_argument("--serve-qps", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=20.0)
    ap.add_argument("--serve-warmup", type=float, default=2.0)
    ap.add_argument("--serve-oracle", type=int, default=1000,
                    help="queries the oracle re-runs for CPU latency and parity")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(asked for --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        import torch
        torch.cuda.set_device(0)
        n = args.calibrate_copy << 18            # int32 elements
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied %d MiB x 4" % args.calibrate_copy)
        return

    # inputs (host), and the oracle's worker processes, before anything
    # touches the GPU
    t0 = time.perf_counter()
    g, sp, sn, sc, desc = workload(args.workload)
    wl_key = "xl" if args.workload.startswith("xl") else args.workload
    prof_key = ("xl%d" % int(args.workload[2:] or XL_STRIDE)) if wl_key == "xl" else wl_key
    g_n, g_nnz = int(g.n), int(g.nnz)
    log("workload %s ready in %.1f s: n=%d nnz=%d sets=%d scales=%d"
        % (args.workload, time.perf_counter() - t0, g.n, g.nnz, sp.size - 1, sc.size))
    cpu_job = None
    if not args.no_cpu_baseline:
        cores = args.cpu_cores or min(16, os.cpu_count() or 1)
        n_sample = args.cpu_sets or CPU_SETS_PER_CORE[wl_key] * cores
        cpu_job = CpuBaseline(g, sp, sn, sc, n_sample, cores)
        log("cpu baseline: %d oracle processes forked for %d seed sets" % (cpu_job.cores, cpu_job.ids.size))

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    from paper_1301_0955_amd import lcd

    t0 = time.perf_counter()
    G = lcd.Graph.from_workload(g)
    log("graph uploaded in %.1f s" % (time.perf_counter() - t0))
    d_sc = torch.as_tensor(sc, dtype=torch.float64, device="cuda")
    d_sp = torch.as_tensor(sp, dtype=torch.int32, device="cuda")
    d_sn = torch.as_tensor(sn, dtype=torch.int32, device="cuda")
    prm = dict(lds_capacity=args.lds_capacity, waves_per_block=args.waves_per_block,
               blocks_per_cu=args.blocks_per_cu)
    tuned = None
    # the 10M-node share keeps the library's static sizing for graphs of
    # millions of nodes (deterministic, so the committed counter profile of
    # this configuration applies to every run)
    do_tune = not any(prm.values()) and not args.no_tune and (wl_key != "xl" or args.tune)
    if do_tune:
        t0 = time.perf_counter()
        tuned = lcd.lcd_tune(G, sc, sp, sn)
        log("autotuned in %.1f s: %s (sample of every %d-th set)"
            % (time.perf_counter() - t0, tuned["best"], tuned["sample_stride"]))
    torch.cuda.synchronize()
    # member pool as deltas between scales (the sorted list only at a set's
    # first scale), or whole lists at every changed scale
    prm["output_mode"] = lcd.LCD_OUT_DELTA if args.output == "delta" else lcd.LCD_OUT_FULL

    # one result object; every step re-runs the whole sweep into it (inputs
    # and outputs stay on the device; the first call allocates and sizes the
    # member pool)
    t0 = time.perf_counter()
    res = lcd.lcd_sweep(G, d_sc, d_sp, d_sn, **prm)
    log("first call %.1f s (reruns for pool growth: %d)" % (time.perf_counter() - t0, res.stats()["reruns"]))
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
        log("step %d: device %.2f ms" % (i, stats[-1]["ms_total"]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / max(args.steps, 1)
    totals = res.counters()
    log("timed %d steps: %.2f ms/step wall" % (args.steps, ms_step))

    # the same sweep captured in a hipGraph and replayed (two replays)
    graph_ms, graph_same = None, None
    if not args.no_hipgraph:
        rg = lcd.lcd_sweep(G, d_sc, d_sp, d_sn, use_graph=1, **prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(2):
            rg.rerun()
        torch.cuda.synchronize()
        graph_ms = 1e3 * (time.perf_counter() - t0) / 2
        graph_same = bool(np.array_equal(rg.counters(), totals))
        rg.free()
        log("hipGraph replay %.2f ms/step" % graph_ms)

    gains = totals[0]
    ms_dev = float(np.mean([s["ms_total"] for s in stats]))
    st0 = stats[0]
    S = sc.size
    weighted = g.w is not None
    nt = st0["tiers"]
    ms_tier = [float(np.mean([s["ms_tier"][k] for s in stats])) for k in range(nt)]
    k_dom = int(np.argmax(ms_tier))
    t_dom = st0["tier"][k_dom]
    kbytes = gather_bytes(t_dom, weighted)
    kname = kernel_of(st0["tier_kind"][k_dom], st0["tier_capacity"][k_dom])
    kms = ms_tier[k_dom]
    achieved = kbytes / (kms * 1e-3) / 1e9
    n_rec = (sp.size - 1) * S
    all_bytes = (sum(gather_bytes(st0["tier"][k], weighted) for k in range(nt))
                 + output_bytes(int(totals[2]), int(sn.size), n_rec))
    scanned = [int(st0["tier"][k]["entries_scanned"]) for k in range(nt)]
    traffic = profiled_traffic(kname, st0["tier_capacity"][:nt], prof_key)
    roofline = dict(bound="hbm", kernel=kname, tier=k_dom, achieved=round(achieved, 3), peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 7), traffic=traffic,
                    traffic_GBs=None if traffic is None else round(traffic / (kms * 1e-3) / 1e9, 2),
                    algorithmic_bytes=int(kbytes), kernel_ms=round(kms, 4),
                    bytes_rule="per CSR row gathered by a move or a seed member: 8 B offsets + (4 + 1 if "
                               "weighted) B per entry; 4 B per table entry created; rows regathered by resumed "
                               "sets and work of overflowed scales excluded; the kernel's own output not "
                               "attributed (it is in all_tiers)",
                    all_tiers=dict(algorithmic_bytes=int(all_bytes), ms=round(ms_dev, 4),
                                   achieved=round(all_bytes / (ms_dev * 1e-3) / 1e9, 3),
                                   frac=round(all_bytes / (ms_dev * 1e-3) / 1e9 / HBM_PEAK_GBS, 7),
                                   output_rule="4 B per member change between scales (at most seeds + moves) "
                                               "+ 24 B (K, V, f) per (set, scale)"),
                    scanned_entries=scanned, scanned_over_gains=round(sum(scanned) / max(gains, 1), 3),
                    secondary=profiled_utilisation(kname, prof_key),
                    tiers=[dict(kernel=kernel_of(st0["tier_kind"][k], st0["tier_capacity"][k]),
                                table_entries=st0["tier_capacity"][k], ms=round(ms_tier[k], 3),
                                sets_finished=st0["tier"][k]["sets_finished"],
                                entries_scanned=scanned[k],
                                algorithmic_bytes=int(gather_bytes(st0["tier"][k], weighted)))
                           for k in range(nt)])

    loop = None
    if not args.no_loop_compare and wl_key != "xl":
        r = lcd.lcd_sweep(G, d_sc, d_sp, d_sn, mode=lcd.LCD_PER_SCALE_LOOP, **prm)
        lst = r.stats()
        same = lcd.sweep_to_numpy(r)
        r.free()
        got = lcd.sweep_to_numpy(res)
        identical = (np.array_equal(same["K"], got["K"]) and np.array_equal(same["ctr"], got["ctr"])
                     and np.array_equal(same["cnt"], got["cnt"]))
        loop = dict(device_ms=round(lst["ms_total"], 3), launches=lst["launches"],
                    persistent_speedup=round(lst["ms_total"] / ms_dev, 3),
                    identical_results=bool(identical))
        log("per-scale loop: %.2f ms device (%d launches)" % (lst["ms_total"], lst["launches"]))

    cpu = None
    if cpu_job is not None:
        log("cpu baseline: oracle on %d seed sets over %d processes" % (cpu_job.ids.size, cpu_job.cores))
        cpu = cpu_job.run(lambda ids: res.sets_to_numpy(ids))
        log("cpu baseline: %s; parity %s" % (cpu["sample"], cpu["parity_on_sample"]))
    res.free()

    # seed selection (initialisation of Algorithm 2) on the device vs the oracle
    # (on the 100k-node graph when the headline graph is the 10M one, whose
    # rule-2 oracle run alone would take minutes)
    seeds_info = {}
    if wl_key != "xl":
        seeds_info = seeds_bench(lcd, G, g, not args.no_cpu_baseline)
        seeds_info["graph"] = desc
        log("seed selection: %s" % seeds_info)
    G.free()
    del g

    medium = None if (args.no_medium or wl_key == "medium") else medium_compare(
        lcd, 2, with_seeds=wl_key == "xl", with_oracle=not args.no_cpu_baseline)
    if medium:
        log("lfr2-100k sweep: %.1f ms device, per-scale loop %.1f ms"
            % (medium["sweep_ms_device"], medium["per_scale_loop_ms_device"]))
        if "seed_selection" in medium:
            seeds_info = dict(medium.pop("seed_selection"), graph="lfr2-100k")
            log("seed selection (lfr2-100k): %s" % seeds_info)

    merge = None
    if not args.no_merge:
        from paper_1301_0955_amd import workloads as W
        gm, spm, snm, scm = W.workload_medium()
        GM = lcd.Graph.from_workload(gm)
        merge = merge_bench(lcd, GM, gm, spm, snm, scm, not args.no_cpu_baseline)
        GM.free()
    nmi = None if args.no_nmi else nmi_bench(lcd)
    if nmi:
        log("nmi: successive(3) %s; device vs oracle max diff %.2e" % (nmi["nmi_successive_3"],
                                                                      nmi["max_abs_diff_vs_oracle"]))

    large = serving = None
    if not (args.no_large and args.no_serve) and wl_key != "large":
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
    if not args.no_multigraph:
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
        for _ in range(2):
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
        "config": None,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    out["config"] = {"workload": desc, "n": g_n, "nnz": g_nnz, "seed_sets": int(sp.size - 1), "scales": int(S),
                     "lds_capacity": st0["lds_capacity"], "waves_per_block": st0["waves_per_block"],
                     "grid_blocks": st0["grid_blocks"], "tiers": nt,
                     "tier_capacity": st0["tier_capacity"][:nt], "output": args.output,
                     "tuned": tuned["best"] if tuned else None}
    out.update({
        "sweep_ms_device": round(ms_dev, 4),
        "hipgraph_ms_per_step": round(graph_ms, 4) if graph_ms is not None else None,
        "hipgraph_identical_counters": graph_same,
        "gains_per_step": int(gains),
        "counters": {"G": totals[0], "R": totals[1], "M": totals[2], "C": totals[3]},
        "gains_per_s_device": gains / (ms_dev * 1e-3),
        "spilled_sets": st0["n_spilled"],
        "pool_entries": st0["pool_used"],
        "per_scale_loop": loop,
        "seed_selection": seeds_info,
        "medium_sweep": medium,
        "large_sweep": large,
        "merge": merge,
        "nmi": nmi,
        "serving": serving,
        "multigraph": multi,
    })
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
