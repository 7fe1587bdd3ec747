// Host side of the C ABI declared in include/lcd.h: validation, device
// memory, launch sizing, the launch sequence of a sweep and the readout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <iterator>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "lcd.h"
#include "lcd_host.h"
#include "lcd_internal.h"

using namespace lcd;

namespace {
thread_local std::string t_err;
}  // namespace

namespace lcd {

lcd_status fail(lcd_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    t_err = buf;
    return s;
}

lcd_status device_info(DevInfo &d) {
    HIPCHK(hipGetDevice(&d.device));
    int v = 0;
    HIPCHK(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, d.device));
    d.cus = v;
    HIPCHK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, d.device));
    d.lds_cu = v;
    HIPCHK(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, d.device));
    d.lds_block = v;
    HIPCHK(hipDeviceGetAttribute(&v, hipDeviceAttributeWallClockRate, d.device));
    if (v > 0)
        d.wall_khz = v;
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, d.device));
    std::snprintf(d.arch, sizeof(d.arch), "%s", prop.gcnArchName);
    if (d.lds_cu <= 0)
        d.lds_cu = 65536;
    if (d.lds_block <= 0)
        d.lds_block = 65536;
    return LCD_OK;
}

lcd_status ensure_slab(Slab &sl, int32_t cap, int32_t slots, hipStream_t st) {
    const int32_t hbits = next_pow2_bits(2 * (int64_t)cap);
    const int64_t stride = slab_stride(cap);
    if (sl.buf && sl.cap == cap && sl.slots == slots && !sl.dirty)
        return LCD_OK;
    if (!(sl.buf && sl.cap == cap && sl.slots == slots)) {
        dev_free(sl.buf);
        CHK(dev_alloc(&sl.buf, (size_t)(stride * slots)));
    }
    sl.stride = stride;
    sl.cap = cap;
    sl.hbits = hbits;
    sl.slots = slots;
    // all-ones bytes: every hash slot empty (-1); other arrays need no init
    HIPCHK(launch_fill_i32((int32_t *)sl.buf, -1, stride * slots / 4, st));
    sl.dirty = false;
    return LCD_OK;
}

lcd_status plan_tiers(const DevInfo &dev, int32_t n, const lcd_params &p, TierPlan &tp) {
    int32_t cap = p.lds_capacity > 0 ? p.lds_capacity : 512;
    if (cap % 64 != 0 || cap < 64 || cap > 8192)
        return fail(LCD_EINVAL, "lds_capacity must be a multiple of 64 in [64, 8192]");
    if (p.spill_mode < 0 || p.spill_mode > 2)
        return fail(LCD_EINVAL, "spill_mode must be 0, 1 or 2");
    const int32_t hbits0 = next_pow2_bits(2 * (int64_t)cap);
    const int64_t tb = table_bytes(cap, hbits0);
    int32_t wpb = p.waves_per_block > 0 ? p.waves_per_block
                                        : (int32_t)std::max<int64_t>(1, std::min<int64_t>(4, dev.lds_block / tb));
    if (wpb > 4)
        return fail(LCD_EINVAL, "waves_per_block must be at most 4");
    if (wpb * tb > dev.lds_block)
        return fail(LCD_EINVAL, "LDS table of %lld bytes x %d waves exceeds %lld bytes per block",
                    (long long)tb, wpb, (long long)dev.lds_block);
    int32_t bpc = p.blocks_per_cu > 0 ? p.blocks_per_cu
                                      : (int32_t)std::max<int64_t>(1, dev.lds_cu / (wpb * tb));
    bpc = std::min(bpc, 32);
    tp.n = 0;
    tp.t[tp.n++] = TierSpec{TIER_WAVE_LDS, cap, hbits0, wpb, dev.cus * bpc, 0, -1};
    const int64_t need = std::max<int64_t>(64, n);
    const int32_t capn = (int32_t)((int64_t)1 << next_pow2_bits(need));
    int32_t have = cap;   // largest table so far
    auto add_global = [&](int32_t kind, int32_t c, int32_t waves, int32_t slots, int32_t slab) {
        tp.t[tp.n++] = TierSpec{kind, c, next_pow2_bits(2 * (int64_t)c), waves, 0, slots, slab};
        have = c;
    };
    if (p.team_waves < 0 || 64 * p.team_waves > kTeamMaxThreads)
        return fail(LCD_EINVAL, "team_waves must be in [0, %d]", kTeamMaxThreads / 64);
    // graphs of millions of nodes: their sets are chains of thousands of
    // dependent steps on global tables, and two waves per set keep twice as
    // many sets in flight at a step cost little above four waves'
    const int32_t team_waves = p.team_waves > 0 ? p.team_waves : (n >= (4 << 20) ? 2 : 4);
    // workgroups of a workgroup tier that stay resident on the whole chip
    auto resident = [&](int32_t kind, int32_t waves, size_t lds) -> int32_t {
        int32_t nb = 0;
        if (tier_blocks_per_cu(kind, waves, lds, &nb) != hipSuccess || nb < 1)
            nb = 1;
        return dev.cus * nb;
    };
    if (p.spill_mode == 1 || p.spill_mode == 2) {
        const int32_t c1 = std::min<int32_t>(16384, capn);
        if (c1 > have && n > have)
            add_global(TIER_WAVE_GLOBAL, c1, 4, 4096, 0);
        if (capn > have && n > have) {
            int64_t slots = ((int64_t)4 << 30) / slab_stride(capn);
            if (p.spill_mode == 1)
                add_global(TIER_WAVE_GLOBAL, capn, 4, (int32_t)std::max<int64_t>(4, std::min<int64_t>(256, slots)), 1);
            else
                add_global(TIER_TEAM_GLOBAL, capn, team_waves,
                           (int32_t)std::max<int64_t>(4, std::min<int64_t>(resident(TIER_TEAM_GLOBAL, team_waves, 0), slots)), 1);
        }
        return LCD_OK;
    }
    // workgroup tiers: an LDS table per workgroup, then global tables
    int32_t cl = std::max(1024, 2 * cap);
    if (p.team_capacity > 0) {
        cl = p.team_capacity;
        if (cl % 64 != 0 || cl > 8192 ||
            table_bytes(cl, next_pow2_bits(2 * (int64_t)cl)) + 1024 > dev.lds_block)
            return fail(LCD_EINVAL, "team_capacity must be a multiple of 64 whose table fits one workgroup's LDS");
    } else {
        while (cl > 64 && table_bytes(cl, next_pow2_bits(2 * (int64_t)cl)) + 1024 > dev.lds_block)
            cl >>= 1;
    }
    if (cl > have && n > have) {
        const int32_t hb = next_pow2_bits(2 * (int64_t)cl);
        tp.t[tp.n++] = TierSpec{TIER_TEAM_LDS, cl, hb, team_waves,
                                resident(TIER_TEAM_LDS, team_waves, (size_t)table_bytes(cl, hb)), 0, -1};
        have = cl;
    }
    // graphs of millions of nodes grow communities of thousands of members
    // whose tables hold tens of thousands of entries: there the first global
    // tier takes 131,072 entries, so that such sets run one per resident
    // workgroup instead of waiting for the few whole-graph tables
    const int32_t c2 = std::min<int32_t>(n >= (4 << 20) ? 131072 : 16384, capn);
    if (c2 > have && n > have)
        add_global(TIER_TEAM_GLOBAL, c2, team_waves, resident(TIER_TEAM_GLOBAL, team_waves, 0), 0);
    if (capn > have && n > have) {
        // the whole-graph tier gets the few largest communities, whose
        // step-by-step chain is the tier's time: the widest workgroups
        const int32_t wide = kTeamMaxThreads / 64;
        int64_t slots = ((int64_t)4 << 30) / slab_stride(capn);
        add_global(TIER_TEAM_GLOBAL, capn, wide,
                   (int32_t)std::max<int64_t>(4, std::min<int64_t>(resident(TIER_TEAM_GLOBAL, wide, 0), slots)), 1);
    }
    return LCD_OK;
}

lcd_status enqueue_tiers(const SweepArgs &a0, const TierPlan &tp, int first, int last, int32_t blocks0,
                         Slab *slabs, int32_t *const *work, int32_t *const *ordered, hipStream_t st,
                         hipEvent_t *ev, int32_t *launches) {
    // ordering pays only when a launch spans several scales
    const bool order = ordered && a0.S >= 2 && a0.S <= 1024 && a0.s_end - a0.s_begin >= 2 && a0.n_sets > 0;
    if (first < 0 || last > tp.n || first > last)
        return fail(LCD_EINVAL, "tier range [%d, %d) outside the plan of %d tiers", first, last, tp.n);
    for (int k = first; k < last; ++k) {
        const TierSpec &T = tp.t[k];
        if (ev)
            HIPCHK(hipEventRecord(ev[k], st));
        SweepArgs b = a0;
        b.tier = k;
        b.kind = T.kind;
        b.in_from = k > 0 ? k - 1 : 0;
        b.work_in = k > 0 ? work[k - 1] : nullptr;
        if (k > 0 && order && ordered[k - 1]) {
            HIPCHK(launch_order_spills(work[k - 1], &a0.ctl->ovf_count[k - 1], (uint32_t)a0.n_sets, a0.S,
                                       ordered[k - 1], st));
            b.work_in = ordered[k - 1];
        }
        b.work_out = k + 1 < tp.n ? work[k] : nullptr;
        b.cap = T.cap;
        b.hbits = T.hbits;
        int32_t blocks = k == 0 ? blocks0 : T.blocks;
        if (T.slab >= 0) {
            const Slab &sl = slabs[T.slab];
            if (sl.cap != T.cap || !sl.buf)
                return fail(LCD_EDEVICE, "tier %d: table workspace not prepared", k);
            b.gtab = sl.buf;
            b.gtab_stride = sl.stride;
            b.n_slots = sl.slots;
            blocks = T.kind == TIER_WAVE_GLOBAL ? (sl.slots + T.waves - 1) / T.waves : sl.slots;
        } else {
            b.gtab = nullptr;
            b.gtab_stride = 0;
            b.n_slots = 0;
        }
        HIPCHK(launch_sweep(b, blocks, T.waves, st));
        *launches += 1;
    }
    if (ev)
        HIPCHK(hipEventRecord(ev[last], st));
    return LCD_OK;
}

bool params_are_auto(const lcd_params &p) {
    return p.lds_capacity == 0 && p.waves_per_block == 0 && p.blocks_per_cu == 0 && p.spill_mode == 0 &&
           p.team_capacity == 0 && p.team_waves == 0;
}

void apply_tuned(const lcd_graph *g, lcd_params &p) {
    if (!g->tuned || !params_are_auto(p))
        return;
    p.lds_capacity = g->tuned_prm.lds_capacity;
    p.waves_per_block = g->tuned_prm.waves_per_block;
    p.blocks_per_cu = g->tuned_prm.blocks_per_cu;
    p.spill_mode = g->tuned_prm.spill_mode;
    p.team_capacity = g->tuned_prm.team_capacity;
    p.team_waves = g->tuned_prm.team_waves;
}

}  // namespace lcd

struct lcd_result {
    const lcd_graph *g = nullptr;
    int32_t n_sets = 0;
    int32_t S = 0;
    lcd_params prm;
    double *scales = nullptr;
    int32_t *seed_ptr = nullptr;
    int32_t *seed_nodes = nullptr;
    int64_t n_seed_nodes = 0;
    Records rec{};
    int32_t *pool = nullptr;
    int64_t pool_cap = 0;
    Counters *ctl = nullptr;          // one per launch group
    int32_t n_ctl = 0;
    unsigned long long *cursor = nullptr;
    uint32_t *err = nullptr;
    int32_t *work[kMaxTiers - 1] = {nullptr, nullptr, nullptr};
    int32_t *ordered[kMaxTiers - 1] = {nullptr, nullptr, nullptr};   // work, by overflow scale
    std::vector<double> scales_h;
    lcd_sweep_stats stats{};
    int32_t *into = nullptr;          // merge mode: per record, -1 live or the live id merged into
    // use_graph: the captured launch sequence and the buffers it refers to
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // buffer addresses and sizes baked into the captured launches (a freed
    // and reallocated buffer can come back at the same address)
    int64_t cap_key[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};

namespace {


lcd_status prepare_slabs(lcd_graph *g, const TierPlan &tp, hipStream_t st) {
    for (int k = 0; k < tp.n; ++k)
        if (tp.t[k].slab >= 0)
            CHK(ensure_slab(g->slab[tp.t[k].slab], tp.t[k].cap, tp.t[k].slots, st));
    return LCD_OK;
}

lcd_status run_group(lcd_result *r, const TierPlan &tp, int32_t s_begin, int32_t s_end, int32_t gi,
                     hipStream_t st, hipEvent_t *ev) {
    lcd_graph *g = const_cast<lcd_graph *>(r->g);
    SweepArgs a{};
    a.g = graph_dev(g);
    a.scales = r->scales;
    a.alpha_set = nullptr;
    a.S = r->S;
    a.s_begin = s_begin;
    a.s_end = s_end;
    a.seed_ptr = r->seed_ptr;
    a.seed_nodes = r->seed_nodes;
    a.n_sets = r->n_sets;
    a.k_prune = r->prm.k_prune;
    a.max_calls = r->prm.grow_calls > 0 ? (uint32_t)r->prm.grow_calls : 0u;
    a.queue_min = queue_min_of(r->prm);
    a.resume = s_begin > 0 ? 1 : 0;
    a.rec = r->rec;
    a.pool = r->pool;
    a.pool_cap = r->pool_cap;
    a.ctl = r->ctl + gi;
    a.pool_cursor = r->cursor;
    a.err = r->err;
    a.budget_ticks = r->prm.watchdog_ms < 0 ? 0 : g->dev.wall_khz * (int64_t)r->prm.watchdog_ms;
    a.stat = r->cursor + 2;
    return enqueue_tiers(a, tp, 0, tp.n, tp.t[0].blocks, g->slab, r->work, r->ordered, st, ev,
                         &r->stats.launches);
}

void capture_key(const lcd_result *r, int64_t key[8]) {
    const lcd_graph *g = r->g;
    key[0] = (int64_t)(intptr_t)g->slab[0].buf;
    key[1] = g->slab[0].stride * g->slab[0].slots + g->slab[0].cap;
    key[2] = (int64_t)(intptr_t)g->slab[1].buf;
    key[3] = g->slab[1].stride * g->slab[1].slots + g->slab[1].cap;
    key[4] = (int64_t)(intptr_t)r->pool;
    key[5] = r->pool_cap;
    key[6] = 0;
    key[7] = 0;
}

void drop_graph(lcd_result *r) {
    if (r->gexec)
        (void)hipGraphExecDestroy(r->gexec);
    if (r->graph)
        (void)hipGraphDestroy(r->graph);
    r->gexec = nullptr;
    r->graph = nullptr;
}

// Capture the whole persistent sweep (queue and counter reset by fill
// kernels, then every tier) into a hipGraph on a private stream.
lcd_status capture_sweep(lcd_result *r, const TierPlan &tp) {
    drop_graph(r);
    hipStream_t cs = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    lcd_status s = LCD_OK;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        e = launch_zero_bytes(r->ctl, (int64_t)sizeof(Counters) * r->n_ctl, cs);
        if (e == hipSuccess)
            e = launch_zero_bytes(r->cursor, 8 * kCursorWords, cs);
        if (e == hipSuccess)
            s = run_group(r, tp, 0, r->S, 0, cs, nullptr);
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (e == hipSuccess && s == LCD_OK && e2 == hipSuccess) {
            e = hipGraphInstantiate(&r->gexec, graph, nullptr, nullptr, 0);
            if (e == hipSuccess)
                r->graph = graph;
            else
                (void)hipGraphDestroy(graph);
        } else {
            if (graph)
                (void)hipGraphDestroy(graph);
            if (e == hipSuccess)
                e = e2;
        }
    }
    (void)hipStreamDestroy(cs);
    if (s != LCD_OK)
        return s;
    if (e != hipSuccess) {
        r->gexec = nullptr;
        return fail(LCD_EDEVICE, "graph capture: %s", hipGetErrorString(e));
    }
    capture_key(r, r->cap_key);
    return LCD_OK;
}

lcd_status run_sweep(lcd_result *r, hipStream_t st) {
    lcd_graph *g = const_cast<lcd_graph *>(r->g);
    TierPlan tp;
    CHK(plan_tiers(g->dev, g->n, r->prm, tp));
    CHK(prepare_slabs(g, tp, st));
    r->stats = lcd_sweep_stats{};
    r->stats.lds_capacity = tp.t[0].cap;
    r->stats.waves_per_block = tp.t[0].waves;
    r->stats.grid_blocks = tp.t[0].blocks;
    r->stats.tiers = tp.n;
    for (int k = 0; k < tp.n; ++k) {
        r->stats.tier_kind[k] = tp.t[k].kind;
        r->stats.tier_capacity[k] = tp.t[k].cap;
    }
    // ev[0 .. n]: before each tier and after the last; ev[kMaxTiers + 1]:
    // before the work-queue reset
    hipEvent_t ev[kMaxTiers + 2];
    for (auto &e : ev)
        HIPCHK(hipEventCreate(&e));
    hipEvent_t &ev_begin = ev[kMaxTiers + 1];
    hipEvent_t &ev_end = ev[tp.n];
    lcd_status status = LCD_OK;
    for (int attempt = 0; attempt < 8; ++attempt) {
        r->stats.launches = 0;
        const bool use_graph = r->prm.use_graph != 0 && r->prm.mode == LCD_PERSISTENT && r->n_sets > 0;
        if (use_graph) {
            int64_t key[8];
            capture_key(r, key);
            if (!r->gexec || std::memcmp(key, r->cap_key, sizeof(key)) != 0)
                CHK(capture_sweep(r, tp));
        }
        r->stats.launches = 0;
        HIPCHK(hipEventRecord(ev_begin, st));
        const bool timed = r->n_sets > 0 && r->prm.mode != LCD_PER_SCALE_LOOP && !use_graph;
        if (use_graph) {
            // zero fills and every tier, as captured
            HIPCHK(hipGraphLaunch(r->gexec, st));
            r->stats.launches = 2 + tp.n;
            HIPCHK(hipEventRecord(ev_end, st));
        } else {
        // zero the work queues, the pool cursor and the error word
        HIPCHK(launch_zero_bytes(r->ctl, (int64_t)sizeof(Counters) * r->n_ctl, st));
        HIPCHK(launch_zero_bytes(r->cursor, 8 * kCursorWords, st));
        if (r->n_sets > 0) {
            if (r->prm.mode == LCD_PER_SCALE_LOOP) {
                for (int32_t s = 0; s < r->S; ++s) {
                    CHK(run_group(r, tp, s, s + 1, s, st, nullptr));
                }
                HIPCHK(hipEventRecord(ev_end, st));
            } else {
                CHK(run_group(r, tp, 0, r->S, 0, st, ev));
            }
        } else {
            HIPCHK(hipEventRecord(ev_end, st));
        }
        }
        HIPCHK(hipEventSynchronize(ev_end));
        unsigned long long cur[kCursorWords] = {};
        HIPCHK(hipMemcpy(cur, r->cursor, 8 * kCursorWords, hipMemcpyDeviceToHost));
        std::vector<Counters> ctl(r->n_ctl);
        HIPCHK(hipMemcpy(ctl.data(), r->ctl, sizeof(Counters) * r->n_ctl, hipMemcpyDeviceToHost));
        float ms_total = 0.f, ms_main = 0.f, ms_spill = 0.f;
        HIPCHK(hipEventElapsedTime(&ms_total, ev_begin, ev_end));
        for (int k = 0; k < kMaxTiers; ++k)
            r->stats.ms_tier[k] = 0.0;
        if (timed) {
            HIPCHK(hipEventElapsedTime(&ms_main, ev[0], ev[1]));
            if (tp.n > 1)
                HIPCHK(hipEventElapsedTime(&ms_spill, ev[1], ev_end));
            for (int k = 0; k < tp.n; ++k) {
                float x = 0.f;
                HIPCHK(hipEventElapsedTime(&x, ev[k], ev[k + 1]));
                r->stats.ms_tier[k] = x;
            }
        }
        const uint32_t err = (uint32_t)(cur[1] & 0xffffffffu);
        if (err) {
            g->slab[0].dirty = g->slab[1].dirty = true;
            status = fail(err & ERR_CAPACITY ? LCD_ECAPACITY : LCD_EDEVICE,
                          "sweep kernel reported error bits 0x%x%s", err,
                          err & ERR_TIMEOUT ? " (watchdog: a seed set ran past its time budget)" : "");
            break;
        }
        r->stats.ms_total = ms_total;
        r->stats.ms_main = ms_main;
        r->stats.ms_spill = ms_spill;
        int64_t sp = 0, spb = 0;
        for (auto &c : ctl) {
            sp += c.ovf_count[0];
            spb += tp.n >= 3 ? c.ovf_count[tp.n - 2] : 0;
        }
        r->stats.n_spilled = sp;
        r->stats.n_spilled_big = spb;
        r->stats.pool_used = (int64_t)cur[0];
        for (int t = 0; t < kMaxTiers; ++t) {
            const unsigned long long *x = cur + 2 + kStatWords * t;
            r->stats.tier[t].rows_gathered = (int64_t)x[0];
            r->stats.tier[t].row_entries = (int64_t)x[1];
            r->stats.tier[t].entries_created = (int64_t)x[2];
            r->stats.tier[t].members_written = (int64_t)x[3];
            r->stats.tier[t].sets_finished = (int64_t)x[4];
            r->stats.tier[t].entries_scanned = (int64_t)x[5];
            r->stats.tier[t].move_rows = (int64_t)x[6];
            r->stats.tier[t].move_row_entries = (int64_t)x[7];
            r->stats.tier[t].seed_rows = (int64_t)x[8];
            r->stats.tier[t].seed_row_entries = (int64_t)x[9];
            r->stats.tier[t].entries_committed = (int64_t)x[10];
        }
        if ((int64_t)cur[0] <= r->pool_cap)
            break;
        // the pool was too small: grow it and run again
        r->stats.reruns += 1;
        int64_t want = std::max<int64_t>((int64_t)cur[0] + (int64_t)cur[0] / 8 + 1024, 2 * r->pool_cap);
        drop_graph(r);
        dev_free(r->pool);
        r->pool_cap = 0;
        CHK(dev_alloc(&r->pool, (size_t)want));
        r->pool_cap = want;
        if (attempt == 7)
            status = fail(LCD_ECAPACITY, "member pool did not converge");
    }
    for (auto &e : ev)
        (void)hipEventDestroy(e);
    if (status == LCD_OK)
        g->pool_hint = std::max(g->pool_hint, r->stats.pool_used);
    return status;
}

void result_release(lcd_result *r) {
    if (!r)
        return;
    drop_graph(r);
    dev_free(r->scales);
    dev_free(r->seed_ptr);
    dev_free(r->seed_nodes);
    dev_free(r->into);
    dev_free(r->rec.off);
    dev_free(r->rec.cnt);
    dev_free(r->rec.K);
    dev_free(r->rec.V);
    dev_free(r->rec.f);
    dev_free(r->rec.ctr);
    dev_free(r->rec.dadd);
    dev_free(r->rec.drem);
    dev_free(r->pool);
    dev_free(r->ctl);
    dev_free(r->cursor);
    for (auto &w : r->work)
        dev_free(w);
    for (auto &w : r->ordered)
        dev_free(w);
    delete r;
}

}  // namespace

extern "C" {

void lcd_params_default(lcd_params *p) {
    if (!p)
        return;
    std::memset(p, 0, sizeof(*p));
    p->mode = LCD_PERSISTENT;
    p->watchdog_ms = 20000;
}

const char *lcd_last_error(void) { return t_err.c_str(); }

const char *lcd_version(void) { return "lcd-mi355x 0.1 (gfx950)"; }

lcd_status lcd_device_info(int32_t *compute_units, int64_t *lds_per_cu, int64_t *lds_per_block,
                           char *arch, int32_t arch_len) {
    DevInfo d;
    CHK(device_info(d));
    if (compute_units)
        *compute_units = d.cus;
    if (lds_per_cu)
        *lds_per_cu = d.lds_cu;
    if (lds_per_block)
        *lds_per_block = d.lds_block;
    if (arch && arch_len > 0)
        std::snprintf(arch, (size_t)arch_len, "%s", d.arch);
    return LCD_OK;
}

}  // extern "C"

namespace {

// Validate a host CSR and make it resident (the body of lcd_graph_upload).
lcd_status build_graph(int32_t n, int64_t nnz, const std::vector<int32_t> &rp,
                       const std::vector<int32_t> &cl, const uint8_t *wp, hipStream_t st,
                       lcd_graph **out) {
    const bool has_w = wp != nullptr;
    const uint8_t *w = wp;
    std::vector<uint8_t> ww;
    if (has_w)
        ww.assign(wp, wp + nnz);
    // --- validation ---
    if (rp[0] != 0 || rp[n] != nnz)
        return fail(LCD_EINVAL, "row_ptr must start at 0 and end at nnz");
    for (int32_t u = 0; u < n; ++u)
        if (rp[u + 1] < rp[u])
            return fail(LCD_EINVAL, "row_ptr decreases at node %d", u);
    // rows are checked in parallel blocks; the first failing row of the
    // lowest block is reported
    struct RowCheck {
        int32_t row = -1;
        int code = 0;
        int32_t v = 0;
        int64_t maxk = 0, vol = 0;
    };
    auto check_rows = [&](int32_t u0, int32_t u1, RowCheck &rc) {
        for (int32_t u = u0; u < u1; ++u) {
            const int32_t b = rp[u], e = rp[u + 1];
            int64_t k = 0;
            for (int32_t j = b; j < e; ++j) {
                const int32_t v = cl[j];
                int code = 0;
                if (v < 0 || v >= n)
                    code = 1;
                else if (v == u)
                    code = 2;
                else if (j > b && cl[j - 1] >= v)
                    code = 3;
                else if ((w ? (int)ww[j] : 1) < 1)
                    code = 4;
                else {
                    // symmetry: u must appear in row v with the same weight
                    const int32_t *rb = cl.data() + rp[v];
                    const int32_t *re = cl.data() + rp[v + 1];
                    const int32_t *it = std::lower_bound(rb, re, u);
                    if (it == re || *it != u)
                        code = 5;
                    else if (w && ww[it - cl.data()] != ww[j])
                        code = 6;
                }
                if (code) {
                    rc.row = u;
                    rc.code = code;
                    rc.v = v;
                    return;
                }
                k += w ? (int)ww[j] : 1;
            }
            rc.maxk = std::max(rc.maxk, k);
            rc.vol += k;
        }
    };
    const int32_t nthr = (int32_t)std::max<int64_t>(1, std::min<int64_t>(16, (int64_t)n / 65536));
    std::vector<RowCheck> rcs((size_t)nthr);
    {
        std::vector<std::thread> th;
        for (int32_t t = 0; t < nthr; ++t) {
            const int32_t u0 = (int32_t)((int64_t)n * t / nthr), u1 = (int32_t)((int64_t)n * (t + 1) / nthr);
            th.emplace_back(check_rows, u0, u1, std::ref(rcs[(size_t)t]));
        }
        for (auto &x : th)
            x.join();
    }
    int64_t maxk = 0, vol = 0;
    for (const RowCheck &rc : rcs) {
        if (rc.code) {
            const int32_t u = rc.row, v = rc.v;
            switch (rc.code) {
            case 1: return fail(LCD_EINVAL, "neighbour id %d of node %d out of range", v, u);
            case 2: return fail(LCD_EINVAL, "self-loop at node %d", u);
            case 3: return fail(LCD_EINVAL, "row %d is not strictly ascending", u);
            case 4: return fail(LCD_EINVAL, "zero weight on edge %d-%d", u, v);
            case 5: return fail(LCD_EINVAL, "edge %d-%d has no reverse entry", u, v);
            default: return fail(LCD_EINVAL, "edge %d-%d has unequal weights", u, v);
            }
        }
        maxk = std::max(maxk, rc.maxk);
        vol += rc.vol;
    }
    if (maxk >= ((int64_t)1 << 27))
        return fail(LCD_EINVAL, "weighted degree %lld exceeds 2^27", (long long)maxk);
    // --- device copies ---
    lcd_graph *g = new (std::nothrow) lcd_graph();
    if (!g)
        return fail(LCD_ENOMEM, "host allocation failed");
    auto bail = [&](lcd_status s) {
        dev_free(g->row_ptr);
        dev_free(g->col);
        dev_free(g->w);
        dev_free(g->kdeg);
        dev_free(g->logtab);
        delete g;
        return s;
    };
    lcd_status s;
    if ((s = device_info(g->dev)) != LCD_OK)
        return bail(s);
    g->n = n;
    g->nnz = nnz;
    g->maxk = maxk;
    g->volume = vol;
    g->device = g->dev.device;
    g->logtab_n = (int32_t)(2 * maxk + 2);
    if ((s = dev_alloc(&g->row_ptr, (size_t)n + 1)) != LCD_OK ||
        (s = dev_alloc(&g->col, (size_t)nnz)) != LCD_OK ||
        (s = dev_alloc(&g->kdeg, (size_t)std::max(n, 1))) != LCD_OK ||
        (s = dev_alloc(&g->logtab, (size_t)g->logtab_n)) != LCD_OK)
        return bail(s);
    if (w && (s = dev_alloc(&g->w, (size_t)nnz)) != LCD_OK)
        return bail(s);
    hipError_t e = hipSuccess;
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->row_ptr, rp.data(), sizeof(int32_t) * ((size_t)n + 1),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess && nnz)
        e = hipMemcpyAsync(g->col, cl.data(), sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && w && nnz)
        e = hipMemcpyAsync(g->w, ww.data(), (size_t)nnz, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = launch_degrees(g->row_ptr, g->w, g->kdeg, n, st);
    if (e == hipSuccess)
        e = launch_logtab(g->logtab, g->logtab_n, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        return bail(fail(LCD_EDEVICE, "graph upload: %s", hipGetErrorString(e)));
    *out = g;
    return LCD_OK;
}

}  // namespace

extern "C" {

lcd_status lcd_graph_upload(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col,
                            const uint8_t *w, int32_t mem_kind, void *stream, lcd_graph **out) {
    if (!out)
        return fail(LCD_EINVAL, "out is null");
    *out = nullptr;
    if (n < 0 || nnz < 0 || nnz >= ((int64_t)1 << 31))
        return fail(LCD_EINVAL, "n and nnz must be in [0, 2^31)");
    if (mem_kind != LCD_MEM_HOST && mem_kind != LCD_MEM_DEVICE)
        return fail(LCD_EINVAL, "unknown mem_kind %d", mem_kind);
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> rp, cl;
    std::vector<uint8_t> ww;
    CHK(fetch(rp, row_ptr, (size_t)n + 1, mem_kind, st));
    CHK(fetch(cl, col, (size_t)nnz, mem_kind, st));
    if (w)
        CHK(fetch(ww, w, (size_t)nnz, mem_kind, st));
    return build_graph(n, nnz, rp, cl, w ? ww.data() : nullptr, st, out);
}

lcd_status lcd_graph_upload_batch(int32_t n_graphs, const int64_t *node_off, const int64_t *edge_off,
                                  const int32_t *row_ptr, const int32_t *col, const uint8_t *w,
                                  int32_t mem_kind, void *stream, lcd_graph **out) {
    if (!out)
        return fail(LCD_EINVAL, "out is null");
    *out = nullptr;
    if (n_graphs < 1)
        return fail(LCD_EINVAL, "n_graphs must be >= 1");
    if (mem_kind != LCD_MEM_HOST && mem_kind != LCD_MEM_DEVICE)
        return fail(LCD_EINVAL, "unknown mem_kind %d", mem_kind);
    hipStream_t st = (hipStream_t)stream;
    std::vector<int64_t> no, eo;
    CHK(fetch(no, node_off, (size_t)n_graphs + 1, mem_kind, st));
    CHK(fetch(eo, edge_off, (size_t)n_graphs + 1, mem_kind, st));
    if (no[0] != 0 || eo[0] != 0)
        return fail(LCD_EINVAL, "node_off and edge_off must start at 0");
    for (int32_t i = 0; i < n_graphs; ++i)
        if (no[i + 1] < no[i] || eo[i + 1] < eo[i])
            return fail(LCD_EINVAL, "node_off / edge_off decrease at graph %d", i);
    const int64_t N = no[n_graphs], E = eo[n_graphs];
    if (N >= ((int64_t)1 << 31) || E >= ((int64_t)1 << 31))
        return fail(LCD_EINVAL, "total nodes and entries must be below 2^31");
    std::vector<int32_t> lrp, lcl;
    std::vector<uint8_t> lw;
    CHK(fetch(lrp, row_ptr, (size_t)(N + n_graphs), mem_kind, st));
    CHK(fetch(lcl, col, (size_t)E, mem_kind, st));
    if (w)
        CHK(fetch(lw, w, (size_t)E, mem_kind, st));
    // the disjoint union: graph i's nodes at node_off[i] + local id
    std::vector<int32_t> rp((size_t)N + 1), cl((size_t)E);
    for (int32_t i = 0; i < n_graphs; ++i) {
        const int64_t ni = no[i + 1] - no[i], ei = eo[i + 1] - eo[i];
        const int32_t *r = lrp.data() + no[i] + i;
        if (r[0] != 0 || r[ni] != ei)
            return fail(LCD_EINVAL, "graph %d: row_ptr must start at 0 and end at its %lld entries", i,
                        (long long)ei);
        for (int64_t u = 0; u < ni; ++u) {
            if (r[u + 1] < r[u])
                return fail(LCD_EINVAL, "graph %d: row_ptr decreases at node %lld", i, (long long)u);
            rp[no[i] + u] = (int32_t)(eo[i] + r[u]);
        }
        for (int64_t j = eo[i]; j < eo[i + 1]; ++j) {
            const int32_t v = lcl[j];
            if (v < 0 || v >= ni)
                return fail(LCD_EINVAL, "graph %d: neighbour id %d out of range", i, v);
            cl[j] = (int32_t)(no[i] + v);
        }
    }
    rp[N] = (int32_t)E;
    lcd_graph *g = nullptr;
    CHK(build_graph((int32_t)N, E, rp, cl, w ? lw.data() : nullptr, st, &g));
    g->node_off = no;
    g->edge_off = eo;
    *out = g;
    return LCD_OK;
}

lcd_status lcd_graph_batch_info(const lcd_graph *g, int32_t *n_graphs, int64_t *node_off) {
    if (!g)
        return fail(LCD_EINVAL, "null graph");
    const int32_t k = g->node_off.empty() ? 1 : (int32_t)g->node_off.size() - 1;
    if (n_graphs)
        *n_graphs = k;
    if (node_off) {
        if (g->node_off.empty()) {
            node_off[0] = 0;
            node_off[1] = g->n;
        } else {
            std::memcpy(node_off, g->node_off.data(), sizeof(int64_t) * (size_t)(k + 1));
        }
    }
    return LCD_OK;
}

lcd_status lcd_graph_info(const lcd_graph *g, int32_t *n, int64_t *nnz, int64_t *max_degree,
                          int64_t *volume) {
    if (!g)
        return fail(LCD_EINVAL, "null graph");
    if (n)
        *n = g->n;
    if (nnz)
        *nnz = g->nnz;
    if (max_degree)
        *max_degree = g->maxk;
    if (volume)
        *volume = g->volume;
    return LCD_OK;
}

lcd_status lcd_graph_free(lcd_graph *g) {
    if (!g)
        return LCD_OK;
    dev_free(g->row_ptr);
    dev_free(g->col);
    dev_free(g->w);
    dev_free(g->kdeg);
    dev_free(g->logtab);
    dev_free(g->slab[0].buf);
    dev_free(g->slab[1].buf);
    dev_free(g->seed_ws);
    delete g;
    return LCD_OK;
}

lcd_status lcd_sweep(const lcd_graph *g, const double *scales, int32_t n_scales,
                     const int32_t *seed_ptr, const int32_t *seed_nodes, int32_t n_sets,
                     int32_t mem_kind, const lcd_params *params, void *stream, lcd_result **out) {
    if (!out)
        return fail(LCD_EINVAL, "out is null");
    *out = nullptr;
    if (!g)
        return fail(LCD_EINVAL, "null graph");
    if (n_scales < 1)
        return fail(LCD_EINVAL, "n_scales must be >= 1");
    if (n_sets < 0)
        return fail(LCD_EINVAL, "n_sets must be >= 0");
    // the tiers hand a spilled set on as set * n_scales + scale (int32)
    if ((int64_t)n_sets * n_scales >= ((int64_t)1 << 31))
        return fail(LCD_EINVAL, "n_sets x n_scales must stay below 2^31");
    if (mem_kind != LCD_MEM_HOST && mem_kind != LCD_MEM_DEVICE)
        return fail(LCD_EINVAL, "unknown mem_kind %d", mem_kind);
    lcd_params prm;
    lcd_params_default(&prm);
    if (params)
        prm = *params;
    if (prm.mode != LCD_PERSISTENT && prm.mode != LCD_PER_SCALE_LOOP)
        return fail(LCD_EINVAL, "unknown mode %d", prm.mode);
    if (prm.watchdog_ms == 0)
        prm.watchdog_ms = 20000;
    if (prm.grow_calls < 0)
        return fail(LCD_EINVAL, "grow_calls must be >= 0");
    if (prm.output_mode != LCD_OUT_FULL && prm.output_mode != LCD_OUT_DELTA)
        return fail(LCD_EINVAL, "unknown output_mode %d", prm.output_mode);
    apply_tuned(g, prm);
    hipStream_t st = (hipStream_t)stream;
    std::vector<double> sc;
    CHK(fetch(sc, scales, (size_t)n_scales, mem_kind, st));
    for (int32_t s = 0; s < n_scales; ++s) {
        if (!std::isfinite(sc[s]) || sc[s] < 0.0 || sc[s] > 1000.0)
            return fail(LCD_EINVAL, "scale %d must be finite and in [0, 1000]", s);
        if (s > 0 && !(sc[s] < sc[s - 1]))
            return fail(LCD_EINVAL, "scales must be strictly decreasing (finest first)");
    }
    std::vector<int32_t> sp, sn;
    CHK(fetch(sp, seed_ptr, (size_t)n_sets + 1, mem_kind, st));
    if (sp[0] != 0)
        return fail(LCD_EINVAL, "seed_ptr[0] must be 0");
    for (int32_t j = 0; j < n_sets; ++j)
        if (sp[j + 1] <= sp[j])
            return fail(LCD_EINVAL, "seed set %d is empty or seed_ptr decreases", j);
    const int64_t total = sp[n_sets];
    CHK(fetch(sn, seed_nodes, (size_t)total, mem_kind, st));
    {
        std::vector<int32_t> stamp((size_t)std::max(g->n, 1), -1);
        for (int32_t j = 0; j < n_sets; ++j)
            for (int32_t q = sp[j]; q < sp[j + 1]; ++q) {
                const int32_t u = sn[q];
                if (u < 0 || u >= g->n)
                    return fail(LCD_EINVAL, "seed node %d of set %d out of range", u, j);
                if (stamp[u] == j)
                    return fail(LCD_EINVAL, "seed node %d repeated in set %d", u, j);
                stamp[u] = j;
            }
    }
    lcd_result *r = new (std::nothrow) lcd_result();
    if (!r)
        return fail(LCD_ENOMEM, "host allocation failed");
    r->g = g;
    r->n_sets = n_sets;
    r->S = n_scales;
    r->prm = prm;
    r->scales_h = sc;
    r->n_seed_nodes = total;
    const size_t R = (size_t)n_sets * (size_t)n_scales;
    r->n_ctl = prm.mode == LCD_PER_SCALE_LOOP ? n_scales : 1;
    int64_t est = std::max<int64_t>(1 << 16, (int64_t)n_sets * (n_scales / 4 + 2) * 32);
    est = std::max(est, g->pool_hint + g->pool_hint / 16);
    if (prm.pool_hint > 0)
        est = prm.pool_hint;
    lcd_status s = LCD_OK;
    if ((s = dev_alloc(&r->scales, (size_t)n_scales)) != LCD_OK ||
        (s = dev_alloc(&r->seed_ptr, (size_t)n_sets + 1)) != LCD_OK ||
        (s = dev_alloc(&r->seed_nodes, (size_t)total)) != LCD_OK ||
        (s = dev_alloc(&r->rec.off, R)) != LCD_OK || (s = dev_alloc(&r->rec.cnt, R)) != LCD_OK ||
        (s = dev_alloc(&r->rec.K, R)) != LCD_OK || (s = dev_alloc(&r->rec.V, R)) != LCD_OK ||
        (s = dev_alloc(&r->rec.f, R)) != LCD_OK || (s = dev_alloc(&r->rec.ctr, 4 * R)) != LCD_OK ||
        (s = dev_alloc(&r->pool, (size_t)est)) != LCD_OK ||
        (s = dev_alloc(&r->ctl, (size_t)r->n_ctl)) != LCD_OK ||
        (s = dev_alloc(&r->cursor, kCursorWords)) != LCD_OK ||
        (s = dev_alloc(&r->work[0], (size_t)std::max(n_sets, 1))) != LCD_OK ||
        (s = dev_alloc(&r->work[1], (size_t)std::max(n_sets, 1))) != LCD_OK ||
        (s = dev_alloc(&r->work[2], (size_t)std::max(n_sets, 1))) != LCD_OK ||
        (s = dev_alloc(&r->ordered[0], (size_t)std::max(n_sets, 1))) != LCD_OK ||
        (s = dev_alloc(&r->ordered[1], (size_t)std::max(n_sets, 1))) != LCD_OK ||
        (s = dev_alloc(&r->ordered[2], (size_t)std::max(n_sets, 1))) != LCD_OK ||
        (prm.output_mode == LCD_OUT_DELTA &&
         ((s = dev_alloc(&r->rec.dadd, std::max<size_t>(R, 1))) != LCD_OK ||
          (s = dev_alloc(&r->rec.drem, std::max<size_t>(R, 1))) != LCD_OK))) {
        result_release(r);
        return s;
    }
    r->pool_cap = est;
    r->err = (uint32_t *)(r->cursor + 1);
    hipError_t e = hipMemcpyAsync(r->scales, sc.data(), sizeof(double) * n_scales,
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(r->seed_ptr, sp.data(), sizeof(int32_t) * ((size_t)n_sets + 1),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess && total)
        e = hipMemcpyAsync(r->seed_nodes, sn.data(), sizeof(int32_t) * (size_t)total,
                           hipMemcpyHostToDevice, st);
    if (e != hipSuccess) {
        result_release(r);
        return fail(LCD_EDEVICE, "input copy: %s", hipGetErrorString(e));
    }
    s = run_sweep(r, st);
    if (s != LCD_OK) {
        result_release(r);
        return s;
    }
    *out = r;
    return LCD_OK;
}

// rounds of seed selection queued between two reads of the undecided count
constexpr int32_t kSeedBatch = 64;

lcd_status lcd_seeds(const lcd_graph *g, int32_t rule, const int32_t *perm, int32_t mem_kind, void *stream,
                     int32_t *out_seeds, int32_t *n_seeds) {
    if (!g || !out_seeds || !n_seeds)
        return fail(LCD_EINVAL, "null argument");
    if (rule != 1 && rule != 2)
        return fail(LCD_EINVAL, "rule must be 1 or 2");
    if (mem_kind != LCD_MEM_HOST && mem_kind != LCD_MEM_DEVICE)
        return fail(LCD_EINVAL, "unknown mem_kind %d", mem_kind);
    hipStream_t st = (hipStream_t)stream;
    const int32_t n = g->n;
    if (n > 0 && !perm)
        return fail(LCD_EINVAL, "null input array");
    // the permutation is checked on the host: in place when it is host
    // memory, from a copy when it is device memory
    std::vector<int32_t> ph;
    const int32_t *hp = perm;
    if (mem_kind == LCD_MEM_DEVICE) {
        CHK(fetch(ph, perm, (size_t)n, mem_kind, st));
        hp = ph.data();
    }
    {
        std::vector<uint64_t> seen(((size_t)std::max(n, 1) + 63) / 64, 0);
        for (int32_t i = 0; i < n; ++i) {
            const int32_t v = hp[i];
            if (v < 0 || v >= n || (seen[v >> 6] >> (v & 63) & 1u))
                return fail(LCD_EINVAL, "perm is not a permutation of the node ids (entry %d)", i);
            seen[v >> 6] |= (uint64_t)1 << (v & 63);
        }
    }
    *n_seeds = 0;
    if (n == 0)
        return LCD_OK;
    const int nb = (int)(((int64_t)n + 1023) / 1024);
    // one device workspace per graph, allocated on the first call: perm,
    // pos, flag (also the round's one-hop minima), at, block sums, out
    // (int32), state, selection, activity and two-hop marks (uint8), the
    // round counters
    auto al = [](int64_t x) { return (x + 255) / 256 * 256; };
    const int64_t n4 = al(4 * (int64_t)n), n1 = al((int64_t)n);
    const int64_t ws = 5 * n4 + al(4 * ((int64_t)nb + 1)) + 4 * n1 + al(4 * (int64_t)kSeedBatch);
    lcd_graph *gw = const_cast<lcd_graph *>(g);
    if (gw->seed_ws_bytes < ws) {
        dev_free(gw->seed_ws);
        gw->seed_ws_bytes = 0;
        CHK(dev_alloc(&gw->seed_ws, (size_t)ws));
        gw->seed_ws_bytes = ws;
    }
    char *p = gw->seed_ws;
    int32_t *d_perm = (int32_t *)p;
    int32_t *pos = (int32_t *)(p + n4);
    int32_t *flag = (int32_t *)(p + 2 * n4);
    int32_t *at = (int32_t *)(p + 3 * n4);
    int32_t *out = mem_kind == LCD_MEM_HOST ? (int32_t *)(p + 4 * n4) : out_seeds;
    int32_t *bs = (int32_t *)(p + 5 * n4);
    uint8_t *stt = (uint8_t *)(p + 5 * n4 + al(4 * ((int64_t)nb + 1)));
    uint8_t *sel = stt + n1;
    uint8_t *act = sel + n1;
    uint8_t *near = act + n1;
    unsigned *cnt = (unsigned *)(near + n1);
    hipError_t e = hipMemcpyAsync(d_perm, perm, sizeof(int32_t) * (size_t)n,
                                  mem_kind == LCD_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = launch_seed_init(g->row_ptr, d_perm, n, pos, stt, act, st);
    // each round settles at least the first undecided candidate in visiting
    // order, so at most n rounds run; usually a few dozen.  Rounds are queued
    // in batches (4, 8, ... up to kSeedBatch): round k of a batch counts the
    // undecided candidates into cnt[k] and does nothing once the round before
    // counted none, and the host reads the batch's last count only.
    int64_t rounds = 0;
    bool settled = false;
    for (int32_t batch = 4; e == hipSuccess && !settled && rounds <= (int64_t)n;
         batch = std::min(2 * batch, kSeedBatch)) {
        unsigned undecided = 0;
        e = launch_zero_bytes(cnt, 4 * (int64_t)batch, st);
        for (int32_t k = 0; k < batch && e == hipSuccess; ++k)
            e = launch_seed_round(rule, g->row_ptr, g->col, pos, stt, sel, act, near, flag, n,
                                  k > 0 ? cnt + (k - 1) : nullptr, cnt + k, st);
        rounds += batch;
        if (e == hipSuccess)
            e = hipMemcpyAsync(&undecided, cnt + (batch - 1), sizeof(unsigned), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        settled = e == hipSuccess && undecided == 0;
    }
    int32_t total = 0;
    if (e == hipSuccess)
        e = launch_seed_collect(d_perm, stt, n, flag, at, bs, out, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&total, bs + nb, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    // host output: the seeds only, not all n slots
    if (e == hipSuccess && mem_kind == LCD_MEM_HOST && total > 0) {
        e = hipMemcpyAsync(out_seeds, out, sizeof(int32_t) * (size_t)total, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
    }
    if (e != hipSuccess)
        return fail(LCD_EDEVICE, "seed selection: %s", hipGetErrorString(e));
    if (!settled)
        return fail(LCD_EDEVICE, "seed selection did not settle in %lld rounds", (long long)rounds);
    *n_seeds = total;
    return LCD_OK;
}

lcd_status lcd_sweep_batch(const lcd_graph *g, const double *scales, int32_t n_scales,
                           const int32_t *seed_ptr, const int32_t *seed_nodes, const int32_t *seed_graph,
                           int32_t n_sets, int32_t mem_kind, const lcd_params *params, void *stream,
                           lcd_result **out) {
    if (!out)
        return fail(LCD_EINVAL, "out is null");
    *out = nullptr;
    if (!g)
        return fail(LCD_EINVAL, "null graph");
    if (n_sets < 0)
        return fail(LCD_EINVAL, "n_sets must be >= 0");
    if (mem_kind != LCD_MEM_HOST && mem_kind != LCD_MEM_DEVICE)
        return fail(LCD_EINVAL, "unknown mem_kind %d", mem_kind);
    hipStream_t st = (hipStream_t)stream;
    const int32_t k = g->node_off.empty() ? 1 : (int32_t)g->node_off.size() - 1;
    std::vector<int32_t> sp, sn, sg;
    std::vector<double> sc;
    CHK(fetch(sc, scales, (size_t)std::max(n_scales, 0), mem_kind, st));
    CHK(fetch(sp, seed_ptr, (size_t)n_sets + 1, mem_kind, st));
    if (sp[0] != 0)
        return fail(LCD_EINVAL, "seed_ptr[0] must be 0");
    for (int32_t j = 0; j < n_sets; ++j)
        if (sp[j + 1] < sp[j])
            return fail(LCD_EINVAL, "seed_ptr decreases at set %d", j);
    CHK(fetch(sn, seed_nodes, (size_t)sp[n_sets], mem_kind, st));
    if (n_sets > 0 && !seed_graph)
        return fail(LCD_EINVAL, "seed_graph is null");
    CHK(fetch(sg, seed_graph, (size_t)n_sets, mem_kind, st));
    for (int32_t j = 0; j < n_sets; ++j) {
        const int32_t gi = sg[j];
        if (gi < 0 || gi >= k)
            return fail(LCD_EINVAL, "seed set %d names graph %d of %d", j, gi, k);
        const int64_t base = g->node_off.empty() ? 0 : g->node_off[gi];
        const int64_t ni = g->node_off.empty() ? g->n : g->node_off[gi + 1] - base;
        for (int32_t q = sp[j]; q < sp[j + 1]; ++q) {
            if (sn[q] < 0 || sn[q] >= ni)
                return fail(LCD_EINVAL, "seed node %d of set %d outside graph %d", sn[q], j, gi);
            sn[q] = (int32_t)(base + sn[q]);
        }
    }
    return lcd_sweep(g, sc.data(), n_scales, sp.data(), sn.data(), n_sets, LCD_MEM_HOST, params, stream, out);
}

// ---------------------------------------------------------------------------
// Multi-scale loop with the check-and-merge phase (Sec. 3, Algorithm 2 with
// the overlap pre-test of Algorithm 3).  Per scale, rounds until a round
// neither grows nor merges: memberships of the live communities (device
// readout kernels); overlap partner of every live community (device,
// partner_kernel) -> those with a partner skip growth; the others that need
// it make one growth call at the scale (the sweep kernels, one scale, one
// call, from their member lists); memberships again and the partners of the pre-tested
// or changed communities -> pairs; the pairs merge into their lower ids in
// passes of pairwise disjoint pairs.  The bookkeeping between launches
// (member lists, unions of merged pairs, pair passes) is host code.
// ---------------------------------------------------------------------------
lcd_status lcd_sweep_merge(const lcd_graph *g, const double *scales, int32_t n_scales, const int32_t *seed_ptr,
                           const int32_t *seed_nodes, int32_t n_sets, int32_t eta_num, int32_t eta_den,
                           int32_t mem_kind, const lcd_params *params, void *stream, lcd_result **out) {
    if (!out)
        return fail(LCD_EINVAL, "out is null");
    *out = nullptr;
    if (!g)
        return fail(LCD_EINVAL, "null graph");
    if (n_scales < 1 || n_sets < 0)
        return fail(LCD_EINVAL, "n_scales must be >= 1 and n_sets >= 0");
    if (eta_num < 1 || eta_den < 1)
        return fail(LCD_EINVAL, "eta_num and eta_den must be positive");
    if (mem_kind != LCD_MEM_HOST && mem_kind != LCD_MEM_DEVICE)
        return fail(LCD_EINVAL, "unknown mem_kind %d", mem_kind);
    hipStream_t st = (hipStream_t)stream;
    const int32_t n = g->n, ns = n_sets, S = n_scales;
    std::vector<double> sc;
    std::vector<int32_t> sp, sn;
    CHK(fetch(sc, scales, (size_t)S, mem_kind, st));
    for (int32_t s = 0; s < S; ++s) {
        if (!std::isfinite(sc[s]) || sc[s] < 0.0 || sc[s] > 1000.0)
            return fail(LCD_EINVAL, "scale %d must be finite and in [0, 1000]", s);
        if (s > 0 && !(sc[s] < sc[s - 1]))
            return fail(LCD_EINVAL, "scales must be strictly decreasing (finest first)");
    }
    CHK(fetch(sp, seed_ptr, (size_t)ns + 1, mem_kind, st));
    if (sp[0] != 0)
        return fail(LCD_EINVAL, "seed_ptr[0] must be 0");
    for (int32_t j = 0; j < ns; ++j)
        if (sp[j + 1] <= sp[j])
            return fail(LCD_EINVAL, "seed set %d is empty or seed_ptr decreases", j);
    CHK(fetch(sn, seed_nodes, (size_t)sp[ns], mem_kind, st));
    lcd_params prm;
    lcd_params_default(&prm);
    if (params)
        prm = *params;
    prm.mode = LCD_PERSISTENT;
    prm.use_graph = 0;
    prm.grow_calls = 1;   // one growth call per community and round
    // state of every community (host)
    std::vector<std::vector<int32_t>> lists((size_t)ns);
    {
        std::vector<int32_t> stamp((size_t)std::max(n, 1), -1);
        for (int32_t j = 0; j < ns; ++j) {
            for (int32_t q = sp[j]; q < sp[j + 1]; ++q) {
                const int32_t u = sn[q];
                if (u < 0 || u >= n)
                    return fail(LCD_EINVAL, "seed node %d of set %d out of range", u, j);
                if (stamp[u] == j)
                    return fail(LCD_EINVAL, "seed node %d repeated in set %d", u, j);
                stamp[u] = j;
            }
            lists[j].assign(sn.begin() + sp[j], sn.begin() + sp[j + 1]);
            std::sort(lists[j].begin(), lists[j].end());
        }
    }
    std::vector<uint8_t> alive((size_t)ns, 1), need((size_t)ns), flag((size_t)ns), changed((size_t)ns);
    std::vector<int32_t> into((size_t)ns, -1);
    std::vector<int64_t> K((size_t)ns, 0), V((size_t)ns, 0);
    std::vector<uint64_t> acc((size_t)ns * 4);
    const size_t R = (size_t)ns * S;
    std::vector<int64_t> h_off(R), h_K(R), h_V(R);
    std::vector<int32_t> h_cnt(R), h_into(R);
    std::vector<double> h_f(R);
    std::vector<uint64_t> h_ctr(4 * R);
    std::vector<int32_t> pool;
    // device scratch
    const int nbk = (int)(((int64_t)n + 1 + 1023) / 1024) + 1;
    int32_t *d_ptr = nullptr, *d_mem = nullptr, *d_node_ptr = nullptr, *d_node_sets = nullptr, *d_cnt = nullptr,
            *d_bs = nullptr, *d_list = nullptr, *d_partner = nullptr, *d_cnt_all = nullptr;
    unsigned *d_next = nullptr;
    int64_t mem_cap = 0;
    const int32_t slots = (int32_t)std::max<int64_t>(
        1, std::min<int64_t>(4 * (int64_t)g->dev.cus, ((int64_t)1 << 30) / (4 * (int64_t)std::max(ns, 1))));
    auto release = [&]() {
        dev_free(d_ptr);
        dev_free(d_mem);
        dev_free(d_node_ptr);
        dev_free(d_node_sets);
        dev_free(d_cnt);
        dev_free(d_bs);
        dev_free(d_list);
        dev_free(d_partner);
        dev_free(d_cnt_all);
        dev_free(d_next);
    };
    lcd_status status = LCD_OK;
#define MCHK(expr)                         \
    do {                                   \
        lcd_status s_ = (expr);            \
        if (s_ != LCD_OK) {                \
            release();                     \
            return s_;                     \
        }                                  \
    } while (0)
#define MHIP(expr)                                                                             \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) {                                                                \
            release();                                                                         \
            return fail(LCD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));          \
        }                                                                                      \
    } while (0)
    MCHK(dev_alloc(&d_ptr, (size_t)ns + 1));
    MCHK(dev_alloc(&d_node_ptr, (size_t)n + 1));
    MCHK(dev_alloc(&d_cnt, (size_t)n + 1));
    MCHK(dev_alloc(&d_bs, (size_t)nbk + 1));
    MCHK(dev_alloc(&d_list, (size_t)std::max(ns, 1)));
    MCHK(dev_alloc(&d_partner, (size_t)std::max(ns, 1)));
    MCHK(dev_alloc(&d_cnt_all, (size_t)slots * (size_t)std::max(ns, 1)));
    MCHK(dev_alloc(&d_next, 1));
    MHIP(launch_zero_bytes(d_cnt_all, 4 * (int64_t)slots * std::max(ns, 1), st));
    std::vector<int32_t> h_ptr((size_t)ns + 1), h_list, h_partner;
    std::vector<int32_t> flat;
    // upload the live member lists and build the memberships node -> ids
    auto memberships = [&]() -> lcd_status {
        int64_t total = 0;
        for (int32_t j = 0; j < ns; ++j)
            total += alive[j] ? (int64_t)lists[j].size() : 0;
        if (total > INT32_MAX)
            return fail(LCD_ECAPACITY, "live communities hold %lld members in all; at most 2^31 - 1",
                        (long long)total);
        h_ptr[0] = 0;
        for (int32_t j = 0; j < ns; ++j)
            h_ptr[j + 1] = h_ptr[j] + (alive[j] ? (int32_t)lists[j].size() : 0);
        flat.resize((size_t)std::max<int64_t>(total, 1));
        for (int32_t j = 0; j < ns; ++j)
            if (alive[j])
                std::copy(lists[j].begin(), lists[j].end(), flat.begin() + h_ptr[j]);
        if (total > mem_cap) {
            dev_free(d_mem);
            dev_free(d_node_sets);
            mem_cap = std::max<int64_t>(total, 2 * mem_cap);
            CHK(dev_alloc(&d_mem, (size_t)mem_cap));
            CHK(dev_alloc(&d_node_sets, (size_t)mem_cap));
        }
        HIPCHK(hipMemcpyAsync(d_ptr, h_ptr.data(), sizeof(int32_t) * ((size_t)ns + 1), hipMemcpyHostToDevice, st));
        if (total)
            HIPCHK(hipMemcpyAsync(d_mem, flat.data(), sizeof(int32_t) * (size_t)total, hipMemcpyHostToDevice, st));
        HIPCHK(launch_overlap(d_ptr, d_mem, total, ns, n, d_node_ptr, d_node_sets, d_cnt, d_bs, st));
        return LCD_OK;
    };
    // partners of the listed communities (host ids in h_list)
    auto partners = [&]() -> lcd_status {
        h_partner.assign(h_list.size(), -1);
        if (h_list.empty()) {
            // the host lists are rewritten next: the uploads must have landed
            HIPCHK(hipStreamSynchronize(st));
            return LCD_OK;
        }
        HIPCHK(hipMemcpyAsync(d_list, h_list.data(), sizeof(int32_t) * h_list.size(), hipMemcpyHostToDevice, st));
        HIPCHK(launch_partner(d_ptr, d_mem, d_node_ptr, d_node_sets, d_list, (int32_t)h_list.size(), ns, eta_num,
                              eta_den, d_cnt_all, slots, d_next, d_partner, st));
        HIPCHK(hipMemcpyAsync(h_partner.data(), d_partner, sizeof(int32_t) * h_list.size(), hipMemcpyDeviceToHost,
                              st));
        HIPCHK(hipStreamSynchronize(st));
        return LCD_OK;
    };
    const bool trace = std::getenv("LCD_TRACE") != nullptr;
    for (int32_t s = 0; s < S && status == LCD_OK; ++s) {
        const double alpha = sc[s];
        std::fill(acc.begin(), acc.end(), 0);
        for (int32_t j = 0; j < ns; ++j)
            need[j] = alive[j];
        for (int64_t round = 0;; ++round) {
            if (round > 100000) {
                release();
                return fail(LCD_EDEVICE, "scale %d did not settle", s);
            }
            // pre-test
            MCHK(memberships());
            h_list.clear();
            for (int32_t j = 0; j < ns; ++j)
                if (alive[j])
                    h_list.push_back(j);
            MCHK(partners());
            std::fill(flag.begin(), flag.end(), 0);
            for (size_t t = 0; t < h_list.size(); ++t)
                flag[h_list[t]] = h_partner[t] >= 0;
            // growth of the others that need it
            std::vector<int32_t> grow_ids;
            for (int32_t j = 0; j < ns; ++j) {
                changed[j] = 0;
                if (alive[j] && need[j] && !flag[j])
                    grow_ids.push_back(j);
            }
            bool grew = false;
            if (!grow_ids.empty()) {
                std::vector<int32_t> gp(grow_ids.size() + 1, 0), gn;
                for (size_t t = 0; t < grow_ids.size(); ++t) {
                    const auto &L = lists[grow_ids[t]];
                    gn.insert(gn.end(), L.begin(), L.end());
                    gp[t + 1] = (int32_t)gn.size();
                }
                lcd_result *res = nullptr;
                MCHK(lcd_sweep(g, &alpha, 1, gp.data(), gn.data(), (int32_t)grow_ids.size(), LCD_MEM_HOST, &prm,
                               stream, &res));
                // the round's results in bulk: one scale readout and one
                // counter readout (a few copies, whatever the number of sets)
                const int32_t ng = (int32_t)grow_ids.size();
                std::vector<int32_t> rcp((size_t)ng + 1);
                std::vector<int64_t> rk((size_t)ng), rv((size_t)ng);
                std::vector<uint64_t> rct(4 * (size_t)ng), tot4(4);
                int64_t needm = 0;
                lcd_status s1 = lcd_result_sizes(res, 0, &needm);
                std::vector<int32_t> rm((size_t)std::max<int64_t>(needm, 1));
                if (s1 == LCD_OK)
                    s1 = lcd_result_membership(res, 0, rcp.data(), rm.data(), rk.data(), rv.data(), nullptr,
                                               LCD_MEM_HOST, stream);
                if (s1 == LCD_OK)
                    s1 = lcd_result_counters(res, tot4.data(), rct.data(), LCD_MEM_HOST, stream);
                lcd_result_free(res);
                MCHK(s1);
                std::vector<int64_t> ro((size_t)ng);
                std::vector<int32_t> rc((size_t)ng);
                for (int32_t t = 0; t < ng; ++t) {
                    ro[t] = rcp[t];
                    rc[t] = rcp[t + 1] - rcp[t];
                }
                for (int32_t t = 0; t < ng; ++t) {
                    const int32_t j = grow_ids[t];
                    const int32_t *a = rm.data() + ro[t];
                    const bool same = (size_t)rc[t] == lists[j].size() && std::equal(a, a + rc[t], lists[j].begin());
                    if (!same) {
                        lists[j].assign(a, a + rc[t]);
                        changed[j] = 1;
                        grew = true;
                    }
                    K[j] = rk[t];
                    V[j] = rv[t];
                    for (int q = 0; q < 4; ++q)
                        acc[4 * j + q] += rct[4 * t + q];
                    need[j] = changed[j];   // a call that changed it calls for another
                }
            }
            // check
            MCHK(memberships());
            h_list.clear();
            for (int32_t j = 0; j < ns; ++j)
                if (alive[j] && (flag[j] || changed[j]))
                    h_list.push_back(j);
            MCHK(partners());
            std::vector<std::pair<int32_t, int32_t>> pairs;
            for (size_t t = 0; t < h_list.size(); ++t)
                if (h_partner[t] >= 0)
                    pairs.emplace_back(std::min(h_list[t], h_partner[t]), std::max(h_list[t], h_partner[t]));
            const bool merged = !pairs.empty();
            // merge passes of pairwise disjoint pairs, in ascending order
            std::vector<uint8_t> used((size_t)ns, 0);
            while (!pairs.empty()) {
                std::sort(pairs.begin(), pairs.end());
                pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
                std::vector<std::pair<int32_t, int32_t>> rest, ren;
                for (auto &p : pairs)
                    used[p.first] = used[p.second] = 0;
                for (auto &p : pairs) {
                    const int32_t a = p.first, b = p.second;
                    if (!used[a] && !used[b]) {
                        used[a] = used[b] = 1;
                        std::vector<int32_t> u;
                        u.reserve(lists[a].size() + lists[b].size());
                        std::set_union(lists[a].begin(), lists[a].end(), lists[b].begin(), lists[b].end(),
                                       std::back_inserter(u));
                        lists[a].swap(u);
                        lists[b].clear();
                        alive[b] = 0;
                        into[b] = a;
                        need[a] = 1;
                        ren.emplace_back(b, a);
                    } else {
                        rest.push_back(p);
                    }
                }
                pairs.clear();
                for (auto p : rest) {
                    for (auto &r : ren) {
                        if (p.first == r.first)
                            p.first = r.second;
                        if (p.second == r.first)
                            p.second = r.second;
                    }
                    if (p.first != p.second)
                        pairs.emplace_back(std::min(p.first, p.second), std::max(p.first, p.second));
                }
            }
            if (trace) {
                int32_t nl = 0, nf = 0;
                for (int32_t j = 0; j < ns; ++j) {
                    nl += alive[j];
                    nf += alive[j] && flag[j];
                }
                std::fprintf(stderr, "[lcd merge] scale %d round %lld: live %d, pre-tested %d, grown %zu%s, %s\n",
                             s, (long long)round, nl, nf, grow_ids.size(), grew ? " (changed)" : "",
                             merged ? "merged" : "no merge");
            }
            if (!grew && !merged)
                break;
        }
        for (int32_t j = 0; j < ns; ++j) {
            const size_t r = (size_t)j * S + s;
            int32_t to = j;
            while (!alive[to])
                to = into[to];
            h_into[r] = alive[j] ? -1 : to;
            h_off[r] = (int64_t)pool.size();
            for (int q = 0; q < 4; ++q)
                h_ctr[4 * r + q] = acc[4 * j + q];
            if (alive[j]) {
                h_cnt[r] = (int32_t)lists[j].size();
                h_K[r] = K[j];
                h_V[r] = V[j];
                h_f[r] = K[j] == 0 ? 0.0 : (double)K[j] / pow((double)V[j], alpha);
                pool.insert(pool.end(), lists[j].begin(), lists[j].end());
            } else {
                h_cnt[r] = 0;
                h_K[r] = h_V[r] = 0;
                h_f[r] = 0.0;
            }
        }
    }
    release();
#undef MCHK
#undef MHIP
    // the result object: records and member pool on the device
    lcd_result *r = new (std::nothrow) lcd_result();
    if (!r)
        return fail(LCD_ENOMEM, "host allocation failed");
    r->g = g;
    r->n_sets = ns;
    r->S = S;
    r->prm = prm;
    r->scales_h = sc;
    lcd_status s2 = LCD_OK;
    if ((s2 = dev_alloc(&r->scales, (size_t)S)) != LCD_OK || (s2 = dev_alloc(&r->rec.off, R)) != LCD_OK ||
        (s2 = dev_alloc(&r->rec.cnt, R)) != LCD_OK || (s2 = dev_alloc(&r->rec.K, R)) != LCD_OK ||
        (s2 = dev_alloc(&r->rec.V, R)) != LCD_OK || (s2 = dev_alloc(&r->rec.f, R)) != LCD_OK ||
        (s2 = dev_alloc(&r->rec.ctr, 4 * R)) != LCD_OK || (s2 = dev_alloc(&r->into, R)) != LCD_OK ||
        (s2 = dev_alloc(&r->pool, std::max<size_t>(pool.size(), 1))) != LCD_OK ||
        (s2 = dev_alloc(&r->cursor, kCursorWords)) != LCD_OK) {
        result_release(r);
        return s2;
    }
    r->pool_cap = (int64_t)std::max<size_t>(pool.size(), 1);
    r->err = (uint32_t *)(r->cursor + 1);
    hipError_t e = hipMemcpy(r->scales, sc.data(), sizeof(double) * S, hipMemcpyHostToDevice);
    if (e == hipSuccess && R)
        e = hipMemcpy(r->rec.off, h_off.data(), sizeof(int64_t) * R, hipMemcpyHostToDevice);
    if (e == hipSuccess && R)
        e = hipMemcpy(r->rec.cnt, h_cnt.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice);
    if (e == hipSuccess && R)
        e = hipMemcpy(r->rec.K, h_K.data(), sizeof(int64_t) * R, hipMemcpyHostToDevice);
    if (e == hipSuccess && R)
        e = hipMemcpy(r->rec.V, h_V.data(), sizeof(int64_t) * R, hipMemcpyHostToDevice);
    if (e == hipSuccess && R)
        e = hipMemcpy(r->rec.f, h_f.data(), sizeof(double) * R, hipMemcpyHostToDevice);
    if (e == hipSuccess && R)
        e = hipMemcpy(r->rec.ctr, h_ctr.data(), sizeof(uint64_t) * 4 * R, hipMemcpyHostToDevice);
    if (e == hipSuccess && R)
        e = hipMemcpy(r->into, h_into.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice);
    if (e == hipSuccess && !pool.empty())
        e = hipMemcpy(r->pool, pool.data(), sizeof(int32_t) * pool.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        result_release(r);
        return fail(LCD_EDEVICE, "merge result upload: %s", hipGetErrorString(e));
    }
    r->stats.pool_used = (int64_t)pool.size();
    *out = r;
    return LCD_OK;
}

lcd_status lcd_result_merged_into(const lcd_result *r, int32_t scale_idx, int32_t *into) {
    if (!r || !into)
        return fail(LCD_EINVAL, "null argument");
    if (scale_idx < 0 || scale_idx >= r->S)
        return fail(LCD_EINVAL, "scale index out of range");
    if (!r->into) {
        for (int32_t j = 0; j < r->n_sets; ++j)
            into[j] = -1;
        return LCD_OK;
    }
    std::vector<int32_t> all((size_t)r->n_sets * r->S);
    if (!all.empty())
        HIPCHK(hipMemcpy(all.data(), r->into, sizeof(int32_t) * all.size(), hipMemcpyDeviceToHost));
    for (int32_t j = 0; j < r->n_sets; ++j)
        into[j] = all[(size_t)j * r->S + scale_idx];
    return LCD_OK;
}

lcd_status lcd_tune(lcd_graph *g, const double *scales, int32_t n_scales, const int32_t *seed_ptr,
                    const int32_t *seed_nodes, int32_t n_sets, int32_t mem_kind, const lcd_params *base,
                    void *stream, lcd_tune_report *report) {
    if (!g)
        return fail(LCD_EINVAL, "null graph");
    if (n_sets < 1 || n_scales < 1)
        return fail(LCD_EINVAL, "tuning needs at least one seed set and one scale");
    if (mem_kind != LCD_MEM_HOST && mem_kind != LCD_MEM_DEVICE)
        return fail(LCD_EINVAL, "unknown mem_kind %d", mem_kind);
    hipStream_t st = (hipStream_t)stream;
    std::vector<double> sc;
    std::vector<int32_t> sp, sn;
    CHK(fetch(sc, scales, (size_t)n_scales, mem_kind, st));
    CHK(fetch(sp, seed_ptr, (size_t)n_sets + 1, mem_kind, st));
    if (sp[0] != 0 || sp[n_sets] < sp[0])
        return fail(LCD_EINVAL, "malformed seed_ptr");
    CHK(fetch(sn, seed_nodes, (size_t)sp[n_sets], mem_kind, st));
    // a deterministic sample: every stride-th seed set, at most ~16k sets
    const int32_t stride = std::max<int32_t>(1, n_sets / 16384);
    std::vector<int32_t> sp2{0}, sn2;
    for (int32_t j = 0; j < n_sets; j += stride) {
        if (sp[j + 1] < sp[j])
            return fail(LCD_EINVAL, "seed_ptr decreases at set %d", j);
        sn2.insert(sn2.end(), sn.begin() + sp[j], sn.begin() + sp[j + 1]);
        sp2.push_back((int32_t)sn2.size());
    }
    const int32_t ns2 = (int32_t)sp2.size() - 1;
    lcd_params b;
    lcd_params_default(&b);
    if (base)
        b = *base;
    b.mode = LCD_PERSISTENT;
    // candidate sizings: {tier-0 table, spill mode, workgroup LDS table, waves per community}
    static const int32_t cand[][4] = {
        {256, 0, 1024, 2}, {256, 0, 1024, 4}, {512, 0, 1024, 2}, {512, 0, 1024, 4},
        {512, 0, 2048, 4}, {1024, 0, 2048, 4}, {256, 0, 768, 2},  {256, 0, 768, 4},
        {512, 0, 768, 2},  {512, 0, 768, 4},  {256, 2, 0, 8},     {512, 2, 0, 8},
        {512, 1, 0, 0},    {1024, 1, 0, 0},
    };
    const int nc = (int)(sizeof(cand) / sizeof(cand[0]));
    lcd_tune_report rep{};
    rep.sample_stride = stride;
    auto time_one = [&](const lcd_params &q, const std::vector<int32_t> &p_, const std::vector<int32_t> &n_,
                        int32_t ns, int reps, double *ms) -> lcd_status {
        double best = 1e300;
        for (int r = 0; r < reps; ++r) {
            lcd_result *res = nullptr;
            CHK(lcd_sweep(g, sc.data(), n_scales, p_.data(), n_.data(), ns, LCD_MEM_HOST, &q, stream, &res));
            best = std::min(best, res->stats.ms_total);
            lcd_result_free(res);
        }
        *ms = best;
        return LCD_OK;
    };
    int bestc = -1;
    for (int c = 0; c < nc && c < 16; ++c) {
        lcd_params q = b;
        q.lds_capacity = cand[c][0];
        q.spill_mode = cand[c][1];
        q.team_capacity = cand[c][2];
        q.team_waves = cand[c][3];
        q.waves_per_block = 0;
        q.blocks_per_cu = 0;
        double ms = 0.0;
        CHK(time_one(q, sp2, sn2, ns2, 2, &ms));
        rep.tried[rep.n_tried] = q;
        rep.ms[rep.n_tried] = ms;
        rep.n_tried += 1;
        if (bestc < 0 || ms < rep.ms[bestc])
            bestc = c;
    }
    // a sampled timing can rank close candidates differently from the full
    // sweep: when the full sweep is short, re-time the leaders on every set
    if (stride > 1 && rep.ms[bestc] * stride < 5000.0) {
        std::vector<int> order(rep.n_tried);
        for (int i = 0; i < rep.n_tried; ++i)
            order[i] = i;
        std::sort(order.begin(), order.end(), [&](int x, int y) { return rep.ms[x] < rep.ms[y]; });
        double best_full = 1e300;
        for (int i = 0; i < std::min(3, rep.n_tried); ++i) {
            double ms = 0.0;
            CHK(time_one(rep.tried[order[i]], sp, sn, n_sets, 1, &ms));
            if (ms < best_full) {
                best_full = ms;
                bestc = order[i];
            }
        }
        rep.full_checked = 1;
    }
    rep.best = rep.tried[bestc];
    rep.ms_best = rep.ms[bestc];
    g->tuned_prm = rep.best;
    g->tuned = true;
    if (report)
        *report = rep;
    return LCD_OK;
}

lcd_status lcd_graph_untune(lcd_graph *g) {
    if (!g)
        return fail(LCD_EINVAL, "null graph");
    g->tuned = false;
    return LCD_OK;
}

lcd_status lcd_result_shape(const lcd_result *r, int32_t *n_sets, int32_t *n_scales) {
    if (!r)
        return fail(LCD_EINVAL, "null result");
    if (n_sets)
        *n_sets = r->n_sets;
    if (n_scales)
        *n_scales = r->S;
    return LCD_OK;
}

}  // extern "C"

namespace {

// Offsets of one scale's member lists into cp (device, n_sets + 1 entries)
// and their exact total.  The int32 offsets wrap when the total passes
// 2^31 - 1, so callers that use them must check the total first.
lcd_status scale_offsets(const lcd_result *r, int32_t scale_idx, int32_t *cp, hipStream_t st,
                         int64_t *total) {
    long long *d_tot = nullptr;
    CHK(dev_alloc(&d_tot, 1));
    long long tot = 0;
    hipError_t e = launch_scale_scan(r->rec, r->S, scale_idx, r->n_sets, cp, d_tot, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&tot, d_tot, sizeof(long long), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    dev_free(d_tot);
    if (e != hipSuccess)
        return fail(LCD_EDEVICE, "scale offsets: %s", hipGetErrorString(e));
    *total = (int64_t)tot;
    return LCD_OK;
}

lcd_status check_int32_total(int64_t total, int32_t scale_idx) {
    if (total > (int64_t)INT32_MAX)
        return fail(LCD_ECAPACITY, "scale %d lists %lld members; int32 offsets address at most 2^31 - 1",
                    scale_idx, (long long)total);
    return LCD_OK;
}

// Sorted member lists of scale s at the offsets out_ptr (device) for the
// listed sets (nullptr: every set, n = n_sets).  Full output copies them
// from the pool (every set only); delta output rebuilds them on the device
// from each set's records.
lcd_status scale_members(const lcd_result *r, int32_t s, const int32_t *sets, int32_t n, const int32_t *out_ptr,
                         int32_t *members, hipStream_t st) {
    if (!r->rec.drem) {
        if (sets)
            return fail(LCD_ESTATE, "internal: listed sets need delta output");
        const hipError_t e = launch_scale_gather(r->rec, r->pool, r->scales, r->S, s, r->n_sets, out_ptr, members,
                                                 nullptr, nullptr, nullptr, st);
        if (e != hipSuccess)
            return fail(LCD_EDEVICE, "member readout: %s", hipGetErrorString(e));
        return LCD_OK;
    }
    int64_t *ev = nullptr, *ev_off = nullptr;
    uint32_t *err = nullptr;
    int32_t *scr = nullptr;
    int64_t total = 0;
    uint32_t h_err = 0;
    lcd_status x = LCD_OK;
    hipError_t e = hipSuccess;
    if ((x = dev_alloc(&ev, (size_t)std::max(n, 1))) != LCD_OK || (x = dev_alloc(&ev_off, (size_t)n + 1)) != LCD_OK ||
        (x = dev_alloc(&err, 1)) != LCD_OK)
        goto done;
    e = launch_zero_bytes(err, 4, st);
    if (e == hipSuccess)
        e = launch_delta_events(r->rec, r->S, s, sets, n, ev, ev_off, err, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&total, ev_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        x = fail(LCD_EDEVICE, "delta readout: %s", hipGetErrorString(e));
        goto done;
    }
    if ((x = dev_alloc(&scr, (size_t)std::max<int64_t>(total, 1))) != LCD_OK)
        goto done;
    e = launch_delta_rebuild(r->rec, r->pool, r->S, s, sets, n, ev_off, scr, out_ptr, members, err, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&h_err, err, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        x = fail(LCD_EDEVICE, "delta readout: %s", hipGetErrorString(e));
    else if (h_err)
        x = fail(LCD_EDEVICE, "delta readout of scale %d: %s", s,
                 h_err & 1u ? "a set has no full member list before this scale"
                            : "a rebuilt list disagrees with its recorded size");
done:
    dev_free(ev);
    dev_free(ev_off);
    dev_free(err);
    dev_free(scr);
    return x;
}

}  // namespace

extern "C" {

lcd_status lcd_result_sizes(const lcd_result *r, int32_t scale_idx, int64_t *total_members) {
    if (!r || !total_members)
        return fail(LCD_EINVAL, "null argument");
    if (scale_idx < 0 || scale_idx >= r->S)
        return fail(LCD_EINVAL, "scale index %d out of range", scale_idx);
    int32_t *cp = nullptr;
    CHK(dev_alloc(&cp, (size_t)r->n_sets + 1));
    int64_t tot = 0;
    const lcd_status s = scale_offsets(r, scale_idx, cp, nullptr, &tot);
    dev_free(cp);
    CHK(s);
    *total_members = tot;
    return LCD_OK;
}

lcd_status lcd_result_membership(const lcd_result *r, int32_t scale_idx, int32_t *comm_ptr,
                                 int32_t *members, int64_t *k_in, int64_t *vol, double *f,
                                 int32_t mem_kind, void *stream) {
    if (!r)
        return fail(LCD_EINVAL, "null result");
    if (scale_idx < 0 || scale_idx >= r->S)
        return fail(LCD_EINVAL, "scale index %d out of range", scale_idx);
    if (mem_kind != LCD_MEM_HOST && mem_kind != LCD_MEM_DEVICE)
        return fail(LCD_EINVAL, "unknown mem_kind %d", mem_kind);
    hipStream_t st = (hipStream_t)stream;
    const size_t ns = (size_t)r->n_sets;
    const bool host = mem_kind == LCD_MEM_HOST;
    int32_t *cp = comm_ptr;
    int32_t *tmp_cp = nullptr, *tmp_m = nullptr;
    int64_t *tmp_k = nullptr, *tmp_v = nullptr;
    double *tmp_f = nullptr;
    if (host || !comm_ptr) {
        CHK(dev_alloc(&tmp_cp, ns + 1));
        cp = tmp_cp;
    }
    int64_t tot = 0;
    lcd_status s = scale_offsets(r, scale_idx, cp, st, &tot);
    if (s == LCD_OK)
        s = check_int32_total(tot, scale_idx);
    if (s != LCD_OK) {
        dev_free(tmp_cp);
        return s;
    }
    int32_t *m = members;
    int64_t *kk = k_in, *vv = vol;
    double *ff = f;
    if (host) {
        if (members && (s = dev_alloc(&tmp_m, (size_t)tot)) != LCD_OK)
            goto done;
        if (k_in && (s = dev_alloc(&tmp_k, ns)) != LCD_OK)
            goto done;
        if (vol && (s = dev_alloc(&tmp_v, ns)) != LCD_OK)
            goto done;
        if (f && (s = dev_alloc(&tmp_f, ns)) != LCD_OK)
            goto done;
        m = members ? tmp_m : nullptr;
        kk = k_in ? tmp_k : nullptr;
        vv = vol ? tmp_v : nullptr;
        ff = f ? tmp_f : nullptr;
    }
    if (m && r->rec.drem && (s = scale_members(r, scale_idx, nullptr, r->n_sets, cp, m, st)) != LCD_OK)
        goto done;
    {
        hipError_t e = launch_scale_gather(r->rec, r->pool, r->scales, r->S, scale_idx, r->n_sets, cp,
                                           r->rec.drem ? nullptr : m, kk, vv, ff, st);
        if (e == hipSuccess && host) {
            if (comm_ptr)
                e = hipMemcpyAsync(comm_ptr, cp, sizeof(int32_t) * (ns + 1), hipMemcpyDeviceToHost, st);
            if (e == hipSuccess && members && tot)
                e = hipMemcpyAsync(members, m, sizeof(int32_t) * (size_t)tot, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess && k_in && ns)
                e = hipMemcpyAsync(k_in, kk, sizeof(int64_t) * ns, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess && vol && ns)
                e = hipMemcpyAsync(vol, vv, sizeof(int64_t) * ns, hipMemcpyDeviceToHost, st);
            if (e == hipSuccess && f && ns)
                e = hipMemcpyAsync(f, ff, sizeof(double) * ns, hipMemcpyDeviceToHost, st);
        }
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            s = fail(LCD_EDEVICE, "membership: %s", hipGetErrorString(e));
    }
done:
    dev_free(tmp_cp);
    dev_free(tmp_m);
    dev_free(tmp_k);
    dev_free(tmp_v);
    dev_free(tmp_f);
    return s;
}

lcd_status lcd_result_overlap(const lcd_result *r, int32_t scale_idx, int32_t *node_ptr,
                              int32_t *node_sets, int32_t mem_kind, void *stream) {
    if (!r)
        return fail(LCD_EINVAL, "null result");
    if (scale_idx < 0 || scale_idx >= r->S)
        return fail(LCD_EINVAL, "scale index %d out of range", scale_idx);
    if (mem_kind != LCD_MEM_HOST && mem_kind != LCD_MEM_DEVICE)
        return fail(LCD_EINVAL, "unknown mem_kind %d", mem_kind);
    if (!node_ptr || !node_sets)
        return fail(LCD_EINVAL, "null output");
    hipStream_t st = (hipStream_t)stream;
    const int32_t n = r->g->n;
    const size_t ns = (size_t)r->n_sets;
    int32_t *cp = nullptr, *mem = nullptr, *cnt = nullptr, *bs = nullptr, *np = nullptr, *nsets = nullptr;
    lcd_status s = LCD_OK;
    int64_t tot = 0;
    const int nb = (int)(((int64_t)n + 1 + 1023) / 1024);
    hipError_t e;
    if ((s = dev_alloc(&cp, ns + 1)) != LCD_OK)
        goto done;
    if ((s = scale_offsets(r, scale_idx, cp, st, &tot)) != LCD_OK || (s = check_int32_total(tot, scale_idx)) != LCD_OK)
        goto done;
    if ((s = dev_alloc(&mem, (size_t)tot)) != LCD_OK || (s = dev_alloc(&cnt, (size_t)n + 1)) != LCD_OK ||
        (s = dev_alloc(&bs, (size_t)nb + 1)) != LCD_OK)
        goto done;
    np = node_ptr;
    nsets = node_sets;
    if (mem_kind == LCD_MEM_HOST) {
        if ((s = dev_alloc(&np, (size_t)n + 1)) != LCD_OK || (s = dev_alloc(&nsets, (size_t)tot)) != LCD_OK)
            goto done;
    }
    if ((s = scale_members(r, scale_idx, nullptr, r->n_sets, cp, mem, st)) != LCD_OK)
        goto done;
    e = launch_overlap(cp, mem, tot, r->n_sets, n, np, nsets, cnt, bs, st);
    if (e == hipSuccess && mem_kind == LCD_MEM_HOST) {
        e = hipMemcpyAsync(node_ptr, np, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && tot)
            e = hipMemcpyAsync(node_sets, nsets, sizeof(int32_t) * (size_t)tot, hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        s = fail(LCD_EDEVICE, "overlap: %s", hipGetErrorString(e));
done:
    dev_free(cp);
    dev_free(mem);
    dev_free(cnt);
    dev_free(bs);
    if (mem_kind == LCD_MEM_HOST) {
        dev_free(np);
        dev_free(nsets);
    }
    return s;
}

lcd_status lcd_result_counters(const lcd_result *r, uint64_t *totals, uint64_t *per_record,
                               int32_t mem_kind, void *stream) {
    if (!r)
        return fail(LCD_EINVAL, "null result");
    if (mem_kind != LCD_MEM_HOST && mem_kind != LCD_MEM_DEVICE)
        return fail(LCD_EINVAL, "unknown mem_kind %d", mem_kind);
    hipStream_t st = (hipStream_t)stream;
    const int64_t R = (int64_t)r->n_sets * r->S;
    if (totals) {
        unsigned long long *tot = nullptr;
        CHK(dev_alloc(&tot, 4));
        hipError_t e = launch_zero_bytes(tot, 32, st);
        if (e == hipSuccess)
            e = launch_counter_sum(r->rec.ctr, R, tot, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(totals, tot, 32, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        dev_free(tot);
        if (e != hipSuccess)
            return fail(LCD_EDEVICE, "counters: %s", hipGetErrorString(e));
    }
    if (per_record && R) {
        HIPCHK(hipMemcpyAsync(per_record, r->rec.ctr, sizeof(uint64_t) * 4 * (size_t)R,
                              mem_kind == LCD_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                              st));
        HIPCHK(hipStreamSynchronize(st));
    }
    return LCD_OK;
}

lcd_status lcd_result_sets(const lcd_result *r, const int32_t *set_ids, int32_t n_ids,
                           int64_t *rec_off, int32_t *rec_cnt, int32_t *members, int64_t members_cap,
                           int64_t *members_needed, int64_t *k_in, int64_t *vol, double *f,
                           uint64_t *ctr) {
    if (!r || (n_ids > 0 && (!set_ids || !rec_off || !rec_cnt || !members_needed)))
        return fail(LCD_EINVAL, "null argument");
    const int32_t S = r->S;
    std::vector<int64_t> off((size_t)S);
    std::vector<int32_t> cnt((size_t)S);
    int64_t pos = 0;
    for (int32_t q = 0; q < n_ids; ++q) {
        const int32_t j = set_ids[q];
        if (j < 0 || j >= r->n_sets)
            return fail(LCD_EINVAL, "set id %d out of range", j);
        const size_t r0 = (size_t)j * S;
        HIPCHK(hipMemcpy(off.data(), r->rec.off + r0, sizeof(int64_t) * S, hipMemcpyDeviceToHost));
        HIPCHK(hipMemcpy(cnt.data(), r->rec.cnt + r0, sizeof(int32_t) * S, hipMemcpyDeviceToHost));
        const size_t o = (size_t)q * S;
        if (k_in)
            HIPCHK(hipMemcpy(k_in + o, r->rec.K + r0, sizeof(int64_t) * S, hipMemcpyDeviceToHost));
        if (vol)
            HIPCHK(hipMemcpy(vol + o, r->rec.V + r0, sizeof(int64_t) * S, hipMemcpyDeviceToHost));
        if (f)
            HIPCHK(hipMemcpy(f + o, r->rec.f + r0, sizeof(double) * S, hipMemcpyDeviceToHost));
        if (ctr)
            HIPCHK(hipMemcpy(ctr + 4 * o, r->rec.ctr + 4 * r0, sizeof(uint64_t) * 4 * S,
                             hipMemcpyDeviceToHost));
        for (int32_t s = 0; s < S; ++s) {
            rec_off[o + s] = pos;
            rec_cnt[o + s] = cnt[s];
            if (!r->rec.drem && members && pos + cnt[s] <= members_cap && cnt[s] > 0)
                HIPCHK(hipMemcpy(members + pos, r->pool + off[s], sizeof(int32_t) * (size_t)cnt[s],
                                 hipMemcpyDeviceToHost));
            pos += cnt[s];
        }
    }
    *members_needed = pos;
    if (members && pos > members_cap)
        return fail(LCD_ECAPACITY, "members buffer holds %lld entries, %lld needed",
                    (long long)members_cap, (long long)pos);
    if (r->rec.drem && members && n_ids > 0 && pos > 0) {
        // delta output: every scale's lists rebuilt on the device straight
        // to their places in one buffer, then one copy
        if (pos > (int64_t)INT32_MAX)
            return fail(LCD_ECAPACITY, "selected sets list %lld members; at most 2^31 - 1 per call", (long long)pos);
        int32_t *d_ids = nullptr, *d_ptr = nullptr, *d_mem = nullptr;
        std::vector<int32_t> ptr((size_t)n_ids);
        lcd_status x = LCD_OK;
        if ((x = dev_alloc(&d_ids, (size_t)n_ids)) != LCD_OK || (x = dev_alloc(&d_ptr, (size_t)n_ids)) != LCD_OK ||
            (x = dev_alloc(&d_mem, (size_t)pos)) != LCD_OK) {
            dev_free(d_ids);
            dev_free(d_ptr);
            return x;
        }
        hipError_t e = hipMemcpy(d_ids, set_ids, sizeof(int32_t) * (size_t)n_ids, hipMemcpyHostToDevice);
        for (int32_t s = 0; s < S && e == hipSuccess && x == LCD_OK; ++s) {
            for (int32_t q = 0; q < n_ids; ++q)
                ptr[q] = (int32_t)rec_off[(size_t)q * S + s];
            e = hipMemcpy(d_ptr, ptr.data(), sizeof(int32_t) * (size_t)n_ids, hipMemcpyHostToDevice);
            if (e == hipSuccess)
                x = scale_members(r, s, d_ids, n_ids, d_ptr, d_mem, nullptr);
        }
        if (e == hipSuccess && x == LCD_OK)
            e = hipMemcpy(members, d_mem, sizeof(int32_t) * (size_t)pos, hipMemcpyDeviceToHost);
        dev_free(d_ids);
        dev_free(d_ptr);
        dev_free(d_mem);
        if (x != LCD_OK)
            return x;
        if (e != hipSuccess)
            return fail(LCD_EDEVICE, "sets readout: %s", hipGetErrorString(e));
    }
    return LCD_OK;
}

lcd_status lcd_result_delta_sizes(const lcd_result *r, int32_t scale_idx, int64_t *n_added, int64_t *n_removed) {
    if (!r || !n_added || !n_removed)
        return fail(LCD_EINVAL, "null argument");
    if (scale_idx < 0 || scale_idx >= r->S)
        return fail(LCD_EINVAL, "scale index %d out of range", scale_idx);
    if (!r->rec.drem)
        return fail(LCD_ESTATE, "the sweep stored full lists (output_mode LCD_OUT_DELTA gives deltas)");
    const size_t n = (size_t)r->n_sets;
    int64_t *na = nullptr, *nr = nullptr, *ao = nullptr, *ro = nullptr;
    lcd_status x = LCD_OK;
    int64_t h[2] = {0, 0};
    if ((x = dev_alloc(&na, std::max<size_t>(n, 1))) == LCD_OK && (x = dev_alloc(&nr, std::max<size_t>(n, 1))) == LCD_OK &&
        (x = dev_alloc(&ao, n + 1)) == LCD_OK && (x = dev_alloc(&ro, n + 1)) == LCD_OK) {
        hipError_t e = launch_delta_lists(r->rec, r->pool, r->S, scale_idx, r->n_sets, na, nr, ao, ro, nullptr,
                                          nullptr, nullptr);
        if (e == hipSuccess)
            e = hipMemcpy(&h[0], ao + n, sizeof(int64_t), hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            e = hipMemcpy(&h[1], ro + n, sizeof(int64_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            x = fail(LCD_EDEVICE, "delta sizes: %s", hipGetErrorString(e));
    }
    dev_free(na);
    dev_free(nr);
    dev_free(ao);
    dev_free(ro);
    CHK(x);
    *n_added = h[0];
    *n_removed = h[1];
    return LCD_OK;
}

lcd_status lcd_result_delta(const lcd_result *r, int32_t scale_idx, int64_t *add_ptr, int32_t *added,
                            int64_t *rem_ptr, int32_t *removed, int32_t mem_kind, void *stream) {
    if (!r || !add_ptr || !rem_ptr)
        return fail(LCD_EINVAL, "null argument");
    if (scale_idx < 0 || scale_idx >= r->S)
        return fail(LCD_EINVAL, "scale index %d out of range", scale_idx);
    if (mem_kind != LCD_MEM_HOST && mem_kind != LCD_MEM_DEVICE)
        return fail(LCD_EINVAL, "unknown mem_kind %d", mem_kind);
    if (!r->rec.drem)
        return fail(LCD_ESTATE, "the sweep stored full lists (output_mode LCD_OUT_DELTA gives deltas)");
    int64_t ta = 0, tr = 0;
    CHK(lcd_result_delta_sizes(r, scale_idx, &ta, &tr));
    if ((ta > 0 && !added) || (tr > 0 && !removed))
        return fail(LCD_EINVAL, "null output");
    hipStream_t st = (hipStream_t)stream;
    const size_t n = (size_t)r->n_sets;
    const bool host = mem_kind == LCD_MEM_HOST;
    int64_t *na = nullptr, *nr = nullptr, *ao = add_ptr, *ro = rem_ptr;
    int32_t *da = added, *dr = removed;
    lcd_status x = LCD_OK;
    hipError_t e = hipSuccess;
    if ((x = dev_alloc(&na, std::max<size_t>(n, 1))) != LCD_OK || (x = dev_alloc(&nr, std::max<size_t>(n, 1))) != LCD_OK)
        goto done;
    if (host) {
        ao = ro = nullptr;
        da = dr = nullptr;
        if ((x = dev_alloc(&ao, n + 1)) != LCD_OK || (x = dev_alloc(&ro, n + 1)) != LCD_OK ||
            (x = dev_alloc(&da, (size_t)std::max<int64_t>(ta, 1))) != LCD_OK ||
            (x = dev_alloc(&dr, (size_t)std::max<int64_t>(tr, 1))) != LCD_OK)
            goto done;
    }
    e = launch_delta_lists(r->rec, r->pool, r->S, scale_idx, r->n_sets, na, nr, ao, ro, da, dr, st);
    if (e == hipSuccess && host) {
        e = hipMemcpyAsync(add_ptr, ao, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(rem_ptr, ro, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && ta)
            e = hipMemcpyAsync(added, da, sizeof(int32_t) * (size_t)ta, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && tr)
            e = hipMemcpyAsync(removed, dr, sizeof(int32_t) * (size_t)tr, hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    if (e != hipSuccess)
        x = fail(LCD_EDEVICE, "delta readout: %s", hipGetErrorString(e));
done:
    dev_free(na);
    dev_free(nr);
    if (host) {
        dev_free(ao);
        dev_free(ro);
        dev_free(da);
        dev_free(dr);
    }
    return x;
}

}  // extern "C"

namespace {

// NMI of two well-formed covers given as device CSR arrays (int32 offsets,
// tx and ty members); the value goes to the device double d_out.
lcd_status cover_nmi_dev(int32_t n, int32_t cus, int32_t kx, const int32_t *px, const int32_t *mx, int64_t tx,
                         int32_t ky, const int32_t *py, const int32_t *my, int64_t ty, double *d_out, hipStream_t st) {
    double *h = nullptr, *term = nullptr, *res = nullptr;
    int32_t *np_x = nullptr, *ns_x = nullptr, *np_y = nullptr, *ns_y = nullptr, *cnt = nullptr, *bs = nullptr,
            *cnt_all = nullptr;
    unsigned *next = nullptr;
    const int32_t kmax = std::max(std::max(kx, ky), 1);
    const int nb = (int)(((int64_t)n + 1 + 1023) / 1024) + 1;
    const int32_t slots = (int32_t)std::max<int64_t>(
        1, std::min<int64_t>(4 * (int64_t)cus, ((int64_t)1 << 30) / (4 * (int64_t)kmax)));
    auto release = [&]() {
        dev_free(h);
        dev_free(term);
        dev_free(res);
        dev_free(np_x);
        dev_free(ns_x);
        dev_free(np_y);
        dev_free(ns_y);
        dev_free(cnt);
        dev_free(bs);
        dev_free(cnt_all);
        dev_free(next);
    };
    lcd_status s;
    if ((s = dev_alloc(&h, (size_t)n + 1)) != LCD_OK || (s = dev_alloc(&term, (size_t)kmax)) != LCD_OK ||
        (s = dev_alloc(&res, 4)) != LCD_OK || (s = dev_alloc(&np_x, (size_t)n + 1)) != LCD_OK ||
        (s = dev_alloc(&ns_x, (size_t)std::max<int64_t>(tx, 1))) != LCD_OK ||
        (s = dev_alloc(&np_y, (size_t)n + 1)) != LCD_OK ||
        (s = dev_alloc(&ns_y, (size_t)std::max<int64_t>(ty, 1))) != LCD_OK ||
        (s = dev_alloc(&cnt, (size_t)n + 1)) != LCD_OK || (s = dev_alloc(&bs, (size_t)nb + 1)) != LCD_OK ||
        (s = dev_alloc(&cnt_all, (size_t)slots * (size_t)kmax)) != LCD_OK || (s = dev_alloc(&next, 1)) != LCD_OK) {
        release();
        return s;
    }
    hipError_t e = launch_nmi_htab(h, n, st);
    if (e == hipSuccess)
        e = launch_overlap(py, my, ty, ky, n, np_y, ns_y, cnt, bs, st);
    if (e == hipSuccess)
        e = launch_overlap(px, mx, tx, kx, n, np_x, ns_x, cnt, bs, st);
    if (e == hipSuccess)
        e = launch_zero_bytes(cnt_all, 4 * (int64_t)slots * kmax, st);
    if (e == hipSuccess)
        e = launch_nmi_half(px, mx, kx, py, ky, np_y, ns_y, h, n, cnt_all, slots, next, term, res, st);
    if (e == hipSuccess)
        e = launch_nmi_half(py, my, ky, px, kx, np_x, ns_x, h, n, cnt_all, slots, next, term, res + 2, st);
    if (e == hipSuccess)
        e = launch_nmi_final(res, res + 2, d_out, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    release();
    if (e != hipSuccess)
        return fail(LCD_EDEVICE, "nmi: %s", hipGetErrorString(e));
    return LCD_OK;
}

// One scale of a result as a device cover (offsets and members, owned by
// the caller of this helper).
lcd_status scale_cover(const lcd_result *r, int32_t s, hipStream_t st, int32_t **ptr, int32_t **mem, int64_t *tot) {
    *ptr = nullptr;
    *mem = nullptr;
    CHK(dev_alloc(ptr, (size_t)r->n_sets + 1));
    lcd_status x = scale_offsets(r, s, *ptr, st, tot);
    if (x == LCD_OK)
        x = check_int32_total(*tot, s);
    if (x == LCD_OK)
        x = dev_alloc(mem, (size_t)std::max<int64_t>(*tot, 1));
    if (x == LCD_OK)
        x = scale_members(r, s, nullptr, r->n_sets, *ptr, *mem, st);
    if (x != LCD_OK) {
        dev_free(*ptr);
        dev_free(*mem);
    }
    return x;
}

}  // namespace

extern "C" {

lcd_status lcd_cover_nmi(int32_t n, int32_t kx, const int32_t *ptr_x, const int32_t *mem_x, int32_t ky,
                         const int32_t *ptr_y, const int32_t *mem_y, double *out, void *stream) {
    if (!out || n < 1 || kx < 0 || ky < 0 || !ptr_x || !ptr_y)
        return fail(LCD_EINVAL, "bad arguments (n >= 1, counts >= 0, offsets and out not null)");
    hipStream_t st = (hipStream_t)stream;
    int32_t tt[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(&tt[0], ptr_x + kx, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(&tt[1], ptr_y + ky, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if ((tt[0] > 0 && !mem_x) || (tt[1] > 0 && !mem_y))
        return fail(LCD_EINVAL, "null members array");
    DevInfo d;
    CHK(device_info(d));
    uint32_t *bad = nullptr;
    double *dv = nullptr;
    CHK(dev_alloc(&bad, 2));
    uint32_t hb[2] = {0, 0};
    hipError_t e = launch_cover_check(ptr_x, mem_x, kx, tt[0], n, bad, st);
    if (e == hipSuccess)
        e = launch_cover_check(ptr_y, mem_y, ky, tt[1], n, bad + 1, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(hb, bad, sizeof(hb), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    dev_free(bad);
    if (e != hipSuccess)
        return fail(LCD_EDEVICE, "cover check: %s", hipGetErrorString(e));
    if (hb[0] || hb[1])
        return fail(LCD_EINVAL, "a cover is malformed (offsets from 0 to the total, ascending ids in [0, n))");
    CHK(dev_alloc(&dv, 1));
    lcd_status s = cover_nmi_dev(n, d.cus, kx, ptr_x, mem_x, tt[0], ky, ptr_y, mem_y, tt[1], dv, st);
    if (s == LCD_OK) {
        e = hipMemcpyAsync(out, dv, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            s = fail(LCD_EDEVICE, "nmi readout: %s", hipGetErrorString(e));
    }
    dev_free(dv);
    return s;
}

lcd_status lcd_result_nmi(const lcd_result *r, int32_t s1, int32_t s2, double *out, void *stream) {
    if (!r || !out)
        return fail(LCD_EINVAL, "null argument");
    if (s1 < 0 || s1 >= r->S || s2 < 0 || s2 >= r->S)
        return fail(LCD_EINVAL, "scale index out of range");
    hipStream_t st = (hipStream_t)stream;
    int32_t *p1 = nullptr, *m1 = nullptr, *p2 = nullptr, *m2 = nullptr;
    double *dv = nullptr;
    int64_t t1 = 0, t2 = 0;
    CHK(scale_cover(r, s1, st, &p1, &m1, &t1));
    lcd_status s = scale_cover(r, s2, st, &p2, &m2, &t2);
    if (s == LCD_OK)
        s = dev_alloc(&dv, 1);
    if (s == LCD_OK)
        s = cover_nmi_dev(r->g->n, r->g->dev.cus, r->n_sets, p1, m1, t1, r->n_sets, p2, m2, t2, dv, st);
    if (s == LCD_OK) {
        hipError_t e = hipMemcpyAsync(out, dv, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            s = fail(LCD_EDEVICE, "nmi readout: %s", hipGetErrorString(e));
    }
    dev_free(p1);
    dev_free(m1);
    dev_free(p2);
    dev_free(m2);
    dev_free(dv);
    return s;
}

lcd_status lcd_result_nmi_successive(const lcd_result *r, int32_t p, double *out, void *stream) {
    if (!r || !out)
        return fail(LCD_EINVAL, "null argument");
    if (p < 2 || p > r->S)
        return fail(LCD_EINVAL, "p must be in [2, n_scales]");
    hipStream_t st = (hipStream_t)stream;
    double *pair = nullptr, *win = nullptr;
    CHK(dev_alloc(&pair, (size_t)r->S));
    lcd_status s = dev_alloc(&win, (size_t)r->S);
    int32_t *pa = nullptr, *ma = nullptr;
    int64_t ta = 0;
    if (s == LCD_OK)
        s = scale_cover(r, 0, st, &pa, &ma, &ta);
    for (int32_t t = 0; t + 1 < r->S && s == LCD_OK; ++t) {
        int32_t *pb = nullptr, *mb = nullptr;
        int64_t tb = 0;
        s = scale_cover(r, t + 1, st, &pb, &mb, &tb);
        if (s == LCD_OK)
            s = cover_nmi_dev(r->g->n, r->g->dev.cus, r->n_sets, pa, ma, ta, r->n_sets, pb, mb, tb, pair + t, st);
        dev_free(pa);
        dev_free(ma);
        pa = pb;
        ma = mb;
        ta = tb;
    }
    if (s == LCD_OK) {
        hipError_t e = launch_nmi_windows(pair, r->S, p, win, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(out, win, sizeof(double) * (size_t)(r->S - p + 1), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            s = fail(LCD_EDEVICE, "nmi windows: %s", hipGetErrorString(e));
    }
    dev_free(pa);
    dev_free(ma);
    dev_free(pair);
    dev_free(win);
    return s;
}

lcd_status lcd_result_nmi_cover(const lcd_result *r, int32_t scale_idx, int32_t k, const int32_t *ptr,
                                const int32_t *mem, double *out, void *stream) {
    if (!r || !out || !ptr || k < 0)
        return fail(LCD_EINVAL, "bad arguments");
    if (scale_idx < 0 || scale_idx >= r->S)
        return fail(LCD_EINVAL, "scale index out of range");
    hipStream_t st = (hipStream_t)stream;
    int32_t tk = 0;
    HIPCHK(hipMemcpyAsync(&tk, ptr + k, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (tk > 0 && !mem)
        return fail(LCD_EINVAL, "null members array");
    uint32_t *bad = nullptr;
    CHK(dev_alloc(&bad, 1));
    uint32_t hb = 0;
    hipError_t e = launch_cover_check(ptr, mem, k, tk, r->g->n, bad, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&hb, bad, sizeof(hb), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess)
        e = hipStreamSynchronize(st);
    dev_free(bad);
    if (e != hipSuccess)
        return fail(LCD_EDEVICE, "cover check: %s", hipGetErrorString(e));
    if (hb)
        return fail(LCD_EINVAL, "the cover is malformed (offsets from 0 to the total, ascending ids in [0, n))");
    int32_t *p1 = nullptr, *m1 = nullptr;
    double *dv = nullptr;
    int64_t t1 = 0;
    CHK(scale_cover(r, scale_idx, st, &p1, &m1, &t1));
    lcd_status s = dev_alloc(&dv, 1);
    if (s == LCD_OK)
        s = cover_nmi_dev(r->g->n, r->g->dev.cus, r->n_sets, p1, m1, t1, k, ptr, mem, tk, dv, st);
    if (s == LCD_OK) {
        e = hipMemcpyAsync(out, dv, sizeof(double), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipStreamSynchronize(st);
        if (e != hipSuccess)
            s = fail(LCD_EDEVICE, "nmi readout: %s", hipGetErrorString(e));
    }
    dev_free(p1);
    dev_free(m1);
    dev_free(dv);
    return s;
}

lcd_status lcd_result_stats(const lcd_result *r, lcd_sweep_stats *out) {
    if (!r || !out)
        return fail(LCD_EINVAL, "null argument");
    *out = r->stats;
    return LCD_OK;
}

lcd_status lcd_result_rerun(lcd_result *r, void *stream) {
    if (!r)
        return fail(LCD_EINVAL, "null result");
    if (r->into)
        return fail(LCD_EINVAL, "a result of lcd_sweep_merge cannot be rerun");
    return run_sweep(r, (hipStream_t)stream);
}

lcd_status lcd_result_free(lcd_result *r) {
    result_release(r);
    return LCD_OK;
}

lcd_status lcd_log_device(const uint64_t *x, double *out, int64_t n, void *stream) {
    if (n < 0 || (n > 0 && (!x || !out)))
        return fail(LCD_EINVAL, "bad arguments");
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(launch_log(x, out, n, st));
    HIPCHK(hipStreamSynchronize(st));
    return LCD_OK;
}

}  // extern "C"
