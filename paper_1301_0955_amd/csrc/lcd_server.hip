// Local-community query server: a resident graph answers (seed set, scale)
// queries (growth to a fixpoint at one scale, the per-scale step of the
// method in Sec. 2 and Algorithm 1, without chaining).
//
// Continuous batching over a small number of launch lanes.  Each lane owns
// a HIP stream, device buffers for one batch (seeds, scales, records, member
// pool, spill-tier tables) and pinned host staging.  One worker thread
//   * retires lanes whose batch finished (records and member lists back to
//     the host, tickets completed),
//   * admits pending queries into every idle lane at once, as many as the
//     lane's memory, the batch limit and the free query slots allow, and
//     launches the batch on that lane's stream,
// so queries that arrive while others run start in another lane without
// waiting for them, and batches of different lanes overlap on the device.
// A query's result does not depend on its batch: every set is grown by its
// own wavefront from its own seeds, and the kernels are the sweep kernels
// with a per-set scale.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lcd.h"
#include "lcd_host.h"
#include "lcd_internal.h"

using namespace lcd;

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Query {
    uint64_t ticket = 0;
    std::vector<int32_t> seeds;
    double alpha = 0.0;
    int64_t reserve = 0;        // member-pool entries reserved at admission
    bool solo = false;          // rerun alone after its batch's pool overflowed
    bool cancel = false;        // withdrawn while on the device: drop its result
    bool done = false;
    lcd_status status = LCD_EAGAIN;
    std::string msg;
    std::vector<int32_t> members;
    lcd_query_info info{};
};

template <typename T>
lcd_status host_alloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0)
        count = 1;
    hipError_t e = hipHostMalloc((void **)p, count * sizeof(T), hipHostMallocDefault);
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(LCD_ENOMEM, "hipHostMalloc of %zu bytes failed", count * sizeof(T));
    }
    return LCD_OK;
}

// Pinned host memory the device writes while a kernel runs and the host
// reads as soon as a flag says so (fine-grained, coherent); *dev gets the
// device's address of it.
template <typename T>
lcd_status host_alloc_coherent(T **p, T **dev, size_t count) {
    *p = nullptr;
    *dev = nullptr;
    if (count == 0)
        count = 1;
    hipError_t e = hipHostMalloc((void **)p, count * sizeof(T), hipHostMallocCoherent | hipHostMallocMapped);
    if (e == hipSuccess)
        e = hipHostGetDevicePointer((void **)dev, (void *)*p, 0);
    if (e != hipSuccess) {
        if (*p)
            (void)hipHostFree((void *)*p);
        *p = nullptr;
        *dev = nullptr;
        (void)hipGetLastError();
        return fail(LCD_ENOMEM, "coherent hipHostMalloc of %zu bytes failed", count * sizeof(T));
    }
    return LCD_OK;
}

template <typename T>
void host_free(T *&p) {
    if (p)
        (void)hipHostFree((void *)p);
    p = nullptr;
}

// A stage runs the tiers [first, last) of the plan; queries whose table
// overflows its last tier go on to the next stage.
struct Stage {
    int first = 0, last = 0;
};
constexpr int kMaxStages = kMaxTiers;
constexpr int kMaxLanes = 8;

struct Lane {
    int id = 0;
    int stage = 0;
    hipStream_t st = nullptr;
    hipEvent_t done = nullptr;
    int32_t max_q = 0;
    int64_t max_seed = 0;
    int64_t pool_cap = 0;
    // device
    double *alpha = nullptr;
    int32_t *seed_ptr = nullptr;
    int32_t *seed_nodes = nullptr;
    // records, member pool and completion flags: coherent pinned host
    // memory written by the kernels (device addresses here, host ones in
    // h_off .. h_pool, h_flags), so that a query completes when its own
    // flag is set, not when its batch ends
    Records rec{};
    int32_t *pool = nullptr;
    uint32_t *flags = nullptr;
    Counters *ctl = nullptr;
    unsigned long long *cursor = nullptr;
    int32_t *work[kMaxTiers - 1] = {nullptr, nullptr, nullptr};
    Slab slab[2];
    // pinned host staging
    double *h_alpha = nullptr;
    int32_t *h_seed_ptr = nullptr;
    int32_t *h_seed_nodes = nullptr;
    int64_t *h_off = nullptr;
    int32_t *h_cnt = nullptr;
    int64_t *h_K = nullptr;
    int64_t *h_V = nullptr;
    double *h_f = nullptr;
    uint64_t *h_ctr = nullptr;
    unsigned long long *h_cursor = nullptr;
    int32_t *h_pool = nullptr;
    Counters *h_ctl = nullptr;
    int32_t *h_work0 = nullptr;
    uint32_t *h_flags = nullptr;
    // batch in flight; taken[i]: query i already completed from its flag
    std::vector<Query *> batch;
    std::vector<char> taken;
    bool busy = false;
    int64_t t_start = 0;
};

void lane_release(Lane &L) {
    dev_free(L.alpha);
    dev_free(L.seed_ptr);
    dev_free(L.seed_nodes);
    dev_free(L.ctl);
    dev_free(L.cursor);
    for (auto &w : L.work)
        dev_free(w);
    dev_free(L.slab[0].buf);
    dev_free(L.slab[1].buf);
    host_free(L.h_alpha);
    host_free(L.h_seed_ptr);
    host_free(L.h_seed_nodes);
    host_free(L.h_off);
    host_free(L.h_cnt);
    host_free(L.h_K);
    host_free(L.h_V);
    host_free(L.h_f);
    host_free(L.h_ctr);
    host_free(L.h_cursor);
    host_free(L.h_pool);
    host_free(L.h_ctl);
    host_free(L.h_work0);
    host_free(L.h_flags);
    if (L.done)
        (void)hipEventDestroy(L.done);
    if (L.st)
        (void)hipStreamDestroy(L.st);
    L.done = nullptr;
    L.st = nullptr;
}

// Device bytes of one lane's buffers (without the spill tables; records
// and member pool are host memory).
int64_t lane_bytes(int32_t max_q, int64_t max_seed, int64_t pool_cap) {
    (void)pool_cap;
    return (int64_t)max_q * (8 + 4 + 4 + 4 * (kMaxTiers - 1)) + max_seed * 4 + 8 * kCursorWords +
           (int64_t)sizeof(Counters) + 256 * 16;
}

}  // namespace

struct lcd_server {
    const lcd_graph *g = nullptr;
    lcd_params prm{};
    TierPlan tp{};
    int32_t max_slots = 0;
    int64_t mem_budget = 0;
    int64_t mem_held = 0;
    std::vector<Lane> lanes;
    std::mutex mu;
    std::condition_variable cv_work;
    std::condition_variable cv_done;
    std::deque<Query *> pending;         // submitted, waiting for a stage-0 lane
    Stage stages[kMaxStages];
    int n_stages = 1;
    std::deque<Query *> forwarded[kMaxStages];   // waiting for a lane of stage k (k >= 1)
    std::unordered_map<uint64_t, Query *> tickets;
    uint64_t next_ticket = 1;
    int64_t in_flight = 0;
    bool stop = false;
    std::thread worker;
    lcd_server_stats stats{};
    // start-stage routing: host copy of the CSR and each stage's table size
    bool route = false;
    std::vector<int32_t> h_row_ptr, h_col;
    int32_t stage_cap[kMaxStages] = {0};
};

namespace {

// Launch the batch already placed in L.batch; called without the lock.
// An entry lane runs tier 0 only; the sets that overflow it are listed in
// work[0] and leave for a spill lane.  A spill lane runs the later tiers on
// its whole batch, fed as if tier 0 had pushed every set.
lcd_status launch_lane(lcd_server *S, Lane &L) {
    const lcd_graph *g = S->g;
    const int32_t nq = (int32_t)L.batch.size();
    int64_t pos = 0;
    for (int32_t i = 0; i < nq; ++i) {
        const Query *q = L.batch[i];
        L.h_alpha[i] = q->alpha;
        L.h_seed_ptr[i] = (int32_t)pos;
        std::memcpy(L.h_seed_nodes + pos, q->seeds.data(), sizeof(int32_t) * q->seeds.size());
        pos += (int64_t)q->seeds.size();
    }
    L.h_seed_ptr[nq] = (int32_t)pos;
    for (int32_t i = 0; i < nq; ++i)
        __atomic_store_n(&L.h_flags[i], 0u, __ATOMIC_RELAXED);
    L.taken.assign((size_t)nq, 0);
    hipStream_t st = L.st;
    HIPCHK(hipMemcpyAsync(L.alpha, L.h_alpha, sizeof(double) * nq, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(L.seed_ptr, L.h_seed_ptr, sizeof(int32_t) * (nq + 1), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(L.seed_nodes, L.h_seed_nodes, sizeof(int32_t) * pos, hipMemcpyHostToDevice, st));
    HIPCHK(launch_zero_bytes(L.cursor, 8 * kCursorWords, st));
    const Stage &G = S->stages[L.stage];
    if (G.first > 0) {
        // as if tier first-1 had pushed every set of the batch
        std::memset(L.h_ctl, 0, sizeof(Counters));
        L.h_ctl->ovf_count[G.first - 1] = (uint32_t)nq;
        for (int32_t i = 0; i < nq; ++i)
            L.h_work0[i] = i;
        HIPCHK(hipMemcpyAsync(L.ctl, L.h_ctl, sizeof(Counters), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(L.work[G.first - 1], L.h_work0, sizeof(int32_t) * nq, hipMemcpyHostToDevice, st));
    } else {
        HIPCHK(launch_zero_bytes(L.ctl, (int64_t)sizeof(Counters), st));
    }
    for (int k = 0; k < S->tp.n; ++k)
        if (S->tp.t[k].slab >= 0 && L.slab[S->tp.t[k].slab].buf) {
            Slab &sl = L.slab[S->tp.t[k].slab];
            CHK(ensure_slab(sl, sl.cap, sl.slots, st));
        }
    SweepArgs a{};
    a.g = graph_dev(g);
    a.scales = L.alpha;
    a.alpha_set = L.alpha;
    a.S = 1;
    a.s_begin = 0;
    a.s_end = 1;
    a.seed_ptr = L.seed_ptr;
    a.seed_nodes = L.seed_nodes;
    a.n_sets = nq;
    a.k_prune = S->prm.k_prune;
    a.queue_min = queue_min_of(S->prm);
    a.resume = 0;
    a.rec = L.rec;
    a.pool = L.pool;
    a.pool_cap = L.pool_cap;
    a.ctl = L.ctl;
    a.pool_cursor = L.cursor;
    a.err = (uint32_t *)(L.cursor + 1);
    a.stat = L.cursor + 2;
    a.budget_ticks = S->prm.watchdog_ms < 0 ? 0 : g->dev.wall_khz * (int64_t)S->prm.watchdog_ms;
    a.done_flags = L.flags;
    const TierSpec &T0 = S->tp.t[0];
    const int32_t blocks0 = std::min<int32_t>(T0.blocks, (nq + T0.waves - 1) / T0.waves);
    int32_t launches = 0;
    CHK(enqueue_tiers(a, S->tp, G.first, G.last, blocks0, L.slab, L.work, nullptr, st, nullptr, &launches));
    HIPCHK(hipMemcpyAsync(L.h_cursor, L.cursor, 8 * kCursorWords, hipMemcpyDeviceToHost, st));
    if (G.last < S->tp.n) {
        HIPCHK(hipMemcpyAsync(L.h_ctl, L.ctl, sizeof(Counters), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(L.h_work0, L.work[G.last - 1], sizeof(int32_t) * nq, hipMemcpyDeviceToHost, st));
    }
    HIPCHK(hipEventRecord(L.done, st));
    return LCD_OK;
}

// Result of query i of the lane's batch from the host-visible records and
// pool; false when its members did not fit the pool.
bool fill_query(Lane &L, int32_t i, Query *q, int64_t t_done) {
    const int64_t off = L.h_off[i];
    const int32_t cnt = L.h_cnt[i];
    if (off < 0 || cnt < 0 || off + cnt > L.pool_cap)
        return false;
    q->members.assign(L.h_pool + off, L.h_pool + off + cnt);
    q->info.n_members = cnt;
    q->info.k_in = L.h_K[i];
    q->info.vol = L.h_V[i];
    q->info.f = L.h_f[i];
    for (int c = 0; c < 4; ++c)
        q->info.ctr[c] = L.h_ctr[4 * i + c];
    q->info.t_done_ns = t_done;
    q->info.batch_size = (int32_t)L.batch.size();
    q->info.lane = L.id;
    q->status = LCD_OK;
    return true;
}

// The lane's batch has finished on the device: fill the queries not yet
// completed from their flags.  Called without the lock.  `again`: queries to run again
// alone (the batch outgrew the lane's pool); `forward`: queries that
// overflowed the last tier of the lane's stage.
lcd_status collect_lane(lcd_server *S, Lane &L, std::vector<Query *> &again,
                        std::vector<Query *> &forward) {
    const int32_t nq = (int32_t)L.batch.size();
    const uint32_t err = (uint32_t)(L.h_cursor[1] & 0xffffffffu);
    if (err) {
        L.slab[0].dirty = L.slab[1].dirty = true;
        return fail(err & ERR_CAPACITY ? LCD_ECAPACITY : LCD_EDEVICE,
                    "query kernel reported error bits 0x%x%s", err,
                    err & ERR_TIMEOUT ? " (watchdog: a query ran past its time budget)" : "");
    }
    std::vector<char> spilled((size_t)nq, 0);
    const Stage &G = S->stages[L.stage];
    if (G.last < S->tp.n) {
        const uint32_t nf = std::min<uint32_t>(L.h_ctl->ovf_count[G.last - 1], (uint32_t)nq);
        for (uint32_t j = 0; j < nf; ++j) {
            const int32_t i = L.h_work0[j];
            if (i < 0 || i >= nq)
                return fail(LCD_EDEVICE, "overflow list holds set %d of a batch of %d", i, nq);
            spilled[i] = 1;
        }
    }
    const int64_t t_done = now_ns();
    for (int32_t i = 0; i < nq; ++i) {
        Query *q = L.batch[i];
        if (L.taken[i])
            continue;
        if (spilled[i]) {
            forward.push_back(q);
            continue;
        }
        if (!fill_query(L, i, q, t_done)) {
            // the batch outgrew the lane's pool: this query runs again alone
            q->solo = true;
            q->reserve = L.pool_cap;
            again.push_back(q);
        }
    }
    return LCD_OK;
}

// Queries of a running batch whose flags are set: results straight from
// the coherent host buffers.  Called without the lock; the queries it
// returns are completed by the caller.
void harvest_lane(Lane &L, std::vector<Query *> &out) {
    const int32_t nq = (int32_t)L.batch.size();
    int64_t t_done = 0;
    for (int32_t i = 0; i < nq; ++i) {
        if (L.taken[i] || __atomic_load_n(&L.h_flags[i], __ATOMIC_ACQUIRE) == 0u)
            continue;
        if (t_done == 0)
            t_done = now_ns();
        if (fill_query(L, i, L.batch[i], t_done)) {
            L.taken[i] = 1;
            out.push_back(L.batch[i]);
        }
    }
}

// Fill L.batch from queue (FIFO) within the lane's limits.  Lock held.
void admit(lcd_server *S, Lane &L, std::deque<Query *> &queue, bool count_slots) {
    int64_t seeds = 0, reserved = 0;
    while (!queue.empty() && (int32_t)L.batch.size() < L.max_q &&
           (!count_slots || S->in_flight < S->max_slots)) {
        Query *q = queue.front();
        const int64_t ns = (int64_t)q->seeds.size();
        if (!L.batch.empty() && (q->solo || seeds + ns > L.max_seed || reserved + q->reserve > L.pool_cap))
            break;
        queue.pop_front();
        L.batch.push_back(q);
        if (count_slots)
            S->in_flight += 1;
        seeds += ns;
        reserved += q->reserve;
        if (q->solo)
            break;
    }
}

// A query leaves the server's bookkeeping (lock held): done, counted; one
// withdrawn while it ran ends cancelled instead.
void finish_query(lcd_server *S, Query *q) {
    if (q->cancel) {
        q->status = LCD_ECANCELED;
        q->msg = "query cancelled";
        q->members.clear();
        S->stats.cancelled += 1;
    } else if (q->status == LCD_OK) {
        S->stats.completed += 1;
    } else {
        S->stats.failed += 1;
    }
    q->done = true;
}

void worker_main(lcd_server *S) {
    (void)hipSetDevice(S->g->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        bool progress = false;
        // 1. retire finished lanes
        for (Lane &L : S->lanes) {
            if (!L.busy)
                continue;
            lk.unlock();
            std::vector<Query *> early;
            harvest_lane(L, early);
            if (!early.empty()) {
                lk.lock();
                for (Query *qq : early) {
                    finish_query(S, qq);
                    S->in_flight -= 1;
                }
                S->cv_done.notify_all();
                progress = true;
                lk.unlock();
            }
            const hipError_t q = hipEventQuery(L.done);
            std::vector<Query *> again, forward;
            lcd_status s = LCD_OK;
            std::string msg;
            bool finished = false;
            if (q == hipSuccess) {
                s = collect_lane(S, L, again, forward);
                finished = true;
            } else if (q != hipErrorNotReady) {
                s = fail(LCD_EDEVICE, "query batch failed: %s", hipGetErrorString(q));
                finished = true;
            }
            if (s != LCD_OK)
                msg = lcd_last_error();
            lk.lock();
            if (!finished)
                continue;
            progress = true;
            if (s != LCD_OK) {
                again.clear();
                forward.clear();
            }
            for (size_t bi = 0; bi < L.batch.size(); ++bi) {
                Query *qq = L.batch[bi];
                if (L.taken[bi])
                    continue;   // completed from its flag
                bool moved = false;
                for (Query *a : again)
                    moved |= a == qq;
                for (Query *a : forward)
                    moved |= a == qq;
                if (moved)
                    continue;
                if (s != LCD_OK) {
                    qq->status = s;
                    qq->msg = msg;
                }
                finish_query(S, qq);
                S->in_flight -= 1;
            }
            // withdrawn queries go no further
            for (auto *lst : {&again, &forward})
                for (auto it = lst->begin(); it != lst->end();) {
                    if ((*it)->cancel) {
                        finish_query(S, *it);
                        S->in_flight -= 1;
                        it = lst->erase(it);
                    } else {
                        ++it;
                    }
                }
            // queries to run again keep their place at the front of their stage
            std::deque<Query *> &back = L.stage == 0 ? S->pending : S->forwarded[L.stage];
            for (auto it = again.rbegin(); it != again.rend(); ++it)
                back.push_front(*it);
            if (L.stage + 1 < S->n_stages)
                for (Query *f : forward)
                    S->forwarded[L.stage + 1].push_back(f);
            if (L.stage == 0)
                S->in_flight -= (int64_t)again.size();   // re-admitted from `pending`
            S->stats.requeued += (int64_t)again.size();
            S->stats.forwarded += (int64_t)forward.size();
            L.batch.clear();
            L.busy = false;
            S->cv_done.notify_all();
        }
        if (S->stop) {
            bool any = false;
            for (Lane &L : S->lanes)
                any |= L.busy;
            bool waiting = false;
            for (int k = 1; k < S->n_stages; ++k)
                waiting |= !S->forwarded[k].empty();
            if (!any && !waiting)
                break;
        }
        // 2. admit waiting queries into idle lanes
        for (Lane &L : S->lanes) {
            if (L.busy)
                continue;
            if (L.stage > 0) {
                if (S->forwarded[L.stage].empty())
                    continue;
                admit(S, L, S->forwarded[L.stage], false);
                S->stats.spill_batches += 1;
            } else {
                if (S->stop || S->pending.empty() || S->in_flight >= S->max_slots)
                    continue;
                admit(S, L, S->pending, true);
            }
            if (L.batch.empty())
                continue;
            L.busy = true;
            S->stats.batches += 1;
            S->stats.max_batch = std::max<int32_t>(S->stats.max_batch, (int32_t)L.batch.size());
            int32_t nbusy = 0;
            for (Lane &M : S->lanes)
                nbusy += M.busy ? 1 : 0;
            S->stats.max_lanes_busy = std::max(S->stats.max_lanes_busy, nbusy);
            L.t_start = now_ns();
            for (Query *q : L.batch)
                if (q->info.t_start_ns == 0)
                    q->info.t_start_ns = L.t_start;
            lk.unlock();
            const lcd_status s = launch_lane(S, L);
            std::string msg = s != LCD_OK ? std::string(lcd_last_error()) : std::string();
            lk.lock();
            progress = true;
            if (s != LCD_OK) {
                lk.unlock();
                (void)hipStreamSynchronize(L.st);
                lk.lock();
                L.slab[0].dirty = L.slab[1].dirty = true;
                for (Query *qq : L.batch) {
                    qq->status = s;
                    qq->msg = msg;
                    qq->done = true;
                    S->stats.failed += 1;
                    S->in_flight -= 1;
                }
                L.batch.clear();
                L.busy = false;
                S->cv_done.notify_all();
            }
        }
        if (progress)
            continue;
        bool any = false;
        for (Lane &L : S->lanes)
            any |= L.busy;
        if (any)
            S->cv_work.wait_for(lk, std::chrono::microseconds(20));
        else
            S->cv_work.wait(lk, [S] {
                // new work: a submitted query, or one queued straight to a
                // later stage
                bool later = false;
                for (int k = 1; k < S->n_stages; ++k)
                    later |= !S->forwarded[k].empty();
                return S->stop || !S->pending.empty() || later;
            });
    }
    // fail whatever is still queued
    for (Query *q : S->pending) {
        q->status = LCD_ESTATE;
        q->msg = "server destroyed";
        q->done = true;
    }
    S->pending.clear();
    S->cv_done.notify_all();
}

lcd_status lane_init(lcd_server *S, Lane &L, int id, int32_t max_q, int64_t max_seed,
                     int64_t pool_cap, const int32_t *slots) {
    L.id = id;
    L.max_q = max_q;
    L.max_seed = max_seed;
    L.pool_cap = pool_cap;
    HIPCHK(hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&L.done, hipEventDisableTiming));
    CHK(dev_alloc(&L.alpha, max_q));
    CHK(dev_alloc(&L.seed_ptr, (size_t)max_q + 1));
    CHK(dev_alloc(&L.seed_nodes, (size_t)max_seed));
    CHK(host_alloc_coherent(&L.h_off, &L.rec.off, max_q));
    CHK(host_alloc_coherent(&L.h_cnt, &L.rec.cnt, max_q));
    CHK(host_alloc_coherent(&L.h_K, &L.rec.K, max_q));
    CHK(host_alloc_coherent(&L.h_V, &L.rec.V, max_q));
    CHK(host_alloc_coherent(&L.h_f, &L.rec.f, max_q));
    CHK(host_alloc_coherent(&L.h_ctr, &L.rec.ctr, 4 * (size_t)max_q));
    CHK(host_alloc_coherent(&L.h_pool, &L.pool, (size_t)pool_cap));
    CHK(host_alloc_coherent(&L.h_flags, &L.flags, max_q));
    CHK(dev_alloc(&L.ctl, 1));
    CHK(dev_alloc(&L.cursor, kCursorWords));
    for (auto &w : L.work)
        CHK(dev_alloc(&w, max_q));
    CHK(host_alloc(&L.h_alpha, max_q));
    CHK(host_alloc(&L.h_seed_ptr, (size_t)max_q + 1));
    CHK(host_alloc(&L.h_seed_nodes, (size_t)max_seed));
    CHK(host_alloc(&L.h_cursor, kCursorWords));
    CHK(host_alloc(&L.h_ctl, 1));
    CHK(host_alloc(&L.h_work0, max_q));
    for (int k = 0; k < S->tp.n; ++k)
        if (S->tp.t[k].slab >= 0 && slots[S->tp.t[k].slab] > 0)
            CHK(ensure_slab(L.slab[S->tp.t[k].slab], S->tp.t[k].cap, slots[S->tp.t[k].slab], L.st));
    HIPCHK(hipStreamSynchronize(L.st));
    return LCD_OK;
}

void server_release(lcd_server *S) {
    for (Lane &L : S->lanes)
        lane_release(L);
    for (auto &kv : S->tickets)
        delete kv.second;
    delete S;
}

}  // namespace

extern "C" {

lcd_status lcd_server_create(const lcd_graph *g, int64_t mem_budget, int32_t max_slots,
                             const lcd_params *params, lcd_server **out) {
    if (!out)
        return fail(LCD_EINVAL, "out is null");
    *out = nullptr;
    if (!g)
        return fail(LCD_EINVAL, "null graph");
    if (mem_budget < 0 || max_slots < 0)
        return fail(LCD_EINVAL, "mem_budget and max_slots must be >= 0");
    lcd_params prm;
    lcd_params_default(&prm);
    if (params)
        prm = *params;
    if (prm.watchdog_ms == 0)
        prm.watchdog_ms = 20000;
    if (mem_budget == 0)
        mem_budget = (int64_t)1 << 30;
    if (max_slots == 0)
        max_slots = 1024;
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != g->device)
        return fail(LCD_EINVAL, "the graph lives on device %d, the current device is %d", g->device, dev);
    size_t free_b = 0, total_b = 0;
    HIPCHK(hipMemGetInfo(&free_b, &total_b));
    if ((int64_t)free_b < mem_budget)
        return fail(LCD_ENOMEM, "mem_budget %lld exceeds the free device memory %lld",
                    (long long)mem_budget, (long long)free_b);
    lcd_server *S = new (std::nothrow) lcd_server();
    if (!S)
        return fail(LCD_ENOMEM, "host allocation failed");
    S->g = g;
    S->prm = prm;
    S->max_slots = max_slots;
    S->mem_budget = mem_budget;
    // serving sizing: the tuned sweep sizing favours throughput over many
    // sets; a query stream wants most queries done by tier 0
    if (params_are_auto(prm)) {
        prm.lds_capacity = 1024;
        prm.team_waves = 8;
    }
    S->prm = prm;
    lcd_status s = plan_tiers(g->dev, g->n, prm, S->tp);
    if (s != LCD_OK) {
        delete S;
        return s;
    }
    // Lanes are HIP streams, and HIP spreads a process's streams over a fixed
    // number of hardware queues (GPU_MAX_HW_QUEUES, 4 unless set before the
    // runtime starts); lanes that share a queue run their batches in turn,
    // so a short batch can wait behind a long one.
    //  * >= 8 queues: one stage per tier (a batch lasts as long as its
    //    slowest query, so a query that fits a small table never waits for
    //    one that needs a large table) and six lanes: one per LDS tier,
    //    three for the 16,384-entry tier (about a third of a query stream
    //    ends there), one for the whole-graph tier; with 10 or more queues
    //    five lanes for the 16,384-entry tier (eight in all), so that a
    //    query leaving an earlier stage finds a free lane sooner.
    //  * fewer: tier 0, then all later tiers; four lanes, one for tier 0.
    int hw_queues = 4;
    if (const char *e = std::getenv("GPU_MAX_HW_QUEUES"))
        hw_queues = std::max(1, std::atoi(e));
    const bool per_tier = hw_queues >= 8 && S->tp.n >= 2;
    S->n_stages = 0;
    if (per_tier) {
        for (int k = 0; k < S->tp.n && k < kMaxStages; ++k)
            S->stages[S->n_stages++] = Stage{k, k + 1};
    } else {
        S->stages[S->n_stages++] = Stage{0, 1};
        if (S->tp.n >= 2)
            S->stages[S->n_stages++] = Stage{1, S->tp.n};
    }
    static const int kPerTierLanes[6] = {0, 1, 2, 2, 2, 3};
    static const int kPerTierWide[8] = {0, 1, 2, 2, 2, 2, 2, 3};
    static const int kTwoStageLanes[4] = {0, 1, 1, 1};
    const bool wide = per_tier && hw_queues >= 10;
    const int n_lanes = per_tier ? (wide ? 8 : 6) : 4;
    int lane_stage[kMaxLanes] = {0};
    for (int i = 0; i < n_lanes; ++i)
        lane_stage[i] = std::min(per_tier ? (wide ? kPerTierWide[i] : kPerTierLanes[i]) : kTwoStageLanes[i],
                                 S->n_stages - 1);
    const int32_t max_q = std::max<int32_t>(1, std::min<int32_t>(1024, max_slots));
    const int64_t max_seed = std::max<int64_t>(65536, (int64_t)g->n);
    const int64_t pool_cap = std::max<int64_t>((int64_t)g->n, 1 << 22);
    int64_t tb[2] = {0, 0};
    int32_t want[2] = {0, 0};
    for (int k = 0; k < S->tp.n; ++k)
        if (S->tp.t[k].slab >= 0) {
            tb[S->tp.t[k].slab] = slab_stride(S->tp.t[k].cap);
            want[S->tp.t[k].slab] = S->tp.t[k].slots;
        }
    const int64_t fixed = lane_bytes(max_q, max_seed, pool_cap);
    // a lane whose stage runs a global tier holds at least one table of it;
    // the rest of the budget buys more (half for the first global tier)
    auto stage_uses = [&](int st, int slab) {
        for (int k = S->stages[st].first; k < S->stages[st].last; ++k)
            if (S->tp.t[k].slab == slab)
                return true;
        return false;
    };
    int64_t need_min = n_lanes * fixed;
    int users[2] = {0, 0};
    for (int i = 0; i < n_lanes; ++i)
        for (int sl = 0; sl < 2; ++sl)
            if (tb[sl] && stage_uses(lane_stage[i], sl)) {
                need_min += tb[sl];
                users[sl] += 1;
            }
    const int64_t left_all = mem_budget - need_min;
    if (left_all < 0) {
        delete S;
        return fail(LCD_ENOMEM, "mem_budget %lld is below the %lld bytes the lanes need on this graph",
                    (long long)mem_budget, (long long)need_min);
    }
    int32_t slots[2] = {0, 0};
    {
        const int64_t half = left_all / 2;
        if (users[0])
            slots[0] = (int32_t)std::min<int64_t>(std::max(1, want[0]), 1 + half / users[0] / tb[0]);
        const int64_t left2 = left_all - (users[0] ? (int64_t)(slots[0] - 1) * tb[0] * users[0] : 0);
        if (users[1])
            slots[1] = (int32_t)std::min<int64_t>(std::max(1, want[1]), 1 + left2 / users[1] / tb[1]);
    }
    S->lanes.resize(n_lanes);
    S->mem_held = n_lanes * fixed;
    for (int i = 0; i < n_lanes; ++i) {
        Lane &L = S->lanes[i];
        L.stage = lane_stage[i];
        int32_t mine[2] = {0, 0};
        for (int sl = 0; sl < 2; ++sl)
            if (tb[sl] && stage_uses(L.stage, sl)) {
                mine[sl] = slots[sl];
                S->mem_held += (int64_t)slots[sl] * tb[sl];
            }
        s = lane_init(S, L, i, max_q, max_seed, pool_cap, mine);
        if (s != LCD_OK) {
            server_release(S);
            return s;
        }
    }
    S->stats.lanes = n_lanes;
    S->stats.spill_lanes = 0;
    for (int i = 0; i < n_lanes; ++i)
        S->stats.spill_lanes += lane_stage[i] > 0 ? 1 : 0;
    S->stats.max_slots = max_slots;
    S->stats.mem_held = S->mem_held;
    S->stats.spill_tables[0] = slots[0];
    S->stats.spill_tables[1] = slots[1];
    // start-stage routing needs the adjacency on the host: kept for graphs
    // of up to 2^28 entries (1 GiB)
    for (int k = 0; k < S->n_stages; ++k)
        S->stage_cap[k] = S->tp.t[S->stages[k].first].cap;
    if (S->n_stages >= 2 && g->nnz <= ((int64_t)1 << 28)) {
        try {
            S->h_row_ptr.resize((size_t)g->n + 1);
            S->h_col.resize((size_t)std::max<int64_t>(g->nnz, 1));
        } catch (...) {
            server_release(S);
            return fail(LCD_ENOMEM, "host allocation failed");
        }
        hipError_t e = hipMemcpy(S->h_row_ptr.data(), g->row_ptr, sizeof(int32_t) * ((size_t)g->n + 1),
                                 hipMemcpyDeviceToHost);
        if (e == hipSuccess && g->nnz > 0)
            e = hipMemcpy(S->h_col.data(), g->col, sizeof(int32_t) * (size_t)g->nnz, hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            server_release(S);
            return fail(LCD_EDEVICE, "copying the graph to the host: %s", hipGetErrorString(e));
        }
        S->route = true;
    }
    try {
        S->worker = std::thread(worker_main, S);
    } catch (...) {
        server_release(S);
        return fail(LCD_ENOMEM, "could not start the server thread");
    }
    *out = S;
    return LCD_OK;
}

// The first stage whose table holds the query's initial table (its seeds
// and their neighbours): every earlier stage would overflow at once.
// Counting stops past the largest table that leaves a later stage.
static int start_stage(const lcd_server *S, const std::vector<int32_t> &seeds) {
    if (!S->route || S->n_stages < 2)
        return 0;
    const int32_t n = S->g->n;
    thread_local std::vector<uint32_t> stamp;
    thread_local uint32_t epoch = 0;
    if ((int32_t)stamp.size() != n) {
        stamp.assign((size_t)n, 0u);
        epoch = 0;
    }
    if (++epoch == 0) {
        std::fill(stamp.begin(), stamp.end(), 0u);
        epoch = 1;
    }
    const int64_t limit = S->stage_cap[S->n_stages - 2];
    int64_t cnt = 0;
    auto see = [&](int32_t v) {
        if (stamp[v] != epoch) {
            stamp[v] = epoch;
            ++cnt;
        }
    };
    for (int32_t v : seeds) {
        see(v);
        for (int32_t j = S->h_row_ptr[v]; j < S->h_row_ptr[v + 1] && cnt <= limit; ++j)
            see(S->h_col[j]);
        if (cnt > limit)
            break;
    }
    int k = 0;
    while (k + 1 < S->n_stages && cnt > S->stage_cap[k])
        ++k;
    return k;
}

lcd_status lcd_server_submit(lcd_server *S, const int32_t *seeds, int32_t n, double alpha,
                             uint64_t *ticket) {
    if (!S || !ticket)
        return fail(LCD_EINVAL, "null argument");
    if (n < 1 || !seeds)
        return fail(LCD_EINVAL, "a query needs at least one seed node");
    if (!std::isfinite(alpha) || alpha < 0.0 || alpha > 1000.0)
        return fail(LCD_EINVAL, "alpha must be finite and in [0, 1000]");
    Query *q = new (std::nothrow) Query();
    if (!q)
        return fail(LCD_ENOMEM, "host allocation failed");
    q->seeds.assign(seeds, seeds + n);
    std::vector<int32_t> srt(q->seeds);
    std::sort(srt.begin(), srt.end());
    for (int32_t i = 0; i < n; ++i) {
        if (srt[i] < 0 || srt[i] >= S->g->n || (i > 0 && srt[i] == srt[i - 1])) {
            delete q;
            return fail(LCD_EINVAL, "seed nodes must be distinct ids in [0, n)");
        }
    }
    if ((int64_t)n > S->lanes[0].max_seed) {
        delete q;
        return fail(LCD_EINVAL, "a query may hold at most %lld seed nodes", (long long)S->lanes[0].max_seed);
    }
    q->alpha = alpha;
    q->reserve = std::min<int64_t>(S->lanes[0].pool_cap, 4 * (int64_t)n + 2048);
    q->info.t_submit_ns = now_ns();
    const int start = start_stage(S, q->seeds);
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) {
            delete q;
            return fail(LCD_ESTATE, "server is shutting down");
        }
        q->ticket = S->next_ticket++;
        S->tickets[q->ticket] = q;
        if (start > 0 && S->in_flight < S->max_slots) {
            // admitted here, as a query forwarded to that stage would be
            S->in_flight += 1;
            S->forwarded[start].push_back(q);
            S->stats.routed += 1;
        } else {
            S->pending.push_back(q);
        }
        S->stats.submitted += 1;
        *ticket = q->ticket;
    }
    S->cv_work.notify_one();
    return LCD_OK;
}

lcd_status lcd_server_poll(lcd_server *S, uint64_t ticket, int32_t *members, int32_t cap,
                           lcd_query_info *info) {
    if (!S)
        return fail(LCD_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end())
        return fail(LCD_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Query *q = it->second;
    if (!q->done)
        return LCD_EAGAIN;
    if (q->status != LCD_OK) {
        const lcd_status s = fail(q->status, "%s", q->msg.c_str());
        S->tickets.erase(it);
        delete q;
        return s;
    }
    if (info)
        *info = q->info;
    if ((int64_t)cap < (int64_t)q->members.size() || (!members && !q->members.empty()))
        return fail(LCD_ECAPACITY, "the result has %zu members, the buffer holds %d",
                    q->members.size(), cap);
    if (!q->members.empty())
        std::memcpy(members, q->members.data(), sizeof(int32_t) * q->members.size());
    S->tickets.erase(it);
    delete q;
    return LCD_OK;
}

lcd_status lcd_server_wait(lcd_server *S, uint64_t ticket, int32_t timeout_ms) {
    if (!S)
        return fail(LCD_EINVAL, "null server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end())
        return fail(LCD_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Query *q = it->second;
    auto ready = [q] { return q->done; };
    if (timeout_ms < 0)
        S->cv_done.wait(lk, ready);
    else if (!S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
        return LCD_EAGAIN;
    return LCD_OK;
}

lcd_status lcd_server_cancel(lcd_server *S, uint64_t ticket) {
    if (!S)
        return fail(LCD_EINVAL, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end())
        return fail(LCD_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Query *q = it->second;
    if (q->done)
        return q->status == LCD_ECANCELED ? LCD_OK : fail(LCD_ESTATE, "the query has already completed");
    q->cancel = true;
    // waiting for a lane: drop it now (a stage-0 query holds no slot yet, a
    // forwarded one does)
    auto drop = [q](std::deque<Query *> &dq) {
        for (auto d = dq.begin(); d != dq.end(); ++d)
            if (*d == q) {
                dq.erase(d);
                return true;
            }
        return false;
    };
    bool dropped = drop(S->pending);
    for (int k = 1; k < S->n_stages && !dropped; ++k)
        if (drop(S->forwarded[k])) {
            dropped = true;
            S->in_flight -= 1;
        }
    if (dropped) {
        finish_query(S, q);
        S->cv_done.notify_all();
    }
    return LCD_OK;
}

lcd_status lcd_server_get_stats(lcd_server *S, lcd_server_stats *out) {
    if (!S || !out)
        return fail(LCD_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->stats;
    out->pending = (int64_t)S->pending.size();
    out->in_flight = S->in_flight;
    return LCD_OK;
}

lcd_status lcd_server_destroy(lcd_server *S) {
    if (!S)
        return LCD_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable())
        S->worker.join();
    server_release(S);
    return LCD_OK;
}

}  // extern "C"
