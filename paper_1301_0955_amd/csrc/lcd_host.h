// Host-side internals shared by the sweep API (lcd_api.hip) and the query
// server (lcd_server.hip): error reporting, device memory helpers, launch
// planning and the launch sequence of the table tiers.  Not installed.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "lcd.h"
#include "lcd_internal.h"

namespace lcd {

// Sets the calling thread's lcd_last_error() message and returns s.
lcd_status fail(lcd_status s, const char *fmt, ...);

#define HIPCHK(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::lcd::fail(LCD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define CHK(expr)                      \
    do {                               \
        lcd_status s_ = (expr);        \
        if (s_ != LCD_OK)              \
            return s_;                 \
    } while (0)

template <typename T>
lcd_status dev_alloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0)
        count = 1;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(LCD_ENOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T),
                    hipGetErrorString(e));
    }
    return LCD_OK;
}

template <typename T>
void dev_free(T *&p) {
    if (p)
        (void)hipFree((void *)p);
    p = nullptr;
}

// Copy n elements from caller memory (host or device) to a host vector.
template <typename T>
lcd_status fetch(std::vector<T> &dst, const T *src, size_t n, int32_t mem_kind, hipStream_t st) {
    dst.resize(n);
    if (n == 0)
        return LCD_OK;
    if (!src)
        return fail(LCD_EINVAL, "null input array");
    if (mem_kind == LCD_MEM_DEVICE) {
        HIPCHK(hipMemcpyAsync(dst.data(), src, n * sizeof(T), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    } else {
        std::memcpy(dst.data(), src, n * sizeof(T));
    }
    return LCD_OK;
}

inline int next_pow2_bits(int64_t x) {
    int b = 0;
    while (((int64_t)1 << b) < x)
        ++b;
    return b;
}

struct DevInfo {
    int64_t wall_khz = 100000;   // wall_clock64() rate
    int device = -1;
    int cus = 0;
    int64_t lds_cu = 0;
    int64_t lds_block = 0;
    char arch[64] = {0};
};

lcd_status device_info(DevInfo &d);

// Global-memory table workspace of one spill tier.
struct Slab {
    char *buf = nullptr;
    int64_t stride = 0;
    int32_t cap = 0;
    int32_t hbits = 0;
    int32_t slots = 0;
    bool dirty = false;
};

// pool cursor, error word, then kStatWords statistics per tier
constexpr int kCursorWords = 2 + kStatWords * kMaxTiers;

// The table size from which a growth call keeps its queue bucketed by rank.
inline int32_t queue_min_of(const lcd_params &p) {
    return p.queue_min_entries > 0 ? p.queue_min_entries : 1024;
}

// One tier of the launch chain.
struct TierSpec {
    int32_t kind;      // TIER_*
    int32_t cap;       // table entries per community
    int32_t hbits;     // hash slots = 2^hbits
    int32_t waves;     // waves per workgroup
    int32_t blocks;    // workgroups of an LDS tier (tier 0: the full-size grid)
    int32_t slots;     // global tiers: tables wanted in the slab
    int32_t slab;      // global tiers: slab index; -1 for LDS tiers
};

struct TierPlan {
    int32_t n = 0;
    TierSpec t[kMaxTiers];
};

inline int64_t slab_stride(int32_t cap) {
    return (global_table_bytes(cap, next_pow2_bits(2 * (int64_t)cap)) + 255) / 256 * 256;
}

// The tier chain for a graph of n nodes: tier 0 one wave per community with
// an LDS table (lds_capacity entries), then tiers with larger tables.
// spill_mode 0: workgroup tiers (LDS table of 4,096 entries, global tables of
// 16,384 entries, global tables that hold every node); 1: one-wave global
// tiers (16,384 entries x 4,096 tables, then every node).
lcd_status plan_tiers(const DevInfo &dev, int32_t n, const lcd_params &p, TierPlan &tp);

// (Re)allocate a slab for cap entries x slots tables and mark every hash
// slot empty; a clean slab of the same shape is kept as it is.
lcd_status ensure_slab(Slab &sl, int32_t cap, int32_t slots, hipStream_t st);

// Enqueue one launch group on st: tiers first .. last-1 of tp in order, tier
// k > 0 fed by the overflow queue work[k - 1] (count in ctl->ovf_count[k-1])
// of the tier before it; tier 0 runs with blocks0 workgroups.  With
// `ordered` (null, or one buffer per queue) and a launch over several
// scales, each queue is first copied into ordered[k - 1] by ascending
// overflow scale and the tier reads that.  ev (null, or one event per tier
// plus one) is recorded before each tier and at the end.
lcd_status enqueue_tiers(const SweepArgs &a, const TierPlan &tp, int first, int last, int32_t blocks0,
                         Slab *slabs, int32_t *const *work, int32_t *const *ordered, hipStream_t st,
                         hipEvent_t *ev, int32_t *launches);

}  // namespace lcd

struct lcd_graph;

namespace lcd {
// Launch parameters all left at 0: the sizing fields come from the graph's
// tuned set when lcd_tune() has run on it.
bool params_are_auto(const lcd_params &p);
void apply_tuned(const lcd_graph *g, lcd_params &p);
}  // namespace lcd

struct lcd_graph {
    int32_t n = 0;
    int64_t nnz = 0;
    int64_t maxk = 0;
    int64_t volume = 0;
    int device = -1;
    int32_t *row_ptr = nullptr;
    int32_t *col = nullptr;
    uint8_t *w = nullptr;
    int32_t *kdeg = nullptr;
    double *logtab = nullptr;
    int32_t logtab_n = 0;
    lcd::DevInfo dev;
    lcd::Slab slab[2];          // spill-tier tables of lcd_sweep on this graph
    int64_t pool_hint = 0;
    // batch graphs: node and edge offsets of each member graph (host copy)
    std::vector<int64_t> node_off, edge_off;
    // launch sizing chosen by lcd_tune() for this graph
    bool tuned = false;
    lcd_params tuned_prm{};
    // lcd_seeds' device workspace, kept for the next call
    char *seed_ws = nullptr;
    int64_t seed_ws_bytes = 0;
};

static inline lcd::GraphDev graph_dev(const lcd_graph *g) {
    lcd::GraphDev d;
    d.row_ptr = g->row_ptr;
    d.col = g->col;
    d.w = g->w;
    d.kdeg = g->kdeg;
    d.logtab = g->logtab;
    d.n = g->n;
    d.logtab_n = g->logtab_n;
    return d;
}
