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

// pool cursor, error word, then 5 statistics per tier
constexpr int kCursorWords = 2 + 5 * 3 + 1;

struct TierPlan {
    int32_t cap0, hbits0, wpb0, blocks0;
    int32_t cap1, cap2;
    bool use1, use2;
};

// LDS table size, waves per block and grid of the LDS tier, and which
// global-memory tiers a graph of n nodes needs.
lcd_status plan_tiers(const DevInfo &dev, int32_t n, const lcd_params &p, TierPlan &tp);

// (Re)allocate a slab for cap entries x slots tables and mark every hash
// slot empty; a clean slab of the same shape is kept as it is.
lcd_status ensure_slab(Slab &sl, int32_t cap, int32_t slots, hipStream_t st);

// Enqueue one launch group on st: the LDS tier over a.n_sets items with
// blocks0 workgroups, then every global-memory tier tp enables, each fed by
// the overflow queue of the tier before it.  ev (3 events, or null) is
// recorded before the LDS tier, between the tiers and at the end.
lcd_status enqueue_tiers(const SweepArgs &a, const TierPlan &tp, int32_t blocks0, Slab *slabs,
                         int32_t *const work[2], hipStream_t st, hipEvent_t *ev,
                         int32_t *launches);

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
    // tuned launch parameters, keyed by the sweep shape they were tuned on
    bool tuned = false;
    int32_t tuned_n_sets = 0, tuned_S = 0;
    int32_t tuned_cap = 0, tuned_wpb = 0;
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
