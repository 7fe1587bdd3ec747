// lcd_sweep_into: the sweep of lcd_sweep for callers that cannot allocate
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  The caller passes device inputs and device outputs; the
// library's own working memory (work queues, counters, the global-memory
// tables of the workgroup tier) lives in one static device array of fixed
// size, `scratch`, and nothing is allocated on the device or the host.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "lcd.h"
#include "lcd_host.h"
#include "lcd_internal.h"

namespace lcd {
namespace {

// Limits of the static working memory (also stated in lcd.h).
constexpr int32_t kNaMaxSets = LCD_NOALLOC_MAX_SETS;
constexpr int32_t kNaMaxScales = LCD_NOALLOC_MAX_SCALES;
constexpr int32_t kNaMaxSeedSet = LCD_NOALLOC_MAX_SEED_SET;
constexpr int32_t kNaTableCap = LCD_NOALLOC_TABLE_ENTRIES;
constexpr int32_t kNaTables = LCD_NOALLOC_TABLES;

// Layout of the scratch array (byte offsets, each 256-aligned).
constexpr int64_t kNaCtl = 0;                                    // Counters
constexpr int64_t kNaCursor = 256;                               // kCursorWords x u64
constexpr int64_t kNaCheck = kNaCursor + 512;                    // validation verdict (u32)
constexpr int64_t kNaWork = kNaCheck + 256;                      // 6 x kNaMaxSets int32
constexpr int64_t kNaSlab = kNaWork + (int64_t)6 * kNaMaxSets * 4;
constexpr int64_t kNaStride = (global_table_bytes(kNaTableCap, 15) + 255) / 256 * 256;
constexpr int64_t kNaBytes = kNaSlab + kNaTables * kNaStride;
static_assert(kCursorWords * 8 <= 512, "cursor words fit their slot");
static_assert(((int64_t)1 << 15) >= 2 * (int64_t)kNaTableCap, "hash bits of the workgroup tier");
static_assert(kNaBytes <= LCD_NOALLOC_SCRATCH_BYTES, "scratch layout fits the stated size");

// The working memory of every call on one GPU.  In host code this name is a
// host-side stand-in, not a device address: host code only ever uses the
// per-device address that hipGetSymbolAddress returns for it.
static __device__ __align__(256) char scratch[LCD_NOALLOC_SCRATCH_BYTES];

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;
char *g_na_ptr[kNaMaxDevices] = {};

// The scratch array's device address on the current device, looked up once
// per device with that device current.
lcd_status scratch_ptr(int device, char **out) {
    if (device < 0 || device >= kNaMaxDevices)
        return fail(LCD_EDEVICE, "device %d outside the %d the library tracks", device, kNaMaxDevices);
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LCD_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_na_ptr[device] = (char *)p;
    }
    *out = g_na_ptr[device];
    return LCD_OK;
}

enum : uint32_t {
    NA_BAD_PTR = 1u,        // seed_ptr[0] != 0 or a set is empty
    NA_BAD_SEED = 2u,       // a seed id outside [0, n)
    NA_DUP_SEED = 4u,       // a seed id repeated within its set
    NA_BAD_SCALE = 8u,      // a scale not finite, outside [0, 1000] or not decreasing
    NA_BIG_SET = 16u        // a seed set longer than LCD_NOALLOC_MAX_SEED_SET
};

// The input rules of lcd_sweep, checked on the device (reading the inputs
// on the host would need a host buffer).  One thread per seed position
// (repeats: compared with the earlier positions of its set), one per scale
// and one per set boundary; any breach ORs its bit into *verdict.
__global__ void check_inputs_kernel(const int32_t *seed_ptr, const int32_t *seed_nodes, int32_t n_sets,
                                    const double *scales, int32_t n_scales, int32_t n, int64_t total,
                                    uint32_t *verdict) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_sets; t += stride) {
        const int32_t a = seed_ptr[t], b = seed_ptr[t + 1];
        uint32_t bad = 0;
        if (b <= a)
            bad |= NA_BAD_PTR;
        if (b - a > kNaMaxSeedSet)
            bad |= NA_BIG_SET;
        if ((t == 0 && a != 0) || (t == n_sets - 1 && (int64_t)b != total))
            bad |= NA_BAD_PTR;
        if (bad)
            atomicOr(verdict, bad);
    }
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_scales; s += stride) {
        const double x = scales[s];
        if (!(x >= 0.0 && x <= 1000.0) || (s > 0 && !(x < scales[s - 1])))
            atomicOr(verdict, NA_BAD_SCALE);
    }
    // positions are checked only when the offsets are sane (seed_ptr has
    // been read above by other threads; a broken one is reported first)
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += stride) {
        const int32_t u = seed_nodes[q];
        if (u < 0 || u >= n) {
            atomicOr(verdict, NA_BAD_SEED);
            continue;
        }
        // the set holding position q, by binary search over the offsets
        int32_t lo = 0, hi = n_sets - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if ((int64_t)seed_ptr[mid] <= q)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int64_t a = seed_ptr[lo];
        if (a < 0 || a > q || q - a > kNaMaxSeedSet)
            continue;   // broken offsets or a long set: reported above
        for (int64_t p = a; p < q; ++p)
            if (seed_nodes[p] == u) {
                atomicOr(verdict, NA_DUP_SEED);
                break;
            }
    }
}

}  // namespace
}  // namespace lcd

using namespace lcd;

extern "C" lcd_status lcd_sweep_into(const lcd_graph *g, const double *scales, int32_t n_scales,
                                     const int32_t *seed_ptr, const int32_t *seed_nodes, int32_t n_sets,
                                     int64_t n_seed_nodes, const lcd_params *params, int64_t *rec_off,
                                     int32_t *rec_cnt, int64_t *rec_k, int64_t *rec_v, double *rec_f,
                                     uint64_t *rec_ctr, int32_t *members, int64_t members_cap,
                                     int64_t *members_used, void *stream) {
    if (!g || !members_used)
        return fail(LCD_EINVAL, "null graph or members_used");
    if (n_scales < 1 || n_scales > kNaMaxScales)
        return fail(LCD_EINVAL, "n_scales must be in [1, %d]", kNaMaxScales);
    if (n_sets < 0 || n_sets > kNaMaxSets)
        return fail(LCD_EINVAL, "n_sets must be in [0, %d]", kNaMaxSets);
    if (n_seed_nodes < n_sets || n_seed_nodes > (int64_t)n_sets * kNaMaxSeedSet)
        return fail(LCD_EINVAL, "n_seed_nodes must lie between n_sets and n_sets x %d", kNaMaxSeedSet);
    if (members_cap < 0)
        return fail(LCD_EINVAL, "members_cap must be >= 0");
    if (n_sets > 0 && (!scales || !seed_ptr || !seed_nodes || !rec_off || !rec_cnt || !rec_k || !rec_v ||
                       !rec_f || !rec_ctr || (members_cap > 0 && !members)))
        return fail(LCD_EINVAL, "null device array");
    lcd_params prm;
    lcd_params_default(&prm);
    if (params)
        prm = *params;
    if (prm.mode != LCD_PERSISTENT || prm.use_graph)
        return fail(LCD_EINVAL, "lcd_sweep_into runs the persistent launch only (no mode, no use_graph)");
    if (prm.watchdog_ms == 0)
        prm.watchdog_ms = 20000;
    if (prm.grow_calls < 0)
        return fail(LCD_EINVAL, "grow_calls must be >= 0");
    apply_tuned(g, prm);
    if (prm.spill_mode != 0)
        return fail(LCD_EINVAL, "lcd_sweep_into supports spill_mode 0 (workgroup tiers) only");
    *members_used = 0;
    if (n_sets == 0)
        return LCD_OK;
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev != g->device)
        return fail(LCD_EINVAL, "the graph lives on device %d, the current device is %d", g->device, dev);
    char *base = nullptr;
    CHK(scratch_ptr(dev, &base));
    hipStream_t st = (hipStream_t)stream;

    // the tier chain of lcd_sweep, cut after its first global-memory tier,
    // whose tables come from the scratch array
    TierPlan full;
    CHK(plan_tiers(g->dev, g->n, prm, full));
    TierPlan tp;
    for (int k = 0; k < full.n; ++k) {
        TierSpec T = full.t[k];
        if (T.slab >= 0) {
            if (T.kind != TIER_TEAM_GLOBAL || T.cap > kNaTableCap)
                break;
            T.cap = kNaTableCap;
            T.hbits = 15;
            T.slots = kNaTables;
            T.slab = 0;
            tp.t[tp.n++] = T;
            break;
        }
        tp.t[tp.n++] = T;
    }
    Slab slab[2];
    slab[0].buf = base + kNaSlab;
    slab[0].stride = kNaStride;
    slab[0].cap = kNaTableCap;
    slab[0].hbits = 15;
    slab[0].slots = kNaTables;

    // check the inputs, then clear the queues, counters and table hashes
    uint32_t *verdict = (uint32_t *)(base + kNaCheck);
    HIPCHK(launch_zero_bytes(verdict, 4, st));
    hipLaunchKernelGGL(check_inputs_kernel, dim3(256), dim3(256), 0, st, seed_ptr, seed_nodes, n_sets, scales,
                       n_scales, g->n, n_seed_nodes, verdict);
    HIPCHK(hipGetLastError());
    uint32_t bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, verdict, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad)
        return fail(bad & NA_BIG_SET ? LCD_ECAPACITY : LCD_EINVAL,
                    "inputs rejected (0x%x: %s%s%s%s%s)", bad, bad & NA_BAD_PTR ? "seed_ptr " : "",
                    bad & NA_BAD_SEED ? "seed id out of range " : "", bad & NA_DUP_SEED ? "repeated seed " : "",
                    bad & NA_BAD_SCALE ? "scales " : "", bad & NA_BIG_SET ? "seed set too long" : "");
    HIPCHK(launch_zero_bytes(base + kNaCtl, sizeof(Counters), st));
    HIPCHK(launch_zero_bytes(base + kNaCursor, 8 * kCursorWords, st));
    if (tp.n > 0 && tp.t[tp.n - 1].slab >= 0)
        HIPCHK(launch_fill_i32((int32_t *)slab[0].buf, -1, kNaStride * kNaTables / 4, st));

    SweepArgs a{};
    a.g = graph_dev(g);
    a.scales = scales;
    a.alpha_set = nullptr;
    a.S = n_scales;
    a.s_begin = 0;
    a.s_end = n_scales;
    a.seed_ptr = seed_ptr;
    a.seed_nodes = seed_nodes;
    a.n_sets = n_sets;
    a.k_prune = prm.k_prune;
    a.max_calls = prm.grow_calls > 0 ? (uint32_t)prm.grow_calls : 0u;
    a.queue_min = queue_min_of(prm);
    a.resume = 0;
    a.rec.off = rec_off;
    a.rec.cnt = rec_cnt;
    a.rec.K = rec_k;
    a.rec.V = rec_v;
    a.rec.f = rec_f;
    a.rec.ctr = rec_ctr;
    a.pool = members;
    a.pool_cap = members_cap;
    a.ctl = (Counters *)(base + kNaCtl);
    unsigned long long *cursor = (unsigned long long *)(base + kNaCursor);
    a.pool_cursor = cursor;
    a.err = (uint32_t *)(cursor + 1);
    a.stat = cursor + 2;
    a.budget_ticks = prm.watchdog_ms < 0 ? 0 : g->dev.wall_khz * (int64_t)prm.watchdog_ms;
    int32_t *work[kMaxTiers - 1], *ordered[kMaxTiers - 1];
    for (int k = 0; k < kMaxTiers - 1; ++k) {
        work[k] = (int32_t *)(base + kNaWork) + (int64_t)k * kNaMaxSets;
        ordered[k] = (int32_t *)(base + kNaWork) + (int64_t)(3 + k) * kNaMaxSets;
    }
    int32_t launches = 0;
    CHK(enqueue_tiers(a, tp, 0, tp.n, tp.t[0].blocks, slab, work, ordered, st, nullptr, &launches));
    unsigned long long cur[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(cur, cursor, sizeof(cur), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *members_used = (int64_t)cur[0];
    const uint32_t err = (uint32_t)(cur[1] & 0xffffffffu);
    if (err & ERR_CAPACITY)
        return fail(LCD_ECAPACITY, "a seed set's table outgrew %d entries, the largest that lcd_sweep_into holds",
                    kNaTableCap);
    if (err)
        return fail(LCD_EDEVICE, "sweep kernel reported error bits 0x%x%s", err,
                    err & ERR_TIMEOUT ? " (watchdog: a seed set ran past its time budget)" : "");
    if ((int64_t)cur[0] > members_cap)
        return fail(LCD_ECAPACITY, "members buffer holds %lld entries, %lld needed", (long long)members_cap,
                    (long long)cur[0]);
    return LCD_OK;
}
