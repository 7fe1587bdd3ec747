// Kernels of the multi-scale local community sweep for gfx950 (CDNA4, wave64).
//
// One wavefront grows one community through every scale (paper Sec. 2,
// Algorithm 1, chained over scales as in Algorithm 2).  Per community the
// wave keeps a table of every node it has touched:
//   open-addressing hash  node id -> dense index   (int32 slots, 2^hbits >= 2 cap)
//   dense arrays          node id, d_in | flags, weighted degree k, rank R
// held in LDS (tier 0) or, for communities that outgrow the LDS table, in a
// per-wave slab of global memory (tiers 1 and 2, same code).
//
// The sequential priority queue of Algorithm 1 is emulated exactly:
//   * every live (queued) entry is tested against the current (K, V); the
//     highest-ranked improving entry e* is the one the queue would add next,
//     and every live entry ranked above e* would have been popped and
//     rejected against the same state first.  Those pops are applied lazily:
//     the next pass drops a live entry ranked above the previous e* unless
//     the addition of e* touched it (flag FRESH), which is exactly the
//     queue update that Algorithm 1 applies to the neighbours of an added
//     node.
//   * the number of pops G is counted where entries enter the queue (every
//     entry that enters is popped exactly once before the queue empties).
//   * a removal pass visits members in ascending id: each step finds the
//     smallest removable id above the cursor with a wave min-reduction.
// Decisions use only exact integer sums and the integer log L below, in
// the same IEEE operation order as the specification, so the result is
// bit-identical to a sequential evaluation.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lcd_internal.h"

namespace lcd {

namespace {

constexpr double kMargin = 0x1p-40;   // improvement threshold on the log-fitness gain
constexpr double kFilter = 1e-9;      // certified pre-test margin (see improves_add)
constexpr uint32_t kDMask = (1u << 27) - 1;   // d (weighted degrees stay below 2^27)
constexpr uint32_t kMember = 1u << 31;
constexpr uint32_t kLive = 1u << 30;
constexpr uint32_t kFresh = 1u << 29;
// delta output: member at the set's last emitted record
constexpr uint32_t kWas = 1u << 28;
// bucketed queue: re-ranked by the latest addition, not yet seen by a
// fresh-list scan
constexpr uint32_t kTouch = 1u << 27;

// ---------------------------------------------------------------------------
// L(x): natural log of an integer 1 <= x < 2^53.  x = m 2^e with m in
// (sqrt(2)/2, sqrt(2)]; ln m = 2 atanh(s), s = (m-1)/(m+1), by the series
// 2 s (1 + z/3 + ... + z^11/23) with z = s^2; ln 2 as a Cody-Waite pair so
// that e * ln2_hi is exact.  Plain IEEE operations, no contraction.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double ilog(uint64_t x) {
    int e = 63 - __builtin_clzll(x);
    double m = (double)x * __longlong_as_double((long long)(1023 - e) << 52);
    if (m > 0x1.6a09e667f3bcdp+0) {
        m = m * 0.5;
        e = e + 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
    double p = 1.0 / 23.0;
    p = p * z + 1.0 / 21.0;
    p = p * z + 1.0 / 19.0;
    p = p * z + 1.0 / 17.0;
    p = p * z + 1.0 / 15.0;
    p = p * z + 1.0 / 13.0;
    p = p * z + 1.0 / 11.0;
    p = p * z + 1.0 / 9.0;
    p = p * z + 1.0 / 7.0;
    p = p * z + 1.0 / 5.0;
    p = p * z + 1.0 / 3.0;
    p = p * z + 1.0;
    double h = s * p;
    double lnm = h + h;
    double de = (double)e;
    return de * 6.93147180369123816490e-01 + (de * 1.90821492927058770002e-10 + lnm);
}

__device__ __forceinline__ uint64_t lanes_below(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Ordering point between table phases of one wave.  LDS operations of a
// wave execute in order, so only the compiler must be fenced; global
// tables additionally wait for outstanding memory operations.
template <bool GLOBAL>
__device__ __forceinline__ void wsync() {
    if constexpr (GLOBAL)
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    else
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t hash_of(int32_t u, int hbits) {
    return ((uint32_t)u * 2654435761u) >> (32 - hbits);
}

// true when (r, u) pops before (pr, pu): higher rank, then smaller id
__device__ __forceinline__ bool before(double r, int32_t u, double pr, int32_t pu) {
    return r > pr || (r == pr && u < pu);
}

// A community's table.  Field f of entry i is at fb + i * fs: separate
// arrays in LDS tables and small global tables (a scan reads one field of
// consecutive entries), one 32-byte record per entry in global tables of
// kRecordMinEntries or more (a step reads the fields of entries it reaches
// through the queue or the fresh list at random: one cache line per entry
// instead of four; 19 % off the 10M-node sweep, 2 % slower on 16,384-entry
// tables, which stay arrays).
struct Tab {
    char *rkb, *nodeb, *dvb, *kvb;
    uint32_t rks, nodes, dvs, kvs;
    __device__ __forceinline__ double &RK(int32_t i) const { return *(double *)(rkb + (uint32_t)i * rks); }
    __device__ __forceinline__ int32_t &NODE(int32_t i) const { return *(int32_t *)(nodeb + (uint32_t)i * nodes); }
    __device__ __forceinline__ uint32_t &DV(int32_t i) const { return *(uint32_t *)(dvb + (uint32_t)i * dvs); }
    __device__ __forceinline__ int32_t &KV(int32_t i) const { return *(int32_t *)(kvb + (uint32_t)i * kvs); }
    int32_t *scr;
    int32_t *hs;      // hash slots: entry index (LDS and array-layout tables)
    uint64_t *hp;     // hash slots: node id << 32 | entry index (record tables)
    int32_t *sq;      // global tables: rank-bucketed queue (entry indices)
    int32_t *fr;      // global tables: fresh list (entry indices)
    uint32_t hmask;
    int hbits;
    int cap;
};

// LDS table: rank f64[cap], node i32[cap], d|flags u32[cap], degree
// i32[cap], scratch i32[cap], hash slots i32[2^hbits].
__device__ __forceinline__ Tab carve(char *base, int cap, int hbits) {
    Tab t;
    t.rkb = base;
    t.nodeb = base + (size_t)cap * 8;
    t.dvb = base + (size_t)cap * 12;
    t.kvb = base + (size_t)cap * 16;
    t.rks = 8;
    t.nodes = t.dvs = t.kvs = 4;
    t.scr = (int32_t *)(base + (size_t)cap * 20);
    t.hs = (int32_t *)(base + (size_t)cap * 24);
    t.hp = nullptr;
    t.sq = nullptr;
    t.fr = nullptr;
    t.hbits = hbits;
    t.hmask = (1u << hbits) - 1;
    t.cap = cap;
    return t;
}

// Global table: the LDS layout then the bucketed queue i32[cap] and the
// fresh list i32[cap]; from kRecordMinEntries entries on, records
// {d|flags u32, node i32, degree i32, -, rank f64, -} of kRecordBytes, then
// scratch i32[cap] (padded to 8 bytes), hash slots u64[2^hbits] of
// node << 32 | index, queue and fresh list.
template <bool REC>
__device__ __forceinline__ Tab carve_global_as(char *base, int cap, int hbits) {
    if constexpr (!REC) {
        Tab t = carve(base, cap, hbits);
        char *q = base + table_bytes(cap, hbits);
        t.sq = (int32_t *)q;
        t.fr = (int32_t *)(q + (size_t)cap * 4);
        return t;
    } else {
        Tab t;
        t.dvb = base;
        t.nodeb = base + 4;
        t.kvb = base + 8;
        t.rkb = base + 16;
        t.rks = t.nodes = t.dvs = t.kvs = kRecordBytes;
        char *p = base + (size_t)cap * kRecordBytes;
        t.scr = (int32_t *)p;
        const size_t scr_bytes = ((size_t)cap * 4 + 7) & ~(size_t)7;
        t.hs = nullptr;
        t.hp = (uint64_t *)(p + scr_bytes);
        char *q = p + scr_bytes + ((size_t)1 << hbits) * kPairSlotBytes;
        t.sq = (int32_t *)q;
        t.fr = (int32_t *)(q + (size_t)cap * 4);
        t.hbits = hbits;
        t.hmask = (1u << hbits) - 1;
        t.cap = cap;
        return t;
    }
}

// The layout a global table of cap entries has.
__device__ __forceinline__ Tab carve_global(char *base, int cap, int hbits) {
    return cap >= kRecordMinEntries ? carve_global_as<true>(base, cap, hbits)
                                    : carve_global_as<false>(base, cap, hbits);
}

template <bool GLOBAL>
__device__ __forceinline__ int32_t hs_load(const int32_t *p) {
    if constexpr (GLOBAL)
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        return *p;
}

template <bool GLOBAL>
__device__ __forceinline__ void hs_store(int32_t *p, int32_t v) {
    if constexpr (GLOBAL)
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

// Per-wave state.  Every field except the lane partial counters holds the
// same value in all lanes.
struct St {
    int32_t count;     // dense entries in use
    int32_t nmem;      // members
    int64_t K, V;      // k_in and volume of the community
    double LK, LV;     // L(K), L(V) when positive
    double alpha;
    double pr;         // rank and id of the entry added last in this call
    int32_t pu;
    uint32_t Gl, Rl;   // lane partial counts of pops and rank computations
    uint64_t Gu;       // wave-uniform part of G (removal-pass visits)
    uint64_t M;        // moves in this (set, scale)
    bool ovf;          // the table ran out of entries
    uint32_t err;
    int64_t move_limit; // guard against a runaway loop in one (set, scale)
    uint64_t t0;        // wall clock when the set started
    uint64_t budget;    // wall-clock ticks the set may take
    uint64_t rows;      // CSR rows gathered (moves and initial members)
    uint64_t row_len;   // ... and their total length
    uint64_t inserted;  // table entries created (one degree read each)
    uint64_t written;   // member ids written to the pool
    uint64_t scanned;   // table entries visited by the growth scans
    // algorithmic work, committed when a scale's record is written (work of
    // a scale that overflows is redone in the next tier and not counted)
    uint64_t mrows, mrow_len;       // rows gathered by moves, running totals
    uint64_t c_mrows, c_mrow_len;   // ... at the last record written
    uint64_t ins_mark, c_ins;       // entries created: not counted before ins_mark;
                                    // committed count at the last record written
    uint64_t srows, srow_len;       // seed-set rows of a set in its first tier
    bool emitted;                   // a record was written in this tier
};

// Watchdog: a seed set that runs past its budget stops with ERR_TIMEOUT, so
// a logic error ends the sweep with an error instead of running on.
__device__ __forceinline__ bool over_budget(St &st) {
    if (wall_clock64() - st.t0 > st.budget) {
        st.err |= ERR_TIMEOUT;
        return true;
    }
    return false;
}

struct Ctx {
    const int32_t *row_ptr;
    const int32_t *col;
    const uint8_t *w;
    const int32_t *kdeg;
    const double *logtab;
    int32_t logtab_last;   // largest valid index of logtab
    int32_t n;             // nodes
};

// queue rank R(d, k) = L(2d) - alpha L(k); 2d <= 2k <= 2 max degree, so both
// logs come from the table (the clamp only keeps a broken table in bounds)
__device__ __forceinline__ double rank_of(const Ctx &c, int32_t d, int32_t k, double alpha) {
    const int32_t i2 = min(2 * d, c.logtab_last);
    const int32_t ik = min(k, c.logtab_last);
    return c.logtab[i2] - alpha * c.logtab[ik];
}

constexpr uint64_t kEmptyPair = ~0ull;   // node -1, index -1

template <bool GLOBAL>
__device__ __forceinline__ int32_t tab_find(const Tab &t, int32_t u, uint32_t &err) {
    uint32_t p = hash_of(u, t.hbits);
    if constexpr (GLOBAL) {
        if (t.hp) {
            for (uint32_t it = 0; it <= t.hmask; ++it) {
                const uint64_t s = __hip_atomic_load(&t.hp[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (s == kEmptyPair)
                    return -1;
                if ((int32_t)(uint32_t)(s >> 32) == u)
                    return (int32_t)(uint32_t)s;
                p = (p + 1) & t.hmask;
            }
            err |= ERR_PROBE;
            return -1;
        }
    }
    for (uint32_t it = 0; it <= t.hmask; ++it) {
        int32_t i = hs_load<GLOBAL>(&t.hs[p]);
        if (i < 0)
            return -1;
        if (t.NODE(i) == u)
            return i;
        p = (p + 1) & t.hmask;
    }
    err |= ERR_PROBE;
    return -1;
}

// Put entry idx of node u into its hash slot (linear probing).
template <bool GLOBAL>
__device__ __forceinline__ void tab_slot_insert(const Tab &t, int32_t u, int32_t idx, uint32_t &err) {
    uint32_t p = hash_of(u, t.hbits);
    uint32_t it = 0;
    if (GLOBAL && t.hp) {
        const uint64_t v = ((uint64_t)(uint32_t)u << 32) | (uint32_t)idx;
        for (; it <= t.hmask; ++it) {
            if (atomicCAS((unsigned long long *)&t.hp[p], (unsigned long long)kEmptyPair,
                          (unsigned long long)v) == (unsigned long long)kEmptyPair)
                break;
            p = (p + 1) & t.hmask;
        }
    } else {
        for (; it <= t.hmask; ++it) {
            if (atomicCAS(&t.hs[p], -1, idx) == -1)
                break;
            p = (p + 1) & t.hmask;
        }
    }
    if (it > t.hmask)
        err |= ERR_PROBE;
}

// Empty the hash slot of entry i (global tables, before the slab's next
// community).
template <bool GLOBAL>
__device__ __forceinline__ void tab_slot_clear(const Tab &t, int32_t i) {
    uint32_t p = hash_of(t.NODE(i), t.hbits);
    for (uint32_t it = 0; it <= t.hmask; ++it) {
        if (t.hp) {
            const uint64_t s = __hip_atomic_load(&t.hp[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((int32_t)(uint32_t)s == i) {
                __hip_atomic_store(&t.hp[p], kEmptyPair, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
        } else if (hs_load<GLOBAL>(&t.hs[p]) == i) {
            hs_store<GLOBAL>(&t.hs[p], -1);
            return;
        }
        p = (p + 1) & t.hmask;
    }
}

// Dense index of u for every active lane, inserting absent ids.  All active
// ids of one call are distinct.  Returns -1 for inactive lanes, and for all
// lanes when the table would overflow (st.ovf is then set).
template <bool GLOBAL>
__device__ int32_t tab_ensure(const Tab &t, St &st, const Ctx &c, bool act, int32_t u, int lane) {
    int32_t idx = act ? tab_find<GLOBAL>(t, u, st.err) : -1;
    bool need = act && idx < 0;
    uint64_t m = __ballot(need);
    if (m == 0)
        return idx;
    int nn = __popcll(m);
    if (st.count + nn > t.cap) {
        st.ovf = true;
        return -1;
    }
    st.inserted += (uint64_t)nn;
    if (need) {
        idx = st.count + __popcll(m & lanes_below(lane));
        t.NODE(idx) = u;
        t.KV(idx) = c.kdeg[u];
        t.DV(idx) = 0u;
        tab_slot_insert<GLOBAL>(t, u, idx, st.err);
    }
    st.count += nn;
    wsync<GLOBAL>();
    return idx;
}

enum { ROW_INIT = 0, ROW_ADD = 1, ROW_REMOVE = 2 };

// Apply the edges of node n to the table: d_in += w for INIT and ADD,
// d_in -= w for REMOVE.  For ADD, every non-member neighbour is (re)queued
// with its new rank (the queue update of Algorithm 1).
template <bool GLOBAL, int MODE>
__device__ void row_update(const Tab &t, St &st, const Ctx &c, int32_t n, int lane) {
    const int32_t beg = c.row_ptr[n];
    const int32_t end = c.row_ptr[n + 1];
    st.rows += 1;
    st.row_len += (uint64_t)(end - beg);
    if constexpr (MODE != ROW_INIT) {
        st.mrows += 1;
        st.mrow_len += (uint64_t)(end - beg);
    }
    for (int32_t base = beg; base < end; base += 64) {
        const int32_t j = base + lane;
        const bool act = j < end;
        const int32_t u = act ? c.col[j] : 0;
        const int32_t wt = act ? (c.w ? (int32_t)c.w[j] : 1) : 0;
        int32_t idx;
        if constexpr (MODE == ROW_REMOVE) {
            idx = act ? tab_find<GLOBAL>(t, u, st.err) : -1;
            if (act && idx < 0)
                st.err |= ERR_MISSING;
        } else {
            idx = tab_ensure<GLOBAL>(t, st, c, act, u, lane);
            if (st.ovf)
                return;
        }
        if (act && idx >= 0) {
            const uint32_t v = t.DV(idx);
            int32_t d = (int32_t)(v & kDMask);
            if constexpr (MODE == ROW_REMOVE) {
                d -= wt;
                t.DV(idx) = (v & ~kDMask) | (uint32_t)d;
            } else if constexpr (MODE == ROW_INIT) {
                d += wt;
                t.DV(idx) = (v & ~kDMask) | (uint32_t)d;
            } else {
                d += wt;
                if (v & kMember) {
                    t.DV(idx) = (v & ~kDMask) | (uint32_t)d;
                } else {
                    // still queued unless popped and rejected above the node just added
                    const bool queued = (v & kLive) && !before(t.RK(idx), u, st.pr, st.pu);
                    if (!queued)
                        st.Gl += 1;
                    const int32_t k = t.KV(idx);
                    t.RK(idx) = rank_of(c, d, k, st.alpha);
                    st.Rl += 1;
                    t.DV(idx) = (v & kWas) | (uint32_t)d | kLive | kFresh;
                }
            }
        }
    }
    wsync<GLOBAL>();
}

// Full decision "f(Kp, Vp) > f(K, V)" in the log domain (K, V > 0 here).
__device__ __forceinline__ bool decide(const St &st, int64_t Kp, int64_t Vp) {
    if (Kp == 0)
        return false;
    if (st.K == 0)
        return true;
    const double a = ilog((uint64_t)Kp) - st.LK;
    const double b = ilog((uint64_t)Vp) - st.LV;
    const double cc = st.alpha * b;
    const double t = a - cc;
    return t > kMargin;
}

// Would adding a non-member with (d, k) raise f?  The pre-test uses
// ln(1+x) <= x and ln(1+y) >= y/(1+y):  the exact gain is at most
//   2d/K - alpha k/(V+k),
// evaluated multiplied out by K (V+k) (every product of integers below 2^53
// is exact); when that bound is below -1e-9 the exact gain, and therefore
// the computed one (error < 1e-11 for alpha <= 1000), is far below the
// threshold, so the full test would reject as well.
__device__ __forceinline__ bool improves_add(const St &st, int32_t d, int32_t k) {
    if (st.K == 0)
        return true;
    const int64_t Kp = st.K + 2 * (int64_t)d;
    const int64_t Vp = st.V + k;
    const double X = (double)(2 * (int64_t)d) * (double)Vp - st.alpha * ((double)k * (double)st.K);
    if (X < -kFilter * ((double)st.K * (double)Vp))
        return false;
    return decide(st, Kp, Vp);
}

// Would removing a member with internal weight d and degree k raise f?
// Bound: ln(1-x) <= -x and -ln(1-y) <= y/(1-y) give a gain of at most
//   -2d/K + alpha k/(V-k).
__device__ __forceinline__ bool improves_remove(const St &st, int32_t d, int32_t k) {
    const int64_t Kp = st.K - 2 * (int64_t)d;
    if (Kp <= 0)
        return false;
    const int64_t Vp = st.V - k;
    const double X = -(double)(2 * (int64_t)d) * (double)Vp + st.alpha * ((double)k * (double)st.K);
    if (X < -kFilter * ((double)st.K * (double)Vp))
        return false;
    return decide(st, Kp, Vp);
}

__device__ __forceinline__ void set_logs(St &st) {
    st.LK = st.K > 0 ? ilog((uint64_t)st.K) : 0.0;
    st.LV = st.V > 0 ? ilog((uint64_t)st.V) : 0.0;
}

__device__ __forceinline__ void wave_argmax(double &r, int32_t &u, int32_t &i) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double r2 = __shfl_xor(r, off);
        const int32_t u2 = __shfl_xor(u, off);
        const int32_t i2 = __shfl_xor(i, off);
        if (before(r2, u2, r, u)) {
            r = r2;
            u = u2;
            i = i2;
        }
    }
}

__device__ __forceinline__ void wave_argmin(int32_t &u, int32_t &i) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int32_t u2 = __shfl_xor(u, off);
        const int32_t i2 = __shfl_xor(i, off);
        if (u2 < u) {
            u = u2;
            i = i2;
        }
    }
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v |= __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off);
    return v;
}

// One call of the growth function (Algorithm 1) at st.alpha.
// Returns the number of moves; stops early on table overflow.
template <bool GLOBAL>
__device__ int64_t grow(const Tab &t, St &st, const Ctx &c, uint32_t k_prune, int lane) {
    int64_t moves = 0;
    bool creation = true;
    for (;;) {
        double br = -__builtin_huge_val();
        int32_t bu = INT32_MAX;
        int32_t bi = -1;
        st.scanned += (uint64_t)st.count;
        for (int32_t i = lane; i < st.count; i += 64) {
            uint32_t v = t.DV(i);
            double r;
            if (creation) {
                // the queue is built from every non-member with a link into c
                if ((v & kMember) || (v & kDMask) == 0) {
                    if (v & (kLive | kFresh))
                        t.DV(i) = v & ~(kLive | kFresh);
                    continue;
                }
                const int32_t d = (int32_t)(v & kDMask);
                r = rank_of(c, d, t.KV(i), st.alpha);
                t.RK(i) = r;
                st.Rl += 1;
                st.Gl += 1;
                v = (v | kLive) & ~kFresh;
                t.DV(i) = v;
            } else {
                if (!(v & kLive))
                    continue;
                r = t.RK(i);
                if (v & kFresh) {
                    v &= ~kFresh;
                    t.DV(i) = v;
                } else if (before(r, t.NODE(i), st.pr, st.pu)) {
                    t.DV(i) = v & ~kLive;      // popped and rejected last step
                    continue;
                }
            }
            const int32_t u = t.NODE(i);
            if (before(r, u, br, bu) && improves_add(st, (int32_t)(v & kDMask), t.KV(i))) {
                br = r;
                bu = u;
                bi = i;
            }
        }
        creation = false;
        wave_argmax(br, bu, bi);
        wsync<GLOBAL>();
        if (bi < 0)
            break;
        // add the best improving node
        const uint32_t v = t.DV(bi);
        const int32_t d = (int32_t)(v & kDMask);
        const int32_t k = t.KV(bi);
        wsync<GLOBAL>();
        if (lane == 0)
            t.DV(bi) = (v | kMember) & ~(kLive | kFresh);
        st.K += 2 * (int64_t)d;
        st.V += k;
        st.nmem += 1;
        st.M += 1;
        moves += 1;
        st.pr = br;
        st.pu = bu;
        set_logs(st);
        wsync<GLOBAL>();
        row_update<GLOBAL, ROW_ADD>(t, st, c, bu, lane);
        if (st.ovf)
            return moves;
        if ((int64_t)st.M > st.move_limit) {
            st.err |= ERR_LIMIT;
            return moves;
        }
        if (over_budget(st))
            return moves;
    }
    if (moves == 0)
        return 0;
    // removal passes over the members in ascending id
    for (uint32_t pass = 0; k_prune == 0 || pass < k_prune; ++pass) {
        st.Gu += (uint64_t)st.nmem;
        int32_t cursor = -1;
        bool removed = false;
        for (;;) {
            int32_t cu = INT32_MAX;
            int32_t ci = -1;
            st.scanned += (uint64_t)st.count;
            for (int32_t i = lane; i < st.count; i += 64) {
                const uint32_t v = t.DV(i);
                if (!(v & kMember))
                    continue;
                const int32_t u = t.NODE(i);
                if (u <= cursor || u >= cu)
                    continue;
                if (improves_remove(st, (int32_t)(v & kDMask), t.KV(i))) {
                    cu = u;
                    ci = i;
                }
            }
            wave_argmin(cu, ci);
            wsync<GLOBAL>();
            if (ci < 0)
                break;
            const uint32_t v = t.DV(ci);
            const int32_t d = (int32_t)(v & kDMask);
            const int32_t k = t.KV(ci);
            wsync<GLOBAL>();
            if (lane == 0)
                t.DV(ci) = v & ~kMember;
            st.K -= 2 * (int64_t)d;
            st.V -= k;
            st.nmem -= 1;
            st.M += 1;
            moves += 1;
            set_logs(st);
            wsync<GLOBAL>();
            row_update<GLOBAL, ROW_REMOVE>(t, st, c, cu, lane);
            removed = true;
            cursor = cu;
            if ((int64_t)st.M > st.move_limit) {
                st.err |= ERR_LIMIT;
                return moves;
            }
            if (over_budget(st))
                return moves;
        }
        if (!removed)
            break;
    }
    return moves;
}

// Ascending sort of a[0..m) by one wave: bitonic network in its all-ascending
// form (each merge starts with a "flip" stage), with virtual +inf padding to
// the next power of two so comparators that touch the padding are no-ops.
template <bool GLOBAL>
__device__ void wave_sort(int32_t *a, int32_t m, int lane) {
    int32_t P = 1;
    while (P < m)
        P <<= 1;
    const int32_t half_n = P >> 1;
    for (int32_t k = 2; k <= P; k <<= 1) {
        const int32_t hk = k >> 1;
        for (int32_t t = lane; t < half_n; t += 64) {
            const int32_t blk = t / hk;
            const int32_t off = t - blk * hk;
            const int32_t i = blk * k + off;
            const int32_t l = blk * k + k - 1 - off;
            if (l < m) {
                const int32_t x = a[i], y = a[l];
                if (x > y) {
                    a[i] = y;
                    a[l] = x;
                }
            }
        }
        wsync<GLOBAL>();
        for (int32_t j = k >> 2; j >= 1; j >>= 1) {
            for (int32_t t = lane; t < half_n; t += 64) {
                const int32_t i = (t / j) * 2 * j + (t % j);
                const int32_t l = i + j;
                if (l < m) {
                    const int32_t x = a[i], y = a[l];
                    if (x > y) {
                        a[i] = y;
                        a[l] = x;
                    }
                }
            }
            wsync<GLOBAL>();
        }
    }
}

// PERSET: each set carries its own scale (query batches, one record per
// set); otherwise every set runs through scales[s_begin, s_end).
// Delta output: the first scale of the set's last full list at or before
// scale s_last (-1 if there is none), and the pool span of record r.
__device__ __forceinline__ int32_t delta_key_scale(const Records &rec, int32_t S, int32_t set, int32_t s_last) {
    int32_t sk = s_last;
    while (sk >= 0 && rec.drem[(int64_t)set * S + sk] >= 0)
        --sk;
    return sk;
}

__device__ __forceinline__ int32_t record_len(const Records &rec, int64_t r) {
    return rec.drem[r] < 0 ? rec.cnt[r] : rec.dadd[r] + rec.drem[r];
}

// Delta output, one wave: rebuild in the table the members recorded for
// scale s_last by toggling kMember | kWas for every id of the last full
// list and of each delta after it (an id joins and leaves alternately, so
// the members are the ids seen an odd number of times).  False when a
// record lies outside the pool (it overflowed: the host runs the sweep
// again); no full list before s_last is an error (ERR_MISSING).
template <bool GLOBAL>
__device__ bool wave_toggle_records(const SweepArgs &A, const Tab &t, St &st, const Ctx &c, int32_t set,
                                    int32_t s_last, int lane) {
    const int32_t sk = delta_key_scale(A.rec, A.S, set, s_last);
    if (sk < 0) {
        st.err |= ERR_MISSING;
        return true;
    }
    for (int32_t s = sk; s <= s_last; ++s) {
        const int64_t r = (int64_t)set * A.S + s;
        const int64_t off = A.rec.off[r];
        const int32_t len = record_len(A.rec, r);
        if (off < 0 || len < 0 || off + len > A.pool_cap)
            return false;
        for (int32_t base = 0; base < len; base += 64) {
            const bool act = base + lane < len;
            const int32_t u = act ? A.pool[off + base + lane] : 0;
            const int32_t idx = tab_ensure<GLOBAL>(t, st, c, act, u, lane);
            if (st.ovf)
                return true;
            if (act && idx >= 0)
                t.DV(idx) ^= (kMember | kWas);
            wsync<GLOBAL>();
        }
    }
    return true;
}

template <bool GLOBAL, bool PERSET>
__device__ void run_wave(const SweepArgs &A, const Tab &t, int lane) {
    Ctx c;
    c.row_ptr = A.g.row_ptr;
    c.col = A.g.col;
    c.w = A.g.w;
    c.kdeg = A.g.kdeg;
    c.logtab = A.g.logtab;
    c.logtab_last = A.g.logtab_n - 1;
    c.n = A.g.n;
    const uint32_t n_items = A.tier == 0 ? (uint32_t)A.n_sets : A.ctl->ovf_count[A.in_from];
    // What one item leaves for the device-wide counters is published by
    // lane 0 at the top of the next iteration, in the same lane-0 block that
    // takes the next item.  The item loop so has exactly one lane-0 block,
    // and its exits test wave-uniform (scalar) values: a lane-0 block at
    // both ends of such a loop lets the compiler thread them into a second
    // back edge that lanes 1..63 take without lane 0.
    bool pend = false;          // an item's epilogue is waiting
    uint32_t pend_push = 0;     // overflow item to push (valid if pend_ovf)
    bool pend_ovf = false;
    uint32_t pend_err = 0;
    uint64_t pend_stat[kStatWords] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (;;) {
        uint32_t item = 0;
        if (lane == 0) {
            if (pend) {
                if (pend_ovf) {
                    if (A.work_out) {
                        const uint32_t pos = atomicAdd(&A.ctl->ovf_count[A.tier], 1u);
                        A.work_out[pos] = (int32_t)pend_push;
                    } else {
                        atomicOr(A.err, ERR_CAPACITY);
                    }
                }
                if (pend_err)
                    atomicOr(A.err, pend_err);
                unsigned long long *sx = A.stat + kStatWords * A.tier;
                for (int q = 0; q < kStatWords; ++q)
                    if (q >= 6 || !pend_ovf)
                        atomicAdd(&sx[q], (unsigned long long)pend_stat[q]);
            }
            item = atomicAdd(&A.ctl->work_next[A.tier], 1u);
        }
        pend = false;
        item = (uint32_t)__builtin_amdgcn_readfirstlane((int)item);
        // another wave hit the watchdog: stop taking work
        const uint32_t abort = (uint32_t)__builtin_amdgcn_readfirstlane(
            (int)(__hip_atomic_load(A.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_TIMEOUT));
        if (item >= n_items || abort)
            break;
        // a later tier's item is set * S + s: the set overflowed the tier
        // before during scale s and resumes there from its scale s - 1 record
        const uint32_t wi = A.tier == 0 ? item : (uint32_t)A.work_in[item];
        const int32_t set = A.tier == 0 ? (int32_t)item : (int32_t)(wi / (uint32_t)A.S);
        const int32_t s0 = A.tier == 0 ? A.s_begin : (int32_t)(wi % (uint32_t)A.S);

        if constexpr (!GLOBAL) {
            for (uint32_t i = lane; i <= t.hmask; i += 64)
                t.hs[i] = -1;
            wsync<GLOBAL>();
        }
        St st;
        st.count = 0;
        st.nmem = 0;
        st.K = 0;
        st.V = 0;
        st.LK = st.LV = 0.0;
        st.alpha = 0.0;
        st.pr = 0.0;
        st.pu = 0;
        st.Gl = st.Rl = 0;
        st.Gu = 0;
        st.M = 0;
        st.ovf = false;
        st.err = 0;
        st.move_limit = 8 * (int64_t)A.g.n + 65536;
        st.t0 = wall_clock64();
        st.budget = (uint64_t)A.budget_ticks;
        st.rows = st.row_len = st.inserted = st.written = st.scanned = 0;
        st.mrows = st.mrow_len = st.c_mrows = st.c_mrow_len = st.ins_mark = st.c_ins = 0;
        st.srows = st.srow_len = 0;
        st.emitted = false;

        // initial community: the seed set, or the members recorded at the
        // previous scale when resuming
        const int32_t *init = nullptr;
        int32_t n_init = 0;
        bool bad = false;
        // delta output: the table's kWas flags hold the last record's members
        bool keyed = false;
        if ((s0 > A.s_begin || A.resume) && A.rec.drem) {
            // the members of scale s0 - 1 from its full list and deltas,
            // then gathered (any order) for the initialisation below
            bad = !wave_toggle_records<GLOBAL>(A, t, st, c, set, s0 - 1, lane);
            if (!bad && !st.ovf && !st.err) {
                int32_t m = 0;
                for (int32_t base = 0; base < st.count; base += 64) {
                    const int32_t i = base + lane;
                    const bool ism = i < st.count && (t.DV(i) & kMember);
                    const uint64_t bm = __ballot(ism);
                    if (ism)
                        t.scr[m + __popcll(bm & lanes_below(lane))] = t.NODE(i);
                    m += __popcll(bm);
                }
                wsync<GLOBAL>();
                init = t.scr;
                n_init = m;
                keyed = true;
            }
        } else if (s0 > A.s_begin || A.resume) {
            const int64_t r = (int64_t)set * A.S + (s0 - 1);
            const int64_t off = A.rec.off[r];
            n_init = A.rec.cnt[r];
            if (off < 0 || off + n_init > A.pool_cap)
                bad = true;   // the pool overflowed earlier: the host reruns
            else
                init = A.pool + off;
        } else {
            init = A.seed_nodes + A.seed_ptr[set];
            n_init = A.seed_ptr[set + 1] - A.seed_ptr[set];
        }
        for (int32_t q = 0; q < n_init && !bad && !st.ovf; ++q) {
            const int32_t u = init[q];
            const int32_t idx = tab_ensure<GLOBAL>(t, st, c, lane == 0, u, lane);
            if (st.ovf)
                break;
            const int32_t i0 = __shfl(idx, 0);
            const uint32_t v = t.DV(i0);
            wsync<GLOBAL>();
            if (lane == 0)
                t.DV(i0) = v | kMember;
            st.K += 2 * (int64_t)(v & kDMask);
            st.V += c.kdeg[u];
            st.nmem += 1;
            wsync<GLOBAL>();
            row_update<GLOBAL, ROW_INIT>(t, st, c, u, lane);
            if (st.ovf)
                break;
        }

        st.err = wave_or(st.err);
        // a seed set's initial gathers are part of the method; a set resumed
        // from an earlier tier's record gathers its members again (overhead)
        if (!(s0 > A.s_begin || A.resume)) {
            st.srows = st.rows;
            st.srow_len = st.row_len;
        } else {
            st.ins_mark = st.inserted;
        }
        int64_t last_off = -1;
        int32_t last_cnt = 0;
        int32_t s_at = s0;   // the scale being grown (where an overflow happened)
        for (int32_t s = s0; s < A.s_end && !st.ovf && !bad && !st.err; ++s) {
            s_at = s;
            if constexpr (PERSET)
                st.alpha = A.alpha_set[set];
            else
                st.alpha = A.scales[s];
            set_logs(st);
            st.Gl = st.Rl = 0;
            st.Gu = 0;
            st.M = 0;
            uint64_t calls = 0;
            int64_t moved = 0;
            for (;;) {
                calls += 1;
                const int64_t mv = grow<GLOBAL>(t, st, c, A.k_prune, lane);
                st.err = wave_or(st.err);   // probe failures are per lane
                moved += mv;
                if (st.ovf || st.err || mv == 0)
                    break;
                if (A.max_calls != 0 && calls >= (uint64_t)A.max_calls)
                    break;
                if ((int64_t)calls > st.move_limit) {
                    st.err |= ERR_LIMIT;
                    break;
                }
                if (over_budget(st))
                    break;
            }
            if (st.ovf || st.err)
                break;
            const int64_t r = (int64_t)set * A.S + s;
            const uint64_t G = wave_sum((uint64_t)st.Gl) + st.Gu;
            const uint64_t R = wave_sum((uint64_t)st.Rl);
            int32_t dadd = 0, drem = 0;
            if ((s == s0 || moved > 0) && keyed) {
                // delta output: ids that joined (from the front of the
                // scratch array) and left (from its back) since the last
                // record, each run sorted, into the pool
                int32_t na = 0, nr = 0;
                for (int32_t base = 0; base < st.count; base += 64) {
                    const int32_t i = base + lane;
                    const uint32_t v = i < st.count ? t.DV(i) : 0u;
                    const bool add = (v & kMember) && !(v & kWas);
                    const bool rem = (v & kWas) && !(v & kMember);
                    const uint64_t ba = __ballot(add);
                    const uint64_t br = __ballot(rem);
                    if (add)
                        t.scr[na + __popcll(ba & lanes_below(lane))] = t.NODE(i);
                    if (rem)
                        t.scr[t.cap - 1 - (nr + __popcll(br & lanes_below(lane)))] = t.NODE(i);
                    if (add || rem)
                        t.DV(i) = v ^ kWas;
                    na += __popcll(ba);
                    nr += __popcll(br);
                }
                wsync<GLOBAL>();
                wave_sort<GLOBAL>(t.scr, na, lane);
                wave_sort<GLOBAL>(t.scr + (t.cap - nr), nr, lane);
                unsigned long long off = 0;
                if (lane == 0)
                    off = atomicAdd(A.pool_cursor, (unsigned long long)(na + nr));
                off = __shfl(off, 0);
                if ((int64_t)off + na + nr <= A.pool_cap) {
                    for (int32_t i = lane; i < na; i += 64)
                        A.pool[off + i] = t.scr[i];
                    for (int32_t i = lane; i < nr; i += 64)
                        A.pool[off + na + i] = t.scr[t.cap - nr + i];
                }
                last_off = (int64_t)off;
                last_cnt = st.nmem;
                dadd = na;
                drem = nr;
                st.written += (uint64_t)(na + nr);
            } else if (s == s0 || moved > 0) {
                // members, sorted, into the pool (delta output: the set's
                // full list, and kWas := kMember)
                int32_t m = 0;
                for (int32_t base = 0; base < st.count; base += 64) {
                    const int32_t i = base + lane;
                    const uint32_t v = i < st.count ? t.DV(i) : 0u;
                    const bool ism = v & kMember;
                    const uint64_t bm = __ballot(ism);
                    if (ism)
                        t.scr[m + __popcll(bm & lanes_below(lane))] = t.NODE(i);
                    if (A.rec.drem && i < st.count && ism != (bool)(v & kWas))
                        t.DV(i) = v ^ kWas;
                    m += __popcll(bm);
                }
                wsync<GLOBAL>();
                wave_sort<GLOBAL>(t.scr, m, lane);
                unsigned long long off = 0;
                if (lane == 0)
                    off = atomicAdd(A.pool_cursor, (unsigned long long)m);
                off = __shfl(off, 0);
                if ((int64_t)off + m <= A.pool_cap) {
                    for (int32_t i = lane; i < m; i += 64)
                        A.pool[off + i] = t.scr[i];
                }
                last_off = (int64_t)off;
                last_cnt = m;
                dadd = m;
                drem = -1;
                keyed = A.rec.drem != nullptr;
                st.written += (uint64_t)m;
            } else if (keyed) {
                // delta output, nothing moved: an empty delta
                last_cnt = st.nmem;
            }
            if (lane == 0) {
                A.rec.off[r] = last_off;
                A.rec.cnt[r] = last_cnt;
                if (A.rec.drem) {
                    A.rec.dadd[r] = dadd;
                    A.rec.drem[r] = drem;
                }
                A.rec.K[r] = st.K;
                A.rec.V[r] = st.V;
                A.rec.f[r] = st.K == 0 ? 0.0 : (double)st.K / pow((double)st.V, st.alpha);
                A.rec.ctr[4 * r + 0] = G;
                A.rec.ctr[4 * r + 1] = R;
                A.rec.ctr[4 * r + 2] = st.M;
                A.rec.ctr[4 * r + 3] = calls;
            }
            if constexpr (PERSET) {
                // a query's record and members are final: publish them to
                // the host (every lane's stores, then the flag)
                if (A.done_flags) {
                    __threadfence_system();
                    if (lane == 0)
                        __hip_atomic_store(&A.done_flags[set], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                }
            }
            st.c_mrows = st.mrows;
            st.c_mrow_len = st.mrow_len;
            st.c_ins = st.inserted - st.ins_mark;
            st.emitted = true;
        }
        pend = true;
        pend_ovf = st.ovf;
        pend_push = (uint32_t)(set * A.S + s_at);
        pend_err = st.err;
        pend_stat[0] = st.rows;
        pend_stat[1] = st.row_len;
        pend_stat[2] = st.inserted;
        pend_stat[3] = st.written;
        pend_stat[4] = 1;
        pend_stat[5] = st.scanned;
        pend_stat[6] = st.c_mrows;
        pend_stat[7] = st.c_mrow_len;
        pend_stat[8] = st.emitted ? st.srows : 0;
        pend_stat[9] = st.emitted ? st.srow_len : 0;
        pend_stat[10] = st.c_ins;
        if constexpr (GLOBAL) {
            // leave the slab's hash empty for the next community
            wsync<GLOBAL>();
            for (int32_t i = lane; i < st.count; i += 64)
                tab_slot_clear<GLOBAL>(t, i);
            wsync<GLOBAL>();
        }
    }
}

__global__ void __launch_bounds__(256) sweep_lds_kernel(SweepArgs A) {
    extern __shared__ __align__(16) char smem[];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t tb = table_bytes(A.cap, A.hbits);
    Tab t = carve(smem + wave * tb, A.cap, A.hbits);
    run_wave<false, false>(A, t, lane);
}

__global__ void __launch_bounds__(256) sweep_global_kernel(SweepArgs A) {
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int slot = blockIdx.x * (blockDim.x >> 6) + wave;
    if (slot >= A.n_slots)
        return;
    Tab t = carve_global(A.gtab + (int64_t)slot * A.gtab_stride, A.cap, A.hbits);
    run_wave<true, false>(A, t, lane);
}

// The same growth for query batches: set j grows once at alpha_set[j].
__global__ void __launch_bounds__(256) query_lds_kernel(SweepArgs A) {
    extern __shared__ __align__(16) char smem[];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t tb = table_bytes(A.cap, A.hbits);
    Tab t = carve(smem + wave * tb, A.cap, A.hbits);
    run_wave<false, true>(A, t, lane);
}

__global__ void __launch_bounds__(256) query_global_kernel(SweepArgs A) {
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int slot = blockIdx.x * (blockDim.x >> 6) + wave;
    if (slot >= A.n_slots)
        return;
    Tab t = carve_global(A.gtab + (int64_t)slot * A.gtab_stride, A.cap, A.hbits);
    run_wave<true, true>(A, t, lane);
}

// ---------------------------------------------------------------------------
// Team growth: one workgroup of up to kTeamMaxWaves waves grows one
// community, for sets whose table outgrew the one-wave tier.  Same exact
// queue emulation, decisions and outputs as run_wave; every table scan is
// split over all threads of the workgroup and the per-wave results are
// combined through LDS.  Every branch that decides how many barriers a
// thread reaches depends only on values that all threads computed
// identically or read from LDS after a barrier.
// ---------------------------------------------------------------------------

constexpr int kTeamMaxWaves = 8;
// Rank buckets of the queue of a workgroup on a global-memory table.
constexpr int kBuckets = 256;

struct TeamSh {
    double r[kTeamMaxWaves];
    int32_t u[kTeamMaxWaves];
    int32_t i[kTeamMaxWaves];
    unsigned long long v[kTeamMaxWaves];
    unsigned long long off;
    int32_t count;    // dense entries claimed (may pass cap on overflow)
    int32_t m;        // members gathered for emission
    int32_t m2;       // delta output: ids that left, gathered for emission
    int32_t bidx;     // broadcast dense index
    uint32_t item;
    uint32_t ovf;
    uint32_t stop;
    uint32_t abort;
    // rank-bucketed queue (global tables)
    int32_t flen;                       // fresh-list appends (may pass the capacity)
    uint32_t ev;                        // the chosen addition's d|flags and degree
    int32_t ek;
    int32_t bstart[kBuckets + 1];       // queue positions of each bucket
    uint32_t fill[kBuckets];            // bucket counts, then fill cursors
    double r2[2 * kTeamMaxWaves];       // more reduction slots
    int32_t u2[2 * kTeamMaxWaves];
    int32_t i2[2 * kTeamMaxWaves];
};

struct TeamId {
    int tid, nt, lane, wid, nw;
};

__device__ __forceinline__ uint64_t team_sum(TeamSh &sh, const TeamId &id, uint64_t v) {
    v = wave_sum(v);
    if (id.lane == 0)
        sh.v[id.wid] = v;
    __syncthreads();
    uint64_t s = 0;
    for (int w = 0; w < id.nw; ++w)
        s += sh.v[w];
    __syncthreads();
    return s;
}

__device__ __forceinline__ uint32_t team_or(TeamSh &sh, const TeamId &id, uint32_t v) {
    v = wave_or(v);
    if (id.lane == 0)
        sh.v[id.wid] = v;
    __syncthreads();
    uint32_t s = 0;
    for (int w = 0; w < id.nw; ++w)
        s |= (uint32_t)sh.v[w];
    __syncthreads();
    return s;
}

// Watchdog decided by thread 0 and broadcast, so that all threads leave
// their loops together.
__device__ __forceinline__ bool team_over_budget(TeamSh &sh, const TeamId &id, St &st) {
    __syncthreads();
    if (id.tid == 0 && wall_clock64() - st.t0 > st.budget)
        sh.stop = 1u;
    __syncthreads();
    if (sh.stop) {
        st.err |= ERR_TIMEOUT;
        return true;
    }
    return false;
}

// Dense index of u for every active thread, inserting absent ids (all
// active ids of one call are distinct).  All probes finish before any
// insert.  On overflow sh.ovf is set (read it after the call).
template <bool GLOBAL>
__device__ int32_t team_ensure(const Tab &t, TeamSh &sh, St &st, const Ctx &c, bool act, int32_t u) {
    int32_t idx = act ? tab_find<GLOBAL>(t, u, st.err) : -1;
    __syncthreads();
    if (act && idx < 0) {
        const int32_t k = atomicAdd(&sh.count, 1);
        if (k >= t.cap) {
            atomicOr(&sh.ovf, 1u);
        } else {
            idx = k;
            t.NODE(idx) = u;
            t.KV(idx) = c.kdeg[u];
            t.DV(idx) = 0u;
            st.inserted += 1;
            tab_slot_insert<GLOBAL>(t, u, idx, st.err);
        }
    }
    __syncthreads();
    return idx;
}

// bqm: the table's queue is the rank-bucketed one (global tables only);
// otherwise pops are applied lazily, by the next table scan.
template <bool GLOBAL, int MODE>
__device__ void team_row(const Tab &t, TeamSh &sh, St &st, const Ctx &c, const TeamId &id, int32_t n,
                         bool bqm = false) {
    const int32_t beg = c.row_ptr[n];
    const int32_t end = c.row_ptr[n + 1];
    st.rows += 1;
    st.row_len += (uint64_t)(end - beg);
    if constexpr (MODE != ROW_INIT) {
        st.mrows += 1;
        st.mrow_len += (uint64_t)(end - beg);
    }
    for (int32_t base = beg; base < end; base += id.nt) {
        const int32_t j = base + id.tid;
        const bool act = j < end;
        const int32_t u = act ? c.col[j] : 0;
        const int32_t wt = act ? (c.w ? (int32_t)c.w[j] : 1) : 0;
        int32_t idx;
        if constexpr (MODE == ROW_REMOVE) {
            idx = act ? tab_find<GLOBAL>(t, u, st.err) : -1;
            if (act && idx < 0)
                st.err |= ERR_MISSING;
        } else {
            idx = team_ensure<GLOBAL>(t, sh, st, c, act, u);
            if (sh.ovf) {
                st.ovf = true;
                return;
            }
        }
        if (act && idx >= 0) {
            const uint32_t v = t.DV(idx);
            int32_t d = (int32_t)(v & kDMask);
            if constexpr (MODE == ROW_REMOVE) {
                d -= wt;
                t.DV(idx) = (v & ~kDMask) | (uint32_t)d;
            } else if constexpr (MODE == ROW_INIT) {
                d += wt;
                t.DV(idx) = (v & ~kDMask) | (uint32_t)d;
            } else {
                d += wt;
                if (v & kMember) {
                    t.DV(idx) = (v & ~kDMask) | (uint32_t)d;
                } else if (GLOBAL && bqm) {
                    // bucketed queue: queue entries are popped eagerly (flag
                    // cleared); fresh-list entries ranked above the addition
                    // just made were popped before it, which the next
                    // fresh-list scan applies.  An entry whose rank changes
                    // moves to the fresh list (its queue slot is stale while
                    // kFresh is set), marked kTouch until that scan.
                    const bool popped = !(v & kLive) || ((v & kFresh) && before(t.RK(idx), u, st.pr, st.pu));
                    if (popped)
                        st.Gl += 1;
                    const int32_t k = t.KV(idx);
                    t.RK(idx) = rank_of(c, d, k, st.alpha);
                    st.Rl += 1;
                    if (!(v & kFresh)) {
                        const int32_t pos = atomicAdd(&sh.flen, 1);
                        if (pos < t.cap)
                            t.fr[pos] = idx;
                    }
                    t.DV(idx) = (v & kWas) | (uint32_t)d | kLive | kFresh | kTouch;
                } else {
                    const bool queued = (v & kLive) && !before(t.RK(idx), u, st.pr, st.pu);
                    if (!queued)
                        st.Gl += 1;
                    const int32_t k = t.KV(idx);
                    t.RK(idx) = rank_of(c, d, k, st.alpha);
                    st.Rl += 1;
                    t.DV(idx) = (v & kWas) | (uint32_t)d | kLive | kFresh;
                }
            }
        }
    }
    __syncthreads();
    st.count = min(sh.count, t.cap);
}

// Block argmax of (rank, -id); also reads d|flags and k of the winner
// before the closing barrier, so that thread 0 may update the winner's flags
// right after it without another barrier.
__device__ __forceinline__ void team_pick_max(TeamSh &sh, const TeamId &id, const Tab &t, double &r,
                                              int32_t &u, int32_t &i, uint32_t &v, int32_t &k) {
    wave_argmax(r, u, i);
    if (id.lane == 0) {
        sh.r[id.wid] = r;
        sh.u[id.wid] = u;
        sh.i[id.wid] = i;
    }
    __syncthreads();
    r = sh.r[0];
    u = sh.u[0];
    i = sh.i[0];
    for (int w = 1; w < id.nw; ++w) {
        if (before(sh.r[w], sh.u[w], r, u)) {
            r = sh.r[w];
            u = sh.u[w];
            i = sh.i[w];
        }
    }
    if (i >= 0) {
        v = t.DV(i);
        k = t.KV(i);
    }
    __syncthreads();
}

// Workgroup minimum of v (every thread gets it).
__device__ __forceinline__ int32_t team_min_i32(TeamSh &sh, const TeamId &id, int32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        v = min(v, __shfl_xor(v, off));
    if (id.lane == 0)
        sh.u[id.wid] = v;
    __syncthreads();
    v = sh.u[0];
    for (int w = 1; w < id.nw; ++w)
        v = min(v, sh.u[w]);
    __syncthreads();
    return v;
}

__device__ __forceinline__ void team_pick_min(TeamSh &sh, const TeamId &id, const Tab &t, int32_t &u,
                                              int32_t &i, uint32_t &v, int32_t &k) {
    wave_argmin(u, i);
    if (id.lane == 0) {
        sh.u[id.wid] = u;
        sh.i[id.wid] = i;
    }
    __syncthreads();
    u = sh.u[0];
    i = sh.i[0];
    for (int w = 1; w < id.nw; ++w) {
        if (sh.u[w] < u) {
            u = sh.u[w];
            i = sh.i[w];
        }
    }
    if (i >= 0) {
        v = t.DV(i);
        k = t.KV(i);
    }
    __syncthreads();
}

// Entries each thread loads ahead in a table scan (independent loads in
// flight per thread; the scans are latency-bound).
constexpr int kScanAhead = 4;

// Removal passes of one growth call over the whole table: members in
// ascending id, each removal applied at once.  False when the call must
// end early (move limit, budget).
template <bool GLOBAL>
__device__ bool removal_scan(const Tab &t, TeamSh &sh, St &st, const Ctx &c, const TeamId &id,
                             uint32_t k_prune, int64_t &moves) {
    for (uint32_t pass = 0; k_prune == 0 || pass < k_prune; ++pass) {
        st.Gu += (uint64_t)st.nmem;
        int32_t cursor = -1;
        bool removed = false;
        for (;;) {
            int32_t cu = INT32_MAX;
            int32_t ci = -1;
            st.scanned += (uint64_t)st.count;
            for (int32_t base = id.tid; base < st.count; base += kScanAhead * id.nt) {
                uint32_t vv[kScanAhead];
                int32_t nn[kScanAhead], kk[kScanAhead];
#pragma unroll
                for (int q = 0; q < kScanAhead; ++q) {
                    const int32_t i = base + q * id.nt;
                    vv[q] = 0u;
                    nn[q] = 0;
                    kk[q] = 0;
                    if (i < st.count) {
                        vv[q] = t.DV(i);
                        nn[q] = t.NODE(i);
                        kk[q] = t.KV(i);
                    }
                }
#pragma unroll
                for (int q = 0; q < kScanAhead; ++q) {
                    const int32_t i = base + q * id.nt;
                    if (i >= st.count || !(vv[q] & kMember))
                        continue;
                    const int32_t u = nn[q];
                    if (u <= cursor || u >= cu)
                        continue;
                    if (improves_remove(st, (int32_t)(vv[q] & kDMask), kk[q])) {
                        cu = u;
                        ci = i;
                    }
                }
            }
            uint32_t v = 0;
            int32_t k = 0;
            team_pick_min(sh, id, t, cu, ci, v, k);
            if (ci < 0)
                break;
            const int32_t d = (int32_t)(v & kDMask);
            if (id.tid == 0)
                t.DV(ci) = v & ~kMember;
            st.K -= 2 * (int64_t)d;
            st.V -= k;
            st.nmem -= 1;
            st.M += 1;
            moves += 1;
            set_logs(st);
            team_row<GLOBAL, ROW_REMOVE>(t, sh, st, c, id, cu);
            removed = true;
            cursor = cu;
            if ((int64_t)st.M > st.move_limit) {
                st.err |= ERR_LIMIT;
                return false;
            }
            if ((st.M & 15) == 0 && team_over_budget(sh, id, st))
                return false;
        }
        if (!removed)
            break;
    }
    return true;
}

// ---------------------------------------------------------------------------
// Growth on a global-memory table with a rank-bucketed queue.
//
// A table of thousands of entries makes a full scan per addition the cost
// that dominates (a community adding A nodes scans its table A times).  For
// global tables the queue is therefore kept ordered enough that a step only
// looks at its head:
//   * the queue: every queued entry's index, counting-sorted into kBuckets
//     rank buckets (bucket(r) is monotone non-increasing in r, so every
//     entry of a later bucket ranks strictly below every entry of an earlier
//     one); positions before q.cp hold only popped entries;
//   * the fresh list: entries re-ranked by an addition since the queue was
//     built (flag kFresh; their queue slot is stale);
//   * a step takes the best improving fresh entry and walks the queue from
//     q.cp in windows of whole buckets (the best improving entry of a window
//     is the first improving entry of the queue, if it ranks above the fresh
//     candidate; a window with no improving entry ranked above the fresh
//     candidate is popped whole), so it pops exactly the entries the
//     sequential queue pops;
//   * the queue is rebuilt (three table passes, read in order) when the
//     fresh list grows past max(512, entries / 32): a rebuild costs fewer
//     bytes than the random reads of a longer fresh list.
// Removal passes walk a list of the members instead of the whole table.
// Same decisions, counters and results as the scan-driven additions.
// ---------------------------------------------------------------------------
struct BQ {
    double rtop;     // rank of bucket 0's upper end
    double scale;    // buckets per unit of rank
    int32_t ns;      // entries in the bucketed queue
    int32_t cp;      // queue positions before cp hold only popped entries
};

__device__ __forceinline__ int32_t bucket_of(double r, const BQ &q) {
    const double x = (q.rtop - r) * q.scale;
    if (!(x > 0.0))
        return 0;
    if (x >= (double)(kBuckets - 1))
        return kBuckets - 1;
    return (int32_t)x;
}

// true when (r, u) pops after (pr, pu)
__device__ __forceinline__ bool pops_after(double r, int32_t u, double pr, int32_t pu) {
    return before(pr, pu, r, u);
}

// largest b in [lo, hi] with bstart[b] <= pos (bstart non-decreasing, bstart[lo] <= pos)
__device__ __forceinline__ int32_t bucket_at(const TeamSh &sh, int32_t lo, int32_t hi, int32_t pos) {
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (sh.bstart[mid] <= pos)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Team argmax of (r, u, i) plus the team minimum and maximum of lo and hi.
__device__ __forceinline__ void team_max_range(TeamSh &sh, const TeamId &id, double &r, int32_t &u, int32_t &i,
                                               double &lo, double &hi) {
    wave_argmax(r, u, i);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off));
        hi = fmax(hi, __shfl_xor(hi, off));
    }
    if (id.lane == 0) {
        sh.r[id.wid] = r;
        sh.u[id.wid] = u;
        sh.i[id.wid] = i;
        sh.r2[id.wid] = lo;
        sh.r2[kTeamMaxWaves + id.wid] = hi;
    }
    __syncthreads();
    r = sh.r[0];
    u = sh.u[0];
    i = sh.i[0];
    lo = sh.r2[0];
    hi = sh.r2[kTeamMaxWaves];
    for (int w = 1; w < id.nw; ++w) {
        if (before(sh.r[w], sh.u[w], r, u)) {
            r = sh.r[w];
            u = sh.u[w];
            i = sh.i[w];
        }
        lo = fmin(lo, sh.r2[w]);
        hi = fmax(hi, sh.r2[kTeamMaxWaves + w]);
    }
    __syncthreads();
}

// Team reduction of one queue window: the best improving fresh entry (f),
// the best improving window entry (w) and the window entry that pops last
// (m; mi < 0: none).
__device__ __forceinline__ void team_window(TeamSh &sh, const TeamId &id, double &fr, int32_t &fu, int32_t &fi,
                                            double &wr, int32_t &wu, int32_t &wi, double &mr, int32_t &mi,
                                            int32_t &mu) {
    wave_argmax(fr, fu, fi);
    wave_argmax(wr, wu, wi);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double r2 = __shfl_xor(mr, off);
        const int32_t u2 = __shfl_xor(mu, off);
        const int32_t i2 = __shfl_xor(mi, off);
        if (i2 >= 0 && (mi < 0 || pops_after(r2, u2, mr, mu))) {
            mr = r2;
            mu = u2;
            mi = i2;
        }
    }
    if (id.lane == 0) {
        sh.r[id.wid] = fr;
        sh.u[id.wid] = fu;
        sh.i[id.wid] = fi;
        sh.r2[id.wid] = wr;
        sh.u2[id.wid] = wu;
        sh.i2[id.wid] = wi;
        sh.r2[kTeamMaxWaves + id.wid] = mr;
        sh.u2[kTeamMaxWaves + id.wid] = mu;
        sh.i2[kTeamMaxWaves + id.wid] = mi;
    }
    __syncthreads();
    fr = sh.r[0];
    fu = sh.u[0];
    fi = sh.i[0];
    wr = sh.r2[0];
    wu = sh.u2[0];
    wi = sh.i2[0];
    mr = sh.r2[kTeamMaxWaves];
    mu = sh.u2[kTeamMaxWaves];
    mi = sh.i2[kTeamMaxWaves];
    for (int w = 1; w < id.nw; ++w) {
        if (before(sh.r[w], sh.u[w], fr, fu)) {
            fr = sh.r[w];
            fu = sh.u[w];
            fi = sh.i[w];
        }
        if (before(sh.r2[w], sh.u2[w], wr, wu)) {
            wr = sh.r2[w];
            wu = sh.u2[w];
            wi = sh.i2[w];
        }
        const int32_t i2 = sh.i2[kTeamMaxWaves + w];
        const double r2 = sh.r2[kTeamMaxWaves + w];
        const int32_t u2 = sh.u2[kTeamMaxWaves + w];
        if (i2 >= 0 && (mi < 0 || pops_after(r2, u2, mr, mu))) {
            mr = r2;
            mu = u2;
            mi = i2;
        }
    }
    __syncthreads();
}

// Which queued entries a build pops first: those that pop before the last
// addition (pr, pu) and were not re-ranked by it.  After lazy-scan
// additions that is an entry without kFresh; in the bucketed queue, a
// fresh-list entry without kTouch.
enum { POP_LAZY_SCAN = 1, POP_FRESH_LIST = 2 };

__device__ __forceinline__ bool build_pops(uint32_t v, int pop_mode) {
    if (pop_mode == POP_LAZY_SCAN)
        return !(v & kFresh);
    if (pop_mode == POP_FRESH_LIST)
        return (v & kFresh) && !(v & kTouch);
    return false;
}

// Counting-sort the queued entries into rank buckets, ranks in [rbot, rtop].
// Entries that build_pops names and that pop before (pr, pu) are popped
// instead.  Clears every kFresh and kTouch flag and empties the fresh list.
__device__ void bq_build(const Tab &t, TeamSh &sh, St &st, const TeamId &id, BQ &q, double rtop,
                         double rbot, int pop_mode, double pr, int32_t pu) {
    q.rtop = rtop;
    q.scale = rtop > rbot ? (double)kBuckets / (rtop - rbot) : 0.0;
    st.scanned += 2 * (uint64_t)st.count;
    for (int32_t b = id.tid; b < kBuckets; b += id.nt)
        sh.fill[b] = 0u;
    if (id.tid == 0)
        sh.flen = 0;
    __syncthreads();
    for (int32_t i = id.tid; i < st.count; i += id.nt) {
        const uint32_t v = t.DV(i);
        if (!(v & kLive) || (v & kMember)) {
            if (v & (kFresh | kTouch))
                t.DV(i) = v & ~(kFresh | kTouch);   // a popped fresh-list entry
            continue;
        }
        const double r = t.RK(i);
        if (build_pops(v, pop_mode) && before(r, t.NODE(i), pr, pu)) {
            t.DV(i) = v & ~(kLive | kFresh | kTouch);
            continue;
        }
        if (v & (kFresh | kTouch))
            t.DV(i) = v & ~(kFresh | kTouch);
        atomicAdd(&sh.fill[bucket_of(r, q)], 1u);
    }
    __syncthreads();
    // exclusive prefix of the bucket counts (wave 0: four buckets per lane)
    if (id.wid == 0) {
        const int32_t b0 = 4 * id.lane;
        uint32_t c4[4];
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            c4[j] = sh.fill[b0 + j];
            sum += c4[j];
        }
        uint32_t incl = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t x = __shfl_up(incl, off);
            if (id.lane >= off)
                incl += x;
        }
        uint32_t run = incl - sum;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            sh.bstart[b0 + j] = (int32_t)run;
            sh.fill[b0 + j] = run;
            run += c4[j];
        }
        if (id.lane == 63)
            sh.bstart[kBuckets] = (int32_t)incl;
    }
    __syncthreads();
    for (int32_t i = id.tid; i < st.count; i += id.nt) {
        const uint32_t v = t.DV(i);
        if (!(v & kLive) || (v & kMember))
            continue;
        const uint32_t pos = atomicAdd(&sh.fill[bucket_of(t.RK(i), q)], 1u);
        t.sq[pos] = i;
    }
    __syncthreads();
    q.ns = sh.bstart[kBuckets];
    q.cp = 0;
}

// Rebuild the queue from every queued entry (fresh ones included), right
// after an addition (st.pr, st.pu): the fresh-list pops still pending are
// applied first.
__device__ void bq_rebuild(const Tab &t, TeamSh &sh, St &st, const TeamId &id, BQ &q) {
    double lo = __builtin_huge_val(), hi = -__builtin_huge_val();
    st.scanned += (uint64_t)st.count;
    for (int32_t i = id.tid; i < st.count; i += id.nt) {
        const uint32_t v = t.DV(i);
        if ((v & kLive) && !(v & kMember)) {
            const double r = t.RK(i);
            if (build_pops(v, POP_FRESH_LIST) && before(r, t.NODE(i), st.pr, st.pu))
                continue;
            lo = fmin(lo, r);
            hi = fmax(hi, r);
        }
    }
    double r = -__builtin_huge_val();
    int32_t u = INT32_MAX, i = -1;
    team_max_range(sh, id, r, u, i, lo, hi);
    bq_build(t, sh, st, id, q, hi, lo, POP_FRESH_LIST, st.pr, st.pu);
}

// Up to kScanAhead entries of an index list per thread (positions
// j0 + q * nt below lim), all loads issued before any is used: the index
// loads, then the entries' fields (i < 0: no entry).
struct Batch {
    int32_t i[kScanAhead];
    uint32_t v[kScanAhead];
    double r[kScanAhead];
    int32_t u[kScanAhead];
    int32_t k[kScanAhead];
};

__device__ __forceinline__ void load_batch(const Tab &t, const int32_t *list, int32_t j0, int32_t lim, int32_t nt,
                                           Batch &b) {
#pragma unroll
    for (int q = 0; q < kScanAhead; ++q) {
        const int32_t j = j0 + q * nt;
        b.i[q] = j < lim ? list[j] : -1;
    }
#pragma unroll
    for (int q = 0; q < kScanAhead; ++q) {
        b.v[q] = 0u;
        b.r[q] = 0.0;
        b.u[q] = 0;
        b.k[q] = 0;
        if (b.i[q] >= 0) {
            const int32_t i = b.i[q];
            b.v[q] = t.DV(i);
            b.r[q] = t.RK(i);
            b.u[q] = t.NODE(i);
            b.k[q] = t.KV(i);
        }
    }
}

// Switch a call from lazy pops to the bucketed queue right after an
// addition (st.pr, st.pu): the entries the lazy scan would drop next (not
// re-ranked, ranked above the addition) are popped, every other queued entry
// is bucketed.
__device__ void bq_switch(const Tab &t, TeamSh &sh, St &st, const TeamId &id, BQ &q) {
    double lo = __builtin_huge_val(), hi = -__builtin_huge_val();
    st.scanned += (uint64_t)st.count;
    for (int32_t i = id.tid; i < st.count; i += id.nt) {
        const uint32_t v = t.DV(i);
        if (!(v & kLive) || (v & kMember))
            continue;
        const double r = t.RK(i);
        if (build_pops(v, POP_LAZY_SCAN) && before(r, t.NODE(i), st.pr, st.pu))
            continue;
        lo = fmin(lo, r);
        hi = fmax(hi, r);
    }
    double r = -__builtin_huge_val();
    int32_t u = INT32_MAX, i = -1;
    team_max_range(sh, id, r, u, i, lo, hi);
    bq_build(t, sh, st, id, q, hi, lo, POP_LAZY_SCAN, st.pr, st.pu);
}

// The next addition: the entry the sequential queue would add next (the
// first improving entry in rank order), popping every queued entry ranked
// above it.  Returns its index, or -1 when no queued entry improves (every
// queued entry is popped then); er, eu, ev, ek get its rank, id, d|flags,
// degree.  The fresh list's pops are applied lazily: its scan drops the
// entries that an addition did not re-rank and that rank above it (the
// last addition is st.pr, st.pu).  A first window of at most one entry per
// thread keeps its entry in registers for its pops.
__device__ int32_t bq_step(const Tab &t, TeamSh &sh, St &st, const TeamId &id, BQ &q, double &er, int32_t &eu,
                           uint32_t &ev, int32_t &ek) {
    const int32_t flen = min(sh.flen, t.cap);
    st.scanned += (uint64_t)flen;
    double fr = -__builtin_huge_val();
    int32_t fu = INT32_MAX, fi = -1;
    uint32_t my_fv = 0u;
    int32_t my_fk = 0;
    for (int32_t j = id.tid; j < flen; j += id.nt) {
        const int32_t i = t.fr[j];
        uint32_t v = t.DV(i);
        if ((v & (kLive | kFresh | kMember)) != (kLive | kFresh))
            continue;
        const double r = t.RK(i);
        const int32_t u = t.NODE(i);
        const int32_t k = t.KV(i);
        if (v & kTouch) {
            v &= ~kTouch;
            t.DV(i) = v;
        } else if (before(r, u, st.pr, st.pu)) {
            // popped before the last addition; it keeps kFresh (and its
            // slot in the list), so that a later re-rank does not list it
            // twice
            t.DV(i) = v & ~kLive;
            continue;
        }
        if (before(r, u, fr, fu) && improves_add(st, (int32_t)(v & kDMask), k)) {
            fr = r;
            fu = u;
            fi = i;
            my_fv = v;
            my_fk = k;
        }
    }
    const int32_t my_fi = fi;
    int32_t my_wi = -1;
    uint32_t my_wv = 0u;
    int32_t my_wk = 0;
    int32_t cp = q.cp;
    int32_t win = id.nt;
    bool first = true;
    int32_t e = -1;
    bool from_q = false;
    for (;;) {
        // the window: whole buckets from cp, at most win entries unless its
        // first bucket alone holds more
        int32_t end = cp;
        if (cp < q.ns) {
            const int32_t b0 = bucket_at(sh, 0, kBuckets - 1, cp);
            int32_t b1 = bucket_at(sh, b0, kBuckets, cp + win);
            if (b1 <= b0)
                b1 = b0 + 1;
            end = sh.bstart[b1];
        }
        // a window of at most one entry per thread stays in registers
        const bool cached = end - cp <= id.nt;
        int32_t ci = -1;
        uint32_t cv = 0u;
        double cr = 0.0;
        int32_t cu = 0;
        double wr = -__builtin_huge_val(), mr = 0.0;
        int32_t wu = INT32_MAX, wi = -1, mu = 0, mi = -1;
        my_wi = -1;
        st.scanned += (uint64_t)(end - cp);
        for (int32_t j = cp + id.tid; j < end; j += id.nt) {
            const int32_t i = t.sq[j];
            const uint32_t v = t.DV(i);
            if ((v & (kLive | kFresh | kMember)) != kLive)
                continue;
            const double r = t.RK(i);
            const int32_t u = t.NODE(i);
            const int32_t k = t.KV(i);
            ci = i;
            cv = v;
            cr = r;
            cu = u;
            if (mi < 0 || pops_after(r, u, mr, mu)) {
                mr = r;
                mu = u;
                mi = i;
            }
            if (before(r, u, wr, wu) && improves_add(st, (int32_t)(v & kDMask), k)) {
                wr = r;
                wu = u;
                wi = i;
                my_wv = v;
                my_wk = k;
            }
        }
        my_wi = wi;
        if (!first) {
            fr = -__builtin_huge_val();
            fu = INT32_MAX;
            fi = -1;
        }
        team_window(sh, id, fr, fu, fi, wr, wu, wi, mr, mi, mu);
        if (first) {
            // the fresh candidate, kept for later windows
            er = fr;
            eu = fu;
            e = fi;
            first = false;
        }
        const bool has_f = e >= 0 && !from_q;
        const bool last = end >= q.ns;
        bool decided = false;
        if (wi >= 0 && (!has_f || before(wr, wu, er, eu))) {
            e = wi;
            er = wr;
            eu = wu;
            from_q = true;
            decided = true;
        } else if (has_f && ((mi >= 0 && before(er, eu, mr, mu)) || last)) {
            decided = true;
        } else if (last) {
            e = -1;
            decided = true;
        }
        // pops in the window: entries ranked above the addition, or all
        if (cached) {
            if (ci >= 0 && ci != e && (!decided || e < 0 || before(cr, cu, er, eu)))
                t.DV(ci) = cv & ~kLive;
        } else {
            for (int32_t j = cp + id.tid; j < end; j += id.nt) {
                const int32_t i = t.sq[j];
                const uint32_t v = t.DV(i);
                if ((v & (kLive | kFresh | kMember)) != kLive || i == e)
                    continue;
                if (!decided || e < 0 || before(t.RK(i), t.NODE(i), er, eu))
                    t.DV(i) = v & ~kLive;
            }
        }
        if (decided)
            break;
        cp = end;
        win *= 2;
        __syncthreads();
    }
    // buckets before the addition's hold only popped entries now
    q.cp = (e >= 0 && from_q) ? sh.bstart[bucket_of(er, q)] : cp;
    // the thread that found the addition hands on its flags and degree
    if (e >= 0 && (from_q ? my_wi == e : my_fi == e)) {
        sh.ev = from_q ? my_wv : my_fv;
        sh.ek = from_q ? my_wk : my_fk;
    }
    __syncthreads();
    if (e >= 0) {
        ev = sh.ev;
        ek = sh.ek;
    }
    return e;
}

// Additions from the bucketed queue until no queued entry improves (true)
// or the call must end early (false: overflow, move limit, budget).
template <bool GLOBAL>
__device__ bool bq_additions(const Tab &t, TeamSh &sh, St &st, const Ctx &c, const TeamId &id, BQ &q,
                             int64_t &moves) {
    for (;;) {
        if (sh.flen > max(512, st.count >> 5))
            bq_rebuild(t, sh, st, id, q);
        double br;
        int32_t bu;
        uint32_t v;
        int32_t k;
        const int32_t bi = bq_step(t, sh, st, id, q, br, bu, v, k);
        if (bi < 0)
            return true;
        // add bi; no thread reads its flags again before the row update's barriers
        const int32_t d = (int32_t)(v & kDMask);
        if (id.tid == 0)
            t.DV(bi) = (v | kMember) & ~(kLive | kFresh | kTouch);
        st.K += 2 * (int64_t)d;
        st.V += k;
        st.nmem += 1;
        st.M += 1;
        moves += 1;
        st.pr = br;
        st.pu = bu;
        set_logs(st);
        team_row<GLOBAL, ROW_ADD>(t, sh, st, c, id, bu, true);
        if (st.ovf)
            return false;
        if ((int64_t)st.M > st.move_limit) {
            st.err |= ERR_LIMIT;
            return false;
        }
        if ((st.M & 15) == 0 && team_over_budget(sh, id, st))
            return false;
    }
}

// Removal passes of one growth call over a list of the members gathered
// once (global tables), same order and decisions as removal_scan.  Record
// tables of more than by_id_min entries (16 queue_min: 16,384 at the default)
// sort the list into kBuckets ranges of node id (the queue's bucket arrays
// are free once the additions are over), so that a search for the smallest
// removable id above the cursor walks whole buckets from the cursor's one
// and stops at the first that holds one; smaller tables scan their whole
// list per search, which costs less than the sort and the extra barriers
// there.
template <bool GLOBAL>
__device__ bool removal_members(const Tab &t, TeamSh &sh, St &st, const Ctx &c, const TeamId &id,
                                uint32_t k_prune, int32_t by_id_min, int64_t &moves) {
    // record tables only (their lists run to tens of thousands of members);
    // the same in all threads
    const bool by_id = t.hp != nullptr && st.count > by_id_min;
    const int shift = max(0, (32 - __builtin_clz((uint32_t)max(c.n - 1, 1))) - 8);
    int32_t ml;
    if (by_id) {
        for (int32_t b = id.tid; b < kBuckets; b += id.nt)
            sh.fill[b] = 0u;
        __syncthreads();
        for (int32_t i = id.tid; i < st.count; i += id.nt) {
            if (t.DV(i) & kMember)
                atomicAdd(&sh.fill[t.NODE(i) >> shift], 1u);
        }
        __syncthreads();
        if (id.wid == 0) {
            const int32_t b0 = 4 * id.lane;
            uint32_t c4[4];
            uint32_t sum = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                c4[j] = sh.fill[b0 + j];
                sum += c4[j];
            }
            uint32_t incl = sum;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t x = __shfl_up(incl, off);
                if (id.lane >= off)
                    incl += x;
            }
            uint32_t run = incl - sum;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                sh.bstart[b0 + j] = (int32_t)run;
                sh.fill[b0 + j] = run;
                run += c4[j];
            }
            if (id.lane == 63)
                sh.bstart[kBuckets] = (int32_t)incl;
        }
        __syncthreads();
        for (int32_t i = id.tid; i < st.count; i += id.nt) {
            if (t.DV(i) & kMember)
                t.scr[atomicAdd(&sh.fill[t.NODE(i) >> shift], 1u)] = i;
        }
        __syncthreads();
        ml = sh.bstart[kBuckets];
        st.scanned += 2 * (uint64_t)st.count;
    } else {
        if (id.tid == 0)
            sh.m = 0;
        __syncthreads();
        for (int32_t i = id.tid; i < st.count; i += id.nt) {
            if (t.DV(i) & kMember)
                t.scr[atomicAdd(&sh.m, 1)] = i;
        }
        __syncthreads();
        ml = sh.m;
        st.scanned += (uint64_t)st.count;
    }
    for (uint32_t pass = 0; k_prune == 0 || pass < k_prune; ++pass) {
        st.Gu += (uint64_t)st.nmem;
        int32_t cursor = -1;
        bool removed = false;
        int32_t pos = 0;   // list positions before pos hold only ids at or below the cursor
        for (;;) {
            int32_t cu = INT32_MAX;
            int32_t ci = -1;
            // windows of whole buckets from pos until one holds a removable
            // id (unsorted: one window, the whole list)
            while (pos < ml) {
                int32_t end = ml;
                if (by_id) {
                    const int32_t b0 = bucket_at(sh, 0, kBuckets - 1, pos);
                    int32_t b1 = bucket_at(sh, b0, kBuckets, pos + kScanAhead * id.nt);
                    if (b1 <= b0)
                        b1 = b0 + 1;
                    end = sh.bstart[b1];
                }
                st.scanned += (uint64_t)(end - pos);
                for (int32_t j0 = pos + id.tid; j0 < end; j0 += kScanAhead * id.nt) {
                    Batch b;
                    load_batch(t, t.scr, j0, end, id.nt, b);
#pragma unroll
                    for (int x = 0; x < kScanAhead; ++x) {
                        if (b.i[x] < 0 || !(b.v[x] & kMember))
                            continue;
                        const int32_t u = b.u[x];
                        if (u <= cursor || u >= cu)
                            continue;
                        if (improves_remove(st, (int32_t)(b.v[x] & kDMask), b.k[x])) {
                            cu = u;
                            ci = b.i[x];
                        }
                    }
                }
                if (end >= ml)
                    break;   // the last window: the pick below decides
                const int32_t found = team_min_i32(sh, id, ci < 0 ? INT32_MAX : cu);
                if (found != INT32_MAX)
                    break;
                pos = end;
            }
            uint32_t vm = 0;
            int32_t km = 0;
            team_pick_min(sh, id, t, cu, ci, vm, km);
            if (ci < 0)
                break;
            const int32_t d = (int32_t)(vm & kDMask);
            if (id.tid == 0)
                t.DV(ci) = vm & ~kMember;
            st.K -= 2 * (int64_t)d;
            st.V -= km;
            st.nmem -= 1;
            st.M += 1;
            moves += 1;
            set_logs(st);
            team_row<GLOBAL, ROW_REMOVE>(t, sh, st, c, id, cu);
            removed = true;
            cursor = cu;
            pos = by_id ? sh.bstart[cu >> shift] : 0;
            if ((int64_t)st.M > st.move_limit) {
                st.err |= ERR_LIMIT;
                return false;
            }
            if ((st.M & 15) == 0 && team_over_budget(sh, id, st))
                return false;
        }
        if (!removed)
            break;
    }
    return true;
}


// One call of the growth function (Algorithm 1) by the whole workgroup.
// Additions start with full-table scans and lazy pops; on a global table
// whose entry count reaches queue_min (the count is the same in all
// threads) the call switches to the bucketed queue for the rest of its
// additions and to member-list removal passes.
template <bool GLOBAL>
__device__ int64_t team_grow(const Tab &t, TeamSh &sh, St &st, const Ctx &c, const TeamId &id,
                             uint32_t k_prune, int32_t queue_min) {
    int64_t moves = 0;
    bool creation = true;
    bool bucketed = false;
    for (;;) {
        double br = -__builtin_huge_val();
        int32_t bu = INT32_MAX;
        int32_t bi = -1;
        st.scanned += (uint64_t)st.count;
        for (int32_t base = id.tid; base < st.count; base += kScanAhead * id.nt) {
            uint32_t vv[kScanAhead];
            double rr[kScanAhead];
            int32_t nn[kScanAhead], kk[kScanAhead];
#pragma unroll
            for (int q = 0; q < kScanAhead; ++q) {
                const int32_t i = base + q * id.nt;
                vv[q] = 0u;
                rr[q] = 0.0;
                nn[q] = 0;
                kk[q] = 0;
                if (i < st.count) {
                    vv[q] = t.DV(i);
                    rr[q] = t.RK(i);
                    nn[q] = t.NODE(i);
                    kk[q] = t.KV(i);
                }
            }
#pragma unroll
            for (int q = 0; q < kScanAhead; ++q) {
                const int32_t i = base + q * id.nt;
                if (i >= st.count)
                    continue;
                uint32_t v = vv[q];
                double r = rr[q];
                if (creation) {
                    // the queue is built from every non-member with a link into c
                    if ((v & kMember) || (v & kDMask) == 0) {
                        if (v & (kLive | kFresh | kTouch))
                            t.DV(i) = v & ~(kLive | kFresh | kTouch);
                        continue;
                    }
                    r = rank_of(c, (int32_t)(v & kDMask), kk[q], st.alpha);
                    t.RK(i) = r;
                    st.Rl += 1;
                    st.Gl += 1;
                    v = (v | kLive) & ~(kFresh | kTouch);
                    t.DV(i) = v;
                } else {
                    if (!(v & kLive))
                        continue;
                    if (v & kFresh) {
                        v &= ~kFresh;
                        t.DV(i) = v;
                    } else if (before(r, nn[q], st.pr, st.pu)) {
                        t.DV(i) = v & ~kLive;      // popped and rejected last step
                        continue;
                    }
                }
                if (before(r, nn[q], br, bu) && improves_add(st, (int32_t)(v & kDMask), kk[q])) {
                    br = r;
                    bu = nn[q];
                    bi = i;
                }
            }
        }
        creation = false;
        uint32_t v = 0;
        int32_t k = 0;
        team_pick_max(sh, id, t, br, bu, bi, v, k);
        if (bi < 0)
            break;
        // add the best improving node; no thread reads its flags again
        // before the barriers of the row update below
        const int32_t d = (int32_t)(v & kDMask);
        if (id.tid == 0)
            t.DV(bi) = (v | kMember) & ~(kLive | kFresh);
        st.K += 2 * (int64_t)d;
        st.V += k;
        st.nmem += 1;
        st.M += 1;
        moves += 1;
        st.pr = br;
        st.pu = bu;
        set_logs(st);
        team_row<GLOBAL, ROW_ADD>(t, sh, st, c, id, bu);
        if (st.ovf)
            return moves;
        if ((int64_t)st.M > st.move_limit) {
            st.err |= ERR_LIMIT;
            return moves;
        }
        if ((st.M & 15) == 0 && team_over_budget(sh, id, st))
            return moves;
        if constexpr (GLOBAL) {
            if (st.count >= queue_min) {
                BQ q;
                bq_switch(t, sh, st, id, q);
                if (!bq_additions<GLOBAL>(t, sh, st, c, id, q, moves))
                    return moves;
                bucketed = true;
                break;
            }
        }
    }
    if (moves == 0)
        return 0;
    if constexpr (GLOBAL) {
        if (bucketed) {
            const int32_t by_id_min = (int32_t)min<int64_t>(16 * (int64_t)queue_min, INT32_MAX);
            removal_members<GLOBAL>(t, sh, st, c, id, k_prune, by_id_min, moves);
            return moves;
        }
    }
    removal_scan<GLOBAL>(t, sh, st, c, id, k_prune, moves);
    return moves;
}

// One compare-exchange round of the bitonic network over a[0..m): pair q
// of the round compares positions (i, l); kScanAhead pairs per thread with
// all loads issued first (the pairs of a round are disjoint).
template <typename PairOf>
__device__ __forceinline__ void team_sort_round(int32_t *a, int32_t m, int32_t half_n, const TeamId &id,
                                                PairOf pair_of) {
    for (int32_t q0 = id.tid; q0 < half_n; q0 += kScanAhead * id.nt) {
        int32_t ii[kScanAhead], ll[kScanAhead], xx[kScanAhead], yy[kScanAhead];
#pragma unroll
        for (int x = 0; x < kScanAhead; ++x) {
            const int32_t q = q0 + x * id.nt;
            ii[x] = -1;
            ll[x] = -1;
            if (q < half_n) {
                pair_of(q, ii[x], ll[x]);
                if (ll[x] >= m)
                    ii[x] = -1;
            }
            xx[x] = 0;
            yy[x] = 0;
            if (ii[x] >= 0) {
                xx[x] = a[ii[x]];
                yy[x] = a[ll[x]];
            }
        }
#pragma unroll
        for (int x = 0; x < kScanAhead; ++x) {
            if (ii[x] >= 0 && xx[x] > yy[x]) {
                a[ii[x]] = yy[x];
                a[ll[x]] = xx[x];
            }
        }
    }
    __syncthreads();
}

// Ascending sort of a[0..m) by the workgroup (same network as wave_sort).
__device__ void team_sort(int32_t *a, int32_t m, const TeamId &id) {
    int32_t P = 1;
    while (P < m)
        P <<= 1;
    const int32_t half_n = P >> 1;
    for (int32_t k = 2; k <= P; k <<= 1) {
        const int32_t hk = k >> 1;
        team_sort_round(a, m, half_n, id, [=](int32_t q, int32_t &i, int32_t &l) {
            const int32_t blk = q / hk;
            const int32_t off = q - blk * hk;
            i = blk * k + off;
            l = blk * k + k - 1 - off;
        });
        for (int32_t j = k >> 2; j >= 1; j >>= 1) {
            team_sort_round(a, m, half_n, id, [=](int32_t q, int32_t &i, int32_t &l) {
                i = (q / j) * 2 * j + (q % j);
                l = i + j;
            });
        }
    }
}

// Delta output, one workgroup: wave_toggle_records for the workgroup.
template <bool GLOBAL>
__device__ bool team_toggle_records(const SweepArgs &A, const Tab &t, TeamSh &sh, St &st, const Ctx &c,
                                    const TeamId &id, int32_t set, int32_t s_last) {
    const int32_t sk = delta_key_scale(A.rec, A.S, set, s_last);
    if (sk < 0) {
        st.err |= ERR_MISSING;
        return true;
    }
    for (int32_t s = sk; s <= s_last; ++s) {
        const int64_t r = (int64_t)set * A.S + s;
        const int64_t off = A.rec.off[r];
        const int32_t len = record_len(A.rec, r);
        if (off < 0 || len < 0 || off + len > A.pool_cap)
            return false;
        for (int32_t base = 0; base < len; base += id.nt) {
            const bool act = base + id.tid < len;
            const int32_t u = act ? A.pool[off + base + id.tid] : 0;
            const int32_t idx = team_ensure<GLOBAL>(t, sh, st, c, act, u);
            if (sh.ovf) {
                st.ovf = true;
                return true;
            }
            if (act && idx >= 0)
                t.DV(idx) ^= (kMember | kWas);
            st.count = min(sh.count, t.cap);
            __syncthreads();
        }
    }
    return true;
}

// Sort a[0..m) (global memory) through the LDS buffer lbuf when it fits:
// the bitonic network's rounds then wait on LDS, not on memory.
constexpr int kLdsSort = 2048;

__device__ void team_sort_via(int32_t *a, int32_t m, const TeamId &id, int32_t *lbuf) {
    if (m <= 1)
        return;
    if (!lbuf || m > kLdsSort) {
        team_sort(a, m, id);
        return;
    }
    for (int32_t i = id.tid; i < m; i += id.nt)
        lbuf[i] = a[i];
    __syncthreads();
    team_sort(lbuf, m, id);
    for (int32_t i = id.tid; i < m; i += id.nt)
        a[i] = lbuf[i];
    __syncthreads();
}

// lbuf: LDS sort buffer of kLdsSort entries (global tables), or nullptr.
template <bool GLOBAL, bool PERSET>
__device__ void run_team(const SweepArgs &A, const Tab &t, TeamSh &sh, int32_t *lbuf) {
    TeamId id;
    id.tid = (int)threadIdx.x;
    id.nt = (int)blockDim.x;
    id.lane = id.tid & 63;
    id.wid = id.tid >> 6;
    id.nw = id.nt >> 6;
    Ctx c;
    c.row_ptr = A.g.row_ptr;
    c.col = A.g.col;
    c.w = A.g.w;
    c.kdeg = A.g.kdeg;
    c.logtab = A.g.logtab;
    c.logtab_last = A.g.logtab_n - 1;
    c.n = A.g.n;
    const uint32_t n_items = A.tier == 0 ? (uint32_t)A.n_sets : A.ctl->ovf_count[A.in_from];
    for (;;) {
        __syncthreads();
        if (id.tid == 0) {
            sh.item = atomicAdd(&A.ctl->work_next[A.tier], 1u);
            sh.abort = __hip_atomic_load(A.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & ERR_TIMEOUT;
            sh.count = 0;
            sh.ovf = 0u;
            sh.stop = 0u;
        }
        if constexpr (!GLOBAL) {
            for (uint32_t i = id.tid; i <= t.hmask; i += id.nt)
                t.hs[i] = -1;
        }
        __syncthreads();
        const uint32_t item = sh.item;
        if (item >= n_items || sh.abort)
            break;
        // a later tier's item is set * S + s (see run_wave)
        const uint32_t wi = A.tier == 0 ? item : (uint32_t)A.work_in[item];
        const int32_t set = A.tier == 0 ? (int32_t)item : (int32_t)(wi / (uint32_t)A.S);
        const int32_t s0 = A.tier == 0 ? A.s_begin : (int32_t)(wi % (uint32_t)A.S);

        St st;
        st.count = 0;
        st.nmem = 0;
        st.K = 0;
        st.V = 0;
        st.LK = st.LV = 0.0;
        st.alpha = 0.0;
        st.pr = 0.0;
        st.pu = 0;
        st.Gl = st.Rl = 0;
        st.Gu = 0;
        st.M = 0;
        st.ovf = false;
        st.err = 0;
        st.move_limit = 8 * (int64_t)A.g.n + 65536;
        st.t0 = wall_clock64();
        st.budget = (uint64_t)A.budget_ticks;
        st.rows = st.row_len = st.inserted = st.written = st.scanned = 0;
        st.mrows = st.mrow_len = st.c_mrows = st.c_mrow_len = st.ins_mark = st.c_ins = 0;
        st.srows = st.srow_len = 0;
        st.emitted = false;

        const int32_t *init = nullptr;
        int32_t n_init = 0;
        bool bad = false;
        bool keyed = false;   // delta output (see run_wave)
        if ((s0 > A.s_begin || A.resume) && A.rec.drem) {
            bad = !team_toggle_records<GLOBAL>(A, t, sh, st, c, id, set, s0 - 1);
            st.err = team_or(sh, id, st.err);
            if (!bad && !st.ovf && !st.err) {
                if (id.tid == 0)
                    sh.m = 0;
                __syncthreads();
                for (int32_t i = id.tid; i < st.count; i += id.nt) {
                    if (t.DV(i) & kMember)
                        t.scr[atomicAdd(&sh.m, 1)] = t.NODE(i);
                }
                __syncthreads();
                init = t.scr;
                n_init = sh.m;
                keyed = true;
            }
        } else if (s0 > A.s_begin || A.resume) {
            const int64_t r = (int64_t)set * A.S + (s0 - 1);
            const int64_t off = A.rec.off[r];
            n_init = A.rec.cnt[r];
            if (off < 0 || off + n_init > A.pool_cap)
                bad = true;
            else
                init = A.pool + off;
        } else {
            init = A.seed_nodes + A.seed_ptr[set];
            n_init = A.seed_ptr[set + 1] - A.seed_ptr[set];
        }
        for (int32_t q = 0; q < n_init && !bad && !st.ovf; ++q) {
            const int32_t u = init[q];
            const int32_t idx = team_ensure<GLOBAL>(t, sh, st, c, id.tid == 0, u);
            if (sh.ovf) {
                st.ovf = true;
                break;
            }
            if (id.tid == 0)
                sh.bidx = idx;
            __syncthreads();
            const int32_t i0 = sh.bidx;
            const uint32_t v = t.DV(i0);
            __syncthreads();
            if (id.tid == 0)
                t.DV(i0) = v | kMember;
            st.K += 2 * (int64_t)(v & kDMask);
            st.V += c.kdeg[u];
            st.nmem += 1;
            st.count = min(sh.count, t.cap);
            __syncthreads();
            team_row<GLOBAL, ROW_INIT>(t, sh, st, c, id, u);
            if (st.ovf)
                break;
        }
        st.err = team_or(sh, id, st.err);
        // seed-set gathers are the method's; a resumed set's are overhead
        if (!(s0 > A.s_begin || A.resume)) {
            st.srows = st.rows;
            st.srow_len = st.row_len;
        } else {
            st.ins_mark = st.inserted;
        }

        int64_t last_off = -1;
        int32_t last_cnt = 0;
        int32_t s_at = s0;   // the scale being grown (where an overflow happened)
        for (int32_t s = s0; s < A.s_end && !st.ovf && !bad && !st.err; ++s) {
            s_at = s;
            if constexpr (PERSET)
                st.alpha = A.alpha_set[set];
            else
                st.alpha = A.scales[s];
            set_logs(st);
            st.Gl = st.Rl = 0;
            st.Gu = 0;
            st.M = 0;
            uint64_t calls = 0;
            int64_t moved = 0;
            for (;;) {
                calls += 1;
                const int64_t mv = team_grow<GLOBAL>(t, sh, st, c, id, A.k_prune, A.queue_min);
                st.err = team_or(sh, id, st.err);
                moved += mv;
                if (st.ovf || st.err || mv == 0)
                    break;
                if (A.max_calls != 0 && calls >= (uint64_t)A.max_calls)
                    break;
                if ((int64_t)calls > st.move_limit) {
                    st.err |= ERR_LIMIT;
                    break;
                }
                if (team_over_budget(sh, id, st))
                    break;
            }
            if (st.ovf || st.err)
                break;
            const int64_t r = (int64_t)set * A.S + s;
            const uint64_t G = team_sum(sh, id, (uint64_t)st.Gl) + st.Gu;
            const uint64_t R = team_sum(sh, id, (uint64_t)st.Rl);
            int32_t dadd = 0, drem = 0;
            if ((s == s0 || moved > 0) && keyed) {
                // delta output (see run_wave)
                if (id.tid == 0) {
                    sh.m = 0;
                    sh.m2 = 0;
                }
                __syncthreads();
                for (int32_t i = id.tid; i < st.count; i += id.nt) {
                    const uint32_t v = t.DV(i);
                    const bool add = (v & kMember) && !(v & kWas);
                    const bool rem = (v & kWas) && !(v & kMember);
                    if (add)
                        t.scr[atomicAdd(&sh.m, 1)] = t.NODE(i);
                    if (rem)
                        t.scr[t.cap - 1 - atomicAdd(&sh.m2, 1)] = t.NODE(i);
                    if (add || rem)
                        t.DV(i) = v ^ kWas;
                }
                __syncthreads();
                const int32_t na = sh.m, nr = sh.m2;
                team_sort_via(t.scr, na, id, lbuf);
                team_sort_via(t.scr + (t.cap - nr), nr, id, lbuf);
                if (id.tid == 0)
                    sh.off = atomicAdd(A.pool_cursor, (unsigned long long)(na + nr));
                __syncthreads();
                const unsigned long long off = sh.off;
                if ((int64_t)off + na + nr <= A.pool_cap) {
                    for (int32_t i = id.tid; i < na; i += id.nt)
                        A.pool[off + i] = t.scr[i];
                    for (int32_t i = id.tid; i < nr; i += id.nt)
                        A.pool[off + na + i] = t.scr[t.cap - nr + i];
                }
                last_off = (int64_t)off;
                last_cnt = st.nmem;
                dadd = na;
                drem = nr;
                st.written += (uint64_t)(na + nr);
                __syncthreads();
            } else if (s == s0 || moved > 0) {
                if (id.tid == 0)
                    sh.m = 0;
                __syncthreads();
                for (int32_t i = id.tid; i < st.count; i += id.nt) {
                    const uint32_t v = t.DV(i);
                    const bool ism = v & kMember;
                    if (ism) {
                        const int32_t p = atomicAdd(&sh.m, 1);
                        t.scr[p] = t.NODE(i);
                    }
                    if (A.rec.drem && ism != (bool)(v & kWas))
                        t.DV(i) = v ^ kWas;
                }
                __syncthreads();
                const int32_t m = sh.m;
                team_sort_via(t.scr, m, id, lbuf);
                if (id.tid == 0)
                    sh.off = atomicAdd(A.pool_cursor, (unsigned long long)m);
                __syncthreads();
                const unsigned long long off = sh.off;
                if ((int64_t)off + m <= A.pool_cap) {
                    for (int32_t i = id.tid; i < m; i += id.nt)
                        A.pool[off + i] = t.scr[i];
                }
                last_off = (int64_t)off;
                last_cnt = m;
                dadd = m;
                drem = -1;
                keyed = A.rec.drem != nullptr;
                st.written += (uint64_t)m;
                __syncthreads();
            } else if (keyed) {
                last_cnt = st.nmem;
            }
            if (id.tid == 0) {
                A.rec.off[r] = last_off;
                A.rec.cnt[r] = last_cnt;
                if (A.rec.drem) {
                    A.rec.dadd[r] = dadd;
                    A.rec.drem[r] = drem;
                }
                A.rec.K[r] = st.K;
                A.rec.V[r] = st.V;
                A.rec.f[r] = st.K == 0 ? 0.0 : (double)st.K / pow((double)st.V, st.alpha);
                A.rec.ctr[4 * r + 0] = G;
                A.rec.ctr[4 * r + 1] = R;
                A.rec.ctr[4 * r + 2] = st.M;
                A.rec.ctr[4 * r + 3] = calls;
            }
            if constexpr (PERSET) {
                // see run_wave: every thread's stores, then the flag
                if (A.done_flags) {
                    __threadfence_system();
                    __syncthreads();
                    if (id.tid == 0)
                        __hip_atomic_store(&A.done_flags[set], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                }
            }
            st.c_mrows = st.mrows;
            st.c_mrow_len = st.mrow_len;
            st.c_ins = st.inserted - st.ins_mark;
            st.emitted = true;
        }
        const uint64_t inserted = team_sum(sh, id, st.inserted);
        const uint64_t cins = team_sum(sh, id, st.c_ins);
        if (id.tid == 0) {
            if (st.ovf) {
                if (A.work_out) {
                    const uint32_t pos = atomicAdd(&A.ctl->ovf_count[A.tier], 1u);
                    A.work_out[pos] = set * A.S + s_at;
                } else {
                    atomicOr(A.err, ERR_CAPACITY);
                }
            }
            if (st.err)
                atomicOr(A.err, st.err);
            if (!st.ovf) {
                unsigned long long *sx = A.stat + kStatWords * A.tier;
                atomicAdd(&sx[0], (unsigned long long)st.rows);
                atomicAdd(&sx[1], (unsigned long long)st.row_len);
                atomicAdd(&sx[2], (unsigned long long)inserted);
                atomicAdd(&sx[3], (unsigned long long)st.written);
                atomicAdd(&sx[4], 1ull);
                atomicAdd(&sx[5], (unsigned long long)st.scanned);
            }
            unsigned long long *sa = A.stat + kStatWords * A.tier;
            atomicAdd(&sa[6], (unsigned long long)st.c_mrows);
            atomicAdd(&sa[7], (unsigned long long)st.c_mrow_len);
            if (st.emitted) {
                atomicAdd(&sa[8], (unsigned long long)st.srows);
                atomicAdd(&sa[9], (unsigned long long)st.srow_len);
            }
            atomicAdd(&sa[10], (unsigned long long)cins);
        }
        if constexpr (GLOBAL) {
            // leave the slab's hash empty for the next community
            const int32_t cnt = min(sh.count, t.cap);
            for (int32_t i = id.tid; i < cnt; i += id.nt)
                tab_slot_clear<GLOBAL>(t, i);
        }
    }
}

template <bool PERSET>
__device__ __forceinline__ void team_lds_entry(const SweepArgs &A) {
    extern __shared__ __align__(16) char smem[];
    __shared__ TeamSh sh;
    Tab t = carve(smem, A.cap, A.hbits);
    run_team<false, PERSET>(A, t, sh, nullptr);
}

// REC: the tables are of the record layout (cap >= kRecordMinEntries); one
// kernel per layout, so that each is compiled with its own strides.
template <bool PERSET, bool REC>
__device__ __forceinline__ void team_global_entry(const SweepArgs &A) {
    __shared__ TeamSh sh;
    __shared__ int32_t lsort[kLdsSort];
    const int slot = blockIdx.x;
    if (slot >= A.n_slots)
        return;
    Tab t = carve_global_as<REC>(A.gtab + (int64_t)slot * A.gtab_stride, A.cap, A.hbits);
    run_team<true, PERSET>(A, t, sh, lsort);
}

// Register bounds: a workgroup steps through one community as a chain of
// dependent scans, reductions and table updates, so more communities in
// flight per CU is what hides the latency, up to the point where spilled
// values reloaded inside the steps cost more than the extra communities
// win.  Both kinds take at most 128 VGPRs (four waves per SIMD): LDS tables
// of 1,024 entries allow four workgroups per CU anyway, and for the
// global-table kernels 96 VGPRs (five waves) spilled about 130 registers
// into scratch that the steps reload (measured: 128 is 7 % faster on the
// 100k- and 10M-node graphs, 1 % on the 1M one; 168 is slower on the 1M
// one).
#define LCD_TEAM_KERNEL(w) __global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(w)))
LCD_TEAM_KERNEL(4) sweep_team_lds_kernel(SweepArgs A) { team_lds_entry<false>(A); }
LCD_TEAM_KERNEL(4) sweep_team_global_kernel(SweepArgs A) { team_global_entry<false, false>(A); }
LCD_TEAM_KERNEL(4) sweep_team_global_rec_kernel(SweepArgs A) { team_global_entry<false, true>(A); }
LCD_TEAM_KERNEL(4) query_team_lds_kernel(SweepArgs A) { team_lds_entry<true>(A); }
LCD_TEAM_KERNEL(4) query_team_global_kernel(SweepArgs A) { team_global_entry<true, false>(A); }
LCD_TEAM_KERNEL(4) query_team_global_rec_kernel(SweepArgs A) { team_global_entry<true, true>(A); }
#undef LCD_TEAM_KERNEL

// ---------------------------------------------------------------------------
// Graph preparation
// ---------------------------------------------------------------------------
__global__ void degrees_kernel(const int32_t *row_ptr, const uint8_t *w, int32_t *kdeg, int32_t n) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n)
        return;
    const int32_t b = row_ptr[u], e = row_ptr[u + 1];
    if (!w) {
        kdeg[u] = e - b;
        return;
    }
    int32_t s = 0;
    for (int32_t j = b; j < e; ++j)
        s += w[j];
    kdeg[u] = s;
}

__global__ void logtab_kernel(double *tab, int32_t m) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= m)
        return;
    tab[x] = x == 0 ? 0.0 : ilog((uint64_t)x);
}

__global__ void log_kernel(const uint64_t *x, double *out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const uint64_t v = x[i];
    out[i] = v == 0 ? 0.0 : ilog(v);
}

__global__ void fill_i32_kernel(int32_t *p, int32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
// Readout
// ---------------------------------------------------------------------------

// exclusive scan of the member counts of one scale (single workgroup); the
// exact int64 total goes to *total, so the host can refuse a scale whose
// int32 offsets would wrap before it sizes or gathers anything
__global__ void __launch_bounds__(1024) scale_scan_kernel(const int32_t *cnt, int32_t S, int32_t s,
                                                          int32_t n_sets, int32_t *comm_ptr,
                                                          long long *total) {
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    const int64_t per = ((int64_t)n_sets + 1023) / 1024;
    const int64_t lo = tid * per;
    const int64_t hi = lo + per < n_sets ? lo + per : n_sets;
    int64_t sum = 0;
    for (int64_t j = lo; j < hi; ++j)
        sum += cnt[j * S + s];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = part[tid] - sum;
    for (int64_t j = lo; j < hi; ++j) {
        comm_ptr[j] = (int32_t)run;
        run += cnt[j * S + s];
    }
    if (tid == 1023) {
        comm_ptr[n_sets] = (int32_t)part[1023];
        *total = (long long)part[1023];
    }
}

__global__ void __launch_bounds__(256) scale_gather_kernel(Records rec, const int32_t *pool,
                                                           const double *scales, int32_t S,
                                                           int32_t s, int32_t n_sets,
                                                           const int32_t *comm_ptr, int32_t *members,
                                                           int64_t *k_in, int64_t *vol, double *f) {
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (j >= n_sets)
        return;
    const int64_t r = j * S + s;
    const int64_t off = rec.off[r];
    const int32_t m = rec.cnt[r];
    const int32_t dst = comm_ptr[j];
    if (members)
        for (int32_t i = lane; i < m; i += 64)
            members[dst + i] = pool[off + i];
    if (lane == 0) {
        if (k_in)
            k_in[j] = rec.K[r];
        if (vol)
            vol[j] = rec.V[r];
        if (f)
            f[j] = rec.f[r];
    }
}

// Delta output readout.  The members of scale s of a set are the ids that
// occur an odd number of times among the ids of its records from its last
// full list at or before s through s (every id alternately joins and
// leaves).  sets: listed set ids (nullptr: set q for q < n).

// Per listed set: ids in those records (ev[q]); a set with no full list
// before s sets bit 1 of *err.
__global__ void delta_events_kernel(Records rec, int32_t S, int32_t s, const int32_t *sets, int32_t n,
                                    int64_t *ev, uint32_t *err) {
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t set = sets ? sets[q] : (int32_t)q;
        const int32_t sk = delta_key_scale(rec, S, set, s);
        int64_t e = 0;
        if (sk < 0)
            atomicOr(err, 1u);
        else
            for (int32_t x = sk; x <= s; ++x)
                e += record_len(rec, (int64_t)set * S + x);
        ev[q] = e;
    }
}

// Exclusive prefix sums of x[0..n) into out[0..n] (one block).
__global__ void __launch_bounds__(1024) scan_i64_kernel(const int64_t *x, int64_t n, int64_t *out) {
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t lo = tid * per;
    const int64_t hi = lo + per < n ? lo + per : n;
    int64_t sum = 0;
    for (int64_t j = lo; j < hi; ++j)
        sum += x[j];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = part[tid] - sum;
    for (int64_t j = lo; j < hi; ++j) {
        const int64_t v = x[j];
        out[j] = run;
        run += v;
    }
    if (tid == 1023)
        out[n] = part[1023];
}

// One workgroup per listed set: its records' ids into scratch[ev_off[q]..),
// sorted, then the ids of odd multiplicity, in order, to
// members[out_ptr[q]..).  A count other than the record's sets bit 2 of
// *err.
__global__ void __launch_bounds__(256) delta_rebuild_kernel(Records rec, const int32_t *pool, int32_t S,
                                                            int32_t s, const int32_t *sets, int32_t n,
                                                            const int64_t *ev_off, int32_t *scratch,
                                                            const int32_t *out_ptr, int32_t *members,
                                                            uint32_t *err) {
    TeamId id;
    id.tid = (int)threadIdx.x;
    id.nt = (int)blockDim.x;
    id.lane = id.tid & 63;
    id.wid = id.tid >> 6;
    id.nw = id.nt >> 6;
    __shared__ int32_t wcount[kTeamMaxWaves];
    for (int64_t q = blockIdx.x; q < n; q += gridDim.x) {
        const int32_t set = sets ? sets[q] : (int32_t)q;
        const int32_t sk = delta_key_scale(rec, S, set, s);
        if (sk < 0)
            continue;   // reported by delta_events_kernel
        int32_t *a = scratch + ev_off[q];
        int64_t pos = 0;
        for (int32_t x = sk; x <= s; ++x) {
            const int64_t r = (int64_t)set * S + x;
            const int64_t off = rec.off[r];
            const int32_t len = record_len(rec, r);
            for (int32_t i = id.tid; i < len; i += id.nt)
                a[pos + i] = pool[off + i];
            pos += len;
        }
        const int32_t E = (int32_t)pos;
        __syncthreads();
        team_sort(a, E, id);
        int32_t outn = 0;
        const int32_t dst = out_ptr[q];
        for (int32_t base = 0; base < E; base += id.nt) {
            const int32_t p = base + id.tid;
            bool keep = false;
            if (p < E && (p == 0 || a[p - 1] != a[p])) {
                int32_t L = 1;
                while (p + L < E && a[p + L] == a[p])
                    ++L;
                keep = (L & 1) != 0;
            }
            const uint64_t bm = __ballot(keep);
            if (id.lane == 0)
                wcount[id.wid] = __popcll(bm);
            __syncthreads();
            int32_t before_w = 0, total = 0;
            for (int w = 0; w < id.nw; ++w) {
                if (w < id.wid)
                    before_w += wcount[w];
                total += wcount[w];
            }
            if (keep)
                members[dst + outn + before_w + __popcll(bm & lanes_below(id.lane))] = a[p];
            outn += total;
            __syncthreads();
        }
        if (id.tid == 0 && outn != rec.cnt[(int64_t)set * S + s])
            atomicOr(err, 2u);
        __syncthreads();
    }
}

// Per set: the ids added and removed at scale s (a full list counts as
// added), their counts first.
__global__ void delta_counts_kernel(Records rec, int32_t S, int32_t s, int32_t n, int64_t *na, int64_t *nr) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = j * S + s;
        const bool full = rec.drem[r] < 0;
        na[j] = full ? rec.cnt[r] : rec.dadd[r];
        nr[j] = full ? 0 : rec.drem[r];
    }
}

__global__ void __launch_bounds__(256) delta_gather_kernel(Records rec, const int32_t *pool, int32_t S,
                                                           int32_t s, int32_t n, const int64_t *add_off,
                                                           int32_t *added, const int64_t *rem_off,
                                                           int32_t *removed) {
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (j >= n)
        return;
    const int64_t r = j * S + s;
    const int64_t off = rec.off[r];
    const int32_t a = (int32_t)(add_off[j + 1] - add_off[j]);
    const int32_t m = (int32_t)(rem_off[j + 1] - rem_off[j]);
    if (added)
        for (int32_t i = lane; i < a; i += 64)
            added[add_off[j] + i] = pool[off + i];
    if (removed)
        for (int32_t i = lane; i < m; i += 64)
            removed[rem_off[j] + i] = pool[off + a + i];
}

__global__ void overlap_count_kernel(const int32_t *members, int64_t total, int32_t *cnt) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[members[i]], 1);
}

// ---------------------------------------------------------------------------
// Seed selection (Sec. 3, initialisation of Algorithm 2) in parallel rounds.
// Candidate nodes (at least two neighbours) are visited in the order perm;
// the sequential rule keeps a node that is still a candidate and drops its
// neighbours (rule 1) or everything within two hops (rule 2).  That set is
// the first independent set in visiting order of the conflict graph (two
// candidates conflict within 1 or 2 hops), which rounds of "an undecided
// candidate joins when it comes first among the undecided candidates it
// conflicts with" produce exactly (Blelloch, Fineman and Shun, SPAA 2012).
// st: 0 undecided candidate, 1 seed, 2 not a seed.
// ---------------------------------------------------------------------------

__global__ void seed_init_kernel(const int32_t *row_ptr, const int32_t *perm, int32_t n, int32_t *pos,
                                 uint8_t *st, uint8_t *act) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        pos[perm[i]] = (int32_t)i;
        st[i] = (row_ptr[i + 1] - row_ptr[i]) >= 2 ? 0 : 2;
        act[i] = 1;
    }
}

// A round whose previous round counted no undecided candidate (*prev == 0)
// does nothing, so that the host can queue many rounds and read the count
// once.  A candidate comes first among the undecided candidates within R
// hops iff the smallest visiting position of an undecided candidate in its
// closed R-hop neighbourhood is its own.  That minimum is built one hop at a
// time: m1[u] = min over the closed neighbourhood of u (undecided
// candidates only), then, for rule 2, the min of m1 over the closed
// neighbourhood of v: two passes over the edges instead of a walk over
// every two-hop path.  Candidates never become undecided again, so a node
// whose closed neighbourhood holds none keeps m1 = INT32_MAX for good and
// is skipped from then on (act[v] = 0).
__global__ void seed_min1_kernel(const int32_t *row_ptr, const int32_t *col, const int32_t *pos,
                                 const uint8_t *st, uint8_t *act, int32_t n, int32_t *m1, const unsigned *prev,
                                 unsigned *undecided) {
    if (prev && *prev == 0u)
        return;
    unsigned cnt = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        if (!act[v])
            continue;
        int32_t m = INT32_MAX;
        if (st[v] == 0) {
            cnt += 1;
            m = pos[v];
        }
        for (int32_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
            const int32_t u = col[j];
            if (st[u] == 0)
                m = min(m, pos[u]);
        }
        m1[v] = m;
        if (m == INT32_MAX)
            act[v] = 0;
    }
    if (cnt)
        atomicAdd(undecided, cnt);
}

// Rule 2: sel[v] for undecided v whose closed two-hop minimum is its own.
__global__ void seed_min2_kernel(const int32_t *row_ptr, const int32_t *col, const int32_t *pos,
                                 const uint8_t *st, const int32_t *m1, uint8_t *sel, int32_t n,
                                 const unsigned *undecided) {
    if (*undecided == 0u)
        return;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        uint8_t ok = 0;
        if (st[v] == 0) {
            const int32_t pv = pos[v];
            ok = m1[v] == pv;
            for (int32_t j = row_ptr[v]; j < row_ptr[v + 1] && ok; ++j)
                ok = m1[col[j]] >= pv;
        }
        sel[v] = ok;
    }
}

// Rule 1: the selected candidates (m1 == own position) become seeds and
// their undecided neighbours are dropped.  Selected nodes are pairwise
// further apart than one hop, so a selected node's flag is written by its
// own thread only, and every other write is the same value from whichever
// thread makes it.
__global__ void seed_apply1_kernel(const int32_t *row_ptr, const int32_t *col, const int32_t *pos,
                                   const int32_t *m1, uint8_t *st, int32_t n, const unsigned *undecided) {
    if (*undecided == 0u)
        return;   // the round found nothing to decide
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        if (st[v] != 0 || m1[v] != pos[v])
            continue;
        st[v] = 1;
        for (int32_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
            const int32_t u = col[j];
            if (st[u] == 0)
                st[u] = 2;
        }
    }
}

// Rule 2 in two one-hop passes instead of a walk over the two-hop paths of
// each selected node (one thread per selected node walked up to max-degree
// squared entries in turn): near[v] = some selected node in the closed
// neighbourhood of v; an undecided candidate then becomes a seed if
// selected, and is dropped if some node of its closed neighbourhood is
// near a selected one, i.e. if a selected node lies within two hops.
// Nodes with no undecided candidate within one hop (act[v] = 0) are never
// read by the second pass and are skipped.
__global__ void seed_near_kernel(const int32_t *row_ptr, const int32_t *col, const uint8_t *sel,
                                 const uint8_t *act, int32_t n, uint8_t *near, const unsigned *undecided) {
    if (*undecided == 0u)
        return;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        if (!act[v])
            continue;
        uint8_t x = sel[v];
        for (int32_t j = row_ptr[v]; j < row_ptr[v + 1] && !x; ++j)
            x = sel[col[j]];
        near[v] = x;
    }
}

__global__ void seed_apply2_kernel(const int32_t *row_ptr, const int32_t *col, const uint8_t *sel,
                                   const uint8_t *near, uint8_t *st, int32_t n, const unsigned *undecided) {
    if (*undecided == 0u)
        return;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        if (st[v] != 0)
            continue;
        if (sel[v]) {
            st[v] = 1;
            continue;
        }
        uint8_t x = near[v];
        for (int32_t j = row_ptr[v]; j < row_ptr[v + 1] && !x; ++j)
            x = near[col[j]];
        if (x)
            st[v] = 2;
    }
}

__global__ void seed_flag_kernel(const int32_t *perm, const uint8_t *st, int32_t n, int32_t *flag) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        flag[i] = st[perm[i]] == 1 ? 1 : 0;
}

__global__ void seed_scatter_kernel(const int32_t *perm, const int32_t *flag, const int32_t *at, int32_t n,
                                    int32_t *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (flag[i])
            out[at[i]] = perm[i];
}

// ---------------------------------------------------------------------------
// Overlap partner of a community (check phase of Algorithm 2, and the
// overlap pre-test of Algorithm 3).  One wave per listed community c: walk
// c's members in ascending order and, for each member v, the communities
// holding v in ascending order, counting per community; the first community
// i != c whose count x reaches x * den >= num * min(|c|, |i|) is the partner
// (-1: none).  The order of the walk decides which partner is "first", so
// lanes take consecutive entries of one member's list and the lowest lane
// that reaches the threshold wins.  cnt_all: one int32[n_comms] per wave
// slot, zero on entry and left zero.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) partner_kernel(const int32_t *comm_ptr, const int32_t *members,
                                                      const int32_t *node_ptr, const int32_t *node_sets,
                                                      const int32_t *list, int32_t n_list, int32_t n_comms,
                                                      int32_t eta_num, int32_t eta_den, int32_t *cnt_all,
                                                      int32_t n_slots, unsigned *next, int32_t *partner) {
    const int lane = threadIdx.x & 63;
    const int slot = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slot >= n_slots)
        return;
    int32_t *cnt = cnt_all + (int64_t)slot * n_comms;
    // item and found are held wave-uniform (scalar registers), and the loop
    // has no lane-0-only block at its end: a lane-0 block at both ends of the
    // loop lets the compiler thread them into a second back edge that lanes
    // 1..63 take alone, with no exit for them while lane 0 waits outside.
    for (;;) {
        unsigned item = 0;
        if (lane == 0)
            item = atomicAdd(next, 1u);
        item = (unsigned)__builtin_amdgcn_readfirstlane((int)item);
        if (item >= (unsigned)n_list)
            break;
        const int32_t c = list[item];
        const int32_t c0 = comm_ptr[c], c1 = comm_ptr[c + 1];
        const int64_t sc = c1 - c0;
        int32_t found = -1;
        for (int32_t q = c0; q < c1 && found < 0; ++q) {
            const int32_t v = members[q];
            const int32_t t1 = node_ptr[v + 1];
            for (int32_t t0 = node_ptr[v]; t0 < t1 && found < 0; t0 += 64) {
                const int32_t t = t0 + lane;
                const int32_t i = t < t1 ? node_sets[t] : -1;
                bool hit = false;
                if (i >= 0 && i != c) {
                    const int64_t x = (int64_t)atomicAdd(&cnt[i], 1) + 1;
                    const int64_t si = comm_ptr[i + 1] - comm_ptr[i];
                    const int64_t small = sc < si ? sc : si;
                    hit = x * eta_den >= (int64_t)eta_num * small;
                }
                const uint64_t m = __ballot(hit);
                if (m)
                    found = __builtin_amdgcn_readlane(i, (int)__builtin_ctzll(m));
            }
        }
        // leave the counts at zero for the next community
        for (int32_t q = c0; q < c1; ++q) {
            const int32_t v = members[q];
            for (int32_t t = node_ptr[v] + lane; t < node_ptr[v + 1]; t += 64) {
                const int32_t i = node_sets[t];
                if (i != c)
                    atomicExch(&cnt[i], 0);
            }
        }
        // every lane stores the same value (no lane-0 branch, see above)
        partner[item] = found;
    }
}

// Order one tier's overflow list for the next tier: items set * S + s by
// ascending s, so that the sets with the most scales left start first (a
// tier lasts as long as its slowest workgroup).  One workgroup; the order
// never changes a result.
__global__ void __launch_bounds__(1024) order_spills_kernel(const int32_t *in, const uint32_t *count,
                                                            uint32_t n_max, int32_t S, int32_t *out) {
    __shared__ uint32_t hist[1024];
    const uint32_t n = min(*count, n_max);
    const uint32_t tid = threadIdx.x;
    for (int32_t s = (int32_t)tid; s < S; s += 1024)
        hist[s] = 0u;
    __syncthreads();
    for (uint32_t i = tid; i < n; i += 1024)
        atomicAdd(&hist[(uint32_t)in[i] % (uint32_t)S], 1u);
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int32_t s = 0; s < S; ++s) {
            const uint32_t c = hist[s];
            hist[s] = run;
            run += c;
        }
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += 1024) {
        const int32_t w = in[i];
        const uint32_t pos = atomicAdd(&hist[(uint32_t)w % (uint32_t)S], 1u);
        out[pos] = w;
    }
}

// three-phase exclusive scan of n counts into ptr[0..n]
__global__ void __launch_bounds__(1024) scan_blocks_kernel(const int32_t *cnt, int64_t n,
                                                           int32_t *ptr, int32_t *block_sums) {
    __shared__ int32_t part[1024];
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const int32_t v = i < n ? cnt[i] : 0;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int32_t x = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += x;
        __syncthreads();
    }
    if (i < n)
        ptr[i] = part[threadIdx.x] - v;
    if (threadIdx.x == 1023)
        block_sums[blockIdx.x] = part[1023];
}

__global__ void __launch_bounds__(1024) scan_sums_kernel(int32_t *block_sums, int32_t nb,
                                                         int32_t *total_out) {
    __shared__ int32_t part[1024];
    const int tid = threadIdx.x;
    const int per = (nb + 1023) / 1024;
    const int lo = tid * per;
    const int hi = lo + per < nb ? lo + per : nb;
    int32_t sum = 0;
    for (int j = lo; j < hi; ++j)
        sum += block_sums[j];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int32_t x = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += x;
        __syncthreads();
    }
    int32_t run = part[tid] - sum;
    for (int j = lo; j < hi; ++j) {
        const int32_t b = block_sums[j];
        block_sums[j] = run;
        run += b;
    }
    if (tid == 1023)
        *total_out = part[1023];
}

__global__ void scan_add_kernel(int32_t *ptr, int64_t n, const int32_t *block_sums) {
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    if (i < n)
        ptr[i] += block_sums[blockIdx.x];
}

__global__ void __launch_bounds__(256) overlap_scatter_kernel(const int32_t *comm_ptr,
                                                              const int32_t *members, int32_t n_sets,
                                                              const int32_t *node_ptr, int32_t *fill,
                                                              int32_t *node_sets) {
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t j = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (j >= n_sets)
        return;
    for (int32_t i = comm_ptr[j] + lane; i < comm_ptr[j + 1]; i += 64) {
        const int32_t u = members[i];
        const int32_t pos = atomicAdd(&fill[u], 1);
        node_sets[node_ptr[u] + pos] = (int32_t)j;
    }
}

// Sort every node's list: lanes sort short lists alone; each long list is
// then sorted by the whole wave.
__global__ void __launch_bounds__(256) overlap_sort_kernel(const int32_t *node_ptr, int32_t n,
                                                           int32_t *node_sets) {
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t u = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wave) * 64 + lane;
    int32_t lo = 0, len = 0;
    if (u < n) {
        lo = node_ptr[u];
        len = node_ptr[u + 1] - lo;
    }
    const bool longl = len > 32;
    if (!longl && len > 1) {
        int32_t *a = node_sets + lo;
        for (int32_t i = 1; i < len; ++i) {
            const int32_t x = a[i];
            int32_t j = i - 1;
            while (j >= 0 && a[j] > x) {
                a[j + 1] = a[j];
                --j;
            }
            a[j + 1] = x;
        }
    }
    uint64_t todo = __ballot(longl);
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    while (todo) {
        const int src = __builtin_ctzll(todo);
        todo &= todo - 1;
        const int32_t l0 = __shfl(lo, src);
        const int32_t n0 = __shfl(len, src);
        wave_sort<true>(node_sets + l0, n0, lane);
    }
}

__global__ void counter_sum_kernel(const uint64_t *ctr, int64_t n_rec, unsigned long long *tot) {
    unsigned long long s[4] = {0, 0, 0, 0};
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_rec;
         r += (int64_t)gridDim.x * blockDim.x) {
        for (int q = 0; q < 4; ++q)
            s[q] += ctr[4 * r + q];
    }
    for (int q = 0; q < 4; ++q) {
        unsigned long long v = s[q];
        for (int off = 32; off >= 1; off >>= 1)
            v += __shfl_xor(v, off);
        if ((threadIdx.x & 63) == 0 && v)
            atomicAdd(&tot[q], v);
    }
}

// ---------------------------------------------------------------------------
// Normalised mutual information of two covers (Sec. 4 compares community
// sets of successive scales with the overlapping-community NMI of
// Lancichinetti, Fortunato and Kertesz, 2009).  Entropies are in nats,
// h(c) = (c / n) (L(n) - L(c)) for a count c of n nodes, taken from a table
// built with the specified integer log, so that the admission test
// h(a) + h(e) > h(b) + h(c) decides exactly as in any other implementation
// of the same specification.  Empty communities are skipped.
// ---------------------------------------------------------------------------
__global__ void nmi_htab_kernel(double *h, int32_t n) {
    const double ln_n = n > 0 ? ilog((uint64_t)n) : 0.0;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c <= n;
         c += (int64_t)gridDim.x * blockDim.x) {
        if (c == 0) {
            h[c] = 0.0;
            continue;
        }
        const double t = ln_n - ilog((uint64_t)c);
        const double p = (double)c / (double)n;
        h[c] = p * t;
    }
}

// H(X_k | Y) / H(X_k) for every community k of X, one wave per community
// from a work counter: the wave counts X_k's intersections with every Y_l
// through Y's node -> communities lists (cnt: one zeroed int32[ky] row per
// wave slot, left zeroed), then takes the least admitted conditional
// entropy over all non-empty Y_l.  term[k] = -1 marks an empty X_k.
__global__ void __launch_bounds__(256) nmi_half_kernel(const int32_t *px, const int32_t *mx, int32_t kx,
                                                       const int32_t *py, int32_t ky, const int32_t *node_ptr,
                                                       const int32_t *node_sets, const double *h, int32_t n,
                                                       int32_t *cnt_all, int32_t n_slots, unsigned *next,
                                                       double *term) {
    const int lane = threadIdx.x & 63;
    const int slot = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (slot >= n_slots)
        return;
    int32_t *cnt = cnt_all + (int64_t)slot * ky;
    // the item is wave-uniform and the loop has no lane-0 block at its end
    for (;;) {
        unsigned item = 0;
        if (lane == 0)
            item = atomicAdd(next, 1u);
        item = (unsigned)__builtin_amdgcn_readfirstlane((int)item);
        if (item >= (unsigned)kx)
            break;
        const int32_t k = (int32_t)item;
        const int32_t x0 = px[k], x1 = px[k + 1];
        const int32_t sx = x1 - x0;
        double out = -1.0;
        if (sx > 0) {
            for (int32_t q = x0 + lane; q < x1; q += 64) {
                const int32_t v = mx[q];
                for (int32_t t = node_ptr[v]; t < node_ptr[v + 1]; ++t)
                    atomicAdd(&cnt[node_sets[t]], 1);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
            const double hx = h[sx] + h[n - sx];
            double best = 0.0;
            int found = 0;
            for (int32_t l = lane; l < ky; l += 64) {
                const int32_t sy = py[l + 1] - py[l];
                if (sy == 0)
                    continue;
                const int32_t a = atomicExch(&cnt[l], 0);   // read at L2 and leave it zero
                const int32_t b = sx - a, c = sy - a, e = n - a - b - c;
                const double ha = h[a], hb = h[b], hc = h[c], he = h[e];
                if (!(ha + he > hb + hc))
                    continue;
                const double hxy = ((ha + hb) + hc) + he;
                const double hy = h[sy] + h[n - sy];
                const double cond = hxy - hy;
                if (!found || cond < best) {
                    best = cond;
                    found = 1;
                }
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                const double b2 = __shfl_xor(best, off);
                const int f2 = __shfl_xor(found, off);
                if (f2 && (!found || b2 < best)) {
                    best = b2;
                    found = 1;
                }
            }
            if (!found)
                best = hx;
            out = hx > 0.0 ? best / hx : 0.0;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
        // every lane stores the same value
        term[k] = out;
    }
}

// Mean of the terms that are not -1 (one workgroup, fixed order), written
// with its count: res[0] = mean, res[1] = count.
__global__ void __launch_bounds__(1024) nmi_mean_kernel(const double *term, int32_t k, double *res) {
    __shared__ double s[1024];
    __shared__ int c[1024];
    double acc = 0.0;
    int cc = 0;
    for (int32_t i = threadIdx.x; i < k; i += 1024) {
        const double x = term[i];
        if (x >= 0.0) {
            acc += x;
            cc += 1;
        }
    }
    s[threadIdx.x] = acc;
    c[threadIdx.x] = cc;
    __syncthreads();
    for (int off = 512; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) {
            s[threadIdx.x] += s[threadIdx.x + off];
            c[threadIdx.x] += c[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        res[0] = c[0] > 0 ? s[0] / (double)c[0] : 0.0;
        res[1] = (double)c[0];
    }
}

// Checks a cover given as CSR: offsets from 0 to total, non-decreasing;
// every community strictly ascending with ids in [0, n).  Any breach sets
// *bad.
__global__ void cover_check_kernel(const int32_t *ptr, const int32_t *mem, int32_t k, int64_t total, int32_t n,
                                   uint32_t *bad) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < k; j += stride) {
        const int32_t a = ptr[j], b = ptr[j + 1];
        if (b < a || a < 0 || (int64_t)b > total || (j == 0 && a != 0) || (j == k - 1 && (int64_t)b != total)) {
            atomicOr(bad, 1u);
            continue;
        }
        for (int32_t q = a; q < b; ++q) {
            const int32_t v = mem[q];
            if (v < 0 || v >= n || (q > a && v <= mem[q - 1])) {
                atomicOr(bad, 1u);
                break;
            }
        }
    }
}

// Means of the p - 1 consecutive pair values of each window of p scales.
__global__ void nmi_windows_kernel(const double *pair, int32_t S, int32_t p, double *out) {
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s > S - p)
        return;
    double acc = 0.0;
    for (int32_t t = s; t < s + p - 1; ++t)
        acc += pair[t];
    out[s] = acc / (double)(p - 1);
}

// NMI from the two halves (N4: a cover without a non-empty community).
__global__ void nmi_final_kernel(const double *hx, const double *hy, double *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const bool ex = hx[1] > 0.0, ey = hy[1] > 0.0;
        if (!ex || !ey)
            *out = (!ex && !ey) ? 1.0 : 0.0;
        else
            *out = 1.0 - (hx[0] + hy[0]) / 2.0;
    }
}

inline int grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g < 1)
        g = 1;
    if (g > 65535 * 64)
        g = 65535 * 64;
    return (int)g;
}

}  // namespace

hipError_t launch_degrees(const int32_t *row_ptr, const uint8_t *w, int32_t *kdeg, int32_t n,
                          hipStream_t st) {
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(degrees_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, row_ptr, w, kdeg, n);
    return hipGetLastError();
}

hipError_t launch_logtab(double *tab, int32_t m, hipStream_t st) {
    hipLaunchKernelGGL(logtab_kernel, dim3(grid_for(m, 256)), dim3(256), 0, st, tab, m);
    return hipGetLastError();
}

hipError_t launch_log(const uint64_t *x, double *out, int64_t n, hipStream_t st) {
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(log_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, x, out, n);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st) {
    if (n == 0)
        return hipSuccess;
    int64_t g = (n + 255) / 256;
    if (g > 16384)
        g = 16384;
    hipLaunchKernelGGL(fill_i32_kernel, dim3((int)g), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t launch_zero_bytes(void *p, int64_t bytes, hipStream_t st) {
    // callers pass 4-byte multiples
    return launch_fill_i32((int32_t *)p, 0, bytes / 4, st);
}

hipError_t launch_sweep(const SweepArgs &a, int32_t blocks, int32_t waves_per_block, hipStream_t st) {
    if (blocks <= 0)
        return hipSuccess;
    const bool q = a.alpha_set != nullptr;
    if (q && (a.S != 1 || a.s_begin != 0 || a.s_end != 1 || a.resume))
        return hipErrorInvalidValue;
    const dim3 grid(blocks), block(64 * waves_per_block);
    switch (a.kind) {
    case TIER_WAVE_LDS: {
        if (waves_per_block < 1 || waves_per_block > 4)
            return hipErrorInvalidValue;
        const size_t smem = (size_t)waves_per_block * (size_t)table_bytes(a.cap, a.hbits);
        hipLaunchKernelGGL(q ? query_lds_kernel : sweep_lds_kernel, grid, block, smem, st, a);
        break;
    }
    case TIER_WAVE_GLOBAL:
        if (waves_per_block < 1 || waves_per_block > 4 || a.gtab == nullptr)
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(q ? query_global_kernel : sweep_global_kernel, grid, block, 0, st, a);
        break;
    case TIER_TEAM_LDS: {
        if (waves_per_block < 1 || 64 * waves_per_block > kTeamMaxThreads)
            return hipErrorInvalidValue;
        const size_t smem = (size_t)table_bytes(a.cap, a.hbits);
        hipLaunchKernelGGL(q ? query_team_lds_kernel : sweep_team_lds_kernel, grid, block, smem, st, a);
        break;
    }
    case TIER_TEAM_GLOBAL:
        if (waves_per_block < 1 || 64 * waves_per_block > kTeamMaxThreads || a.gtab == nullptr)
            return hipErrorInvalidValue;
        if (a.cap >= kRecordMinEntries)
            hipLaunchKernelGGL(q ? query_team_global_rec_kernel : sweep_team_global_rec_kernel, grid, block, 0, st,
                               a);
        else
            hipLaunchKernelGGL(q ? query_team_global_kernel : sweep_team_global_kernel, grid, block, 0, st, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t tier_blocks_per_cu(int32_t kind, int32_t waves, size_t lds_bytes, int32_t *out) {
    const void *f = nullptr;
    switch (kind) {
    case TIER_WAVE_LDS: f = reinterpret_cast<const void *>(&sweep_lds_kernel); break;
    case TIER_WAVE_GLOBAL: f = reinterpret_cast<const void *>(&sweep_global_kernel); break;
    case TIER_TEAM_LDS: f = reinterpret_cast<const void *>(&sweep_team_lds_kernel); break;
    case TIER_TEAM_GLOBAL: f = reinterpret_cast<const void *>(&sweep_team_global_kernel); break;
    default: return hipErrorInvalidValue;
    }
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, 64 * waves, lds_bytes);
    *out = nb;
    return e;
}

hipError_t launch_scale_scan(const Records &rec, int32_t S, int32_t s, int32_t n_sets,
                             int32_t *comm_ptr, long long *total, hipStream_t st) {
    hipLaunchKernelGGL(scale_scan_kernel, dim3(1), dim3(1024), 0, st, rec.cnt, S, s, n_sets, comm_ptr, total);
    return hipGetLastError();
}

hipError_t launch_scale_gather(const Records &rec, const int32_t *pool, const double *scales,
                               int32_t S, int32_t s, int32_t n_sets, const int32_t *comm_ptr,
                               int32_t *members, int64_t *k_in, int64_t *vol, double *f,
                               hipStream_t st) {
    if (n_sets == 0)
        return hipSuccess;
    hipLaunchKernelGGL(scale_gather_kernel, dim3((n_sets + 3) / 4), dim3(256), 0, st, rec, pool, scales,
                       S, s, n_sets, comm_ptr, members, k_in, vol, f);
    return hipGetLastError();
}

hipError_t launch_delta_events(const Records &rec, int32_t S, int32_t s, const int32_t *sets, int32_t n,
                               int64_t *ev, int64_t *ev_off, uint32_t *err, hipStream_t st) {
    if (n > 0) {
        hipLaunchKernelGGL(delta_events_kernel, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)), dim3(256),
                           0, st, rec, S, s, sets, n, ev, err);
    }
    hipLaunchKernelGGL(scan_i64_kernel, dim3(1), dim3(1024), 0, st, ev, (int64_t)n, ev_off);
    return hipGetLastError();
}

hipError_t launch_delta_rebuild(const Records &rec, const int32_t *pool, int32_t S, int32_t s,
                                const int32_t *sets, int32_t n, const int64_t *ev_off, int32_t *scratch,
                                const int32_t *out_ptr, int32_t *members, uint32_t *err, hipStream_t st) {
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(delta_rebuild_kernel, dim3((unsigned)std::min<int64_t>(65536, n)), dim3(256), 0, st, rec,
                       pool, S, s, sets, n, ev_off, scratch, out_ptr, members, err);
    return hipGetLastError();
}

hipError_t launch_delta_lists(const Records &rec, const int32_t *pool, int32_t S, int32_t s, int32_t n,
                              int64_t *na, int64_t *nr, int64_t *add_off, int64_t *rem_off, int32_t *added,
                              int32_t *removed, hipStream_t st) {
    if (n > 0)
        hipLaunchKernelGGL(delta_counts_kernel, dim3((unsigned)std::min<int64_t>(4096, (n + 255) / 256)),
                           dim3(256), 0, st, rec, S, s, n, na, nr);
    hipLaunchKernelGGL(scan_i64_kernel, dim3(1), dim3(1024), 0, st, na, (int64_t)n, add_off);
    hipLaunchKernelGGL(scan_i64_kernel, dim3(1), dim3(1024), 0, st, nr, (int64_t)n, rem_off);
    if ((added || removed) && n > 0)
        hipLaunchKernelGGL(delta_gather_kernel, dim3((n + 3) / 4), dim3(256), 0, st, rec, pool, S, s, n, add_off,
                           added, rem_off, removed);
    return hipGetLastError();
}

hipError_t launch_overlap(const int32_t *comm_ptr, const int32_t *members, int64_t total,
                               int32_t n_sets, int32_t n, int32_t *node_ptr, int32_t *node_sets,
                               int32_t *cnt, int32_t *block_sums, hipStream_t st) {
    hipError_t e;
    if ((e = launch_fill_i32(cnt, 0, (int64_t)n + 1, st)) != hipSuccess)
        return e;
    if (total > 0) {
        hipLaunchKernelGGL(overlap_count_kernel, dim3(grid_for(total, 256) < 8192 ? grid_for(total, 256) : 8192),
                           dim3(256), 0, st, members, total, cnt);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    const int64_t nn = (int64_t)n + 1;
    const int nb = (int)((nn + 1023) / 1024);
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(nb), dim3(1024), 0, st, cnt, nn, node_ptr, block_sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, st, block_sums, nb, block_sums + nb);
    hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(1024), 0, st, node_ptr, nn, block_sums);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if ((e = launch_fill_i32(cnt, 0, (int64_t)n + 1, st)) != hipSuccess)
        return e;
    if (n_sets > 0) {
        hipLaunchKernelGGL(overlap_scatter_kernel, dim3((n_sets + 3) / 4), dim3(256), 0, st, comm_ptr,
                           members, n_sets, node_ptr, cnt, node_sets);
    }
    if (n > 0) {
        const int64_t waves = ((int64_t)n + 63) / 64;
        hipLaunchKernelGGL(overlap_sort_kernel, dim3((int)((waves + 3) / 4)), dim3(256), 0, st, node_ptr,
                           n, node_sets);
    }
    return hipGetLastError();
}

hipError_t launch_order_spills(const int32_t *in, const uint32_t *count, uint32_t n_max, int32_t S,
                               int32_t *out, hipStream_t st) {
    if (S < 2 || S > 1024 || n_max == 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(order_spills_kernel, dim3(1), dim3(1024), 0, st, in, count, n_max, S, out);
    return hipGetLastError();
}

hipError_t launch_exclusive_scan(const int32_t *in, int64_t n, int32_t *out, int32_t *block_sums,
                                 hipStream_t st) {
    const int nb = (int)((n + 1023) / 1024);
    if (nb == 0)
        return hipSuccess;
    if (nb > 1024 * 1024)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(scan_blocks_kernel, dim3(nb), dim3(1024), 0, st, in, n, out, block_sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, st, block_sums, nb, block_sums + nb);
    hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(1024), 0, st, out, n, block_sums);
    return hipGetLastError();
}

hipError_t launch_seed_init(const int32_t *row_ptr, const int32_t *perm, int32_t n, int32_t *pos,
                            uint8_t *st, uint8_t *act, hipStream_t s) {
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(seed_init_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, row_ptr, perm, n, pos, st, act);
    return hipGetLastError();
}

hipError_t launch_seed_round(int32_t rule, const int32_t *row_ptr, const int32_t *col, const int32_t *pos,
                             uint8_t *st, uint8_t *sel, uint8_t *act, uint8_t *near, int32_t *m1, int32_t n,
                             const unsigned *prev, unsigned *undecided, hipStream_t s) {
    if (n == 0)
        return hipSuccess;
    if (rule != 1 && rule != 2)
        return hipErrorInvalidValue;
    const dim3 g(grid_for(n, 256)), b(256);
    hipLaunchKernelGGL(seed_min1_kernel, g, b, 0, s, row_ptr, col, pos, st, act, n, m1, prev, undecided);
    if (rule == 1) {
        hipLaunchKernelGGL(seed_apply1_kernel, g, b, 0, s, row_ptr, col, pos, m1, st, n, undecided);
    } else {
        hipLaunchKernelGGL(seed_min2_kernel, g, b, 0, s, row_ptr, col, pos, st, m1, sel, n, undecided);
        hipLaunchKernelGGL(seed_near_kernel, g, b, 0, s, row_ptr, col, sel, act, n, near, undecided);
        hipLaunchKernelGGL(seed_apply2_kernel, g, b, 0, s, row_ptr, col, sel, near, st, n, undecided);
    }
    return hipGetLastError();
}

hipError_t launch_seed_collect(const int32_t *perm, const uint8_t *st, int32_t n, int32_t *flag, int32_t *at,
                               int32_t *block_sums, int32_t *out, hipStream_t s) {
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(seed_flag_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, perm, st, n, flag);
    hipError_t e = launch_exclusive_scan(flag, n, at, block_sums, s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(seed_scatter_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, perm, flag, at, n, out);
    return hipGetLastError();
}

hipError_t launch_partner(const int32_t *comm_ptr, const int32_t *members, const int32_t *node_ptr,
                          const int32_t *node_sets, const int32_t *list, int32_t n_list, int32_t n_comms,
                          int32_t eta_num, int32_t eta_den, int32_t *cnt_all, int32_t n_slots, unsigned *next,
                          int32_t *partner, hipStream_t st) {
    if (n_list == 0)
        return hipSuccess;
    hipError_t e = launch_zero_bytes(next, 4, st);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(partner_kernel, dim3((n_slots + 3) / 4), dim3(256), 0, st, comm_ptr, members, node_ptr,
                       node_sets, list, n_list, n_comms, eta_num, eta_den, cnt_all, n_slots, next, partner);
    return hipGetLastError();
}

hipError_t launch_nmi_htab(double *h, int32_t n, hipStream_t st) {
    hipLaunchKernelGGL(nmi_htab_kernel, dim3(grid_for((int64_t)n + 1, 256)), dim3(256), 0, st, h, n);
    return hipGetLastError();
}

hipError_t launch_nmi_half(const int32_t *px, const int32_t *mx, int32_t kx, const int32_t *py, int32_t ky,
                           const int32_t *node_ptr, const int32_t *node_sets, const double *h, int32_t n,
                           int32_t *cnt_all, int32_t n_slots, unsigned *next, double *term, double *res,
                           hipStream_t st) {
    hipError_t e = launch_zero_bytes(next, 4, st);
    if (e != hipSuccess)
        return e;
    if (kx > 0)
        hipLaunchKernelGGL(nmi_half_kernel, dim3((n_slots + 3) / 4), dim3(256), 0, st, px, mx, kx, py, ky, node_ptr,
                           node_sets, h, n, cnt_all, n_slots, next, term);
    hipLaunchKernelGGL(nmi_mean_kernel, dim3(1), dim3(1024), 0, st, term, kx, res);
    return hipGetLastError();
}

hipError_t launch_nmi_final(const double *hx, const double *hy, double *out, hipStream_t st) {
    hipLaunchKernelGGL(nmi_final_kernel, dim3(1), dim3(64), 0, st, hx, hy, out);
    return hipGetLastError();
}

hipError_t launch_cover_check(const int32_t *ptr, const int32_t *mem, int32_t k, int64_t total, int32_t n,
                              uint32_t *bad, hipStream_t st) {
    hipError_t e = launch_zero_bytes(bad, 4, st);
    if (e != hipSuccess || k == 0)
        return e;
    hipLaunchKernelGGL(cover_check_kernel, dim3(grid_for(k, 256) < 4096 ? grid_for(k, 256) : 4096), dim3(256), 0, st,
                       ptr, mem, k, total, n, bad);
    return hipGetLastError();
}

hipError_t launch_nmi_windows(const double *pair, int32_t S, int32_t p, double *out, hipStream_t st) {
    if (p < 2 || p > S)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(nmi_windows_kernel, dim3((S - p + 1 + 255) / 256), dim3(256), 0, st, pair, S, p, out);
    return hipGetLastError();
}

hipError_t launch_counter_sum(const uint64_t *ctr, int64_t n_rec, unsigned long long *tot,
                              hipStream_t st) {
    if (n_rec == 0)
        return hipSuccess;
    hipLaunchKernelGGL(counter_sum_kernel, dim3(grid_for(n_rec, 256) < 4096 ? grid_for(n_rec, 256) : 4096),
                       dim3(256), 0, st, ctr, n_rec, tot);
    return hipGetLastError();
}

}  // namespace lcd
