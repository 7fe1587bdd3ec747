// Internal interface between the host API (lcd_api.hip) and the kernels
// (lcd_kernels.hip).  Not installed; the public ABI is include/lcd.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lcd {

// Graph resident in device memory.
struct GraphDev {
    const int32_t *row_ptr;   // [n+1]
    const int32_t *col;       // [nnz]
    const uint8_t *w;         // [nnz] or nullptr (all weights 1)
    const int32_t *kdeg;      // [n] weighted degree
    const double *logtab;     // [logtab_n] L(x) for x < logtab_n
    int32_t n;
    int32_t logtab_n;
};

// Per-record outputs; record r = set * S + s.
//
// Full output: the pool holds record r's sorted member list at off[r]
// (cnt[r] ids; a scale where nothing moved shares the list before it).
// Delta output (dadd, drem non-null): drem[r] < 0 marks a full sorted list
// of cnt[r] ids at off[r] (the first scale a set grew from its seeds);
// otherwise off[r] holds dadd[r] sorted ids that joined since record r - 1,
// then drem[r] sorted ids that left.  cnt[r] is the member count either way.
struct Records {
    int64_t *off;             // member-pool offset of the record's ids
    int32_t *cnt;             // number of members
    int64_t *K;               // k_in
    int64_t *V;               // k_in + k_out
    double *f;                // K / pow(V, alpha)
    uint64_t *ctr;            // G, R, M, C
    int32_t *dadd;            // delta output: ids added (nullptr: full output)
    int32_t *drem;            // delta output: ids removed, -1 for a full list
};

// Error bits written by the kernels.
enum : uint32_t {
    ERR_PROBE = 1u,           // hash probe exceeded the table size
    ERR_MISSING = 2u,         // a neighbour of a member was absent from the table
    ERR_LIMIT = 4u,           // move or growth-call limit of one (set, scale) hit
    ERR_CAPACITY = 8u,        // the largest tier ran out of entries
    ERR_TIMEOUT = 16u         // a seed set ran past the watchdog budget (sweep aborted)
};

// Work-queue state of one launch group (all tiers of one scale range),
// zeroed before the group runs.
struct Counters {
    uint32_t work_next[4];    // per tier: next work item
    uint32_t ovf_count[4];    // per tier: items pushed to the next tier
};

struct SweepArgs {
    GraphDev g;
    const double *scales;
    int32_t S;                // records per set
    int32_t s_begin, s_end;   // scale range of this launch
    const int32_t *seed_ptr;
    const int32_t *seed_nodes;
    int32_t n_sets;
    uint32_t k_prune;
    uint32_t max_calls;       // growth calls per (set, scale); 0 = until one changes nothing
    int32_t queue_min;        // workgroup tiers on global tables: a growth call switches to
                              // the bucketed queue once its table holds this many entries
    int32_t resume;           // 1: start from the records of scale s_begin - 1
    Records rec;
    int32_t *pool;
    int64_t pool_cap;
    Counters *ctl;
    unsigned long long *pool_cursor;   // entries claimed in the pool (may pass pool_cap)
    uint32_t *err;                     // ERR_* bits
    unsigned long long *stat;          // per tier (kStatWords each), over the sets the tier
                                       // finished: rows gathered, their length, entries
                                       // created, pool entries written, sets finished, table
                                       // entries scanned; over every set the tier ran, for
                                       // the scales whose records it wrote: rows gathered by
                                       // moves, their length, seed-set rows, their length,
                                       // entries created after the set's start
    int32_t tier;             // 0 = LDS; 1, 2 = global-memory tiers
    int32_t in_from;          // tier > 0: the tier whose pushes this one consumes
    const int32_t *work_in;   // tier > 0: set ids pushed by that tier
    int32_t *work_out;        // sets pushed to the next tier (nullptr for the last)
    int32_t cap;              // table entries per community
    int32_t hbits;            // hash slots = 2^hbits >= 2 * cap
    char *gtab;               // global tiers: table workspace
    int64_t gtab_stride;      // bytes per table
    int32_t n_slots;          // global tiers: number of tables
    int64_t budget_ticks;     // watchdog: wall-clock ticks one seed set may take
    const double *alpha_set;  // query kernels: one scale per set (S = 1); nullptr for sweeps
    uint32_t *done_flags;     // query kernels: set to 1 (system scope) once set j's record
                              // and members are final; nullptr for none
    int32_t kind;             // TIER_* below: which kernel runs this tier
};

// Table tiers.  A set starts in tier 0 and moves to the next tier (starting
// over from its seeds) when its table would overflow.
enum : int32_t {
    TIER_WAVE_LDS = 0,        // one wave per community, table in LDS
    TIER_WAVE_GLOBAL = 1,     // one wave per community, table in global memory
    TIER_TEAM_LDS = 2,        // one workgroup per community, table in LDS
    TIER_TEAM_GLOBAL = 3      // one workgroup per community, table in global memory
};
constexpr int kMaxTiers = 4;
constexpr int kStatWords = 11;  // statistics words per tier
constexpr int kTeamMaxThreads = 512;

// LDS tables: bytes per entry (one array per field + scratch) and per hash
// slot.
constexpr int kEntryBytes = 4 /*node*/ + 4 /*d|flags*/ + 4 /*k*/ + 8 /*rank*/ + 4 /*scratch*/;
constexpr int kSlotBytes = 4;

__host__ __device__ constexpr int64_t table_bytes(int32_t cap, int32_t hbits) {
    return (int64_t)cap * kEntryBytes + ((int64_t)1 << hbits) * kSlotBytes;
}

// Global tables hold the LDS layout plus the workgroup kernel's
// rank-bucketed queue and fresh list (one int32 entry index per table entry
// each); from kRecordMinEntries entries on, the fields of an entry are one
// 32-byte record instead (d|flags, node, k, rank), since the steps on such
// tables reach most entries at random through the queue.
// Their hash slots hold the node id beside the entry index (8 bytes), so a
// lookup is one load.
constexpr int kRecordBytes = 32;
constexpr int32_t kRecordMinEntries = 65536;
constexpr int kPairSlotBytes = 8;
constexpr int kQueueBytes = 4 /*bucketed queue*/ + 4 /*fresh list*/;

__host__ __device__ constexpr int64_t global_table_bytes(int32_t cap, int32_t hbits) {
    return cap >= kRecordMinEntries
               ? (int64_t)cap * (kRecordBytes + kQueueBytes) + (((int64_t)cap * 4 /*scratch*/ + 7) & ~(int64_t)7) +
                     ((int64_t)1 << hbits) * kPairSlotBytes
               : table_bytes(cap, hbits) + (int64_t)cap * kQueueBytes;
}

hipError_t launch_degrees(const int32_t *row_ptr, const uint8_t *w, int32_t *kdeg, int32_t n,
                          hipStream_t st);
hipError_t launch_logtab(double *tab, int32_t m, hipStream_t st);
hipError_t launch_log(const uint64_t *x, double *out, int64_t n, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t st);
hipError_t launch_zero_bytes(void *p, int64_t bytes, hipStream_t st);
hipError_t launch_sweep(const SweepArgs &a, int32_t blocks, int32_t waves_per_block,
                        hipStream_t st);
// Resident workgroups per compute unit of a tier kernel (TIER_* kind) at the
// given waves per workgroup and dynamic LDS bytes.
hipError_t tier_blocks_per_cu(int32_t kind, int32_t waves, size_t lds_bytes, int32_t *out);
// readout
// comm_ptr[0..n_sets] (int32, wraps past 2^31 - 1) and the exact total in *total
hipError_t launch_scale_scan(const Records &rec, int32_t S, int32_t s, int32_t n_sets,
                             int32_t *comm_ptr, long long *total, hipStream_t st);
// Delta output readout (see Records): ids per listed set in the records
// that rebuild scale s (ev) and their exclusive prefix (ev_off, n + 1
// entries; bit 1 of *err: a set without a full list); the rebuilt sorted
// member lists at out_ptr offsets (scratch holds ev_off[n] ids; bit 2 of
// *err: a count that disagrees with the record); and the added / removed
// ids of scale s with their offsets (n + 1 entries each; a full list counts
// as added; a null added or removed skips that side).
hipError_t launch_delta_events(const Records &rec, int32_t S, int32_t s, const int32_t *sets, int32_t n,
                               int64_t *ev, int64_t *ev_off, uint32_t *err, hipStream_t st);
hipError_t launch_delta_rebuild(const Records &rec, const int32_t *pool, int32_t S, int32_t s,
                                const int32_t *sets, int32_t n, const int64_t *ev_off, int32_t *scratch,
                                const int32_t *out_ptr, int32_t *members, uint32_t *err, hipStream_t st);
hipError_t launch_delta_lists(const Records &rec, const int32_t *pool, int32_t S, int32_t s, int32_t n,
                              int64_t *na, int64_t *nr, int64_t *add_off, int64_t *rem_off, int32_t *added,
                              int32_t *removed, hipStream_t st);
hipError_t launch_scale_gather(const Records &rec, const int32_t *pool, const double *scales,
                               int32_t S, int32_t s, int32_t n_sets, const int32_t *comm_ptr,
                               int32_t *members, int64_t *k_in, int64_t *vol, double *f,
                               hipStream_t st);
// node_ptr[n+1] and node_sets[total] from one scale's member lists; cnt has
// n+1 entries of scratch, block_sums ceil((n+1)/1024)+1.
hipError_t launch_overlap(const int32_t *comm_ptr, const int32_t *members, int64_t total,
                          int32_t n_sets, int32_t n, int32_t *node_ptr, int32_t *node_sets,
                          int32_t *cnt, int32_t *block_sums, hipStream_t st);
hipError_t launch_counter_sum(const uint64_t *ctr, int64_t n_rec, unsigned long long *tot,
                              hipStream_t st);
// NMI of two covers: h[c] for c = 0..n; one half H(X|Y)_norm into res[0]
// (with the number of non-empty X communities in res[1]; term has kx
// entries, cnt_all n_slots zeroed int32[ky] rows, left zeroed); the NMI
// from both halves into *out.
hipError_t launch_nmi_htab(double *h, int32_t n, hipStream_t st);
hipError_t launch_nmi_half(const int32_t *px, const int32_t *mx, int32_t kx, const int32_t *py, int32_t ky,
                           const int32_t *node_ptr, const int32_t *node_sets, const double *h, int32_t n,
                           int32_t *cnt_all, int32_t n_slots, unsigned *next, double *term, double *res,
                           hipStream_t st);
hipError_t launch_nmi_final(const double *hx, const double *hy, double *out, hipStream_t st);
// *bad = 1 unless the cover (CSR with total members) is well formed over n nodes
hipError_t launch_cover_check(const int32_t *ptr, const int32_t *mem, int32_t k, int64_t total, int32_t n,
                              uint32_t *bad, hipStream_t st);
// out[s] = mean of pair[s .. s + p - 2] for s = 0 .. S - p
hipError_t launch_nmi_windows(const double *pair, int32_t S, int32_t p, double *out, hipStream_t st);
// overlap partner of each listed community (check phase); cnt_all holds
// n_slots zeroed int32[n_comms] arrays and is left zeroed
hipError_t launch_partner(const int32_t *comm_ptr, const int32_t *members, const int32_t *node_ptr,
                          const int32_t *node_sets, const int32_t *list, int32_t n_list, int32_t n_comms,
                          int32_t eta_num, int32_t eta_den, int32_t *cnt_all, int32_t n_slots, unsigned *next,
                          int32_t *partner, hipStream_t st);
// exclusive scan of n int32 into out[0..n); block_sums: ceil(n/1024)+1 entries,
// the total lands in block_sums[ceil(n/1024)]
// Reorder the overflow list in[0 .. min(*count, n_max)) of items set * S + s
// into out by ascending s (2 <= S <= 1024).
hipError_t launch_order_spills(const int32_t *in, const uint32_t *count, uint32_t n_max, int32_t S,
                               int32_t *out, hipStream_t st);
hipError_t launch_exclusive_scan(const int32_t *in, int64_t n, int32_t *out, int32_t *block_sums,
                                 hipStream_t st);
// seed selection: pos/st/act setup, one selection round (adds the number of
// undecided candidates at its start to *undecided; does nothing when prev
// is non-null and *prev is 0), and the ordered output.  act[v] = 0 once no
// undecided candidate is left within one hop of v (it stays so); near is
// rule 2's per-round scratch (n bytes).
hipError_t launch_seed_init(const int32_t *row_ptr, const int32_t *perm, int32_t n, int32_t *pos,
                            uint8_t *st, uint8_t *act, hipStream_t s);
hipError_t launch_seed_round(int32_t rule, const int32_t *row_ptr, const int32_t *col, const int32_t *pos,
                             uint8_t *st, uint8_t *sel, uint8_t *act, uint8_t *near, int32_t *m1, int32_t n,
                             const unsigned *prev, unsigned *undecided, hipStream_t s);
hipError_t launch_seed_collect(const int32_t *perm, const uint8_t *st, int32_t n, int32_t *flag, int32_t *at,
                               int32_t *block_sums, int32_t *out, hipStream_t s);

}  // namespace lcd
