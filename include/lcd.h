/*
 * lcd.h — C ABI of the MI355X multi-scale local community sweep.
 *
 * The library grows communities under the LFK fitness
 *     f_c = k_in / (k_in + k_out)^alpha                (paper Sec. 2, Eq. 1)
 * by the growth function of Algorithm 1 (priority-queue additions ranked by
 * 2 d_in / (d_in + d_out)^alpha, then removal passes), repeated until
 * nothing changes at one scale and chained from each scale to the next
 * coarser one (Sec. 2 and the growth half of Algorithm 2).  In lcd_sweep and
 * the query server every seed set is an independent community;
 * lcd_sweep_merge adds the check-and-merge phase of Algorithm 2.
 * Paper: E. Le Martelot and C. Hankin, "Fast Multi-Scale Community
 * Detection based on Local Criteria within a Multi-Threaded Algorithm",
 * arXiv:1301.0955.  Each call below names the passage that defines what it
 * computes.
 *
 * Exact semantics (shared with the test oracle, written independently):
 *   - k_in counts internal edges from both ends: adding node n raises it by
 *     2 d_in(n); k_in + k_out is the volume V (sum of member degrees).
 *     Weights are integers 1..255 (or all 1), so every term is an exact
 *     integer.
 *   - "n improves f_c" is  t = (L(K')-L(K)) - alpha (L(V')-L(V)) > 2^-40
 *     in IEEE double, where L is the integer natural log given in the
 *     design notes; K' = 0 never improves, K = 0 < K' always does.
 *   - queue rank R = L(2 d_in) - alpha L(k); equal ranks pop the smaller id;
 *     a node that was popped and rejected returns to the queue only when a
 *     later addition changes its d_in.
 *   - removal passes visit the members present at the start of the pass in
 *     ascending id; at most k_prune passes (0 = until nothing is removed);
 *     no pass when the call added nothing.
 *
 * Conventions for every call:
 *   - Every function returns an lcd_status; nothing aborts or throws across
 *     the ABI.  lcd_last_error() gives a thread-local message for the last
 *     non-OK status of the calling thread.
 *   - Input arrays stay owned by the caller and are copied before the call
 *     returns; the library never keeps a caller pointer.
 *   - mem_kind says where caller arrays live: LCD_MEM_HOST (pageable or
 *     pinned host memory) or LCD_MEM_DEVICE (device memory of the current
 *     HIP device).
 *   - stream is a hipStream_t (NULL = the null stream).  Work is queued on
 *     it; calls documented as blocking synchronise that stream before they
 *     return.
 *   - Handles are owned by the library and freed by their *_free call.
 */
#ifndef LCD_H
#define LCD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LCD_OK = 0,
    LCD_EINVAL = 1,     /* an argument breaks its documented contract */
    LCD_ENOMEM = 2,     /* device or host allocation failed */
    LCD_EDEVICE = 3,    /* a HIP call failed or a kernel reported an error */
    LCD_EAGAIN = 4,     /* result not ready yet (server poll) */
    LCD_ECAPACITY = 5,  /* a caller buffer or a fixed capacity is too small */
    LCD_ESTATE = 6,     /* the handle is not in a state that allows the call */
    LCD_ECANCELED = 7   /* a server query that lcd_server_cancel withdrew */
} lcd_status;

enum { LCD_MEM_HOST = 0, LCD_MEM_DEVICE = 1 };

/* lcd_params.mode */
enum {
    LCD_PERSISTENT = 0,     /* all scales and seed sets in one persistent launch */
    LCD_PER_SCALE_LOOP = 1  /* one launch per scale, state re-read from memory */
};

/* lcd_params.output_mode: how a sweep stores each (seed set, scale) community.
 * Either way the readout calls return whole sorted member lists. */
enum {
    LCD_OUT_FULL = 0,   /* a scale where anything moved stores its sorted member list */
    LCD_OUT_DELTA = 1   /* a set's first scale stores its sorted member list; every
                           later scale only the sorted ids that joined and left since
                           the scale before (lcd_result_delta reads them) */
};

typedef struct lcd_graph lcd_graph;
typedef struct lcd_result lcd_result;
typedef struct lcd_server lcd_server;

typedef struct {
    uint32_t k_prune;        /* removal passes per growth call; 0 = unbounded */
    int32_t mode;            /* LCD_PERSISTENT or LCD_PER_SCALE_LOOP */
    int32_t lds_capacity;    /* tier 0: table entries per community held in LDS;
                                0 = tuned (lcd_tune) or 512 */
    int32_t waves_per_block; /* communities (one wave each) per workgroup; 0 = default */
    int32_t blocks_per_cu;   /* resident workgroups per compute unit; 0 = default */
    int32_t use_graph;       /* 1 (persistent mode): capture the sweep's launch sequence
                                (fill kernels and every tier) in a hipGraph, launch
                                it, and replay it on lcd_result_rerun() */
    int64_t pool_hint;       /* initial member-pool size in entries; 0 = estimate */
    int32_t watchdog_ms;     /* wall-clock budget of one seed set; past it the sweep
                                stops with LCD_EDEVICE.  0 = default (20000);
                                negative = no budget at all (tests the error path) */
    int32_t spill_mode;      /* sets whose table outgrows tier 0: 0 = workgroup tiers
                                (one workgroup per community: an LDS table of
                                team_capacity entries, then global-memory tables);
                                1 = one-wave global-memory tiers; 2 = one-wave
                                global tables of 16,384 entries, then workgroups
                                on tables that hold every node */
    int32_t team_capacity;   /* spill_mode 0: entries of the workgroup tier's LDS table;
                                0 = max(1,024, 2 lds_capacity), within one workgroup's LDS */
    int32_t team_waves;      /* waves per community in the workgroup tiers, 1..8;
                                0 = 4 (2 on graphs of 4M+ nodes) */
    int32_t grow_calls;      /* growth calls per (seed set, scale): 0 = until a call
                                changes nothing (the default); n > 0 stops after
                                n calls (lcd_sweep_merge makes one per round) */
    int32_t queue_min_entries; /* workgroup tiers on global tables: once the table of a
                                growth call holds this many entries (checked after
                                each addition) the call keeps its queue bucketed by
                                rank (a step looks at the queue's head, not the
                                whole table); 0 = default (1,024); results never
                                depend on it */
    int32_t output_mode;     /* LCD_OUT_FULL (default) or LCD_OUT_DELTA: lcd_sweep and
                                lcd_sweep_batch only (the other calls store full
                                lists); it changes what the member pool holds, never
                                the communities read back */
} lcd_params;

/* Work of one table tier (0 = one wave per community with an LDS table; the
 * later tiers hold larger tables, see lcd_params.spill_mode), counted over
 * the seed sets that tier finished. */
typedef struct {
    int64_t rows_gathered;    /* CSR rows read: one per move and per initial member */
    int64_t row_entries;      /* total length of those rows */
    int64_t entries_created;  /* table entries created (one degree read each) */
    int64_t members_written;  /* member ids written to the output pool */
    int64_t sets_finished;    /* seed sets completed in this tier */
    int64_t entries_scanned;  /* table entries the tier's growth scans visited (the
                                 sequential algorithm's own visits are the counter G) */
    /* Algorithmic work, over every set the tier ran (finished or passed on),
     * for the scales whose records the tier wrote: a scale whose table
     * overflowed is redone by the next tier and counted there. */
    int64_t move_rows;        /* CSR rows gathered by additions and removals */
    int64_t move_row_entries; /* ... their total length */
    int64_t seed_rows;        /* rows of the seed-set members, in a set's first tier
                                 (a set resumed from a record gathers again: overhead) */
    int64_t seed_row_entries; /* ... their total length */
    int64_t entries_committed;/* table entries created for those scales (one degree read
                                 each; entries rebuilt when a set resumes excluded) */
} lcd_tier_stats;

/* Timing and bookkeeping of one sweep (filled by lcd_result_stats). */
typedef struct {
    double ms_total;          /* device time of the whole sweep (hipEvents on the caller's stream) */
    double ms_main;           /* device time of tier 0 */
    double ms_spill;          /* device time of the later tiers */
    int64_t n_spilled;        /* seed sets that left tier 0 */
    int64_t n_spilled_big;    /* ... of which reached the last tier */
    int64_t pool_used;        /* member-pool entries written */
    int32_t reruns;           /* relaunches after the member pool had to grow */
    int32_t lds_capacity;     /* table entries per community in LDS actually used */
    int32_t waves_per_block;
    int32_t grid_blocks;      /* workgroups of the LDS-resident launch */
    int32_t launches;         /* kernel launches of the sweep (excluding readout) */
    int32_t tiers;            /* tiers in the launch chain */
    lcd_tier_stats tier[4];
    double ms_tier[4];        /* device time of each tier (persistent mode, no hipGraph) */
    int32_t tier_kind[4];     /* 0 one wave + LDS table, 1 one wave + global table,
                                 2 workgroup + LDS table, 3 workgroup + global table */
    int32_t tier_capacity[4]; /* table entries per community of each tier */
} lcd_sweep_stats;

/* Fill *p with the defaults (k_prune 0, persistent mode, autotuned sizes). */
void lcd_params_default(lcd_params *p);

/*
 * Upload an undirected graph in symmetric CSR form and keep it resident.
 * Paper: Sec. 2 (the graph is undirected and weighted: d_in, d_out and the
 * node degree k in the fitness of Eq. 1 and the queue factor of Algorithm 1
 * are sums of edge weights); Sec. 3 (complexity: direct access to each
 * node's neighbours).
 *   n        nodes, 0 <= n < 2^31
 *   nnz      directed entries (twice the undirected edges), < 2^31
 *   row_ptr  int32[n+1], row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz
 *   col      int32[nnz], each row strictly ascending, ids in [0, n), no
 *            self-loops; symmetric (v in row u <=> u in row v)
 *   w        uint8[nnz] weights >= 1, equal on both directions, or NULL for
 *            all weights 1
 * Validation (host side, before any device work) returns LCD_EINVAL when
 * any rule above is broken, or the weighted degree exceeds 2^27.
 * Blocking.  Derived data built on the device: weighted degrees and the
 * table L(x) for x <= 2 * max weighted degree.
 */
lcd_status lcd_graph_upload(int32_t n, int64_t nnz, const int32_t *row_ptr,
                            const int32_t *col, const uint8_t *w, int32_t mem_kind,
                            void *stream, lcd_graph **out);

/*
 * Upload n_graphs independent graphs as one resident batch (sweeps over all
 * of them run in one launch).  Each member graph obeys the rules of
 * lcd_graph_upload in its own local ids:
 *   node_off, edge_off  int64[n_graphs+1], starting at 0, non-decreasing:
 *                       graph i has node_off[i+1]-node_off[i] nodes and
 *                       edge_off[i+1]-edge_off[i] directed entries
 *   row_ptr  int32[node_off[n_graphs] + n_graphs]: graph i's local offsets
 *            (n_i + 1 of them, from 0 to its entry count) at row_ptr + node_off[i] + i
 *   col      int32[edge_off[n_graphs]]: graph-local neighbour ids, graph i's
 *            at col + edge_off[i]
 *   w        uint8[edge_off[n_graphs]] or NULL
 * The batch is stored as the disjoint union: node u of graph i has batch id
 * node_off[i] + u, and member lists of sweeps over it use batch ids.
 */
lcd_status lcd_graph_upload_batch(int32_t n_graphs, const int64_t *node_off, const int64_t *edge_off,
                                  const int32_t *row_ptr, const int32_t *col, const uint8_t *w,
                                  int32_t mem_kind, void *stream, lcd_graph **out);

/* Member graphs of a batch (1 for a plain graph) and node_off[n_graphs+1]
 * (host memory; may be NULL). */
lcd_status lcd_graph_batch_info(const lcd_graph *g, int32_t *n_graphs, int64_t *node_off);

/* n, nnz, max weighted degree and total volume (sum of weighted degrees). */
lcd_status lcd_graph_info(const lcd_graph *g, int32_t *n, int64_t *nnz,
                          int64_t *max_degree, int64_t *volume);

lcd_status lcd_graph_free(lcd_graph *g);

/*
 * Grow every seed set through every scale.
 * Paper: Sec. 2, Eq. 1 (fitness) and Eq. 2 (node fitness, the add and
 * remove tests); Algorithm 1 (one growth call: queue ranked by
 * 2 d_in / (d_in + d_out)^alpha, additions, then removal passes);
 * Algorithm 2 (initial communities given as input; for each scale, growth
 * repeated while it changes something, then the next scale starts from the
 * result), without its check-and-merge phase.
 *   scales      double[n_scales], finite, >= 0, <= 1000, strictly decreasing
 *               (finest first: large alpha = small communities)
 *   seed_ptr    int32[n_sets+1] offsets into seed_nodes; set j is
 *               seed_nodes[seed_ptr[j] .. seed_ptr[j+1]) (non-empty, ids in
 *               range, no repeats inside a set).  n_sets may be 0;
 *               n_sets x n_scales must stay below 2^31.
 *   params      NULL for defaults
 * The result holds, for each record r = j * n_scales + s: the sorted member
 * list, K = k_in, V = k_in + k_out, f = K / pow(V, alpha_s) and the work
 * counters (criterion evaluations G, rank updates R, moves M, growth calls C).
 * Blocking: the work is queued on stream and the call returns after the
 * sweep has finished there (the library reads the device's error word and
 * member-pool fill to grow the pool and run again if it overflowed).
 * Errors: LCD_EINVAL for an argument outside the rules above;
 * LCD_ENOMEM when device memory runs out; LCD_ECAPACITY when a set's table
 * outgrows the largest tier; LCD_EDEVICE for a failed launch or a kernel
 * error (watchdog, probe failure).  On error *out is NULL.
 */
lcd_status lcd_sweep(const lcd_graph *g, const double *scales, int32_t n_scales,
                     const int32_t *seed_ptr, const int32_t *seed_nodes, int32_t n_sets,
                     int32_t mem_kind, const lcd_params *params, void *stream,
                     lcd_result **out);

/*
 * lcd_sweep for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same sweep and
 * the same records, written into caller buffers; the library allocates
 * nothing, on the device or the host.  Its working memory (work queues,
 * counters, LCD_NOALLOC_TABLES global-memory tables of the workgroup tier)
 * is one static device array of LCD_NOALLOC_SCRATCH_BYTES that each GPU the
 * library runs on holds until the process ends.  Every call on a GPU uses
 * that GPU's array, so calls that overlap on one GPU race: issue them in
 * order.
 *   scales, seed_ptr, seed_nodes  device arrays, rules as in lcd_sweep;
 *            n_seed_nodes = seed_ptr[n_sets] (the length of seed_nodes)
 *   rec_off int64, rec_cnt int32, rec_k int64, rec_v int64, rec_f double
 *            (n_sets * n_scales each) and rec_ctr uint64 (4 per record):
 *            device arrays; record r = set * n_scales + s as in lcd_sweep:
 *            members of r at members[rec_off[r] .. + rec_cnt[r]), ascending
 *   members  device int32[members_cap]; *members_used (host) receives the
 *            entries the sweep wrote or needed
 *   params   as lcd_sweep (spill_mode 0, persistent mode, no use_graph)
 * Limits: n_sets <= LCD_NOALLOC_MAX_SETS, n_scales <= LCD_NOALLOC_MAX_SCALES,
 * seed sets of at most LCD_NOALLOC_MAX_SEED_SET nodes, and tables of at most
 * LCD_NOALLOC_TABLE_ENTRIES entries per community (larger communities need
 * lcd_sweep's whole-graph tier).
 * Errors: LCD_EINVAL for arguments outside the rules (inputs are checked on
 * the device); LCD_ECAPACITY when a limit above is passed or members_cap is
 * too small (*members_used then holds the size needed; the records are not
 * valid); LCD_EDEVICE for a failed launch or a kernel error.  Blocking.
 */
#define LCD_NOALLOC_SCRATCH_BYTES (24 << 20)
#define LCD_NOALLOC_MAX_SETS 65536
#define LCD_NOALLOC_MAX_SCALES 1024
#define LCD_NOALLOC_MAX_SEED_SET 4096
#define LCD_NOALLOC_TABLE_ENTRIES 16384
#define LCD_NOALLOC_TABLES 32
lcd_status lcd_sweep_into(const lcd_graph *g, const double *scales, int32_t n_scales,
                          const int32_t *seed_ptr, const int32_t *seed_nodes, int32_t n_sets,
                          int64_t n_seed_nodes, const lcd_params *params, int64_t *rec_off,
                          int32_t *rec_cnt, int64_t *rec_k, int64_t *rec_v, double *rec_f,
                          uint64_t *rec_ctr, int32_t *members, int64_t members_cap,
                          int64_t *members_used, void *stream);

/* Result of lcd_tune(). */
typedef struct {
    lcd_params best;          /* the chosen sizing (the graph keeps it) */
    double ms_best;           /* device time of one sweep of the sample with it */
    int32_t n_tried;
    int32_t sample_stride;    /* every sample_stride-th seed set was timed */
    int32_t full_checked;     /* 1: the three fastest were re-timed on every set */
    int32_t pad;
    double ms[16];            /* device time of the sample per candidate */
    lcd_params tried[16];
} lcd_tune_report;

/*
 * Autotuner: time one sweep of a sample of the given seed sets (every
 * stride-th set, at most ~16k sets) with each of a fixed list of launch
 * sizings (tier-0 LDS table, spill mode, workgroup table, waves per
 * community) and keep the fastest on the graph.  Later lcd_sweep() and
 * lcd_server_create() calls whose params leave every sizing field at 0 use
 * it.  k_prune and watchdog_ms come from base (NULL = defaults).  Results
 * of a sweep never depend on the sizing; only the time does.  Blocking;
 * runs 2 x 14 sample sweeps, then the three fastest sizings once on every
 * set when that full sweep is expected to take under 5 s.
 */
lcd_status lcd_tune(lcd_graph *g, const double *scales, int32_t n_scales, const int32_t *seed_ptr,
                    const int32_t *seed_nodes, int32_t n_sets, int32_t mem_kind, const lcd_params *base,
                    void *stream, lcd_tune_report *report);

/* Forget the tuned sizing (later calls use the static defaults). */
lcd_status lcd_graph_untune(lcd_graph *g);

/*
 * Seed selection of the initialisation step of Algorithm 2 (Sec. 3) on the
 * device.  Candidates are the nodes with at least two neighbours; nodes are
 * visited in the order perm (int32[n], a permutation of 0..n-1: the random
 * choice, drawn by the caller); a visited node that is still a candidate
 * becomes a seed and drops its neighbours (rule 1) or every node within two
 * hops (rule 2) from the candidates.  out_seeds (int32[n], mem_kind memory)
 * receives the seeds in order of selection, *n_seeds their number (entries
 * past it are not written); seed j is the singleton seed set j of a sweep.
 * Computed in parallel rounds that give exactly the sequential result.
 * LCD_EINVAL if perm is not a permutation.  The graph keeps the call's
 * device workspace (about 24 bytes per node) for the next call, so calls on
 * one graph must not overlap.
 * Blocking.
 */
lcd_status lcd_seeds(const lcd_graph *g, int32_t rule, const int32_t *perm, int32_t mem_kind, void *stream,
                     int32_t *out_seeds, int32_t *n_seeds);

/*
 * lcd_sweep over a batch graph with graph-local seeds: seed set j lives in
 * member graph seed_graph[j] (int32[n_sets], in mem_kind memory) and its
 * seed ids are local to that graph.  The result is that of lcd_sweep() on
 * the batch with the seeds translated to batch ids; every community stays
 * inside its own member graph (no edges join them).
 */
lcd_status lcd_sweep_batch(const lcd_graph *g, const double *scales, int32_t n_scales,
                           const int32_t *seed_ptr, const int32_t *seed_nodes, const int32_t *seed_graph,
                           int32_t n_sets, int32_t mem_kind, const lcd_params *params, void *stream,
                           lcd_result **out);

/*
 * The multi-scale loop with its check-and-merge phase (Sec. 3, Algorithm 2
 * with the overlap pre-test of Algorithm 3).  At each scale, rounds until a
 * round neither grows nor merges:
 *   - a live community that shares, counted over its members in ascending
 *     order, at least eta * min(|c|, |i|) nodes with another live
 *     community i (eta = eta_num / eta_den; the paper's 0.5 is 1 / 2) is
 *     not grown in that round;
 *   - every other community that needs it makes one call of the growth
 *     function at the scale (each live one at the start of a scale, then
 *     those that the last call changed and the survivors of merges); the
 *     round repeats while a call changed something or a pair merged;
 *   - each pre-tested or changed community with such a partner forms the
 *     pair (lower id, higher id); the pairs, ascending, merge in passes of
 *     pairwise disjoint pairs into their lower ids (union of members; the
 *     higher id dies and is renamed in the remaining pairs).
 * The result is read like lcd_sweep's; a community that died reports no
 * members and K = V = 0 from that scale on, and lcd_result_merged_into()
 * names the live id it went into.  Seeds, scales, params as in lcd_sweep
 * (mode and use_graph ignored); every seed set must be non-empty.  Blocking.
 * The result is freed with lcd_result_free() and cannot be rerun.
 * Errors: LCD_EINVAL for a null graph or out, eta_num or eta_den < 1, scales
 * not finite, outside [0, 1000] or not strictly decreasing, an empty seed
 * set, a seed out of range or repeated within its set; LCD_ECAPACITY when the
 * live communities of a round hold 2^31 members or more in all; LCD_ENOMEM
 * when device memory runs out; LCD_EDEVICE for a failed launch or copy, or a
 * scale that has not settled after 100,000 rounds.
 */
lcd_status lcd_sweep_merge(const lcd_graph *g, const double *scales, int32_t n_scales, const int32_t *seed_ptr,
                           const int32_t *seed_nodes, int32_t n_sets, int32_t eta_num, int32_t eta_den,
                           int32_t mem_kind, const lcd_params *params, void *stream, lcd_result **out);

/* For each seed set at one scale: -1 if its community is live, else the live
 * id it was merged into (host memory, int32[n_sets]).  All -1 for results of
 * lcd_sweep. */
lcd_status lcd_result_merged_into(const lcd_result *r, int32_t scale_idx, int32_t *into);

/*
 * Sweep shape, and the total number of members listed at one scale (the
 * size the members buffer of lcd_result_membership needs).
 * Paper: Algorithm 2 stores the community set and its quality for every
 * scale.  LCD_EINVAL for a null result or a scale index out of range.
 * Blocking.
 */
lcd_status lcd_result_shape(const lcd_result *r, int32_t *n_sets, int32_t *n_scales);
lcd_status lcd_result_sizes(const lcd_result *r, int32_t scale_idx, int64_t *total_members);

/*
 * Communities at one scale, in caller buffers (all in mem_kind memory).
 * Paper: Algorithm 2 (the community set and its quality stored per scale);
 * Sec. 3 (community nodes kept sorted); f is Eq. 1 at that scale.
 * LCD_ECAPACITY when the scale lists 2^31 members or more in all (int32
 * offsets cannot address them); nothing is written then.
 *   comm_ptr int32[n_sets+1]    offsets into members
 *   members  int32[total]       each community ascending
 *   k_in, vol int64[n_sets], f double[n_sets]   (each may be NULL)
 * Blocking.
 */
lcd_status lcd_result_membership(const lcd_result *r, int32_t scale_idx, int32_t *comm_ptr,
                                 int32_t *members, int64_t *k_in, int64_t *vol, double *f,
                                 int32_t mem_kind, void *stream);

/*
 * Overlap at one scale: for every node, the seed sets whose community holds
 * it.  Paper: Sec. 3 (the per-node membership sets that the check phase of
 * Algorithm 2 reads).  LCD_ECAPACITY, as for lcd_result_membership, when
 * the scale lists 2^31 members or more.
 *   node_ptr  int32[n+1], node_sets int32[total members], ascending per node.
 * Blocking.
 */
lcd_status lcd_result_overlap(const lcd_result *r, int32_t scale_idx, int32_t *node_ptr,
                              int32_t *node_sets, int32_t mem_kind, void *stream);

/*
 * Work counters: totals[4] = sums of G, R, M, C over all records (host
 * memory); per_record (n_sets * n_scales * 4, in mem_kind memory) may be NULL.
 * Paper: the counts are those of a sequential run of Algorithm 1 and the
 * scale loop of Algorithm 2: G = queue pops plus members visited by the
 * removal passes (one evaluation of Eq. 2 each), R = queue (re)insertions
 * with a fresh rank, M = nodes added or removed, C = growth calls.
 * Blocking.
 */
lcd_status lcd_result_counters(const lcd_result *r, uint64_t *totals, uint64_t *per_record,
                               int32_t mem_kind, void *stream);

/*
 * What changed at one scale, for a sweep run with output_mode = LCD_OUT_DELTA
 * (LCD_ESTATE otherwise).  Paper: Sec. 2 and Algorithm 2 (the community of
 * one scale is the starting point of the next, so consecutive scales differ
 * by the nodes the growth function added and removed).  For set j: the ids
 * that joined its community between scale_idx - 1 and scale_idx at
 * added[add_ptr[j] .. add_ptr[j+1]), those that left at
 * removed[rem_ptr[j] .. rem_ptr[j+1]), each run ascending; at scale 0 (and at
 * any scale stored as a full list) the whole community counts as added.
 *   add_ptr, rem_ptr int64[n_sets+1]; added, removed int32 (sizes from
 *   lcd_result_delta_sizes); all in mem_kind memory.
 * Blocking.
 */
lcd_status lcd_result_delta_sizes(const lcd_result *r, int32_t scale_idx, int64_t *n_added,
                                  int64_t *n_removed);
lcd_status lcd_result_delta(const lcd_result *r, int32_t scale_idx, int64_t *add_ptr, int32_t *added,
                            int64_t *rem_ptr, int32_t *removed, int32_t mem_kind, void *stream);

/*
 * Every scale of selected seed sets, in host memory.  For the q-th id and
 * scale s (record o = q * n_scales + s): members[rec_off[o] .. +rec_cnt[o])
 * ascending, k_in[o], vol[o], f[o], ctr[4*o .. 4*o+4) (G, R, M, C).
 * members may be NULL to learn *members_needed first; k_in, vol, f, ctr may
 * be NULL.  LCD_ECAPACITY (with *members_needed set) when members_cap is too
 * small.  Blocking.
 */
lcd_status lcd_result_sets(const lcd_result *r, const int32_t *set_ids, int32_t n_ids,
                           int64_t *rec_off, int32_t *rec_cnt, int32_t *members, int64_t members_cap,
                           int64_t *members_needed, int64_t *k_in, int64_t *vol, double *f,
                           uint64_t *ctr);

lcd_status lcd_result_stats(const lcd_result *r, lcd_sweep_stats *out);

/* ------------------------------------------------------------------------
 * Multi-scale relevance analysis.  Paper: Sec. 4 compares the community sets
 * of successive scales, and with the planted ones, by the normalised mutual
 * information for overlapping communities of Lancichinetti, Fortunato and
 * Kertesz (2009), averaged over p successive scales (p = 3 and 5 there).
 * The paper cites the definition without printing it; restated: each
 * community is a binary variable over the n nodes; H(X_k | Y_l) counts only
 * when h(a) + h(e) > h(b) + h(c) for the intersection counts a, b, c, e;
 * H(X_k | Y) is the least counting one (H(X_k) if none); NMI = 1 - (mean_k
 * H(X_k|Y)/H(X_k) + mean_l H(Y_l|X)/H(Y_l)) / 2.  Entropies are in nats,
 * h(c) = (c / n)(L(n) - L(c)) with the integer log L of the decisions, so
 * the admission test decides the same way in every implementation of this
 * specification.  Empty communities are skipped; a cover without a
 * non-empty community gives 1 against another such cover, else 0.  Cost
 * O(kx * ky + intersections).  All blocking; *out in host memory.
 * ------------------------------------------------------------------------ */

/* Two covers of n nodes as device CSR arrays: community j of X is
 * mem_x[ptr_x[j] .. ptr_x[j+1]), strictly ascending ids in [0, n).
 * LCD_EINVAL for a malformed cover. */
lcd_status lcd_cover_nmi(int32_t n, int32_t kx, const int32_t *ptr_x, const int32_t *mem_x, int32_t ky,
                         const int32_t *ptr_y, const int32_t *mem_y, double *out, void *stream);

/* The community sets of scales s1 and s2 of a result (one community per
 * record, empty records skipped). */
lcd_status lcd_result_nmi(const lcd_result *r, int32_t s1, int32_t s2, double *out, void *stream);

/* The NMI averaged over p successive scales: out[s] (s = 0 .. n_scales - p)
 * is the mean of NMI(scale t, scale t + 1) for t = s .. s + p - 2. */
lcd_status lcd_result_nmi_successive(const lcd_result *r, int32_t p, double *out, void *stream);

/* One scale's community set against a given cover of the graph's nodes
 * (device CSR as in lcd_cover_nmi), e.g. the planted communities. */
lcd_status lcd_result_nmi_cover(const lcd_result *r, int32_t scale_idx, int32_t k, const int32_t *ptr,
                                const int32_t *mem, double *out, void *stream);

/*
 * Run the same sweep again (same graph, scales and seed sets, still on the
 * device) into the same result, overwriting it; with use_graph the captured
 * hipGraph is replayed (captured again if the member pool or the graph's
 * spill tables were reallocated since).  Sweeps of one graph must not run
 * concurrently: they share its spill-tier tables.  Blocking.  LCD_EINVAL for
 * a result of lcd_sweep_merge().
 */
lcd_status lcd_result_rerun(lcd_result *r, void *stream);

lcd_status lcd_result_free(lcd_result *r);

/* ------------------------------------------------------------------------
 * Query server.  A resident graph answers local-community queries: a query
 * (S, alpha) starts from the seed set S and applies the growth function of
 * Algorithm 1 at the single scale alpha until nothing changes (the per-scale
 * step of Sec. 2 without chaining), with k_prune as in lcd_params.  The
 * result (members ascending, K, V, f, counters) is exactly that of
 * lcd_sweep() with n_scales = 1 and the same seed set; it does not depend on
 * which other queries run at the same time.
 *
 * Queries are batched as they arrive: a worker thread owned by the server
 * admits waiting queries into any idle launch lane (each lane a HIP stream
 * with its own buffers), limited by max_slots queries in flight and by the
 * lane's member pool, so batches of several lanes run on the device at once.
 * Entry lanes run tier 0 (one wave per query, LDS table); queries whose
 * table outgrows it go on to spill lanes running the larger tiers, so that
 * a few large communities do not hold back the batches of small ones.
 * ------------------------------------------------------------------------ */

/* Outcome of one query (filled by lcd_server_poll). */
typedef struct {
    int32_t n_members;
    int32_t batch_size;       /* queries in the launch that answered it */
    int64_t k_in, vol;
    double f;                 /* K / pow(V, alpha) */
    uint64_t ctr[4];          /* G, R, M, C */
    int64_t t_submit_ns;      /* CLOCK_MONOTONIC stamps: submitted, launched, done */
    int64_t t_start_ns;
    int64_t t_done_ns;
    int32_t lane;             /* launch lane (stream) that ran it */
    int32_t pad;
} lcd_query_info;

typedef struct {
    int64_t submitted, completed, failed;
    int64_t batches;          /* launches of query batches (both lane kinds) */
    int64_t requeued;         /* queries run again alone after a pool overflow */
    int64_t pending;          /* waiting for an entry lane now */
    int64_t in_flight;        /* admitted and not finished now */
    int64_t mem_held;         /* device bytes the server holds */
    int64_t forwarded;        /* moves of a query to the next stage (it outgrew its
                                 stage's table); one stage per tier */
    int64_t spill_batches;    /* launches of lanes of stages after the first */
    int32_t lanes, spill_lanes, max_slots;
    int32_t max_batch;        /* largest batch launched */
    int32_t max_lanes_busy;   /* most lanes with a batch on the device at once */
    int32_t spill_tables[2];  /* global-memory tables per spill lane, per global tier */
    int32_t pad;
    int64_t cancelled;        /* queries withdrawn by lcd_server_cancel */
    int64_t routed;           /* queries queued straight to a later stage: their
                                 seeds and the seeds' neighbours alone
                                 already overflow the earlier stages' tables */
} lcd_server_stats;

/*
 * Create a server on the current device (the graph's device).
 *   mem_budget  device bytes the server may allocate (0 = 1 GiB); it must
 *               not exceed the free device memory (LCD_ENOMEM) and must
 *               cover the lanes, each able to hold any single query
 * Lanes are HIP streams; HIP spreads a process's streams over
 * GPU_MAX_HW_QUEUES hardware queues (4 unless set before the HIP runtime
 * starts).  With 8 or more the server runs one stage per table tier on six
 * lanes (a query moves to the next stage's lane when it outgrows its
 * stage's table), otherwise tier 0 on one lane and the later tiers on three.
 * A query whose seeds and their neighbours outnumber a stage's table starts
 * at the first stage whose table holds them (graphs of up to 2^28 adjacency
 * entries, whose CSR the server keeps a host copy of; the stage never
 * changes a result).
 *   max_slots   queries admitted and unfinished at once (0 = 1024)
 *   params      k_prune, lds_capacity, waves_per_block, watchdog_ms used;
 *               NULL for defaults
 * The graph must outlive the server.
 */
lcd_status lcd_server_create(const lcd_graph *g, int64_t mem_budget, int32_t max_slots,
                             const lcd_params *params, lcd_server **out);

/*
 * Queue one query: n >= 1 distinct seed ids in [0, n_nodes) in host memory
 * (copied), alpha finite in [0, 1000].  Returns at once with a ticket.
 * Thread-safe.
 */
lcd_status lcd_server_submit(lcd_server *s, const int32_t *seeds, int32_t n, double alpha,
                             uint64_t *ticket);

/*
 * Result of a ticket.  LCD_EAGAIN while it runs.  When done: *info is
 * filled (if not NULL) and the members are copied to members[0 .. cap);
 * with cap too small the call returns LCD_ECAPACITY (info->n_members set)
 * and the ticket stays valid.  LCD_OK and a query's own error status
 * retire the ticket.  Thread-safe.
 */
lcd_status lcd_server_poll(lcd_server *s, uint64_t ticket, int32_t *members, int32_t cap,
                           lcd_query_info *info);

/* Block until the ticket is done (LCD_OK) or timeout_ms passes (LCD_EAGAIN);
 * timeout_ms < 0 waits without limit.  Does not retire the ticket. */
lcd_status lcd_server_wait(lcd_server *s, uint64_t ticket, int32_t timeout_ms);

/*
 * Withdraw a query.  Not part of the paper's method: serving plumbing for
 * callers that no longer need an answer.  A query still waiting for a lane
 * is dropped at once; one already on the device finishes there and its
 * result is discarded.  Either way the ticket then ends with
 * LCD_ECANCELED (poll retires it).  Returns LCD_OK when the query was
 * withdrawn, LCD_ESTATE when it had already completed (its result stays
 * available), LCD_EINVAL for an unknown ticket.  Thread-safe.
 */
lcd_status lcd_server_cancel(lcd_server *s, uint64_t ticket);

lcd_status lcd_server_get_stats(lcd_server *s, lcd_server_stats *out);

/* Finish the batches on the device, fail queries still waiting
 * (LCD_ESTATE), free everything.  Outstanding tickets become invalid. */
lcd_status lcd_server_destroy(lcd_server *s);

/*
 * The library's integer logarithm L(x) evaluated on the device, for
 * x in [1, 2^53): x and out are device arrays of n entries.  Blocking.
 * Exposed so the decision arithmetic can be checked bit for bit.
 */
lcd_status lcd_log_device(const uint64_t *x, double *out, int64_t n, void *stream);

/* Device properties used for launch sizing: compute units and LDS per CU. */
lcd_status lcd_device_info(int32_t *compute_units, int64_t *lds_per_cu,
                           int64_t *lds_per_block, char *arch, int32_t arch_len);

const char *lcd_last_error(void);
const char *lcd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LCD_H */
