/*
 * CPU oracle for the multi-scale LFK community growth sweep.
 *
 * TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg build, load or call this file.
 * The HIP library shares nothing with it: no header, helper, table or
 * constant.
 *
 * Source: E. Le Martelot and C. Hankin, "Fast Multi-Scale Community
 * Detection based on Local Criteria within a Multi-Threaded Algorithm"
 * (arXiv:1301.0955).
 *
 *   f_c   = k_in / (k_in + k_out)^alpha               Sec. 2, Eq. (1)
 *   f_c^i = f_{c+i} - f_{c-i}; a node joins or leaves   Sec. 2, Eq. (2)
 *           c only if that raises f_c
 *   growth: max priority queue ranked by              Sec. 2, Algorithm 1
 *           2 d_in / (d_in + d_out)^alpha, then passes
 *           that drop members whose removal raises f_c
 *   chain:  the result at one scale is the start of    Sec. 2 (method); Sec. 3
 *           the next, scales ordered by coarseness      (Algorithm 2, growth half)
 *
 * Readings of points the paper leaves open (each is also stated where used):
 *   R1 k_in counts every internal edge from both ends (so adding node n
 *      raises it by 2 d_in(n)) and k_in + k_out is the community volume
 *      V = sum of member degrees.  All of K = k_in, V, d_in, degrees are
 *      exact integers (edge weights are positive integers).
 *   R2 whether adding n raises the fitness of the community is decided in
 *      the log domain:
 *        t = (L(K') - L(K)) - alpha * (L(V') - L(V)),  improve <=> t > 2^-40
 *      with K' = 0 never improving and K = 0 (< K') always improving.  L is
 *      lcdo_log below, a fully specified natural log of a positive integer,
 *      evaluated with IEEE double operations in a fixed order (no FMA).
 *   R3 rank R(d, k) = L(2d) - alpha * L(k); equal ranks pop the smaller id.
 *   R4 a popped node that does not improve Q_c is re-queued only when a
 *      later addition changes its d_in (the queue update of Algorithm 1).
 *   R5 removal passes visit the members present at the start of the pass in
 *      ascending id and apply each removal at once; at most k_prune passes
 *      (0 = until a pass removes nothing); no pass if nothing was added.
 *   R6 without the merge phase, the repetition of Algorithm 2 until nothing
 *      changes is the fixpoint of the growth function at each scale.
 *   R7 the reported criterion value is f = K / pow(V, alpha) (0 when K = 0).
 *
 * Work counters (the definition the GPU must reproduce):
 *   G  one per criterion evaluation: each queue pop and each member visited
 *      by a removal pass;
 *   R  one per rank (re)computation: each node put in the queue when it is
 *      built and each non-member neighbour of an added node;
 *   M  one per node added or removed;
 *   C  one per call of the growth function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* R2: L(x), natural log of an integer 1 <= x < 2^53.                        */
/* x = m * 2^e with m in (sqrt(2)/2, sqrt(2)]; ln m = 2 atanh(s),            */
/* s = (m - 1) / (m + 1), summed as 2 s (1 + z/3 + ... + z^11/23), z = s^2;   */
/* ln 2 is split in a high part with trailing zero bits and a low part       */
/* (Cody and Waite) so that e * ln2_hi is exact.                             */
/* ------------------------------------------------------------------------ */
#define LCDO_SQRT2 0x1.6a09e667f3bcdp+0
#define LCDO_LN2_HI 6.93147180369123816490e-01
#define LCDO_LN2_LO 1.90821492927058770002e-10

double lcdo_log(uint64_t x)
{
    int e = 63;
    while (!((x >> e) & 1u))
        --e;
    double m = (double)x;
    double scale = 1.0;
    for (int i = 0; i < e; ++i)
        scale *= 0.5;               /* exact: a power of two */
    m = m * scale;                  /* exact */
    if (m > LCDO_SQRT2) {
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
    return de * LCDO_LN2_HI + (de * LCDO_LN2_LO + lnm);
}

/* ------------------------------------------------------------------------ */
/* Tracing hook for the audits in the test suite.                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t K, V, Kp, Vp;
    double alpha, t;
    int32_t kind;      /* 0 = add test, 1 = removal test */
    int32_t result;    /* 1 = improves */
    int32_t node;      /* the node tested */
    int32_t pad;
    uint64_t mask;     /* member set after the decision, bit u (n <= 64) */
} lcdo_trace_rec;

typedef struct {
    lcdo_trace_rec *rec;
    int64_t cap;
    int64_t count;     /* may exceed cap: records past cap are dropped */
} lcdo_trace;

/* R2: "is f(K', V') > f(K, V)" at scale alpha. */
static int lcdo_improves(int64_t Kp, int64_t Vp, int64_t K, int64_t V,
                         double alpha, double *t_out)
{
    if (Kp == 0) {
        *t_out = NAN;
        return 0;
    }
    if (K == 0) {
        *t_out = INFINITY;
        return 1;
    }
    double a = lcdo_log((uint64_t)Kp) - lcdo_log((uint64_t)K);
    double b = lcdo_log((uint64_t)Vp) - lcdo_log((uint64_t)V);
    double c = alpha * b;
    double t = a - c;
    *t_out = t;
    return t > 0x1p-40;
}

double lcdo_rank(int64_t d, int64_t k, double alpha)
{
    double c = alpha * lcdo_log((uint64_t)k);
    return lcdo_log((uint64_t)(2 * d)) - c;
}

int lcdo_improves_export(int64_t Kp, int64_t Vp, int64_t K, int64_t V,
                         double alpha, double *t_out)
{
    return lcdo_improves(Kp, Vp, K, V, alpha, t_out);
}

/* ------------------------------------------------------------------------ */
/* Graph and per-community working state                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    double r;
    int32_t u;
    uint32_t ver;
} lcdo_qent;

typedef struct {
    int32_t n;
    const int32_t *row_ptr;
    const int32_t *col;
    const uint8_t *w;      /* NULL: all weights 1 */
    int64_t *k;            /* weighted degree of every node */
    /* state of the community being grown; every array indexed by node id */
    int64_t *d;            /* d_in: weight from the node into c */
    uint8_t *in_c;
    uint8_t *queued;
    uint32_t *ver;
    uint8_t *seen;
    int32_t *touched;      /* nodes whose entries above may be non-zero */
    int64_t n_touched;
    int32_t *members;      /* scratch for one removal pass */
    lcdo_qent *heap;
    int64_t heap_n, heap_cap;
    int64_t K, V;
    int32_t size;
    uint64_t G, R, M;
    lcdo_trace *trace;
} lcdo_ctx;

static int64_t lcdo_w(const lcdo_ctx *g, int64_t j)
{
    return g->w ? (int64_t)g->w[j] : 1;
}

lcdo_ctx *lcdo_ctx_new(int32_t n, const int32_t *row_ptr, const int32_t *col,
                       const uint8_t *w)
{
    lcdo_ctx *g = (lcdo_ctx *)calloc(1, sizeof(lcdo_ctx));
    if (!g)
        return NULL;
    g->n = n;
    g->row_ptr = row_ptr;
    g->col = col;
    g->w = w;
    size_t nn = (size_t)(n > 0 ? n : 1);
    g->k = (int64_t *)calloc(nn, sizeof(int64_t));
    g->d = (int64_t *)calloc(nn, sizeof(int64_t));
    g->in_c = (uint8_t *)calloc(nn, 1);
    g->queued = (uint8_t *)calloc(nn, 1);
    g->ver = (uint32_t *)calloc(nn, sizeof(uint32_t));
    g->seen = (uint8_t *)calloc(nn, 1);
    g->touched = (int32_t *)malloc(nn * sizeof(int32_t));
    g->members = (int32_t *)malloc(nn * sizeof(int32_t));
    g->heap_cap = 1024;
    g->heap = (lcdo_qent *)malloc((size_t)g->heap_cap * sizeof(lcdo_qent));
    if (!g->k || !g->d || !g->in_c || !g->queued || !g->ver || !g->seen ||
        !g->touched || !g->members || !g->heap)
        return NULL;
    for (int32_t u = 0; u < n; ++u) {
        int64_t s = 0;
        for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j)
            s += lcdo_w(g, j);
        g->k[u] = s;
    }
    return g;
}

void lcdo_ctx_free(lcdo_ctx *g)
{
    if (!g)
        return;
    free(g->k);
    free(g->d);
    free(g->in_c);
    free(g->queued);
    free(g->ver);
    free(g->seen);
    free(g->touched);
    free(g->members);
    free(g->heap);
    free(g);
}

const int64_t *lcdo_degrees(const lcdo_ctx *g) { return g->k; }

static void lcdo_touch(lcdo_ctx *g, int32_t u)
{
    if (!g->seen[u]) {
        g->seen[u] = 1;
        g->touched[g->n_touched++] = u;
    }
}

/* --- max priority queue: higher rank first, equal rank -> smaller id --- */
static int lcdo_before(const lcdo_qent *a, const lcdo_qent *b)
{
    return a->r > b->r || (a->r == b->r && a->u < b->u);
}

static void lcdo_push(lcdo_ctx *g, double r, int32_t u, uint32_t ver)
{
    if (g->heap_n == g->heap_cap) {
        g->heap_cap *= 2;
        g->heap = (lcdo_qent *)realloc(g->heap, (size_t)g->heap_cap * sizeof(lcdo_qent));
    }
    int64_t i = g->heap_n++;
    lcdo_qent e = {r, u, ver};
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!lcdo_before(&e, &g->heap[p]))
            break;
        g->heap[i] = g->heap[p];
        i = p;
    }
    g->heap[i] = e;
}

static lcdo_qent lcdo_pop(lcdo_ctx *g)
{
    lcdo_qent top = g->heap[0];
    lcdo_qent last = g->heap[--g->heap_n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, b = i;
        const lcdo_qent *best = &last;
        if (l < g->heap_n && lcdo_before(&g->heap[l], best)) {
            b = l;
            best = &g->heap[l];
        }
        if (r < g->heap_n && lcdo_before(&g->heap[r], best)) {
            b = r;
            best = &g->heap[r];
        }
        if (b == i)
            break;
        g->heap[i] = g->heap[b];
        i = b;
    }
    if (g->heap_n > 0)
        g->heap[i] = last;
    return top;
}

/* Put u in the queue, or move it to its new rank if it is there already. */
static void lcdo_queue(lcdo_ctx *g, int32_t u, double alpha)
{
    g->ver[u] += 1;
    g->queued[u] = 1;
    lcdo_push(g, lcdo_rank(g->d[u], g->k[u], alpha), u, g->ver[u]);
    g->R += 1;
}

static uint64_t lcdo_mask(const lcdo_ctx *g)
{
    uint64_t m = 0;
    if (g->n > 64)
        return 0;
    for (int32_t u = 0; u < g->n; ++u)
        if (g->in_c[u])
            m |= (uint64_t)1 << u;
    return m;
}

static int lcdo_decide(lcdo_ctx *g, int kind, int32_t node, int64_t Kp, int64_t Vp,
                       double alpha)
{
    double t;
    int r = lcdo_improves(Kp, Vp, g->K, g->V, alpha, &t);
    if (g->trace) {
        lcdo_trace *tr = g->trace;
        if (tr->count < tr->cap) {
            lcdo_trace_rec *x = &tr->rec[tr->count];
            x->K = g->K;
            x->V = g->V;
            x->Kp = Kp;
            x->Vp = Vp;
            x->alpha = alpha;
            x->t = t;
            x->kind = kind;
            x->result = r;
            x->node = node;
            x->pad = 0;
            x->mask = 0;
        }
        tr->count += 1;
    }
    return r;
}

static void lcdo_trace_mask(lcdo_ctx *g)
{
    if (g->trace && g->trace->count <= g->trace->cap && g->trace->count > 0)
        g->trace->rec[g->trace->count - 1].mask = lcdo_mask(g);
}

static void lcdo_add(lcdo_ctx *g, int32_t u, double alpha)
{
    g->in_c[u] = 1;
    g->K += 2 * g->d[u];
    g->V += g->k[u];
    g->size += 1;
    g->M += 1;
    for (int64_t j = g->row_ptr[u]; j < g->row_ptr[u + 1]; ++j) {
        int32_t v = g->col[j];
        g->d[v] += lcdo_w(g, j);
        lcdo_touch(g, v);
        if (!g->in_c[v])
            lcdo_queue(g, v, alpha);   /* R4: update or (re)insert */
    }
}

static void lcdo_remove(lcdo_ctx *g, int32_t u)
{
    g->in_c[u] = 0;
    g->K -= 2 * g->d[u];
    g->V -= g->k[u];
    g->size -= 1;
    g->M += 1;
    for (int64_t j = g->row_ptr[u]; j < g->row_ptr[u + 1]; ++j)
        g->d[g->col[j]] -= lcdo_w(g, j);
}

static int lcdo_cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Algorithm 1: one call of the growth function at scale alpha.
 * Returns the number of nodes added or removed. */
static int64_t lcdo_grow(lcdo_ctx *g, double alpha, uint32_t k_prune)
{
    int64_t moves = 0;
    int added = 0;
    g->heap_n = 0;
    /* build the queue from every non-member with a link into c */
    for (int64_t i = 0; i < g->n_touched; ++i) {
        int32_t u = g->touched[i];
        g->queued[u] = 0;
        if (!g->in_c[u] && g->d[u] > 0)
            lcdo_queue(g, u, alpha);
    }
    while (g->heap_n > 0) {
        lcdo_qent e = lcdo_pop(g);
        int32_t u = e.u;
        if (!g->queued[u] || e.ver != g->ver[u])
            continue;               /* superseded entry */
        g->queued[u] = 0;
        g->G += 1;
        if (lcdo_decide(g, 0, u, g->K + 2 * g->d[u], g->V + g->k[u], alpha)) {
            lcdo_add(g, u, alpha);
            lcdo_trace_mask(g);
            moves += 1;
            added = 1;
        }
    }
    if (added) {
        for (uint32_t pass = 0; k_prune == 0 || pass < k_prune; ++pass) {
            int32_t m = 0;
            for (int64_t i = 0; i < g->n_touched; ++i)
                if (g->in_c[g->touched[i]])
                    g->members[m++] = g->touched[i];
            qsort(g->members, (size_t)m, sizeof(int32_t), lcdo_cmp_i32);
            int removed = 0;
            for (int32_t i = 0; i < m; ++i) {
                int32_t u = g->members[i];
                g->G += 1;
                if (lcdo_decide(g, 1, u, g->K - 2 * g->d[u], g->V - g->k[u], alpha)) {
                    lcdo_remove(g, u);
                    lcdo_trace_mask(g);
                    moves += 1;
                    removed = 1;
                }
            }
            if (!removed)
                break;
        }
    }
    return moves;
}

static void lcdo_reset(lcdo_ctx *g)
{
    for (int64_t i = 0; i < g->n_touched; ++i) {
        int32_t u = g->touched[i];
        g->d[u] = 0;
        g->in_c[u] = 0;
        g->queued[u] = 0;
        g->seen[u] = 0;
    }
    g->n_touched = 0;
    g->heap_n = 0;
    g->K = g->V = 0;
    g->size = 0;
}

/*
 * Grow one initial community (one of the starting sets of Algorithm 2, or a
 * seed) through every scale in order.
 *
 * seeds[0..ns)      distinct node ids forming the initial community
 * scales[0..S)      alpha values, finest first (decreasing alpha)
 * k_prune           removal passes per growth call, 0 = unbounded (R5)
 * out_members       members of scale s, ascending, at
 *                   [out_off[s], out_off[s+1]); out_off has S+1 entries
 * members_cap       capacity of out_members; on overflow returns -1 and
 *                   out_off[S] still holds the size needed
 * out_K, out_V      K and V per scale; out_f the reported f (R7)
 * out_ctr           per scale: G, R, M, C (4 entries each)
 */
static int lcdo_run_set_calls(lcdo_ctx *g, const int32_t *seeds, int32_t ns,
                              const double *scales, int32_t S, uint32_t k_prune,
                              uint64_t max_calls, int32_t *out_members,
                              int64_t members_cap, int64_t *out_off, int64_t *out_K,
                              int64_t *out_V, double *out_f, uint64_t *out_ctr,
                              lcdo_trace *trace);

int lcdo_run_set(lcdo_ctx *g, const int32_t *seeds, int32_t ns,
                 const double *scales, int32_t S, uint32_t k_prune,
                 int32_t *out_members, int64_t members_cap, int64_t *out_off,
                 int64_t *out_K, int64_t *out_V, double *out_f,
                 uint64_t *out_ctr, lcdo_trace *trace)
{
    return lcdo_run_set_calls(g, seeds, ns, scales, S, k_prune, 0, out_members,
                              members_cap, out_off, out_K, out_V, out_f, out_ctr, trace);
}

/* The same with at most max_calls growth calls per scale (0 = until a call
 * changes nothing, R6); the check-and-merge loop makes one call per round. */
static int lcdo_run_set_calls(lcdo_ctx *g, const int32_t *seeds, int32_t ns,
                              const double *scales, int32_t S, uint32_t k_prune,
                              uint64_t max_calls, int32_t *out_members,
                              int64_t members_cap, int64_t *out_off, int64_t *out_K,
                              int64_t *out_V, double *out_f, uint64_t *out_ctr,
                              lcdo_trace *trace)
{
    lcdo_reset(g);
    g->trace = trace;
    /* initial community: add the seed nodes without any test */
    for (int32_t i = 0; i < ns; ++i) {
        int32_t u = seeds[i];
        lcdo_touch(g, u);
        g->in_c[u] = 1;
        g->K += 2 * g->d[u];
        g->V += g->k[u];
        g->size += 1;
        for (int64_t j = g->row_ptr[u]; j < g->row_ptr[u + 1]; ++j) {
            g->d[g->col[j]] += lcdo_w(g, j);
            lcdo_touch(g, g->col[j]);
        }
    }
    int64_t off = 0;
    int overflow = 0;
    for (int32_t s = 0; s < S; ++s) {
        double alpha = scales[s];
        g->G = g->R = g->M = 0;
        uint64_t calls = 0;
        for (;;) {                   /* R6: grow until nothing changes */
            calls += 1;
            if (lcdo_grow(g, alpha, k_prune) == 0)
                break;
            if (max_calls != 0 && calls >= max_calls)
                break;
        }
        out_ctr[4 * s + 0] = g->G;
        out_ctr[4 * s + 1] = g->R;
        out_ctr[4 * s + 2] = g->M;
        out_ctr[4 * s + 3] = calls;
        out_K[s] = g->K;
        out_V[s] = g->V;
        out_f[s] = g->K == 0 ? 0.0 : (double)g->K / pow((double)g->V, alpha);
        out_off[s] = off;
        int32_t m = 0;
        for (int64_t i = 0; i < g->n_touched; ++i)
            if (g->in_c[g->touched[i]])
                g->members[m++] = g->touched[i];
        qsort(g->members, (size_t)m, sizeof(int32_t), lcdo_cmp_i32);
        if (off + m <= members_cap)
            memcpy(out_members + off, g->members, (size_t)m * sizeof(int32_t));
        else
            overflow = 1;
        off += m;
    }
    out_off[S] = off;
    g->trace = NULL;
    return overflow ? -1 : 0;
}

/*
 * Many independent initial communities.  Set j is seed_nodes[seed_ptr[j] ..
 * seed_ptr[j+1]).  Records are indexed j * S + s; the members of record r
 * are out_members[out_off[r] .. out_off[r] + out_cnt[r]).  Returns 0, or -1
 * when members_cap was too small (*needed then holds the size required).
 */
int lcdo_run_sets(lcdo_ctx *g, const int32_t *seed_ptr, const int32_t *seed_nodes,
                  int32_t n_sets, const double *scales, int32_t S, uint32_t k_prune,
                  int32_t *out_members, int64_t members_cap, int64_t *needed,
                  int64_t *out_off, int32_t *out_cnt, int64_t *out_K, int64_t *out_V,
                  double *out_f, uint64_t *out_ctr)
{
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(S + 1));
    if (!off)
        return -2;
    int64_t base = 0;
    int status = 0;
    for (int32_t j = 0; j < n_sets; ++j) {
        int64_t room = members_cap - base;
        if (room < 0)
            room = 0;
        int rc = lcdo_run_set(g, seed_nodes + seed_ptr[j], seed_ptr[j + 1] - seed_ptr[j],
                              scales, S, k_prune,
                              out_members ? out_members + (room > 0 ? base : 0) : NULL,
                              out_members ? room : 0, off,
                              out_K + (int64_t)j * S, out_V + (int64_t)j * S,
                              out_f + (int64_t)j * S, out_ctr + (int64_t)j * S * 4, NULL);
        if (rc != 0)
            status = -1;
        for (int32_t s = 0; s < S; ++s) {
            out_off[(int64_t)j * S + s] = base + off[s];
            out_cnt[(int64_t)j * S + s] = (int32_t)(off[s + 1] - off[s]);
        }
        base += off[S];
    }
    *needed = base;
    free(off);
    return status;
}

/* L(x) over an array (for the accuracy pins and the device comparison). */
void lcdo_log_many(const uint64_t *x, double *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = lcdo_log(x[i]);
}

/* ------------------------------------------------------------------------ */
/* Seed selection (Sec. 3, initialisation part of Algorithm 2)              */
/* ------------------------------------------------------------------------ */
/*
 * Candidates are the nodes with at least two neighbours.  Nodes are visited
 * in the order perm[0 .. n) (the random choice of the paper, drawn by the
 * caller); a visited node that is still a candidate becomes the next seed and
 * leaves the candidate set together with its neighbours (rule 1), or with
 * every node at most two hops away (rule 2: neighbours of neighbours too).
 * Writes the seeds in order of selection to out (room for n ids) and returns
 * their number; -1 if rule is not 1 or 2 or perm is not a permutation.
 */
int64_t lcdo_seeds(const lcdo_ctx *g, const int32_t *perm, int rule, int32_t *out)
{
    const int32_t n = g->n;
    if (rule != 1 && rule != 2)
        return -1;
    uint8_t *cand = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!cand)
        return -1;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t v = perm[i];
        if (v < 0 || v >= n || cand[v] == 2) {
            free(cand);
            return -1;
        }
        cand[v] = 2; /* seen once */
    }
    for (int32_t u = 0; u < n; ++u)
        cand[u] = (g->row_ptr[u + 1] - g->row_ptr[u]) >= 2;
    int64_t ns = 0;
    for (int32_t i = 0; i < n; ++i) {
        const int32_t v = perm[i];
        if (!cand[v])
            continue;
        out[ns++] = v;
        cand[v] = 0;
        for (int64_t j = g->row_ptr[v]; j < g->row_ptr[v + 1]; ++j) {
            const int32_t u = g->col[j];
            cand[u] = 0;
            if (rule == 2)
                for (int64_t q = g->row_ptr[u]; q < g->row_ptr[u + 1]; ++q)
                    cand[g->col[q]] = 0;
        }
    }
    free(cand);
    return ns;
}

/* ------------------------------------------------------------------------ */
/* Check-and-merge phase (Sec. 3, Algorithm 2; overlap pre-test of          */
/* Algorithm 3)                                                              */
/* ------------------------------------------------------------------------ */
/*
 * Reading (each point also in the design notes):
 *   M1 the scale loop of Algorithm 2 runs rounds until a round neither grows
 *      a community nor merges two;
 *   M2 memberships M[v] = the live communities holding v, ascending ids,
 *      rebuilt at the start of a round and again after its growth;
 *   M3 overlap count of c with i: walk c's members ascending and, for each,
 *      M[v] ascending; c and i "reach the threshold" when the running count
 *      x satisfies x * eta_den >= eta_num * min(|c|, |i|) (eta = 1/2 by
 *      default: at least half of the smaller one); the first such i is c's
 *      partner;
 *   M4 pre-test (Algorithm 3): a live community with a partner under the
 *      round's first M is not grown in that round;
 *   M5 growth: every other community that needs it makes one call of the
 *      growth function at the scale, from its members (Algorithm 2 calls
 *      growth once per community and round, and repeats the round while
 *      anything changes); a live community needs a call at the start of a
 *      scale, after a call that changed it and after a merge it survived
 *      (a call on an unchanged community changes nothing again: the call
 *      is a function of the member set);
 *   M6 check: for each pre-tested or changed community, ascending, its
 *      partner under the post-growth M gives the pair (min, max);
 *   M7 merge: the pairs sorted ascending without repeats; repeatedly take,
 *      in order, the pairs that share no community, merge each into its
 *      lower id (union of members; the higher id dies and is renamed to the
 *      lower one in the remaining pairs), until no pair is left;
 *   M8 records: a live community reports its members, K, V, f at the scale
 *      and the counters summed over its growths at that scale; a dead one
 *      reports no members, K = V = 0, and the live id it was merged into.
 */
typedef struct {
    int32_t ns;
    int32_t **mem;
    int32_t *msz, *mcap;
    uint8_t *alive;
    int32_t *into;
    int64_t *node_ptr;   /* memberships, n + 1 */
    int32_t *node_list;
    int64_t list_cap;
    int32_t *cnt, *touched;
} lcdo_merge;

static int lcdo_mg_memberships(const lcdo_ctx *g, lcdo_merge *m)
{
    const int32_t n = g->n;
    memset(m->node_ptr, 0, sizeof(int64_t) * (size_t)(n + 1));
    for (int32_t j = 0; j < m->ns; ++j)
        if (m->alive[j])
            for (int32_t q = 0; q < m->msz[j]; ++q)
                m->node_ptr[m->mem[j][q] + 1] += 1;
    for (int32_t v = 0; v < n; ++v)
        m->node_ptr[v + 1] += m->node_ptr[v];
    const int64_t total = m->node_ptr[n];
    if (total > m->list_cap) {
        int32_t *p = (int32_t *)realloc(m->node_list, sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
        if (!p)
            return -1;
        m->node_list = p;
        m->list_cap = total;
    }
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!fill)
        return -1;
    memcpy(fill, m->node_ptr, sizeof(int64_t) * (size_t)n);
    for (int32_t j = 0; j < m->ns; ++j)       /* ascending ids per node */
        if (m->alive[j])
            for (int32_t q = 0; q < m->msz[j]; ++q)
                m->node_list[fill[m->mem[j][q]]++] = j;
    free(fill);
    return 0;
}

static int32_t lcdo_mg_partner(lcdo_merge *m, int32_t c, int32_t eta_num, int32_t eta_den)
{
    int32_t nt = 0, found = -1;
    for (int32_t q = 0; q < m->msz[c] && found < 0; ++q) {
        const int32_t v = m->mem[c][q];
        for (int64_t t = m->node_ptr[v]; t < m->node_ptr[v + 1]; ++t) {
            const int32_t i = m->node_list[t];
            if (i == c)
                continue;
            if (m->cnt[i]++ == 0)
                m->touched[nt++] = i;
            const int64_t small = m->msz[c] < m->msz[i] ? m->msz[c] : m->msz[i];
            if ((int64_t)m->cnt[i] * eta_den >= (int64_t)eta_num * small) {
                found = i;
                break;
            }
        }
    }
    for (int32_t t = 0; t < nt; ++t)
        m->cnt[m->touched[t]] = 0;
    return found;
}

static int lcdo_cmp_pair(const void *a, const void *b)
{
    const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
    if (x[0] != y[0])
        return (x[0] > y[0]) - (x[0] < y[0]);
    return (x[1] > y[1]) - (x[1] < y[1]);
}

/* union of two ascending lists into a (reallocated) */
static int lcdo_mg_union(lcdo_merge *m, int32_t a, int32_t b)
{
    const int32_t na = m->msz[a], nb = m->msz[b];
    int32_t *u = (int32_t *)malloc(sizeof(int32_t) * (size_t)(na + nb + 1));
    if (!u)
        return -1;
    int32_t i = 0, j = 0, k = 0;
    while (i < na || j < nb) {
        if (j >= nb || (i < na && m->mem[a][i] < m->mem[b][j]))
            u[k++] = m->mem[a][i++];
        else if (i >= na || m->mem[b][j] < m->mem[a][i])
            u[k++] = m->mem[b][j++];
        else {
            u[k++] = m->mem[a][i++];
            ++j;
        }
    }
    free(m->mem[a]);
    m->mem[a] = u;
    m->msz[a] = k;
    m->mcap[a] = na + nb + 1;
    return 0;
}

/*
 * Seed sets j = seed_nodes[seed_ptr[j] .. seed_ptr[j+1]), scales as in
 * lcdo_run_sets.  Record r = j * S + s: members at out_members[out_off[r] ..
 * out_off[r] + out_cnt[r]), out_K, out_V, out_f, out_ctr (4 per record),
 * out_into (-1 for a live community, else the live id it merged into).
 * out_rounds[s]: rounds the scale took.  Returns 0, -1 when members_cap is
 * too small (*needed set), -2 on allocation failure, -3 when a scale does
 * not settle within max_rounds rounds.
 */
int lcdo_run_merge(lcdo_ctx *g, const int32_t *seed_ptr, const int32_t *seed_nodes, int32_t ns,
                   const double *scales, int32_t S, uint32_t k_prune, int32_t eta_num,
                   int32_t eta_den, int32_t max_rounds, int32_t *out_members, int64_t members_cap,
                   int64_t *needed, int64_t *out_off, int32_t *out_cnt, int64_t *out_K,
                   int64_t *out_V, double *out_f, uint64_t *out_ctr, int32_t *out_into,
                   int32_t *out_rounds)
{
    const int32_t n = g->n;
    lcdo_merge m;
    memset(&m, 0, sizeof(m));
    m.ns = ns;
    size_t nn = (size_t)(ns > 0 ? ns : 1);
    m.mem = (int32_t **)calloc(nn, sizeof(int32_t *));
    m.msz = (int32_t *)calloc(nn, sizeof(int32_t));
    m.mcap = (int32_t *)calloc(nn, sizeof(int32_t));
    m.alive = (uint8_t *)calloc(nn, 1);
    m.into = (int32_t *)calloc(nn, sizeof(int32_t));
    m.node_ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    m.cnt = (int32_t *)calloc(nn, sizeof(int32_t));
    m.touched = (int32_t *)calloc(nn, sizeof(int32_t));
    int64_t *K = (int64_t *)calloc(nn, sizeof(int64_t));
    int64_t *V = (int64_t *)calloc(nn, sizeof(int64_t));
    uint64_t *acc = (uint64_t *)calloc(nn * 4, sizeof(uint64_t));
    uint8_t *need = (uint8_t *)calloc(nn, 1), *flag = (uint8_t *)calloc(nn, 1), *changed = (uint8_t *)calloc(nn, 1);
    int32_t *pairs = (int32_t *)malloc(sizeof(int32_t) * 2 * nn);
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t *used = (int32_t *)calloc(nn, sizeof(int32_t));
    int32_t *ren = (int32_t *)malloc(sizeof(int32_t) * 2 * nn);   /* dead id -> survivor, one pass */
    int status = 0;
    if (!m.mem || !m.msz || !m.mcap || !m.alive || !m.into || !m.node_ptr || !m.cnt || !m.touched || !K ||
        !V || !acc || !need || !flag || !changed || !pairs || !tmp || !used || !ren) {
        status = -2;
        goto done;
    }
    for (int32_t j = 0; j < ns; ++j) {
        const int32_t c = seed_ptr[j + 1] - seed_ptr[j];
        m.mem[j] = (int32_t *)malloc(sizeof(int32_t) * (size_t)(c > 0 ? c : 1));
        if (!m.mem[j]) {
            status = -2;
            goto done;
        }
        memcpy(m.mem[j], seed_nodes + seed_ptr[j], sizeof(int32_t) * (size_t)c);
        qsort(m.mem[j], (size_t)c, sizeof(int32_t), lcdo_cmp_i32);
        m.msz[j] = c;
        m.mcap[j] = c;
        m.alive[j] = 1;
        m.into[j] = -1;
    }
    int64_t base = 0;
    for (int32_t s = 0; s < S; ++s) {
        const double alpha = scales[s];
        memset(acc, 0, sizeof(uint64_t) * 4 * nn);
        for (int32_t j = 0; j < ns; ++j)
            need[j] = m.alive[j];
        int32_t rounds = 0;
        for (;;) {
            if (++rounds > max_rounds) {
                status = -3;
                goto done;
            }
            if (lcdo_mg_memberships(g, &m) != 0) {
                status = -2;
                goto done;
            }
            for (int32_t j = 0; j < ns; ++j)
                flag[j] = m.alive[j] && lcdo_mg_partner(&m, j, eta_num, eta_den) >= 0;
            int grew = 0;
            for (int32_t j = 0; j < ns; ++j) {
                changed[j] = 0;
                if (!m.alive[j] || !need[j] || flag[j])
                    continue;
                int64_t off2[2];
                int64_t k1, v1;
                double f1;
                uint64_t c4[4];
                if (lcdo_run_set_calls(g, m.mem[j], m.msz[j], &alpha, 1, k_prune, 1, tmp, n, off2, &k1,
                                       &v1, &f1, c4, NULL) != 0) {
                    status = -2;
                    goto done;
                }
                const int32_t sz = (int32_t)(off2[1] - off2[0]);
                changed[j] = sz != m.msz[j] || memcmp(tmp, m.mem[j], sizeof(int32_t) * (size_t)sz) != 0;
                if (sz > m.mcap[j]) {
                    int32_t *p = (int32_t *)realloc(m.mem[j], sizeof(int32_t) * (size_t)sz);
                    if (!p) {
                        status = -2;
                        goto done;
                    }
                    m.mem[j] = p;
                    m.mcap[j] = sz;
                }
                memcpy(m.mem[j], tmp, sizeof(int32_t) * (size_t)sz);
                m.msz[j] = sz;
                K[j] = k1;
                V[j] = v1;
                for (int q = 0; q < 4; ++q)
                    acc[4 * j + q] += c4[q];
                need[j] = changed[j];
                grew |= changed[j];
            }
            if (lcdo_mg_memberships(g, &m) != 0) {
                status = -2;
                goto done;
            }
            int32_t np = 0;
            for (int32_t j = 0; j < ns; ++j) {
                if (!m.alive[j] || !(flag[j] || changed[j]))
                    continue;
                const int32_t i = lcdo_mg_partner(&m, j, eta_num, eta_den);
                if (i >= 0) {
                    pairs[2 * np] = i < j ? i : j;
                    pairs[2 * np + 1] = i < j ? j : i;
                    ++np;
                }
            }
            const int merged = np > 0;
            while (np > 0) {
                qsort(pairs, (size_t)np, 2 * sizeof(int32_t), lcdo_cmp_pair);
                int32_t w = 0;       /* drop repeats */
                for (int32_t p = 0; p < np; ++p)
                    if (w == 0 || pairs[2 * p] != pairs[2 * (w - 1)] || pairs[2 * p + 1] != pairs[2 * (w - 1) + 1]) {
                        pairs[2 * w] = pairs[2 * p];
                        pairs[2 * w + 1] = pairs[2 * p + 1];
                        ++w;
                    }
                np = w;
                /* take, in order, the pairs sharing no community */
                for (int32_t p = 0; p < np; ++p)
                    used[pairs[2 * p]] = used[pairs[2 * p + 1]] = 0;
                int32_t rest = 0;
                int32_t nren = 0;
                for (int32_t p = 0; p < np; ++p) {
                    const int32_t a = pairs[2 * p], b = pairs[2 * p + 1];
                    if (!used[a] && !used[b]) {
                        used[a] = used[b] = 1;
                        if (lcdo_mg_union(&m, a, b) != 0) {
                            status = -2;
                            goto done;
                        }
                        m.alive[b] = 0;
                        m.into[b] = a;
                        need[a] = 1;
                        ren[2 * nren] = b;
                        ren[2 * nren + 1] = a;
                        ++nren;
                    } else {
                        pairs[2 * rest] = a;
                        pairs[2 * rest + 1] = b;
                        ++rest;
                    }
                }
                /* rename the dead ids in the remaining pairs */
                np = 0;
                for (int32_t p = 0; p < rest; ++p) {
                    int32_t a = pairs[2 * p], b = pairs[2 * p + 1];
                    for (int32_t r = 0; r < nren; ++r) {
                        if (a == ren[2 * r])
                            a = ren[2 * r + 1];
                        if (b == ren[2 * r])
                            b = ren[2 * r + 1];
                    }
                    if (a == b)
                        continue;
                    pairs[2 * np] = a < b ? a : b;
                    pairs[2 * np + 1] = a < b ? b : a;
                    ++np;
                }
            }
            if (!grew && !merged)
                break;
        }
        out_rounds[s] = rounds;
        for (int32_t j = 0; j < ns; ++j) {
            const int64_t r = (int64_t)j * S + s;
            int32_t to = j;
            while (!m.alive[to])
                to = m.into[to];
            out_into[r] = m.alive[j] ? -1 : to;
            out_off[r] = base;
            for (int q = 0; q < 4; ++q)
                out_ctr[4 * r + q] = acc[4 * j + q];
            if (m.alive[j]) {
                out_cnt[r] = m.msz[j];
                out_K[r] = K[j];
                out_V[r] = V[j];
                out_f[r] = K[j] == 0 ? 0.0 : (double)K[j] / pow((double)V[j], alpha);
                if (base + m.msz[j] <= members_cap)
                    memcpy(out_members + base, m.mem[j], sizeof(int32_t) * (size_t)m.msz[j]);
                else
                    status = -1;
                base += m.msz[j];
            } else {
                out_cnt[r] = 0;
                out_K[r] = 0;
                out_V[r] = 0;
                out_f[r] = 0.0;
            }
        }
    }
    *needed = base;
done:
    if (m.mem)
        for (int32_t j = 0; j < ns; ++j)
            free(m.mem[j]);
    free(m.mem);
    free(m.msz);
    free(m.mcap);
    free(m.alive);
    free(m.into);
    free(m.node_ptr);
    free(m.node_list);
    free(m.cnt);
    free(m.touched);
    free(K);
    free(V);
    free(acc);
    free(need);
    free(flag);
    free(changed);
    free(pairs);
    free(tmp);
    free(used);
    free(ren);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Normalised mutual information of two covers (Sec. 4)                      */
/* ------------------------------------------------------------------------ */
/*
 * Sec. 4 compares community sets of successive scales, and with the planted
 * ones, by the normalised mutual information for overlapping communities of
 * Lancichinetti, Fortunato and Kertesz (2009), which the paper cites without
 * printing.  Restated from that definition: every community X_k of a cover
 * X of n nodes is a binary variable (a node is in X_k or not); for X_k and
 * Y_l the joint distribution comes from the counts a = |X_k & Y_l|,
 * b = |X_k| - a, c = |Y_l| - a, e = n - a - b - c; the conditional entropy
 * H(X_k | Y_l) = H(X_k, Y_l) - H(Y_l) is admitted only when
 * h(a) + h(e) > h(b) + h(c); H(X_k | Y) is the least admitted one, or
 * H(X_k) when none is; H(X|Y)_norm is the mean over k of H(X_k|Y) / H(X_k),
 * and NMI = 1 - (H(X|Y)_norm + H(Y|X)_norm) / 2.
 * Readings (also in the design notes):
 *   N1 entropies in nats: h(c) = (c / n) * (L(n) - L(c)) for a count c of n
 *      nodes, h(0) = 0, with L the integer log of R2 (the log base cancels
 *      in every ratio; a specified log makes the admission test decide the
 *      same way in every implementation); the operations are rounded in
 *      the order written below;
 *   N2 a cover is taken as listed: every community counts, a repeated one
 *      each time it is listed;
 *   N3 an empty community is no community: it is skipped on both sides (it
 *      adds no term and does not count in the mean); a community of every
 *      node (H(X_k) = 0) adds 0 to its mean;
 *   N4 a cover without a non-empty community: the NMI is 1 if both are so,
 *      else 0.
 */
static double lcdo_h(int64_t c, int64_t n)
{
    if (c <= 0)
        return 0.0;
    double t = lcdo_log((uint64_t)n) - lcdo_log((uint64_t)c);
    double p = (double)c / (double)n;
    return p * t;
}

/* H(X|Y)_norm for covers given as CSR (community j = mem[ptr[j] .. ptr[j+1]),
 * distinct node ids in [0, n)); -1 on allocation failure. */
static double lcdo_nmi_half(int32_t n, int32_t kx, const int64_t *px, const int32_t *mx, int32_t ky,
                            const int64_t *py, const int32_t *my)
{
    int64_t *node_ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *cnt = (int32_t *)calloc((size_t)(ky > 0 ? ky : 1), sizeof(int32_t));
    int64_t total = py[ky];
    int32_t *node_sets = (int32_t *)malloc(sizeof(int32_t) * (size_t)(total > 0 ? total : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!node_ptr || !cnt || !node_sets || !fill) {
        free(node_ptr);
        free(cnt);
        free(node_sets);
        free(fill);
        return -1.0;
    }
    for (int32_t l = 0; l < ky; ++l)
        for (int64_t q = py[l]; q < py[l + 1]; ++q)
            node_ptr[my[q] + 1] += 1;
    for (int32_t v = 0; v < n; ++v)
        node_ptr[v + 1] += node_ptr[v];
    memcpy(fill, node_ptr, sizeof(int64_t) * (size_t)n);
    for (int32_t l = 0; l < ky; ++l)
        for (int64_t q = py[l]; q < py[l + 1]; ++q)
            node_sets[fill[my[q]]++] = l;
    double sum = 0.0;
    int32_t counted = 0;
    for (int32_t k = 0; k < kx; ++k) {
        const int64_t sx = px[k + 1] - px[k];
        if (sx == 0)
            continue;
        counted += 1;
        for (int64_t q = px[k]; q < px[k + 1]; ++q) {
            const int32_t v = mx[q];
            for (int64_t t = node_ptr[v]; t < node_ptr[v + 1]; ++t)
                cnt[node_sets[t]] += 1;
        }
        const double hx = lcdo_h(sx, n) + lcdo_h(n - sx, n);
        double best = hx;
        int found = 0;
        for (int32_t l = 0; l < ky; ++l) {
            const int64_t sy = py[l + 1] - py[l];
            if (sy == 0)
                continue;
            const int64_t a = cnt[l];
            const int64_t b = sx - a, c = sy - a, e = n - a - b - c;
            const double ha = lcdo_h(a, n), hb = lcdo_h(b, n), hc = lcdo_h(c, n), he = lcdo_h(e, n);
            cnt[l] = 0;
            if (!(ha + he > hb + hc))
                continue;
            const double hxy = ((ha + hb) + hc) + he;
            const double hy = lcdo_h(sy, n) + lcdo_h(n - sy, n);
            const double cond = hxy - hy;
            if (!found || cond < best) {
                best = cond;
                found = 1;
            }
        }
        if (hx > 0.0)
            sum += best / hx;
    }
    free(node_ptr);
    free(cnt);
    free(node_sets);
    free(fill);
    return counted > 0 ? sum / (double)counted : 0.0;
}

static int32_t lcdo_nonempty(int32_t k, const int64_t *p)
{
    int32_t c = 0;
    for (int32_t j = 0; j < k; ++j)
        c += p[j + 1] > p[j];
    return c;
}

/* NMI of covers X and Y of n nodes (N1-N4 above); returns -2 on allocation
 * failure. */
double lcdo_nmi(int32_t n, int32_t kx, const int64_t *px, const int32_t *mx, int32_t ky, const int64_t *py,
                const int32_t *my)
{
    const int32_t ex = lcdo_nonempty(kx, px), ey = lcdo_nonempty(ky, py);
    if (ex == 0 || ey == 0)
        return (ex == 0 && ey == 0) ? 1.0 : 0.0;
    const double hxy = lcdo_nmi_half(n, kx, px, mx, ky, py, my);
    const double hyx = lcdo_nmi_half(n, ky, py, my, kx, px, mx);
    if (hxy < 0.0 || hyx < 0.0)
        return -2.0;
    return 1.0 - (hxy + hyx) / 2.0;
}
