/*
 * Fast parts of the seeded input generator (workloads.py): stub matching
 * inside buckets with rejection of self-loops and repeated pairs, symmetric
 * CSR assembly with per-edge weights, and the rule-1 seed scan.  Used for
 * graphs too large for the numpy generator (10^7 nodes, 10^8 edges).
 *
 * This file makes inputs only.  It holds none of the method's arithmetic
 * (no fitness, rank or growth) and is shared by nothing but the input
 * module.  Randomness: splitmix64 (Steele, Lea and Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014) on a counter, one stream per
 * purpose, so a (parameters, seed) pair always yields the same graph.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

typedef struct {
    uint64_t s;
} rng_t;

static uint64_t rng_next(rng_t *r)
{
    r->s += 0x9e3779b97f4a7c15ull;
    return mix64(r->s);
}

/* uniform integer in [0, m), m >= 1 (Lemire's multiply-shift with rejection) */
static uint64_t rng_below(rng_t *r, uint64_t m)
{
    for (;;) {
        const uint64_t x = rng_next(r);
        const unsigned __int128 p = (unsigned __int128)x * m;
        const uint64_t lo = (uint64_t)p;
        if (lo >= m || lo >= (0ull - m) % m)
            return (uint64_t)(p >> 64);
    }
}

/* --- open-addressing set of undirected pairs (key = lo * n + hi) --- */
typedef struct {
    uint64_t *slot;
    uint64_t mask;
} pairset;

static int pairset_init(pairset *h, int64_t expect)
{
    uint64_t cap = 1024;
    while (cap < (uint64_t)expect * 2)
        cap <<= 1;
    h->slot = (uint64_t *)malloc(cap * sizeof(uint64_t));
    if (!h->slot)
        return -1;
    memset(h->slot, 0xff, cap * sizeof(uint64_t));
    h->mask = cap - 1;
    return 0;
}

/* 1 if inserted, 0 if present */
static int pairset_insert(pairset *h, uint64_t key)
{
    uint64_t p = mix64(key) & h->mask;
    for (;;) {
        const uint64_t v = h->slot[p];
        if (v == ~0ull) {
            h->slot[p] = key;
            return 1;
        }
        if (v == key)
            return 0;
        p = (p + 1) & h->mask;
    }
}

/*
 * Match stubs level by level.  stubs[l * n + u] stubs of node u at level l
 * pair inside bucket[l * n + u] (bucket ids in [0, n)).  Each round shuffles
 * every bucket's remaining stubs (Fisher-Yates) and pairs them in order; a
 * pair that is a self-loop or repeats an accepted pair is undone and its two
 * stubs are matched again in the next round, up to `rounds` rounds or until
 * fewer than 0.2 % of the level's stubs are left.  Accepted pairs go to
 * (out_u[i], out_v[i]), i < returned count (at most cap); -1 on allocation
 * failure, -2 when cap is too small.
 */
int64_t lfrgen_match(int64_t n, int32_t n_levels, const int64_t *stubs, const int64_t *bucket,
                     int32_t rounds, uint64_t seed, int32_t *out_u, int32_t *out_v, int64_t cap)
{
    int64_t total = 0;
    for (int64_t i = 0; i < n * n_levels; ++i)
        total += stubs[i];
    pairset h;
    if (pairset_init(&h, total / 2 + 16) != 0)
        return -1;
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int32_t *pool = NULL;
    int64_t m = 0;
    if (!start || !fill) {
        m = -1;
        goto done;
    }
    for (int32_t l = 0; l < n_levels && m >= 0; ++l) {
        const int64_t *s = stubs + (int64_t)l * n;
        const int64_t *b = bucket + (int64_t)l * n;
        int64_t lv = 0;
        memset(start, 0, sizeof(int64_t) * (size_t)(n + 1));
        for (int64_t u = 0; u < n; ++u) {
            start[b[u] + 1] += s[u];
            lv += s[u];
        }
        for (int64_t k = 0; k < n; ++k)
            start[k + 1] += start[k];
        free(pool);
        pool = (int32_t *)malloc(sizeof(int32_t) * (size_t)(lv > 0 ? lv : 1));
        if (!pool) {
            m = -1;
            break;
        }
        memcpy(fill, start, sizeof(int64_t) * (size_t)(n + 1));
        for (int64_t u = 0; u < n; ++u)
            for (int64_t q = 0; q < s[u]; ++q)
                pool[fill[b[u]]++] = (int32_t)u;
        /* fill[k] = end of bucket k's remaining stubs */
        rng_t r = {mix64(seed * 0x100000001b3ull + (uint64_t)l)};
        int64_t left = lv;
        for (int32_t round = 0; round < rounds && left >= 2; ++round) {
            left = 0;
            for (int64_t k = 0; k < n; ++k) {
                int32_t *a = pool + start[k];
                const int64_t len = fill[k] - start[k];
                if (len < 2) {
                    left += len;
                    continue;
                }
                for (int64_t i = len - 1; i > 0; --i) {
                    const int64_t j = (int64_t)rng_below(&r, (uint64_t)(i + 1));
                    const int32_t t = a[i];
                    a[i] = a[j];
                    a[j] = t;
                }
                int64_t keep = 0;
                int64_t i = 0;
                for (; i + 1 < len; i += 2) {
                    const int64_t x = a[i], y = a[i + 1];
                    const int64_t lo = x < y ? x : y, hi = x < y ? y : x;
                    if (x != y && pairset_insert(&h, (uint64_t)(lo * n + hi))) {
                        if (m >= cap) {
                            m = -2;
                            goto done;
                        }
                        out_u[m] = (int32_t)lo;
                        out_v[m] = (int32_t)hi;
                        ++m;
                    } else {
                        a[keep++] = (int32_t)x;
                        a[keep++] = (int32_t)y;
                    }
                }
                if (i < len)
                    a[keep++] = a[i];
                fill[k] = start[k] + keep;
                left += keep;
            }
            if (left * 500 < lv + 1000)
                break;
        }
    }
done:
    free(h.slot);
    free(start);
    free(fill);
    free(pool);
    return m;
}

/*
 * Symmetric CSR from m undirected pairs (lo < hi, no repeats): rows sorted
 * ascending.  With wmax > 0 every pair gets a weight uniform in [1, wmax]
 * from its own stream (the i-th pair's weight depends on seed and i only),
 * stored on both directions; w may be NULL when wmax is 0.  row_ptr has
 * n + 1 entries, col and w 2 m.  Returns 0, or -1 on allocation failure.
 */
int lfrgen_csr(int64_t n, int64_t m, const int32_t *u, const int32_t *v, int32_t wmax, uint64_t seed,
               int32_t *row_ptr, int32_t *col, uint8_t *w)
{
    const int64_t nnz = 2 * m;
    int64_t *cnt = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int32_t *src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    int32_t *dst = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    uint8_t *ww = (uint8_t *)malloc((size_t)(nnz > 0 ? nnz : 1));
    if (!cnt || !src || !dst || !ww) {
        free(cnt);
        free(src);
        free(dst);
        free(ww);
        return -1;
    }
    /* pass 1: counting sort of the directed entries by destination */
    for (int64_t i = 0; i < m; ++i) {
        cnt[v[i] + 1] += 1;
        cnt[u[i] + 1] += 1;
    }
    for (int64_t k = 0; k < n; ++k)
        cnt[k + 1] += cnt[k];
    for (int64_t i = 0; i < m; ++i) {
        uint8_t wt = 1;
        if (wmax > 0)
            wt = (uint8_t)(1 + mix64(seed ^ mix64((uint64_t)i + 0x632be59bd9b4e019ull)) % (uint64_t)wmax);
        int64_t p = cnt[v[i]]++;
        src[p] = u[i];
        dst[p] = v[i];
        ww[p] = wt;
        p = cnt[u[i]]++;
        src[p] = v[i];
        dst[p] = u[i];
        ww[p] = wt;
    }
    /* pass 2: stable counting sort by source, so each row is ascending */
    memset(cnt, 0, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t i = 0; i < nnz; ++i)
        cnt[src[i] + 1] += 1;
    for (int64_t k = 0; k < n; ++k)
        cnt[k + 1] += cnt[k];
    for (int64_t k = 0; k <= n; ++k)
        row_ptr[k] = (int32_t)cnt[k];
    for (int64_t i = 0; i < nnz; ++i) {
        const int64_t p = cnt[src[i]]++;
        col[p] = dst[i];
        if (w)
            w[p] = ww[i];
    }
    free(cnt);
    free(src);
    free(dst);
    free(ww);
    return 0;
}

/*
 * Seed rule 1 of the input module: nodes with at least two neighbours are
 * candidates; visiting perm in order, a node still a candidate becomes the
 * next seed and it and its neighbours leave the candidates.  Writes the
 * seeds in order to out (room for n) and returns their number.
 */
int64_t lfrgen_seed_rule1(int64_t n, const int32_t *row_ptr, const int32_t *col, const int32_t *perm,
                          int32_t *out)
{
    uint8_t *cand = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    if (!cand)
        return -1;
    for (int64_t x = 0; x < n; ++x)
        cand[x] = (row_ptr[x + 1] - row_ptr[x]) >= 2;
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int32_t x = perm[i];
        if (!cand[x])
            continue;
        out[k++] = x;
        cand[x] = 0;
        for (int64_t j = row_ptr[x]; j < row_ptr[x + 1]; ++j)
            cand[col[j]] = 0;
    }
    free(cand);
    return k;
}

/*
 * Place nodes in communities so that each community can hold its members'
 * internal stubs: node u needs a community of at least need[u] nodes.
 * Nodes are taken in the order `order` (by need, largest first); each goes
 * to a community drawn uniformly among those of size >= need[u] that still
 * have room (communities 0.. are sorted by size, largest first, so the
 * eligible ones are a growing prefix); when none has room it goes to any
 * community with room.  out_comm[u] receives the community index.  Returns
 * 0, or -1 on allocation failure or when the sizes cannot hold n nodes.
 */
int lfrgen_assign(int64_t n, const int64_t *need, const int64_t *order, int64_t n_comms,
                  const int64_t *size, uint64_t seed, int64_t *out_comm)
{
    int64_t *room = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_comms > 0 ? n_comms : 1));
    int64_t *avail = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_comms > 0 ? n_comms : 1));
    int64_t *where = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_comms > 0 ? n_comms : 1));
    if (!room || !avail || !where) {
        free(room);
        free(avail);
        free(where);
        return -1;
    }
    int64_t cap = 0;
    for (int64_t c = 0; c < n_comms; ++c) {
        room[c] = size[c];
        cap += size[c];
        where[c] = -1;
    }
    if (cap < n) {
        free(room);
        free(avail);
        free(where);
        return -1;
    }
    rng_t r = {mix64(seed ^ 0x5851f42d4c957f2dull)};
    int64_t n_avail = 0, next = 0, any = 0;
    for (int64_t q = 0; q < n; ++q) {
        const int64_t u = order[q];
        while (next < n_comms && size[next] >= need[u]) {
            if (room[next] > 0) {
                where[next] = n_avail;
                avail[n_avail++] = next;
            }
            ++next;
        }
        int64_t c;
        if (n_avail > 0) {
            c = avail[rng_below(&r, (uint64_t)n_avail)];
        } else {
            while (room[any] == 0)
                ++any;
            c = any;
        }
        out_comm[u] = c;
        room[c] -= 1;
        if (room[c] == 0 && where[c] >= 0) {
            const int64_t p = where[c];
            const int64_t last = avail[--n_avail];
            avail[p] = last;
            where[last] = p;
            where[c] = -1;
        }
    }
    free(room);
    free(avail);
    free(where);
    return 0;
}
