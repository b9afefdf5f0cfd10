/*
 * CPU oracle for exact (p,q)-biclique counting.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the
 * device library.
 *
 * What it computes (Definition 1 and the problem statement of Section II-A):
 *
 *     count(G, p, q) = #{ (L, R) : L in U, |L| = p, R in V, |R| = q, L x R in E }
 *                    = sum over p-subsets L of U of  C(|intersection of N(x), x in L|, q)
 *
 * The second line is the leaf rule of the Basic model (Section III-A): once p
 * vertices are in L, any q of the common neighbours C_R complete a biclique.
 *
 * How: every p-subset L is visited exactly once, as the increasing sequence
 * of its members under a strict total order ("rank") of U, starting from its
 * lowest-ranked member, the root.  This is the orientation by vertex priority
 * of Section III-B (Definition 2); any strict total order gives the same
 * total.  Along the sequence the common-neighbour set S = C_R is narrowed by
 * a sorted linear merge (the CPU intersection named in Section III-A), and
 * each complete L adds C(|S|, q).
 *
 * With pruning on, three kinds of branch are skipped, each of which can only
 * hold subsets whose contribution is zero:
 *   - candidates w sharing fewer than q neighbours with the root (the root's
 *     2-hop set N_2^q, Section II-A and Algorithm 1): S would end below q;
 *   - a child whose S has fewer than q vertices (first pruning condition of
 *     Section IV; S only shrinks further down);
 *   - a node with fewer remaining candidates than vertices still to add
 *     (no p-subset can be completed there; the root filter of Section III-B
 *     is the case of the root).
 * With pruning off, every higher-ranked vertex is a candidate and every
 * (p-1)-subset of them is visited, which is the definition written out.
 *
 * Counts are exact unsigned 128-bit integers; every addition is checked and
 * an overflow is reported as an error, never wrapped.
 *
 * Per-vertex counts (oracle_count_per_vertex) reduce the output set of
 * Algorithm 1 to membership counts: how many bicliques hold each x in U (in
 * L) and each v in V (in R).  They come from the same leaf rule, visiting
 * every p-subset L once by increasing ids: L's C(n, q) bicliques all hold
 * each member of L, and C(n-1, q-1) of them hold a given common neighbour.
 */
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

enum {
    OR_OK = 0,
    OR_E_ARG = -1,
    OR_E_CSR = -2,
    OR_E_OVERFLOW = -3,
    OR_E_OOM = -4,
    OR_E_BUDGET = -5,   /* a root needed more intersections than allowed */
};

/* ------------------------------------------------------------------ */
/* Checked 128-bit arithmetic and the binomial table (Pascal's rule).  */

static int add_u128(u128 *acc, u128 x)
{
    u128 s = *acc + x;
    if (s < *acc) return OR_E_OVERFLOW;
    *acc = s;
    return OR_OK;
}

typedef struct {
    uint32_t n_max, k_max;
    u128 *val;        /* (n_max+1) x (k_max+1), row-major by n */
    uint8_t *over;    /* 1 where the true value exceeds 2^128 - 1 */
} binom_table;

static int binom_init(binom_table *t, uint32_t n_max, uint32_t k_max)
{
    size_t cells = (size_t)(n_max + 1) * (k_max + 1);
    t->n_max = n_max;
    t->k_max = k_max;
    t->val = (u128 *)calloc(cells, sizeof(u128));
    t->over = (uint8_t *)calloc(cells, 1);
    if (!t->val || !t->over) return OR_E_OOM;
    for (uint32_t n = 0; n <= n_max; ++n) {
        for (uint32_t k = 0; k <= k_max; ++k) {
            size_t c = (size_t)n * (k_max + 1) + k;
            if (k == 0) { t->val[c] = 1; continue; }
            if (n == 0) { t->val[c] = 0; continue; }
            size_t a = (size_t)(n - 1) * (k_max + 1) + (k - 1);   /* C(n-1, k-1) */
            size_t b = (size_t)(n - 1) * (k_max + 1) + k;         /* C(n-1, k)   */
            u128 s = t->val[a];
            int ov = t->over[a] | t->over[b];
            if (add_u128(&s, t->val[b]) != OR_OK) ov = 1;
            t->val[c] = ov ? 0 : s;
            t->over[c] = (uint8_t)ov;
        }
    }
    return OR_OK;
}

static void binom_free(binom_table *t)
{
    free(t->val);
    free(t->over);
}

/* C(n, k) into *out; OR_E_OVERFLOW if it does not fit in 128 bits. */
static int binom_get(const binom_table *t, uint32_t n, uint32_t k, u128 *out)
{
    size_t c = (size_t)n * (t->k_max + 1) + k;
    if (t->over[c]) return OR_E_OVERFLOW;
    *out = t->val[c];
    return OR_OK;
}

/* Binomial coefficient through the same Pascal table, for the pin tests. */
int oracle_binom(uint32_t n, uint32_t k, uint64_t *lo, uint64_t *hi)
{
    if (!lo || !hi || k > 256 || n > 200000) return OR_E_ARG;
    binom_table t;
    int rc = binom_init(&t, n, k);
    if (rc == OR_OK) {
        u128 v = 0;
        rc = binom_get(&t, n, k, &v);
        if (rc == OR_OK) {
            *lo = (uint64_t)v;
            *hi = (uint64_t)(v >> 64);
        }
    }
    binom_free(&t);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Graph: validated copy of the U-side CSR plus its own transpose.     */

typedef struct {
    uint64_t n_u, n_v, nnz;
    uint64_t *ptr_u;
    uint32_t *adj_u;   /* N(u): sorted V ids */
    uint64_t *ptr_v;
    uint32_t *adj_v;   /* N(v): sorted U ids */
    uint32_t max_deg_u;
} og_graph;

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

static void graph_free(og_graph *g)
{
    free(g->ptr_u);
    free(g->adj_u);
    free(g->ptr_v);
    free(g->adj_v);
    memset(g, 0, sizeof(*g));
}

static int graph_load(og_graph *g, uint64_t n_u, uint64_t n_v,
                      const uint64_t *indptr, const uint32_t *indices)
{
    memset(g, 0, sizeof(*g));
    if (!indptr || (n_u > 0 && indptr[n_u] > 0 && !indices)) return OR_E_ARG;
    if (n_u >= (1ull << 32) || n_v >= (1ull << 32)) return OR_E_ARG;
    if (indptr[0] != 0) return OR_E_CSR;
    for (uint64_t u = 0; u < n_u; ++u)
        if (indptr[u + 1] < indptr[u]) return OR_E_CSR;
    uint64_t nnz = indptr[n_u];
    g->n_u = n_u;
    g->n_v = n_v;
    g->nnz = nnz;
    g->ptr_u = (uint64_t *)malloc((n_u + 1) * sizeof(uint64_t));
    g->adj_u = (uint32_t *)malloc((nnz ? nnz : 1) * sizeof(uint32_t));
    g->ptr_v = (uint64_t *)calloc(n_v + 1, sizeof(uint64_t));
    g->adj_v = (uint32_t *)malloc((nnz ? nnz : 1) * sizeof(uint32_t));
    if (!g->ptr_u || !g->adj_u || !g->ptr_v || !g->adj_v) { graph_free(g); return OR_E_OOM; }
    memcpy(g->ptr_u, indptr, (n_u + 1) * sizeof(uint64_t));
    if (nnz) memcpy(g->adj_u, indices, nnz * sizeof(uint32_t));
    for (uint64_t u = 0; u < n_u; ++u) {
        uint64_t b = g->ptr_u[u], e = g->ptr_u[u + 1];
        qsort(g->adj_u + b, e - b, sizeof(uint32_t), cmp_u32);
        for (uint64_t i = b; i < e; ++i) {
            if (g->adj_u[i] >= n_v) { graph_free(g); return OR_E_CSR; }
            if (i > b && g->adj_u[i] == g->adj_u[i - 1]) { graph_free(g); return OR_E_CSR; }
        }
        if (e - b > g->max_deg_u) g->max_deg_u = (uint32_t)(e - b);
    }
    /* Transpose by counting; visiting u in increasing order keeps N(v) sorted. */
    for (uint64_t i = 0; i < nnz; ++i) g->ptr_v[g->adj_u[i] + 1]++;
    for (uint64_t v = 0; v < n_v; ++v) g->ptr_v[v + 1] += g->ptr_v[v];
    uint64_t *fill = (uint64_t *)malloc((n_v + 1) * sizeof(uint64_t));
    if (!fill) { graph_free(g); return OR_E_OOM; }
    memcpy(fill, g->ptr_v, (n_v + 1) * sizeof(uint64_t));
    for (uint64_t u = 0; u < n_u; ++u)
        for (uint64_t i = g->ptr_u[u]; i < g->ptr_u[u + 1]; ++i)
            g->adj_v[fill[g->adj_u[i]]++] = (uint32_t)u;
    free(fill);
    return OR_OK;
}

/* Sorted linear merge: out = a intersect b; returns |out|. */
static uint32_t merge_intersect(const uint32_t *a, uint32_t na, const uint32_t *b, uint32_t nb,
                                uint32_t *out)
{
    uint32_t i = 0, j = 0, n = 0;
    while (i < na && j < nb) {
        if (a[i] < b[j]) ++i;
        else if (a[i] > b[j]) ++j;
        else { out[n++] = a[i]; ++i; ++j; }
    }
    return n;
}

/* ------------------------------------------------------------------ */
/* Vertex order.  key 0: id.  key 1: (degree, id).  key 2: (|N_2^q|, id),
 * with N_2^q over U without orientation (Definition 2's quantity; its
 * "higher priority first" direction is only a relabelling of the same
 * order and does not change the count).                               */

static _Thread_local const uint64_t *g_sort_key;

static int cmp_by_key(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    uint64_t kx = g_sort_key[x], ky = g_sort_key[y];
    if (kx != ky) return (kx > ky) - (kx < ky);
    return (x > y) - (x < y);
}

static uint64_t two_hop_size(const og_graph *g, uint32_t u, uint32_t q, uint32_t *cnt,
                             uint32_t *touched)
{
    uint64_t nt = 0, size = 0;
    for (uint64_t i = g->ptr_u[u]; i < g->ptr_u[u + 1]; ++i) {
        uint32_t v = g->adj_u[i];
        for (uint64_t j = g->ptr_v[v]; j < g->ptr_v[v + 1]; ++j) {
            uint32_t w = g->adj_v[j];
            if (w == u) continue;
            if (cnt[w]++ == 0) touched[nt++] = w;
        }
    }
    for (uint64_t t = 0; t < nt; ++t) {
        if (cnt[touched[t]] >= q) ++size;
        cnt[touched[t]] = 0;
    }
    return size;
}

/* rank[u] = position of u in the order; by_rank = inverse. */
static int make_order(const og_graph *g, int order_key, uint32_t q, uint32_t *rank, uint32_t *by_rank)
{
    uint64_t n = g->n_u;
    uint64_t *key = (uint64_t *)calloc(n ? n : 1, sizeof(uint64_t));
    if (!key) return OR_E_OOM;
    if (order_key == 1) {
        for (uint64_t u = 0; u < n; ++u) key[u] = g->ptr_u[u + 1] - g->ptr_u[u];
    } else if (order_key == 2) {
        uint32_t *cnt = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
        uint32_t *touched = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
        if (!cnt || !touched) { free(cnt); free(touched); free(key); return OR_E_OOM; }
        for (uint64_t u = 0; u < n; ++u) key[u] = two_hop_size(g, (uint32_t)u, q, cnt, touched);
        free(cnt);
        free(touched);
    } else if (order_key != 0) {
        free(key);
        return OR_E_ARG;
    }
    for (uint64_t u = 0; u < n; ++u) by_rank[u] = (uint32_t)u;
    g_sort_key = key;
    qsort(by_rank, n, sizeof(uint32_t), cmp_by_key);
    for (uint64_t r = 0; r < n; ++r) rank[by_rank[r]] = (uint32_t)r;
    free(key);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* The enumeration.                                                    */

typedef struct {
    const og_graph *g;
    const binom_table *bt;
    const uint32_t *rank, *by_rank;
    uint32_t p, q;
    int prune;
    uint64_t rank_lo, rank_hi;
    const uint64_t *rank_list;   /* if non-NULL: count these ranks one by one */
    uint64_t n_list;
    u128 *per_list;              /* per-entry counts for rank_list */
    int32_t *per_status;         /* per-entry status for rank_list */
    uint64_t max_nodes;          /* per-root intersection budget (0 = none) */
    atomic_uint_fast64_t next;
    /* per-thread results are summed by the caller */
} job_t;

typedef struct {
    job_t *job;
    u128 total;
    uint64_t nodes;
    int status;
    uint64_t node_limit;         /* abort the current root past this count */
    /* scratch */
    uint32_t *cnt, *touched, *cand;
    uint32_t **S;   /* S[d]: common neighbours at depth d (1..p) */
} worker_t;

/* Depth-first extension of L.  S (size nS) = common neighbours of the
 * vertices of L, |L| = depth; cand = candidates ranked after the last vertex
 * of L, in increasing rank order. */
static int extend(worker_t *w, uint32_t depth, const uint32_t *S, uint32_t nS,
                  const uint32_t *cand, uint32_t ncand, u128 *acc)
{
    const job_t *jb = w->job;
    const og_graph *g = jb->g;
    for (uint32_t i = 0; i < ncand; ++i) {
        if (jb->prune && ncand - i < jb->p - depth) break;
        uint32_t c = cand[i];
        uint32_t *S2 = w->S[depth + 1];
        uint32_t n2 = merge_intersect(S, nS, g->adj_u + g->ptr_u[c],
                                      (uint32_t)(g->ptr_u[c + 1] - g->ptr_u[c]), S2);
        if (++w->nodes > w->node_limit) return OR_E_BUDGET;
        if (jb->prune && n2 < jb->q) continue;
        if (depth + 1 == jb->p) {
            u128 c_nq = 0;
            if (n2 >= jb->q) {
                int rc = binom_get(jb->bt, n2, jb->q, &c_nq);
                if (rc != OR_OK) return rc;
            }
            if (add_u128(acc, c_nq) != OR_OK) return OR_E_OVERFLOW;
        } else {
            int rc = extend(w, depth + 1, S2, n2, cand + i + 1, ncand - i - 1, acc);
            if (rc != OR_OK) return rc;
        }
    }
    return OR_OK;
}

/* All p-subsets whose lowest-ranked member is u. */
static int count_root(worker_t *w, uint32_t u, u128 *out)
{
    const job_t *jb = w->job;
    const og_graph *g = jb->g;
    uint32_t du = (uint32_t)(g->ptr_u[u + 1] - g->ptr_u[u]);
    const uint32_t *Nu = g->adj_u + g->ptr_u[u];
    u128 acc = 0;
    *out = 0;
    if (jb->p == 1) {
        if (du >= jb->q) {
            int rc = binom_get(jb->bt, du, jb->q, &acc);
            if (rc != OR_OK) return rc;
        }
        w->nodes++;
        *out = acc;
        return OR_OK;
    }
    if (jb->prune && du < jb->q) return OR_OK;
    uint32_t ru = jb->rank[u];
    uint32_t ncand = 0;
    if (jb->prune) {
        /* Oriented N_2^q(u): common-neighbour counts by a wedge scan u-v-w. */
        uint64_t nt = 0;
        for (uint32_t i = 0; i < du; ++i) {
            uint32_t v = Nu[i];
            for (uint64_t j = g->ptr_v[v]; j < g->ptr_v[v + 1]; ++j) {
                uint32_t x = g->adj_v[j];
                if (jb->rank[x] <= ru) continue;
                if (w->cnt[x]++ == 0) w->touched[nt++] = x;
            }
        }
        for (uint64_t t = 0; t < nt; ++t) {
            uint32_t x = w->touched[t];
            if (w->cnt[x] >= jb->q) w->cand[ncand++] = jb->rank[x];
            w->cnt[x] = 0;
        }
        if (ncand < jb->p - 1) return OR_OK;
        qsort(w->cand, ncand, sizeof(uint32_t), cmp_u32);
        for (uint32_t i = 0; i < ncand; ++i) w->cand[i] = jb->by_rank[w->cand[i]];
    } else {
        for (uint64_t r = (uint64_t)ru + 1; r < g->n_u; ++r) w->cand[ncand++] = jb->by_rank[r];
    }
    memcpy(w->S[1], Nu, du * sizeof(uint32_t));
    int rc = extend(w, 1, w->S[1], du, w->cand, ncand, &acc);
    if (rc != OR_OK) return rc;
    *out = acc;
    return OR_OK;
}

static void *worker_main(void *arg)
{
    worker_t *w = (worker_t *)arg;
    job_t *jb = w->job;
    uint64_t n_items = jb->rank_list ? jb->n_list : jb->rank_hi - jb->rank_lo;
    for (;;) {
        uint64_t it = atomic_fetch_add(&jb->next, 1);
        if (it >= n_items) break;
        uint64_t r = jb->rank_list ? jb->rank_list[it] : jb->rank_lo + it;
        u128 c = 0;
        w->node_limit = jb->max_nodes ? w->nodes + jb->max_nodes : UINT64_MAX;
        int rc = count_root(w, jb->by_rank[r], &c);
        if (rc == OR_E_BUDGET && jb->rank_list) {
            /* Only per-root queries may give up on a root: it is reported as
             * not computed and contributes nothing. */
            jb->per_status[it] = OR_E_BUDGET;
            continue;
        }
        if (rc != OR_OK) { w->status = rc; break; }
        if (jb->rank_list) {
            jb->per_list[it] = c;
            jb->per_status[it] = OR_OK;
            continue;
        }
        if (add_u128(&w->total, c) != OR_OK) { w->status = OR_E_OVERFLOW; break; }
    }
    return NULL;
}

static int run_job(job_t *jb, int threads, u128 *total, uint64_t *nodes)
{
    const og_graph *g = jb->g;
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    worker_t *ws = (worker_t *)calloc((size_t)threads, sizeof(worker_t));
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    int rc = OR_OK;
    if (!ws || !tid) { free(ws); free(tid); return OR_E_OOM; }
    for (int t = 0; t < threads && rc == OR_OK; ++t) {
        worker_t *w = &ws[t];
        w->job = jb;
        w->cnt = (uint32_t *)calloc(g->n_u ? g->n_u : 1, sizeof(uint32_t));
        w->touched = (uint32_t *)malloc((g->n_u ? g->n_u : 1) * sizeof(uint32_t));
        w->cand = (uint32_t *)malloc((g->n_u ? g->n_u : 1) * sizeof(uint32_t));
        w->S = (uint32_t **)calloc(jb->p + 2, sizeof(uint32_t *));
        if (!w->cnt || !w->touched || !w->cand || !w->S) { rc = OR_E_OOM; break; }
        for (uint32_t d = 0; d <= jb->p + 1; ++d) {
            w->S[d] = (uint32_t *)malloc((g->max_deg_u + 1) * sizeof(uint32_t));
            if (!w->S[d]) { rc = OR_E_OOM; break; }
        }
    }
    int started = 0;
    if (rc == OR_OK) {
        for (int t = 0; t < threads; ++t) {
            if (pthread_create(&tid[t], NULL, worker_main, &ws[t]) != 0) break;
            ++started;
        }
        if (started == 0) rc = OR_E_OOM;
        for (int t = 0; t < started; ++t) pthread_join(tid[t], NULL);
    }
    u128 sum = 0;
    uint64_t nsum = 0;
    for (int t = 0; t < threads; ++t) {
        worker_t *w = &ws[t];
        if (rc == OR_OK && w->status != OR_OK) rc = w->status;
        if (rc == OR_OK && add_u128(&sum, w->total) != OR_OK) rc = OR_E_OVERFLOW;
        nsum += w->nodes;
        free(w->cnt);
        free(w->touched);
        free(w->cand);
        if (w->S)
            for (uint32_t d = 0; d <= jb->p + 1; ++d) free(w->S[d]);
        free(w->S);
    }
    free(ws);
    free(tid);
    if (rc == OR_OK) {
        *total = sum;
        if (nodes) *nodes = nsum;
    }
    return rc;
}

/* ------------------------------------------------------------------ */
/* Public entry points (ctypes).                                       */

/*
 * Count (p,q)-bicliques with U as the side of L.  Only roots whose rank lies
 * in [rank_lo, rank_hi) are counted, so disjoint rank ranges give additive
 * partial counts.  order_key selects the rank (0 id, 1 degree, 2 |N_2^q|).
 * threads > 1 spreads roots over POSIX threads.  Result in (*lo, *hi);
 * *nodes (nullable) receives the number of intersections performed.
 */
int oracle_count(uint64_t n_u, uint64_t n_v, const uint64_t *indptr_u, const uint32_t *indices_u,
                 uint32_t p, uint32_t q, int order_key, int prune,
                 uint64_t rank_lo, uint64_t rank_hi, int threads,
                 uint64_t *lo, uint64_t *hi, uint64_t *nodes)
{
    if (!lo || !hi || p == 0 || q == 0 || p > 256 || q > 256) return OR_E_ARG;
    og_graph g;
    int rc = graph_load(&g, n_u, n_v, indptr_u, indices_u);
    if (rc != OR_OK) return rc;
    if (rank_hi > n_u) rank_hi = n_u;
    if (rank_lo > rank_hi) rank_lo = rank_hi;
    uint32_t *rank = (uint32_t *)malloc((n_u ? n_u : 1) * sizeof(uint32_t));
    uint32_t *by_rank = (uint32_t *)malloc((n_u ? n_u : 1) * sizeof(uint32_t));
    binom_table bt = {0};
    if (!rank || !by_rank) rc = OR_E_OOM;
    if (rc == OR_OK) rc = make_order(&g, order_key, q, rank, by_rank);
    if (rc == OR_OK) rc = binom_init(&bt, g.max_deg_u, q);
    u128 total = 0;
    if (rc == OR_OK) {
        job_t jb;
        memset(&jb, 0, sizeof(jb));
        jb.g = &g;
        jb.bt = &bt;
        jb.rank = rank;
        jb.by_rank = by_rank;
        jb.p = p;
        jb.q = q;
        jb.prune = prune;
        jb.rank_lo = rank_lo;
        jb.rank_hi = rank_hi;
        atomic_init(&jb.next, 0);
        rc = run_job(&jb, threads, &total, nodes);
    }
    if (rc == OR_OK) {
        *lo = (uint64_t)total;
        *hi = (uint64_t)(total >> 64);
    }
    binom_free(&bt);
    free(rank);
    free(by_rank);
    graph_free(&g);
    return rc;
}

/*
 * Per-root counts: for each of the n ranks in rank_list, the number of
 * bicliques whose lowest-ranked L member has that rank, into
 * (out_lo[i], out_hi[i]), with out_status[i] = OR_OK.  With max_nodes > 0 a
 * root that needs more than max_nodes intersections is abandoned and gets
 * out_status[i] = OR_E_BUDGET (its count is then not computed).
 */
int oracle_count_ranks(uint64_t n_u, uint64_t n_v, const uint64_t *indptr_u,
                       const uint32_t *indices_u, uint32_t p, uint32_t q, int order_key,
                       const uint64_t *rank_list, uint64_t n, int threads, uint64_t max_nodes,
                       uint64_t *out_lo, uint64_t *out_hi, int32_t *out_status)
{
    if (p == 0 || q == 0 || p > 256 || q > 256 ||
        (n && (!rank_list || !out_lo || !out_hi || !out_status)))
        return OR_E_ARG;
    og_graph g;
    int rc = graph_load(&g, n_u, n_v, indptr_u, indices_u);
    if (rc != OR_OK) return rc;
    for (uint64_t i = 0; i < n; ++i)
        if (rank_list[i] >= n_u) { graph_free(&g); return OR_E_ARG; }
    uint32_t *rank = (uint32_t *)malloc((n_u ? n_u : 1) * sizeof(uint32_t));
    uint32_t *by_rank = (uint32_t *)malloc((n_u ? n_u : 1) * sizeof(uint32_t));
    u128 *per = (u128 *)calloc(n ? n : 1, sizeof(u128));
    binom_table bt = {0};
    if (!rank || !by_rank || !per) rc = OR_E_OOM;
    if (rc == OR_OK) rc = make_order(&g, order_key, q, rank, by_rank);
    if (rc == OR_OK) rc = binom_init(&bt, g.max_deg_u, q);
    if (rc == OR_OK) {
        job_t jb;
        memset(&jb, 0, sizeof(jb));
        jb.g = &g;
        jb.bt = &bt;
        jb.rank = rank;
        jb.by_rank = by_rank;
        jb.p = p;
        jb.q = q;
        jb.prune = 1;
        jb.rank_list = rank_list;
        jb.n_list = n;
        jb.per_list = per;
        jb.per_status = out_status;
        jb.max_nodes = max_nodes;
        atomic_init(&jb.next, 0);
        u128 total = 0;
        rc = run_job(&jb, threads, &total, NULL);
    }
    if (rc == OR_OK)
        for (uint64_t i = 0; i < n; ++i) {
            out_lo[i] = (uint64_t)per[i];
            out_hi[i] = (uint64_t)(per[i] >> 64);
        }

    free(per);
    binom_free(&bt);
    free(rank);
    free(by_rank);
    graph_free(&g);
    return rc;
}

/*
 * The rank order itself (for tests of the ordering rule): by_rank[r] = the U
 * vertex of rank r.
 */
int oracle_order(uint64_t n_u, uint64_t n_v, const uint64_t *indptr_u, const uint32_t *indices_u,
                 int order_key, uint32_t q, uint32_t *by_rank_out)
{
    if (!by_rank_out) return OR_E_ARG;
    og_graph g;
    int rc = graph_load(&g, n_u, n_v, indptr_u, indices_u);
    if (rc != OR_OK) return rc;
    uint32_t *rank = (uint32_t *)malloc((n_u ? n_u : 1) * sizeof(uint32_t));
    if (!rank) rc = OR_E_OOM;
    if (rc == OR_OK) rc = make_order(&g, order_key, q, rank, by_rank_out);
    free(rank);
    graph_free(&g);
    return rc;
}

/*
 * Candidate sets of the Basic model (Section III-A) after the vertices of L
 * (in the given order) have been added, with no orientation:
 *   C_R = intersection of N(x) over x in L,
 *   C_L = intersection of N_2^q(x) over x in L, minus L,
 * where N_2^q(x) = { w in U, w != x : |N(x) n N(w)| >= q }.
 * Sorted ids go to out_cr / out_cl (capacity n_v / n_u); sizes to *n_cr, *n_cl.
 */
int oracle_basic_sets(uint64_t n_u, uint64_t n_v, const uint64_t *indptr_u,
                      const uint32_t *indices_u, uint32_t q, const uint32_t *L, uint32_t n_l,
                      uint32_t *out_cr, uint32_t *n_cr, uint32_t *out_cl, uint32_t *n_cl)
{
    if (!L || n_l == 0 || !out_cr || !n_cr || !out_cl || !n_cl) return OR_E_ARG;
    og_graph g;
    int rc = graph_load(&g, n_u, n_v, indptr_u, indices_u);
    if (rc != OR_OK) return rc;
    for (uint32_t i = 0; i < n_l; ++i)
        if (L[i] >= n_u) { graph_free(&g); return OR_E_ARG; }
    uint32_t *in_cl = (uint32_t *)calloc(n_u ? n_u : 1, sizeof(uint32_t));
    uint32_t *tmp = (uint32_t *)malloc((n_v ? n_v : 1) * sizeof(uint32_t));
    uint32_t *tmp2 = (uint32_t *)malloc((n_v ? n_v : 1) * sizeof(uint32_t));
    if (!in_cl || !tmp || !tmp2) rc = OR_E_OOM;
    if (rc == OR_OK) {
        /* C_R */
        uint32_t n = (uint32_t)(g.ptr_u[L[0] + 1] - g.ptr_u[L[0]]);
        memcpy(tmp, g.adj_u + g.ptr_u[L[0]], n * sizeof(uint32_t));
        for (uint32_t i = 1; i < n_l; ++i) {
            n = merge_intersect(tmp, n, g.adj_u + g.ptr_u[L[i]],
                                (uint32_t)(g.ptr_u[L[i] + 1] - g.ptr_u[L[i]]), tmp2);
            memcpy(tmp, tmp2, n * sizeof(uint32_t));
        }
        memcpy(out_cr, tmp, n * sizeof(uint32_t));
        *n_cr = n;
        /* C_L: w is kept when it is in N_2^q(x) for every x in L. */
        for (uint32_t w = 0; w < n_u; ++w) {
            uint32_t ok = 1;
            for (uint32_t i = 0; i < n_l && ok; ++i) {
                if (w == L[i]) { ok = 0; break; }
                uint32_t c = merge_intersect(g.adj_u + g.ptr_u[w],
                                             (uint32_t)(g.ptr_u[w + 1] - g.ptr_u[w]),
                                             g.adj_u + g.ptr_u[L[i]],
                                             (uint32_t)(g.ptr_u[L[i] + 1] - g.ptr_u[L[i]]), tmp2);
                if (c < q) ok = 0;
            }
            in_cl[w] = ok;
        }
        uint32_t m = 0;
        for (uint32_t w = 0; w < n_u; ++w)
            if (in_cl[w]) out_cl[m++] = w;
        *n_cl = m;
    }
    free(in_cl);
    free(tmp);
    free(tmp2);
    graph_free(&g);
    return rc;
}

/*
 * Hierarchical truncated bitmap of one sorted id list (Section V-A): id x
 * goes to word i = x / word_bits at bit j = x % word_bits (bit weight 2^j).
 * Writes the distinct word indices (Idx) and the words (Val) in increasing
 * index order; returns their number in *n_words.  word_bits is 32 or 64.
 */
int oracle_htb_encode(const uint32_t *ids, uint32_t n, uint32_t word_bits,
                      uint64_t *out_idx, uint64_t *out_val, uint32_t *n_words)
{
    if ((word_bits != 32 && word_bits != 64) || !n_words || (n && (!ids || !out_idx || !out_val)))
        return OR_E_ARG;
    uint32_t m = 0;
    for (uint32_t k = 0; k < n; ++k) {
        if (k > 0 && ids[k] <= ids[k - 1]) return OR_E_ARG;
        uint64_t i = ids[k] / word_bits, j = ids[k] % word_bits;
        if (m == 0 || out_idx[m - 1] != i) {
            out_idx[m] = i;
            out_val[m] = 0;
            ++m;
        }
        out_val[m - 1] |= (uint64_t)1 << j;
    }
    *n_words = m;
    return OR_OK;
}

/*
 * Two-phase intersection of two HTB lists (Section V-A): matching word
 * indices are found first, then the words are combined by bitwise AND.
 * Result words with at least one bit set are written in index order.
 */
int oracle_htb_intersect(const uint64_t *idx_a, const uint64_t *val_a, uint32_t na,
                         const uint64_t *idx_b, const uint64_t *val_b, uint32_t nb,
                         uint64_t *out_idx, uint64_t *out_val, uint32_t *n_out)
{
    if (!n_out || (na && (!idx_a || !val_a)) || (nb && (!idx_b || !val_b))) return OR_E_ARG;
    uint32_t i = 0, j = 0, m = 0;
    while (i < na && j < nb) {
        if (idx_a[i] < idx_b[j]) ++i;
        else if (idx_a[i] > idx_b[j]) ++j;
        else {
            uint64_t v = val_a[i] & val_b[j];
            if (v) {
                out_idx[m] = idx_a[i];
                out_val[m] = v;
                ++m;
            }
            ++i;
            ++j;
        }
    }
    *n_out = m;
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Per-vertex counts: the output set of Algorithm 1 reduced to how many
 * bicliques each vertex belongs to.                                   */

typedef struct {
    const og_graph *g;
    const binom_table *bt;
    uint32_t p, q;
    uint32_t *L;       /* L[0 .. depth): members chosen so far, increasing ids */
    uint32_t **S;      /* S[d]: common neighbours of L[0 .. d) */
    uint32_t *nS;      /* |S[d]| */
    u128 *cu, *cv;     /* per-vertex totals of U and V */
} pv_t;

/* Extends L (depth members, S = S[depth]) by every x > the last member.  A
 * complete L with n = |S| common neighbours holds C(n, q) bicliques (any q of
 * S as R): each member of L is in all of them, and each v in S is in the
 * C(n-1, q-1) of them whose R contains v.  A subset whose S has fewer than q
 * vertices holds none and neither does any subset that extends it, so it is
 * not extended. */
static int pv_extend(pv_t *w, uint32_t depth, uint32_t from)
{
    const og_graph *g = w->g;
    for (uint64_t x = from; x < g->n_u; ++x) {
        const uint32_t *Nx = g->adj_u + g->ptr_u[x];
        const uint32_t dx = (uint32_t)(g->ptr_u[x + 1] - g->ptr_u[x]);
        uint32_t n;
        if (depth == 0) {
            memcpy(w->S[1], Nx, dx * sizeof(uint32_t));
            n = dx;
        } else {
            n = merge_intersect(w->S[depth], w->nS[depth], Nx, dx, w->S[depth + 1]);
        }
        if (n < w->q) continue;
        w->nS[depth + 1] = n;
        w->L[depth] = (uint32_t)x;
        if (depth + 1 == w->p) {
            u128 all = 0, with_v = 0;
            int rc = binom_get(w->bt, n, w->q, &all);
            if (rc == OR_OK) rc = binom_get(w->bt, n - 1, w->q - 1, &with_v);
            if (rc != OR_OK) return rc;
            for (uint32_t i = 0; i < w->p; ++i)
                if (add_u128(&w->cu[w->L[i]], all) != OR_OK) return OR_E_OVERFLOW;
            for (uint32_t i = 0; i < n; ++i)
                if (add_u128(&w->cv[w->S[depth + 1][i]], with_v) != OR_OK) return OR_E_OVERFLOW;
        } else {
            int rc = pv_extend(w, depth + 1, (uint32_t)x + 1);
            if (rc != OR_OK) return rc;
        }
    }
    return OR_OK;
}

/*
 * Per-vertex counts: for every x in U, the number of (p,q)-bicliques (L, R)
 * with x in L, into (u_lo[x], u_hi[x]); for every v in V, the number with v in
 * R, into (v_lo[v], v_hi[v]).  Single-threaded, for small graphs.
 */
int oracle_count_per_vertex(uint64_t n_u, uint64_t n_v, const uint64_t *indptr_u, const uint32_t *indices_u,
                            uint32_t p, uint32_t q, uint64_t *u_lo, uint64_t *u_hi, uint64_t *v_lo,
                            uint64_t *v_hi)
{
    if (!u_lo || !u_hi || !v_lo || !v_hi || p == 0 || q == 0 || p > 256 || q > 256) return OR_E_ARG;
    og_graph g;
    int rc = graph_load(&g, n_u, n_v, indptr_u, indices_u);
    if (rc != OR_OK) return rc;
    binom_table bt = {0};
    pv_t w;
    memset(&w, 0, sizeof(w));
    w.g = &g;
    w.bt = &bt;
    w.p = p;
    w.q = q;
    w.L = (uint32_t *)calloc(p + 1, sizeof(uint32_t));
    w.S = (uint32_t **)calloc(p + 2, sizeof(uint32_t *));
    w.nS = (uint32_t *)calloc(p + 2, sizeof(uint32_t));
    w.cu = (u128 *)calloc(n_u ? n_u : 1, sizeof(u128));
    w.cv = (u128 *)calloc(n_v ? n_v : 1, sizeof(u128));
    if (!w.L || !w.S || !w.nS || !w.cu || !w.cv) rc = OR_E_OOM;
    for (uint32_t d = 0; rc == OR_OK && d <= p + 1; ++d) {
        w.S[d] = (uint32_t *)malloc((g.max_deg_u + 1) * sizeof(uint32_t));
        if (!w.S[d]) rc = OR_E_OOM;
    }
    if (rc == OR_OK) rc = binom_init(&bt, g.max_deg_u, q);
    if (rc == OR_OK) rc = pv_extend(&w, 0, 0);
    if (rc == OR_OK) {
        for (uint64_t x = 0; x < n_u; ++x) {
            u_lo[x] = (uint64_t)w.cu[x];
            u_hi[x] = (uint64_t)(w.cu[x] >> 64);
        }
        for (uint64_t v = 0; v < n_v; ++v) {
            v_lo[v] = (uint64_t)w.cv[v];
            v_hi[v] = (uint64_t)(w.cv[v] >> 64);
        }
    }
    if (w.S)
        for (uint32_t d = 0; d <= p + 1; ++d) free(w.S[d]);
    free(w.S);
    free(w.nS);
    free(w.L);
    free(w.cu);
    free(w.cv);
    binom_free(&bt);
    graph_free(&g);
    return rc;
}
