/*
 * bc.h -- exact (p,q)-biclique counting on AMD Instinct MI355X (gfx950).
 *
 * Problem (Section II-A, Definition 1 and the problem statement): given a
 * bipartite graph G = (U, V, E) and two integers p, q, return the number of
 * pairs (L, R) with L a p-subset of U, R a q-subset of V and every (u, v) in
 * L x R an edge of E.  Equivalently, the sum over p-subsets L of U of
 * C(|common neighbours of L|, q) -- the leaf rule of the Basic model
 * (Section III-A), which is what the device path evaluates.
 *
 * Plain C99 ABI: fixed-width integers and plain pointers only.  Every call
 * returns a bc_status (0 = BC_OK, negative = error); nothing throws across
 * the boundary.  On error no output argument is written, and
 * bc_last_error() returns a detail message for the calling thread.
 *
 * Counts are exact unsigned 128-bit integers (count = hi * 2^64 + lo).  If the
 * true count does not fit in 128 bits the call fails with BC_E_OVERFLOW.
 * No floating point takes part in any count.
 */
#ifndef BC_H
#define BC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bc_status;
enum {
    BC_OK = 0,
    BC_E_INVALID_ARG = -1,   /* NULL pointer, p or q outside 1..32, bad option value */
    BC_E_BAD_CSR = -2,       /* indptr not a prefix array, id out of range, duplicate edge */
    BC_E_INCONSISTENT = -3,  /* the U-side and V-side CSRs are not transposes */
    BC_E_OOM = -4,           /* host or device allocation failed */
    BC_E_DEVICE = -5,        /* a HIP runtime error; the HIP message is in bc_last_error() */
    BC_E_OVERFLOW = -6,      /* the count needs more than 128 bits */
    BC_E_REJECTED = -7,      /* server: query refused by admission control */
    BC_E_TIMEOUT = -8,       /* the time limit or deadline passed before the count finished */
    BC_E_CANCELLED = -9,     /* server: shut down before the query ran */
    BC_E_PENDING = -10,      /* server: non-blocking poll, result not ready yet */
    BC_E_NOT_FOUND = -11     /* server: unknown ticket or graph id */
};

typedef struct { uint64_t lo, hi; } bc_u128;

/* One side of the graph in CSR form, in HOST memory.  Row r lists the ids
 * (in [0, n_cols)) of the other side adjacent to vertex r; rows may be
 * unsorted, duplicates are rejected.  indptr has n_rows + 1 nondecreasing
 * entries with indptr[0] == 0 and indptr[n_rows] == nnz. */
typedef struct {
    uint64_t n_rows, n_cols, nnz;
    const uint64_t *indptr;
    const uint32_t *indices;
} bc_csr;

typedef struct bc_graph bc_graph;   /* opaque; immutable after bc_build */

/* Anchor: the side that L is drawn from.  The count never depends on it.
 * AUTO takes the side with the smaller of p, q as L's (U when p < q, V when
 * q < p, U when p == q <= 2).  For p == q >= 3 it takes the side with the
 * smaller planning cost (sum over roots of k^min(p-1,3) times the root's row
 * words, k = the root's candidates).  When the two sides have at least 65536
 * roots together it is estimated from 1 in 16 roots of each side; estimates
 * within 15 % of each other go to the side whose candidate pass scans fewer
 * wedges (sum over the other side's vertices of C(d,2)).  Smaller graphs take
 * the cost from a candidate pass over all roots of both sides. */
enum { BC_ANCHOR_AUTO = -1, BC_ANCHOR_U = 0, BC_ANCHOR_V = 1 };

/*
 * Device-memory hook (e.g. a framework's caching allocator).  alloc returns
 * `bytes` of device memory usable by work queued on `stream` (a hipStream_t),
 * or NULL when it cannot (the call then fails with BC_E_OOM after releasing
 * everything it took).  free gives back a block alloc returned; the library
 * calls it with the same stream once all work it queued on the block is on
 * that stream, so a stream-ordered allocator may reuse the block at once.
 * Blocks a graph keeps (bc_build) are freed by bc_free with stream NULL.
 * The hook object and ctx must outlive every call and graph that uses them.
 */
typedef struct {
    void *ctx;
    void *(*alloc)(void *ctx, size_t bytes, void *stream);
    void (*free)(void *ctx, void *ptr, void *stream);
} bc_allocator;

/* Vertex order keys of bc_build (Definition 2: vertex priority). */
enum {
    BC_ORDER_DEGREE = 0,    /* ascending degree, ties by id (default) */
    BC_ORDER_TWO_HOP = 1,   /* ascending |N_2^k(x)|: same-side vertices sharing >= k neighbours with x,
                               k = bc_opts.order_k (0 = 2); ties by original id */
    BC_ORDER_BORDER = 2     /* Border (Algorithm 2, Section V-B): the degree order, then up to
                               bc_opts.border_iters (0 = 4096) greedy swaps per side that each remove
                               the most 1-blocks (32-id blocks of a row holding one neighbour) */
};

/* Root-build paths (bc_opts.root_build). */
enum {
    BC_ROOT_BUILD_AUTO = 0,      /* one fused kernel per root (LDS hash table) when the device has the LDS */
    BC_ROOT_BUILD_TWO_PASS = 1   /* candidate counts, host plan, then rows: two kernels with HBM counters */
};

/* Set representations of the enumeration (bc_opts.sets). */
enum {
    BC_SETS_LOCAL_BITMAP = 0,   /* per-root bitmap rows over the root's own neighbourhood (default) */
    BC_SETS_HTB = 1,            /* the graph's hierarchical truncated bitmaps (Section V-A): a set is
                                   32-bit words, each with its index; intersections binary-search the
                                   indices, then AND the words */
    BC_SETS_SORTED = 2          /* sorted adjacency lists intersected by binary search (Section III-B) */
};

/* Options.  Pass NULL for all defaults.  No field changes any count.
 * Fields after timeout_ms are read only when struct_size covers them. */
typedef struct {
    uint32_t struct_size;      /* sizeof(bc_opts), for forward compatibility */
    void *stream;              /* hipStream_t to run on; NULL = the library's own stream */
    int32_t anchor;            /* BC_ANCHOR_AUTO / _U / _V */
    uint32_t lds_words;        /* per-wavefront LDS budget in 64-bit words; 0 = default */
    uint32_t waves_per_cu;     /* persistent-grid occupancy target, 1..12 wavefronts per CU (larger is
                                  capped); 0 = default (12) */
    uint32_t instrument;       /* nonzero: fill the work counters of bc_stats */
    uint32_t timeout_ms;       /* device-side time limit of the call (0 = none); past it the
                                  call fails with BC_E_TIMEOUT and no count is returned */
    const bc_allocator *alloc; /* device memory for the call's scratch (and, in bc_build, the
                                  graph's arrays); NULL = hipMallocAsync on the stream */
    int32_t order_key;         /* bc_build: BC_ORDER_DEGREE or BC_ORDER_TWO_HOP */
    uint32_t order_k;          /* bc_build, BC_ORDER_TWO_HOP: the sharing threshold k (0 = 2) */
    uint32_t roots_per_wave;   /* enumeration tasks a wavefront takes per queue pop, 1..64;
                                  0 = auto (8 on launches with >= 1024 tasks per wave, else 4) */
    uint32_t switch_depth;     /* levels above the leaves that a small node expands breadth-first in
                                  one matrix-core sweep instead of depth-first: 2 (pairs of the last
                                  candidate list) or 3 (triples, nodes of <= 96 rows); 0 = auto (3) */
    uint32_t split_rows;       /* runtime split of heavy tasks (p_A >= 5): a (root, second vertex)
                                  task whose level-2 block keeps more rows than this pushes one
                                  subtask per child row to a device queue that idle wavefronts
                                  drain; 0 or 0xffffffff = never split (the default) */
    uint32_t root_build;       /* BC_ROOT_BUILD_AUTO / _TWO_PASS */
    uint32_t sets;             /* BC_SETS_LOCAL_BITMAP / _HTB / _SORTED (the last two send every root
                                  through the global-set path) */
    uint32_t bitmap_bits;      /* BC_SETS_LOCAL_BITMAP: the widest root bitmap, in bits (= neighbours
                                  of the root); roots with more neighbours take the HTB path
                                  instead; 0 = no limit */
    uint32_t border_iters;     /* bc_build, BC_ORDER_BORDER: swap steps per side (0 = 4096) */
    uint64_t scratch_cap_bytes;/* device scratch the call may take (0 = no cap): the enumeration grid
                                  shrinks to fit, and a call that cannot fit fails with BC_E_OOM */
    uint32_t pure_dfs;         /* global-set path: nonzero visits a node's candidates one at a time, the
                                  wavefront's lanes sharing each intersection (no BFS over siblings) */
} bc_opts;

/* Timings (milliseconds, measured with HIP events on the stream) and work
 * counters of one count. */
typedef struct {
    double ms_total, ms_candidates, ms_plan, ms_rows, ms_enumerate;
    int32_t anchor;            /* side actually used */
    uint64_t roots;            /* roots of the anchor side visited */
    uint64_t roots_active;     /* roots that own at least one task */
    uint64_t tasks;            /* (root, second vertex) tasks enumerated */
    uint64_t candidate_edges;  /* oriented 2-hop pairs sharing >= q (or p) neighbours */
    uint64_t row_words;        /* 64-bit words of per-root candidate bitmaps */
    uint64_t pair_ops;         /* instrumented: 64-bit word ANDs+popcounts of the fused leaf pairs */
    uint64_t filter_ops;       /* instrumented: 64-bit word ANDs+popcounts of the child filters */
    uint64_t cyc_setup, cyc_compact, cyc_pair, cyc_filter;  /* instrumented: shader-clock cycles summed
                                  over wavefronts in task setup, row compaction, leaf pairs, filters */
    uint64_t pairs;            /* instrumented: leaf pairs evaluated */
    uint64_t pair_slots;       /* instrumented: lane-slots spent on them (pairs / pair_slots = lane use) */
    uint64_t cyc_pack;         /* instrumented: the part of cyc_compact spent in tasks whose common
                                  neighbourhood had to be bit-packed (spread over more words than it needs) */
    uint64_t scratch_bytes;    /* device scratch the call took (all of it held until the call ends) */
    double ms_wave_makespan;   /* instrumented: first wavefront start to last wavefront end of the
                                  local-bitmap enumeration (device real-time clock) */
    double ms_wave_spread;     /* instrumented: first to last wavefront end (load imbalance) */
} bc_stats;

/*
 * bc_build -- validate a bipartite graph and copy it to the device.
 *
 * U lists N(u) for every u in U (n_rows = |U|, n_cols = |V|); V lists N(v)
 * for every v in V and must be the exact transpose of U (BC_E_INCONSISTENT
 * otherwise).  Rows are sorted and each side is relabelled by its vertex
 * order: ascending degree, ties by original id (BC_ORDER_DEGREE), or
 * ascending |N_2^k| (BC_ORDER_TWO_HOP, Definition 2's priority, computed on
 * the host by wedge counting).  A vertex's position in that order is its
 * "rank", which fixes the orientation of the search (vertex priority,
 * Section III-B).  Both CSR sides are then copied to device memory on
 * opts->stream (through opts->alloc when given).  The caller keeps ownership
 * of its arrays; nothing refers to them after return.  *out receives a graph
 * that owns its device memory until bc_free.
 */
bc_status bc_build(const bc_csr *U, const bc_csr *V, const bc_opts *opts, bc_graph **out);

/* Releases a graph and its device memory.  NULL is ignored. */
void bc_free(bc_graph *g);

/* Sizes of a built graph. */
bc_status bc_graph_info(const bc_graph *g, uint64_t *n_u, uint64_t *n_v, uint64_t *n_edges);

/*
 * Size of the hierarchical truncated bitmap (Section V-A) of one side's rows
 * (0 = U's rows over V ids, 1 = V's rows over U ids) under the graph's
 * vertex order: *words = 32-bit words over all rows, *one_blocks = those
 * holding a single neighbour (the 1-blocks that Border reduces).  Builds the
 * HTB if no count has needed it yet (it is kept with the graph).
 */
bc_status bc_htb_stats(bc_graph *g, int32_t side, uint64_t *words, uint64_t *one_blocks);

/*
 * rank_of[x] for every vertex x of one side (0 = U, 1 = V), in original ids:
 * the rank that orients the search.  rank_of must hold n entries.
 */
bc_status bc_ranks(const bc_graph *g, int32_t side, uint32_t *rank_of);

/*
 * bc_count -- number of (p,q)-bicliques of g, 1 <= p, q <= 32.
 *
 * Runs entirely on the device (Algorithm 1 restated for CDNA4): per-root
 * 2-hop candidate collection, bitmap rows of the common neighbours,
 * enumeration whose child filters are AND + popcount on the vector units,
 * and leaves adding C(|S|, q) from an exact table.  The leaf intersection
 * sizes of a candidate list come, pair by pair, from an int8 product of its
 * 0/1 rows on the matrix cores when every leaf value is below 2^28 (exact
 * integer arithmetic), else from AND + popcount.  p > |U| or q > |V| gives
 * 0.  The call returns when the count is on the host.  *st (nullable)
 * receives timings and counters.
 */
bc_status bc_count(const bc_graph *g, uint32_t p, uint32_t q, const bc_opts *opts,
                   bc_u128 *out, bc_stats *st);

/*
 * bc_count_roots -- the part of the count whose lowest-ranked L vertex has
 * rank in [rank_lo, rank_hi) on the given anchor side (BC_ANCHOR_U or _V;
 * AUTO is rejected).  Disjoint rank ranges give partial counts that add up
 * exactly to bc_count; with a one-rank range it is the per-root count.
 */
bc_status bc_count_roots(const bc_graph *g, uint32_t p, uint32_t q, int32_t anchor,
                         uint64_t rank_lo, uint64_t rank_hi, const bc_opts *opts,
                         bc_u128 *out, bc_stats *st);

/*
 * bc_count_batch -- n independent counts (graphs[i], p[i], q[i]) in one set
 * of persistent launches sharing one task queue.  out[i] and item_status[i]
 * receive each result; every out[i] with item_status[i] == BC_OK equals what
 * bc_count would return (out[i] is 0 otherwise).  Items with a bad graph
 * pointer or p, q outside 1..32 get BC_E_INVALID_ARG and the rest still run.
 * When the call as a whole fails before the counts are read back (device
 * error, BC_E_OOM, ...), it returns that status and every item that was to
 * run gets the same status: no item reports BC_OK unless its count was
 * computed.  BC_E_DEVICE with per-item statuses is also returned when an
 * item hit an internal bound.  st (nullable) receives the timings of the
 * whole call and work counters summed over all items (anchor: that of the
 * first item).
 */
bc_status bc_count_batch(const bc_graph *const *graphs, const uint32_t *p, const uint32_t *q,
                         size_t n, const bc_opts *opts, bc_u128 *out, bc_status *item_status, bc_stats *st);

/*
 * bc_count_per_vertex -- per-vertex counts (the output set B of Algorithm 1
 * reduced to how many bicliques each vertex belongs to): for
 * every vertex x of `side` (BC_ANCHOR_U or BC_ANCHOR_V), the number of
 * (p,q)-bicliques (L, R), L in U with |L| = p and R in V with |R| = q, that
 * hold x (in L for side U, in R for side V).  counts (host, one entry per
 * vertex of that side, indexed by the caller's vertex id) receives them;
 * their sum is p (side U) or q (side V) times bc_count.  The search runs with
 * `side` as the anchor: a leaf's C(n, q_A) bicliques are added to each of its
 * p_A members.  With p_A = 2 the candidate pass does it as it counts each
 * root's candidates; deeper searches run on the global-set path, which
 * visits every leaf with its members known; p_A = 1 is the closed form
 * C(d(x), q_A).  opts->sets picks HTB (default) or sorted lists; pure_dfs is
 * ignored.  Device scratch of 16
 * bytes per vertex of the side comes on top of the count's.  Errors as for
 * bc_count; on error counts is untouched.
 */
bc_status bc_count_per_vertex(const bc_graph *g, uint32_t p, uint32_t q, int32_t side, const bc_opts *opts,
                              bc_u128 *counts);

/*
 * bc_partition -- BCPar (Algorithm 3, Section VI): groups the roots of one
 * anchor side (BC_ANCHOR_U or _V; the anchor's depth, p for U and q for V,
 * must be at least 3) so that each group's closure -- its roots, their
 * oriented 2-hop candidates (ranked after the root, sharing at least q
 * neighbours for anchor U, p for V) and the neighbourhoods of all of them --
 * takes at most budget_bytes, counting 4 bytes per adjacency entry and per
 * candidate entry of each member (w(u) = |N(u)| + |N_2(u)|).  Greedy: a
 * group starts from the unassigned root of highest average candidate
 * weight and keeps taking the unassigned root that shares the most weight
 * with its closure while the budget holds (a root whose closure alone is
 * over budget forms a group by itself).  part_of_rank[r] (one entry per
 * vertex of the side) receives the group of the root of rank r; *n_parts
 * the number of groups.  Candidate sets are computed on the host.
 */
bc_status bc_partition(const bc_graph *g, uint32_t p, uint32_t q, int32_t anchor, uint64_t budget_bytes,
                       uint32_t *part_of_rank, uint32_t *n_parts);

/*
 * bc_count_partition -- the part of the count whose lowest-ranked L vertex
 * is a root of group `part` (part_of_rank as from bc_partition), computed on
 * the group's closure alone: that subgraph is built, uploaded, counted with
 * only the group's roots owning tasks, and freed.  Over all groups these
 * counts add up to bc_count.  *closure_edges (nullable) receives the
 * closure's edge count.  Same argument rules as bc_partition.
 */
bc_status bc_count_partition(const bc_graph *g, uint32_t p, uint32_t q, int32_t anchor,
                             const uint32_t *part_of_rank, uint32_t part, const bc_opts *opts, bc_u128 *out,
                             uint64_t *closure_edges);

/*
 * bc_scratch_estimate -- an upper bound on the device scratch of bc_count(g,
 * p, q) run with opts->waves_per_cu (0 = 12) and scratch_cap_bytes set to
 * that bound (a capped call never takes more; the server admits queries by
 * these estimates and caps each batch at their sum).  Per-root sizes are
 * taken at their bounds over the graph (candidates, row words), for either
 * anchor; the enumeration slabs are charged at most 8 GiB.
 */
bc_status bc_scratch_estimate(const bc_graph *g, uint32_t p, uint32_t q, const bc_opts *opts, uint64_t *bytes);

/*
 * bc_tune_batch -- chooses a schedule for bc_count_batch over the same items
 * (the paper has no batching; this is the batched path's autotuner).  It
 * times bc_count_batch on an evenly spaced sample of the items (every 16th,
 * at least 8) and tunes one option after another, each keeping the value
 * with the shortest sample time (coordinate descent, after one warm-up run):
 * waves_per_cu (12, 8, 4), lds_words (default, 256), roots_per_wave (auto,
 * 2, 4, 16), switch_depth (3, 2) and, when a sampled item has min(p, q) >= 5,
 * split_rows (default, 64, 256, 1024).  When the choice differs from base,
 * both are then timed once over all n items and the faster is kept (a
 * sample has fewer tasks per wavefront than the whole batch, so a schedule
 * can win on the sample and lose on the batch).  *tuned receives base (NULL
 * = defaults) with the chosen values.  No count depends on these options.
 * A sample item that fails (e.g. over base's time limit) counts as taking
 * the whole limit.  Returns argument or device errors.
 */
bc_status bc_tune_batch(const bc_graph *const *graphs, const uint32_t *p, const uint32_t *q, size_t n,
                        const bc_opts *base, bc_opts *tuned);

/*
 * bc_count_noalloc -- bc_count for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  It calls no hipMalloc, hipFree or other allocating routine:
 * every scratch buffer of the call (job table, binomial table, result slot,
 * task queue, candidate counters, bitmap rows, per-wavefront slabs) is carved
 * from one fixed device array of BC_NOALLOC_SCRATCH_BYTES that the library
 * keeps on each device it runs on until the process ends.  The caller passes
 * the graph and receives the count as with bc_count; the grid of the
 * enumeration shrinks to what the remaining scratch can hold.
 *
 * A count whose scratch does not fit fails with BC_E_OOM (bc_last_error says
 * so) and writes nothing.  opts->alloc must be NULL (BC_E_INVALID_ARG
 * otherwise); work runs on opts->stream, or on the null stream when it is
 * NULL, and the call returns once the count is on the host.  All calls on one
 * device share the array, which keeps the last call's contents (whatever must
 * start at zero is cleared by each call): calls that overlapped on one device
 * would race, so the library serialises them with a lock per device.
 */
#define BC_NOALLOC_SCRATCH_BYTES (64ull << 20)
bc_status bc_count_noalloc(const bc_graph *g, uint32_t p, uint32_t q, const bc_opts *opts, bc_u128 *out);

/* Human-readable name of a status code (static storage). */
const char *bc_status_string(bc_status s);

/* Detail of the last error on the calling thread ("" if none). */
const char *bc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BC_H */
