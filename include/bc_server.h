/*
 * bc_server.h -- a counting service over device-resident graphs.
 *
 * Graphs stay on the device; count queries (graph, p, q) arrive at any time
 * and are answered with the same exact counts bc_count returns.  Admission
 * and batching: pending queries are grouped into batches that run through
 * the batched device path (bc_count_batch).  Up to max_inflight batches run
 * at once, each on its own HIP stream, so queries that arrive while others
 * are on the GPU are admitted as soon as a batch slot and enough of the
 * memory budget are free, and their work overlaps on the device with the
 * batches already running (continuous batching).  The paper has no serving
 * layer; the counting work inside each batch is the one of Algorithm 1.
 *
 * Sharing: each of the max_inflight workers runs its enumeration on its
 * share of the device's wave slots (bc_opts.waves_per_cu), so batches in
 * flight progress together instead of waiting for the GPU in turn.
 *
 * Order: a free batch slot takes the newest pending queries first.  Under
 * overload the oldest would start with little of their deadline left and
 * expire one after another; newest-first keeps answering some queries.
 *
 * Memory admission: each query is charged an estimate of its device scratch
 * (candidate-pass scratch + bitmap rows + enumeration slabs, from the graph's
 * sizes); a batch only starts while the estimates in flight stay within
 * memory_budget_bytes.  A query whose estimate alone exceeds the budget, or
 * that arrives while max_pending queries wait, is refused (BC_E_REJECTED).
 *
 * Deadlines: a query carries an absolute deadline on the steady clock in
 * nanoseconds (0 = none).  A query still waiting at its deadline completes
 * with BC_E_TIMEOUT; one already running is bounded by the device-side
 * time limit of its batch (bc_opts.timeout_ms semantics) and also completes
 * with BC_E_TIMEOUT if that limit is reached.
 *
 * Thread safety: every function may be called from any thread.  The server
 * does not own the graphs; they must outlive it.
 */
#ifndef BC_SERVER_H
#define BC_SERVER_H

#include "bc.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bc_server bc_server;

typedef struct {
    uint32_t struct_size;          /* sizeof(bc_server_opts) */
    uint32_t max_inflight;         /* concurrent batches on the device (streams); 0 = 2 */
    uint32_t max_batch;            /* queries per batch; 0 = 256 */
    uint32_t max_pending;          /* waiting queries before new ones are refused; 0 = 65536 */
    uint64_t memory_budget_bytes;  /* admission budget; 0 = half of the free device memory */
    uint32_t batch_timeout_ms;     /* device-side time limit per batch; 0 = none */
    uint32_t pad;
} bc_server_opts;

typedef struct {
    double queue_ms;      /* submit -> batch start */
    double run_ms;        /* batch start -> result */
    double total_ms;      /* submit -> result */
    uint64_t batch_id;    /* batch the query ran in */
    uint32_t batch_size;  /* queries in that batch */
    uint32_t pad;
} bc_query_stats;

typedef struct {
    uint64_t submitted, completed, rejected, timed_out, failed, batches;
    double p50_ms, p99_ms, mean_ms;   /* latency (submit -> result) of completed queries */
    double qps;                       /* completed queries per second since creation */
    double mean_batch;                /* mean queries per batch */
    uint32_t max_overlap;             /* most batches seen in flight at once */
    uint32_t pad;
} bc_server_summary;

bc_status bc_server_create(const bc_server_opts *opts, bc_server **out);

/* Registers a built graph; *graph_id receives its id (0, 1, ...). */
bc_status bc_server_add_graph(bc_server *s, const bc_graph *g, uint32_t *graph_id);

/* Queues one count.  *ticket identifies it for bc_server_poll. */
bc_status bc_server_submit(bc_server *s, uint32_t graph_id, uint32_t p, uint32_t q,
                           uint64_t deadline_ns, uint64_t *ticket);

/*
 * Result of a ticket.  block != 0 waits for it.  Returns the query's own
 * status (BC_OK, BC_E_TIMEOUT, BC_E_OVERFLOW, ...), or BC_E_PENDING when
 * block == 0 and it is not done, or BC_E_NOT_FOUND for an unknown ticket.
 * A ticket can be read once: it is released when its final status is
 * returned.
 */
bc_status bc_server_poll(bc_server *s, uint64_t ticket, int block, bc_u128 *out, bc_query_stats *st);

/* Counters and latency percentiles so far. */
bc_status bc_server_stats(bc_server *s, bc_server_summary *out);

/* Current value of the clock deadlines are measured on (steady, ns). */
uint64_t bc_server_now_ns(void);

/* Stops the workers; queries not yet started complete with BC_E_CANCELLED. */
void bc_server_destroy(bc_server *s);

#ifdef __cplusplus
}
#endif

#endif /* BC_SERVER_H */
