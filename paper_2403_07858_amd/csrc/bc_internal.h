// Internal entry points shared by the C ABI implementation and the server.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "bc.h"
#include "bc_server.h"

namespace bcint {

struct Query {
    const bc_graph *g;
    uint32_t p, q;
    uint64_t deadline_ns;   // steady clock; 0 = none
};

// Steady clock in nanoseconds (the clock deadlines use).
uint64_t steady_ns();

// n counts through one batched device pass; per-query status in status[i].
bc_status count_queries(const Query *qs, size_t n, const bc_opts *opts, bc_u128 *out, bc_status *status);

// Admission estimate of the device scratch one count of g at (p, q) takes when
// run with waves_per_cu wavefronts per CU under a cap of that size.
uint64_t estimate_scratch_bytes(const bc_graph *g, uint32_t p, uint32_t q, uint32_t waves_per_cu);

int graph_device(const bc_graph *g);
// Relative time of one (p,q) count on g, from the graph alone (no device
// work): the wedges the candidate pass scans for the cheaper anchor, times 4
// per level of L beyond two and halved per common neighbour asked beyond two.
double query_cost(const bc_graph *g, uint32_t p, uint32_t q);

// What the serving scheduler needs from the device side.  The library uses
// hip_server_backend(); the scheduler itself touches no device API, so it can
// also run against a host-only stand-in (the CPU stress test does).
struct ServerBackend {
    // one batch of counts on `stream` (opts->stream); per-query status and value
    bc_status (*count)(const Query *qs, size_t n, const bc_opts *opts, bc_u128 *out, bc_status *status);
    // admission estimate of the device scratch of one count on waves_per_cu wavefronts per CU
    uint64_t (*estimate)(const bc_graph *g, uint32_t p, uint32_t q, uint32_t waves_per_cu);
    int (*device)(const bc_graph *g);
    // a stream of the worker's own on `device` (NULL if none could be made), and its release
    void *(*stream_create)(int device);
    void (*stream_destroy)(void *stream);
    // default memory budget: half of the device memory free after the caches are trimmed
    uint64_t (*default_budget)();
    // relative time of one count, known before any device work: the queue is
    // served cheapest first (NULL: newest first)
    double (*cost)(const bc_graph *g, uint32_t p, uint32_t q);
};

const ServerBackend *hip_server_backend();

// bc_server_create with an explicit backend.
bc_status server_create(const bc_server_opts *opts, const ServerBackend *backend, bc_server **out);

}  // namespace bcint
