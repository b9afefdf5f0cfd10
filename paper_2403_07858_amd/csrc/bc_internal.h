// Internal entry points shared by the C ABI implementation and the server.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "bc.h"

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

// Admission estimate of the device scratch one count of g may need.
uint64_t estimate_scratch_bytes(const bc_graph *g, uint32_t p, uint32_t q);

int graph_device(const bc_graph *g);

}  // namespace bcint
