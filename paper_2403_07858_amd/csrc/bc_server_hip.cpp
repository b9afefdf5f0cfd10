// The serving scheduler's device side on HIP (bcint::ServerBackend), and the
// C entry point that creates a server with it.
#include <hip/hip_runtime.h>

#include "bc_internal.h"

namespace {

void *hip_stream_create(int device)
{
    if (hipSetDevice(device) != hipSuccess) return nullptr;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    return s;
}

void hip_stream_destroy(void *s) { (void)hipStreamDestroy((hipStream_t)s); }

uint64_t hip_default_budget()
{
    // memory cached by earlier counts is not in use: give it back first
    int dev = 0;
    hipMemPool_t pool;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceSynchronize() == hipSuccess &&
        hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess)
        (void)hipMemPoolTrimTo(pool, 0);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || free_b == 0) free_b = 8ull << 30;
    return free_b / 2;
}

const bcint::ServerBackend kHipBackend = {
    bcint::count_queries, bcint::estimate_scratch_bytes, bcint::graph_device,
    hip_stream_create,    hip_stream_destroy,            hip_default_budget,
    bcint::query_cost,
};

}  // namespace

const bcint::ServerBackend *bcint::hip_server_backend() { return &kHipBackend; }

extern "C" bc_status bc_server_create(const bc_server_opts *opts, bc_server **out)
{
    return bcint::server_create(opts, &kHipBackend, out);
}
