// Microbenchmarks of the two on-chip rates the enumeration is measured
// against: LDS read bandwidth and 32-bit integer VALU issue rate, on every
// CU of the device at once.  Each kernel runs many blocks of independent
// work whose result is kept only under a condition the host never makes
// true, so that no load or operation can be dropped by the compiler.
#include "bc_peaks.h"

#include <hip/hip_runtime.h>

namespace {

constexpr int kThreads = 256;
constexpr uint32_t kLdsVec = 2048;   // 16-byte elements: 32 KiB of LDS per block
constexpr int kLdsUnroll = 16;

// Every thread reads 16 bytes 16 times per step (ds_read_b128) at 16
// distinct addresses; lanes of a wave read consecutive elements (no bank
// conflicts); the start index moves by a whole wave each step.
__global__ __launch_bounds__(kThreads) void k_lds_read(uint32_t iters, uint32_t never, uint4 *sink)
{
    __shared__ uint4 buf[kLdsVec];
    const uint32_t t = threadIdx.x;
    for (uint32_t i = t; i < kLdsVec; i += kThreads) buf[i] = make_uint4(i, i * 3u, i * 5u, i * 7u);
    __syncthreads();
    uint4 acc = make_uint4(0, 0, 0, 0);
    uint32_t base = t;
    for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < kLdsUnroll; ++u) {
            const uint4 v = buf[(base + (uint32_t)u * (kLdsVec / kLdsUnroll)) & (kLdsVec - 1)];
            acc.x += v.x;
            acc.y ^= v.y;
            acc.z += v.z;
            acc.w ^= v.w;
        }
        base = (base + 64u) & (kLdsVec - 1);
    }
    if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == never) sink[blockIdx.x * kThreads + t] = acc;
}

// Eight independent chains of v_and_b32 and v_bcnt_u32_b32 (popcount plus
// accumulate): 16 integer VALU instructions per step and lane, written in
// one asm block so that the count is exact.
__global__ __launch_bounds__(kThreads) void k_valu_int(uint32_t iters, uint32_t seed, uint32_t never,
                                                        uint32_t *sink)
{
    const uint32_t t = blockIdx.x * kThreads + threadIdx.x;
    uint32_t a0 = t ^ seed, a1 = t * 3u, a2 = t * 5u, a3 = t * 7u, a4 = t * 11u, a5 = t * 13u, a6 = t * 17u,
             a7 = t * 19u;
    const uint32_t m = seed | 0x5bd1e995u;
    for (uint32_t it = 0; it < iters; ++it) {
        asm volatile(
            "v_and_b32 %0, %0, %8\n\t"
            "v_and_b32 %1, %1, %8\n\t"
            "v_and_b32 %2, %2, %8\n\t"
            "v_and_b32 %3, %3, %8\n\t"
            "v_and_b32 %4, %4, %8\n\t"
            "v_and_b32 %5, %5, %8\n\t"
            "v_and_b32 %6, %6, %8\n\t"
            "v_and_b32 %7, %7, %8\n\t"
            "v_bcnt_u32_b32 %0, %0, %1\n\t"
            "v_bcnt_u32_b32 %1, %1, %2\n\t"
            "v_bcnt_u32_b32 %2, %2, %3\n\t"
            "v_bcnt_u32_b32 %3, %3, %4\n\t"
            "v_bcnt_u32_b32 %4, %4, %5\n\t"
            "v_bcnt_u32_b32 %5, %5, %6\n\t"
            "v_bcnt_u32_b32 %6, %6, %7\n\t"
            "v_bcnt_u32_b32 %7, %7, %0\n\t"
            : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
            : "v"(m));
    }
    const uint32_t r = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
    if (r == never) sink[t] = r;
}

struct Timed {
    hipEvent_t a = nullptr, b = nullptr;
    Timed()
    {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~Timed()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

int blocks_for(int per_cu)
{
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
        ncu = 256;
    return ncu * per_cu;
}

}  // namespace

extern "C" int bc_peak_lds(uint32_t iters, double *bytes_per_s, double *ms)
{
    if (!bytes_per_s || !ms || iters == 0) return (int)hipErrorInvalidValue;
    const int blocks = blocks_for(32);   // 5 resident per CU (LDS bound): several waves of blocks
    void *sink = nullptr;
    hipError_t e = hipMalloc(&sink, (size_t)blocks * kThreads * sizeof(uint4));
    if (e != hipSuccess) return (int)e;
    Timed tm;
    // warm-up launch, then the timed one
    hipLaunchKernelGGL(k_lds_read, dim3(blocks), dim3(kThreads), 0, nullptr, 1u, 0xfeedf00du, (uint4 *)sink);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(tm.a, nullptr);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_lds_read, dim3(blocks), dim3(kThreads), 0, nullptr, iters, 0xfeedf00du, (uint4 *)sink);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(tm.b, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(tm.b);
    float f = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, tm.a, tm.b);
    (void)hipFree(sink);
    if (e != hipSuccess) return (int)e;
    *ms = f;
    *bytes_per_s = (double)blocks * kThreads * (double)iters * kLdsUnroll * 16.0 / (f * 1e-3);
    return 0;
}

extern "C" int bc_peak_valu_int(uint32_t iters, double *ops_per_s, double *ms)
{
    if (!ops_per_s || !ms || iters == 0) return (int)hipErrorInvalidValue;
    const int blocks = blocks_for(64);
    void *sink = nullptr;
    hipError_t e = hipMalloc(&sink, (size_t)blocks * kThreads * sizeof(uint32_t));
    if (e != hipSuccess) return (int)e;
    Timed tm;
    hipLaunchKernelGGL(k_valu_int, dim3(blocks), dim3(kThreads), 0, nullptr, 1u, 12345u, 0xfeedf00du,
                       (uint32_t *)sink);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(tm.a, nullptr);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_valu_int, dim3(blocks), dim3(kThreads), 0, nullptr, iters, 12345u, 0xfeedf00du,
                           (uint32_t *)sink);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(tm.b, nullptr);
    if (e == hipSuccess) e = hipEventSynchronize(tm.b);
    float f = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&f, tm.a, tm.b);
    (void)hipFree(sink);
    if (e != hipSuccess) return (int)e;
    *ms = f;
    *ops_per_s = (double)blocks * kThreads * (double)iters * 16.0 / (f * 1e-3);
    return 0;
}
