// HIP kernels of the (p,q)-biclique counter for CDNA4 (gfx950, wave64).
//
// The search follows Algorithm 1 (GBC) restated for this hardware:
//   k_root_build  per root u: oriented 2-hop candidates w > u sharing at least
//                 qA neighbours with u (N_2^q(u) of Section II-A with the
//                 vertex-priority orientation of Section III-B), and one
//                 bitmap row per candidate over the neighbours of u (column
//                 d(u) - 1 - j set when the j-th neighbour of u is also a
//                 neighbour of w) -- a truncated bitmap in the spirit of the
//                 HTB of Section V-A, dense over the root's own neighbourhood.
//                 For pA == 2 the leaves C(|N(u) n N(w)|, qA) are summed
//                 right here.  k_cand_count + k_rows_build do the same in two
//                 kernels with global counters (fallback).
//   k_enumerate   persistent wavefronts pop (root, second vertex) tasks -- the
//                 edge-oriented pre-runtime split of Section V-C -- from one
//                 device queue (runtime balancing, Section V-C), compact the
//                 rows to the common neighbours of the two vertices, then run
//                 the hybrid DFS-BFS of Section IV: DFS over levels, all
//                 siblings of a node intersected at once by the 64 lanes
//                 (AND + popcount), and the last two levels fused into one
//                 pairwise sum of C(|S|, q) (leaf rule of Section III-A) whose
//                 intersection sizes come from the matrix cores.
#include "bc_device.h"

#include <type_traits>

namespace bcdev {

constexpr uint32_t kLdsWordsPerWave = 960;    // LDS arena per wavefront (64-bit words): with the spread table,
                                              // 3 blocks of 4 waves fill 160 KiB
constexpr uint32_t kTileWords = 4;            // widest row (64-bit words) of the tiled leaf sum
constexpr uint32_t kTableLen = 64 * kTileWords + 4;   // per-wave LDS copy of C(n, q), n < kTableLen
constexpr uint32_t kStackWords = 128;         // DFS stack at the start of each wave's LDS
constexpr uint32_t kFilterDepth = 4;          // 64-row chunks loaded at once by the level-2 filter


uint32_t max_lds_words_per_wave() { return kLdsWordsPerWave; }

// ---------------------------------------------------------------------------
// Wave-level helpers.

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWaveSize - 1); }

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint32_t bcast32(uint32_t v, int src) { return __shfl(v, src); }

__device__ __forceinline__ uint64_t bcast64(uint64_t v, int src)
{
    uint32_t lo = __shfl((uint32_t)v, src), hi = __shfl((uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// Orders this wave's earlier LDS / global writes before its later reads.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v)
{
    const uint32_t ln = lane_id();
#pragma unroll
    for (int off = 1; off < kWaveSize; off <<= 1) {
        uint32_t t = __shfl_up(v, off);
        if (ln >= (uint32_t)off) v += t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v)
{
#pragma unroll
    for (int off = kWaveSize / 2; off > 0; off >>= 1) {
        uint32_t lo = __shfl_xor((uint32_t)v, off), hi = __shfl_xor((uint32_t)(v >> 32), off);
        v += ((uint64_t)hi << 32) | lo;
    }
    return v;
}

// Exact wave-wide sum of per-lane u128 values; *ovf is set if the sum does
// not fit in 128 bits.  Returned in every lane.
__device__ u128 wave_sum_u128(u128 v, bool *ovf)
{
    uint64_t l0 = (uint64_t)(v & 0xffffffffu), l1 = (uint64_t)((v >> 32) & 0xffffffffu);
    uint64_t l2 = (uint64_t)((v >> 64) & 0xffffffffu), l3 = (uint64_t)(v >> 96);
    l0 = wave_sum_u64(l0);
    l1 = wave_sum_u64(l1);
    l2 = wave_sum_u64(l2);
    l3 = wave_sum_u64(l3);
    // each limb sum < 2^38
    bool o = (l3 >> 32) != 0;
    u128 t = (u128)l0;
    o |= __builtin_add_overflow(t, (u128)l1 << 32, &t);
    o |= __builtin_add_overflow(t, (u128)l2 << 64, &t);
    o |= __builtin_add_overflow(t, (u128)(l3 & 0xffffffffu) << 96, &t);
    *ovf = o;
    return t;
}

// Adds v into a result slot with two 64-bit atomics; the carry out of the
// low limb goes into the high limb, a carry out of the high limb is overflow.
__device__ void slot_add(Slot *s, u128 v, bool ovf)
{
    const uint64_t lo = (uint64_t)v, hi = (uint64_t)(v >> 64);
    bool over = ovf;
    uint64_t add_hi = hi;
    if (lo) {
        unsigned long long old = atomicAdd(&s->lo, (unsigned long long)lo);
        if ((uint64_t)old + lo < (uint64_t)old) {
            add_hi += 1;
            if (add_hi == 0) over = true;
        }
    }
    if (add_hi) {
        unsigned long long old = atomicAdd(&s->hi, (unsigned long long)add_hi);
        if ((uint64_t)old + add_hi < (uint64_t)old) over = true;
    }
    if (over) atomicOr(&s->flags, FLAG_OVERFLOW);
}

// Wave-uniform flush of per-lane accumulators into a slot.
__device__ void wave_flush(Slot *slots, uint32_t slot, u128 acc, bool ovf,
                           unsigned long long pair_ops, unsigned long long filter_ops)
{
    bool o = false;
    u128 tot = wave_sum_u128(acc, &o);
    uint64_t any_ovf = __ballot(ovf);
    if (lane_id() == 0) {
        slot_add(&slots[slot], tot, o || any_ovf != 0);
        if (pair_ops) atomicAdd(&slots[slot].pair_ops, pair_ops);
        if (filter_ops) atomicAdd(&slots[slot].filter_ops, filter_ops);
    }
}

// True once the device real-time clock has passed a nonzero deadline.
// Adds v to vertex x's per-vertex count (two 64-bit atomics; the carry out of
// the low word goes into the high one).  A count never exceeds the query's
// total, which the result slot checks for overflow.
__device__ __forceinline__ void pv_add(uint64_t *pv, uint32_t x, u128 v)
{
    unsigned long long *c = (unsigned long long *)(pv + 2ull * x);
    const uint64_t lo = (uint64_t)v;
    uint64_t hi = (uint64_t)(v >> 64);
    if (lo) {
        const unsigned long long old = atomicAdd(&c[0], (unsigned long long)lo);
        if ((uint64_t)old + lo < (uint64_t)old) hi += 1;
    }
    if (hi) atomicAdd(&c[1], (unsigned long long)hi);
}

__device__ __forceinline__ bool past_deadline(uint64_t deadline)
{
    if (deadline == 0) return false;
    const uint64_t now = __builtin_amdgcn_s_memrealtime();
    // wave-uniform by construction (scalar clock read); make it explicit
    return __builtin_amdgcn_readfirstlane((uint32_t)(now > deadline)) != 0u;
}

__global__ void k_read_clock(uint64_t *out)
{
    if (threadIdx.x == 0) out[0] = __builtin_amdgcn_s_memrealtime();
}

hipError_t launch_read_clock(uint64_t *out, hipStream_t stream)
{
    hipLaunchKernelGGL(k_read_clock, dim3(1), dim3(64), 0, stream, out);
    return hipGetLastError();
}

// Largest j in [0, n) with prefix[j] <= x (prefix nondecreasing, prefix[0] == 0).
__device__ __forceinline__ uint32_t find_segment(const uint64_t *prefix, uint32_t n, uint64_t x)
{
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Slots.

__global__ void k_fill_slots(Slot *slots, uint32_t n)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        slots[i].lo = 0;
        slots[i].hi = 0;
        slots[i].flags = 0;
        slots[i].pad = 0;
        slots[i].pair_ops = 0;
        slots[i].filter_ops = 0;
        slots[i].cyc_setup = 0;
        slots[i].cyc_compact = 0;
        slots[i].cyc_pair = 0;
        slots[i].cyc_filter = 0;
        slots[i].pairs = 0;
        slots[i].pair_slots = 0;
        slots[i].cyc_pack = 0;
        slots[i].pad3 = 0;
    }
}

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t stream)
{
    if (!n) return hipSuccess;
    const uint64_t blocks = min((n + 255) / 256, (uint64_t)4096);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_slots(Slot *slots, uint32_t n, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_slots, dim3((n + 255) / 256), dim3(256), 0, stream, slots, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// pA == 1: every root alone is an L; the count is sum_u C(d(u), qA).

__global__ __launch_bounds__(kBlockThreads) void k_degree_sum(const Job *jobs, const uint32_t *job_ids,
                                                              Slot *slots)
{
    const Job jb = jobs[job_ids[blockIdx.y]];
    u128 acc = 0;
    bool ovf = false;
    for (uint64_t u = (uint64_t)jb.root_lo + blockIdx.x * blockDim.x + threadIdx.x; u < jb.root_hi;
         u += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t d = (uint32_t)(jb.ptrA[u + 1] - jb.ptrA[u]);
        if (d >= jb.qA) {
            if (d >= jb.n_ovf) ovf = true;
            else ovf |= __builtin_add_overflow(acc, jb.binom[d], &acc);
        }
    }
    wave_flush(slots, jb.slot, acc, ovf, 0, 0);
}

hipError_t launch_degree_sum(const Job *jobs, const uint32_t *job_ids, uint32_t n_jobs, Slot *slots,
                             hipStream_t stream)
{
    if (n_jobs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_degree_sum, dim3(64, n_jobs), dim3(kBlockThreads), 0, stream, jobs, job_ids, slots);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Wedge scan shared by the two-kernel per-root path: for every neighbour v_j
// of u and every w in N(v_j) with w > u, call f(c, w), where c = d(u) - 1 - j
// is v_j's column (bit position) in the root's rows: the highest-ranked
// neighbours, which most candidates share, take the first word, so common
// neighbourhoods tend to need no bit-packing.  Waves take the j's round
// robin; lanes stride over the oriented part of N(v_j), which starts right
// after u (its position within N(v_j) is stored per edge).
template <typename F>
__device__ __forceinline__ void oriented_wedges(const Job &jb, uint32_t u, uint64_t ub, uint32_t du, F f)
{
    const uint32_t wv = threadIdx.x / kWaveSize, ln = lane_id();
    for (uint32_t j = wv; j < du; j += kWavesPerBlock) {
        const uint32_t v = jb.adjA[ub + j];
        const uint64_t s = jb.ptrB[v] + jb.rposA[ub + j] + 1, ve = jb.ptrB[v + 1];
        for (uint64_t x = s + ln; x < ve; x += kWaveSize) f(du - 1 - j, jb.adjB[x]);
    }
}

// The same wedges (and columns) spread evenly over the NW waves of a block.  The
// neighbours of u are taken 64 at a time, one per lane; a wave scan lays the
// 64 oriented parts of their rows end to end, and the waves take 64-element
// windows of that concatenation round robin, two windows per step.  Each lane
// finds the part holding its element by a binary search over the lanes'
// exclusive offsets.
template <int NW, typename F>
__device__ __forceinline__ void wedges_flat(const Job &jb, uint64_t ub, uint32_t du, F f)
{
    const uint32_t wv = threadIdx.x / kWaveSize, ln = lane_id();
    for (uint32_t j0 = 0; j0 < du; j0 += kWaveSize) {
        const uint32_t j = j0 + ln;
        uint64_t s = 0;
        uint32_t len = 0;
        if (j < du) {
            const uint32_t v = jb.adjA[ub + j];
            s = jb.ptrB[v] + jb.rposA[ub + j] + 1;
            len = (uint32_t)(jb.ptrB[v + 1] - s);
        }
        const uint32_t inc = wave_inclusive_scan(len);
        const uint32_t excl = inc - len;
        const uint64_t base = s - excl;   // element x of this lane's part is adjB[base + x] (mod 2^64)
        const uint32_t total = __shfl(inc, kWaveSize - 1);
        for (uint32_t x0 = wv * kWaveSize; x0 < total; x0 += 2 * NW * kWaveSize) {
            const uint32_t xa = x0 + ln, xb = xa + NW * kWaveSize;
            uint32_t la = 0, lb = 0;
#pragma unroll
            for (uint32_t b = 32; b; b >>= 1) {
                // la + b <= 63: the larger steps already taken add up to at most 64 - 2b
                if (__shfl(excl, (int)(la + b)) <= xa) la += b;
                if (__shfl(excl, (int)(lb + b)) <= xb) lb += b;
            }
            const uint64_t pa = bcast64(base, (int)la) + xa, pb = bcast64(base, (int)lb) + xb;
            uint32_t wa = 0, wb = 0;
            if (xa < total) wa = jb.adjB[pa];
            if (xb < total) wb = jb.adjB[pb];
            if (xa < total) f(du - 1 - (j0 + la), wa);
            if (xb < total) f(du - 1 - (j0 + lb), wb);
        }
    }
}

// wedges_flat that stops early once *over is raised (by f or another wave).
// With Count, f returns true when its wedge claimed a new table slot; each
// wave adds its claims per step, and once the block total passes cap the
// waves raise *over (the caller then discards the table).
template <int NW, bool Count, typename F>
__device__ __forceinline__ void wedges_flat_capped(const Job &jb, uint64_t ub, uint32_t du, uint32_t cap,
                                                   uint32_t *claimed, volatile uint32_t *over, F f)
{
    const uint32_t wv = threadIdx.x / kWaveSize, ln = lane_id();
    for (uint32_t j0 = 0; j0 < du; j0 += kWaveSize) {
        const uint32_t j = j0 + ln;
        uint64_t s = 0;
        uint32_t len = 0;
        if (j < du) {
            const uint32_t v = jb.adjA[ub + j];
            s = jb.ptrB[v] + jb.rposA[ub + j] + 1;
            len = (uint32_t)(jb.ptrB[v + 1] - s);
        }
        const uint32_t inc = wave_inclusive_scan(len);
        const uint32_t excl = inc - len;
        const uint64_t base = s - excl;
        const uint32_t total = __shfl(inc, kWaveSize - 1);
        for (uint32_t x0 = wv * kWaveSize; x0 < total; x0 += 2 * NW * kWaveSize) {
            const uint32_t xa = x0 + ln, xb = xa + NW * kWaveSize;
            uint32_t la = 0, lb = 0;
#pragma unroll
            for (uint32_t b = 32; b; b >>= 1) {
                if (__shfl(excl, (int)(la + b)) <= xa) la += b;
                if (__shfl(excl, (int)(lb + b)) <= xb) lb += b;
            }
            const uint64_t pa = bcast64(base, (int)la) + xa, pb = bcast64(base, (int)lb) + xb;
            uint32_t wa = 0, wb = 0;
            if (xa < total) wa = jb.adjB[pa];
            if (xb < total) wb = jb.adjB[pb];
            bool na = false, nb = false;
            if (xa < total) na = f(du - 1 - (j0 + la), wa);
            if (xb < total) nb = f(du - 1 - (j0 + lb), wb);
            if constexpr (Count) {
                const uint32_t nn = (uint32_t)__popcll(__ballot(na)) + (uint32_t)__popcll(__ballot(nb));
                uint32_t tot = 0;
                if (nn) {
                    if (ln == 0) tot = atomicAdd(claimed, nn) + nn;
                    tot = __shfl(tot, 0);
                    if (tot > cap && ln == 0) *over = 1u;
                }
            }
            if (*over) return;
        }
    }
}

// k_cand_count: for every root of every job, k(u) = #{w > u : |N(u) n N(w)| >= qA}.
// Common-neighbour counts live in a per-block dense counter array (all zero
// between roots); the ids touched are listed so that only they are reset.
__global__ __launch_bounds__(kBlockThreads) void k_cand_count(const Job *jobs, const uint64_t *job_root_prefix,
                                                              uint32_t n_jobs, uint64_t total_roots,
                                                              RootScratch sc, unsigned long long *queue,
                                                              uint32_t *out_k, Slot *slots)
{
    __shared__ unsigned long long s_item;
    __shared__ uint32_t s_nt, s_k, s_late;
    uint32_t *cnt = sc.cnt + (uint64_t)blockIdx.x * sc.stride;
    uint32_t *touched = sc.touched + (uint64_t)blockIdx.x * sc.stride;
    const uint32_t tid = threadIdx.x;
    u128 acc = 0;
    bool ovf = false;
    uint32_t cur_job = 0xffffffffu;
    for (;;) {
        if (tid == 0) {
            s_item = atomicAdd(queue, 1ull);
            s_nt = 0;
            s_k = 0;
        }
        __syncthreads();
        const uint64_t item = s_item;
        if (item >= total_roots) break;
        const uint32_t j = find_segment(job_root_prefix, n_jobs, item);
        if (j != cur_job) {
            if (cur_job != 0xffffffffu) wave_flush(slots, jobs[cur_job].slot, acc, ovf, 0, 0);
            acc = 0;
            ovf = false;
            cur_job = j;
        }
        const Job jb = jobs[j];
        const uint32_t u = jb.root_lo + (uint32_t)(item - job_root_prefix[j]);
        const uint64_t ub = jb.ptrA[u];
        const uint32_t du = (uint32_t)(jb.ptrA[u + 1] - ub);
        uint32_t k = 0;
        // one thread reads the clock so that the whole block takes the same branch
        if (tid == 0) {
            s_late = past_deadline(jb.deadline) ? 1u : 0u;
            if (s_late) atomicOr(&slots[jb.slot].flags, FLAG_TIMEOUT);
        }
        __syncthreads();
        const bool late = s_late != 0;
        if (du >= jb.qA && !late) {
            oriented_wedges(jb, u, ub, du, [&](uint32_t, uint32_t w) {
                if (atomicAdd(&cnt[w], 1u) == 0u) touched[atomicAdd(&s_nt, 1u)] = w;
            });
            __syncthreads();
            const uint32_t nt = s_nt;
            for (uint32_t t = tid; t < nt; t += kBlockThreads) {
                const uint32_t w = touched[t];
                const uint32_t c = atomicExch(&cnt[w], 0u);
                if (c >= jb.qA) {
                    atomicAdd(&s_k, 1u);
                    if (jb.pA == 2) {
                        if (c >= jb.n_ovf) ovf = true;
                        else ovf |= __builtin_add_overflow(acc, jb.binom[c], &acc);
                    }
                }
            }
            __syncthreads();
            k = s_k;
        }
        if (tid == 0) out_k[item] = k;
        __syncthreads();
    }
    if (cur_job != 0xffffffffu) wave_flush(slots, jobs[cur_job].slot, acc, ovf, 0, 0);
}

hipError_t launch_cand_count(const Job *jobs, const uint64_t *job_root_prefix, uint32_t n_jobs,
                             uint64_t total_roots, RootScratch scratch, uint32_t n_blocks,
                             unsigned long long *queue, uint32_t *out_k, Slot *slots, hipStream_t stream)
{
    if (total_roots == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cand_count, dim3(n_blocks), dim3(kBlockThreads), 0, stream, jobs, job_root_prefix,
                       n_jobs, total_roots, scratch, queue, out_k, slots);
    return hipGetLastError();
}

// Block-wide bitonic sort of s[0, n) ascending by a block of NT threads;
// pads to a power of two, so s must hold that many entries.
template <int NT>
__device__ void block_sort_u32(uint32_t *s, uint32_t n)
{
    uint32_t n2 = 1;
    while (n2 < n) n2 <<= 1;
    for (uint32_t i = n + threadIdx.x; i < n2; i += NT) s[i] = 0xffffffffu;
    __syncthreads();
    for (uint32_t size = 2; size <= n2; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t pr = threadIdx.x; pr < (n2 >> 1); pr += NT) {
                const uint32_t i = 2 * stride * (pr / stride) + (pr % stride);
                const uint32_t l = i + stride;
                const bool asc = (i & size) == 0;
                const uint32_t a = s[i], b = s[l];
                if ((a > b) == asc) {
                    s[i] = b;
                    s[l] = a;
                }
            }
            __syncthreads();
        }
    }
}

// k_rows_build: candidate rows of every active root, column-major in the pool
// (word w of row s at pool[off + w*k + s]), rows in increasing rank order of
// the candidates whenever k <= kSortCap.
__global__ __launch_bounds__(kBlockThreads) void k_rows_build(const Job *jobs, const ActiveRoot *roots,
                                                              uint32_t n_roots, uint64_t *pool,
                                                              RootScratch sc, unsigned long long *queue,
                                                              Slot *slots)
{
    __shared__ unsigned long long s_item;
    __shared__ uint32_t s_nt, s_k, s_late;
    __shared__ uint32_t s_cand[kSortCap];
    uint32_t *cnt = sc.cnt + (uint64_t)blockIdx.x * sc.stride;
    uint32_t *touched = sc.touched + (uint64_t)blockIdx.x * sc.stride;
    uint32_t *cand_g = sc.cand + (uint64_t)blockIdx.x * sc.stride;
    const uint32_t tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            s_item = atomicAdd(queue, 1ull);
            s_nt = 0;
            s_k = 0;
        }
        __syncthreads();
        const uint64_t item = s_item;
        if (item >= n_roots) break;
        const ActiveRoot ar = roots[item];
        const Job jb = jobs[ar.job];
        // one thread reads the clock so that the whole block takes the same branch
        if (tid == 0) {
            s_late = past_deadline(jb.deadline) ? 1u : 0u;
            if (s_late) atomicOr(&slots[jb.slot].flags, FLAG_TIMEOUT);
        }
        __syncthreads();
        if (s_late) {
            // rows stay unwritten; the enumeration sees the same passed deadline
            __syncthreads();
            continue;
        }
        const uint32_t u = ar.root;
        const uint64_t ub = jb.ptrA[u];
        const uint32_t du = (uint32_t)(jb.ptrA[u + 1] - ub);
        const uint32_t W1 = (du + 63) >> 6;
        const uint32_t kexp = ar.k;
        uint64_t *base = pool + ar.pool_off;

        oriented_wedges(jb, u, ub, du, [&](uint32_t, uint32_t w) {
            if (atomicAdd(&cnt[w], 1u) == 0u) touched[atomicAdd(&s_nt, 1u)] = w;
        });
        __syncthreads();
        const uint32_t nt = s_nt;
        const bool in_lds = kexp <= (uint32_t)kSortCap;
        uint32_t *cand = in_lds ? s_cand : cand_g;
        for (uint32_t t = tid; t < nt; t += kBlockThreads) {
            const uint32_t w = touched[t];
            const uint32_t c = atomicAdd(&cnt[w], 0u);
            if (c >= jb.qA) {
                const uint32_t s = atomicAdd(&s_k, 1u);
                if (s < kexp) cand[s] = w;
            } else {
                atomicExch(&cnt[w], 0u);
            }
        }
        __syncthreads();
        const uint32_t k = s_k;
        if (k != kexp) {
            // Cannot happen unless the two wedge passes disagree; leave the
            // scratch clean and report.
            for (uint32_t t = tid; t < nt; t += kBlockThreads) atomicExch(&cnt[touched[t]], 0u);
            if (tid == 0) atomicOr(&slots[jb.slot].flags, FLAG_MISMATCH);
            __syncthreads();
            continue;
        }
        if (in_lds) block_sort_u32<kBlockThreads>(s_cand, k);
        __syncthreads();
        for (uint32_t s = tid; s < k; s += kBlockThreads) atomicExch(&cnt[cand[s]], kSlotFlag | s);
        const uint64_t words = (uint64_t)k * W1;
        for (uint64_t x = tid; x < words; x += kBlockThreads) base[x] = 0;
        __threadfence();
        __syncthreads();
        oriented_wedges(jb, u, ub, du, [&](uint32_t j, uint32_t w) {
            const uint32_t e = atomicAdd(&cnt[w], 0u);
            if (e & kSlotFlag) {
                const uint32_t s = e & ~kSlotFlag;
                atomicOr((unsigned long long *)&base[(uint64_t)(j >> 6) * k + s], 1ull << (j & 63));
            }
        });
        __syncthreads();
        for (uint32_t s = tid; s < k; s += kBlockThreads) atomicExch(&cnt[cand[s]], 0u);
        __syncthreads();
    }
}

hipError_t launch_rows_build(const Job *jobs, const ActiveRoot *roots, uint32_t n_roots, uint64_t *pool,
                             RootScratch scratch, uint32_t n_blocks, unsigned long long *queue, Slot *slots,
                             hipStream_t stream)
{
    if (n_roots == 0) return hipSuccess;
    hipLaunchKernelGGL(k_rows_build, dim3(n_blocks), dim3(kBlockThreads), 0, stream, jobs, roots, n_roots,
                       pool, scratch, queue, slots);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_root_build: the candidate count and the candidate rows of every root in
// one kernel, one root per block of kRbWaves waves at a time.
//
// The 2-hop vertices of u live in an LDS open-addressing table (key w + 1,
// linear probing).  When u has at most 64 neighbours (one row word), the
// table entry accumulates w's row itself -- v_j's column set for the wedge
// u - v_j - w -- so one wedge pass yields both |N(u) n N(w)| (the popcount)
// and the row.
// Wider roots count in the first pass, index their candidates, and set the
// row bits in a second pass into LDS (or the pool when the rows do not fit).
// Roots whose 2-hop set overflows the table fall back to the per-block dense
// counter array in HBM.  Row storage is taken from the pool with one atomic
// bump per root, so counting and row building need no host round trip.

constexpr uint32_t kHashSlots = 8192;       // LDS table entries
constexpr uint32_t kHashProbes = 128;       // longest probe sequence before falling back
constexpr uint32_t kSlotsPerThread = kHashSlots / kRbThreads;
constexpr uint16_t kNoRow = 0xffffu;
constexpr uint32_t kHintDistinct = 8192;    // 2-hop vertices above which the next root starts with id ranges
constexpr uint32_t kCapRange = 5120;        // distinct 2-hop vertices of one id range
constexpr uint32_t kRowsCap = 4096;         // candidates of a root counted by id ranges

__device__ __forceinline__ uint32_t hash_slot(uint32_t w) { return (w * 0x9E3779B1u) >> (32 - 13); }

// Slot of w, inserting it if new; -1 when the probe limit is reached.
__device__ __forceinline__ int hash_insert(uint32_t *key, uint32_t w)
{
    const uint32_t kv = w + 1u;
    uint32_t h = hash_slot(w);
    for (uint32_t p = 0; p < kHashProbes; ++p, h = (h + 1) & (kHashSlots - 1)) {
        const uint32_t e = key[h];
        if (e == kv) return (int)h;
        if (e == 0u) {
            const uint32_t old = atomicCAS(&key[h], 0u, kv);
            if (old == 0u || old == kv) return (int)h;
        }
    }
    return -1;
}

// As hash_insert; *fresh tells whether this call claimed the slot.
__device__ __forceinline__ int hash_insert_new(uint32_t *key, uint32_t w, bool *fresh)
{
    const uint32_t kv = w + 1u;
    uint32_t h = hash_slot(w);
    *fresh = false;
    for (uint32_t p = 0; p < kHashProbes; ++p, h = (h + 1) & (kHashSlots - 1)) {
        const uint32_t e = key[h];
        if (e == kv) return (int)h;
        if (e == 0u) {
            const uint32_t old = atomicCAS(&key[h], 0u, kv);
            if (old == 0u) {
                *fresh = true;
                return (int)h;
            }
            if (old == kv) return (int)h;
        }
    }
    return -1;
}

// Slot of w, or -1 when w is absent (the table must have an empty slot).
__device__ __forceinline__ int hash_lookup(const uint32_t *key, uint32_t w)
{
    const uint32_t kv = w + 1u;
    uint32_t h = hash_slot(w);
    for (;;) {
        const uint32_t e = key[h];
        if (e == kv) return (int)h;
        if (e == 0u) return -1;
        h = (h + 1) & (kHashSlots - 1);
    }
}

// Slot of w (w must be present).
__device__ __forceinline__ uint32_t hash_find(const uint32_t *key, uint32_t w)
{
    const uint32_t kv = w + 1u;
    uint32_t h = hash_slot(w);
    while (key[h] != kv) h = (h + 1) & (kHashSlots - 1);
    return h;
}

// Exclusive prefix of v over the block (thread order); *total gets the sum.
// Uses s_wsum[kRbWaves]; the caller separates consecutive uses by a barrier.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_wsum, uint32_t *total)
{
    const uint32_t wv = threadIdx.x / kWaveSize;
    const uint32_t inc = wave_inclusive_scan(v);
    if (lane_id() == kWaveSize - 1) s_wsum[wv] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (uint32_t w = 0; w < (uint32_t)kRbWaves; ++w) {
        const uint32_t t = s_wsum[w];
        before += w < wv ? t : 0u;
        tot += t;
    }
    *total = tot;
    return before + inc - v;
}

// PV: per-vertex counts for p_A = 2 jobs that ask for them (each leaf {u, w}
// adds its C(|N(u) n N(w)|, q_A) to w at once and, summed per wave, to u).
template <bool PV>
__global__ __launch_bounds__(kRbThreads) void k_root_build(const Job *jobs, const uint64_t *job_root_prefix,
                                                           uint32_t n_jobs, uint64_t total_roots, RootScratch sc,
                                                           uint64_t *pool, uint64_t pool_cap,
                                                           unsigned long long *counters, uint32_t *out_k,
                                                           uint64_t *out_off, Slot *slots)
{
    __shared__ uint32_t s_key[kHashSlots];               // w + 1, 0 = empty
    __shared__ unsigned long long s_row[kHashSlots];     // row word or count of the slot; later LDS rows
    __shared__ uint16_t s_map[kHashSlots];               // row index of the slot's vertex, kNoRow if none
    __shared__ uint32_t s_sort[kHashSlots];              // candidates being sorted
    __shared__ uint32_t s_wsum[kRbWaves];
    __shared__ unsigned long long s_item, s_off;
    __shared__ uint32_t s_k, s_nt, s_flag, s_claimed;
    unsigned long long *queue = counters;        // roots
    unsigned long long *pool_head = counters + 1;
    uint32_t *cnt = sc.cnt + (uint64_t)blockIdx.x * sc.stride;
    uint32_t *touched = sc.touched + (uint64_t)blockIdx.x * sc.stride;
    uint32_t *cand_g = sc.cand + (uint64_t)blockIdx.x * sc.stride;
    const uint32_t tid = threadIdx.x;
    const uint32_t h0 = tid * kSlotsPerThread;   // this thread's slots in the per-root scans
    for (uint32_t x = tid; x < kHashSlots; x += kRbThreads) {
        s_key[x] = 0;
        s_row[x] = 0;
    }
    u128 acc = 0;
    bool ovf = false;
    uint32_t cur_job = 0xffffffffu;
    uint32_t parts_hint = 1;   // id ranges the previous root needed
    for (;;) {
        if (tid == 0) {
            s_item = atomicAdd(queue, 1ull);
            s_k = 0;
            s_nt = 0;
            s_flag = 0;
            s_off = ~0ull;
            s_claimed = 0;
        }
        __syncthreads();
        const uint64_t item = s_item;
        if (item >= total_roots) break;
        const uint32_t j = find_segment(job_root_prefix, n_jobs, item);
        if (j != cur_job) {
            if (cur_job != 0xffffffffu) wave_flush(slots, jobs[cur_job].slot, acc, ovf, 0, 0);
            acc = 0;
            ovf = false;
            cur_job = j;
        }
        const Job jb = jobs[j];
        const uint32_t u = jb.root_lo + (uint32_t)(item - job_root_prefix[j]);
        const uint64_t ub = jb.ptrA[u];
        const uint32_t du = (uint32_t)(jb.ptrA[u + 1] - ub);
        const uint32_t W1 = (du + 63) >> 6;
        // one thread reads the clock so that the whole block takes the same branch
        if (tid == 0 && past_deadline(jb.deadline)) {
            s_flag = 4;
            atomicOr(&slots[jb.slot].flags, FLAG_TIMEOUT);
        }
        __syncthreads();
        if (du < jb.qA || s_flag == 4) {
            if (tid == 0) {
                out_k[item] = 0;
                out_off[item] = ~0ull;
            }
            __syncthreads();
            continue;
        }
        const bool one = W1 == 1;
        const bool rows = jb.pA >= 3;
        u128 rsum = 0;   // PV: this thread's part of the root's leaves

        // pass 1: insert every 2-hop vertex; one-word roots OR in the row bit,
        // wider ones count.  It gives up at the first insert that finds no
        // slot within kHashProbes, and is skipped when the previous root of
        // this block needed several id ranges.
        volatile uint32_t *flag = &s_flag;
        bool in_lds = false;
        if (parts_hint == 1) {
            wedges_flat_capped<kRbWaves, false>(jb, ub, du, 0, &s_claimed, flag, [&](uint32_t jj, uint32_t w) {
                const int h = hash_insert(s_key, w);
                if (h < 0) *flag = 1u;
                else if (one) atomicOr(&s_row[h], 1ull << jj);
                else atomicAdd(&s_row[h], 1ull);
                return false;
            });
            __syncthreads();
            in_lds = s_flag == 0;
            if (in_lds) parts_hint = 1;
        }
        uint32_t k = 0;
        uint64_t off = ~0ull;
        bool build = false;
        bool done = in_lds;
        if (!in_lds) {
            // The candidates are the ids above u.  Take them in id ranges, each
            // counted in a fresh table of at most kCapRange distinct vertices;
            // a range that passes it is halved and counted again, and the width
            // doubles after a sparse range.  Candidates are listed in s_sort.
            const uint32_t lo0 = u + 1u, span = jb.nA - lo0;
            const uint32_t parts = parts_hint > 2u ? parts_hint : 2u;
            uint32_t width = (uint32_t)(((uint64_t)span + parts - 1) / parts);
            uint32_t lo = lo0, distinct = 0;
            bool fits = true;
            while (lo < jb.nA) {
                const uint32_t hi = lo + (width < jb.nA - lo ? width : jb.nA - lo);
                for (uint32_t x = tid; x < kHashSlots; x += kRbThreads) {
                    s_key[x] = 0;
                    s_row[x] = 0;
                }
                if (tid == 0) {
                    s_flag = 0;
                    s_claimed = 0;
                }
                __syncthreads();
                wedges_flat_capped<kRbWaves, true>(jb, ub, du, kCapRange, &s_claimed, flag, [&](uint32_t jj, uint32_t w) {
                    if (w < lo || w >= hi) return false;
                    bool fresh;
                    const int h = hash_insert_new(s_key, w, &fresh);
                    if (h < 0) {
                        *flag = 1u;
                        return false;
                    }
                    if (one) atomicOr(&s_row[h], 1ull << jj);
                    else atomicAdd(&s_row[h], 1ull);
                    return fresh;
                });
                __syncthreads();
                const uint32_t over = s_flag, d = s_claimed;
                __syncthreads();   // read by all before thread 0 resets them
                if (over) {
                    width = (hi - lo) >> 1;   // a range of one id cannot overflow
                    if (width == 0) width = 1;
                    continue;
                }
                distinct += d;
                uint32_t mine = 0;
#pragma unroll
                for (uint32_t i = 0; i < kSlotsPerThread; ++i) {
                    const uint32_t h = h0 + i;
                    const unsigned long long e = s_row[h];
                    const uint32_t c = one ? (uint32_t)__popcll(e) : (uint32_t)e;
                    if (s_key[h] != 0u && c >= jb.qA) {
                        ++mine;
                        if (rows) continue;
                        if (c >= jb.n_ovf) ovf = true;
                        else ovf |= __builtin_add_overflow(acc, jb.binom[c], &acc);
                        if constexpr (PV) {
                            if (jb.pv && c < jb.n_ovf) {
                                pv_add(jb.pv, s_key[h] - 1u, jb.binom[c]);
                                rsum += jb.binom[c];
                            }
                        }
                    }
                }
                uint32_t kk;
                uint32_t pos = block_excl_scan(mine, s_wsum, &kk);
                if (rows) {
                    if (k + kk > kRowsCap) {
                        fits = false;
                        break;
                    }
#pragma unroll
                    for (uint32_t i = 0; i < kSlotsPerThread; ++i) {
                        const uint32_t h = h0 + i;
                        const unsigned long long e = s_row[h];
                        const uint32_t c = one ? (uint32_t)__popcll(e) : (uint32_t)e;
                        const uint32_t kv = s_key[h];
                        if (kv != 0u && c >= jb.qA) s_sort[k + pos++] = kv - 1u;
                    }
                }
                k += kk;
                lo = hi;
                if (4u * d < kCapRange) width = (uint32_t)(2ull * width < span ? 2ull * width : span);
                __syncthreads();   // table and s_wsum reads done before the next range
            }
            parts_hint = distinct > kHintDistinct ? (distinct + kCapRange - 1) / kCapRange : 1u;
            done = fits;
            if (fits) {
                build = rows && k >= jb.pA - 1;
                if (build && tid == 0) {
                    const unsigned long long need = (unsigned long long)k * W1;
                    const unsigned long long o = atomicAdd(pool_head, need);
                    if (o + need <= pool_cap) s_off = o;
                }
                __syncthreads();
                off = s_off;
                if (build && off != ~0ull) {
                    // rows in increasing id order; a table of the candidates alone
                    // (at most half full) maps an id to its row
                    block_sort_u32<kRbThreads>(s_sort, k);
                    for (uint32_t x = tid; x < kHashSlots; x += kRbThreads) s_key[x] = 0;
                    __syncthreads();
                    for (uint32_t x = tid; x < k; x += kRbThreads) {
                        const uint32_t kv = s_sort[x] + 1u;
                        uint32_t h = hash_slot(kv - 1u);
                        while (atomicCAS(&s_key[h], 0u, kv) != 0u) h = (h + 1) & (kHashSlots - 1);
                        s_map[h] = (uint16_t)x;
                    }
                    const uint64_t words = (uint64_t)k * W1;
                    const bool lds_rows = words <= kHashSlots;
                    if (lds_rows)
                        for (uint32_t x = tid; x < words; x += kRbThreads) s_row[x] = 0;
                    else
                        for (uint64_t x = tid; x < words; x += kRbThreads) pool[off + x] = 0;
                    __threadfence();
                    __syncthreads();
                    wedges_flat<kRbWaves>(jb, ub, du, [&](uint32_t jj, uint32_t w) {
                        const int h = hash_lookup(s_key, w);
                        if (h >= 0) {
                            const uint64_t x = (uint64_t)(jj >> 6) * k + s_map[h];
                            if (lds_rows) atomicOr(&s_row[x], 1ull << (jj & 63));
                            else atomicOr((unsigned long long *)&pool[off + x], 1ull << (jj & 63));
                        }
                    });
                    __syncthreads();
                    if (lds_rows)
                        for (uint32_t x = tid; x < words; x += kRbThreads) pool[off + x] = s_row[x];
                }
            } else {
                k = 0;
            }
        }
        if (in_lds) {
            // candidates: count >= qA, indexed in slot order (pA == 2 sums its leaves here)
            uint32_t mine = 0;
#pragma unroll
            for (uint32_t i = 0; i < kSlotsPerThread; ++i) {
                const uint32_t h = h0 + i;
                const unsigned long long e = s_row[h];
                const uint32_t c = one ? (uint32_t)__popcll(e) : (uint32_t)e;
                if (s_key[h] != 0u && c >= jb.qA) {
                    ++mine;
                    if (rows) continue;
                    if (c >= jb.n_ovf) ovf = true;
                    else ovf |= __builtin_add_overflow(acc, jb.binom[c], &acc);
                    if constexpr (PV) {
                        if (jb.pv && c < jb.n_ovf) {
                            pv_add(jb.pv, s_key[h] - 1u, jb.binom[c]);
                            rsum += jb.binom[c];
                        }
                    }
                }
            }
            uint32_t pos = block_excl_scan(mine, s_wsum, &k);
            build = rows && k >= jb.pA - 1;
            if (build && tid == 0) {
                const unsigned long long need = (unsigned long long)k * W1;
                const unsigned long long o = atomicAdd(pool_head, need);
                if (o + need <= pool_cap) s_off = o;
            }
            __syncthreads();
            off = s_off;
            if (build && off != ~0ull) {
                // rows in increasing rank order of the candidates: list and sort them
#pragma unroll
                for (uint32_t i = 0; i < kSlotsPerThread; ++i) {
                    const uint32_t h = h0 + i;
                    const unsigned long long e = s_row[h];
                    const uint32_t c = one ? (uint32_t)__popcll(e) : (uint32_t)e;
                    const uint32_t kv = s_key[h];
                    const bool cand = kv != 0u && c >= jb.qA;
                    if (cand) s_sort[pos++] = kv - 1u;
                    if (!one) s_map[h] = kNoRow;
                }
                block_sort_u32<kRbThreads>(s_sort, k);
                // one-word roots write their rows now; wider ones record the row index
                for (uint32_t x = tid; x < k; x += kRbThreads) {
                    const uint32_t h = hash_find(s_key, s_sort[x]);
                    if (one) pool[off + x] = s_row[h];
                    else s_map[h] = (uint16_t)x;
                }
                if (!one) {
                    const uint64_t words = (uint64_t)k * W1;
                    const bool lds_rows = words <= kHashSlots;
                    __syncthreads();   // every count has been read
                    if (lds_rows)
                        for (uint32_t x = tid; x < words; x += kRbThreads) s_row[x] = 0;
                    else
                        for (uint64_t x = tid; x < words; x += kRbThreads) pool[off + x] = 0;
                    __threadfence();
                    __syncthreads();
                    // pass 2: set v_j's column bit of row(w) for every wedge u - v_j - w with w a candidate
                    wedges_flat<kRbWaves>(jb, ub, du, [&](uint32_t jj, uint32_t w) {
                        const uint32_t m = s_map[hash_find(s_key, w)];
                        if (m != kNoRow) {
                            const uint64_t x = (uint64_t)(jj >> 6) * k + m;
                            if (lds_rows) atomicOr(&s_row[x], 1ull << (jj & 63));
                            else atomicOr((unsigned long long *)&pool[off + x], 1ull << (jj & 63));
                        }
                    });
                    __syncthreads();
                    if (lds_rows)
                        for (uint32_t x = tid; x < words; x += kRbThreads) pool[off + x] = s_row[x];
                }
            }
        }
        if (!done) {
            // too many candidates for the id ranges: count again in the dense array
            wedges_flat<kRbWaves>(jb, ub, du, [&](uint32_t, uint32_t w) {
                if (atomicAdd(&cnt[w], 1u) == 0u) touched[atomicAdd(&s_nt, 1u)] = w;
            });
            __syncthreads();
            const uint32_t nt = s_nt;
            for (uint32_t t = tid; t < nt; t += kRbThreads) {
                const uint32_t w = touched[t];
                const uint32_t c = atomicAdd(&cnt[w], 0u);
                if (c >= jb.qA) {
                    const uint32_t s = atomicAdd(&s_k, 1u);
                    if (rows) {
                        cand_g[s] = w;
                        atomicExch(&cnt[w], kSlotFlag | s);
                    } else {
                        if (c >= jb.n_ovf) ovf = true;
                        else ovf |= __builtin_add_overflow(acc, jb.binom[c], &acc);
                        if constexpr (PV) {
                            if (jb.pv && c < jb.n_ovf) {
                                pv_add(jb.pv, w, jb.binom[c]);
                                rsum += jb.binom[c];
                            }
                        }
                        atomicExch(&cnt[w], 0u);
                    }
                } else {
                    atomicExch(&cnt[w], 0u);
                }
            }
            __syncthreads();
            k = s_k;
            build = rows && k >= jb.pA - 1;
            if (build && tid == 0) {
                const unsigned long long need = (unsigned long long)k * W1;
                const unsigned long long o = atomicAdd(pool_head, need);
                if (o + need <= pool_cap) s_off = o;
            }
            __syncthreads();
            off = s_off;
            if (build && off != ~0ull) {
                const uint64_t words = (uint64_t)k * W1;
                for (uint64_t x = tid; x < words; x += kRbThreads) pool[off + x] = 0;
                __threadfence();
                __syncthreads();
                wedges_flat<kRbWaves>(jb, ub, du, [&](uint32_t jj, uint32_t w) {
                    const uint32_t e = atomicAdd(&cnt[w], 0u);
                    if (e & kSlotFlag)
                        atomicOr((unsigned long long *)&pool[off + (uint64_t)(jj >> 6) * k + (e & ~kSlotFlag)],
                                 1ull << (jj & 63));
                });
                __syncthreads();
            }
            // reset the candidates' counters
            if (rows)
                for (uint32_t s = tid; s < k; s += kRbThreads) atomicExch(&cnt[cand_g[s]], 0u);
        }
        if (build && off == ~0ull && tid == 0) atomicOr(&slots[jb.slot].flags, FLAG_POOL);
        if constexpr (PV) {
            // the root's own count: its leaves summed per wave, one add per wave
            if (jb.pv && jb.pA == 2) {
                bool o = false;
                const u128 t = wave_sum_u128(rsum, &o);
                ovf |= o;
                if (lane_id() == 0 && t != 0) pv_add(jb.pv, u, t);
            }
        }
        if (tid == 0) {
            out_k[item] = k;
            out_off[item] = build ? off : ~0ull;
        }
        __syncthreads();
        for (uint32_t x = tid; x < kHashSlots; x += kRbThreads) {
            s_key[x] = 0;
            s_row[x] = 0;
        }
        __syncthreads();
    }
    if (cur_job != 0xffffffffu) wave_flush(slots, jobs[cur_job].slot, acc, ovf, 0, 0);
}

hipError_t launch_root_build(const Job *jobs, const uint64_t *job_root_prefix, uint32_t n_jobs,
                             uint64_t total_roots, RootScratch scratch, uint64_t *pool, uint64_t pool_cap,
                             uint32_t n_blocks, unsigned long long *counters, uint32_t *out_k, uint64_t *out_off,
                             Slot *slots, bool per_vertex, hipStream_t stream)
{
    if (total_roots == 0) return hipSuccess;
    if (per_vertex)
        hipLaunchKernelGGL(k_root_build<true>, dim3(n_blocks), dim3(kRbThreads), 0, stream, jobs, job_root_prefix,
                           n_jobs, total_roots, scratch, pool, pool_cap, counters, out_k, out_off, slots);
    else
        hipLaunchKernelGGL(k_root_build<false>, dim3(n_blocks), dim3(kRbThreads), 0, stream, jobs, job_root_prefix,
                           n_jobs, total_roots, scratch, pool, pool_cap, counters, out_k, out_off, slots);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Enumeration.

// Per-lane leaf accumulators.  The u128 total takes the fallback path (table
// entries of 128 bits read from HBM) and every flush; the hot path adds 64-bit
// table entries into lo and counts carries in hi.
struct Acc {
    u128 v;
    bool ovf;
    u128 t;   // 64-bit leaf values of the current task: fewer than 2^64 of them, so t cannot wrap
};

__device__ __forceinline__ void acc_flush(Acc &a)
{
    a.ovf |= __builtin_add_overflow(a.v, a.t, &a.v);
    a.t = 0;
}

__device__ __forceinline__ void leaf_add(Acc &a, const u128 *binom, uint32_t n_ovf, uint32_t n)
{
    if (n >= n_ovf) {
        a.ovf = true;
        return;
    }
    a.ovf |= __builtin_add_overflow(a.v, binom[n], &a.v);
}

__device__ __forceinline__ uint64_t readlane64(uint64_t v, uint32_t lane)
{
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, (int)lane);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)lane);
    return ((uint64_t)hi << 32) | lo;
}

// Per-wave copy of the low 64 bits of C(n, q) for n < len, valid for the job
// it was loaded for while every entry needed is below 2^64.
struct Table {
    uint64_t *t;         // LDS
    uint32_t *t32;       // LDS: low 32 bits of the same entries
    uint64_t *tile;      // LDS staging of one 64-row tile (64 x kTileWords words)
    uint32_t job, len;
};

// Makes tbl hold entries [0, need) of job j; false if they do not all fit
// (table too short or some entry >= 2^64), in which case the caller uses the
// u128 table in HBM.
__device__ bool table_ready(Table &tb, const Job &jb, uint32_t j, uint32_t need)
{
    if (need > kTableLen || need > jb.n_u64 + 1 || need > jb.binom_n) return false;
    if (tb.job == j && tb.len >= need) return true;
    const uint32_t len = min(kTableLen, min(jb.binom_n, jb.n_u64 + 1));
    for (uint32_t n = lane_id(); n < len; n += kWaveSize) {
        const uint64_t x = (uint64_t)jb.binom[n];
        tb.t[n] = x;
        tb.t32[n] = (uint32_t)x;
    }
    wave_sync();
    tb.job = j;
    tb.len = len;
    return true;
}

// sum over a < b < m of C(popcount(row_a & row_b), q), rows column-major in
// blk (stride), W <= WR words.  64-row tiles of a are loaded coalesced and
// broadcast row by row with readlane; each lane owns one b; the leaf value
// comes from the wave's LDS table.
template <int W>
__device__ __forceinline__ uint32_t and_popcount(const uint64_t *row, const uint64_t (&rb)[W])
{
    uint32_t n = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) n += __popcll(row[w] & rb[w]);
    return n;
}

// sum over a < b < m of C(popcount(row_a & row_b), q), rows of exactly W
// words column-major in blk (stride).  Each lane owns one b; 64-row tiles of
// a are loaded coalesced, staged row-major in the wave's LDS tile and read
// back row by row with one broadcast LDS read per word; the leaf value comes
// from the wave's LDS table.  Lanes past m hold zero rows, so they add
// C(0, q) = 0 and need no mask.
//
// The diagonal tile (the t <= 64 rows b0 .. b0+t-1 paired among themselves)
// is folded round-robin: in step d = 1, 2, ... lane b pairs with row
// (b + d) mod t.  Every unordered pair has exactly one difference d <= t/2
// (both differences equal t/2 when t is even, where only lanes b < t/2
// count), so floor(t/2) steps with all lanes busy replace t - 1 masked ones.
//
// Small: every table entry is below 2^58, so 64 of them add up in 64 bits;
// the tile sums go into the 128-bit task sum once per tile.
template <int W, bool Small>
__device__ void pair_sum_tile(const uint64_t *blk, uint32_t stride, uint32_t m, const uint64_t *tbl,
                              uint64_t *tile, Acc &acc)
{
    const uint32_t ln = lane_id();
    for (uint32_t b0 = 0; b0 < m; b0 += kWaveSize) {
        const uint32_t b = b0 + ln;
        const bool bv = b < m;
        uint64_t rb[W];
#pragma unroll
        for (int w = 0; w < W; ++w) rb[w] = bv ? blk[(uint64_t)w * stride + b] : 0ull;
        for (uint32_t a0 = 0; a0 < b0; a0 += kWaveSize) {
#pragma unroll
            for (int w = 0; w < W; ++w) tile[ln * W + w] = blk[(uint64_t)w * stride + a0 + ln];
            wave_sync();
            uint64_t s = 0;
            for (uint32_t j = 0; j < (uint32_t)kWaveSize; j += 8) {
                uint32_t n[8];
#pragma unroll
                for (int r = 0; r < 8; ++r) n[r] = and_popcount<W>(tile + (j + r) * W, rb);
                uint64_t x[8];
#pragma unroll
                for (int r = 0; r < 8; ++r) x[r] = tbl[n[r]];
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    if (Small) s += x[r];
                    else acc.t += x[r];
                }
            }
            if (Small) acc.t += s;
            wave_sync();
        }
        // diagonal tile, folded round-robin
        const uint32_t t = min((uint32_t)kWaveSize, m - b0);
#pragma unroll
        for (int w = 0; w < W; ++w) tile[ln * W + w] = rb[w];
        wave_sync();
        const uint32_t half = t >> 1;
        uint64_t s = 0;
        uint32_t a = ln;
        for (uint32_t d = 1; d <= half; ++d) {
            a = (a + 1 == t) ? 0u : a + 1;                    // (ln + d) mod t for lanes ln < t
            const uint32_t n = and_popcount<W>(tile + (ln < t ? a : 0u) * W, rb);
            const bool take = (2 * d != t) || (ln < half);    // d = t/2: each pair once
            const uint64_t x = take ? tbl[n] : 0ull;
            if (Small) s += x;
            else acc.t += x;
        }
        if (Small) acc.t += s;
        wave_sync();
    }
    acc_flush(acc);
}

// The same sum as a product on the matrix cores.  With the rows as 0/1
// vectors, |row_a & row_b| is entry (a, b) of R R^T, so 16 x 16 blocks of
// intersection sizes come out of v_mfma_i32_16x16x64_i8 (one instruction per
// 64-bit row word).  Operand layout: lane l holds row (l mod 16) of a 16-row
// block, bits [16 (l / 16), 16 (l / 16) + 16) of each word spread to one byte
// per bit; the A and B operands of a block are built the same way, so every
// bit position meets its partner.  One operand is spread as 0/4 bytes (the
// one built once per column group or pair block) and the other, streamed
// one, as 0/1 bytes through a table; the accumulator starts at the LDS byte
// address of the C(n, q) table, so each result is already the address of its
// leaf value.  Result register i of
// lane l is entry (4 (l / 16) + i, l mod 16) of the block; in a diagonal
// block only entries above the diagonal count.  Rows past m are zero and add
// C(0, q) = 0.
//
// G column blocks stay in registers while the row blocks stream by.  Every
// table entry is below 2^28, so the 4 G <= 16 leaf values a lane takes per
// row block add up in 32 bits.
typedef int v4i __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const uint32_t lds_u32;

__device__ __forceinline__ uint32_t lds_addr(const uint32_t *p) { return (uint32_t)(uintptr_t)(lds_u32 *)p; }
__device__ __forceinline__ uint32_t lds_load_u32(uint32_t a) { return *(lds_u32 *)(uintptr_t)a; }

// Bits [off, off + 16) of x (off = 16 (lane / 16)) as 16 bytes of value
// `one` (1 or 4): nibble t of the chunk times the spreading multiplier puts
// its bit k at bit 8k (+2 for the value 4) of dword t, with no carries.
template <uint32_t One>
__device__ __forceinline__ v4i spread_bits(uint64_t x, uint32_t ln)
{
    constexpr uint32_t mul = One == 1 ? 0x00204081u : 0x00810204u;
    constexpr uint32_t msk = One == 1 ? 0x01010101u : 0x04040404u;
    const uint32_t half = (ln & 32) ? (uint32_t)(x >> 32) : (uint32_t)x;
    const uint32_t c = half >> (ln & 16);
    v4i e;
#pragma unroll
    for (int t = 0; t < 4; ++t) e[t] = (int)((((c >> (4 * t)) & 0xfu) * mul) & msk);
    return e;
}

template <int W>
__device__ __forceinline__ v4i mfma_block(const v4i (&ei)[W], const v4i (&ej)[W], v4i c0)
{
    v4i d = __builtin_amdgcn_mfma_i32_16x16x64_i8(ei[0], ej[0], c0, 0, 0, 0);
#pragma unroll
    for (int w = 1; w < W; ++w) d = __builtin_amdgcn_mfma_i32_16x16x64_i8(ei[w], ej[w], d, 0, 0, 0);
    return d;
}

typedef __attribute__((address_space(1))) const uint64_t glb_u64;
typedef __attribute__((address_space(3))) const uint64_t lds_u64;

// Eight-bit spreads for the matrix-core operands, one table per block
// (k_enumerate fills it before its first task): entry v holds bit k of v in
// byte k, as 0 or 1.
__shared__ uint64_t spread_lut[256];

__device__ __forceinline__ uint64_t spread_lut_entry(uint32_t v)
{
    uint64_t e = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) e |= (uint64_t)((v >> k) & 1u) << (8 * k);
    return e;
}

// spread_bits<1> through the table: bits [sh, sh + 16) of x (sh = 16 (lane /
// 16)) as 16 bytes of value 0 or 1, in two LDS reads instead of twelve ALU
// operations.
__device__ __forceinline__ v4i spread1_lut(uint64_t x, uint32_t sh)
{
    const uint32_t c = (uint32_t)(x >> sh);
    const uint32_t base = (uint32_t)(uintptr_t)(lds_u64 *)spread_lut;
    const uint64_t lo = *(lds_u64 *)(uintptr_t)(base + ((c & 0xffu) << 3));
    const uint64_t hi = *(lds_u64 *)(uintptr_t)(base + (((c >> 8) & 0xffu) << 3));
    v4i e;
    e[0] = (int)(uint32_t)lo;
    e[1] = (int)(uint32_t)(lo >> 32);
    e[2] = (int)(uint32_t)hi;
    e[3] = (int)(uint32_t)(hi >> 32);
    return e;
}

// Rows in LDS or in the wave's slab: typed loads, so that row fetches from
// the slab count only against vmcnt and the leaf-table reads' lgkmcnt waits
// do not wait for them.
template <bool Lds>
__device__ __forceinline__ uint64_t row_word(const uint64_t *blk, uint64_t x)
{
    if constexpr (Lds) return ((lds_u64 *)blk)[x];
    else return ((glb_u64 *)blk)[x];
}

template <int W, int G, bool Lds>
__device__ void pair_sum_mfma(const uint64_t *blk, uint32_t stride, uint32_t m, const uint32_t *t32, Acc &acc)
{
    const uint32_t ln = lane_id();
    const uint32_t r16 = ln & 15;
    const uint32_t nb = __builtin_amdgcn_readfirstlane((m + 15) >> 4);   // the group bounds below stay scalar
    const uint32_t sh = 16 * (ln >> 4);
    const int tb = (int)lds_addr(t32);   // t32[0] = C(0, q) = 0
    const v4i c0 = {tb, tb, tb, tb};
    bool above[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) above[i] = 4 * (ln >> 4) + (uint32_t)i < r16;
    // the W words of this lane's row in row block I (zero past m)
    auto fetch = [&](uint32_t I, uint64_t (&x)[W]) {
        const uint32_t row = 16 * I + r16;
        const uint32_t rr = row < m ? row : m - 1;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint64_t v = row_word<Lds>(blk, (uint64_t)w * stride + rr);
            x[w] = row < m ? v : 0ull;
        }
    };
    // Column groups end at the last block: when G does not divide nb the
    // first group starts below block 0.  Its blocks J < 0 are zero rows that
    // meet no row block (row blocks I < 0 are skipped, and a row block I
    // meets only the columns J >= I), so no product is spent past m.
    const uint32_t part = nb % G;
    for (int J0 = part ? (int)part - G : 0; J0 < (int)nb; J0 += G) {
        v4i ej[G][W];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            uint64_t x[W];
            fetch(J0 + g >= 0 ? (uint32_t)(J0 + g) : nb, x);   // block nb lies past m: zero rows
#pragma unroll
            for (int w = 0; w < W; ++w) ej[g][w] = spread_bits<4>(x[w], ln);
        }
        uint64_t s64 = 0;
        // row blocks up to the group's last (J0 + G - 1 <= nb - 1); the next
        // block's words are fetched one step ahead
        uint64_t nx[W];
        fetch(0, nx);
        // row blocks before the group: every entry is above the diagonal
        for (int I = 0; I < J0; ++I) {
            v4i ei[W];
#pragma unroll
            for (int w = 0; w < W; ++w) ei[w] = spread1_lut(nx[w], sh);
            fetch((uint32_t)I + 1, nx);
            v4i d[G];
#pragma unroll
            for (int g = 0; g < G; ++g) d[g] = mfma_block<W>(ei, ej[g], c0);
            uint32_t s = 0;
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int i = 0; i < 4; ++i) s += lds_load_u32((uint32_t)d[g][i]);
            s64 += s;
        }
        // row blocks inside the group: row block J0 + i meets the column
        // blocks J0 + g with g >= i, and only g = i is a diagonal block
#pragma unroll
        for (int i = 0; i < G; ++i) {
            if (J0 + i < 0) continue;   // wave-uniform: blocks below 0 (first group only)
            const uint32_t I = (uint32_t)(J0 + i);
            v4i ei[W];
#pragma unroll
            for (int w = 0; w < W; ++w) ei[w] = spread1_lut(nx[w], sh);
            if (i + 1 < G) fetch(I + 1, nx);
            uint32_t s = 0;
#pragma unroll
            for (int g = i; g < G; ++g) {
                const v4i d = mfma_block<W>(ei, ej[g], c0);
#pragma unroll
                for (int k = 0; k < 4; ++k) s += lds_load_u32((g > i || above[k]) ? (uint32_t)d[k] : (uint32_t)tb);
            }
            s64 += s;
        }
        acc.t += s64;
    }
    acc_flush(acc);
}

template <int W, int G>
__device__ __forceinline__ void pair_sum_mfma_any(const uint64_t *blk, bool in_lds, uint32_t stride, uint32_t m,
                                                  const uint32_t *t32, Acc &acc)
{
    if (in_lds) pair_sum_mfma<W, G, true>(blk, stride, m, t32, acc);
    else pair_sum_mfma<W, G, false>(blk, stride, m, t32, acc);
}

// Same sum through the u128 table in HBM (wide rows or entries >= 2^64).
__device__ void pair_sum_mem(const uint64_t *blk, uint32_t stride, uint32_t m, uint32_t W, const u128 *binom,
                             uint32_t q, uint32_t n_ovf, Acc &acc)
{
    const uint32_t ln = lane_id();
    for (uint32_t b0 = 1; b0 < m; b0 += kWaveSize) {
        const uint32_t b = b0 + ln;
        const bool valid = b < m;
        const uint32_t bb = valid ? b : 0;
        const uint32_t amax = min(m - 1, b0 + kWaveSize - 1);
        for (uint32_t a = 0; a < amax; ++a) {
            uint32_t n = 0;
            for (uint32_t w = 0; w < W; ++w)
                n += __popcll(blk[(uint64_t)w * stride + a] & blk[(uint64_t)w * stride + bb]);
            if (valid && a < b && n >= q) leaf_add(acc, binom, n_ovf, n);
        }
    }
}

// Returns the column-group width G of the matrix-core path, 0 for the others.
__device__ uint32_t pair_sum(const uint64_t *blk, bool in_lds, uint32_t stride, uint32_t m, uint32_t W,
                             uint32_t nbits, const Job &jb, uint32_t j, Table &tb, Acc &acc)
{
    if (m < 2) return 0;
    // every popcount is at most nbits (the compacted universe)
    if (W <= kTileWords && table_ready(tb, jb, j, nbits + 1)) {
        if (nbits <= jb.n_u28) {
            switch (W) {
            case 1: pair_sum_mfma_any<1, 4>(blk, in_lds, stride, m, tb.t32, acc); return 4;
            case 2: pair_sum_mfma_any<2, 2>(blk, in_lds, stride, m, tb.t32, acc); return 2;
            case 3: pair_sum_mfma_any<3, 1>(blk, in_lds, stride, m, tb.t32, acc); return 1;
            default: pair_sum_mfma_any<4, 1>(blk, in_lds, stride, m, tb.t32, acc); return 1;
            }
        } else if (nbits <= jb.n_u58) {
            switch (W) {
            case 1: pair_sum_tile<1, true>(blk, stride, m, tb.t, tb.tile, acc); break;
            case 2: pair_sum_tile<2, true>(blk, stride, m, tb.t, tb.tile, acc); break;
            case 3: pair_sum_tile<3, true>(blk, stride, m, tb.t, tb.tile, acc); break;
            default: pair_sum_tile<4, true>(blk, stride, m, tb.t, tb.tile, acc); break;
            }
        } else {
            switch (W) {
            case 1: pair_sum_tile<1, false>(blk, stride, m, tb.t, tb.tile, acc); break;
            case 2: pair_sum_tile<2, false>(blk, stride, m, tb.t, tb.tile, acc); break;
            case 3: pair_sum_tile<3, false>(blk, stride, m, tb.t, tb.tile, acc); break;
            default: pair_sum_tile<4, false>(blk, stride, m, tb.t, tb.tile, acc); break;
            }
        }
    } else {
        pair_sum_mem(blk, stride, m, W, jb.binom, jb.qA, jb.n_ovf, acc);
    }
    return 0;
}

// The last three levels of a small node at once: over the node's rows
// r_0 .. r_{m-1} (W words each), sum over a < b < c of C(|r_a & r_b & r_c|, q).
// This equals what the children of the node and their leaf sums add up to
// (a child a keeps b when |r_a & r_b| >= q; dropped pairs only had zero
// leaves).  Pair rows p_ab = r_a & r_b with at least q bits are listed in
// order of b (rows of P, b in Pb); then each 16-pair block of P meets the
// 16-row blocks of the node's rows c on the matrix cores exactly like
// pair_sum_mfma, keeping entries with c > b.  One sweep replaces m leaf sums
// over short lists.  P holds pcap pair rows (W words each, stride pcap)
// followed by pcap u32 values of b.
template <int W, bool Lds>
__device__ void triple_sum_mfma(const uint64_t *blk, uint32_t stride, uint32_t m, uint32_t q, uint64_t *P,
                                uint32_t pcap, const uint32_t *t32, Acc &acc, unsigned long long *pairs)
{
    const uint32_t ln = lane_id();
    const uint32_t r16 = ln & 15;
    uint32_t *Pb = (uint32_t *)(P + (uint64_t)W * pcap);
    // 1. pair rows, b-major
    uint32_t np = 0;
    unsigned long long useful = 0;
    for (uint32_t b = 1; b < m; ++b) {
        uint64_t rb[W];
#pragma unroll
        for (int w = 0; w < W; ++w) rb[w] = row_word<Lds>(blk, (uint64_t)w * stride + b);
        for (uint32_t a0 = 0; a0 < b; a0 += kWaveSize) {
            const uint32_t a = a0 + ln;
            const bool valid = a < b;
            const uint32_t aa = valid ? a : 0u;
            uint64_t v[W];
            uint32_t n = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) {
                v[w] = row_word<Lds>(blk, (uint64_t)w * stride + aa) & rb[w];
                n += (uint32_t)__popcll(v[w]);
            }
            const bool keep = valid && n >= q;
            const uint64_t mask = __ballot(keep);
            if (keep) {
                const uint32_t idx = np + mbcnt64(mask);
#pragma unroll
                for (int w = 0; w < W; ++w) P[(uint64_t)w * pcap + idx] = v[w];
                Pb[idx] = b;
            }
            const uint32_t kept = (uint32_t)__popcll(mask);
            np += kept;
            useful += (unsigned long long)kept * (m - 1 - b);
        }
    }
    *pairs += useful;
    wave_sync();
    // 2. pair-row blocks against row blocks c > b
    const uint32_t nbc = (m + 15) >> 4;
    const uint32_t sh = 16 * (ln >> 4);
    const int tb = (int)lds_addr(t32);   // t32[0] = C(0, q) = 0
    const v4i c0 = {tb, tb, tb, tb};
    for (uint32_t i0 = 0; i0 < np; i0 += 16) {
        const uint32_t pr = i0 + r16;
        const bool pv = pr < np;
        const uint32_t prr = pv ? pr : np - 1;
        v4i ea[W];
#pragma unroll
        for (int w = 0; w < W; ++w) ea[w] = spread_bits<4>(pv ? P[(uint64_t)w * pcap + prr] : 0ull, ln);
        const uint32_t bmine = pv ? Pb[prr] : 0xffffffffu;
        uint32_t brow[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) brow[i] = (uint32_t)__shfl((int)bmine, (int)(4 * (ln >> 4) + i));
        const uint32_t bmin = __builtin_amdgcn_readfirstlane(Pb[i0]);   // b-major: the block's smallest b
        uint64_t s64 = 0;
        for (uint32_t J = (bmin + 1) >> 4; J < nbc; ++J) {
            const uint32_t c = 16 * J + r16;
            const uint32_t cc = c < m ? c : m - 1;
            v4i eb[W];
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint64_t x = row_word<Lds>(blk, (uint64_t)w * stride + cc);
                eb[w] = spread1_lut(c < m ? x : 0ull, sh);
            }
            const v4i dd = mfma_block<W>(ea, eb, c0);
            uint32_t s = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i) s += lds_load_u32(c > brow[i] ? (uint32_t)dd[i] : (uint32_t)tb);
            s64 += s;
        }
        acc.t += s64;
    }
    acc_flush(acc);
    wave_sync();
}

// One row block of the pair sum over m rows (W words, column-major with
// stride), on the matrix cores: rows a in [16 I, 16 I + 16) against every
// row b > a, adding C(|row_a & row_b|, q).  The row blocks I = 0, 1, ...
// together give the whole pair sum; rows past m are zero and add nothing.
template <int W, bool Lds>
__device__ void pair_row_block_mfma(const uint64_t *blk, uint32_t stride, uint32_t m, uint32_t I,
                                    const uint32_t *t32, Acc &acc)
{
    const uint32_t ln = lane_id();
    const uint32_t r16 = ln & 15;
    const uint32_t nb = (m + 15) >> 4;
    const uint32_t sh = 16 * (ln >> 4);
    const int tb = (int)lds_addr(t32);
    const v4i c0 = {tb, tb, tb, tb};
    auto fetch = [&](uint32_t B, uint64_t (&x)[W]) {
        const uint32_t row = 16 * B + r16;
        const uint32_t rr = row < m ? row : m - 1;
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint64_t v = row_word<Lds>(blk, (uint64_t)w * stride + rr);
            x[w] = row < m ? v : 0ull;
        }
    };
    uint64_t x[W];
    fetch(I, x);
    v4i ea[W];
#pragma unroll
    for (int w = 0; w < W; ++w) ea[w] = spread_bits<4>(x[w], ln);
    uint64_t s64 = 0;
    uint64_t nx[W];
    fetch(I, nx);
    for (uint32_t J = I; J < nb; ++J) {
        v4i eb[W];
#pragma unroll
        for (int w = 0; w < W; ++w) eb[w] = spread1_lut(nx[w], sh);
        fetch(J + 1, nx);
        const v4i d = mfma_block<W>(ea, eb, c0);
        uint32_t s = 0;
        if (J > I) {
#pragma unroll
            for (int i = 0; i < 4; ++i) s += lds_load_u32((uint32_t)d[i]);
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                s += lds_load_u32(4 * (ln >> 4) + (uint32_t)i < r16 ? (uint32_t)d[i] : (uint32_t)tb);
        }
        s64 += s;
    }
    acc.t += s64;
    acc_flush(acc);
}

// Children of row a: rows b > a whose AND with row a keeps >= q bits, written
// (ANDed) into nblk (stride nstride) in order.  Returns their number.
__device__ uint32_t filter_children(const uint64_t *blk, uint32_t stride, uint32_t m, uint32_t a, uint32_t W,
                                    uint32_t q, uint64_t *nblk, uint32_t nstride)
{
    const uint32_t ln = lane_id();
    uint32_t out = 0;
    if (W == 1) {   // one-word rows: row a read once, each AND computed once
        const uint64_t ra = blk[a];
        for (uint32_t b0 = a + 1; b0 < m; b0 += kWaveSize) {
            const uint32_t b = b0 + ln;
            const bool valid = b < m;
            const uint64_t v = valid ? ra & blk[b] : 0ull;
            const bool keep = valid && (uint32_t)__popcll(v) >= q;
            const uint64_t mask = __ballot(keep);
            if (keep) nblk[out + mbcnt64(mask)] = v;
            out += (uint32_t)__popcll(mask);
        }
        wave_sync();
        return out;
    }
    for (uint32_t b0 = a + 1; b0 < m; b0 += kWaveSize) {
        const uint32_t b = b0 + ln;
        const bool valid = b < m;
        uint32_t n = 0;
        if (valid)
            for (uint32_t w = 0; w < W; ++w)
                n += __popcll(blk[(uint64_t)w * stride + a] & blk[(uint64_t)w * stride + b]);
        const bool keep = valid && n >= q;
        const uint64_t mask = __ballot(keep);
        if (keep) {
            const uint32_t idx = out + mbcnt64(mask);
            for (uint32_t w = 0; w < W; ++w)
                nblk[(uint64_t)w * nstride + idx] = blk[(uint64_t)w * stride + a] & blk[(uint64_t)w * stride + b];
        }
        out += (uint32_t)__popcll(mask);
    }
    wave_sync();
    return out;
}

// Wave-local bump allocator over the LDS and slab regions of one wavefront.
struct Arena {
    uint64_t *lds;
    uint64_t *slab;
    uint32_t lds_cap, lds_used;
    uint64_t slab_cap, slab_used;
    // true when p was handed out from the LDS part
    __device__ bool holds(const uint64_t *p) const { return p >= lds && p < lds + lds_cap; }
};

__device__ __forceinline__ uint64_t *arena_alloc(Arena &ar, uint64_t words, bool *fail)
{
    if (ar.lds_used + words <= ar.lds_cap) {
        uint64_t *p = ar.lds + ar.lds_used;
        ar.lds_used += (uint32_t)words;
        return p;
    }
    if (ar.slab_used + words <= ar.slab_cap) {
        uint64_t *p = ar.slab + ar.slab_used;
        ar.slab_used += words;
        return p;
    }
    *fail = true;
    return nullptr;
}

// Work and cycle counters of one wavefront (uniform values).
struct Counters {
    unsigned long long pair_words, filter_words;
    unsigned long long cyc_setup, cyc_compact, cyc_pair, cyc_filter;
    unsigned long long pairs, pair_slots;
    unsigned long long cyc_pack;
};

// Work of one pair_sum over m rows: pairs, and pair positions (lane-slots)
// the chosen path spends: 16 x 16 blocks of G column blocks on the matrix
// cores (G > 0), else 64-row tiles with the folded diagonal tile.
__device__ __forceinline__ void count_pairs(Counters &ct, uint32_t m, uint32_t W, uint32_t G)
{
    const unsigned long long pr = (unsigned long long)m * (m - 1) / 2;
    ct.pairs += pr;
    ct.pair_words += pr * W;
    if (G) {   // one 16 x 16 product per block pair I <= J, whatever the group width
        const unsigned long long nb = (m + 15) / 16;
        ct.pair_slots += nb * (nb + 1) / 2 * 256;
        return;
    }
    for (uint32_t b0 = 0; b0 < m; b0 += kWaveSize)   // full tiles, then the folded diagonal tile
        ct.pair_slots += (unsigned long long)(b0 / kWaveSize) * kWaveSize * kWaveSize +
                         (unsigned long long)(min((uint32_t)kWaveSize, m - b0) / 2) * kWaveSize;
}

__device__ __forceinline__ uint64_t cycles() { return __builtin_amdgcn_s_memtime(); }

// Runtime split of heavy tasks: a task whose level-2 block keeps more than
// `rows` rows queues one subtask per kept row in a ring that wavefronts drain
// once the task queue is empty (runtime load balancing, Section V-C).
struct SplitCtx {
    uint4 *ring;                    // {heap offset lo, hi, child row, ready}; ready is stored last
    unsigned long long *tail;       // entries reserved so far
    uint64_t *heap;                 // split tasks' level-2 blocks, each after a 4-word header
    unsigned long long *heap_used;  // words of the heap taken so far
    uint64_t heap_cap;              // heap words
    uint32_t cap;                   // ring entries
    uint32_t rows;                  // split threshold on the kept rows
    uint32_t root_idx;              // index of the task's root in the active-root list
};

constexpr uint32_t kNoJ = 0xffffffffu;   // no restriction to one child

// Reserves n consecutive ring entries (lane 0 decides, every lane learns);
// ~0 when the ring cannot hold them.
__device__ unsigned long long ring_reserve(const SplitCtx &sp, uint32_t n)
{
    unsigned long long got = ~0ull;
    if (lane_id() == 0) {
        unsigned long long cur = __hip_atomic_load(sp.tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (cur + n <= sp.cap) {
            if (__hip_atomic_compare_exchange_strong(sp.tail, &cur, cur + n, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)) {
                got = cur;
                break;
            }
        }
    }
    return bcast64(got, 0);
}

// Publishes one ring entry: the payload first, then the ready word with
// release order, so that a reader that sees ready also sees the payload.
__device__ __forceinline__ void ring_put(uint4 *e, uint64_t off, uint32_t a)
{
    e->x = (uint32_t)off;
    e->y = (uint32_t)(off >> 32);
    e->z = a;
    __hip_atomic_store(&e->w, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Takes n heap words (lane 0 decides, every lane learns); ~0 when the heap
// cannot hold them.
__device__ unsigned long long heap_take(const SplitCtx &sp, uint64_t n)
{
    unsigned long long got = ~0ull;
    if (lane_id() == 0) {
        unsigned long long cur = __hip_atomic_load(sp.heap_used, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (cur + n <= sp.heap_cap) {
            if (__hip_atomic_compare_exchange_strong(sp.heap_used, &cur, cur + n, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                got = cur;
                break;
            }
        }
    }
    return bcast64(got, 0);
}

__device__ __attribute__((always_inline)) inline void dfs_level2(
    const Job &jb, uint32_t jidx, const uint64_t *blk2, uint32_t stride2, uint32_t m2, uint32_t W2, uint32_t s2n,
    uint32_t only_child, Arena &ar, uint64_t *stack, Table &tb, Acc &acc, Counters &ct, bool instrument, bool triple,
    bool *cap_fail, bool *timed_out, uint64_t t0);

// One task: the node {u, c_i} of the search tree.  SPLIT compiles in the
// hand-off of heavy tasks to the subtask ring; without it sp is unused.
template <bool SPLIT>
__device__ void run_task(const Job &jb, uint32_t jidx, const ActiveRoot &rt, uint32_t i, const uint64_t *pool,
                         Arena ar, uint64_t *stack, Table &tb, Acc &acc, Counters &ct, bool instrument, bool triple,
                         const SplitCtx *sp, bool *cap_fail, bool *timed_out)
{
    const uint32_t ln = lane_id();
    const uint32_t u = rt.root;
    const uint32_t du = (uint32_t)(jb.ptrA[u + 1] - jb.ptrA[u]);
    const uint32_t W1 = (du + 63) >> 6;
    const uint32_t k = rt.k;
    glb_u64 *base = (glb_u64 *)(pool + rt.pool_off);   // the root's rows (global: typed loads)
    const uint32_t q = jb.qA, pA = jb.pA;
    uint64_t t0 = instrument ? cycles() : 0;

    const uint32_t s = i;   // the candidates are the rows after i
    const uint32_t rem = k - s - 1;
    if (pA == 3 && W1 <= kTileWords && du <= jb.n_u28 && table_ready(tb, jb, jidx, du + 1)) {
        // the root's leaves {u, c_a, c_b} are the pair sum over its rows:
        // task i = 16 I takes row block I on the matrix cores, the root's
        // other tasks have nothing left to do
        if ((i & 15) == 0) {
            const uint64_t *rows = pool + rt.pool_off;
            switch (W1) {
            case 1: pair_row_block_mfma<1, false>(rows, k, k, i >> 4, tb.t32, acc); break;
            case 2: pair_row_block_mfma<2, false>(rows, k, k, i >> 4, tb.t32, acc); break;
            case 3: pair_row_block_mfma<3, false>(rows, k, k, i >> 4, tb.t32, acc); break;
            default: pair_row_block_mfma<4, false>(rows, k, k, i >> 4, tb.t32, acc); break;
            }
            if (instrument) {
                const uint32_t a1 = min(i + 16, k);
                unsigned long long pr = 0;
                for (uint32_t a = i; a < a1; ++a) pr += k - 1 - a;
                ct.pairs += pr;
                ct.pair_words += pr * W1;
                ct.pair_slots += 256ull * (((k + 15) >> 4) - (i >> 4));
            }
        }
        if (instrument) ct.cyc_pair += cycles() - t0;
        return;
    }
    // S2 = row i (common neighbours of u and c_i).  Its first two nonzero
    // words (s0, s1, at word indices w0, w1) stay in scalar registers; wider
    // roots also get the table of all nonzero words.
    uint32_t s2n, nz;
    uint64_t s0 = 0, s1 = 0;
    uint32_t w0 = 0, w1 = 0;
    uint64_t *nzt = nullptr;
    if (W1 == 1) {
        // one-word root: nothing to scan or tabulate
        const uint64_t x = base[i];
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)x);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
        s0 = ((uint64_t)hi << 32) | lo;
        s2n = (uint32_t)__popcll(s0);
        nz = s0 != 0 ? 1u : 0u;
        if (instrument) {
            const uint64_t t1 = cycles();
            ct.cyc_setup += t1 - t0;
            t0 = t1;
        }
    } else {
        // S2 and its word prefix counts
        uint64_t *s2 = arena_alloc(ar, 2ull * W1, cap_fail);
        if (!s2) return;
        uint64_t *pre = s2 + W1;
        for (uint32_t w = ln; w < W1; w += kWaveSize) s2[w] = base[(uint64_t)w * k + i];
        wave_sync();
        uint32_t running = 0;
        for (uint32_t x0 = 0; x0 < W1; x0 += kWaveSize) {
            const uint32_t w = x0 + ln;
            const uint32_t c = (w < W1) ? (uint32_t)__popcll(s2[w]) : 0u;
            const uint32_t incl = wave_inclusive_scan(c);
            if (w < W1) pre[w] = running + incl - c;
            running += bcast32(incl, kWaveSize - 1);
        }
        wave_sync();
        s2n = running;
        if (instrument) {
            const uint64_t t1 = cycles();
            ct.cyc_setup += t1 - t0;
            t0 = t1;
        }

        // The nonzero words of S2, each with the six masks of the compress
        // operation (Hacker's Delight, "compress" / parallel bit extract) that
        // packs the bits selected by that word to the right: entry e holds
        // {s2 word, mv0..mv5, w | pre << 32}.  Empty words of S2 are skipped.
        nzt = arena_alloc(ar, 8ull * W1, cap_fail);
        if (!nzt) return;
        nz = 0;
        for (uint32_t x0 = 0; x0 < W1; x0 += kWaveSize) {
            const uint32_t w = x0 + ln;
            const uint64_t sw = (w < W1) ? s2[w] : 0ull;
            const uint64_t nzmask = __ballot(sw != 0);
            if (sw != 0) {
                uint64_t *e = nzt + 8ull * (nz + mbcnt64(nzmask));
                e[0] = sw;
                uint64_t m = sw, mk = ~sw << 1;
#pragma unroll
                for (int r = 0; r < 6; ++r) {
                    uint64_t mp = mk ^ (mk << 1);
                    mp ^= mp << 2;
                    mp ^= mp << 4;
                    mp ^= mp << 8;
                    mp ^= mp << 16;
                    mp ^= mp << 32;
                    const uint64_t mv = mp & m;
                    e[1 + r] = mv;
                    m = (m ^ mv) | (mv >> (1 << r));
                    mk &= ~mp;
                }
                e[7] = (uint64_t)w | ((uint64_t)pre[w] << 32);
            }
            nz += (uint32_t)__popcll(nzmask);
        }
        wave_sync();
        if (nz > 0) {
            s0 = nzt[0];
            w0 = (uint32_t)nzt[7];
        }
        if (nz > 1) {
            s1 = nzt[8];
            w1 = (uint32_t)nzt[15];
        }
    }
    const uint32_t W2 = (s2n + 63) >> 6;
    if (instrument) ct.filter_words += (unsigned long long)rem * nz;

    if (pA == 3) {
        // Leaves {u, c_i, c_b}: sum of C(|S2 n row_b|, q).
        for (uint32_t b0 = s + 1; b0 < k; b0 += kWaveSize) {
            const uint32_t b = b0 + ln;
            if (b < k) {
                uint32_t n = 0;
                if (nz <= 2) {
                    if (nz > 0) n += __popcll(s0 & base[(uint64_t)w0 * k + b]);
                    if (nz > 1) n += __popcll(s1 & base[(uint64_t)w1 * k + b]);
                } else {
                    for (uint32_t e = 0; e < nz; ++e) {
                        const uint32_t w = (uint32_t)nzt[8ull * e + 7];
                        n += __popcll(nzt[8ull * e] & base[(uint64_t)w * k + b]);
                    }
                }
                if (n >= q) leaf_add(acc, jb.binom, jb.n_ovf, n);
            }
        }
        if (instrument) ct.cyc_compact += cycles() - t0;
        return;
    }

    // Level-2 block: rows b > i restricted to S2 and renumbered to S2's bits
    // (column-major, stride2 words per column).
    uint64_t *blk2 = nullptr;
    uint32_t stride2 = rem;
    uint32_t m2 = 0;
    if (nz <= 2 && nz == W2) {
        // Common case: S2 lives in at most two words that need no packing.
        // The two masks stay in registers; the row words of kFilterDepth
        // chunks are loaded together before any of them is filtered.  A block
        // too big for the wave's LDS when sized for all rem rows starts there
        // anyway, with room for as many rows as fit (half the free LDS when
        // deeper levels follow, so that their blocks keep the other half);
        // only when more rows than that are kept does it move to a slab
        // block of rem rows.
        const uint32_t room = ar.lds_cap - ar.lds_used;
        uint32_t fit = rem;
        if (W2 != 0 && (uint64_t)rem * W2 > room) fit = (pA == 4 ? room : room / 2) / W2;
        stride2 = fit != 0 ? fit : rem;
        blk2 = arena_alloc(ar, (uint64_t)stride2 * W2, cap_fail);
        if (!blk2) return;
        glb_u64 *r0 = base + (uint64_t)w0 * k;
        glb_u64 *r1 = base + (uint64_t)(nz > 1 ? w1 : w0) * k;
        for (uint32_t b0 = s + 1; b0 < k; b0 += kFilterDepth * kWaveSize) {
            uint64_t x0[kFilterDepth], x1[kFilterDepth];
#pragma unroll
            for (uint32_t c = 0; c < kFilterDepth; ++c) {
                const uint32_t b = b0 + c * kWaveSize + ln;
                x0[c] = (b < k) ? r0[b] : 0ull;
                x1[c] = (nz > 1 && b < k) ? r1[b] : 0ull;
            }
#pragma unroll
            for (uint32_t c = 0; c < kFilterDepth; ++c) {
                const uint32_t b = b0 + c * kWaveSize + ln;
                const uint64_t v0 = x0[c] & s0, v1 = x1[c] & s1;
                const uint32_t n = (uint32_t)(__popcll(v0) + __popcll(v1));
                const bool keep = b < k && n >= q;
                const uint64_t mask = __ballot(keep);
                if (m2 + (uint32_t)__popcll(mask) > stride2) {
                    // the LDS block is full: give its words back and move the
                    // rows kept so far to a slab block of rem rows
                    uint64_t *sb = nullptr;
                    if (ar.holds(blk2) && blk2 + (uint64_t)stride2 * W2 == ar.lds + ar.lds_used) {
                        ar.lds_used -= stride2 * W2;
                        sb = arena_alloc(ar, (uint64_t)rem * W2, cap_fail);
                        if (!sb) return;
                        for (uint32_t w = 0; w < W2; ++w)
                            for (uint32_t x = ln; x < m2; x += kWaveSize)
                                sb[(uint64_t)w * rem + x] = blk2[(uint64_t)w * stride2 + x];
                        wave_sync();
                    }
                    if (!sb) {
                        *cap_fail = true;   // not reached: the block was the arena's last allocation
                        return;
                    }
                    blk2 = sb;
                    stride2 = rem;
                }
                if (keep) {
                    const uint32_t idx = m2 + mbcnt64(mask);
                    blk2[idx] = v0;
                    if (nz > 1) blk2[(uint64_t)stride2 + idx] = v1;
                }
                m2 += (uint32_t)__popcll(mask);
            }
        }
    } else {
        // Filter first, listing the kept rows; then copy or bit-pack only
        // those, 64 per step, so that no lane packs a row that was dropped.
        uint32_t *kept = (uint32_t *)arena_alloc(ar, (rem + 1) / 2, cap_fail);
        if (!kept) return;
        for (uint32_t b0 = s + 1; b0 < k; b0 += kWaveSize) {
            const uint32_t b = b0 + ln;
            const bool valid = b < k;
            const uint32_t bb = valid ? b : s;
            uint32_t n = 0;
            for (uint32_t e = 0; e < nz; ++e) {
                const uint32_t w = (uint32_t)nzt[8ull * e + 7];
                n += __popcll(nzt[8ull * e] & base[(uint64_t)w * k + bb]);
            }
            const bool keep = valid && n >= q;
            const uint64_t mask = __ballot(keep);
            if (keep) kept[m2 + mbcnt64(mask)] = b;
            m2 += (uint32_t)__popcll(mask);
        }
        wave_sync();
        // the block is sized for the kept rows only
        stride2 = m2;
        blk2 = arena_alloc(ar, (uint64_t)m2 * W2, cap_fail);
        if (!blk2) return;
        for (uint32_t c0 = 0; c0 < m2; c0 += kWaveSize) {
            const uint32_t idx = c0 + ln;
            const bool live = idx < m2;
            const uint32_t bb = live ? kept[idx] : s;
            if (nz == W2) {
                // S2's nonzero words are already as few as its bits need: the
                // masked words are the compacted row (word e = S2 word e's bits)
                for (uint32_t e = 0; e < nz; ++e) {
                    const uint32_t w = (uint32_t)nzt[8ull * e + 7];
                    const uint64_t x = nzt[8ull * e] & base[(uint64_t)w * k + bb];
                    if (live) blk2[(uint64_t)e * stride2 + idx] = x;
                }
            } else {
                // every lane walks the same entries (uniform control flow)
                uint32_t ow = 0;
                uint64_t cur = 0;
                for (uint32_t e = 0; e < nz; ++e) {
                    const uint64_t *en = nzt + 8ull * e;
                    const uint64_t sw = en[0];
                    const uint32_t w = (uint32_t)en[7];
                    const uint32_t o = (uint32_t)(en[7] >> 32);   // first output bit of this word
                    uint64_t x = sw & base[(uint64_t)w * k + bb];
#pragma unroll
                    for (int r = 0; r < 6; ++r) {
                        const uint64_t t = x & en[1 + r];
                        x = (x ^ t) | (t >> (1 << r));
                    }
                    const uint32_t cnt = (uint32_t)__popcll(sw);
                    const uint32_t tw = o >> 6, sh = o & 63;
                    while (ow < tw) {
                        if (live) blk2[(uint64_t)ow * stride2 + idx] = cur;
                        cur = 0;
                        ++ow;
                    }
                    cur |= x << sh;
                    if (sh + cnt > 64) {
                        if (live) blk2[(uint64_t)ow * stride2 + idx] = cur;
                        cur = x >> (64 - sh);
                        ++ow;
                    }
                }
                while (ow < W2) {
                    if (live) blk2[(uint64_t)ow * stride2 + idx] = cur;
                    cur = 0;
                    ++ow;
                }
            }
        }
    }
    wave_sync();
    if (instrument) {
        const uint64_t t1 = cycles();
        ct.cyc_compact += t1 - t0;
        if (nz != W2) ct.cyc_pack += t1 - t0;
        t0 = t1;
    }
    if (m2 < pA - 2) return;
    // Heavy task (p_A >= 5): its level-2 block goes to the split heap (4-word
    // header, then the block with stride m2) and each child row a that can
    // still complete L becomes a subtask in the ring, to be finished by
    // whichever wavefront takes it; if the heap or the ring is full, the task
    // carries on here.
    if constexpr (SPLIT) {
    if (pA >= 5 && m2 > sp->rows && !(triple && m2 <= kTripleRows)) {
        const uint32_t n_sub = m2 - (pA - 3);   // children a <= m2 - (pA - 2)
        const unsigned long long off = heap_take(*sp, 4 + (uint64_t)m2 * W2);
        const unsigned long long at = off != ~0ull ? ring_reserve(*sp, n_sub) : ~0ull;
        if (at != ~0ull) {
            uint64_t *hdr = sp->heap + off;
            if (ln == 0) {
                hdr[0] = sp->root_idx;
                hdr[1] = i;
                hdr[2] = (uint64_t)m2 | ((uint64_t)W2 << 32);
                hdr[3] = s2n;
            }
            for (uint32_t w = 0; w < W2; ++w)
                for (uint32_t x = ln; x < m2; x += kWaveSize)
                    hdr[4 + (uint64_t)w * m2 + x] = ar.holds(blk2) ? blk2[(uint64_t)w * stride2 + x]
                                                                   : row_word<false>(blk2, (uint64_t)w * stride2 + x);
            // the block must be visible before any entry naming it
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            for (uint32_t x = ln; x < n_sub; x += kWaveSize) ring_put(sp->ring + at + x, off, x);
            if (instrument) ct.cyc_compact += cycles() - t0;
            return;
        }
        // (a heap block taken without ring room stays unused until the launch ends)
    }
    }
    dfs_level2(jb, jidx, blk2, stride2, m2, W2, s2n, kNoJ, ar, stack, tb, acc, ct, instrument, triple, cap_fail, timed_out,
               t0);
}

// The search below a level-2 node {u, c_i} whose block holds m2 rows of W2
// words (column-major, stride2): pair sums for p_A = 4, else the DFS over
// levels 2 .. pA-3, the node at level pA-2 finished by pair_sum (small nodes
// at level pA-3 by the three-level sweep).  only_child != kNoJ restricts the
// level-2 loop to that one child row (a subtask of a split task).
__device__ __attribute__((always_inline)) inline void dfs_level2(
    const Job &jb, uint32_t jidx, const uint64_t *blk2, uint32_t stride2, uint32_t m2, uint32_t W2, uint32_t s2n,
    uint32_t only_child, Arena &ar, uint64_t *stack, Table &tb, Acc &acc, Counters &ct, bool instrument, bool triple,
    bool *cap_fail, bool *timed_out, uint64_t t0)
{
    const uint32_t q = jb.qA, pA = jb.pA;
    if (pA == 4) {
        const uint32_t G = pair_sum(blk2, ar.holds(blk2), stride2, m2, W2, s2n, jb, jidx, tb, acc);
        if (instrument) count_pairs(ct, m2, W2, G);
        if (instrument) ct.cyc_pair += cycles() - t0;
        return;
    }
    // stack[4*d + 0] = the level's block (pointer), [1] = stride | m << 32,
    // [2] = cursor, [3] = arena marks (lds_used | slab_used << 32).
    auto enc_ptr = [&](const uint64_t *p) -> uint64_t { return (uint64_t)(uintptr_t)p; };
    auto dec_ptr = [&](uint64_t e) -> const uint64_t * { return (const uint64_t *)(uintptr_t)e; };
    const uint32_t a_end = only_child == kNoJ ? 0xffffffffu : only_child + 1;
    uint32_t d = 2;
    stack[4 * 2 + 0] = enc_ptr(blk2);
    stack[4 * 2 + 1] = (uint64_t)stride2 | ((uint64_t)m2 << 32);
    stack[4 * 2 + 2] = only_child == kNoJ ? 0 : only_child;
    stack[4 * 2 + 3] = 0;
    for (;;) {
        if (past_deadline(jb.deadline)) {
            *timed_out = true;
            return;
        }
        const uint64_t *blk = dec_ptr(stack[4 * d + 0]);
        const uint32_t stride = (uint32_t)stack[4 * d + 1];
        const uint32_t m = (uint32_t)(stack[4 * d + 1] >> 32);
        uint32_t a = (uint32_t)stack[4 * d + 2];
        // a small node two levels above the leaves: its last three levels in
        // one matrix-core sweep, then the node is done
        if (triple && d + 3 == pA && a == 0 && m >= 3 && m <= kTripleRows && W2 <= kTileWords && s2n <= jb.n_u28 &&
            table_ready(tb, jb, jidx, s2n + 1)) {
            const uint32_t pcap = m * (m - 1) / 2;
            const uint64_t mark = (uint64_t)ar.lds_used | (ar.slab_used << 32);
            uint64_t *P = arena_alloc(ar, (uint64_t)pcap * W2 + (pcap + 1) / 2, cap_fail);
            if (!P) return;
            if (instrument) t0 = cycles();
            unsigned long long tp = 0;
            const bool lds_blk = ar.holds(blk);
            switch (W2) {
            case 1:
                if (lds_blk) triple_sum_mfma<1, true>(blk, stride, m, q, P, pcap, tb.t32, acc, &tp);
                else triple_sum_mfma<1, false>(blk, stride, m, q, P, pcap, tb.t32, acc, &tp);
                break;
            case 2:
                if (lds_blk) triple_sum_mfma<2, true>(blk, stride, m, q, P, pcap, tb.t32, acc, &tp);
                else triple_sum_mfma<2, false>(blk, stride, m, q, P, pcap, tb.t32, acc, &tp);
                break;
            case 3:
                if (lds_blk) triple_sum_mfma<3, true>(blk, stride, m, q, P, pcap, tb.t32, acc, &tp);
                else triple_sum_mfma<3, false>(blk, stride, m, q, P, pcap, tb.t32, acc, &tp);
                break;
            default:
                if (lds_blk) triple_sum_mfma<4, true>(blk, stride, m, q, P, pcap, tb.t32, acc, &tp);
                else triple_sum_mfma<4, false>(blk, stride, m, q, P, pcap, tb.t32, acc, &tp);
                break;
            }
            if (instrument) {
                ct.pairs += tp;
                ct.pair_words += tp * W2;
                ct.filter_words += (unsigned long long)pcap * W2;
                ct.cyc_pair += cycles() - t0;
            }
            ar.lds_used = (uint32_t)(mark & 0xffffffffu);
            ar.slab_used = mark >> 32;
            a = m;   // exhausted: pop below
        }
        // row a needs pA - d - 1 more rows after it (a subtask does one level-2 child)
        if ((int64_t)a > (int64_t)m - (int64_t)pA + (int64_t)d || (d == 2 && a >= a_end)) {
            if (d == 2) break;
            // pop: release this level's block
            const uint64_t mk = stack[4 * d + 3];
            ar.lds_used = (uint32_t)(mk & 0xffffffffu);
            ar.slab_used = mk >> 32;
            --d;
            continue;
        }
        stack[4 * d + 2] = a + 1;
        const uint32_t cap = m - a - 1;
        const uint64_t mark = (uint64_t)ar.lds_used | (ar.slab_used << 32);
        uint64_t *nb = arena_alloc(ar, (uint64_t)cap * W2, cap_fail);
        if (!nb) return;
        if (instrument) t0 = cycles();
        const uint32_t mc = filter_children(blk, stride, m, a, W2, q, nb, cap);
        if (instrument) ct.filter_words += (unsigned long long)cap * W2;
        if (instrument) {
            const uint64_t t1 = cycles();
            ct.cyc_filter += t1 - t0;
            t0 = t1;
        }
        if (mc >= pA - d - 1) {
            if (d + 1 == pA - 2) {
                const uint32_t G = pair_sum(nb, ar.holds(nb), cap, mc, W2, s2n, jb, jidx, tb, acc);
                if (instrument) count_pairs(ct, mc, W2, G);
                if (instrument) ct.cyc_pair += cycles() - t0;
            } else {
                ++d;
                stack[4 * d + 0] = enc_ptr(nb);
                stack[4 * d + 1] = (uint64_t)cap | ((uint64_t)mc << 32);
                stack[4 * d + 2] = 0;
                stack[4 * d + 3] = mark;
                continue;
            }
        }
        ar.lds_used = (uint32_t)(mark & 0xffffffffu);
        ar.slab_used = mark >> 32;
    }
}

__device__ void enum_flush(Slot *slots, uint32_t slot, Acc &acc, Counters &ct, bool instrument)
{
    acc_flush(acc);
    wave_flush(slots, slot, acc.v, acc.ovf, ct.pair_words, ct.filter_words);
    if (instrument && lane_id() == 0) {
        atomicAdd(&slots[slot].cyc_setup, ct.cyc_setup);
        atomicAdd(&slots[slot].cyc_compact, ct.cyc_compact);
        atomicAdd(&slots[slot].cyc_pair, ct.cyc_pair);
        atomicAdd(&slots[slot].cyc_filter, ct.cyc_filter);
        atomicAdd(&slots[slot].pairs, ct.pairs);
        atomicAdd(&slots[slot].pair_slots, ct.pair_slots);
        atomicAdd(&slots[slot].cyc_pack, ct.cyc_pack);
    }
    acc.v = 0;
    acc.ovf = false;
    ct = Counters{};
}

// Three waves per SIMD (12 per CU): the register budget is capped at 168 VGPRs.
// SPLIT = runtime splitting of heavy tasks (the subtask ring and its drain);
// the plain variant carries none of that code.
template <bool SPLIT>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_enumerate(
    EnumParams prm)
{
    __shared__ uint64_t lds[kWavesPerBlock][kLdsWordsPerWave];
    __shared__ uint64_t tbl[kWavesPerBlock][kTableLen];
    __shared__ uint32_t tbl32[kWavesPerBlock][kTableLen];
    __shared__ uint64_t tiles[kWavesPerBlock][kWaveSize * kTileWords];
    const uint32_t wv = threadIdx.x / kWaveSize, ln = lane_id();
    const uint64_t wave_global = (uint64_t)blockIdx.x * kWavesPerBlock + wv;
    static_assert(kBlockThreads == 256, "one spread-table entry per thread");
    spread_lut[threadIdx.x] = spread_lut_entry(threadIdx.x);
    __syncthreads();
    uint64_t *stack = &lds[wv][0];
    Arena arena;
    arena.lds = &lds[wv][kStackWords];
    arena.lds_cap = (prm.lds_words > kStackWords ? min(prm.lds_words, kLdsWordsPerWave) : kStackWords) - kStackWords;
    arena.lds_used = 0;
    arena.slab = prm.slab + wave_global * prm.slab_words;
    arena.slab_cap = prm.slab_words;
    arena.slab_used = 0;
    Table tb;
    tb.t = &tbl[wv][0];
    tb.t32 = &tbl32[wv][0];
    tb.tile = &tiles[wv][0];
    tb.job = 0xffffffffu;
    tb.len = 0;
    const bool instrument = prm.instrument != 0;

    Acc acc;
    acc.v = 0;
    acc.ovf = false;
    acc.t = 0;
    Counters ct{};
    uint32_t cur_job = 0xffffffffu;
    // With splitting on, a wavefront counts itself as a producer (the high
    // bits of the queue word) in the same atomic that pops its chunk, and
    // leaves that count, with release order after its ring entries, once the
    // chunk is done; the drain below uses the count to know when no more
    // subtasks can appear.
    constexpr bool split = SPLIT;
    const unsigned long long kProducer = 1ull << 40, kPopMask = kProducer - 1;
    const unsigned long long t_start = instrument ? __builtin_amdgcn_s_memrealtime() : 0ull;
    SplitCtx sp;
    sp.ring = prm.ring;
    sp.tail = prm.sub_tail;
    sp.heap = prm.split_heap;
    sp.heap_used = prm.sub_head + 2;
    sp.heap_cap = prm.split_heap_words;
    sp.cap = prm.split_cap;
    sp.rows = prm.split_rows;
    sp.root_idx = 0;
    for (;;) {
        // pop task_chunk consecutive tasks; only the first needs the root
        // search, the rest advance through the (contiguous) task ranges
        unsigned long long t0 = 0;
        if (ln == 0) t0 = atomicAdd(prm.queue, (unsigned long long)prm.task_chunk + (split ? kProducer : 0ull));
        t0 = bcast64(t0, 0) & kPopMask;
        if (t0 >= prm.n_tasks) {
            if (split && ln == 0)
                __hip_atomic_fetch_add(prm.queue, 0ull - kProducer, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            break;
        }
        const unsigned long long t_end = min(t0 + prm.task_chunk, (unsigned long long)prm.n_tasks);
        // root owning task t0: largest r with roots[r].task_begin <= t0
        uint32_t r = 0, hi = prm.n_roots;
        while (hi - r > 1) {
            const uint32_t mid = (r + hi) >> 1;
            if (prm.roots[mid].task_begin <= t0) r = mid;
            else hi = mid;
        }
        ActiveRoot rt = prm.roots[r];
        for (unsigned long long t = t0; t < t_end; ++t) {
            while (t >= rt.task_begin + rt.n_tasks) rt = prm.roots[++r];   // every active root owns >= 1 task
            if (rt.job != cur_job) {
                if (cur_job != 0xffffffffu) enum_flush(prm.slots, prm.jobs[cur_job].slot, acc, ct, instrument);
                cur_job = rt.job;
            }
            const Job jb = prm.jobs[rt.job];
            bool cap_fail = false, timed_out = past_deadline(jb.deadline);
            sp.root_idx = r;
            if (!timed_out)
                run_task<SPLIT>(jb, rt.job, rt, (uint32_t)(t - rt.task_begin), prm.pool, arena, stack, tb, acc, ct,
                                instrument, prm.triple != 0, &sp, &cap_fail, &timed_out);
            if (cap_fail && ln == 0) atomicOr(&prm.slots[jb.slot].flags, FLAG_CAPACITY);
            if (timed_out && ln == 0) atomicOr(&prm.slots[jb.slot].flags, FLAG_TIMEOUT);
        }
        if (split && ln == 0)
            __hip_atomic_fetch_add(prm.queue, 0ull - kProducer, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }

    // Drain the subtask ring.  Each wavefront claims one entry index at a
    // time.  It waits while the entry is reserved but not yet published (its
    // producer is running and publishes it right after the reservation), or
    // while the index is past the reserved entries but some producer is still
    // running a chunk (it may reserve more).  Once no producer is left, the
    // reserved count is final: an index at or past it, or past the ring, will
    // never be filled and the wavefront is done.  Producers only run popped
    // chunks, so every wait ends when they finish their (finite) tasks.
    while (SPLIT) {
        unsigned long long h = 0;
        if (ln == 0) h = atomicAdd(prm.sub_head, 1ull);
        h = bcast64(h, 0);
        uint32_t state = 0;   // 0 wait, 1 entry ready, 2 done
        for (;;) {
            if (ln == 0) {
                if (h >= prm.split_cap) {
                    state = 2;
                } else {
                    const unsigned long long tl =
                        __hip_atomic_load(prm.sub_tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                    if (h < tl) {
                        if (__hip_atomic_load(&prm.ring[h].w, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0)
                            state = 1;
                    } else {
                        const unsigned long long v =
                            __hip_atomic_load(prm.queue, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                        if ((v >> 40) == 0 &&
                            h >= __hip_atomic_load(prm.sub_tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT))
                            state = 2;
                    }
                }
            }
            state = (uint32_t)__builtin_amdgcn_readfirstlane(state);
            if (state != 0) break;
            __builtin_amdgcn_s_sleep(4);
        }
        if (state == 2) break;
        uint32_t elo = 0, ehi = 0, ea = 0;
        if (ln == 0) {
            const uint4 e = prm.ring[h];
            elo = e.x;
            ehi = e.y;
            ea = e.z;
        }
        elo = (uint32_t)__builtin_amdgcn_readfirstlane(elo);
        ehi = (uint32_t)__builtin_amdgcn_readfirstlane(ehi);
        ea = (uint32_t)__builtin_amdgcn_readfirstlane(ea);
        // the parent's level-2 block and its header (written before the entry was published)
        const uint64_t *hdr = prm.split_heap + (((uint64_t)ehi << 32) | elo);
        const uint32_t er = (uint32_t)hdr[0];
        const uint32_t hm2 = (uint32_t)hdr[2], hW2 = (uint32_t)(hdr[2] >> 32), hs2n = (uint32_t)hdr[3];
        const ActiveRoot rt = prm.roots[er];
        if (rt.job != cur_job) {
            if (cur_job != 0xffffffffu) enum_flush(prm.slots, prm.jobs[cur_job].slot, acc, ct, instrument);
            cur_job = rt.job;
        }
        const Job jb = prm.jobs[rt.job];
        bool cap_fail = false, timed_out = past_deadline(jb.deadline);
        if (!timed_out) {
            Arena ar = arena;
            dfs_level2(jb, rt.job, hdr + 4, hm2, hm2, hW2, hs2n, ea, ar, stack, tb, acc, ct, instrument,
                       prm.triple != 0, &cap_fail, &timed_out, instrument ? cycles() : 0);
        }
        if (cap_fail && ln == 0) atomicOr(&prm.slots[jb.slot].flags, FLAG_CAPACITY);
        if (timed_out && ln == 0) atomicOr(&prm.slots[jb.slot].flags, FLAG_TIMEOUT);
    }
    if (cur_job != 0xffffffffu) enum_flush(prm.slots, prm.jobs[cur_job].slot, acc, ct, instrument);
    if (instrument && prm.wave_clock && ln == 0) {
        // when this wavefront started and ran out of work (load balance)
        prm.wave_clock[2 * wave_global] = t_start;
        prm.wave_clock[2 * wave_global + 1] = __builtin_amdgcn_s_memrealtime();
    }
}

hipError_t launch_enumerate(const EnumParams &prm, uint32_t n_blocks, hipStream_t stream)
{
    if (prm.n_tasks == 0) return hipSuccess;
    if (prm.split_cap != 0) hipLaunchKernelGGL(k_enumerate<true>, dim3(n_blocks), dim3(kBlockThreads), 0, stream, prm);
    else hipLaunchKernelGGL(k_enumerate<false>, dim3(n_blocks), dim3(kBlockThreads), 0, stream, prm);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Global-set path: the search of Algorithm 1 with its intersections done on
// the graph's own adjacency instead of per-root local bitmaps.  Candidate
// sets C_L are id lists; common-neighbour sets C_R are kept either as HTB
// words (Section V-A: word index i and a 32-bit value whose bit j is B id
// 32i + j) or as sorted id lists (word = id, value 1).  An intersection
// C_R n N(c) is the two-phase HTB one: each element's index is
// binary-searched in c's row, then the values are ANDed; with sorted lists
// it is the plain binary search of Section III-B (a value of 1 on both
// sides).  Lanes take 64 candidates at a time (Section IV's BFS over
// siblings); descending to a child intersects the node's set with the
// child's row, the wave's lanes taking its elements.

// k_cand_ids: for every global-set root, the ids w > u with |N(u) n N(w)| >=
// qA (dense per-block counters as in k_cand_count), in the order met.
__global__ __launch_bounds__(kBlockThreads) void k_cand_ids(const Job *jobs, const SetRoot *roots, uint32_t n_roots,
                                                            uint32_t *ids, RootScratch sc, unsigned long long *queue,
                                                            Slot *slots)
{
    __shared__ unsigned long long s_item;
    __shared__ uint32_t s_nt, s_k;
    uint32_t *cnt = sc.cnt + (uint64_t)blockIdx.x * sc.stride;
    uint32_t *touched = sc.touched + (uint64_t)blockIdx.x * sc.stride;
    const uint32_t tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            s_item = atomicAdd(queue, 1ull);
            s_nt = 0;
            s_k = 0;
        }
        __syncthreads();
        const uint64_t item = s_item;
        if (item >= n_roots) break;
        const SetRoot rt = roots[item];
        const Job jb = jobs[rt.job];
        const uint32_t u = rt.root;
        const uint64_t ub = jb.ptrA[u];
        const uint32_t du = (uint32_t)(jb.ptrA[u + 1] - ub);
        oriented_wedges(jb, u, ub, du, [&](uint32_t, uint32_t w) {
            if (atomicAdd(&cnt[w], 1u) == 0u) touched[atomicAdd(&s_nt, 1u)] = w;
        });
        __syncthreads();
        const uint32_t nt = s_nt;
        for (uint32_t t = tid; t < nt; t += kBlockThreads) {
            const uint32_t w = touched[t];
            const uint32_t c = atomicExch(&cnt[w], 0u);
            if (c >= jb.qA) {
                const uint32_t at = atomicAdd(&s_k, 1u);
                if (at < rt.k) ids[rt.id_off + at] = w;
            }
        }
        __syncthreads();
        // the candidate pass counted the same set: a different size is an internal error
        if (tid == 0 && s_k != rt.k) atomicOr(&slots[jb.slot].flags, FLAG_MISMATCH);
        __syncthreads();
    }
}

hipError_t launch_cand_ids(const Job *jobs, const SetRoot *roots, uint32_t n_roots, uint32_t *ids,
                           RootScratch scratch, uint32_t n_blocks, unsigned long long *queue, Slot *slots,
                           hipStream_t stream)
{
    if (n_roots == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cand_ids, dim3(n_blocks), dim3(kBlockThreads), 0, stream, jobs, roots, n_roots, ids,
                       scratch, queue, slots);
    return hipGetLastError();
}

template <uint32_t MODE>
__device__ __forceinline__ uint64_t row_begin(const Job &jb, uint32_t x)
{
    return MODE == SETS_HTB ? jb.htb_off[x] : jb.ptrA[x];
}
template <uint32_t MODE>
__device__ __forceinline__ uint32_t row_key(const Job &jb, uint64_t e)
{
    return MODE == SETS_HTB ? jb.htb_idx[e] : jb.adjA[e];
}
template <uint32_t MODE>
__device__ __forceinline__ uint32_t row_val(const Job &jb, uint64_t e)
{
    return MODE == SETS_HTB ? jb.htb_val[e] : 1u;
}

// First position in [lo, hi) of x's row whose key is >= key.
template <uint32_t MODE>
__device__ __forceinline__ uint64_t row_lower_bound(const Job &jb, uint64_t lo, uint64_t hi, uint32_t key)
{
    while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (row_key<MODE>(jb, mid) < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// |S n N(c)| in this lane, S = m packed elements (key << 32 | value) sorted
// by key: each element is searched in what is left of c's row.
template <uint32_t MODE>
__device__ uint32_t set_count(const Job &jb, const uint64_t *S, uint32_t m, uint32_t c)
{
    uint64_t lo = row_begin<MODE>(jb, c);
    const uint64_t hi = row_begin<MODE>(jb, c + 1);
    uint32_t n = 0;
    for (uint32_t e = 0; e < m && lo < hi; ++e) {
        const uint64_t x = S[e];
        const uint32_t key = (uint32_t)(x >> 32);
        lo = row_lower_bound<MODE>(jb, lo, hi, key);
        if (lo < hi && row_key<MODE>(jb, lo) == key) n += (uint32_t)__popc((uint32_t)x & row_val<MODE>(jb, lo));
    }
    return n;
}

// out = S n N(c), its elements with a nonzero value, in key order; the wave's
// lanes take S's elements.  S is either a packed set (from_row false) or the
// row of vertex `from` itself.  Returns the element count; *bits gets the
// number of members.
template <uint32_t MODE>
__device__ uint32_t set_intersect(const Job &jb, const uint64_t *S, uint32_t m, bool from_row, uint32_t from,
                                  uint32_t c, uint64_t *out, uint32_t *bits)
{
    const uint32_t ln = lane_id();
    const uint64_t c0 = row_begin<MODE>(jb, c), c1 = row_begin<MODE>(jb, c + 1);
    const uint64_t f0 = from_row ? row_begin<MODE>(jb, from) : 0;
    uint32_t k = 0, nb = 0;
    for (uint32_t e0 = 0; e0 < m; e0 += kWaveSize) {
        const uint32_t e = e0 + ln;
        uint64_t r = 0;
        if (e < m) {
            uint32_t key, val;
            if (from_row) {
                key = row_key<MODE>(jb, f0 + e);
                val = row_val<MODE>(jb, f0 + e);
            } else {
                key = (uint32_t)(S[e] >> 32);
                val = (uint32_t)S[e];
            }
            const uint64_t pos = row_lower_bound<MODE>(jb, c0, c1, key);
            if (pos < c1 && row_key<MODE>(jb, pos) == key) {
                const uint32_t w = val & row_val<MODE>(jb, pos);
                if (w) r = ((uint64_t)key << 32) | w;
            }
        }
        const bool keep = r != 0;
        const uint64_t mask = __ballot(keep);
        if (keep) out[k + mbcnt64(mask)] = r;
        k += (uint32_t)__popcll(mask);
        nb += (uint32_t)__popc((uint32_t)r);
    }
    wave_sync();
    *bits = (uint32_t)wave_sum_u64(nb);
    return k;
}

// |S n N(c)| with the wave's lanes over S's elements, for one candidate c
// (the search without the BFS over siblings: each intersection in turn).
template <uint32_t MODE>
__device__ uint32_t set_count_wave(const Job &jb, const uint64_t *S, uint32_t m, uint32_t c)
{
    const uint32_t ln = lane_id();
    const uint64_t c0 = row_begin<MODE>(jb, c), c1 = row_begin<MODE>(jb, c + 1);
    uint32_t n = 0;
    for (uint32_t e0 = 0; e0 < m; e0 += kWaveSize) {
        const uint32_t e = e0 + ln;
        if (e < m) {
            const uint64_t x = S[e];
            const uint32_t key = (uint32_t)(x >> 32);
            const uint64_t pos = row_lower_bound<MODE>(jb, c0, c1, key);
            if (pos < c1 && row_key<MODE>(jb, pos) == key) n += (uint32_t)__popc((uint32_t)x & row_val<MODE>(jb, pos));
        }
    }
    return (uint32_t)wave_sum_u64(n);
}

constexpr uint32_t kSetLdsWords = 512;    // LDS part of each wave's arena in the global-set kernel
constexpr uint32_t kSetLevels = 33;       // DFS levels (p_A <= 32)

// One (root, second vertex) task of the global-set path: node {u, c_i},
// then the DFS of Algorithm 1 down to |L| = pA - 1, whose candidates each
// add C(|C_R n N(c)|, q).  Per level: the node's set S (arena), its
// candidate list (a suffix of the parent's kept list), the kept list and a
// cursor.
// HYBRID: the 64 lanes take 64 siblings at a time (Section IV's BFS over
// siblings); otherwise the siblings are visited one at a time and the lanes
// share each intersection (the pure DFS the paper's ablation compares with).
template <uint32_t MODE, bool HYBRID>
__device__ void run_set_task(const Job &jb, const SetRoot &rt, uint32_t i, const uint32_t *ids, Arena ar,
                             uint64_t *stk, Acc &acc, Counters &ct, bool instrument, bool *cap_fail, bool *timed_out)
{
    const uint32_t ln = lane_id();
    const uint32_t q = jb.qA, pA = jb.pA, k = rt.k;
    const uint32_t *cid = ids + rt.id_off;
    const uint32_t u = rt.root;
    // level-2 node {u, c_i}: S = N(u) n N(c_i), candidates c_{i+1} ..
    const uint32_t mu = (uint32_t)(row_begin<MODE>(jb, u + 1) - row_begin<MODE>(jb, u));
    uint64_t *S = arena_alloc(ar, mu, cap_fail);
    if (!S) return;
    uint32_t bits = 0;
    uint32_t m = set_intersect<MODE>(jb, nullptr, mu, true, u, cid[i], S, &bits);
    if (instrument) ct.filter_words += mu;
    if (bits < q) return;
    if (pA == 2) {
        // only with per-vertex counts (the candidate pass sums these leaves):
        // L = {u, c_i} holds C(|S|, q) bicliques
        if (jb.pv && ln == 0) {
            if (bits >= jb.n_ovf) {
                acc.ovf = true;
            } else {
                pv_add(jb.pv, u, jb.binom[bits]);
                pv_add(jb.pv, cid[i], jb.binom[bits]);
            }
        }
        return;
    }
    // Saved per level d while a child is explored (wave-private LDS stack):
    // stk[8d] = S, [8d+1] = its element count, [8d+2] = kept list, [8d+3] =
    // cursor << 32 | kept count, [8d+4] = candidates, [8d+5] = their number,
    // [8d+6], [8d+7] = arena state before the kept list was taken.
    uint32_t d = 2;
    const uint32_t *C = cid + i + 1;
    uint32_t nc = k - i - 1;
    bool fresh = true;
    uint32_t *K = nullptr;
    uint32_t nk = 0, t = 0;
    for (;;) {
        if (fresh) {
            fresh = false;
            if (past_deadline(jb.deadline)) {
                *timed_out = true;
                return;
            }
            if (d + 1 == pA) {
                // leaves: every candidate c of this node adds C(|S n N(c)|, q)
                if (HYBRID) {
                    u128 node = 0;   // per-vertex counts: the node's leaves, for its members
                    for (uint32_t b0 = 0; b0 < nc; b0 += kWaveSize) {
                        const uint32_t b = b0 + ln;
                        if (b < nc) {
                            const uint32_t n = set_count<MODE>(jb, S, m, C[b]);
                            if (n >= q) {
                                leaf_add(acc, jb.binom, jb.n_ovf, n);
                                if (jb.pv && n < jb.n_ovf) {
                                    pv_add(jb.pv, C[b], jb.binom[n]);
                                    acc.ovf |= __builtin_add_overflow(node, jb.binom[n], &node);
                                }
                            }
                        }
                    }
                    if (jb.pv) {
                        // the node's members: the root, c_i and the vertex each
                        // level 2 .. d-1 descended into (its kept list's entry
                        // before the saved cursor)
                        bool o = false;
                        const u128 tot = wave_sum_u128(node, &o);
                        acc.ovf |= o;
                        if (ln == 0 && tot != 0) {
                            pv_add(jb.pv, u, tot);
                            pv_add(jb.pv, cid[i], tot);
                            for (uint32_t dd = 2; dd < d; ++dd) {
                                const uint32_t *Kd = (const uint32_t *)(uintptr_t)stk[8 * dd + 2];
                                pv_add(jb.pv, Kd[(uint32_t)(stk[8 * dd + 3] >> 32) - 1], tot);
                            }
                        }
                    }
                } else {
                    for (uint32_t b = 0; b < nc; ++b) {
                        const uint32_t n = set_count_wave<MODE>(jb, S, m, C[b]);
                        if (ln == 0 && n >= q) leaf_add(acc, jb.binom, jb.n_ovf, n);
                    }
                }
                if (instrument) ct.filter_words += (unsigned long long)nc * m;
                goto pop;
            }
            // keep the candidates that leave at least q common neighbours
            stk[8 * d + 6] = ar.lds_used;
            stk[8 * d + 7] = ar.slab_used;
            K = (uint32_t *)arena_alloc(ar, (nc + 1) / 2 + 1, cap_fail);
            if (!K) return;
            nk = 0;
            if (HYBRID) {
                for (uint32_t b0 = 0; b0 < nc; b0 += kWaveSize) {
                    const uint32_t b = b0 + ln;
                    const bool valid = b < nc;
                    const uint32_t c = valid ? C[b] : 0u;
                    const bool keep = valid && set_count<MODE>(jb, S, m, c) >= q;
                    const uint64_t mask = __ballot(keep);
                    if (keep) K[nk + mbcnt64(mask)] = c;
                    nk += (uint32_t)__popcll(mask);
                }
            } else {
                for (uint32_t b = 0; b < nc; ++b) {
                    const uint32_t c = C[b];
                    if (set_count_wave<MODE>(jb, S, m, c) >= q) {
                        if (ln == 0) K[nk] = c;
                        ++nk;
                    }
                }
            }
            wave_sync();
            if (instrument) ct.filter_words += (unsigned long long)nc * m;
            t = 0;
        }
        // next child {.., K[t]}: it needs pA - d vertices from K[t ..]
        if (nk - t < pA - d) goto pop;
        {
            const uint32_t a = K[t++];
            // save this level, then build the child's set
            stk[8 * d + 0] = (uint64_t)(uintptr_t)S;
            stk[8 * d + 1] = m;
            stk[8 * d + 2] = (uint64_t)(uintptr_t)K;
            stk[8 * d + 3] = ((uint64_t)t << 32) | nk;
            stk[8 * d + 4] = (uint64_t)(uintptr_t)C;
            stk[8 * d + 5] = nc;
            wave_sync();
            uint64_t *S2 = arena_alloc(ar, m, cap_fail);
            if (!S2) return;
            uint32_t nb = 0;
            const uint32_t m2 = set_intersect<MODE>(jb, S, m, false, 0, a, S2, &nb);
            if (instrument) ct.filter_words += m;
            S = S2;
            m = m2;
            C = K + t;
            nc = nk - t;
            ++d;
            fresh = true;
            continue;
        }
    pop:
        if (d == 2) return;
        --d;
        // release the child's allocations (its set and kept list): back to
        // the marks taken before this level's kept list, plus that list
        {
            S = (uint64_t *)(uintptr_t)stk[8 * d + 0];
            m = (uint32_t)stk[8 * d + 1];
            K = (uint32_t *)(uintptr_t)stk[8 * d + 2];
            t = (uint32_t)(stk[8 * d + 3] >> 32);
            nk = (uint32_t)stk[8 * d + 3];
            C = (const uint32_t *)(uintptr_t)stk[8 * d + 4];
            nc = (uint32_t)stk[8 * d + 5];
            const uint32_t kw = (nc + 1) / 2 + 1;
            ar.lds_used = (uint32_t)stk[8 * d + 6];
            ar.slab_used = stk[8 * d + 7];
            // re-take the kept list's words at the same place (it is still there)
            bool f = false;
            uint32_t *K2 = (uint32_t *)arena_alloc(ar, kw, &f);
            if (K2 != K) {   // cannot happen: the same request from the same state
                *cap_fail = true;
                return;
            }
        }
    }
}

template <uint32_t MODE, bool HYBRID>
__global__ __launch_bounds__(kBlockThreads) void k_enumerate_sets(SetParams prm)
{
    __shared__ uint64_t lds[kWavesPerBlock][kSetLdsWords];
    __shared__ uint64_t stk[kWavesPerBlock][8 * kSetLevels];
    const uint32_t wv = threadIdx.x / kWaveSize, ln = lane_id();
    const uint64_t wave_global = (uint64_t)blockIdx.x * kWavesPerBlock + wv;
    Arena arena;
    arena.lds = &lds[wv][0];
    arena.lds_cap = kSetLdsWords;
    arena.lds_used = 0;
    arena.slab = prm.slab + wave_global * prm.slab_words;
    arena.slab_cap = prm.slab_words;
    arena.slab_used = 0;
    const bool instrument = prm.instrument != 0;
    Acc acc;
    acc.v = 0;
    acc.ovf = false;
    acc.t = 0;
    Counters ct{};
    uint32_t cur_job = 0xffffffffu;
    for (;;) {
        unsigned long long t0 = 0;
        if (ln == 0) t0 = atomicAdd(prm.queue, (unsigned long long)prm.task_chunk);
        t0 = bcast64(t0, 0);
        if (t0 >= prm.n_tasks) break;
        const unsigned long long t_end = min(t0 + prm.task_chunk, (unsigned long long)prm.n_tasks);
        uint32_t r = 0, hi = prm.n_roots;
        while (hi - r > 1) {
            const uint32_t mid = (r + hi) >> 1;
            if (prm.roots[mid].task_begin <= t0) r = mid;
            else hi = mid;
        }
        SetRoot rt = prm.roots[r];
        for (unsigned long long t = t0; t < t_end; ++t) {
            while (t >= rt.task_begin + rt.n_tasks) rt = prm.roots[++r];   // every root owns >= 1 task
            if (rt.job != cur_job) {
                if (cur_job != 0xffffffffu) enum_flush(prm.slots, prm.jobs[cur_job].slot, acc, ct, instrument);
                cur_job = rt.job;
            }
            const Job jb = prm.jobs[rt.job];
            bool cap_fail = false, timed_out = past_deadline(jb.deadline);
            if (!timed_out)
                run_set_task<MODE, HYBRID>(jb, rt, (uint32_t)(t - rt.task_begin), prm.ids, arena, &stk[wv][0], acc,
                                           ct, instrument, &cap_fail, &timed_out);
            if (cap_fail && ln == 0) atomicOr(&prm.slots[jb.slot].flags, FLAG_CAPACITY);
            if (timed_out && ln == 0) atomicOr(&prm.slots[jb.slot].flags, FLAG_TIMEOUT);
        }
    }
    if (cur_job != 0xffffffffu) enum_flush(prm.slots, prm.jobs[cur_job].slot, acc, ct, instrument);
}

hipError_t launch_enumerate_sets(const SetParams &prm, uint32_t n_blocks, hipStream_t stream)
{
    if (prm.n_tasks == 0) return hipSuccess;
    const bool hybrid = prm.pure_dfs == 0;
    if (prm.mode == SETS_HTB && hybrid)
        hipLaunchKernelGGL((k_enumerate_sets<SETS_HTB, true>), dim3(n_blocks), dim3(kBlockThreads), 0, stream, prm);
    else if (prm.mode == SETS_HTB)
        hipLaunchKernelGGL((k_enumerate_sets<SETS_HTB, false>), dim3(n_blocks), dim3(kBlockThreads), 0, stream, prm);
    else if (hybrid)
        hipLaunchKernelGGL((k_enumerate_sets<SETS_SORTED, true>), dim3(n_blocks), dim3(kBlockThreads), 0, stream,
                           prm);
    else
        hipLaunchKernelGGL((k_enumerate_sets<SETS_SORTED, false>), dim3(n_blocks), dim3(kBlockThreads), 0, stream,
                           prm);
    return hipGetLastError();
}

}  // namespace bcdev
