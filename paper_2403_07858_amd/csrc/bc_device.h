// Shared declarations between the host library and the HIP kernels of the
// biclique counter.  Device-side structures hold plain pointers into HBM.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bcdev {

typedef unsigned __int128 u128;

// One counting job: (graph side pair, p, q, root range) -> one result slot.
// "A" is the anchor side (L is drawn from it), "B" the other side.  Both CSRs
// are relabelled by rank, so orientation "w ranked after u" is "w > u".
struct Job {
    const uint64_t *ptrA;   // nA + 1
    const uint32_t *adjA;   // N(u) as sorted B ids
    const uint32_t *rposA;  // per edge u - v of adjA: position of u within N(v)
    const uint64_t *ptrB;   // nB + 1
    const uint32_t *adjB;   // N(v) as sorted A ids
    const u128 *binom;      // binom[n] = C(n, qA) for n in [0, binom_n)
    uint32_t nA, nB;
    uint32_t root_lo, root_hi;  // roots counted: ranks in [root_lo, root_hi)
    uint32_t pA, qA;
    uint32_t binom_n;       // table length (max degree of A + 1)
    uint32_t n_ovf;         // smallest n with C(n, qA) >= 2^128 (binom_n if none)
    uint32_t slot;          // result slot
    uint32_t n_u64;         // largest n with C(n, qA) < 2^64
    uint64_t deadline;      // device real-time clock tick after which the job gives up (0 = none)
    uint32_t n_u58;         // largest n with C(n, qA) < 2^58 (64 such values add up in 64 bits)
    uint32_t n_u28;         // largest n with C(n, qA) < 2^28 (16 such values add up in 32 bits)
    // hierarchical truncated bitmap of side A's rows (Section V-A): the row of
    // x is the 32-bit words htb_idx/htb_val[htb_off[x] .. htb_off[x+1]), word
    // i holding B ids 32i .. 32i+31 (bit j = id 32i + j); NULL when unused
    const uint64_t *htb_off;
    const uint32_t *htb_idx;
    const uint32_t *htb_val;
    // per-vertex counts of side A (two 64-bit words per vertex, by rank): the
    // bicliques each vertex is an L member of; NULL when not asked for (only
    // the global-set path fills them)
    uint64_t *pv;
};

// One root of the global-set path (set intersections over the graph's own
// adjacency: HTB words or sorted id lists), in schedule order.
struct SetRoot {
    uint64_t id_off;        // its candidate ids: ids[id_off .. id_off + k)
    uint64_t task_begin;    // global index of its first task
    uint32_t job;
    uint32_t root;
    uint32_t k;
    uint32_t n_tasks;       // k - (pA - 2)
};

enum : uint32_t { SETS_HTB = 1, SETS_SORTED = 2 };

struct Slot;

struct SetParams {
    const Job *jobs;
    const SetRoot *roots;
    uint32_t n_roots;
    uint32_t task_chunk;
    uint64_t n_tasks;
    const uint32_t *ids;    // candidate ids of every root
    uint32_t mode;          // SETS_HTB or SETS_SORTED
    uint32_t instrument;
    uint32_t pure_dfs;      // nonzero: siblings one at a time, the lanes sharing each intersection
    uint32_t pad;
    uint64_t *slab;         // per-wave scratch
    uint64_t slab_words;
    unsigned long long *queue;
    Slot *slots;
};

// One root that owns enumeration tasks, in schedule (cost) order.
struct ActiveRoot {
    uint64_t pool_off;      // first word of its candidate rows in the pool
    uint64_t task_begin;    // global index of its first task
    uint32_t job;
    uint32_t root;          // anchor-side vertex (rank)
    uint32_t k;             // number of candidates (rows)
    uint32_t n_tasks;       // candidates that start a task: k - (pA - 2)
};

// Result slot: exact 128-bit count as two 64-bit limbs plus status flags.
struct Slot {
    unsigned long long lo, hi;
    unsigned int flags;     // FLAG_* bits
    unsigned int pad;
    unsigned long long pair_ops, filter_ops;
    unsigned long long cyc_setup, cyc_compact, cyc_pair, cyc_filter;   // instrumented shader-clock sums
    unsigned long long pairs, pair_slots;   // instrumented: leaf pairs, and lane-slots spent on them
    unsigned long long cyc_pack;            // instrumented: compaction cycles of tasks that bit-pack S2
    unsigned long long pad3;
};

enum : unsigned {
    FLAG_OVERFLOW = 1u,     // count does not fit in 128 bits
    FLAG_CAPACITY = 2u,     // a scratch bound computed on the host was exceeded
    FLAG_MISMATCH = 4u,     // candidate count differs between the two wedge passes
    FLAG_TIMEOUT = 8u,      // the job's deadline passed before it finished
    FLAG_POOL = 16u,        // the row pool was too small for some root (rows built again)
};

constexpr int kWaveSize = 64;
constexpr int kWavesPerBlock = 4;
constexpr uint32_t kTripleRows = 96;   // nodes up to this many rows finish their last three levels at once
constexpr int kBlockThreads = kWaveSize * kWavesPerBlock;
constexpr int kSortCap = 4096;          // candidates sorted in LDS up to this many
constexpr int kRbWaves = 16;            // waves per block of the fused per-root kernel
constexpr int kRbThreads = kWaveSize * kRbWaves;
constexpr uint32_t kSlotFlag = 0x80000000u;

struct RootScratch {
    uint32_t *cnt;          // per block: nA_max counters, all zero between roots
    uint32_t *touched;      // per block: nA_max touched ids
    uint32_t *cand;         // per block: nA_max candidate ids (when k > kSortCap)
    uint64_t stride;        // elements per block in each array
};

struct EnumParams {
    const Job *jobs;
    const ActiveRoot *roots;
    uint32_t n_roots;
    uint32_t task_chunk;    // consecutive tasks taken per queue pop (>= 1)
    uint64_t n_tasks;
    const uint64_t *pool;
    uint64_t *slab;         // per-wave global scratch
    uint64_t slab_words;    // words per wave
    uint32_t lds_words;     // per-wave LDS words actually used (<= compiled cap)
    uint32_t instrument;
    uint32_t triple;        // nonzero: small nodes three levels above the leaves take the triple sweep
    uint32_t split_rows;    // level-2 blocks with more rows are split into queued subtasks
    uint32_t split_cap;     // subtask ring entries (0 = no splitting)
    uint4 *ring;            // subtask ring, split_cap entries, all zero at launch
    unsigned long long *sub_head;   // [0] subtask entries claimed, [2] split heap words taken (zero at launch)
    unsigned long long *sub_tail;   // subtask entries reserved (zero at launch)
    uint64_t *split_heap;   // level-2 blocks of split tasks
    uint64_t split_heap_words;
    unsigned long long *wave_clock; // instrumented: per wavefront {first task start, end} device clock ticks
    unsigned long long *queue;   // task counter: tasks popped in the low 40 bits; with splitting on,
                                 // wavefronts still running a popped chunk in the bits above
    Slot *slots;
};

// Launchers (defined in bc_kernels.hip).  All run on `stream` and return the
// launch status.
hipError_t launch_fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t stream);
hipError_t launch_fill_slots(Slot *slots, uint32_t n, hipStream_t stream);
hipError_t launch_degree_sum(const Job *jobs, const uint32_t *job_ids, uint32_t n_jobs,
                             Slot *slots, hipStream_t stream);
hipError_t launch_cand_count(const Job *jobs, const uint64_t *job_root_prefix, uint32_t n_jobs,
                             uint64_t total_roots, RootScratch scratch, uint32_t n_blocks,
                             unsigned long long *queue, uint32_t *out_k, Slot *slots,
                             hipStream_t stream);
// Candidate counts and rows in one kernel; rows go to pool[out_off[r] ..]
// (bump-allocated from counters[1], capacity pool_cap words; out_off = ~0 when
// a root has no rows).  counters[0] is the root queue.  Blocks of kRbThreads
// threads with 144 KiB of LDS each.
hipError_t launch_root_build(const Job *jobs, const uint64_t *job_root_prefix, uint32_t n_jobs,
                             uint64_t total_roots, RootScratch scratch, uint64_t *pool, uint64_t pool_cap,
                             uint32_t n_blocks, unsigned long long *counters, uint32_t *out_k, uint64_t *out_off,
                             Slot *slots, bool per_vertex, hipStream_t stream);
hipError_t launch_rows_build(const Job *jobs, const ActiveRoot *roots, uint32_t n_roots,
                             uint64_t *pool, RootScratch scratch, uint32_t n_blocks,
                             unsigned long long *queue, Slot *slots, hipStream_t stream);
hipError_t launch_enumerate(const EnumParams &prm, uint32_t n_blocks, hipStream_t stream);
// Candidate ids of the global-set roots: for root r, the w > u sharing >= qA
// neighbours with u, in no particular order, written to ids[roots[r].id_off ..].
hipError_t launch_cand_ids(const Job *jobs, const SetRoot *roots, uint32_t n_roots, uint32_t *ids,
                           RootScratch scratch, uint32_t n_blocks, unsigned long long *queue, Slot *slots,
                           hipStream_t stream);
hipError_t launch_enumerate_sets(const SetParams &prm, uint32_t n_blocks, hipStream_t stream);

uint32_t max_lds_words_per_wave();

// Reads the device real-time clock (s_memrealtime) into *out (device memory).
hipError_t launch_read_clock(uint64_t *out, hipStream_t stream);

}  // namespace bcdev
