// Host side of the biclique counter: input validation, degree-order
// relabelling, device residency of graphs, per-query planning and the C ABI
// declared in include/bc.h.
#include "bc.h"

#include <algorithm>
#include <atomic>
#include <cstddef>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <queue>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bc_device.h"
#include "bc_internal.h"

using bcdev::u128;

namespace {

thread_local std::string g_last_error;

bc_status set_error(bc_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

// A failed HIP call: out of device memory is BC_E_OOM, anything else BC_E_DEVICE.
bc_status hip_error(hipError_t e, const char *what)
{
    return set_error(e == hipErrorOutOfMemory ? BC_E_OOM : BC_E_DEVICE,
                     std::string(what) + ": " + hipGetErrorString(e));
}

#define BC_HIP(call)                                             \
    do {                                                         \
        hipError_t e_ = (call);                                  \
        if (e_ != hipSuccess) return hip_error(e_, #call);       \
    } while (0)

unsigned host_threads()
{
    unsigned n = std::thread::hardware_concurrency();
    return n ? std::min(n, 16u) : 1u;
}

template <typename F>
void parallel_for(uint64_t n, F f)
{
    unsigned t = host_threads();
    if (n < 65536 || t <= 1) {
        f(0, n);
        return;
    }
    std::vector<std::thread> th;
    uint64_t chunk = (n + t - 1) / t;
    for (unsigned i = 0; i < t; ++i) {
        uint64_t b = i * chunk, e = std::min(n, b + chunk);
        if (b >= e) break;
        th.emplace_back([=] { f(b, e); });
    }
    for (auto &x : th) x.join();
}

// ---------------------------------------------------------------------------
// Graph residency.

struct Side {
    uint64_t n = 0;
    uint32_t max_deg = 0;
    double deg_pairs = 0;            // sum over the side's vertices of C(d, 2): the wedges that
                                     // a candidate pass anchored on the other side scans
    uint64_t max_wedges = 0;         // max over the side's vertices u of sum_{v in N(u)} d(v): a
                                     // bound on the candidates of any root
    std::vector<uint32_t> rank_of;   // original id -> rank
    std::vector<uint64_t> h_ptr;     // relabelled CSR on the host (by rank)
    uint64_t *d_ptr = nullptr;
    uint32_t *d_adj = nullptr;
    uint32_t *d_rpos = nullptr;      // per edge (a, b): position of a within N(b)
    // hierarchical truncated bitmap of the rows (Section V-A), built on the
    // first count that needs it: row x is words [htb_off[x], htb_off[x+1])
    bool htb_ready = false;
    std::vector<uint64_t> h_htb_off;
    uint64_t *d_htb_off = nullptr;
    uint32_t *d_htb_idx = nullptr;
    uint32_t *d_htb_val = nullptr;
};

}  // namespace

struct bc_graph {
    Side side[2];
    uint64_t nnz = 0;
    int device = 0;
    std::mutex htb_mu;         // guards the lazy HTB build of both sides
    bool hooked = false;       // device arrays came from `hook` (freed through it)
    bc_allocator hook{};
};

namespace {

hipStream_t own_stream()
{
    thread_local hipStream_t s = nullptr;
    if (!s) {
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) s = nullptr;
    }
    return s;
}

hipStream_t pick_stream(const bc_opts *o)
{
    if (o && o->stream) return (hipStream_t)o->stream;
    return own_stream();
}

// Value of an option field, or dflt when opts is NULL or struct_size does not
// cover the field (callers built against an older, shorter bc_opts).
#define BC_OPT(o, field, dflt) \
    (((o) && (o)->struct_size >= offsetof(bc_opts, field) + sizeof((o)->field)) ? (o)->field : (dflt))

bc_status check_opts(const bc_opts *o)
{
    if (!o) return BC_OK;
    if (o->struct_size != 0 && o->struct_size < sizeof(uint32_t) * 2)
        return set_error(BC_E_INVALID_ARG, "bc_opts.struct_size too small");
    if (o->anchor < -1 || o->anchor > 1) return set_error(BC_E_INVALID_ARG, "bc_opts.anchor must be -1, 0 or 1");
    const bc_allocator *al = BC_OPT(o, alloc, (const bc_allocator *)nullptr);
    if (al && (!al->alloc || !al->free))
        return set_error(BC_E_INVALID_ARG, "bc_opts.alloc needs both alloc and free");
    const int32_t ok = BC_OPT(o, order_key, (int32_t)BC_ORDER_DEGREE);
    if (ok != BC_ORDER_DEGREE && ok != BC_ORDER_TWO_HOP && ok != BC_ORDER_BORDER)
        return set_error(BC_E_INVALID_ARG, "bc_opts.order_key must be BC_ORDER_DEGREE, _TWO_HOP or _BORDER");
    if (BC_OPT(o, roots_per_wave, 0u) > 64) return set_error(BC_E_INVALID_ARG, "bc_opts.roots_per_wave must be 0..64");
    const uint32_t sd = BC_OPT(o, switch_depth, 0u);
    if (sd != 0 && sd != 2 && sd != 3) return set_error(BC_E_INVALID_ARG, "bc_opts.switch_depth must be 0, 2 or 3");
    const uint32_t rb = BC_OPT(o, root_build, 0u);
    if (rb != BC_ROOT_BUILD_AUTO && rb != BC_ROOT_BUILD_TWO_PASS)
        return set_error(BC_E_INVALID_ARG, "bc_opts.root_build must be BC_ROOT_BUILD_AUTO or _TWO_PASS");
    const uint32_t sets = BC_OPT(o, sets, 0u);
    if (sets != BC_SETS_LOCAL_BITMAP && sets != BC_SETS_HTB && sets != BC_SETS_SORTED)
        return set_error(BC_E_INVALID_ARG, "bc_opts.sets must be BC_SETS_LOCAL_BITMAP, _HTB or _SORTED");
    return BC_OK;
}

// Validates one CSR side; writes sorted rows into rows_out (same layout).
bc_status validate_side(const bc_csr *c, const char *name, std::vector<uint32_t> &rows_out)
{
    if (!c->indptr) return set_error(BC_E_INVALID_ARG, std::string(name) + ".indptr is NULL");
    if (c->nnz && !c->indices) return set_error(BC_E_INVALID_ARG, std::string(name) + ".indices is NULL");
    if (c->n_rows >= 0xffffffffull || c->n_cols >= 0xffffffffull)
        return set_error(BC_E_INVALID_ARG, std::string(name) + ": more than 2^32-2 vertices on a side");
    if (c->indptr[0] != 0) return set_error(BC_E_BAD_CSR, std::string(name) + ".indptr[0] != 0");
    for (uint64_t r = 0; r < c->n_rows; ++r)
        if (c->indptr[r + 1] < c->indptr[r])
            return set_error(BC_E_BAD_CSR, std::string(name) + ".indptr decreases at row " + std::to_string(r));
    if (c->indptr[c->n_rows] != c->nnz)
        return set_error(BC_E_BAD_CSR, std::string(name) + ".indptr[n_rows] != nnz");
    rows_out.assign(c->indices, c->indices + c->nnz);
    std::vector<std::string> errs(host_threads() + 1);
    std::mutex mu;
    std::string first_err;
    parallel_for(c->n_rows, [&](uint64_t b, uint64_t e) {
        for (uint64_t r = b; r < e; ++r) {
            uint32_t *lo = rows_out.data() + c->indptr[r], *hi = rows_out.data() + c->indptr[r + 1];
            std::sort(lo, hi);
            for (uint32_t *x = lo; x < hi; ++x) {
                if (*x >= c->n_cols || (x > lo && *x == x[-1])) {
                    std::lock_guard<std::mutex> g(mu);
                    if (first_err.empty())
                        first_err = std::string(name) + ": row " + std::to_string(r) +
                                    (*x >= c->n_cols ? " has an id out of range" : " has a duplicate id");
                    return;
                }
            }
        }
    });
    if (!first_err.empty()) return set_error(BC_E_BAD_CSR, first_err);
    return BC_OK;
}

// Rank order of one side: ascending key, ties by original id.
void key_order(uint64_t n, const std::vector<uint64_t> &key, std::vector<uint32_t> &id_of_rank,
               std::vector<uint32_t> &rank_of)
{
    id_of_rank.resize(n);
    std::iota(id_of_rank.begin(), id_of_rank.end(), 0u);
    std::stable_sort(id_of_rank.begin(), id_of_rank.end(), [&](uint32_t a, uint32_t b) { return key[a] < key[b]; });
    rank_of.resize(n);
    for (uint64_t r = 0; r < n; ++r) rank_of[id_of_rank[r]] = (uint32_t)r;
}

// Border (Algorithm 2, Section V-B): reorders the vertices of one layer so
// that the other layer's rows, cut into blocks of 32 consecutive positions
// (the words of their HTB), have fewer blocks holding a single neighbour
// (1-blocks).  Starts from `order` (positions, e.g. the degree order) and
// repeats at most `iters` times: take the vertex v_m sitting in the most
// 1-blocks; the candidates are the vertices sharing the fewest rows with
// v_m; swap v_m with the candidate whose swap removes the most 1-blocks
// (the profit x_m + x_n - y_m - y_n), if any does.  Rows are given over the
// layer's vertex ids (rows_o with offsets ptr_o); cols_x lists, for each
// vertex of the layer, the rows it is in.  Returns the new order (id at
// each position).
std::vector<uint32_t> border_order(uint64_t n, const std::vector<uint32_t> &order, uint64_t n_rows,
                                   const uint64_t *ptr_o, const std::vector<uint32_t> &rows_o,
                                   const uint64_t *ptr_x, const std::vector<uint32_t> &cols_x, uint64_t iters)
{
    // candidates whose profit is evaluated per step: all of the least-overlap
    // vertices would cost O(|V| d) per swap; the 64 in the most 1-blocks stand for them
    constexpr uint32_t kCand = 64;
    std::vector<uint32_t> xat(order), pos(n);
    for (uint64_t i = 0; i < n; ++i) pos[xat[i]] = (uint32_t)i;
    // per row: occupied blocks and how many of its members each holds
    std::vector<std::unordered_map<uint32_t, uint32_t>> cnt(n_rows);
    for (uint64_t r = 0; r < n_rows; ++r)
        for (uint64_t e = ptr_o[r]; e < ptr_o[r + 1]; ++e) cnt[r][pos[rows_o[e]] >> 5]++;
    std::vector<int64_t> ones(n, 0);   // 1-blocks each vertex sits in
    for (uint64_t x = 0; x < n; ++x)
        for (uint64_t e = ptr_x[x]; e < ptr_x[x + 1]; ++e) ones[x] += cnt[cols_x[e]][pos[x] >> 5] == 1;
    std::vector<char> stuck(n, 0);     // no profitable swap found for it
    std::vector<uint8_t> overlap(n_rows, 0);   // per row: holds a (1), both a and b (2)
    // the single member of block b of row r (the block must hold exactly one)
    auto alone = [&](uint32_t r, uint32_t b) -> uint32_t {
        for (uint64_t e = ptr_o[r]; e < ptr_o[r + 1]; ++e)
            if ((pos[rows_o[e]] >> 5) == b) return rows_o[e];
        return 0xffffffffu;
    };
    // 1-blocks removed by swapping the positions of a and b
    auto profit = [&](uint32_t a, uint32_t b) -> int64_t {
        const uint32_t ba = pos[a] >> 5, bb = pos[b] >> 5;
        if (ba == bb) return 0;
        int64_t delta = 0;   // change in the number of 1-blocks
        auto moved = [&](uint32_t r, uint32_t from, uint32_t to) {
            const auto &m = cnt[r];
            const uint32_t cf = m.count(from) ? m.at(from) : 0, ct = m.count(to) ? m.at(to) : 0;
            delta += (int64_t)(cf - 1 == 1) - (int64_t)(cf == 1);
            delta += (int64_t)(ct + 1 == 1) - (int64_t)(ct == 1);
        };
        // rows of a without b: a leaves ba for bb; rows of b without a: the reverse
        for (uint64_t e = ptr_x[a]; e < ptr_x[a + 1]; ++e) overlap[cols_x[e]] = 1;
        for (uint64_t e = ptr_x[b]; e < ptr_x[b + 1]; ++e) {
            const uint32_t r = cols_x[e];
            if (overlap[r]) overlap[r] = 2;
            else moved(r, bb, ba);
        }
        for (uint64_t e = ptr_x[a]; e < ptr_x[a + 1]; ++e) {
            const uint32_t r = cols_x[e];
            if (overlap[r] == 1) moved(r, ba, bb);
            overlap[r] = 0;
        }
        return -delta;
    };
    for (uint64_t it = 0; it < iters; ++it) {
        // Step 1: the vertex in the most 1-blocks
        uint32_t vm = 0xffffffffu;
        for (uint64_t x = 0; x < n; ++x)
            if (!stuck[x] && ones[x] > 0 && (vm == 0xffffffffu || ones[x] > ones[vm])) vm = (uint32_t)x;
        if (vm == 0xffffffffu) break;
        // Step 2: rows shared with v_m, for every vertex (wedge scan); the
        // candidates have the fewest, best first by their own 1-blocks
        std::vector<uint32_t> shared(n, 0);
        for (uint64_t e = ptr_x[vm]; e < ptr_x[vm + 1]; ++e) {
            const uint32_t r = cols_x[e];
            for (uint64_t f = ptr_o[r]; f < ptr_o[r + 1]; ++f) shared[rows_o[f]]++;
        }
        uint32_t least = 0xffffffffu;
        for (uint64_t x = 0; x < n; ++x)
            if (x != vm) least = std::min(least, shared[x]);
        std::vector<uint32_t> cand;
        for (uint64_t x = 0; x < n; ++x)
            if (x != vm && shared[x] == least && (pos[x] >> 5) != (pos[vm] >> 5)) cand.push_back((uint32_t)x);
        if (cand.size() > kCand) {
            std::partial_sort(cand.begin(), cand.begin() + kCand, cand.end(),
                              [&](uint32_t a, uint32_t b) { return ones[a] != ones[b] ? ones[a] > ones[b] : a < b; });
            cand.resize(kCand);
        }
        // Step 3: the candidate with the highest profit
        int64_t best = 0;
        uint32_t vn = 0xffffffffu;
        for (uint32_t x : cand) {
            const int64_t pr = profit(vm, x);
            if (pr > best) {
                best = pr;
                vn = x;
            }
        }
        if (vn == 0xffffffffu) {
            stuck[vm] = 1;
            continue;
        }
        // Step 4: swap, then update the block counts and the 1-block counts
        // of every vertex whose block changed between one member and more
        const uint32_t ba = pos[vm] >> 5, bb = pos[vn] >> 5;
        std::vector<std::pair<uint32_t, uint32_t>> hit;   // (row, block) whose count changes
        for (uint64_t e = ptr_x[vm]; e < ptr_x[vm + 1]; ++e) hit.push_back({cols_x[e], ba}), hit.push_back({cols_x[e], bb});
        for (uint64_t e = ptr_x[vn]; e < ptr_x[vn + 1]; ++e) hit.push_back({cols_x[e], ba}), hit.push_back({cols_x[e], bb});
        std::sort(hit.begin(), hit.end());
        hit.erase(std::unique(hit.begin(), hit.end()), hit.end());
        for (const auto &h : hit) {   // old singles lose their 1-block
            auto f = cnt[h.first].find(h.second);
            if (f != cnt[h.first].end() && f->second == 1) {
                const uint32_t x = alone(h.first, h.second);
                if (x != 0xffffffffu) ones[x]--;
            }
        }
        for (uint64_t e = ptr_x[vm]; e < ptr_x[vm + 1]; ++e) {
            auto &m = cnt[cols_x[e]];
            if (--m[ba] == 0) m.erase(ba);
            m[bb]++;
        }
        for (uint64_t e = ptr_x[vn]; e < ptr_x[vn + 1]; ++e) {
            auto &m = cnt[cols_x[e]];
            if (--m[bb] == 0) m.erase(bb);
            m[ba]++;
        }
        std::swap(xat[pos[vm]], xat[pos[vn]]);
        std::swap(pos[vm], pos[vn]);
        for (const auto &h : hit) {   // new singles gain one
            auto f = cnt[h.first].find(h.second);
            if (f != cnt[h.first].end() && f->second == 1) {
                const uint32_t x = alone(h.first, h.second);
                if (x != 0xffffffffu) ones[x]++;
            }
        }
        stuck[vn] = 0;
    }
    return xat;
}

// Degree of every vertex of side c.
std::vector<uint64_t> degree_key(const bc_csr *c)
{
    std::vector<uint64_t> key(c->n_rows);
    for (uint64_t x = 0; x < c->n_rows; ++x) key[x] = c->indptr[x + 1] - c->indptr[x];
    return key;
}

// |N_2^k(x)| for every vertex x of side c (Section II-A, Definition 2): the
// vertices y != x of the same side with |N(x) n N(y)| >= k, found by counting
// the wedges x - v - y through the other side's rows (o, sorted in rows_o).
// Threads take vertices in chunks, each with its own dense counter array.
std::vector<uint64_t> two_hop_key(const bc_csr *c, const std::vector<uint32_t> &rows_c, const bc_csr *o,
                                  const std::vector<uint32_t> &rows_o, uint32_t k)
{
    const uint64_t n = c->n_rows;
    std::vector<uint64_t> key(n, 0);
    const unsigned nt = std::max(1u, std::min<unsigned>(host_threads(), (unsigned)std::max<uint64_t>(1, n / 256)));
    std::atomic<uint64_t> next{0};
    auto work = [&] {
        std::vector<uint32_t> cnt(n, 0), touched;
        for (;;) {
            const uint64_t b = next.fetch_add(256), e = std::min(n, b + 256);
            if (b >= n) break;
            for (uint64_t x = b; x < e; ++x) {
                touched.clear();
                for (uint64_t i = c->indptr[x]; i < c->indptr[x + 1]; ++i) {
                    const uint32_t v = rows_c[i];
                    for (uint64_t j = o->indptr[v]; j < o->indptr[v + 1]; ++j) {
                        const uint32_t y = rows_o[j];
                        if (y != x && cnt[y]++ == 0) touched.push_back(y);
                    }
                }
                uint64_t size = 0;
                for (uint32_t y : touched) {
                    size += cnt[y] >= k;
                    cnt[y] = 0;
                }
                key[x] = size;
            }
        }
    };
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nt; ++t) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
    return key;
}

// Relabelled CSR: row r is vertex id_of_rank[r]; neighbours mapped through
// the other side's rank and sorted.
void relabel(const bc_csr *c, const std::vector<uint32_t> &sorted_rows, const std::vector<uint32_t> &id_of_rank,
             const std::vector<uint32_t> &other_rank_of, std::vector<uint64_t> &ptr, std::vector<uint32_t> &adj)
{
    const uint64_t n = c->n_rows;
    ptr.assign(n + 1, 0);
    for (uint64_t r = 0; r < n; ++r) {
        uint32_t x = id_of_rank[r];
        ptr[r + 1] = ptr[r] + (c->indptr[x + 1] - c->indptr[x]);
    }
    adj.resize(c->nnz);
    parallel_for(n, [&](uint64_t b, uint64_t e) {
        for (uint64_t r = b; r < e; ++r) {
            uint32_t x = id_of_rank[r];
            uint64_t s = c->indptr[x], t = c->indptr[x + 1], o = ptr[r];
            for (uint64_t i = s; i < t; ++i) adj[o + (i - s)] = other_rank_of[sorted_rows[i]];
            std::sort(adj.begin() + o, adj.begin() + o + (t - s));
        }
    });
}

// A graph's device arrays: hipMalloc, or the caller's hook when bc_build had one.
hipError_t graph_alloc(bc_graph *g, void **p, uint64_t bytes, hipStream_t st)
{
    if (!g->hooked) return hipMalloc(p, bytes);
    *p = g->hook.alloc(g->hook.ctx, bytes, st);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}

void graph_release(bc_graph *g, void *p)
{
    if (!p) return;
    if (g->hooked) g->hook.free(g->hook.ctx, p, nullptr);
    else (void)hipFree(p);
}

void free_side(bc_graph *g, Side &s)
{
    graph_release(g, s.d_ptr);
    graph_release(g, s.d_adj);
    graph_release(g, s.d_rpos);
    graph_release(g, s.d_htb_off);
    graph_release(g, s.d_htb_idx);
    graph_release(g, s.d_htb_val);
    s.d_ptr = nullptr;
    s.d_adj = nullptr;
    s.d_rpos = nullptr;
    s.d_htb_off = nullptr;
    s.d_htb_idx = nullptr;
    s.d_htb_val = nullptr;
}

// The HTB of one side's rows (Section V-A): each neighbour id b goes to word
// b / 32, bit b % 32; a row keeps its nonzero words in increasing word index
// (Idx) with their values (Val), and Off gives each row's first word.  Built
// once per graph side, on the host from the device rows, under htb_mu.
bc_status ensure_htb(bc_graph *g, int side, hipStream_t st)
{
    std::lock_guard<std::mutex> lk(g->htb_mu);
    Side &sd = g->side[side];
    if (sd.htb_ready) return BC_OK;
    std::vector<uint32_t> adj(g->nnz);
    if (g->nnz) BC_HIP(hipMemcpyAsync(adj.data(), sd.d_adj, g->nnz * 4, hipMemcpyDeviceToHost, st));
    BC_HIP(hipStreamSynchronize(st));
    std::vector<uint64_t> off(sd.n + 1, 0);
    std::vector<uint32_t> idx, val;
    idx.reserve(g->nnz);
    val.reserve(g->nnz);
    for (uint64_t x = 0; x < sd.n; ++x) {
        for (uint64_t e = sd.h_ptr[x]; e < sd.h_ptr[x + 1]; ++e) {
            const uint32_t w = adj[e] >> 5, bit = 1u << (adj[e] & 31);
            if (idx.size() > off[x] && idx.back() == w) val.back() |= bit;   // rows are sorted
            else {
                idx.push_back(w);
                val.push_back(bit);
            }
        }
        off[x + 1] = idx.size();
    }
    const uint64_t words = std::max<uint64_t>(1, idx.size());
    hipError_t e = graph_alloc(g, (void **)&sd.d_htb_off, (sd.n + 1) * 8, st);
    if (e == hipSuccess) e = graph_alloc(g, (void **)&sd.d_htb_idx, words * 4, st);
    if (e == hipSuccess) e = graph_alloc(g, (void **)&sd.d_htb_val, words * 4, st);
    if (e == hipSuccess) e = hipMemcpyAsync(sd.d_htb_off, off.data(), (sd.n + 1) * 8, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !idx.empty())
        e = hipMemcpyAsync(sd.d_htb_idx, idx.data(), idx.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !val.empty())
        e = hipMemcpyAsync(sd.d_htb_val, val.data(), val.size() * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(st);
        graph_release(g, sd.d_htb_off);
        graph_release(g, sd.d_htb_idx);
        graph_release(g, sd.d_htb_val);
        sd.d_htb_off = nullptr;
        sd.d_htb_idx = nullptr;
        sd.d_htb_val = nullptr;
        return hip_error(e, "HTB build");
    }
    sd.h_htb_off.swap(off);
    sd.htb_ready = true;
    return BC_OK;
}

}  // namespace

extern "C" bc_status bc_build(const bc_csr *U, const bc_csr *V, const bc_opts *opts, bc_graph **out)
{
    g_last_error.clear();
    if (!U || !V || !out) return set_error(BC_E_INVALID_ARG, "bc_build: NULL argument");
    if (bc_status s = check_opts(opts)) return s;
    if (U->n_rows != V->n_cols || U->n_cols != V->n_rows)
        return set_error(BC_E_INCONSISTENT, "bc_build: U and V CSR shapes are not transposes");
    if (U->nnz != V->nnz) return set_error(BC_E_INCONSISTENT, "bc_build: U and V have different edge counts");
    std::vector<uint32_t> rowsU, rowsV;
    if (bc_status s = validate_side(U, "U", rowsU)) return s;
    if (bc_status s = validate_side(V, "V", rowsV)) return s;

    // V must be the transpose of U: build the transpose of U (rows come out
    // sorted because u is visited in increasing order) and compare.
    {
        std::vector<uint64_t> tp(V->n_rows + 1, 0);
        for (uint64_t i = 0; i < U->nnz; ++i) tp[rowsU[i] + 1]++;
        for (uint64_t v = 0; v < V->n_rows; ++v) tp[v + 1] += tp[v];
        for (uint64_t v = 0; v <= V->n_rows; ++v)
            if (tp[v] != V->indptr[v])
                return set_error(BC_E_INCONSISTENT, "bc_build: degree of V vertex " +
                                                        std::to_string(v ? v - 1 : 0) + " differs from U's view");
        std::vector<uint64_t> fill(tp.begin(), tp.end() - 1);
        std::vector<uint32_t> tadj(U->nnz);
        for (uint64_t u = 0; u < U->n_rows; ++u)
            for (uint64_t i = U->indptr[u]; i < U->indptr[u + 1]; ++i) tadj[fill[rowsU[i]]++] = (uint32_t)u;
        if (tadj != rowsV) return set_error(BC_E_INCONSISTENT, "bc_build: V is not the transpose of U");
    }

    bc_graph *g = new (std::nothrow) bc_graph();
    if (!g) return set_error(BC_E_OOM, "bc_build: host allocation failed");
    g->nnz = U->nnz;
    (void)hipGetDevice(&g->device);
    if (const bc_allocator *al = BC_OPT(opts, alloc, (const bc_allocator *)nullptr)) {
        g->hooked = true;
        g->hook = *al;
    }
    std::vector<uint32_t> idU, idV;
    const int32_t okey = BC_OPT(opts, order_key, (int32_t)BC_ORDER_DEGREE);
    if (okey == BC_ORDER_BORDER) {
        // degree order first (Section V-B), then Border on each layer for the
        // other layer's rows
        key_order(U->n_rows, degree_key(U), idU, g->side[0].rank_of);
        key_order(V->n_rows, degree_key(V), idV, g->side[1].rank_of);
        const uint64_t it = BC_OPT(opts, border_iters, 0u) ? BC_OPT(opts, border_iters, 0u) : 4096u;
        idU = border_order(U->n_rows, idU, V->n_rows, V->indptr, rowsV, U->indptr, rowsU, it);
        idV = border_order(V->n_rows, idV, U->n_rows, U->indptr, rowsU, V->indptr, rowsV, it);
        for (uint64_t r = 0; r < U->n_rows; ++r) g->side[0].rank_of[idU[r]] = (uint32_t)r;
        for (uint64_t r = 0; r < V->n_rows; ++r) g->side[1].rank_of[idV[r]] = (uint32_t)r;
    } else if (okey == BC_ORDER_TWO_HOP) {
        const uint32_t k = std::max(1u, BC_OPT(opts, order_k, 0u) ? BC_OPT(opts, order_k, 0u) : 2u);
        key_order(U->n_rows, two_hop_key(U, rowsU, V, rowsV, k), idU, g->side[0].rank_of);
        key_order(V->n_rows, two_hop_key(V, rowsV, U, rowsU, k), idV, g->side[1].rank_of);
    } else {
        key_order(U->n_rows, degree_key(U), idU, g->side[0].rank_of);
        key_order(V->n_rows, degree_key(V), idV, g->side[1].rank_of);
    }
    const bc_csr *cs[2] = {U, V};
    const std::vector<uint32_t> *rows[2] = {&rowsU, &rowsV};
    const std::vector<uint32_t> *ids[2] = {&idU, &idV};
    hipStream_t st = pick_stream(opts);
    std::vector<uint32_t> adj[2], rpos[2];
    for (int s = 0; s < 2; ++s) {
        Side &sd = g->side[s];
        sd.n = cs[s]->n_rows;
        relabel(cs[s], *rows[s], *ids[s], g->side[1 - s].rank_of, sd.h_ptr, adj[s]);
        for (uint64_t r = 0; r < sd.n; ++r) {
            const uint64_t d = sd.h_ptr[r + 1] - sd.h_ptr[r];
            sd.max_deg = std::max<uint32_t>(sd.max_deg, (uint32_t)d);
            sd.deg_pairs += 0.5 * (double)d * (double)(d ? d - 1 : 0);
        }
    }
    for (int s = 0; s < 2; ++s) {
        Side &sa = g->side[s];
        const Side &sb = g->side[1 - s];
        for (uint64_t r = 0; r < sa.n; ++r) {
            uint64_t w = 0;
            for (uint64_t e = sa.h_ptr[r]; e < sa.h_ptr[r + 1]; ++e) w += sb.h_ptr[adj[s][e] + 1] - sb.h_ptr[adj[s][e]];
            sa.max_wedges = std::max(sa.max_wedges, w);
        }
    }
    // Reverse positions: for the edge (a, b) stored in a's row, the index of a
    // within b's row.  Visiting b in increasing order meets a's edges in the
    // order a's sorted row stores them, so one cursor per a suffices.
    for (int s = 0; s < 2; ++s) {
        const Side &sa = g->side[s], &sb = g->side[1 - s];
        rpos[s].resize(g->nnz);
        std::vector<uint64_t> cursor(sa.h_ptr.begin(), sa.h_ptr.end() - 1);
        for (uint64_t b = 0; b < sb.n; ++b)
            for (uint64_t i = sb.h_ptr[b]; i < sb.h_ptr[b + 1]; ++i)
                rpos[s][cursor[adj[1 - s][i]]++] = (uint32_t)(i - sb.h_ptr[b]);
    }
    for (int s = 0; s < 2; ++s) {
        Side &sd = g->side[s];
        const uint64_t m = std::max<uint64_t>(1, g->nnz) * sizeof(uint32_t);
        hipError_t e = graph_alloc(g, (void **)&sd.d_ptr, (sd.n + 1) * sizeof(uint64_t), st);
        if (e == hipSuccess) e = graph_alloc(g, (void **)&sd.d_adj, m, st);
        if (e == hipSuccess) e = graph_alloc(g, (void **)&sd.d_rpos, m, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(sd.d_ptr, sd.h_ptr.data(), (sd.n + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, st);
        if (e == hipSuccess && g->nnz)
            e = hipMemcpyAsync(sd.d_adj, adj[s].data(), g->nnz * sizeof(uint32_t), hipMemcpyHostToDevice, st);
        if (e == hipSuccess && g->nnz)
            e = hipMemcpyAsync(sd.d_rpos, rpos[s].data(), g->nnz * sizeof(uint32_t), hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(st);   // no upload may still read a block handed back
            free_side(g, g->side[0]);
            free_side(g, g->side[1]);
            delete g;
            return e == hipErrorOutOfMemory ? set_error(BC_E_OOM, "bc_build: device allocation failed")
                                            : hip_error(e, "bc_build: upload");
        }
    }
    *out = g;
    return BC_OK;
}

extern "C" void bc_free(bc_graph *g)
{
    if (!g) return;
    free_side(g, g->side[0]);
    free_side(g, g->side[1]);
    delete g;
}

extern "C" bc_status bc_graph_info(const bc_graph *g, uint64_t *n_u, uint64_t *n_v, uint64_t *n_edges)
{
    if (!g) return set_error(BC_E_INVALID_ARG, "bc_graph_info: NULL graph");
    if (n_u) *n_u = g->side[0].n;
    if (n_v) *n_v = g->side[1].n;
    if (n_edges) *n_edges = g->nnz;
    return BC_OK;
}

extern "C" bc_status bc_htb_stats(bc_graph *g, int32_t side, uint64_t *words, uint64_t *one_blocks)
{
    g_last_error.clear();
    if (!g || (side != 0 && side != 1) || !words || !one_blocks)
        return set_error(BC_E_INVALID_ARG, "bc_htb_stats: bad argument");
    hipStream_t st = own_stream();
    if (!st) return set_error(BC_E_DEVICE, "could not create a HIP stream");
    BC_HIP(hipSetDevice(g->device));
    if (bc_status e = ensure_htb(g, side, st)) return e;
    const Side &sd = g->side[side];
    const uint64_t n_words = sd.h_htb_off.back();
    std::vector<uint32_t> val(std::max<uint64_t>(1, n_words));
    if (n_words) BC_HIP(hipMemcpyAsync(val.data(), sd.d_htb_val, n_words * 4, hipMemcpyDeviceToHost, st));
    BC_HIP(hipStreamSynchronize(st));
    uint64_t ones = 0;
    for (uint64_t i = 0; i < n_words; ++i) ones += __builtin_popcount(val[i]) == 1;
    *words = n_words;
    *one_blocks = ones;
    return BC_OK;
}

extern "C" bc_status bc_ranks(const bc_graph *g, int32_t side, uint32_t *rank_of)
{
    if (!g || !rank_of || (side != 0 && side != 1)) return set_error(BC_E_INVALID_ARG, "bc_ranks: bad argument");
    const auto &r = g->side[side].rank_of;
    std::copy(r.begin(), r.end(), rank_of);
    return BC_OK;
}

// ---------------------------------------------------------------------------
// Query execution.

namespace {

// Device scratch of one call, released when the call ends.  Three sources:
// stream-ordered hipMallocAsync on the call's stream (default), the caller's
// allocator hook, or a fixed device region carved by bumping an offset (the
// no-allocation entry point; nothing is allocated or freed).  Every request
// is rounded up to 256 bytes.  A failed request returns hipErrorOutOfMemory.
struct DevAlloc {
    std::vector<void *> ptrs;
    hipStream_t st;
    const bc_allocator *hook = nullptr;
    uint8_t *fixed = nullptr;
    uint64_t fixed_cap = 0, fixed_used = 0;
    bool fixed_short = false;    // a request did not fit the fixed region
    uint64_t cap = 0;            // nonzero: at most this many bytes in all (other sources)
    uint64_t total = 0;          // bytes taken so far (nothing is released before the end)
    DevAlloc(hipStream_t s, const bc_allocator *h) : st(s), hook(h) {}
    DevAlloc(hipStream_t s, void *region, uint64_t cap) : st(s), fixed((uint8_t *)region), fixed_cap(cap) {}
    ~DevAlloc()
    {
        for (void *p : ptrs) {
            if (hook) hook->free(hook->ctx, p, st);
            else (void)hipFreeAsync(p, st);
        }
    }
    // bytes left in the fixed region or under the cap (else unbounded)
    uint64_t room() const
    {
        if (fixed) return fixed_cap - fixed_used;
        return cap ? (cap > total ? cap - total : 0) : ~0ull;
    }
    hipError_t raw(void **p, uint64_t bytes)
    {
        bytes = (std::max<uint64_t>(bytes, 1) + 255) & ~255ull;
        *p = nullptr;
        if (fixed) {
            if (bytes > fixed_cap - fixed_used) {
                fixed_short = true;
                return hipErrorOutOfMemory;
            }
            *p = fixed + fixed_used;
            fixed_used += bytes;
            total += bytes;
            return hipSuccess;
        }
        if (cap && bytes > room()) return hipErrorOutOfMemory;
        void *v = nullptr;
        if (hook) {
            v = hook->alloc(hook->ctx, bytes, st);
            if (!v) return hipErrorOutOfMemory;
        } else {
            hipError_t e = hipMallocAsync(&v, bytes, st);
            if (e != hipSuccess) return e;
        }
        ptrs.push_back(v);
        total += bytes;
        *p = v;
        return hipSuccess;
    }
    template <typename T>
    hipError_t get(T **p, uint64_t count)
    {
        void *v = nullptr;
        hipError_t e = raw(&v, count * sizeof(T));
        *p = (T *)v;
        return e;
    }
};

struct JobSpec {
    const bc_graph *g;
    uint32_t p, q;
    int32_t anchor;            // requested (AUTO allowed)
    uint64_t rank_lo, rank_hi; // only used when ranged
    bool ranged;
    uint64_t deadline_ns;      // steady clock, 0 = none
    const std::vector<uint8_t> *root_mask = nullptr;   // p_A >= 3 only: roots (by rank) that get tasks
    bc_u128 *pv_out = nullptr;   // per-vertex counts of the anchor side, by rank (explicit anchor, p_A >= 2)
};

// Device real-time clock against the host steady clock, per device.  The
// counter runs at a constant 100 MHz; two samples 20 ms apart check that
// rate once (a rate off by more than 2 % is used as measured instead).  Each
// call re-anchors the offset with a fresh sample taken on the caller's
// (idle) stream, kept only when its round trip was short, so that an error in
// the rate cannot accumulate over the life of the process.
struct ClockCal {
    bool ok = false;
    double ticks_per_ns = 0.1;
    double offset = 0.0;
};

// One sample: the device tick and the host time at the middle of the round
// trip; false on a HIP error.
bool clock_sample(uint64_t *d, hipStream_t st, uint64_t &tick, double &mid, uint64_t &rtt)
{
    const uint64_t t0 = bcint::steady_ns();
    hipError_t e = bcdev::launch_read_clock(d, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&tick, d, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    const uint64_t t1 = bcint::steady_ns();
    mid = 0.5 * ((double)t0 + (double)t1);
    rtt = t1 - t0;
    return e == hipSuccess;
}

bc_status device_clock(int device, hipStream_t st, DevAlloc &mem, ClockCal &out)
{
    static std::mutex mu;
    static std::vector<ClockCal> cache(64);
    if (device < 0 || device >= 64) return set_error(BC_E_DEVICE, "device id out of range");
    uint64_t *d = nullptr;
    BC_HIP(mem.get(&d, 1));
    uint64_t tick = 0, rtt = 0;
    double mid = 0;
    if (!clock_sample(d, st, tick, mid, rtt)) return set_error(BC_E_DEVICE, "clock calibration failed");
    std::lock_guard<std::mutex> g(mu);
    ClockCal &c = cache[device];
    if (!c.ok) {
        // rate check: a second sample 20 ms later
        std::this_thread::sleep_for(std::chrono::milliseconds(20));
        uint64_t tick2 = 0, rtt2 = 0;
        double mid2 = 0;
        if (!clock_sample(d, st, tick2, mid2, rtt2)) return set_error(BC_E_DEVICE, "clock calibration failed");
        const double rate = (double)(tick2 - tick) / (mid2 - mid);
        c.ticks_per_ns = (rate > 0.098 && rate < 0.102) || !(rate > 0) ? 0.1 : rate;
        c.offset = (double)tick2 - c.ticks_per_ns * mid2;
        c.ok = true;
    } else if (rtt < 2000000) {
        c.offset = (double)tick - c.ticks_per_ns * mid;
    }
    out = c;
    return BC_OK;
}

// C(n, q) for n in [0, nmax] as exact u128; n_ovf = first n that overflows.
void binom_column(uint32_t nmax, uint32_t q, std::vector<u128> &col, uint32_t &n_ovf, uint32_t &n_u64,
                  uint32_t &n_u58, uint32_t &n_u28)
{
    std::vector<u128> c(q + 1, 0);
    std::vector<uint8_t> ov(q + 1, 0);
    c[0] = 1;
    col.assign(nmax + 1, 0);
    n_ovf = nmax + 1;
    for (uint32_t n = 0; n <= nmax; ++n) {
        if (n > 0) {
            for (uint32_t k = std::min(n, q); k >= 1; --k) {
                u128 s = c[k] + c[k - 1];
                bool o = ov[k] || ov[k - 1] || s < c[k];
                c[k] = o ? 0 : s;
                ov[k] = o;
            }
        }
        if (ov[q] && n_ovf > nmax) n_ovf = n;
        col[n] = ov[q] ? 0 : c[q];
        // C(n, q) does not decrease with n, so the entries below 2^64 are a prefix
        if (!ov[q] && (c[q] >> 64) == 0) n_u64 = n;
        if (!ov[q] && (c[q] >> 58) == 0) n_u58 = n;
        if (!ov[q] && (c[q] >> 28) == 0) n_u28 = n;
    }
}

hipError_t fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t st) { return bcdev::launch_fill_u32(p, n, v, st); }

int cu_count(int device)
{
    static std::mutex mu;
    static std::vector<int> cache(64, 0);
    std::lock_guard<std::mutex> g(mu);
    if (device < 0 || device >= 64) return 256;
    if (!cache[device]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || v <= 0) v = 256;
        cache[device] = v;
        // keep up to 32 GiB of stream-ordered allocations cached between
        // calls instead of returning them to the driver at every
        // synchronization (more would starve other users of the device)
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
            uint64_t thr = 32ull << 30;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
    }
    return cache[device];
}

int lds_per_block(int device)
{
    static std::mutex mu;
    static std::vector<int> cache(64, -1);
    std::lock_guard<std::mutex> g(mu);
    if (device < 0 || device >= 64) return 0;
    if (cache[device] < 0) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) v = 0;
        cache[device] = v;
    }
    return cache[device];
}

struct Timer {
    hipEvent_t e[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    bool ok = true;
    explicit Timer(bool on)
    {
        ok = on;
        for (auto &x : e)
            if (ok && hipEventCreate(&x) != hipSuccess) ok = false;
    }
    ~Timer()
    {
        for (auto &x : e)
            if (x) (void)hipEventDestroy(x);
    }
    void mark(int i, hipStream_t s)
    {
        if (ok) (void)hipEventRecord(e[i], s);
    }
    double ms(int a, int b)
    {
        float f = 0;
        if (!ok || hipEventElapsedTime(&f, e[a], e[b]) != hipSuccess) return 0.0;
        return f;
    }
};

// Resolved per-job state on the host.
struct HostJob {
    int spec;                  // index into specs
    int anchor;
    uint32_t pA, qA;
    uint32_t root_lo, root_hi;
    bool trivial_zero;
    bool dropped;              // the other anchor of its spec was chosen from a sample
    uint64_t cost;             // planning proxy after the candidate pass
    uint64_t weight;           // the same over the whole depth (job ordering)
};

// Positions of cost[] in descending cost order, equal costs in ascending
// position (the order a stable sort gives): LSD radix sort over 8-bit digits
// of the complemented key, skipping digits on which all keys agree.
std::vector<uint32_t> order_by_cost_desc(const std::vector<uint64_t> &cost)
{
    const size_t n = cost.size();
    std::vector<uint32_t> a(n), b(n);
    std::vector<uint64_t> key(n), kb(n);
    std::iota(a.begin(), a.end(), 0u);
    uint64_t any = 0, all = ~0ull;
    for (size_t i = 0; i < n; ++i) {
        key[i] = ~cost[i];
        any |= key[i];
        all &= key[i];
    }
    for (int sh = 0; sh < 64; sh += 8) {
        if ((((any ^ all) >> sh) & 0xff) == 0) continue;
        size_t cnt[257] = {0};
        for (size_t i = 0; i < n; ++i) ++cnt[((key[i] >> sh) & 0xff) + 1];
        for (int d = 0; d < 256; ++d) cnt[d + 1] += cnt[d];
        for (size_t i = 0; i < n; ++i) {
            const size_t o = cnt[(key[i] >> sh) & 0xff]++;
            b[o] = a[i];
            kb[o] = key[i];
        }
        a.swap(b);
        key.swap(kb);
    }
    return a;
}

// Cost model of served deadlines: per enumeration depth p_A, the fewest
// nanoseconds per unit of the whole-depth planning proxy (sum over a job's
// roots of k^(p_A - 1) W1) seen so far in a served batch holding that one
// job.  The proxy ignores pruning, so the fewest seen is the optimistic end:
// a job is refused only when even that rate puts it far past its deadline.
struct RateBook {
    std::mutex mu;
    double ns_per_unit[33] = {0};   // 0 = nothing seen yet
};
RateBook &rate_book()
{
    static RateBook rb;
    return rb;
}
constexpr double kRefuseMargin = 4.0;   // refuse when the estimate exceeds 4x the time left

// Where one run_jobs call takes its stream and device scratch from.
struct Exec {
    bool short_first = false;   // served batches: order the tasks job by job, cheapest
                                // job (by the cost proxy) first, so that one job that
                                // cannot meet its deadline does not hold back the others
    void *fixed = nullptr;      // non-NULL: all scratch from this device region
    uint64_t fixed_cap = 0;     //   of this many bytes (no allocation, no timing events)
    bool *fixed_short = nullptr;   // set when the region was too small
    uint64_t scratch_cap = 0;   // nonzero: the call's device scratch stays within this many bytes (the
                                // enumeration grid shrinks to fit; what still does not fit is BC_E_OOM)
};

bc_status run_jobs_impl(const std::vector<JobSpec> &specs, const bc_opts *opts, std::vector<bc_u128> &out,
                        std::vector<bc_status> &item_status, bc_stats *stats, const Exec &ex, bool &read_back,
                        DevAlloc *&mem_out);

// Runs the jobs; item_status[i] is BC_OK only for a count that was read back
// from the device.  When the call fails before that, every item gets the
// call's status.
bc_status run_jobs(const std::vector<JobSpec> &specs, const bc_opts *opts, std::vector<bc_u128> &out,
                   std::vector<bc_status> &item_status, bc_stats *stats, const Exec &ex = Exec())
{
    bool read_back = false;
    DevAlloc *mem = nullptr;
    bc_status s = run_jobs_impl(specs, opts, out, item_status, stats, ex, read_back, mem);
    if (mem && ex.fixed_short && mem->fixed_short) *ex.fixed_short = true;
    delete mem;   // stream-ordered release of the call's scratch
    if (!read_back) {
        const bc_status e = s == BC_OK ? set_error(BC_E_DEVICE, "internal: counts were not read back") : s;
        item_status.assign(specs.size(), e);
        out.assign(specs.size(), bc_u128{0, 0});
        return e;
    }
    return s;
}

bc_status run_jobs_impl(const std::vector<JobSpec> &specs, const bc_opts *opts, std::vector<bc_u128> &out,
                        std::vector<bc_status> &item_status, bc_stats *stats, const Exec &ex, bool &read_back,
                        DevAlloc *&mem_out)
{
    const size_t ns = specs.size();
    out.assign(ns, bc_u128{0, 0});
    item_status.assign(ns, BC_OK);
    if (ns == 0) {
        read_back = true;
        return BC_OK;
    }
    const bool short_first = ex.short_first;
    hipStream_t st = ex.fixed ? (hipStream_t)(opts ? opts->stream : nullptr) : pick_stream(opts);
    if (!st && !ex.fixed) return set_error(BC_E_DEVICE, "could not create a HIP stream");
    const int device = specs[0].g->device;
    BC_HIP(hipSetDevice(device));
    const uint32_t lds_words = (opts && opts->lds_words) ? opts->lds_words : bcdev::max_lds_words_per_wave();
    const uint32_t waves_per_cu = (opts && opts->waves_per_cu) ? std::min(12u, opts->waves_per_cu) : 12u;
    const bool instrument = opts && opts->instrument;
    const uint32_t roots_per_wave = BC_OPT(opts, roots_per_wave, 0u);
    const uint32_t switch_depth = BC_OPT(opts, switch_depth, 0u);
    const uint32_t split_rows = BC_OPT(opts, split_rows, 0u);
    const bool two_pass = BC_OPT(opts, root_build, 0u) == BC_ROOT_BUILD_TWO_PASS;
    const uint64_t scratch_cap = std::max<uint64_t>(ex.scratch_cap, BC_OPT(opts, scratch_cap_bytes, (uint64_t)0));
    const uint32_t sets_opt = BC_OPT(opts, sets, (uint32_t)BC_SETS_LOCAL_BITMAP);
    const uint32_t bitmap_bits = BC_OPT(opts, bitmap_bits, 0u);
    const int ncu = cu_count(device);
    auto t_host0 = std::chrono::steady_clock::now();
    mem_out = ex.fixed ? new DevAlloc(st, ex.fixed, ex.fixed_cap)
                       : new DevAlloc(st, BC_OPT(opts, alloc, (const bc_allocator *)nullptr));
    DevAlloc &mem = *mem_out;
    mem.cap = ex.fixed ? 0 : scratch_cap;

    // 1. Resolve anchors.  A spec with AUTO and p == q (>= 3) gets both sides
    //    as candidate jobs; the cheaper by the candidate-pass proxy is kept.
    std::vector<HostJob> jobs;
    std::vector<std::vector<int>> spec_jobs(ns);
    for (size_t i = 0; i < ns; ++i) {
        const JobSpec &sp = specs[i];
        std::vector<int> sides;
        if (sp.anchor == BC_ANCHOR_U || sp.anchor == BC_ANCHOR_V) sides.push_back(sp.anchor);
        else if (sp.p < sp.q) sides.push_back(0);
        else if (sp.q < sp.p) sides.push_back(1);
        else if (sp.p <= 2) sides.push_back(0);
        else {
            sides.push_back(0);
            sides.push_back(1);
        }
        for (int a : sides) {
            HostJob hj{};
            hj.spec = (int)i;
            hj.anchor = a;
            hj.pA = a == 0 ? sp.p : sp.q;
            hj.qA = a == 0 ? sp.q : sp.p;
            const Side &A = sp.g->side[a];
            const Side &B = sp.g->side[1 - a];
            uint64_t lo = sp.ranged ? std::min<uint64_t>(sp.rank_lo, A.n) : 0;
            uint64_t hi = sp.ranged ? std::min<uint64_t>(sp.rank_hi, A.n) : A.n;
            if (hi < lo) hi = lo;
            hj.root_lo = (uint32_t)lo;
            hj.root_hi = (uint32_t)hi;
            hj.trivial_zero = hj.pA > A.n || hj.qA > B.n || lo == hi || hj.qA > A.max_deg;
            spec_jobs[i].push_back((int)jobs.size());
            jobs.push_back(hj);
        }
    }
    const uint32_t nj = (uint32_t)jobs.size();

    // 2. Device job table and binomial columns.
    ClockCal clock;
    std::vector<bcdev::Job> hjobs(nj);
    std::vector<uint64_t> tab_off(nj + 1, 0);
    std::vector<std::vector<u128>> cols(nj);
    for (uint32_t j = 0; j < nj; ++j) {
        const HostJob &hj = jobs[j];
        const bc_graph *g = specs[hj.spec].g;
        const Side &A = g->side[hj.anchor];
        uint32_t n_ovf = 0, n_u64 = 0, n_u58 = 0, n_u28 = 0;
        binom_column(A.max_deg, hj.qA, cols[j], n_ovf, n_u64, n_u58, n_u28);
        bcdev::Job &d = hjobs[j];
        memset(&d, 0, sizeof(d));
        d.ptrA = A.d_ptr;
        d.adjA = A.d_adj;
        d.rposA = A.d_rpos;
        d.ptrB = g->side[1 - hj.anchor].d_ptr;
        d.adjB = g->side[1 - hj.anchor].d_adj;
        d.nA = (uint32_t)A.n;
        d.nB = (uint32_t)g->side[1 - hj.anchor].n;
        d.root_lo = hj.root_lo;
        d.root_hi = hj.root_hi;
        d.pA = hj.pA;
        d.qA = hj.qA;
        d.binom_n = A.max_deg + 1;
        d.n_ovf = n_ovf;
        d.n_u64 = n_u64;
        d.n_u58 = n_u58;
        d.n_u28 = n_u28;
        d.slot = j;
        d.deadline = 0;
        const uint64_t dl = specs[hj.spec].deadline_ns;
        if (dl) {
            if (!clock.ok) {
                if (bc_status e = device_clock(device, st, mem, clock)) return e;
            }
            const double t = clock.offset + clock.ticks_per_ns * (double)dl;
            d.deadline = t < 1.0 ? 1ull : (uint64_t)t;
        }
        tab_off[j + 1] = tab_off[j] + cols[j].size();
    }
    // per-vertex counters (two 64-bit words per vertex of the anchor side)
    bool any_pv = false;
    std::vector<uint64_t *> d_pv(nj, nullptr);
    for (uint32_t j = 0; j < nj; ++j) {
        if (!specs[jobs[j].spec].pv_out) continue;
        any_pv = true;
        const uint64_t n = specs[jobs[j].spec].g->side[jobs[j].anchor].n;
        BC_HIP(mem.get(&d_pv[j], 2 * std::max<uint64_t>(n, 1)));
        BC_HIP(fill_u32((uint32_t *)d_pv[j], 4 * std::max<uint64_t>(n, 1), 0u, st));
        hjobs[j].pv = d_pv[j];
    }
    bcdev::Job *d_jobs;
    u128 *d_tab;
    bcdev::Slot *d_slots;
    unsigned long long *d_queue;
    BC_HIP(mem.get(&d_jobs, nj));
    BC_HIP(mem.get(&d_tab, tab_off[nj]));
    BC_HIP(mem.get(&d_slots, nj + 1));   // slot nj: sample jobs
    BC_HIP(mem.get(&d_queue, 12));
    {
        std::vector<u128> tab(tab_off[nj]);
        for (uint32_t j = 0; j < nj; ++j) {
            std::copy(cols[j].begin(), cols[j].end(), tab.begin() + tab_off[j]);
            hjobs[j].binom = d_tab + tab_off[j];
        }
        BC_HIP(hipMemcpyAsync(d_tab, tab.data(), tab.size() * sizeof(u128), hipMemcpyHostToDevice, st));
        BC_HIP(hipMemcpyAsync(d_jobs, hjobs.data(), nj * sizeof(bcdev::Job), hipMemcpyHostToDevice, st));
        BC_HIP(hipStreamSynchronize(st));  // host vectors go out of scope
    }
    BC_HIP(bcdev::launch_fill_slots(d_slots, nj + 1, st));
    BC_HIP(fill_u32((uint32_t *)d_queue, 24, 0u, st));

    Timer tm(stats != nullptr && !ex.fixed);
    tm.mark(0, st);

    // 3. pA == 1: degree sums.
    std::vector<uint32_t> deg_jobs;
    for (uint32_t j = 0; j < nj; ++j)
        if (!jobs[j].trivial_zero && jobs[j].pA == 1) deg_jobs.push_back(j);
    if (!deg_jobs.empty()) {
        uint32_t *d_ids;
        BC_HIP(mem.get(&d_ids, deg_jobs.size()));
        BC_HIP(hipMemcpyAsync(d_ids, deg_jobs.data(), deg_jobs.size() * 4, hipMemcpyHostToDevice, st));
        BC_HIP(bcdev::launch_degree_sum(d_jobs, d_ids, (uint32_t)deg_jobs.size(), d_slots, st));
    }

    // The fused per-root kernel (LDS counting, rows bump-allocated on the
    // device) needs 144 KiB of LDS per block and a pool sized up front; the
    // two-kernel path (count, plan, rows) is the fallback.
    const bool fused = !two_pass && lds_per_block(device) >= 148 * 1024;
    // Counter scratch of the candidate passes: per block, three u32 arrays over
    // the widest anchor side of any job (all zero between roots).  Blocks of
    // every candidate-pass launch are capped at rs_blocks.
    bcdev::RootScratch rs{};
    uint32_t rs_blocks = 0;
    {
        uint32_t nA_all = 0;
        for (uint32_t j = 0; j < nj; ++j)
            if (!jobs[j].trivial_zero && jobs[j].pA >= 2) nA_all = std::max(nA_all, hjobs[j].nA);
        if (nA_all) {
            uint64_t nb = (uint64_t)ncu * 2;
            if (ex.fixed || mem.cap)   // at most a quarter of the fixed region or cap
                nb = std::max<uint64_t>(1, std::min<uint64_t>(nb, mem.room() / 4 / (12ull * nA_all)));
            rs_blocks = (uint32_t)nb;
            rs.stride = nA_all;
            BC_HIP(mem.get(&rs.cnt, (uint64_t)rs_blocks * nA_all));
            BC_HIP(mem.get(&rs.touched, (uint64_t)rs_blocks * nA_all));
            BC_HIP(mem.get(&rs.cand, (uint64_t)rs_blocks * nA_all));
            BC_HIP(fill_u32(rs.cnt, (uint64_t)rs_blocks * nA_all, 0u, st));
        }
    }

    // 4a. Specs with both anchors as candidates: estimate each side's
    //     planning cost from a rank-stratified sample of its roots
    //     (kSampleChunk consecutive ranks out of every kSamplePeriod), counted
    //     as candidate-only jobs (p_A = 2, spare slot), and drop a side that is
    //     dearer by more than the margin.  Within the margin the side whose
    //     candidate pass scans fewer wedges is kept.
    if (fused) {
        constexpr uint32_t kSampleChunk = 16, kSamplePeriod = 256;
        constexpr uint64_t kSampleMinRoots = 65536;
        constexpr double kSampleMargin = 1.15;
        std::vector<bcdev::Job> sjobs;
        std::vector<uint32_t> sowner;            // jobs[] index of each sample job
        std::vector<uint64_t> sprefix(1, 0);
        for (size_t i = 0; i < ns; ++i) {
            if (spec_jobs[i].size() != 2) continue;
            const int a = spec_jobs[i][0], b = spec_jobs[i][1];
            if (jobs[a].trivial_zero || jobs[b].trivial_zero || jobs[a].pA < 3 || jobs[b].pA < 3) continue;
            const uint64_t span = (uint64_t)(jobs[a].root_hi - jobs[a].root_lo) + (jobs[b].root_hi - jobs[b].root_lo);
            if (span < kSampleMinRoots) continue;
            for (int j : {a, b}) {
                for (uint64_t c = jobs[j].root_lo; c < jobs[j].root_hi; c += kSamplePeriod) {
                    bcdev::Job sj = hjobs[j];
                    sj.root_lo = (uint32_t)c;
                    sj.root_hi = (uint32_t)std::min<uint64_t>(c + kSampleChunk, jobs[j].root_hi);
                    sj.pA = 2;
                    sj.slot = nj;
                    sj.pv = nullptr;
                    sjobs.push_back(sj);
                    sowner.push_back((uint32_t)j);
                    sprefix.push_back(sprefix.back() + (sj.root_hi - sj.root_lo));
                }
            }
        }
        if (!sjobs.empty()) {
            const uint64_t s_roots = sprefix.back();
            bcdev::Job *d_sj;
            uint64_t *d_sp, *d_soff, *d_spool;
            uint32_t *d_sk;
            BC_HIP(mem.get(&d_sj, sjobs.size()));
            BC_HIP(mem.get(&d_sp, sprefix.size()));
            BC_HIP(mem.get(&d_sk, s_roots));
            BC_HIP(mem.get(&d_soff, s_roots));
            BC_HIP(mem.get(&d_spool, 1));
            BC_HIP(hipMemcpyAsync(d_sj, sjobs.data(), sjobs.size() * sizeof(bcdev::Job), hipMemcpyHostToDevice, st));
            BC_HIP(hipMemcpyAsync(d_sp, sprefix.data(), sprefix.size() * 8, hipMemcpyHostToDevice, st));
            const uint32_t s_blocks = (uint32_t)std::min<uint64_t>(
                std::min<uint64_t>(s_roots, rs_blocks),
                std::max<uint64_t>(1, (uint64_t)ncu * std::min(waves_per_cu, 12u) / 12));
            BC_HIP(bcdev::launch_root_build(d_sj, d_sp, (uint32_t)sjobs.size(), s_roots, rs, d_spool, 1, s_blocks,
                                            d_queue + 6, d_sk, d_soff, d_slots, false, st));
            std::vector<uint32_t> sk(s_roots);
            BC_HIP(hipMemcpyAsync(sk.data(), d_sk, s_roots * 4, hipMemcpyDeviceToHost, st));
            BC_HIP(hipStreamSynchronize(st));
            std::vector<double> est(nj, 0.0), seen(nj, 0.0);
            for (size_t s = 0; s < sjobs.size(); ++s) {
                const uint32_t j = sowner[s];
                const Side &A = specs[jobs[j].spec].g->side[jobs[j].anchor];
                const uint32_t e = std::min<uint32_t>(jobs[j].pA - 1, 3);
                for (uint64_t r = sprefix[s]; r < sprefix[s + 1]; ++r) {
                    const double k = sk[r];
                    const uint64_t u = sjobs[s].root_lo + (r - sprefix[s]);
                    seen[j] += 1.0;
                    if (k < jobs[j].pA - 1) continue;
                    double x = k * (double)((A.h_ptr[u + 1] - A.h_ptr[u] + 63) / 64);
                    for (uint32_t t = 1; t < e; ++t) x *= k;
                    est[j] += x;
                }
            }
            for (size_t i = 0; i < ns; ++i) {
                if (spec_jobs[i].size() != 2) continue;
                const int a = spec_jobs[i][0], b = spec_jobs[i][1];
                if (seen[a] == 0.0 || seen[b] == 0.0) continue;
                const double ca = est[a] * (jobs[a].root_hi - jobs[a].root_lo) / seen[a];
                const double cb = est[b] * (jobs[b].root_hi - jobs[b].root_lo) / seen[b];
                int drop;
                if (ca * kSampleMargin < cb) drop = b;
                else if (cb * kSampleMargin < ca) drop = a;
                else {
                    // a wedge u - v - w of anchor A passes through v on the other side
                    const bc_graph *g = specs[i].g;
                    drop = g->side[1 - jobs[a].anchor].deg_pairs <= g->side[1 - jobs[b].anchor].deg_pairs ? b : a;
                }
                jobs[drop].dropped = true;
                spec_jobs[i] = {drop == a ? b : a};
            }
        }
    }

    // 4b. Candidate pass over all roots of jobs with pA >= 2.
    std::vector<uint32_t> cj;   // jobs in the candidate pass
    std::vector<uint64_t> root_prefix(1, 0);
    for (uint32_t j = 0; j < nj; ++j)
        if (!jobs[j].trivial_zero && !jobs[j].dropped && jobs[j].pA >= 2) cj.push_back(j);
    if (short_first)   // served batches: the small graphs' candidate passes first
        std::stable_sort(cj.begin(), cj.end(), [&](uint32_t a, uint32_t b) {
            return specs[jobs[a].spec].g->nnz < specs[jobs[b].spec].g->nnz;
        });
    for (uint32_t j : cj) {
        root_prefix.push_back(root_prefix.back() + (jobs[j].root_hi - jobs[j].root_lo));
    }
    const uint64_t total_roots = root_prefix.back();
    std::vector<uint32_t> h_k(total_roots);
    std::vector<uint64_t> h_off;
    const uint32_t root_blocks =
        (uint32_t)std::min<uint64_t>(std::max<uint64_t>(total_roots, 1), std::max<uint32_t>(rs_blocks, 1));
    std::vector<bcdev::Job> cjobs;
    bcdev::Job *d_cjobs = nullptr;
    uint64_t *d_pool_fused = nullptr;
    uint64_t pool_cap = 0;
    if (total_roots) {
        // the candidate pass runs over its own compact job table
        cjobs.reserve(cj.size());
        for (uint32_t j : cj) cjobs.push_back(hjobs[j]);
        uint64_t *d_rp;
        uint32_t *d_k;
        BC_HIP(mem.get(&d_cjobs, cjobs.size()));
        BC_HIP(mem.get(&d_rp, root_prefix.size()));
        BC_HIP(mem.get(&d_k, total_roots));
        BC_HIP(hipMemcpyAsync(d_cjobs, cjobs.data(), cjobs.size() * sizeof(bcdev::Job), hipMemcpyHostToDevice, st));
        BC_HIP(hipMemcpyAsync(d_rp, root_prefix.data(), root_prefix.size() * 8, hipMemcpyHostToDevice, st));
        if (fused) {
            // room for the rows of every root: a generous multiple of the
            // edges; a root that finds no room is rebuilt by the two-kernel path
            uint64_t nnz_sum = 0;
            for (uint32_t j : cj) nnz_sum += specs[jobs[j].spec].g->nnz;
            pool_cap = std::max<uint64_t>(1ull << 22, 32 * nnz_sum + (4ull << 20));
            // a fixed region gives the pool at most a third of what is left;
            // roots that find no room are rebuilt into an exactly sized pool
            if (ex.fixed || mem.cap) pool_cap = std::max<uint64_t>(1, std::min<uint64_t>(pool_cap, mem.room() / 3 / 8));
            uint64_t *d_off;
            BC_HIP(mem.get(&d_off, total_roots));
            BC_HIP(mem.get(&d_pool_fused, pool_cap));
            // one block of kRbThreads per CU (its LDS table takes most of the
            // CU's LDS); a reduced waves_per_cu takes the same share of CUs
            const uint32_t fused_blocks = (uint32_t)std::min<uint64_t>(
                std::min<uint64_t>(total_roots, rs_blocks),
                std::max<uint64_t>(1, (uint64_t)ncu * std::min(waves_per_cu, 12u) / 12));
            // per-vertex counts of p_A = 2 jobs are attributed by this pass
            BC_HIP(bcdev::launch_root_build(d_cjobs, d_rp, (uint32_t)cj.size(), total_roots, rs, d_pool_fused, pool_cap,
                                            fused_blocks, d_queue + 4, d_k, d_off, d_slots, any_pv, st));
            h_off.resize(total_roots);
            BC_HIP(hipMemcpyAsync(h_off.data(), d_off, total_roots * 8, hipMemcpyDeviceToHost, st));
        } else {
            BC_HIP(bcdev::launch_cand_count(d_cjobs, d_rp, (uint32_t)cj.size(), total_roots, rs, root_blocks,
                                            d_queue + 0, d_k, d_slots, st));
        }
        BC_HIP(hipMemcpyAsync(h_k.data(), d_k, total_roots * 4, hipMemcpyDeviceToHost, st));
    }
    tm.mark(1, st);
    BC_HIP(hipStreamSynchronize(st));
    auto t_plan0 = std::chrono::steady_clock::now();

    // 5. Plan: per-job cost proxies, anchor choice, active roots, pool.
    std::vector<char> job_live(nj, 1);
    for (uint32_t c = 0; c < cj.size(); ++c) {
        const uint32_t j = cj[c];
        const HostJob &hj = jobs[j];
        const Side &A = specs[hj.spec].g->side[hj.anchor];
        uint64_t cost = 0, weight = 0;
        const uint32_t e = std::min<uint32_t>(hj.pA - 1, 3);
        for (uint64_t r = root_prefix[c]; r < root_prefix[c + 1]; ++r) {
            uint64_t k = h_k[r];
            uint64_t u = hj.root_lo + (r - root_prefix[c]);
            uint64_t w1 = (A.h_ptr[u + 1] - A.h_ptr[u] + 63) / 64;
            uint64_t x = k * w1;
            for (uint32_t t = 1; t < e; ++t) x = std::min<uint64_t>(x * k, 1ull << 62);
            cost = std::min<uint64_t>(cost + x, 1ull << 62);
            // the whole depth, for ordering jobs against each other
            for (uint32_t t = e; t + 1 < hj.pA; ++t) x = std::min<uint64_t>(x * k, 1ull << 62);
            weight = std::min<uint64_t>(weight + x, 1ull << 62);
        }
        jobs[j].cost = cost;
        jobs[j].weight = weight;
    }
    for (size_t i = 0; i < ns; ++i) {
        if (spec_jobs[i].size() == 2) {
            int a = spec_jobs[i][0], b = spec_jobs[i][1];
            if (jobs[b].cost < jobs[a].cost) std::swap(a, b);
            job_live[b] = 0;
            spec_jobs[i] = {a};
        }
    }
    // Served batches: a job that the cost model says cannot finish before its
    // deadline, even at the best rate seen for its depth, is refused here,
    // before the enumeration, instead of holding the device until it expires.
    std::vector<char> refused(nj, 0);
    if (short_first) {
        RateBook &rb = rate_book();
        std::lock_guard<std::mutex> lk(rb.mu);
        const uint64_t now = bcint::steady_ns();
        for (uint32_t j : cj) {
            const uint64_t dl = specs[jobs[j].spec].deadline_ns;
            const uint32_t pA = jobs[j].pA;
            if (!job_live[j] || !dl || pA < 3 || pA > 32 || rb.ns_per_unit[pA] <= 0) continue;
            const double left = dl > now ? (double)(dl - now) : 0.0;
            if ((double)jobs[j].weight * rb.ns_per_unit[pA] > kRefuseMargin * left) {
                refused[j] = 1;
                job_live[j] = 0;
            }
        }
    }
    struct Plan {
        uint32_t c;  // index into cj / cjobs
        uint32_t root, k, w1;
        uint64_t cost;
        uint64_t item;   // index of the root in the candidate pass
    };
    std::vector<Plan> plan;
    uint64_t cand_edges = 0;
    for (uint32_t c = 0; c < cj.size(); ++c) {
        const uint32_t j = cj[c];
        if (!job_live[j]) continue;
        const HostJob &hj = jobs[j];
        const Side &A = specs[hj.spec].g->side[hj.anchor];
        const std::vector<uint8_t> *mask = specs[hj.spec].root_mask;
        for (uint64_t r = root_prefix[c]; r < root_prefix[c + 1]; ++r) {
            cand_edges += h_k[r];
            // per-vertex counts of p_A = 2 jobs: the fused candidate pass
            // attributes their leaves; the two-kernel pass does not, so then
            // their roots take the global-set path
            if (hj.pA < (specs[hj.spec].pv_out && !fused ? 2u : 3u) || h_k[r] < hj.pA - 1) continue;
            uint32_t u = (uint32_t)(hj.root_lo + (r - root_prefix[c]));
            if (mask && !(*mask)[u]) continue;
            uint32_t w1 = (uint32_t)((A.h_ptr[u + 1] - A.h_ptr[u] + 63) / 64);
            uint64_t k = h_k[r];
            uint64_t x = k * w1;
            const uint32_t e = std::min<uint32_t>(hj.pA - 1, 3);
            for (uint32_t t = 1; t < e; ++t) x = std::min<uint64_t>(x * k, 1ull << 62);
            plan.push_back(Plan{c, u, (uint32_t)k, w1, x, r});
        }
    }
    if (short_first)
        std::stable_sort(plan.begin(), plan.end(), [&](const Plan &a, const Plan &b) {
            const uint64_t ca = jobs[cj[a.c]].weight, cb = jobs[cj[b.c]].weight;
            if (ca != cb) return ca < cb;
            if (a.c != b.c) return a.c < b.c;
            return a.cost > b.cost;
        });
    else {
        std::vector<uint64_t> cost(plan.size());
        for (size_t r = 0; r < plan.size(); ++r) cost[r] = plan[r].cost;
        const std::vector<uint32_t> ord = order_by_cost_desc(cost);
        std::vector<Plan> sorted(plan.size());
        for (size_t r = 0; r < plan.size(); ++r) sorted[r] = plan[ord[r]];
        plan.swap(sorted);
    }
    // Roots of the global-set path: all of them with sets = HTB or SORTED;
    // with local bitmaps, those with more neighbours than bitmap_bits (they
    // take HTB).  Jobs with per-vertex counts send all their roots there: it
    // visits every leaf with its members known.  They keep their place in
    // the cost order.
    std::vector<Plan> splan;
    const uint32_t set_mode = sets_opt == BC_SETS_SORTED ? bcdev::SETS_SORTED : bcdev::SETS_HTB;
    if (sets_opt != BC_SETS_LOCAL_BITMAP || bitmap_bits || any_pv) {
        std::vector<Plan> keep;
        for (const Plan &pl : plan) {
            const HostJob &hj = jobs[cj[pl.c]];
            const Side &A = specs[hj.spec].g->side[hj.anchor];
            const uint64_t du = A.h_ptr[pl.root + 1] - A.h_ptr[pl.root];
            const bool to_sets = sets_opt != BC_SETS_LOCAL_BITMAP || (bitmap_bits && du > bitmap_bits) ||
                                 specs[hj.spec].pv_out != nullptr;
            (to_sets ? splan : keep).push_back(pl);
        }
        plan.swap(keep);
    }
    std::vector<bcdev::SetRoot> sroots(splan.size());
    uint64_t set_tasks = 0, set_ids = 0, set_slab_need = 64;
    if (!splan.empty()) {
        if (set_mode == bcdev::SETS_HTB) {
            std::vector<char> done(cj.size(), 0);
            for (const Plan &pl : splan) {
                if (done[pl.c]) continue;
                done[pl.c] = 1;
                const HostJob &hj = jobs[cj[pl.c]];
                bc_graph *g = const_cast<bc_graph *>(specs[hj.spec].g);   // the HTB is a cache of the graph
                if (bc_status e = ensure_htb(g, hj.anchor, st)) return e;
                const Side &A = g->side[hj.anchor];
                cjobs[pl.c].htb_off = A.d_htb_off;
                cjobs[pl.c].htb_idx = A.d_htb_idx;
                cjobs[pl.c].htb_val = A.d_htb_val;
            }
            BC_HIP(hipMemcpyAsync(d_cjobs, cjobs.data(), cjobs.size() * sizeof(bcdev::Job), hipMemcpyHostToDevice, st));
        }
        for (size_t r = 0; r < splan.size(); ++r) {
            const Plan &pl = splan[r];
            const HostJob &hj = jobs[cj[pl.c]];
            const Side &A = specs[hj.spec].g->side[hj.anchor];
            const uint32_t pA = cjobs[pl.c].pA;
            bcdev::SetRoot &a = sroots[r];
            a.id_off = set_ids;
            a.task_begin = set_tasks;
            a.job = pl.c;
            a.root = pl.root;
            a.k = pl.k;
            a.n_tasks = pl.k - (pA - 2);
            set_ids += pl.k;
            set_tasks += a.n_tasks;
            // per task: one set and one kept list per level 2 .. pA-1, each
            // set at most the root's own row (words or ids), each list at most k ids
            const uint64_t mu = set_mode == bcdev::SETS_HTB ? A.h_htb_off[pl.root + 1] - A.h_htb_off[pl.root]
                                                            : A.h_ptr[pl.root + 1] - A.h_ptr[pl.root];
            set_slab_need = std::max<uint64_t>(set_slab_need, (uint64_t)pA * (mu + pl.k / 2 + 2) + 16);
        }
    }
    std::vector<bcdev::ActiveRoot> aroots(plan.size());
    uint64_t pool_words = 0, tasks = 0, slab_need = 64;
    // rows already built by the fused kernel, unless some root found no room
    bool rows_ready = fused;
    for (const Plan &pl : plan)
        if (fused && h_off[pl.item] == ~0ull) rows_ready = false;
    for (size_t r = 0; r < plan.size(); ++r) {
        const Plan &pl = plan[r];
        const uint32_t pA = cjobs[pl.c].pA;
        bcdev::ActiveRoot &a = aroots[r];
        a.pool_off = rows_ready ? h_off[pl.item] : pool_words;
        a.task_begin = tasks;
        a.job = pl.c;
        a.root = pl.root;
        a.k = pl.k;
        a.n_tasks = pl.k - (pA - 2);
        pool_words += (uint64_t)pl.k * pl.w1;
        tasks += a.n_tasks;
        // per task: S2 and its prefix counts (2 W1), the compress table of
        // S2's nonzero words (8 W1), the kept-row list of the level-2 filter
        // (k / 2 + 1), then one block per DFS level 2 .. pA-2, each at most
        // (k - 1) rows of at most W1 words
        // (p_A >= 5: plus the pair rows of one small node's three-level sum,
        // at most kTripleRows (kTripleRows - 1) / 2 rows of at most 4 words
        // and their u32 indices)
        const uint64_t pairs3 = (uint64_t)bcdev::kTripleRows * (bcdev::kTripleRows - 1) / 2;
        uint64_t need = 10ull * pl.w1 + pl.k / 2 + 1 + (pA >= 5 ? pairs3 * 4 + (pairs3 + 1) / 2 : 0) +
                        (pA >= 4 ? (uint64_t)(pA - 3) * (pl.k - 1) * pl.w1 : 0) + 8;
        slab_need = std::max(slab_need, need);
    }
    const double ms_plan =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_plan0).count();

    tm.mark(2, st);
    const uint64_t t_enum0 = bcint::steady_ns();
    unsigned long long *d_wave_clock = nullptr;   // instrumented: per-wave start / end clocks
    uint64_t n_wave_clock = 0;
    if (!plan.empty()) {
        bcdev::ActiveRoot *d_roots;
        uint64_t *d_pool = d_pool_fused;
        BC_HIP(mem.get(&d_roots, aroots.size()));
        BC_HIP(hipMemcpyAsync(d_roots, aroots.data(), aroots.size() * sizeof(bcdev::ActiveRoot), hipMemcpyHostToDevice,
                              st));
        if (!rows_ready) {
            BC_HIP(mem.get(&d_pool, pool_words));
            BC_HIP(bcdev::launch_rows_build(d_cjobs, d_roots, (uint32_t)aroots.size(), d_pool, rs, root_blocks,
                                            d_queue + 1, d_slots, st));
        }
        tm.mark(3, st);
        // Runtime split (queries with p_A >= 5): a subtask ring of up to 4M
        // entries of 16 bytes, cleared before the launch, and a heap of up to
        // 64M words for the split tasks' level-2 blocks.
        uint32_t split_cap = 0;
        uint4 *d_ring = nullptr;
        unsigned long long *d_sub = nullptr;
        uint64_t *d_heap = nullptr;
        uint64_t heap_words = 0;
        bool any_deep = false;
        for (const bcdev::ActiveRoot &a : aroots) any_deep = any_deep || cjobs[a.job].pA >= 5;
        if (any_deep && split_rows != 0 && split_rows != 0xffffffffu) {
            uint64_t cap = 1ull << 22;
            if (ex.fixed || mem.cap) cap = std::min<uint64_t>(cap, mem.room() / 4 / sizeof(uint4));
            uint64_t hw = 1ull << 26;
            if (ex.fixed || mem.cap) hw = std::min<uint64_t>(hw, mem.room() / 4 / 8);
            if (cap >= 1024 && hw >= 4096) {
                BC_HIP(mem.get(&d_ring, cap));
                BC_HIP(mem.get(&d_sub, 4));
                BC_HIP(mem.get(&d_heap, hw));
                BC_HIP(fill_u32((uint32_t *)d_ring, cap * 4, 0u, st));
                BC_HIP(fill_u32((uint32_t *)d_sub, 8, 0u, st));
                split_cap = (uint32_t)cap;
                heap_words = hw;
            }
        }
        // Enumeration grid: waves_per_cu wavefronts per CU; each wave owns a
        // slab big enough for the deepest task of this plan.
        uint32_t blocks = (uint32_t)std::max<uint64_t>(1, (uint64_t)ncu * waves_per_cu / bcdev::kWavesPerBlock);
        uint64_t slab_budget = 64ull << 30;   // bytes of HBM for all slabs
        slab_budget = std::min(slab_budget, mem.room() > 512 ? mem.room() - 512 : 0);
        while (blocks > 1 && (uint64_t)blocks * bcdev::kWavesPerBlock * slab_need * 8 > slab_budget) blocks /= 2;
        uint64_t *d_slab;
        BC_HIP(mem.get(&d_slab, (uint64_t)blocks * bcdev::kWavesPerBlock * slab_need));
        bcdev::EnumParams prm{};
        prm.jobs = d_cjobs;
        prm.roots = d_roots;
        prm.n_roots = (uint32_t)aroots.size();
        prm.n_tasks = tasks;
        // launches with many tasks per wave take them 8 at a time (fewer
        // queue atomics and root searches; consecutive tasks share their
        // root's rows), small ones 4 at a time (a more even spread)
        prm.task_chunk = roots_per_wave ? roots_per_wave
                                        : (tasks >= 1024ull * blocks * bcdev::kWavesPerBlock ? 8u : 4u);
        prm.triple = switch_depth == 2 ? 0u : 1u;
        prm.split_rows = split_rows ? split_rows : 256u;
        prm.split_cap = split_cap;
        prm.ring = d_ring;
        if (instrument) {
            BC_HIP(mem.get(&d_wave_clock, 2ull * blocks * bcdev::kWavesPerBlock));
            BC_HIP(fill_u32((uint32_t *)d_wave_clock, 4ull * blocks * bcdev::kWavesPerBlock, 0u, st));
            n_wave_clock = (uint64_t)blocks * bcdev::kWavesPerBlock;
        }
        prm.wave_clock = d_wave_clock;
        prm.sub_head = d_sub;
        prm.sub_tail = d_sub ? d_sub + 1 : nullptr;
        prm.split_heap = d_heap;
        prm.split_heap_words = heap_words;
        prm.pool = d_pool;
        prm.slab = d_slab;
        prm.slab_words = slab_need;
        prm.lds_words = lds_words;
        prm.instrument = instrument ? 1u : 0u;
        prm.queue = d_queue + 2;
        prm.slots = d_slots;
        BC_HIP(bcdev::launch_enumerate(prm, blocks, st));
    } else {
        tm.mark(3, st);
    }
    if (!splan.empty()) {
        // global-set path: candidate ids, then the enumeration over them
        bcdev::SetRoot *d_sroots;
        uint32_t *d_ids;
        BC_HIP(mem.get(&d_sroots, sroots.size()));
        BC_HIP(mem.get(&d_ids, set_ids));
        BC_HIP(hipMemcpyAsync(d_sroots, sroots.data(), sroots.size() * sizeof(bcdev::SetRoot), hipMemcpyHostToDevice,
                              st));
        BC_HIP(bcdev::launch_cand_ids(d_cjobs, d_sroots, (uint32_t)sroots.size(), d_ids, rs,
                                      (uint32_t)std::min<uint64_t>(sroots.size(), std::max<uint32_t>(rs_blocks, 1)),
                                      d_queue + 8, d_slots, st));
        uint32_t blocks = (uint32_t)std::max<uint64_t>(1, (uint64_t)ncu * waves_per_cu / bcdev::kWavesPerBlock);
        uint64_t slab_budget = 64ull << 30;
        slab_budget = std::min(slab_budget, mem.room() > 512 ? mem.room() - 512 : 0);
        while (blocks > 1 && (uint64_t)blocks * bcdev::kWavesPerBlock * set_slab_need * 8 > slab_budget) blocks /= 2;
        uint64_t *d_sslab;
        BC_HIP(mem.get(&d_sslab, (uint64_t)blocks * bcdev::kWavesPerBlock * set_slab_need));
        bcdev::SetParams sp{};
        sp.jobs = d_cjobs;
        sp.roots = d_sroots;
        sp.n_roots = (uint32_t)sroots.size();
        sp.task_chunk = roots_per_wave ? roots_per_wave : 4u;
        sp.n_tasks = set_tasks;
        sp.ids = d_ids;
        sp.mode = set_mode;
        sp.instrument = instrument ? 1u : 0u;
        sp.pure_dfs = (BC_OPT(opts, pure_dfs, 0u) && !any_pv) ? 1u : 0u;   // per-vertex needs the hybrid
        sp.slab = d_sslab;
        sp.slab_words = set_slab_need;
        sp.queue = d_queue + 9;
        sp.slots = d_slots;
        BC_HIP(bcdev::launch_enumerate_sets(sp, blocks, st));
        tasks += set_tasks;
    }
    tm.mark(4, st);
    std::vector<bcdev::Slot> hs(nj);
    BC_HIP(hipMemcpyAsync(hs.data(), d_slots, nj * sizeof(bcdev::Slot), hipMemcpyDeviceToHost, st));
    std::vector<std::vector<uint64_t>> h_pv(nj);
    for (uint32_t j = 0; j < nj; ++j) {
        if (!d_pv[j]) continue;
        h_pv[j].resize(2 * specs[jobs[j].spec].g->side[jobs[j].anchor].n);
        if (!h_pv[j].empty())
            BC_HIP(hipMemcpyAsync(h_pv[j].data(), d_pv[j], h_pv[j].size() * 8, hipMemcpyDeviceToHost, st));
    }
    BC_HIP(hipStreamSynchronize(st));
    read_back = true;
    for (uint32_t j = 0; j < nj; ++j)
        for (size_t r = 0; 2 * r < h_pv[j].size(); ++r)
            specs[jobs[j].spec].pv_out[r] = bc_u128{h_pv[j][2 * r], h_pv[j][2 * r + 1]};
    if (short_first) {
        // learn from a served batch that enumerated exactly one job to the end
        int only = -1, live = 0;
        for (uint32_t j : cj)
            if (job_live[j] && jobs[j].pA >= 3) {
                only = (int)j;
                ++live;
            }
        if (live == 1 && jobs[only].weight > 0 && !(hs[only].flags & (bcdev::FLAG_TIMEOUT | bcdev::FLAG_CAPACITY))) {
            const double ns = (double)(bcint::steady_ns() - t_enum0) / (double)jobs[only].weight;
            RateBook &rb = rate_book();
            std::lock_guard<std::mutex> lk(rb.mu);
            double &r = rb.ns_per_unit[jobs[only].pA];
            r = r > 0 ? std::min(r, ns) : ns;
        }
    }

    // 6. Results.  Candidate jobs for the same spec: only the live one counts.
    bc_status overall = BC_OK;
    for (size_t i = 0; i < ns; ++i) {
        const int j = spec_jobs[i][0];
        const bcdev::Slot &s = hs[j];
        if (jobs[j].trivial_zero) {
            out[i] = bc_u128{0, 0};
            continue;
        }
        if (refused[j]) {
            item_status[i] = BC_E_REJECTED;
            g_last_error = "refused: the cost model puts the count past its deadline";
        } else if (s.flags & bcdev::FLAG_TIMEOUT) {
            item_status[i] = BC_E_TIMEOUT;
            g_last_error = "time limit reached before the count finished";
        } else if (s.flags & bcdev::FLAG_OVERFLOW) {
            item_status[i] = BC_E_OVERFLOW;
            g_last_error = "count exceeds 128 bits";
        } else if (s.flags & (bcdev::FLAG_CAPACITY | bcdev::FLAG_MISMATCH)) {
            item_status[i] = BC_E_DEVICE;
            g_last_error = (s.flags & bcdev::FLAG_CAPACITY) ? "internal: enumeration scratch bound exceeded"
                                                             : "internal: candidate passes disagree";
            overall = BC_E_DEVICE;
        } else {
            out[i] = bc_u128{s.lo, s.hi};
        }
    }
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->ms_candidates = tm.ms(0, 1);
        stats->ms_plan = ms_plan;
        stats->ms_rows = tm.ms(2, 3);
        stats->ms_enumerate = tm.ms(3, 4);
        stats->ms_total =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_host0).count();
        stats->anchor = jobs[spec_jobs[0][0]].anchor;
        stats->roots = total_roots;
        stats->roots_active = plan.size();
        stats->tasks = tasks;
        stats->candidate_edges = cand_edges;
        stats->row_words = pool_words;
        stats->scratch_bytes = mem.total;
        if (n_wave_clock) {
            // device clock at 100 MHz: 1e5 ticks per millisecond
            std::vector<unsigned long long> wc(2 * n_wave_clock);
            if (hipMemcpy(wc.data(), d_wave_clock, wc.size() * 8, hipMemcpyDeviceToHost) == hipSuccess) {
                unsigned long long s0 = ~0ull, e0 = ~0ull, e1 = 0;
                for (uint64_t w = 0; w < n_wave_clock; ++w) {
                    if (!wc[2 * w + 1]) continue;
                    s0 = std::min(s0, wc[2 * w]);
                    e0 = std::min(e0, wc[2 * w + 1]);
                    e1 = std::max(e1, wc[2 * w + 1]);
                }
                if (e1) {
                    stats->ms_wave_makespan = (double)(e1 - s0) / 1e5;
                    stats->ms_wave_spread = (double)(e1 - e0) / 1e5;
                }
            }
        }
        for (size_t i = 0; i < ns; ++i) {
            const bcdev::Slot &sl = hs[spec_jobs[i][0]];
            stats->pair_ops += sl.pair_ops;
            stats->filter_ops += sl.filter_ops;
            stats->cyc_setup += sl.cyc_setup;
            stats->cyc_compact += sl.cyc_compact;
            stats->cyc_pair += sl.cyc_pair;
            stats->cyc_filter += sl.cyc_filter;
            stats->pairs += sl.pairs;
            stats->pair_slots += sl.pair_slots;
            stats->cyc_pack += sl.cyc_pack;
        }
    }
    return overall;
}

uint64_t opts_deadline(const bc_opts *o)
{
    if (!o || o->struct_size < offsetof(bc_opts, timeout_ms) + sizeof(uint32_t) || o->timeout_ms == 0) return 0;
    return bcint::steady_ns() + (uint64_t)o->timeout_ms * 1000000ull;
}

bc_status check_pq(uint32_t p, uint32_t q)
{
    if (p < 1 || q < 1 || p > 32 || q > 32) return set_error(BC_E_INVALID_ARG, "p and q must be in 1..32");
    return BC_OK;
}

}  // namespace

extern "C" bc_status bc_count(const bc_graph *g, uint32_t p, uint32_t q, const bc_opts *opts, bc_u128 *out,
                              bc_stats *st)
{
    g_last_error.clear();
    if (!g || !out) return set_error(BC_E_INVALID_ARG, "bc_count: NULL argument");
    if (bc_status s = check_pq(p, q)) return s;
    if (bc_status s = check_opts(opts)) return s;
    std::vector<JobSpec> sp{JobSpec{g, p, q, opts ? opts->anchor : BC_ANCHOR_AUTO, 0, 0, false, opts_deadline(opts)}};
    std::vector<bc_u128> res;
    std::vector<bc_status> ist;
    bc_status s = run_jobs(sp, opts, res, ist, st);
    if (s != BC_OK) return s;
    if (ist[0] != BC_OK) return ist[0];
    *out = res[0];
    return BC_OK;
}

extern "C" bc_status bc_count_roots(const bc_graph *g, uint32_t p, uint32_t q, int32_t anchor, uint64_t rank_lo,
                                    uint64_t rank_hi, const bc_opts *opts, bc_u128 *out, bc_stats *st)
{
    g_last_error.clear();
    if (!g || !out) return set_error(BC_E_INVALID_ARG, "bc_count_roots: NULL argument");
    if (bc_status s = check_pq(p, q)) return s;
    if (bc_status s = check_opts(opts)) return s;
    if (anchor != BC_ANCHOR_U && anchor != BC_ANCHOR_V)
        return set_error(BC_E_INVALID_ARG, "bc_count_roots: anchor must be BC_ANCHOR_U or BC_ANCHOR_V");
    if (rank_lo > rank_hi) return set_error(BC_E_INVALID_ARG, "bc_count_roots: rank_lo > rank_hi");
    std::vector<JobSpec> sp{JobSpec{g, p, q, anchor, rank_lo, rank_hi, true, opts_deadline(opts)}};
    std::vector<bc_u128> res;
    std::vector<bc_status> ist;
    bc_status s = run_jobs(sp, opts, res, ist, st);
    if (s != BC_OK) return s;
    if (ist[0] != BC_OK) return ist[0];
    *out = res[0];
    return BC_OK;
}

extern "C" bc_status bc_count_per_vertex(const bc_graph *g, uint32_t p, uint32_t q, int32_t side, const bc_opts *opts,
                                         bc_u128 *counts)
{
    g_last_error.clear();
    if (!g || !counts) return set_error(BC_E_INVALID_ARG, "bc_count_per_vertex: NULL argument");
    if (bc_status s = check_pq(p, q)) return s;
    if (bc_status s = check_opts(opts)) return s;
    if (side != BC_ANCHOR_U && side != BC_ANCHOR_V)
        return set_error(BC_E_INVALID_ARG, "bc_count_per_vertex: side must be BC_ANCHOR_U or BC_ANCHOR_V");
    const Side &A = g->side[side];
    const uint32_t pA = side == BC_ANCHOR_U ? p : q, qA = side == BC_ANCHOR_U ? q : p;
    std::vector<bc_u128> by_rank(A.n, bc_u128{0, 0});
    if (pA == 1) {
        // each vertex x is the whole L of C(d(x), q_A) bicliques
        std::vector<u128> col;
        uint32_t n_ovf = 0, n64 = 0, n58 = 0, n28 = 0;
        binom_column(A.max_deg, qA, col, n_ovf, n64, n58, n28);
        for (uint64_t r = 0; r < A.n; ++r) {
            const uint64_t d = A.h_ptr[r + 1] - A.h_ptr[r];
            if (d >= n_ovf) return set_error(BC_E_OVERFLOW, "count exceeds 128 bits");
            by_rank[r] = bc_u128{(uint64_t)col[d], (uint64_t)(col[d] >> 64)};
        }
    } else {
        std::vector<JobSpec> sp{JobSpec{g, p, q, side, 0, 0, false, opts_deadline(opts)}};
        sp[0].pv_out = by_rank.data();
        std::vector<bc_u128> res;
        std::vector<bc_status> ist;
        bc_status s = run_jobs(sp, opts, res, ist, nullptr);
        if (s != BC_OK) return s;
        if (ist[0] != BC_OK) return ist[0];
    }
    for (uint64_t x = 0; x < A.n; ++x) counts[x] = by_rank[A.rank_of[x]];
    return BC_OK;
}

extern "C" bc_status bc_count_batch(const bc_graph *const *graphs, const uint32_t *p, const uint32_t *q, size_t n,
                                    const bc_opts *opts, bc_u128 *out, bc_status *item_status, bc_stats *st)
{
    g_last_error.clear();
    if (st) memset(st, 0, sizeof(*st));
    if (n == 0) return BC_OK;
    if (!graphs || !p || !q || !out || !item_status) return set_error(BC_E_INVALID_ARG, "bc_count_batch: NULL argument");
    if (bc_status s = check_opts(opts)) return s;
    std::vector<JobSpec> sp;
    std::vector<size_t> idx;
    const uint64_t dl = opts_deadline(opts);
    int device = -1;
    for (size_t i = 0; i < n; ++i) {
        if (!graphs[i]) continue;
        if (device < 0) device = graphs[i]->device;
        if (graphs[i]->device != device)
            return set_error(BC_E_INVALID_ARG, "bc_count_batch: graphs on different devices");
    }
    for (size_t i = 0; i < n; ++i) {
        out[i] = bc_u128{0, 0};
        if (!graphs[i] || p[i] < 1 || q[i] < 1 || p[i] > 32 || q[i] > 32) {
            item_status[i] = BC_E_INVALID_ARG;
            continue;
        }
        item_status[i] = BC_E_PENDING;   // replaced below in every case
        idx.push_back(i);
        sp.push_back(JobSpec{graphs[i], p[i], q[i], opts ? opts->anchor : BC_ANCHOR_AUTO, 0, 0, false, dl});
    }
    std::vector<bc_u128> res;
    std::vector<bc_status> ist;
    if (sp.empty()) return BC_OK;
    // ist holds the call's status for every item unless the counts were read back
    bc_status s = run_jobs(sp, opts, res, ist, st);
    for (size_t t = 0; t < idx.size(); ++t) {
        item_status[idx[t]] = ist[t];
        out[idx[t]] = ist[t] == BC_OK ? res[t] : bc_u128{0, 0};
    }
    return s;
}

extern "C" bc_status bc_scratch_estimate(const bc_graph *g, uint32_t p, uint32_t q, const bc_opts *opts,
                                         uint64_t *bytes)
{
    g_last_error.clear();
    if (!g || !bytes) return set_error(BC_E_INVALID_ARG, "bc_scratch_estimate: NULL argument");
    if (bc_status s = check_pq(p, q)) return s;
    if (bc_status s = check_opts(opts)) return s;
    *bytes = bcint::estimate_scratch_bytes(g, p, q, (opts && opts->waves_per_cu) ? opts->waves_per_cu : 12u);
    return BC_OK;
}

extern "C" bc_status bc_tune_batch(const bc_graph *const *graphs, const uint32_t *p, const uint32_t *q, size_t n,
                                   const bc_opts *base, bc_opts *tuned)
{
    g_last_error.clear();
    if (!tuned || (n && (!graphs || !p || !q))) return set_error(BC_E_INVALID_ARG, "bc_tune_batch: NULL argument");
    if (bc_status s = check_opts(base)) return s;
    bc_opts b{};
    if (base) b = *base;
    b.struct_size = sizeof(bc_opts);
    *tuned = b;
    if (n == 0) return BC_OK;
    // evenly spaced sample: every step-th item, at least 8 items when there are
    const size_t want = std::max<size_t>(8, n / 16);
    const size_t step = std::max<size_t>(1, n / want);
    std::vector<const bc_graph *> sg;
    std::vector<uint32_t> sp, sq;
    bool deep = false;   // some sampled item can take the runtime split (anchor depth min(p, q) >= 5)
    for (size_t i = 0; i < n; i += step) {
        sg.push_back(graphs[i]);
        sp.push_back(p[i]);
        sq.push_back(q[i]);
        deep = deep || std::min(p[i], q[i]) >= 5;
    }
    std::vector<bc_u128> out(sg.size());
    std::vector<bc_status> st(sg.size());
    // sample time of one schedule (items over the base's time limit count as the whole limit)
    auto timed = [&](const bc_opts &c, double *t) -> bc_status {
        const uint64_t t0 = bcint::steady_ns();
        bc_status s = bc_count_batch(sg.data(), sp.data(), sq.data(), sg.size(), &c, out.data(), st.data(), nullptr);
        if (s != BC_OK) return s;
        *t = (double)(bcint::steady_ns() - t0);
        for (bc_status x : st)
            if (x != BC_OK && b.timeout_ms) *t += (double)b.timeout_ms * 1e6;
        return BC_OK;
    };
    // Coordinate descent: each knob in turn takes the value with the shortest
    // sample time, the knobs before it at their chosen values and the ones
    // after it at the base's.  A warm-up run first (first-launch costs).
    bc_opts cur = b;
    double best = 0;
    if (bc_status s = timed(cur, &best)) return s;
    if (bc_status s = timed(cur, &best)) return s;
    struct Knob {
        uint32_t bc_opts::*field;
        std::vector<uint32_t> values;
    };
    std::vector<Knob> knobs = {
        {&bc_opts::waves_per_cu, {12, 8, 4}},
        {&bc_opts::lds_words, {0, 256}},
        {&bc_opts::roots_per_wave, {0, 2, 4, 16}},
        {&bc_opts::switch_depth, {3, 2}},
    };
    if (deep) knobs.push_back({&bc_opts::split_rows, {0, 64, 256, 1024}});
    for (const Knob &kn : knobs) {
        const uint32_t start = cur.*kn.field;
        for (uint32_t v : kn.values) {
            if (v == start) continue;
            bc_opts c = cur;
            c.*kn.field = v;
            double t = 0;
            if (bc_status s = timed(c, &t)) return s;
            if (t < best) {
                best = t;
                cur = c;
            }
        }
    }
    // The sample need not stand for the whole batch (it has fewer tasks per
    // wave, and the automatic chunk size follows that count): the choice is
    // kept only if it also beats the base schedule over all the items.
    bool changed = false;
    for (const Knob &kn : knobs) changed = changed || cur.*kn.field != b.*kn.field;
    if (changed && sg.size() < n) {
        std::vector<bc_u128> aout(n);
        std::vector<bc_status> ast(n);
        auto timed_all = [&](const bc_opts &c, double *t) -> bc_status {
            const uint64_t t0 = bcint::steady_ns();
            bc_status s = bc_count_batch(graphs, p, q, n, &c, aout.data(), ast.data(), nullptr);
            if (s != BC_OK) return s;
            *t = (double)(bcint::steady_ns() - t0);
            for (bc_status x : ast)
                if (x != BC_OK && b.timeout_ms) *t += (double)b.timeout_ms * 1e6;
            return BC_OK;
        };
        double t_base = 0, t_cur = 0;
        if (bc_status s = timed_all(b, &t_base)) return s;
        if (bc_status s = timed_all(cur, &t_cur)) return s;
        if (t_cur >= t_base) cur = b;
    }
    *tuned = cur;
    return BC_OK;
}

// ---------------------------------------------------------------------------
// bc_count_noalloc: every scratch buffer of the call is carved from this
// fixed array (one copy per device, held until the process ends).  In host
// code the array's name is only a stand-in for the device symbol: its device
// address is looked up once per device and used everywhere instead.

constexpr uint64_t kNoAllocScratchBytes = BC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {

struct NoAllocDevice {
    std::mutex mu;           // serialises the calls on one device (they share the array)
    void *ptr = nullptr;     // device address of `scratch` on this device
};

NoAllocDevice &noalloc_device(int device)
{
    static NoAllocDevice devs[64];
    return devs[device];
}

}  // namespace

extern "C" bc_status bc_count_noalloc(const bc_graph *g, uint32_t p, uint32_t q, const bc_opts *opts, bc_u128 *out)
{
    g_last_error.clear();
    if (!g || !out) return set_error(BC_E_INVALID_ARG, "bc_count_noalloc: NULL argument");
    if (bc_status s = check_pq(p, q)) return s;
    if (bc_status s = check_opts(opts)) return s;
    if (BC_OPT(opts, alloc, (const bc_allocator *)nullptr))
        return set_error(BC_E_INVALID_ARG, "bc_count_noalloc: bc_opts.alloc must be NULL (nothing is allocated)");
    if (BC_OPT(opts, sets, 0u) != BC_SETS_LOCAL_BITMAP || BC_OPT(opts, bitmap_bits, 0u) != 0)
        return set_error(BC_E_INVALID_ARG,
                         "bc_count_noalloc: the global-set path (bc_opts.sets, bitmap_bits) is not available here");
    if (g->device < 0 || g->device >= 64) return set_error(BC_E_DEVICE, "bc_count_noalloc: device id out of range");
    NoAllocDevice &dev = noalloc_device(g->device);
    std::lock_guard<std::mutex> lock(dev.mu);
    BC_HIP(hipSetDevice(g->device));
    if (!dev.ptr) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                     "bc_count_noalloc: hipGetSymbolAddress(scratch)");
        dev.ptr = ptr;
    }
    std::vector<JobSpec> sp{JobSpec{g, p, q, opts ? opts->anchor : BC_ANCHOR_AUTO, 0, 0, false, opts_deadline(opts)}};
    std::vector<bc_u128> res;
    std::vector<bc_status> ist;
    bool short_of_room = false;
    Exec ex;
    ex.fixed = dev.ptr;
    ex.fixed_cap = kNoAllocScratchBytes;
    ex.fixed_short = &short_of_room;
    bc_status s = run_jobs(sp, opts, res, ist, nullptr, ex);
    if (short_of_room)
        return set_error(BC_E_OOM, "bc_count_noalloc: the count needs more device scratch than the fixed " +
                                       std::to_string(kNoAllocScratchBytes >> 20) + " MiB buffer");
    if (s != BC_OK) return s;
    if (ist[0] != BC_OK) return ist[0];
    *out = res[0];
    return BC_OK;
}

// ---------------------------------------------------------------------------
// BCPar (Algorithm 3, Section VI): roots of one anchor side grouped so that
// each group's closure -- the roots, their oriented 2-hop candidates and the
// neighbourhoods of both -- fits a memory budget; each group is then counted
// on its closure alone, and the groups' counts add up to the whole count.

namespace {

// Oriented 2-hop candidates of every vertex of side a: the w ranked after u
// sharing at least k neighbours with u (the set a root's search draws from),
// by wedge counting on the host; threads take roots in chunks.
void oriented_candidates(const bc_graph *g, int a, uint32_t k, const std::vector<uint32_t> &adj_a,
                         const std::vector<uint32_t> &adj_b, std::vector<uint64_t> &off, std::vector<uint32_t> &ids)
{
    const Side &A = g->side[a], &B = g->side[1 - a];
    const uint64_t n = A.n;
    std::vector<std::vector<uint32_t>> part(n);
    std::atomic<uint64_t> next{0};
    auto work = [&] {
        std::vector<uint32_t> cnt(n, 0), touched;
        for (;;) {
            const uint64_t b = next.fetch_add(64), e = std::min(n, b + 64);
            if (b >= n) break;
            for (uint64_t u = b; u < e; ++u) {
                touched.clear();
                for (uint64_t x = A.h_ptr[u]; x < A.h_ptr[u + 1]; ++x) {
                    const uint32_t v = adj_a[x];
                    for (uint64_t y = B.h_ptr[v]; y < B.h_ptr[v + 1]; ++y) {
                        const uint32_t w = adj_b[y];
                        if (w > u && cnt[w]++ == 0) touched.push_back(w);
                    }
                }
                std::vector<uint32_t> &out = part[u];
                for (uint32_t w : touched) {
                    if (cnt[w] >= k) out.push_back(w);
                    cnt[w] = 0;
                }
                std::sort(out.begin(), out.end());
            }
        }
    };
    std::vector<std::thread> th;
    for (unsigned t = 1; t < host_threads(); ++t) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
    off.assign(n + 1, 0);
    for (uint64_t u = 0; u < n; ++u) off[u + 1] = off[u] + part[u].size();
    ids.resize(off[n]);
    for (uint64_t u = 0; u < n; ++u) std::copy(part[u].begin(), part[u].end(), ids.begin() + off[u]);
}

bc_status read_rows(const bc_graph *g, int side, std::vector<uint32_t> &adj)
{
    adj.resize(g->nnz);
    hipStream_t st = own_stream();
    if (!st) return set_error(BC_E_DEVICE, "could not create a HIP stream");
    if (g->nnz) BC_HIP(hipMemcpyAsync(adj.data(), g->side[side].d_adj, g->nnz * 4, hipMemcpyDeviceToHost, st));
    BC_HIP(hipStreamSynchronize(st));
    return BC_OK;
}

bc_status partition_args(const bc_graph *g, uint32_t p, uint32_t q, int32_t anchor, uint32_t *kA)
{
    if (!g) return set_error(BC_E_INVALID_ARG, "NULL graph");
    if (bc_status s = check_pq(p, q)) return s;
    if (anchor != BC_ANCHOR_U && anchor != BC_ANCHOR_V)
        return set_error(BC_E_INVALID_ARG, "anchor must be BC_ANCHOR_U or BC_ANCHOR_V");
    const uint32_t pA = anchor == BC_ANCHOR_U ? p : q;
    *kA = anchor == BC_ANCHOR_U ? q : p;
    if (pA < 3) return set_error(BC_E_INVALID_ARG, "partitioned counts need a depth of at least 3 on the anchor side");
    return BC_OK;
}

}  // namespace

extern "C" bc_status bc_partition(const bc_graph *g, uint32_t p, uint32_t q, int32_t anchor, uint64_t budget_bytes,
                                  uint32_t *part_of_rank, uint32_t *n_parts)
{
    g_last_error.clear();
    uint32_t kA = 0;
    if (bc_status s = partition_args(g, p, q, anchor, &kA)) return s;
    if (!part_of_rank || !n_parts) return set_error(BC_E_INVALID_ARG, "bc_partition: NULL argument");
    const int a = anchor;
    const Side &A = g->side[a];
    const uint64_t n = A.n;
    std::vector<uint32_t> adj_a, adj_b;
    if (bc_status s = read_rows(g, a, adj_a)) return s;
    if (bc_status s = read_rows(g, 1 - a, adj_b)) return s;
    std::vector<uint64_t> coff;
    std::vector<uint32_t> cids;
    oriented_candidates(g, a, kA, adj_a, adj_b, coff, cids);
    // w(u) = |N(u)| + |N_2(u)| entries of 4 bytes; avg_w(u) over u's candidates
    std::vector<uint64_t> w(n);
    for (uint64_t u = 0; u < n; ++u) w[u] = 4 * ((A.h_ptr[u + 1] - A.h_ptr[u]) + (coff[u + 1] - coff[u]));
    std::vector<double> avg(n, 0.0);
    for (uint64_t u = 0; u < n; ++u) {
        const uint64_t c = coff[u + 1] - coff[u];
        double sum = 0;
        for (uint64_t x = coff[u]; x < coff[u + 1]; ++x) sum += (double)w[cids[x]];
        avg[u] = c ? sum / (double)c : 0.0;
    }
    // reverse candidate lists: roots whose closure holds w (N_in of Algorithm 3)
    std::vector<uint64_t> roff(n + 1, 0);
    for (uint32_t x : cids) roff[x + 1]++;
    for (uint64_t u = 0; u < n; ++u) roff[u + 1] += roff[u];
    std::vector<uint32_t> rids(cids.size());
    {
        std::vector<uint64_t> fill(roff.begin(), roff.end() - 1);
        for (uint64_t u = 0; u < n; ++u)
            for (uint64_t x = coff[u]; x < coff[u + 1]; ++x) rids[fill[cids[x]]++] = (uint32_t)u;
    }
    std::vector<uint32_t> order(n);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return avg[x] > avg[y]; });
    const uint32_t kNone = 0xffffffffu;
    std::vector<uint32_t> part(n, kNone);
    std::vector<uint32_t> in_closure(n, kNone);   // partition whose closure holds the vertex
    std::vector<double> prio(n, 0.0);
    uint32_t np = 0;
    size_t next = 0;
    for (;;) {
        while (next < n && part[order[next]] != kNone) ++next;
        if (next == n) break;
        // a new partition from the unassigned root of highest average weight
        const uint32_t id = np++;
        uint64_t cost = 0;
        std::vector<uint32_t> touched_q;   // roots given a priority in this partition
        std::priority_queue<std::pair<double, uint32_t>> Q;
        auto add_member = [&](uint32_t x) {   // closure member x: its cost, and the roots that share it
            if (in_closure[x] == id) return;
            in_closure[x] = id;
            cost += w[x];
            for (uint64_t y = roff[x]; y < roff[x + 1]; ++y) {
                const uint32_t v = rids[y];
                if (part[v] != kNone) continue;
                if (prio[v] == 0.0) touched_q.push_back(v);
                prio[v] += (double)w[v];
                Q.push({prio[v], v});
            }
        };
        auto closure_cost = [&](uint32_t u) {   // cost that adding root u would add
            uint64_t c = in_closure[u] == id ? 0 : w[u];
            for (uint64_t x = coff[u]; x < coff[u + 1]; ++x)
                if (in_closure[cids[x]] != id) c += w[cids[x]];
            return c;
        };
        uint32_t u = order[next];
        part[u] = id;
        add_member(u);
        for (uint64_t x = coff[u]; x < coff[u + 1]; ++x) add_member(cids[x]);
        for (;;) {
            // the unassigned root sharing the most (weighted) with the closure,
            // else the next root of the global order
            uint32_t v = kNone;
            while (!Q.empty()) {
                const auto top = Q.top();
                Q.pop();
                if (part[top.second] == kNone && top.first == prio[top.second]) {
                    v = top.second;
                    break;
                }
            }
            if (v == kNone) {
                size_t t = next;
                while (t < n && part[order[t]] != kNone) ++t;
                if (t == n) break;
                v = order[t];
            }
            if (cost + closure_cost(v) > budget_bytes) break;   // the partition is full
            part[v] = id;
            add_member(v);
            for (uint64_t x = coff[v]; x < coff[v + 1]; ++x) add_member(cids[x]);
        }
        for (uint32_t v : touched_q) prio[v] = 0.0;
    }
    for (uint64_t u = 0; u < n; ++u) part_of_rank[u] = part[u];
    *n_parts = np;
    return BC_OK;
}

extern "C" bc_status bc_count_partition(const bc_graph *g, uint32_t p, uint32_t q, int32_t anchor,
                                        const uint32_t *part_of_rank, uint32_t part, const bc_opts *opts,
                                        bc_u128 *out, uint64_t *closure_edges)
{
    g_last_error.clear();
    uint32_t kA = 0;
    if (bc_status s = partition_args(g, p, q, anchor, &kA)) return s;
    if (!part_of_rank || !out) return set_error(BC_E_INVALID_ARG, "bc_count_partition: NULL argument");
    if (bc_status s = check_opts(opts)) return s;
    const int a = anchor;
    const Side &A = g->side[a], &B = g->side[1 - a];
    std::vector<uint32_t> adj_a, adj_b;
    if (bc_status s = read_rows(g, a, adj_a)) return s;
    if (bc_status s = read_rows(g, 1 - a, adj_b)) return s;
    std::vector<uint64_t> coff;
    std::vector<uint32_t> cids;
    oriented_candidates(g, a, kA, adj_a, adj_b, coff, cids);
    // closure: the partition's roots and their candidates, in rank order
    std::vector<uint8_t> in(A.n, 0);
    for (uint64_t u = 0; u < A.n; ++u)
        if (part_of_rank[u] == part) {
            in[u] = 1;
            for (uint64_t x = coff[u]; x < coff[u + 1]; ++x) in[cids[x]] = 1;
        }
    std::vector<uint32_t> xs;
    for (uint64_t u = 0; u < A.n; ++u)
        if (in[u]) xs.push_back((uint32_t)u);
    // the other side: every neighbour of the closure
    std::vector<uint32_t> ymap(B.n, 0xffffffffu), ys;
    for (uint32_t x : xs)
        for (uint64_t e = A.h_ptr[x]; e < A.h_ptr[x + 1]; ++e) {
            const uint32_t v = adj_a[e];
            if (ymap[v] == 0xffffffffu) {
                ymap[v] = (uint32_t)ys.size();
                ys.push_back(v);
            }
        }
    // subgraph CSRs: anchor side rows are the closure vertices in rank order
    // (their ids in the subgraph), with their whole neighbourhoods, so degrees
    // and the (degree, id) order among them are those of g
    std::vector<uint64_t> pa(xs.size() + 1, 0), pb(ys.size() + 1, 0);
    std::vector<uint32_t> ia, ib;
    for (size_t i = 0; i < xs.size(); ++i) {
        for (uint64_t e = A.h_ptr[xs[i]]; e < A.h_ptr[xs[i] + 1]; ++e) ia.push_back(ymap[adj_a[e]]);
        pa[i + 1] = ia.size();
    }
    std::vector<uint64_t> degb(ys.size() + 1, 0);
    for (uint32_t y : ia) degb[y + 1]++;
    for (size_t y = 0; y < ys.size(); ++y) degb[y + 1] += degb[y];
    ib.resize(ia.size());
    {
        std::vector<uint64_t> fill(degb.begin(), degb.end() - 1);
        for (size_t i = 0; i < xs.size(); ++i)
            for (uint64_t e = pa[i]; e < pa[i + 1]; ++e) ib[fill[ia[e]]++] = (uint32_t)i;
    }
    pb = degb;
    bc_csr cu{xs.size(), ys.size(), ia.size(), pa.data(), ia.data()};
    bc_csr cv{ys.size(), xs.size(), ib.size(), pb.data(), ib.data()};
    bc_opts bo{};
    if (opts) bo = *opts;
    bo.struct_size = sizeof(bc_opts);
    bo.order_key = BC_ORDER_DEGREE;
    bc_graph *sub = nullptr;
    bc_status s = a == 0 ? bc_build(&cu, &cv, &bo, &sub) : bc_build(&cv, &cu, &bo, &sub);
    if (s != BC_OK) return s;
    // the partition's roots, by their rank in the subgraph (= position in xs)
    std::vector<uint8_t> mask(xs.size(), 0);
    for (size_t i = 0; i < xs.size(); ++i) mask[sub->side[a].rank_of[i]] = part_of_rank[xs[i]] == part;
    JobSpec js{sub, p, q, anchor, 0, 0, false, opts_deadline(opts)};
    js.root_mask = &mask;
    std::vector<JobSpec> sp{js};
    std::vector<bc_u128> res;
    std::vector<bc_status> ist;
    s = run_jobs(sp, &bo, res, ist, nullptr);
    bc_free(sub);
    if (s != BC_OK) return s;
    if (ist[0] != BC_OK) return ist[0];
    *out = res[0];
    if (closure_edges) *closure_edges = ia.size();
    return BC_OK;
}

namespace bcint {

uint64_t steady_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

bc_status count_queries(const Query *qs, size_t n, const bc_opts *opts, bc_u128 *out, bc_status *status)
{
    std::vector<JobSpec> sp;
    std::vector<size_t> idx;
    for (size_t i = 0; i < n; ++i) {
        if (!qs[i].g || qs[i].p < 1 || qs[i].q < 1 || qs[i].p > 32 || qs[i].q > 32) {
            status[i] = BC_E_INVALID_ARG;
            out[i] = bc_u128{0, 0};
            continue;
        }
        idx.push_back(i);
        sp.push_back(JobSpec{qs[i].g, qs[i].p, qs[i].q, BC_ANCHOR_AUTO, 0, 0, false, qs[i].deadline_ns});
    }
    std::vector<bc_u128> res;
    std::vector<bc_status> ist;
    Exec ex;
    ex.short_first = true;
    // ist holds the call's status for every item unless the counts were read back
    bc_status s = run_jobs(sp, opts, res, ist, nullptr, ex);
    for (size_t t = 0; t < idx.size(); ++t) {
        status[idx[t]] = ist[t];
        out[idx[t]] = status[idx[t]] == BC_OK ? res[t] : bc_u128{0, 0};
    }
    return s;
}

// Admission estimate of the device scratch of one count of g at (p, q) with
// waves_per_cu wavefronts per CU: the sizes run_jobs takes, each per-root
// quantity at its bound over the graph (candidates k <= min(n_A - 1, max
// wedges), row words W1 <= ceil(max degree / 64)), the worse of the two
// anchors, and the row pool twice (a rebuild after an overflow).  The
// enumeration slabs are charged at most 8 GiB: a call capped at the estimate
// (bc_opts.scratch_cap_bytes, as the server does) shrinks its grid to fit.
uint64_t estimate_scratch_bytes(const bc_graph *g, uint32_t p, uint32_t q, uint32_t waves_per_cu)
{
    const uint64_t ncu = (uint64_t)cu_count(g->device);
    const uint64_t waves =
        std::max<uint64_t>(bcdev::kWavesPerBlock, ncu * std::min(12u, std::max(1u, waves_per_cu)));
    const Side &s0 = g->side[0], &s1 = g->side[1];
    const uint64_t n_all = std::max(s0.n, s1.n);
    const uint64_t pool = 8 * std::max<uint64_t>(1ull << 22, 32 * g->nnz + (4ull << 20));
    uint64_t fixed = (1ull << 20) + 32ull * (std::max(s0.max_deg, s1.max_deg) + 1)   // jobs, tables, slots
                     + 2 * ncu * n_all * 12                                          // candidate counters
                     + 48 * (s0.n + s1.n)                                            // per-root arrays
                     + 2 * pool;
    uint64_t worst = 0;
    for (int a = 0; a < 2; ++a) {
        const uint32_t pA = a == 0 ? p : q;
        const Side &A = g->side[a];
        if (pA < 3) continue;
        const double k = (double)std::min<uint64_t>(A.n ? A.n - 1 : 0, A.max_wedges);
        const double w1 = (double)((A.max_deg + 63) / 64);
        const double pairs3 = (double)bcdev::kTripleRows * (bcdev::kTripleRows - 1) / 2;
        const double need = 10 * w1 + k / 2 + 1 + (pA >= 5 ? pairs3 * 4 + pairs3 / 2 + 1 : 0.0) +
                            (pA >= 4 ? (double)(pA - 3) * std::max(0.0, k - 1) * w1 : 0.0) + 8;
        const double slab = std::min((double)(8ull << 30), (double)waves * need * 8);
        const uint64_t ring = pA >= 5 ? (64ull << 20) + 64 : 0;
        worst = std::max<uint64_t>(worst, (uint64_t)slab + ring);
    }
    return fixed + worst;
}

int graph_device(const bc_graph *g) { return g->device; }

double query_cost(const bc_graph *g, uint32_t p, uint32_t q)
{
    double best = 0;
    for (int a = 0; a < 2; ++a) {
        const double pA = a == 0 ? p : q, qA = a == 0 ? q : p;
        // wedges through the other side's vertices: what the candidate pass scans
        const double c = (g->side[1 - a].deg_pairs + 1.0) * std::pow(4.0, std::max(0.0, pA - 2)) /
                         std::pow(2.0, std::max(0.0, std::min(qA, 12.0) - 2));
        best = a == 0 ? c : std::min(best, c);
    }
    return best;
}

}  // namespace bcint

extern "C" const char *bc_status_string(bc_status s)
{
    switch (s) {
    case BC_OK: return "BC_OK";
    case BC_E_INVALID_ARG: return "BC_E_INVALID_ARG";
    case BC_E_BAD_CSR: return "BC_E_BAD_CSR";
    case BC_E_INCONSISTENT: return "BC_E_INCONSISTENT";
    case BC_E_OOM: return "BC_E_OOM";
    case BC_E_DEVICE: return "BC_E_DEVICE";
    case BC_E_OVERFLOW: return "BC_E_OVERFLOW";
    case BC_E_REJECTED: return "BC_E_REJECTED";
    case BC_E_TIMEOUT: return "BC_E_TIMEOUT";
    case BC_E_CANCELLED: return "BC_E_CANCELLED";
    case BC_E_PENDING: return "BC_E_PENDING";
    case BC_E_NOT_FOUND: return "BC_E_NOT_FOUND";
    default: return "BC_E_UNKNOWN";
    }
}

extern "C" const char *bc_last_error(void) { return g_last_error.c_str(); }
