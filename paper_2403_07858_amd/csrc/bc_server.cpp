// Counting service over device-resident graphs: memory-admitted continuous
// batching (include/bc_server.h).  Worker threads each own a stream and run
// one batch at a time through the batched device path; several workers keep
// several batches in flight, so new queries join the device while earlier
// ones are still running.  This file is the scheduler only: every device
// call goes through a bcint::ServerBackend (bc_server_hip.cpp for the HIP
// one), so the scheduler builds and runs on a host without a GPU too.
#include "bc_server.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bc_internal.h"

namespace {

struct Ticket {
    uint32_t gid, p, q;
    uint64_t deadline_ns;
    uint64_t est_bytes;
    double cost;   // the backend's relative time of the count
    uint64_t t_submit, t_start, t_done;
    bc_status status;
    bc_u128 value;
    bool done;
    uint64_t batch_id;
    uint32_t batch_size;
};

}  // namespace

struct bc_server {
    bc_server_opts opts{};
    const bcint::ServerBackend *be = nullptr;
    std::vector<const bc_graph *> graphs;
    std::mutex mu;
    std::condition_variable cv_work;   // pending queue or budget changed
    std::condition_variable cv_done;   // some ticket finished
    std::deque<uint64_t> pending;
    std::unordered_map<uint64_t, Ticket> tickets;
    uint64_t next_ticket = 1;
    uint64_t next_batch = 1;
    uint64_t inflight_bytes = 0;
    uint32_t inflight_batches = 0;
    bool stop = false;
    uint32_t pollers = 0;              // threads inside bc_server_poll (destroy waits for them)
    uint64_t last_deadline_scan = 0;   // steady ns of the last scan of the pending queue for expired deadlines
    std::vector<std::thread> workers;
    // statistics
    uint64_t submitted = 0, completed = 0, rejected = 0, timed_out = 0, failed = 0, batches = 0, batched_queries = 0;
    uint32_t max_overlap = 0;
    std::vector<double> latencies_ms;
    uint64_t t_created = 0;
};

namespace {

// Wave slots per CU of one worker's batches: the enumeration grid is
// persistent, so at full size one batch would hold every CU until it ends
// and the other workers' batches could not start; each takes its share.
uint32_t worker_waves(const bc_server *s) { return std::max(1u, 12u / std::max(1u, s->opts.max_inflight)); }

void finish(bc_server *s, Ticket &t, bc_status st, bc_u128 v, uint64_t now)
{
    t.status = st;
    t.value = v;
    t.done = true;
    t.t_done = now;
    if (st == BC_OK) {
        s->completed++;
        s->latencies_ms.push_back((double)(now - t.t_submit) / 1e6);
    } else if (st == BC_E_TIMEOUT) {
        s->timed_out++;
    } else if (st == BC_E_REJECTED) {
        s->rejected++;   // refused by the cost model after admission
    } else if (st != BC_E_CANCELLED) {
        s->failed++;
    }
}

void worker_main(bc_server *s)
{
    int device = 0;
    {
        // graphs may still be being added (the vector can reallocate)
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->graphs.empty()) device = s->be->device(s->graphs[0]);
    }
    void *stream = s->be->stream_create(device);
    const uint32_t max_batch = s->opts.max_batch ? s->opts.max_batch : 256;
    for (;;) {
        std::vector<uint64_t> batch;
        uint64_t batch_bytes = 0, batch_id = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                if (s->stop) break;
                // drop queries whose deadline passed while they waited (a scan
                // of the whole queue under the lock: at most once a millisecond)
                const uint64_t now = bcint::steady_ns();
                const bool scan = now - s->last_deadline_scan >= 1000000ull;
                if (scan) s->last_deadline_scan = now;
                for (auto it = s->pending.begin(); scan && it != s->pending.end();) {
                    Ticket &t = s->tickets[*it];
                    if (t.deadline_ns && now >= t.deadline_ns) {
                        finish(s, t, BC_E_TIMEOUT, bc_u128{0, 0}, now);
                        it = s->pending.erase(it);
                        s->cv_done.notify_all();
                    } else {
                        ++it;
                    }
                }
                // admit the cheapest first (the backend's cost), newest first
                // among equals, while the memory budget allows: when queries
                // arrive faster than they can be answered, the cheap ones are
                // those that can still finish before their deadlines, and the
                // oldest have the least time left.  Only the newest 4096
                // pending queries are looked at.
                if (!s->pending.empty()) {
                    const size_t n = s->pending.size(), lo = n > 4096 ? n - 4096 : 0;
                    std::vector<std::pair<double, size_t>> order;
                    order.reserve(n - lo);
                    for (size_t i = lo; i < n; ++i) order.push_back({s->tickets[s->pending[i]].cost, i});
                    std::sort(order.begin(), order.end(), [](const std::pair<double, size_t> &a,
                                                             const std::pair<double, size_t> &b) {
                        return a.first != b.first ? a.first < b.first : a.second > b.second;
                    });
                    std::vector<size_t> taken;
                    for (const auto &c : order) {
                        if (batch.size() >= max_batch) break;
                        const Ticket &t = s->tickets[s->pending[c.second]];
                        if (s->inflight_bytes + batch_bytes + t.est_bytes > s->opts.memory_budget_bytes) continue;
                        batch_bytes += t.est_bytes;
                        batch.push_back(s->pending[c.second]);
                        taken.push_back(c.second);
                    }
                    std::sort(taken.begin(), taken.end(), std::greater<size_t>());
                    for (size_t i : taken) s->pending.erase(s->pending.begin() + (std::ptrdiff_t)i);
                }
                if (!batch.empty()) break;
                s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
            }
            if (s->stop && batch.empty()) break;
            if (s->stop) {
                // shutting down: hand the batch back as cancelled
                const uint64_t now = bcint::steady_ns();
                for (uint64_t id : batch) finish(s, s->tickets[id], BC_E_CANCELLED, bc_u128{0, 0}, now);
                s->cv_done.notify_all();
                break;
            }
            s->inflight_bytes += batch_bytes;
            s->inflight_batches++;
            s->max_overlap = std::max(s->max_overlap, s->inflight_batches);
            batch_id = s->next_batch++;
            s->batches++;
            s->batched_queries += batch.size();
        }
        // run the batch outside the lock
        std::vector<bcint::Query> qs(batch.size());
        const uint64_t t_start = bcint::steady_ns();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (size_t i = 0; i < batch.size(); ++i) {
                Ticket &t = s->tickets[batch[i]];
                t.t_start = t_start;
                qs[i] = bcint::Query{s->graphs[t.gid], t.p, t.q, t.deadline_ns};
                if (s->opts.batch_timeout_ms) {
                    const uint64_t cap = t_start + (uint64_t)s->opts.batch_timeout_ms * 1000000ull;
                    if (qs[i].deadline_ns == 0 || cap < qs[i].deadline_ns) qs[i].deadline_ns = cap;
                }
            }
        }
        std::vector<bc_u128> out(batch.size());
        std::vector<bc_status> st(batch.size(), BC_OK);
        bc_opts o{};
        o.struct_size = sizeof(bc_opts);
        o.stream = stream;
        o.anchor = BC_ANCHOR_AUTO;
        o.waves_per_cu = worker_waves(s);
        // the batch may take what admission charged for it, no more
        o.scratch_cap_bytes = batch_bytes;
        s->be->count(qs.data(), qs.size(), &o, out.data(), st.data());
        {
            std::lock_guard<std::mutex> lk(s->mu);
            const uint64_t now = bcint::steady_ns();
            for (size_t i = 0; i < batch.size(); ++i) {
                Ticket &t = s->tickets[batch[i]];
                t.batch_id = batch_id;
                t.batch_size = (uint32_t)batch.size();
                finish(s, t, st[i], out[i], now);   // st[i] is the call's status unless counts were read
            }
            s->inflight_bytes -= batch_bytes;
            s->inflight_batches--;
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
    if (stream) s->be->stream_destroy(stream);
}

}  // namespace

bc_status bcint::server_create(const bc_server_opts *opts, const ServerBackend *backend, bc_server **out)
{
    if (!out || !backend) return BC_E_INVALID_ARG;
    bc_server *s = new (std::nothrow) bc_server();
    if (!s) return BC_E_OOM;
    s->be = backend;
    if (opts) s->opts = *opts;
    if (!s->opts.max_inflight) s->opts.max_inflight = 2;
    if (s->opts.max_inflight > 16) s->opts.max_inflight = 16;
    if (!s->opts.max_batch) s->opts.max_batch = 256;
    if (!s->opts.max_pending) s->opts.max_pending = 65536;
    if (!s->opts.memory_budget_bytes) s->opts.memory_budget_bytes = backend->default_budget();
    s->t_created = bcint::steady_ns();
    *out = s;
    return BC_OK;
}

extern "C" bc_status bc_server_add_graph(bc_server *s, const bc_graph *g, uint32_t *graph_id)
{
    if (!s || !g || !graph_id) return BC_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->graphs.empty() && s->be->device(g) != s->be->device(s->graphs[0])) return BC_E_INVALID_ARG;
    *graph_id = (uint32_t)s->graphs.size();
    s->graphs.push_back(g);
    // workers start with the first graph (they bind to its device)
    if (s->workers.empty())
        for (uint32_t i = 0; i < s->opts.max_inflight; ++i) s->workers.emplace_back(worker_main, s);
    return BC_OK;
}

extern "C" bc_status bc_server_submit(bc_server *s, uint32_t graph_id, uint32_t p, uint32_t q, uint64_t deadline_ns,
                                      uint64_t *ticket)
{
    if (!s || !ticket) return BC_E_INVALID_ARG;
    if (p < 1 || q < 1 || p > 32 || q > 32) return BC_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    if (graph_id >= s->graphs.size()) return BC_E_NOT_FOUND;
    s->submitted++;
    Ticket t{};
    t.gid = graph_id;
    t.p = p;
    t.q = q;
    t.deadline_ns = deadline_ns;
    t.est_bytes = s->be->estimate(s->graphs[graph_id], p, q, worker_waves(s));
    t.cost = s->be->cost ? s->be->cost(s->graphs[graph_id], p, q) : 0.0;
    t.t_submit = bcint::steady_ns();
    t.done = false;
    if (t.est_bytes > s->opts.memory_budget_bytes || s->pending.size() >= s->opts.max_pending) {
        s->rejected++;
        return BC_E_REJECTED;
    }
    const uint64_t id = s->next_ticket++;
    s->tickets.emplace(id, t);
    s->pending.push_back(id);
    *ticket = id;
    s->cv_work.notify_one();
    return BC_OK;
}

extern "C" bc_status bc_server_poll(bc_server *s, uint64_t ticket, int block, bc_u128 *out, bc_query_stats *st)
{
    if (!s) return BC_E_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return BC_E_NOT_FOUND;
    if (!it->second.done) {
        if (!block) return BC_E_PENDING;
        // counted while waiting, so that bc_server_destroy does not free the
        // server under a poll that is about to wake up
        s->pollers++;
        s->cv_done.wait(lk, [&] {
            auto jt = s->tickets.find(ticket);
            return jt == s->tickets.end() || jt->second.done;
        });
        s->pollers--;
        if (s->pollers == 0) s->cv_done.notify_all();
        it = s->tickets.find(ticket);
        if (it == s->tickets.end()) return BC_E_NOT_FOUND;
    }
    const Ticket t = it->second;
    s->tickets.erase(it);
    if (st) {
        st->queue_ms = t.t_start > t.t_submit ? (double)(t.t_start - t.t_submit) / 1e6 : 0.0;
        st->run_ms = t.t_done > t.t_start && t.t_start ? (double)(t.t_done - t.t_start) / 1e6 : 0.0;
        st->total_ms = (double)(t.t_done - t.t_submit) / 1e6;
        st->batch_id = t.batch_id;
        st->batch_size = t.batch_size;
        st->pad = 0;
    }
    if (t.status == BC_OK && out) *out = t.value;
    return t.status;
}

extern "C" bc_status bc_server_stats(bc_server *s, bc_server_summary *out)
{
    if (!s || !out) return BC_E_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->rejected = s->rejected;
    out->timed_out = s->timed_out;
    out->failed = s->failed;
    out->batches = s->batches;
    out->max_overlap = s->max_overlap;
    out->mean_batch = s->batches ? (double)s->batched_queries / (double)s->batches : 0.0;
    if (!s->latencies_ms.empty()) {
        std::vector<double> v = s->latencies_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double f) {
            size_t i = (size_t)std::min<double>((double)v.size() - 1, f * (double)(v.size() - 1) + 0.5);
            return v[i];
        };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        double sum = 0;
        for (double x : v) sum += x;
        out->mean_ms = sum / (double)v.size();
    }
    const double secs = (double)(bcint::steady_ns() - s->t_created) / 1e9;
    out->qps = secs > 0 ? (double)s->completed / secs : 0.0;
    return BC_OK;
}

extern "C" uint64_t bc_server_now_ns(void) { return bcint::steady_ns(); }

extern "C" void bc_server_destroy(bc_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        const uint64_t now = bcint::steady_ns();
        for (uint64_t id : s->pending) finish(s, s->tickets[id], BC_E_CANCELLED, bc_u128{0, 0}, now);
        s->pending.clear();
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    for (auto &w : s->workers) w.join();
    {
        // every query is final now; wait until the pollers woken by it have left
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_done.wait(lk, [&] { return s->pollers == 0; });
    }
    delete s;
}
