// Host-only stress run of the serving scheduler (bc_server.cpp) behind a
// stand-in device backend: many threads submit and poll (blocking and not)
// while workers run batches, deadlines expire, and finally the server is
// destroyed with pollers still blocked on queries in flight.  Every BC_OK
// result must equal the stand-in's count for its (graph, p, q).  Built with
// -fsanitize=thread or -fsanitize=address,undefined by the test.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "bc_internal.h"

namespace bcint {
uint64_t steady_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}
}  // namespace bcint

namespace {

std::atomic<uint64_t> g_batches{0}, g_streams{0};

uint64_t expected(uintptr_t gid, uint32_t p, uint32_t q) { return gid * 1000003ull + p * 101ull + q; }

bc_status fake_count(const bcint::Query *qs, size_t n, const bc_opts *, bc_u128 *out, bc_status *st)
{
    g_batches++;
    // (8,8) queries (only submitted right before the destroy) take long, so
    // that pollers are still blocked on them when the destroy starts
    bool slow = false;
    for (size_t i = 0; i < n; ++i) slow = slow || (qs[i].p == 8 && qs[i].q == 8);
    std::this_thread::sleep_for(std::chrono::microseconds(slow ? 30000 : 50 + 37 * (n % 7)));
    for (size_t i = 0; i < n; ++i) {
        const uint64_t now = bcint::steady_ns();
        if (qs[i].deadline_ns && now > qs[i].deadline_ns) {
            st[i] = BC_E_TIMEOUT;
            out[i] = bc_u128{0, 0};
        } else {
            st[i] = BC_OK;
            out[i] = bc_u128{expected((uintptr_t)qs[i].g, qs[i].p, qs[i].q), 0};
        }
    }
    return BC_OK;
}

uint64_t fake_estimate(const bc_graph *, uint32_t p, uint32_t q, uint32_t) { return 1000ull * (p + q); }
int fake_device(const bc_graph *) { return 0; }
void *fake_stream_create(int)
{
    g_streams++;
    return new int(7);
}
void fake_stream_destroy(void *s)
{
    g_streams--;
    delete (int *)s;
}
uint64_t fake_budget() { return 1ull << 20; }
double fake_cost(const bc_graph *, uint32_t p, uint32_t q) { return (double)(p * q); }

const bcint::ServerBackend kFake = {fake_count,         fake_estimate,       fake_device,
                                    fake_stream_create, fake_stream_destroy, fake_budget,
                                    fake_cost};

}  // namespace

int main(int argc, char **argv)
{
    const int rounds = argc > 1 ? atoi(argv[1]) : 3;
    const int per_thread = argc > 2 ? atoi(argv[2]) : 1500;
    int errors = 0;
    for (int round = 0; round < rounds; ++round) {
        bc_server_opts o{};
        o.struct_size = sizeof(o);
        o.max_inflight = 3;
        o.max_batch = 8;
        o.max_pending = 512;
        o.memory_budget_bytes = 200000;   // admits a few dozen queries at a time
        bc_server *s = nullptr;
        if (bcint::server_create(&o, &kFake, &s) != BC_OK) return 2;
        const int n_graphs = 6;
        for (int g = 0; g < n_graphs; ++g) {
            uint32_t id = 0;
            if (bc_server_add_graph(s, (const bc_graph *)(uintptr_t)(g + 1), &id) != BC_OK || id != (uint32_t)g)
                return 3;
        }
        std::mutex mu;
        std::vector<std::pair<uint64_t, uint64_t>> tickets;   // ticket, expected value
        std::atomic<int> bad{0}, ok{0}, timeouts{0}, rejected{0};
        std::atomic<bool> submitting{true};
        std::vector<std::thread> th;
        for (int t = 0; t < 6; ++t)
            th.emplace_back([&, t] {
                std::mt19937 rng(round * 100 + t);
                for (int k = 0; k < per_thread; ++k) {
                    const uint32_t gid = rng() % n_graphs, p = 1 + rng() % 7, q = 1 + rng() % 7;
                    uint64_t dl = 0;
                    const uint32_t kind = rng() % 10;
                    if (kind == 0) dl = bc_server_now_ns() - 1;                   // already late
                    else if (kind == 1) dl = bc_server_now_ns() + 200000;         // 0.2 ms
                    uint64_t tk = 0;
                    const bc_status st = bc_server_submit(s, gid, p, q, dl, &tk);
                    if (st == BC_E_REJECTED) {
                        rejected++;
                        continue;
                    }
                    if (st != BC_OK) {
                        bad++;
                        continue;
                    }
                    std::lock_guard<std::mutex> g(mu);
                    tickets.emplace_back(tk, expected((uintptr_t)(gid + 1), p, q));
                }
            });
        for (int t = 0; t < 6; ++t)
            th.emplace_back([&, t] {
                std::mt19937 rng(round * 1000 + t);
                for (;;) {
                    std::pair<uint64_t, uint64_t> item{0, 0};
                    {
                        std::lock_guard<std::mutex> g(mu);
                        if (!tickets.empty()) {
                            const size_t i = rng() % tickets.size();
                            item = tickets[i];
                            tickets[i] = tickets.back();
                            tickets.pop_back();
                        }
                    }
                    if (!item.first) {
                        if (!submitting) break;
                        std::this_thread::yield();
                        continue;
                    }
                    bc_u128 v{0, 0};
                    bc_query_stats qs{};
                    bc_status st = bc_server_poll(s, item.first, (int)(rng() % 2), &v, &qs);
                    if (st == BC_E_PENDING) {
                        std::lock_guard<std::mutex> g(mu);
                        tickets.push_back(item);
                        continue;
                    }
                    if (st == BC_OK) {
                        if (v.lo != item.second || v.hi != 0) bad++;
                        else ok++;
                    } else if (st == BC_E_TIMEOUT) {
                        timeouts++;
                    } else {
                        bad++;
                    }
                    if (rng() % 50 == 0) {
                        bc_server_summary sum{};
                        if (bc_server_stats(s, &sum) != BC_OK) bad++;
                    }
                }
            });
        for (int t = 0; t < 6; ++t) th[t].join();
        submitting = false;
        for (size_t t = 6; t < th.size(); ++t) th[t].join();
        // queries in flight at shutdown, with pollers blocked on them
        std::vector<uint64_t> last;
        for (int k = 0; k < 64; ++k) {
            uint64_t tk = 0;
            if (bc_server_submit(s, k % n_graphs, 8, 8, 0, &tk) == BC_OK) last.push_back(tk);
        }
        std::atomic<int> finished{0}, started{0};
        std::vector<std::thread> blocked;
        for (uint64_t tk : last)
            blocked.emplace_back([&, tk] {
                bc_u128 v{0, 0};
                started++;
                const bc_status st = bc_server_poll(s, tk, 1, &v, nullptr);
                if (st != BC_OK && st != BC_E_CANCELLED && st != BC_E_NOT_FOUND) bad++;
                finished++;
            });
        // (the pollers must be inside bc_server_poll before the destroy: a poll
        // that starts after it would use a freed server, the caller's error)
        while (started.load() < (int)last.size()) std::this_thread::yield();
        std::this_thread::sleep_for(std::chrono::milliseconds(5));
        bc_server_destroy(s);
        for (auto &b : blocked) b.join();
        if (g_streams.load() != 0) bad++;
        printf("round %d: ok %d timeouts %d rejected %d bad %d batches %llu blocked-at-destroy %zu\n", round,
               ok.load(), timeouts.load(), rejected.load(), bad.load(), (unsigned long long)g_batches.load(),
               last.size());
        errors += bad.load();
        if (ok.load() == 0) errors++;
    }
    return errors ? 1 : 0;
}
