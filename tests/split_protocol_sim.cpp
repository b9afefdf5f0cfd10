// CPU model of the enumeration kernel's task queue and subtask ring (the
// runtime split): threads stand in for wavefronts and follow the same
// protocol with the same memory orders.  Checks that every queued subtask is
// run exactly once, that every task is popped exactly once, and that every
// thread leaves the drain loop.  Built with -fsanitize=thread by the test.
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <thread>
#include <vector>

struct Entry {
    uint32_t r, i, j;
    std::atomic<uint32_t> ready{0};
};

constexpr uint64_t kProducer = 1ull << 40, kPopMask = kProducer - 1;
constexpr uint32_t kNoJ = 0xffffffffu;

int main(int argc, char **argv)
{
    const int threads = argc > 1 ? atoi(argv[1]) : 16;
    const uint64_t n_tasks = argc > 2 ? strtoull(argv[2], nullptr, 10) : 20000;
    const uint32_t cap = argc > 3 ? (uint32_t)atoi(argv[3]) : 5000;   // small: some pushes must fail
    const uint32_t chunk = 4;
    std::atomic<uint64_t> queue{0}, head{0}, tail{0};
    std::vector<Entry> ring(cap);
    std::vector<std::atomic<uint32_t>> task_runs(n_tasks), sub_runs(n_tasks * 8);
    std::atomic<uint64_t> inline_subs{0}, pushed{0};

    auto wave = [&](int id) {
        std::mt19937 rng(id * 7919 + 1);
        for (;;) {
            const uint64_t t0 = queue.fetch_add(chunk + kProducer) & kPopMask;
            if (t0 >= n_tasks) {
                queue.fetch_add(0ull - kProducer, std::memory_order_release);
                break;
            }
            for (uint64_t t = t0; t < std::min<uint64_t>(t0 + chunk, n_tasks); ++t) {
                task_runs[t].fetch_add(1);
                const uint32_t m = (t % 5 == 0) ? 1 + (uint32_t)(t % 7) : 0;   // subtasks of a heavy task
                if (!m) continue;
                // reserve m entries, CAS as on the device
                uint64_t cur = tail.load(std::memory_order_relaxed), at = ~0ull;
                while (cur + m <= cap) {
                    if (tail.compare_exchange_strong(cur, cur + m, std::memory_order_acq_rel,
                                                     std::memory_order_relaxed)) {
                        at = cur;
                        break;
                    }
                }
                if (at == ~0ull) {   // ring full: the task runs them itself
                    for (uint32_t x = 0; x < m; ++x) sub_runs[t * 8 + x].fetch_add(1);
                    inline_subs += m;
                    continue;
                }
                if (rng() % 3 == 0) std::this_thread::yield();   // a slow publisher
                for (uint32_t x = 0; x < m; ++x) {
                    Entry &e = ring[at + x];
                    e.r = (uint32_t)t;
                    e.i = x;
                    e.j = 1;
                    e.ready.store(1, std::memory_order_release);
                }
                pushed += m;
            }
            queue.fetch_add(0ull - kProducer, std::memory_order_release);
        }
        for (;;) {
            const uint64_t h = head.fetch_add(1);
            int state = 0;
            uint64_t spins = 0;
            while (state == 0) {
                if (h >= cap) {
                    state = 2;
                } else {
                    const uint64_t tl = tail.load(std::memory_order_acquire);
                    if (h < tl) {
                        if (ring[h].ready.load(std::memory_order_acquire)) state = 1;
                    } else {
                        const uint64_t v = queue.load(std::memory_order_acquire);
                        if ((v >> 40) == 0 && h >= tail.load(std::memory_order_acquire)) state = 2;
                    }
                }
                if (state == 0) {
                    std::this_thread::yield();
                    if (++spins > (1ull << 32)) {
                        fprintf(stderr, "thread %d never left the drain\n", id);
                        abort();
                    }
                }
            }
            if (state == 2) break;
            const Entry &e = ring[h];
            if (e.j == kNoJ) continue;
            sub_runs[(uint64_t)e.r * 8 + e.i].fetch_add(1);
        }
    };
    std::vector<std::thread> th;
    for (int i = 0; i < threads; ++i) th.emplace_back(wave, i);
    for (auto &x : th) x.join();

    uint64_t bad = 0, subs = 0;
    for (uint64_t t = 0; t < n_tasks; ++t) {
        bad += task_runs[t].load() != 1;
        const uint32_t m = (t % 5 == 0) ? 1 + (uint32_t)(t % 7) : 0;
        for (uint32_t x = 0; x < 8; ++x) {
            const uint32_t runs = sub_runs[t * 8 + x].load();
            bad += runs != (x < m ? 1u : 0u);
            subs += runs;
        }
    }
    printf("tasks %llu subtasks %llu (ring %llu, inline %llu) errors %llu\n", (unsigned long long)n_tasks,
           (unsigned long long)subs, (unsigned long long)pushed.load(), (unsigned long long)inline_subs.load(),
           (unsigned long long)bad);
    return bad ? 1 : 0;
}
