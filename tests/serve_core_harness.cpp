// CPU harness of the served form's host side (csrc/serve_core.h): worker threads run a
// stand-in for the query (a short sleep), a submitter queues requests of random scratch needs
// (some close to the budget, so idle slots must give their scratch back), and a waiter collects
// every result.  Checks: every request completes with its own result, the charged scratch never
// exceeds the budget, tickets no longer outstanding are refused, and the loop ends.  Built with
// a thread sanitizer by test_serve_core.py.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <random>
#include <thread>
#include <vector>

#include "../paper_1910_00692_amd/csrc/serve_core.h"

int main(int argc, char **argv) {
    const int slots = argc > 1 ? atoi(argv[1]) : 6;
    const int N = argc > 2 ? atoi(argv[2]) : 4000;
    const uint64_t budget = 1000;
    ServeCore C(slots, budget);
    std::atomic<uint64_t> over{0}, bad{0}, releases{0};
    std::vector<std::thread> workers;
    for (int s = 0; s < slots; s++)
        workers.emplace_back([&, s] {
            std::mt19937 rng(1234 + s);
            C.worker(
                s,
                [&](const ServeCore::Req &r, ServeCore::Res &res) -> uint64_t {
                    {
                        std::lock_guard<std::mutex> lk(C.mu);
                        if (C.held_total > C.budget) over++;
                        for (int x = 0; x < ServeCore::PARTS; x++)
                            if (C.held[s].b[x] < r.need[x]) bad++;
                    }
                    std::this_thread::sleep_for(std::chrono::microseconds(rng() % 300));
                    res.rc = TT_OK;
                    res.n_out = 1;
                    res.tri[0].i = (uint32_t)r.ticket;
                    res.tri[0].j = r.k;
                    return r.need[0] + r.need[1];
                },
                [&] { releases++; });
        });
    std::vector<uint64_t> tickets(N, 0);
    std::vector<uint64_t> needs(N), subs(N);
    std::mt19937_64 rng(99);
    for (int i = 0; i < N; i++) {
        const uint64_t x = rng() % 100;
        needs[i] = x < 10 ? 700 + rng() % 150 : x < 40 ? 200 + rng() % 300 : 10 + rng() % 90;
        subs[i] = rng() % 5 == 0 ? 50 + rng() % 100 : 0; // the second part: subset structures
    }
    std::atomic<int> submitted{0};
    std::thread submitter([&] {
        for (int i = 0; i < N; i++) {
            ServeCore::Req r;
            r.k = (uint32_t)(i % 1000 + 1);
            r.need[0] = needs[i];
            r.need[1] = subs[i];
            if (C.submit(std::move(r), &tickets[i]) != TT_OK) bad++;
            submitted.store(i + 1, std::memory_order_release);
            if (i % 64 == 0) std::this_thread::sleep_for(std::chrono::microseconds(rng() % 500));
        }
        ServeCore::Req big;
        big.need[0] = budget;
        big.need[1] = 1;
        uint64_t t = 0;
        if (C.submit(std::move(big), &t) != TT_E_BUDGET) bad++;
    });
    int done = 0;
    for (int i = 0; i < N; i++) {
        while (submitted.load(std::memory_order_acquire) <= i) std::this_thread::yield();
        ServeCore::Res res;
        if (C.wait(tickets[i], res) != TT_OK || res.n_out != 1 || res.tri[0].i != (uint32_t)tickets[i] ||
            res.tri[0].j != (uint32_t)(i % 1000 + 1))
            bad++;
        done++;
    }
    submitter.join();
    // a ticket already handed over, or never issued, is refused (not waited for)
    {
        ServeCore::Res res;
        int d = 1;
        if (N > 0 && (C.wait(tickets[0], res) != TT_E_ARG || C.poll(tickets[0], &d) != TT_E_ARG || d != 0)) bad++;
        if (C.wait(0, res) != TT_E_ARG || C.wait(1ull << 40, res) != TT_E_ARG) bad++;
    }
    C.shutdown();
    for (auto &t : workers) t.join();
    printf("requests %d completed %llu over_budget %llu bad %llu releases %llu peak %llu max_running %u\n", done,
           (unsigned long long)C.completed, (unsigned long long)over.load(), (unsigned long long)bad.load(),
           (unsigned long long)releases.load(), (unsigned long long)C.peak, C.max_running);
    return (done == N && C.completed == (uint64_t)N && over == 0 && bad == 0 && C.peak <= budget) ? 0 : 1;
}
