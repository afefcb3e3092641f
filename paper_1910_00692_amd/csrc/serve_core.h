// serve_core.h — the host side of the served form: the request queue, admission by scratch
// budget and the worker loop, independent of the device.  The library instantiates the worker
// loop with the query (query.hip); a CPU test instantiates it with a stand-in and runs it under
// a thread sanitizer.
//
// Admission.  A request's scratch comes in parts that grow independently (the buffers with k,
// the subset structures with the subset size), and worker (slot) s keeps, part by part, the
// largest it has allocated: held[s].  The budget bounds the sum over the slots of what they
// keep: the request at the front of the FIFO is admitted on an idle slot s when
// total - sum(held[s]) + sum(max(held[s], need)) <= budget.  When the front request fits on no
// slot, not even once a running one finishes, an idle slot that keeps scratch gives it back, so
// that a request the budget admits alone is never left waiting for ever.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/topktri.h"

struct ServeCore {
    static constexpr int PARTS = 2;
    struct Parts {
        uint64_t b[PARTS] = {0, 0};
        uint64_t sum() const {
            uint64_t s = 0;
            for (uint64_t x : b) s += x;
            return s;
        }
        Parts grown(const Parts &o) const {
            Parts r;
            for (int i = 0; i < PARTS; i++) r.b[i] = std::max(b[i], o.b[i]);
            return r;
        }
    };
    struct Req {
        uint64_t ticket = 0;
        uint32_t k = 0;
        double p = 0.0;
        std::vector<uint32_t> subset;
        uint64_t need[PARTS] = {0, 0};
        std::chrono::steady_clock::time_point t_submit;
        Parts parts() const {
            Parts r;
            for (int i = 0; i < PARTS; i++) r.b[i] = need[i];
            return r;
        }
    };
    struct Res {
        bool done = false;
        int rc = TT_OK;
        std::string err;
        std::vector<tt_triangle> tri;
        uint32_t n_out = 0;
        tt_query_stats st{};
    };
    uint64_t budget = 0, held_total = 0, peak = 0, admitted = 0, completed = 0;
    std::vector<Parts> held;      // charged scratch each slot keeps, by part
    std::vector<uint64_t> actual; // device bytes each slot holds (measured by the slot after a request)
    uint32_t max_queue = 0, max_running = 0, running = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::deque<Req> queue;
    std::unordered_map<uint64_t, Res> results;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;

    explicit ServeCore(size_t slots = 0, uint64_t b = 0) : budget(b), held(slots), actual(slots, 0) {}

    // (callers hold mu and the queue is not empty)
    bool fits_on(size_t s) const {
        return held_total - held[s].sum() + held[s].grown(queue.front().parts()).sum() <= budget;
    }
    bool stuck() const {
        for (size_t s = 0; s < held.size(); s++)
            if (fits_on(s)) return false;
        return true;
    }

    // Worker loop of slot s until stop and an empty queue.  run(req, res) executes a request and
    // returns the device bytes the slot holds afterwards; release() gives the slot's scratch back.
    template <class Run, class Release> void worker(size_t s, Run run, Release release) {
        for (;;) {
            Req r;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_work.wait(lk, [&] {
                    return (stop && queue.empty()) ||
                           (!queue.empty() && (fits_on(s) || (held[s].sum() > 0 && stuck())));
                });
                if (queue.empty()) return;
                if (!fits_on(s)) {
                    held_total -= held[s].sum();
                    held[s] = Parts{};
                    lk.unlock();
                    release(); // this slot is idle: nothing queued uses its scratch
                    {
                        std::lock_guard<std::mutex> lk2(mu);
                        actual[s] = 0;
                    }
                    cv_work.notify_all();
                    continue;
                }
                r = std::move(queue.front());
                queue.pop_front();
                const Parts grown = held[s].grown(r.parts());
                held_total += grown.sum() - held[s].sum();
                held[s] = grown;
                peak = std::max(peak, held_total);
                admitted++;
                running++;
                max_running = std::max(max_running, running);
            }
            Res res;
            res.tri.resize(std::max<uint32_t>(r.k, 1));
            const uint64_t bytes = run(r, res);
            res.st.total_ms =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - r.t_submit).count();
            res.done = true;
            {
                std::lock_guard<std::mutex> lk(mu);
                actual[s] = bytes;
                running--;
                completed++;
                results[r.ticket] = std::move(res);
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
    }

    // Queues r (its need already computed); TT_E_BUDGET if it can never fit.
    int submit(Req &&r, uint64_t *ticket) {
        if (r.parts().sum() > budget) return TT_E_BUDGET;
        r.t_submit = std::chrono::steady_clock::now();
        {
            std::lock_guard<std::mutex> lk(mu);
            if (stop) return TT_E_ARG;
            r.ticket = next_ticket++;
            *ticket = r.ticket;
            results[r.ticket] = Res{}; // outstanding until server_wait hands it over
            queue.push_back(std::move(r));
            max_queue = std::max<uint32_t>(max_queue, (uint32_t)queue.size());
        }
        cv_work.notify_all();
        return TT_OK;
    }

    // Blocks until the request has finished and hands its result over (the ticket is released).
    // TT_E_ARG for a ticket that is not outstanding: never issued, or already handed over (also
    // to another thread that waited on the same ticket at the same time).
    int wait(uint64_t ticket, Res &out) {
        std::unique_lock<std::mutex> lk(mu);
        cv_done.wait(lk, [&] {
            auto it = results.find(ticket);
            return it == results.end() || it->second.done;
        });
        auto it = results.find(ticket);
        if (it == results.end()) return TT_E_ARG;
        out = std::move(it->second);
        results.erase(it);
        return TT_OK;
    }

    // TT_E_ARG for a ticket that is not outstanding (as wait).
    int poll(uint64_t ticket, int *done) {
        std::lock_guard<std::mutex> lk(mu);
        auto it = results.find(ticket);
        *done = 0;
        if (it == results.end()) return TT_E_ARG;
        *done = it->second.done;
        return TT_OK;
    }

    uint64_t held_bytes() {
        std::lock_guard<std::mutex> lk(mu);
        uint64_t b = 0;
        for (uint64_t x : actual) b += x;
        return b;
    }

    void shutdown() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv_work.notify_all();
    }
};
