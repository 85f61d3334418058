// Host test of the stream workspace lease (csrc/pa_workspace.h) on a
// simulated stream: no GPU.
//
// The simulated stream is a FIFO of work items run by a device thread in
// enqueue order.  Each call leases the workspace, enqueues an item that
// uses the buffer's address, and releases the lease; an item finding its
// buffer already freed counts as a use after free.  Several host threads
// share the one stream with growing sizes, so growth (wait for the stream,
// free, reallocate) races with the other threads' calls.
//
// Usage: workspace_lease_test [early]
//   early: release the lease right after reading the address, before the
//   work is enqueued (the order the lease exists to prevent); the test then
//   expects to observe uses after free.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "pa_workspace.h"

namespace {

struct SimStream {
    std::mutex mu;
    std::condition_variable cv, idle_cv;
    std::deque<std::function<void()>> q;
    bool running = false, stop = false;
    std::thread dev;

    SimStream() {
        dev = std::thread([this] {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                cv.wait(lk, [this] { return stop || !q.empty(); });
                if (q.empty() && stop) return;
                auto f = std::move(q.front());
                q.pop_front();
                running = true;
                lk.unlock();
                f();
                lk.lock();
                running = false;
                idle_cv.notify_all();
            }
        });
    }
    ~SimStream() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv.notify_all();
        dev.join();
    }
    void enqueue(std::function<void()> f) {
        std::lock_guard<std::mutex> lk(mu);
        q.push_back(std::move(f));
        cv.notify_all();
    }
    void synchronize() {
        std::unique_lock<std::mutex> lk(mu);
        idle_cv.wait(lk, [this] { return q.empty() && !running; });
    }
};

struct Heap {
    std::mutex mu;
    std::set<void *> live;
    std::vector<char *> blocks;  // never returned to the system, so a stale
                                 // address stays a plain number
    ~Heap() {
        for (char *b : blocks) delete[] b;
    }
};

struct SimDev {
    SimStream *s;
    Heap *h;
    const char *what = "";
    bool sync() {
        s->synchronize();
        return true;
    }
    bool release(void *p) {
        std::lock_guard<std::mutex> lk(h->mu);
        if (!h->live.erase(p)) {
            what = "double free";
            return false;
        }
        return true;
    }
    bool allocate(void **p, size_t) {
        std::lock_guard<std::mutex> lk(h->mu);
        char *b = new char[1];
        h->blocks.push_back(b);
        h->live.insert(b);
        *p = b;
        return true;
    }
};

}  // namespace

int main(int argc, char **argv) {
    const bool early = argc > 1 && std::strcmp(argv[1], "early") == 0;
    SimStream stream;
    Heap heap;
    pa::StreamWorkspace<SimDev> ws;
    std::atomic<long> uses{0}, after_free{0}, failures{0};
    const int kThreads = 6, kCalls = 3000;
    std::vector<std::thread> th;
    for (int t = 0; t < kThreads; ++t) {
        th.emplace_back([&, t] {
            std::mt19937 rng(1234 + t);
            SimDev d{&stream, &heap};
            for (int i = 0; i < kCalls; ++i) {
                // sizes grow over the run, so growth keeps happening
                const size_t need = ((size_t)1 << 20) + (size_t)i * 4096 * kThreads + (rng() % 4096) * 512;
                void *p = nullptr;
                std::unique_lock<std::mutex> hold;
                if (!ws.acquire(d, need, &p, &hold)) {
                    ++failures;
                    continue;
                }
                if (early) {
                    hold.unlock();
                    std::this_thread::yield();
                }
                stream.enqueue([&, p] {
                    std::lock_guard<std::mutex> lk(heap.mu);
                    ++uses;
                    if (!heap.live.count(p)) ++after_free;
                });
                // the caller's lease ends when `hold` goes out of scope
            }
        });
    }
    for (auto &x : th) x.join();
    stream.synchronize();
    std::printf("{\"mode\": \"%s\", \"uses\": %ld, \"after_free\": %ld, \"failures\": %ld}\n", early ? "early" : "lease",
                uses.load(), after_free.load(), failures.load());
    if (failures) return 2;
    if (early) return after_free > 0 ? 0 : 3;  // the unsafe order must be detectable
    return after_free == 0 ? 0 : 1;
}
