// A small pool of host threads for the plan-time builds.
#pragma once

#include <algorithm>
#include <atomic>
#include <functional>
#include <thread>
#include <vector>

namespace kafmm {

// Worker threads that live for one host-side build step (operators, tree).  each(f) runs f(t) on
// every thread t in [0, size()) (t = 0 on the caller) and returns when all
// are done; barrier() synchronises the threads inside such a call.
class Pool {
  public:
    explicit Pool(int nt) : nt_(std::max(1, nt)) {
        for (int t = 1; t < nt_; ++t) th_.emplace_back([this, t] { worker(t); });
    }
    ~Pool() {
        stop_.store(true, std::memory_order_release);
        gen_.fetch_add(1, std::memory_order_acq_rel);
        for (auto &x : th_) x.join();
    }
    int size() const { return nt_; }
    void each(const std::function<void(int)> &f) {
        fn_ = &f;
        done_.store(0, std::memory_order_relaxed);
        gen_.fetch_add(1, std::memory_order_acq_rel);
        f(0);
        while (done_.load(std::memory_order_acquire) != nt_ - 1) std::this_thread::yield();
    }
    void barrier() {
        const int g = bgen_.load(std::memory_order_acquire);
        if (bcount_.fetch_add(1, std::memory_order_acq_rel) == nt_ - 1) {
            bcount_.store(0, std::memory_order_relaxed);
            bgen_.fetch_add(1, std::memory_order_acq_rel);
        } else {
            while (bgen_.load(std::memory_order_acquire) == g) std::this_thread::yield();
        }
    }
    // f(i) for i in [0, n), interleaved over the threads
    template <class F>
    void parallel_for(int n, F &&f) {
        each([&](int t) {
            for (int i = t; i < n; i += nt_) f(i);
        });
    }

  private:
    void worker(int t) {
        int seen = 0;
        for (;;) {
            int g;
            while ((g = gen_.load(std::memory_order_acquire)) == seen) std::this_thread::yield();
            seen = g;
            if (stop_.load(std::memory_order_acquire)) return;
            (*fn_)(t);
            done_.fetch_add(1, std::memory_order_acq_rel);
        }
    }
    int nt_;
    std::vector<std::thread> th_;
    std::atomic<int> gen_{0}, done_{0}, bcount_{0}, bgen_{0};
    std::atomic<bool> stop_{false};
    const std::function<void(int)> *fn_ = nullptr;
};

inline int pool_threads() { return int(std::max(1u, std::min(16u, std::thread::hardware_concurrency()))); }

}  // namespace kafmm
