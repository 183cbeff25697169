// Host thread pool of the planner and the batched enqueue (plain C++, no HIP).
#pragma once

#include <stddef.h>

#include <algorithm>
#include <atomic>
#include <exception>
#include <mutex>
#include <thread>
#include <vector>

namespace qsim {

// f(0) .. f(n-1) on up to `threads` threads (the calling one included), each
// taking the next index as it becomes free.  A thread that cannot be started
// leaves its share to the others.  The first exception thrown by f stops the
// handing out of indices and is rethrown in the caller once every thread has
// joined, so no exception ends a worker thread (which would end the process).
template <typename F>
void parallel_for(size_t n, int threads, F &&f) {
    const size_t nt = std::min<size_t>(n, (size_t)std::max(threads, 1));
    std::atomic<size_t> next{0};
    std::exception_ptr err;
    std::mutex err_mu;
    auto run = [&]() noexcept {
        for (size_t k; (k = next.fetch_add(1)) < n;) {
            try {
                f(k);
            } catch (...) {
                std::lock_guard<std::mutex> lk(err_mu);
                if (!err) err = std::current_exception();
                next.store(n);
            }
        }
    };
    std::vector<std::thread> pool;
    for (size_t t = 1; t < nt; ++t) {
        try {
            pool.emplace_back(run);
        } catch (...) {
            break;   // (emplace_back leaves the pool as it was)
        }
    }
    run();
    for (auto &th : pool) th.join();
    if (err) std::rethrow_exception(err);
}

}  // namespace qsim
