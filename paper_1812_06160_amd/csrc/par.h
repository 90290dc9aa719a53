// Fork/join helpers for the host analysis.  Every use splits work whose
// outputs are disjoint (rows of a permuted structure, the two directions of a
// tiling, independent schedules), so the results do not depend on the number
// of threads.  An exception thrown by a worker (std::bad_alloc) is rethrown in
// the calling thread after every worker has joined.
#pragma once

#include <algorithm>
#include <cstdint>
#include <exception>
#include <thread>
#include <vector>

namespace jv {

// Worker threads for one split: the host's hardware threads, at most 16.
inline int host_threads() {
    const unsigned h = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(h, 16u));
}

// Runs a() and b() side by side and returns when both have finished.
template <class A, class B>
void run_pair(A &&a, B &&b) {
    std::exception_ptr eb;
    std::thread t([&] {
        try {
            b();
        } catch (...) {
            eb = std::current_exception();
        }
    });
    std::exception_ptr ea;
    try {
        a();
    } catch (...) {
        ea = std::current_exception();
    }
    t.join();
    if (ea) std::rethrow_exception(ea);
    if (eb) std::rethrow_exception(eb);
}

// Calls f(chunk, lo, hi) over [0, n) cut into at most host_threads()
// contiguous chunks of at least `grain` items; returns the number of chunks.
// Small ranges run inline as one chunk.
template <class F>
int parallel_chunks(int64_t n, int64_t grain, F &&f) {
    const int64_t want = grain > 0 ? n / grain : 1;
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), want));
    if (nt == 1) {
        f(0, (int64_t)0, n);
        return 1;
    }
    std::vector<std::thread> th;
    std::vector<std::exception_ptr> ex(nt);
    th.reserve(nt - 1);
    for (int c = 1; c < nt; ++c)
        th.emplace_back([&, c] {
            try {
                f(c, n * c / nt, n * (c + 1) / nt);
            } catch (...) {
                ex[c] = std::current_exception();
            }
        });
    try {
        f(0, (int64_t)0, n / nt);
    } catch (...) {
        ex[0] = std::current_exception();
    }
    for (auto &t : th) t.join();
    for (auto &e : ex)
        if (e) std::rethrow_exception(e);
    return nt;
}

}  // namespace jv
