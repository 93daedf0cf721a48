// Threads of the host setup (ordering, factorization, layout packing).  Work
// is cut into contiguous chunks, one std::thread each; every result that
// depends on the cut is merged in chunk order, so the output does not depend
// on the number of threads.  Host code only.
#pragma once

#include <algorithm>
#include <cstdint>
#include <exception>
#include <thread>
#include <vector>

namespace hbmc {

// Threads the setup may use: hbmc_set_num_threads, else all hardware threads.
int setup_threads();

// Chunks for n items of work: one per thread, but none smaller than grain.
inline int chunks_for(int64_t n, int64_t grain) {
    const int64_t by_size = std::max<int64_t>(1, n / std::max<int64_t>(1, grain));
    return int(std::min<int64_t>(setup_threads(), by_size));
}

// f(lo, hi, c) for chunk c = 0..chunks-1 of [0, n): lo = n c / chunks,
// hi = n (c + 1) / chunks.  Returns after every chunk is done; rethrows the
// first exception a chunk threw.
template <class F>
void parallel_chunks(int64_t n, int chunks, F &&f) {
    if (chunks <= 1) {
        f(int64_t(0), n, 0);
        return;
    }
    std::vector<std::exception_ptr> err(chunks);
    std::vector<std::thread> th;
    th.reserve(chunks);
    for (int c = 0; c < chunks; ++c)
        th.emplace_back([&, c] {
            try {
                f(n * c / chunks, n * (c + 1) / chunks, c);
            } catch (...) {
                err[c] = std::current_exception();
            }
        });
    for (auto &t : th) t.join();
    for (auto &e : err)
        if (e) std::rethrow_exception(e);
}

// f(i) for every i in [0, n), in chunks of at least grain items.
template <class F>
void parallel_for(int64_t n, int64_t grain, F &&f) {
    parallel_chunks(n, chunks_for(n, grain), [&](int64_t lo, int64_t hi, int) {
        for (int64_t i = lo; i < hi; ++i) f(i);
    });
}

}  // namespace hbmc
