// sched.h -- OpenMP static worksharing arithmetic, shared by the host entry
// points and the device kernels (inlined into both).
//
// Schedules covered: distribute dist_schedule(static[, dc]) over teams, then
// for schedule(static[, c]) over the threads of each team (paper sec. 1: the
// device runtime provides the routines lowered worksharing loops call;
// sec. 3.1: one team = one thread block).  A chunk size of 0 means none was
// given: the iterations are then split into one balanced block per worker,
// the first (m mod p) workers taking one extra iteration.  With a chunk size,
// chunks are dealt round-robin, restarting from worker 0 in every
// distribute block.  Only non-empty chunks are counted.
#pragma once
#include <stdint.h>

#define OMPRT_HD __host__ __device__ __forceinline__

namespace omprt {

struct Range {
    int64_t lo, hi;
};

// Balanced share of worker t when m iterations are split over p workers.
OMPRT_HD Range bal_share(int64_t m, int64_t p, int64_t t) {
    const int64_t q = m / p, r = m - q * p;
    const int64_t lo = t * q + (t < r ? t : r);
    return Range{lo, lo + q + (t < r ? 1 : 0)};
}

// Number of chunks of size c needed to cover m > 0 iterations.
OMPRT_HD int64_t ceil_div_pos(int64_t m, int64_t c) { return (m - 1) / c + 1; }

// Non-empty distribute blocks owned by team k.
OMPRT_HD int64_t team_nblocks(int64_t n, int64_t T, int64_t dc, int64_t k) {
    if (n <= 0) return 0;
    if (dc == 0) {
        const Range r = bal_share(n, T, k);
        return r.hi > r.lo ? 1 : 0;
    }
    const int64_t total = ceil_div_pos(n, dc);
    return k < total ? (total - 1 - k) / T + 1 : 0;
}

// The i-th distribute block of team k (i < team_nblocks).
OMPRT_HD Range team_block(int64_t n, int64_t T, int64_t dc, int64_t k, int64_t i) {
    if (dc == 0) return bal_share(n, T, k);
    const int64_t lo = (k + i * T) * dc;
    const int64_t hi = (n - lo < dc) ? n : lo + dc;
    return Range{lo, hi};
}

// Non-empty chunks thread t executes inside a block of m iterations.
OMPRT_HD int64_t thread_nchunks(int64_t m, int64_t P, int64_t c, int64_t t) {
    if (m <= 0) return 0;
    if (c == 0) {
        const Range r = bal_share(m, P, t);
        return r.hi > r.lo ? 1 : 0;
    }
    const int64_t total = ceil_div_pos(m, c);
    return t < total ? (total - 1 - t) / P + 1 : 0;
}

// The j-th chunk of thread t inside block [a, a+m) (j < thread_nchunks).
OMPRT_HD Range thread_chunk(int64_t a, int64_t m, int64_t P, int64_t c, int64_t t,
                            int64_t j) {
    if (c == 0) {
        const Range r = bal_share(m, P, t);
        return Range{a + r.lo, a + r.hi};
    }
    const int64_t lo = (t + j * P) * c;
    const int64_t hi = (m - lo < c) ? m : lo + c;
    return Range{a + lo, a + hi};
}

// Iterations thread t executes inside a block of m iterations (the sizes of
// its chunks summed in closed form: all but the last have c iterations).
OMPRT_HD int64_t thread_niters(int64_t m, int64_t P, int64_t c, int64_t t) {
    if (m <= 0) return 0;
    if (c == 0) {
        const Range r = bal_share(m, P, t);
        return r.hi - r.lo;
    }
    const int64_t nc = thread_nchunks(m, P, c, t);
    if (nc == 0) return 0;
    const Range last = thread_chunk(0, m, P, c, t, nc - 1);
    return (nc - 1) * c + (last.hi - last.lo);
}

}  // namespace omprt
