// launch.h -- host-side launchers of the gfx950 kernels (internal to the
// library; the public surface is include/omprt.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace omprt {

// Bytes of one cross-team partial slot: 4 tagged 64-bit words (payloads up to
// 16 bytes, 32 bits per word).
constexpr int kSlotBytes = 32;

// Device words a launch of the plain kernels uses for the cross-team step.
struct CrossTeamArgs {
    void* slots;          // teams * kSlotBytes, zero-filled at allocation
    uint32_t* counter;    // election counter, 0 between launches
    uint32_t* epoch;      // launch epoch
    uint32_t* status;     // poll-timeout flag
};

// True if (dtype, op, vec_bytes, unroll) has a compiled reduce kernel.
bool reduce_variant_exists(int dtype, int op, int vec_bytes, int unroll);

// Plain reduction (team-block streaming + wave/LDS tree + last-team combine).
hipError_t launch_reduce(int dtype, int op, int vec_bytes, int unroll, const void* in,
                         int64_t n, void* x, int teams, int threads, const CrossTeamArgs& ct,
                         hipStream_t stream);

// Iteration map of a static schedule (threads = logical P, 1..1024).
hipError_t launch_static_map(int64_t n, int teams, int threads, int64_t dist_chunk,
                             int64_t chunk, int32_t* owner, uint32_t* count,
                             hipStream_t stream);

// The plain reduction (sum, max, min) with every thread reducing exactly its
// schedule(static) run of the team's block (exact.hip).
hipError_t launch_reduce_exact(int dtype, int op, const void* in, int64_t n, void* x, int teams,
                               int threads, const CrossTeamArgs& ct, hipStream_t stream);

// y <- fmaf(a, x, y) with the exact static mapping, fused compensated sum.
hipError_t launch_axpy_sum(float a, const float* x, float* y, float* sum, int64_t n,
                           int teams, int threads, int64_t dist_chunk, int64_t chunk,
                           const CrossTeamArgs& ct, hipStream_t stream);

// Empty target region over n iterations with reduction(+: iters) of one
// count per iteration (iters may be NULL); inconsistencies set status bit 16.
hipError_t launch_empty_region(int64_t n, int teams, int threads, int64_t dist_chunk,
                               int64_t chunk, int64_t* iters, const CrossTeamArgs& ct,
                               hipStream_t stream);

}  // namespace omprt
