// shared_alloc.h -- team-shared dynamic allocation: memory that every
// thread of a team sees, taken at run time (the device runtime's
// alloc_shared entry, paper sec. 2.1's listing).  Requests are served from
// a stack in the team's dynamic LDS and, once that is full, from the team's
// slice of a global pool, so an allocation never fails for lack of LDS
// (only for lack of pool).  Frees are last-in first-out.
//
// Every thread of the team makes the same calls in the same order (they
// are team-collective, with a barrier): thread 0 moves the stack tops and
// the result is read back from LDS by all.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace omprt {

struct TeamStack {
    char* lds;           // the team's dynamic LDS arena
    uint32_t lds_cap;    // its bytes
    uint32_t lds_top;
    char* glob;          // the team's slice of the global pool
    uint64_t glob_cap;
    uint64_t glob_top;
    void* last;          // result of the last allocation, for the other threads
};

constexpr uint32_t kSharedAlign = 16;

__device__ __forceinline__ void team_stack_init(TeamStack* st, char* lds, uint32_t lds_cap,
                                                char* glob, uint64_t glob_cap) {
    if (threadIdx.x == 0) {
        st->lds = lds;
        st->lds_cap = lds_cap;
        st->lds_top = 0;
        st->glob = glob;
        st->glob_cap = glob_cap;
        st->glob_top = 0;
        st->last = nullptr;
    }
    __syncthreads();
}

// Team-collective.  nullptr when neither LDS nor the pool has room.
__device__ __forceinline__ void* team_alloc(TeamStack* st, uint64_t bytes) {
    const uint64_t b = (bytes + kSharedAlign - 1) / kSharedAlign * kSharedAlign;
    __syncthreads();   // every thread has read the previous result
    if (threadIdx.x == 0) {
        void* p = nullptr;
        if (st->lds_top + b <= st->lds_cap) {
            p = st->lds + st->lds_top;
            st->lds_top += (uint32_t)b;
        } else if (st->glob && st->glob_top + b <= st->glob_cap) {
            p = st->glob + st->glob_top;
            st->glob_top += b;
        }
        st->last = p;
    }
    __syncthreads();
    return st->last;
}

// Team-collective; p and bytes as returned / requested by the matching
// team_alloc, which must be the most recent one still live.
__device__ __forceinline__ void team_free(TeamStack* st, void* p, uint64_t bytes) {
    const uint64_t b = (bytes + kSharedAlign - 1) / kSharedAlign * kSharedAlign;
    __syncthreads();   // every thread is done with the memory
    if (threadIdx.x == 0 && p) {
        if ((char*)p >= st->lds && (char*)p < st->lds + st->lds_cap)
            st->lds_top -= (uint32_t)b;
        else
            st->glob_top -= b;
    }
    __syncthreads();
}

}  // namespace omprt
