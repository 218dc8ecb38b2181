// queue.hpp -- the work queue of the persistent cadence kernels.
//
// A class kernel is launched with about as many work-groups as the GPU holds
// at once; each work-group takes items from the queue until it is empty, so
// the time of the launch is set by the work, not by the order in which the
// hardware happens to dispatch work-groups.  The items of a class are split
// over the eight XCDs of the MI355X (each with its own L2): a (station,
// channel) pair's items all sit in one XCD's list, so its taps, voltages and
// partial sums stay in that L2, and the lists are balanced by cost.  Within
// a list items are in descending cost order (longest first).  Work-group b
// serves list b mod 8 first (work-groups are dispatched to the XCDs round
// robin) and then helps the other lists.  Each list has a counter that the
// queue-reset kernel clears before every cadence; a work-group claims an
// item with one atomic add, and every work-group leaves once every list is
// exhausted, so the kernel always ends.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace epic {

constexpr int kXcds = 8;

struct ItemQueue {
    const int4 *items;            // device: the items of all lists, list x at [start[x], start[x + 1])
    int *counters;                // device: kXcds claim counters
    int start[kXcds + 1];
};

// Index of the next item for work-group `home` (its list first), or -1.
__device__ __forceinline__ int queue_claim(const ItemQueue &q, int home)
{
#pragma unroll 1
    for (int k = 0; k < kXcds; ++k) {
        const int x = (home + k) & (kXcds - 1);
        const int len = q.start[x + 1] - q.start[x];
        if (len <= 0) continue;
        const int i = atomicAdd(&q.counters[x], 1);
        if (i < len) return q.start[x] + i;
    }
    return -1;
}

// The item loop of a persistent work-group: `body(item)` for every item it
// claims.  The claim is broadcast through LDS; the barrier after the read
// keeps thread 0 from overwriting it before every thread has read it, and the
// one before the claim keeps the previous item's LDS reads ahead of the next
// item's writes.
// `slot` is one int of LDS; with `shared_slot` the item body may write that
// word too, so a third barrier keeps its first write behind every read of
// the claim.
template <typename F>
__device__ __forceinline__ void for_each_item(const ItemQueue &q, int *slot, F &&body, bool shared_slot = false)
{
    const int home = static_cast<int>(blockIdx.x) & (kXcds - 1);
#pragma unroll 1
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) *slot = queue_claim(q, home);
        __syncthreads();
        // the same value in every lane: a scalar, so the item's tables are
        // read with scalar loads into scalar registers
        const int it = __builtin_amdgcn_readfirstlane(*slot);
        if (shared_slot) __syncthreads();
        if (it < 0) break;
        body(q.items[it]);
    }
}

// The claim slot takes 16 bytes of static LDS, so that the kernels'
// dynamic LDS after it stays 16-byte aligned for their 128-bit accesses.
template <typename F>
__device__ __forceinline__ void for_each_item(const ItemQueue &q, F &&body)
{
    __shared__ __align__(16) int s_item[4];
    for_each_item(q, s_item, body);
}

}  // namespace epic
