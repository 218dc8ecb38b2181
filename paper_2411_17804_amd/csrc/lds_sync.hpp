// lds_sync.hpp -- a work-group barrier for LDS traffic only.
//
// __syncthreads() also orders global memory at work-group scope, so it waits
// for every outstanding global store and atomic of the wave (and for
// prefetched loads) before the barrier.  The fused kernels synchronise only
// their LDS between passes; their global stores (the running sums) and loads
// (the next sample's voltages) may stay in flight across those barriers.
// This barrier waits for the wave's LDS operations and then meets the others;
// uses of global loads are still ordered by the compiler's own waits.
#pragma once

#include <hip/hip_runtime.h>

namespace epic {

__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

}  // namespace epic
