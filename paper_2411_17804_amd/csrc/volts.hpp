// volts.hpp -- exact conversion of one element's voltages (all pols) to FP32.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "epic.h"

namespace epic {

// A pointer to device-global memory that arrived as a plain `const void *`
// (for instance a field of a table in memory) compiles to FLAT loads, whose
// completion the hardware also counts on the LDS counter, so a kernel that
// prefetches through it waits for the prefetch at its next LDS access.  Going
// through the global address space gives global loads instead.
template <typename T>
using gptr = const __attribute__((address_space(1))) T *;

template <typename T>
__device__ __forceinline__ gptr<T> global_ptr(const void *p)
{
    return (gptr<T>)(p);
}

// Element i of a device-global array of a trivially copyable 2-, 4-, 8- or
// 16-byte type (structs and HIP vector types included), as a global load.
template <typename T>
__device__ __forceinline__ T gload(const void *p, size_t i)
{
    if constexpr (sizeof(T) == 2) {
        return __builtin_bit_cast(T, global_ptr<uint16_t>(p)[i]);
    } else if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, global_ptr<uint32_t>(p)[i]);
    } else if constexpr (sizeof(T) == 8) {
        return __builtin_bit_cast(T, global_ptr<uint64_t>(p)[i]);
    } else {
        static_assert(sizeof(T) == 16, "gload: 2, 4, 8 or 16 bytes");
        using u32x4 = __attribute__((ext_vector_type(4))) uint32_t;
        return __builtin_bit_cast(T, global_ptr<u32x4>(p)[i]);
    }
}

// volts layout: [...][n_elem][NP] complex; `idx` counts elements.
template <int NP, int VT>
__device__ __forceinline__ void load_volt(const void *volts, size_t idx, float2 *e)
{
    if constexpr (VT == EPIC_CI8) {
        if constexpr (NP == 2) {
            const int w = global_ptr<int>(volts)[idx];   // re0 im0 re1 im1
            e[0] = make_float2(static_cast<float>(static_cast<int8_t>(w & 0xff)),
                               static_cast<float>(static_cast<int8_t>((w >> 8) & 0xff)));
            e[1] = make_float2(static_cast<float>(static_cast<int8_t>((w >> 16) & 0xff)),
                               static_cast<float>(static_cast<int8_t>((w >> 24) & 0xff)));
        } else {
            const short w = global_ptr<short>(volts)[idx];
            e[0] = make_float2(static_cast<float>(static_cast<int8_t>(w & 0xff)),
                               static_cast<float>(static_cast<int8_t>((w >> 8) & 0xff)));
        }
    } else {
        if constexpr (NP == 2) {
            const float4 w = gload<float4>(volts, idx);
            e[0] = make_float2(w.x, w.y);
            e[1] = make_float2(w.z, w.w);
        } else {
            e[0] = gload<float2>(volts, idx);
        }
    }
}

}  // namespace epic
