// volts.hpp -- exact conversion of one element's voltages (all pols) to FP32.
#pragma once

#include <hip/hip_runtime.h>

#include "epic.h"

namespace epic {

// volts layout: [...][n_elem][NP] complex; `idx` counts elements.
template <int NP, int VT>
__device__ __forceinline__ void load_volt(const void *volts, size_t idx, float2 *e)
{
    if constexpr (VT == EPIC_CI8) {
        if constexpr (NP == 2) {
            const int w = reinterpret_cast<const int *>(volts)[idx];   // re0 im0 re1 im1
            e[0] = make_float2(static_cast<float>(static_cast<int8_t>(w & 0xff)),
                               static_cast<float>(static_cast<int8_t>((w >> 8) & 0xff)));
            e[1] = make_float2(static_cast<float>(static_cast<int8_t>((w >> 16) & 0xff)),
                               static_cast<float>(static_cast<int8_t>((w >> 24) & 0xff)));
        } else {
            const short w = reinterpret_cast<const short *>(volts)[idx];
            e[0] = make_float2(static_cast<float>(static_cast<int8_t>(w & 0xff)),
                               static_cast<float>(static_cast<int8_t>((w >> 8) & 0xff)));
        }
    } else {
        if constexpr (NP == 2) {
            const float4 w = reinterpret_cast<const float4 *>(volts)[idx];
            e[0] = make_float2(w.x, w.y);
            e[1] = make_float2(w.z, w.w);
        } else {
            e[0] = reinterpret_cast<const float2 *>(volts)[idx];
        }
    }
}

}  // namespace epic
