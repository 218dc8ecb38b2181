// mfma_split.hpp -- split-precision complex products on gfx950 matrix cores.
//
// A value x (FP32) is carried as hi + lo with hi = round(x), lo = round(x - hi)
// in FP16 or BF16; a product a.b is formed as hi_a.hi_b + hi_a.lo_b + lo_a.hi_b
// with FP32 accumulation (the lo.lo term is below FP32 resolution of the
// result and is dropped).  Complex products use the real 2x2 block form: the
// K index of a product interleaves (re, im) of the complex summation index.
//
// MFMA v_mfma_f32_16x16x32_{f16,bf16} fragments (64 lanes, g = lane / 16):
//   A (16 x 32): lane holds row lane % 16, K entries 8g .. 8g+7
//   B (32 x 16): lane holds column lane % 16, K entries 8g .. 8g+7
//   D (16 x 16): lane holds column lane % 16, rows 4g .. 4g+3
// Only the D layout matters for correctness: A and B use the same K order,
// and a sum over K does not depend on the order of its terms' indices.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "epic.h"

namespace epic {

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

template <int PREC> struct Split;

template <> struct Split<EPIC_FP16_SPLIT> {
    using scalar = _Float16;
    using vec8 = half8_t;
    // FP16 holds |x| < 65504: inputs are scaled by a power of two first.
    static constexpr bool needs_scale = true;
    __device__ __forceinline__ static scalar round(float x) { return static_cast<scalar>(x); }
    __device__ __forceinline__ static floatx4_t mfma(vec8 a, vec8 b, floatx4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

template <> struct Split<EPIC_BF16_SPLIT> {
    using scalar = __bf16;
    using vec8 = bf16x8_t;
    static constexpr bool needs_scale = false;
    __device__ __forceinline__ static scalar round(float x) { return static_cast<scalar>(x); }
    __device__ __forceinline__ static floatx4_t mfma(vec8 a, vec8 b, floatx4_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

// x -> (hi, lo)
template <int PREC>
__device__ __forceinline__ void split(float x, typename Split<PREC>::scalar &hi,
                                      typename Split<PREC>::scalar &lo)
{
    hi = Split<PREC>::round(x);
    lo = Split<PREC>::round(x - static_cast<float>(hi));
}

// acc += a.b in split precision (three products, small terms first).
template <int PREC>
__device__ __forceinline__ floatx4_t mma3(typename Split<PREC>::vec8 ah, typename Split<PREC>::vec8 al,
                                          typename Split<PREC>::vec8 bh, typename Split<PREC>::vec8 bl,
                                          floatx4_t acc)
{
    acc = Split<PREC>::mfma(al, bh, acc);
    acc = Split<PREC>::mfma(ah, bl, acc);
    acc = Split<PREC>::mfma(ah, bh, acc);
    return acc;
}

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// Two split parts packed into 32 bits (a low, b high): one complex value
// (re, im) of an A or B fragment.
template <int PREC>
__device__ __forceinline__ uint32_t pack2(typename Split<PREC>::scalar a, typename Split<PREC>::scalar b)
{
    return static_cast<uint32_t>(__builtin_bit_cast(uint16_t, a)) |
           (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, b)) << 16);
}

// (re, im) packed -> (re, -im): 2x2 block column for the real output part
__device__ __forceinline__ uint32_t neg_hi(uint32_t w) { return w ^ 0x80000000u; }
// (re, im) packed -> (im, re): 2x2 block column for the imaginary output part
__device__ __forceinline__ uint32_t swap_halves(uint32_t w) { return (w >> 16) | (w << 16); }
// (re, im) packed -> (-re, -im)
__device__ __forceinline__ uint32_t neg_both(uint32_t w) { return w ^ 0x80008000u; }

// Voltage words per (element, pol) in the fused split kernels' LDS: int8
// voltages are held as an exact FP16 pair (one word), float voltages as a
// float pair (two words).
constexpr int volt_words(int vt) { return vt == EPIC_CI8 ? 1 : 2; }

// Power of two s with max_abs * s in [2^14, 2^15) (1 if max_abs is 0 or not
// finite), so scaled FP16 parts cannot overflow and keep full relative
// precision; exact to undo.
__device__ __forceinline__ float pow2_scale(float max_abs)
{
    if (!(max_abs > 0.f) || !(max_abs < 3.0e38f)) return 1.f;
    const int e = ilogbf(max_abs);                  // max_abs in [2^e, 2^(e+1))
    return ldexpf(1.f, min(126, max(-126, 14 - e)));
}

}  // namespace epic
