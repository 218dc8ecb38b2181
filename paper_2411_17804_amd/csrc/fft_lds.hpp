// fft_lds.hpp -- FP32 building blocks of the 2-D transform of Eq. 3 (outer
// sum, + sign, unnormalised): small DFTs in registers and one mixed-radix
// Stockham pass over lines held in LDS.
//
// A length-N line is transformed by passes of radix R_1, R_2, ... (product N).
// Pass i (sub-transform length Ns = R_1 ... R_{i-1} before it) takes, for each
// butterfly j < N/R, the R inputs x[j + r N/R], multiplies input r by
// exp(+2 pi i r (j mod Ns) / (Ns R)), does an R-point DFT and stores output r
// at ((j / Ns) Ns R + j mod Ns) + r Ns.  The result is in natural order
// (Stockham autosort: no bit reversal).
#pragma once

#include <hip/hip_runtime.h>

#include "lds_sync.hpp"

namespace epic {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// cos and sin of 2 pi k / 16, k = 0..15 (exact mathematical constants).
constexpr float kCos16[16] = {1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                              0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                              -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f,
                              0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f};
constexpr float kSin16[16] = {0.0f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
                              1.0f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                              0.0f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f,
                              -1.0f, -0.92387953251128674f, -0.70710678118654752f, -0.38268343236508977f};

// v * exp(+2 pi i K / R) for compile-time K < R/2, R | 16.
template <int K, int R>
__device__ __forceinline__ float2 rot(float2 v)
{
    constexpr int q = K * (16 / R);   // angle in sixteenths of a turn, 0..7
    if constexpr (q == 0) {
        return v;
    } else if constexpr (q == 4) {    // * i
        return make_float2(-v.y, v.x);
    } else if constexpr (q == 2) {    // * (1 + i)/sqrt2
        constexpr float c = kCos16[2];
        return make_float2((v.x - v.y) * c, (v.x + v.y) * c);
    } else if constexpr (q == 6) {    // * (-1 + i)/sqrt2
        constexpr float c = kCos16[2];
        return make_float2((-v.x - v.y) * c, (v.x - v.y) * c);
    } else {
        constexpr float c = kCos16[q], s = kSin16[q];
        return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
    }
}

// In-register R-point DFT with the + sign, R in {2, 4, 8, 16}: radix-2
// decimation in time on the even and odd halves.
template <int R>
struct Dft {
    template <int K>
    __device__ __forceinline__ static void combine(float2 *v, const float2 *e, const float2 *o)
    {
        if constexpr (K < R / 2) {
            const float2 t = rot<K, R>(o[K]);
            v[K] = cadd(e[K], t);
            v[K + R / 2] = csub(e[K], t);
            combine<K + 1>(v, e, o);
        }
    }
    __device__ __forceinline__ static void run(float2 *v)
    {
        float2 e[R / 2], o[R / 2];
#pragma unroll
        for (int i = 0; i < R / 2; ++i) {
            e[i] = v[2 * i];
            o[i] = v[2 * i + 1];
        }
        Dft<R / 2>::run(e);
        Dft<R / 2>::run(o);
        combine<0>(v, e, o);
    }
};

template <>
struct Dft<2> {
    __device__ __forceinline__ static void run(float2 *v)
    {
        const float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
};

template <>
struct Dft<4> {
    __device__ __forceinline__ static void run(float2 *v)
    {
        const float2 y0 = cadd(v[0], v[2]), y1 = csub(v[0], v[2]);
        const float2 y2 = cadd(v[1], v[3]);
        const float2 d = csub(v[1], v[3]);
        const float2 y3 = make_float2(-d.y, d.x);   // * i
        v[0] = cadd(y0, y2);
        v[2] = csub(y0, y2);
        v[1] = cadd(y1, y3);
        v[3] = csub(y1, y3);
    }
};

// Radix split used for each line length (first pass radix, second pass radix).
template <int N> struct Radix;
template <> struct Radix<16> { static constexpr int R1 = 4, R2 = 4; };
template <> struct Radix<32> { static constexpr int R1 = 8, R2 = 4; };
template <> struct Radix<64> { static constexpr int R1 = 8, R2 = 8; };
template <> struct Radix<128> { static constexpr int R1 = 8, R2 = 16; };
template <> struct Radix<256> { static constexpr int R1 = 16, R2 = 16; };

// Describes where the lines of one pass live in LDS: line l of group g starts
// at g * group_stride + (first + l) * line_stride and its points are
// elem_stride apart.  lines_per_group lines per group.
struct LineMap {
    int lines_per_group;
    int first;
    int group_stride;
    int line_stride;
    int elem_stride;
};

// One Stockham pass (radix R, Ns = product of earlier radices) over n_lines
// lines of N points in LDS, in place: every butterfly is read into registers,
// the block synchronises, then all results are written.  MASK: inputs whose
// index along the line lies outside [lo, hi) are taken as zero (used on the
// first pass along y, where rows outside the kernel footprint are zero).
// tw: exp(+2 pi i k / N), k < N, readable by every thread.
template <int N, int R, int NS, int BLOCK, int MAXLINES, bool MASK>
__device__ __forceinline__ void stockham_pass(float2 *buf, const LineMap m, int n_lines,
                                              const float2 *tw, int lo = 0, int hi = 0)
{
    constexpr int NB = N / R;
    constexpr int MAXB = (MAXLINES * NB + BLOCK - 1) / BLOCK;
    const int total = n_lines * NB;
    float2 v[MAXB][R];
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = threadIdx.x + i * BLOCK;
        if (b < total) {
            const int line = b / NB, j = b % NB;
            const int g = line / m.lines_per_group, l = line - g * m.lines_per_group;
            const float2 *src = buf + g * m.group_stride + (m.first + l) * m.line_stride;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int idx = j + r * NB;
                if constexpr (MASK) {
                    v[i][r] = (idx >= lo && idx < hi) ? src[idx * m.elem_stride] : make_float2(0.f, 0.f);
                } else {
                    v[i][r] = src[idx * m.elem_stride];
                }
            }
            if constexpr (NS > 1) {
                const int k = j % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], tw[r * k * (N / (NS * R))]);
            }
            Dft<R>::run(v[i]);
        }
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
        const int b = threadIdx.x + i * BLOCK;
        if (b < total) {
            const int line = b / NB, j = b % NB;
            const int g = line / m.lines_per_group, l = line - g * m.lines_per_group;
            float2 *dst = buf + g * m.group_stride + (m.first + l) * m.line_stride;
            const int d0 = (j / NS) * NS * R + (j % NS);
#pragma unroll
            for (int r = 0; r < R; ++r) dst[(d0 + r * NS) * m.elem_stride] = v[i][r];
        }
    }
    lds_barrier();
}

// Both passes of a length-N transform over the lines described by m.
template <int N, int BLOCK, int MAXLINES, bool MASK_FIRST>
__device__ __forceinline__ void fft_lines(float2 *buf, const LineMap m, int n_lines,
                                          const float2 *tw, int lo = 0, int hi = 0)
{
    constexpr int R1 = Radix<N>::R1, R2 = Radix<N>::R2;
    stockham_pass<N, R1, 1, BLOCK, MAXLINES, MASK_FIRST>(buf, m, n_lines, tw, lo, hi);
    stockham_pass<N, R2, R1, BLOCK, MAXLINES, false>(buf, m, n_lines, tw);
}

}  // namespace epic
