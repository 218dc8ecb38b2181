// accum.hpp -- the time average of Eq. 2 in the fused cadence kernels.
//
// A work-group images one (station, channel) over the whole cadence.  Each
// thread sums the products of the pixels it owns in FP32 registers over a
// block of at most B samples (B = the class's flush interval, 8 or 16), then
// adds the block sums to FP64 running sums; after the last sample the running
// sums times 1/n_time, rounded once to FP32, are the image.  The error of the
// mean is then at most about (B - 1) + 1/2 units in the last place of FP32
// relative to the sum of the magnitudes of the terms (the plain block sums;
// the FP64 sums and the final rounding add no more), whatever n_time is.
//
// The FP64 running sums live in the caller's image buffer: the channel's
// image region [n_pol^2][npix] of float2 has 8 bytes per (product, pixel),
// exactly one double per (real component, pixel) for the components XX,
// Re XY, Im XY, YY (n_pol = 2) or XX (n_pol = 1).  The last step reads all
// components of a pixel and then writes its products over them (XX, XY,
// YX = conj(XY), YY), so a pixel must be finished by one thread that has
// read all its components first.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace epic {

// Running sums of one (station, channel): component q of pixel k at base[q * npix + k].
struct ItemSums {
    double *base;
    int npix;
};

__device__ __forceinline__ ItemSums item_sums(float2 *image, int np, int npix, int c)
{
    return ItemSums{reinterpret_cast<double *>(image + static_cast<size_t>(c) * np * np * npix), npix};
}

// Add a block sum to component q of pixel k (the item's first block: set).
// Both are atomics whose result is not waited for, so the thread goes on with
// the next block while the L2 applies them; only this thread touches the
// address, and atomics of one thread to one address take effect in program
// order, so every sum is formed in the same order on every run.
__device__ __forceinline__ void sums_add(const ItemSums &s, int q, int k, float v, bool first)
{
    double *p = s.base + static_cast<size_t>(q) * s.npix + k;
    if (first)
        (void)atomicExch(reinterpret_cast<unsigned long long *>(p),
                         __double_as_longlong(static_cast<double>(v)));
    else
        (void)atomicAdd(p, static_cast<double>(v));
}

// Every running-sum atomic of this thread has been applied and the memory it
// reads next is not served from a stale cache line: before a thread reads
// the running sums back (and before the barrier after which other threads
// of the work-group read them).
__device__ __forceinline__ void sums_settle() { __threadfence(); }

// Pixel k's mean products over its running sums (inv = 1 / n_time).
template <int NP>
__device__ __forceinline__ void sums_finish(const ItemSums &s, int k, double inv)
{
    float2 *img = reinterpret_cast<float2 *>(s.base);
    const size_t n = static_cast<size_t>(s.npix);
    if constexpr (NP == 1) {
        const double a = s.base[k];
        img[k] = make_float2(static_cast<float>(a * inv), 0.f);
    } else {
        const double a0 = s.base[k], a1 = s.base[n + k], a2 = s.base[2 * n + k], a3 = s.base[3 * n + k];
        const float re = static_cast<float>(a1 * inv), im = static_cast<float>(a2 * inv);
        img[k] = make_float2(static_cast<float>(a0 * inv), 0.f);
        img[n + k] = make_float2(re, im);
        img[2 * n + k] = make_float2(re, -im);
        img[3 * n + k] = make_float2(static_cast<float>(a3 * inv), 0.f);
    }
}

// Whether the sample t (of [0, n_time)) ends a block of B samples.
__device__ __forceinline__ bool block_ends(int t, int n_time, int B)
{
    return (t + 1) % B == 0 || t + 1 == n_time;
}

}  // namespace epic
