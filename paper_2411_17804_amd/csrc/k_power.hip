// k_power.hip -- squaring and temporal averaging (Eq. 2): the polarisation
// outer products F^a conj(F^b) summed over the cadence with compensated
// (error-free two-sum) FP32 accumulation, then scaled by 1/n_time.
//
// Products are kept as four real components per pixel: XX, Re XY, Im XY, YY
// (n_pol = 2) or XX (n_pol = 1).  XX and YY are formed as re^2 + im^2, so their
// imaginary parts are exactly zero; YX is written as the exact conjugate of XY.
#include <algorithm>

#include "internal.hpp"

namespace epic {

// s + c accumulates x exactly up to the final rounding of s + c (Knuth's
// two-sum; only additions, so contraction into FMA cannot change it).
__device__ __forceinline__ void two_sum_acc(float &s, float &c, float x)
{
    const float t = s + x;
    const float bp = t - s;
    const float err = (s - (t - bp)) + (x - bp);
    s = t;
    c += err;
}

// Real components of the products of one pixel.
template <int NP>
__device__ __forceinline__ void products(const float2 *f, float *q)
{
    q[0] = fmaf(f[0].x, f[0].x, f[0].y * f[0].y);
    if constexpr (NP == 2) {
        q[1] = fmaf(f[0].x, f[1].x, f[0].y * f[1].y);       // Re F^X conj(F^Y)
        q[2] = fmaf(f[0].y, f[1].x, -(f[0].x * f[1].y));    // Im F^X conj(F^Y)
        q[3] = fmaf(f[1].x, f[1].x, f[1].y * f[1].y);
    }
}

template <int NP>
__device__ __forceinline__ void store_products(float2 *dst, size_t npix, size_t k, const float *v)
{
    if constexpr (NP == 1) {
        dst[k] = make_float2(v[0], 0.f);
    } else {
        dst[k] = make_float2(v[0], 0.f);
        dst[npix + k] = make_float2(v[1], v[2]);
        dst[2 * npix + k] = make_float2(v[1], -v[2]);
        dst[3 * npix + k] = make_float2(v[3], 0.f);
    }
}

// One thread per (channel, pixel); loops over the nt samples in order, with
// U samples' loads in flight at once (then summed in sample order: the same
// additions in the same order whatever U is).  Short loops (few samples per
// thread, many threads) need the extra loads in flight to keep HBM busy; long
// ones already do one sample at a time and lose to the extra streams (on
// 128 x 128 planes, 2 pols: 64 samples x 256 channels 1.05 -> 0.92 ms with
// U = 4, 256 samples x 64 channels 0.75 -> 0.82 ms).
template <int NP, int U>
__global__ __launch_bounds__(256) void k_power(int npix, int n_chan, int nt,
                                               const float2 *__restrict__ field,
                                               float2 *__restrict__ acc_sum,
                                               float2 *__restrict__ acc_comp, int finalize,
                                               float inv_n, float2 *__restrict__ image)
{
    constexpr int NQ = NP == 2 ? 4 : 1;
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid >= static_cast<int64_t>(n_chan) * npix) return;
    const int c = static_cast<int>(gid / npix);
    const int k = static_cast<int>(gid - static_cast<int64_t>(c) * npix);
    const size_t abase = static_cast<size_t>(c) * NP * NP * npix;
    float s[NQ], cc[NQ];
    {
        const float2 a0 = acc_sum[abase + k], c0 = acc_comp[abase + k];
        s[0] = a0.x;
        cc[0] = c0.x;
        if constexpr (NP == 2) {
            const float2 a1 = acc_sum[abase + npix + k], c1 = acc_comp[abase + npix + k];
            const float2 a3 = acc_sum[abase + 3 * npix + k], c3 = acc_comp[abase + 3 * npix + k];
            s[1] = a1.x; s[2] = a1.y; s[3] = a3.x;
            cc[1] = c1.x; cc[2] = c1.y; cc[3] = c3.x;
        }
    }
    const float2 *f = field + static_cast<size_t>(c) * nt * NP * npix + k;
    int t = 0;
    for (; t + U <= nt; t += U) {
        float2 v[U][NP];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int p = 0; p < NP; ++p) v[u][p] = f[(static_cast<size_t>(t + u) * NP + p) * npix];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            float q[NQ];
            products<NP>(v[u], q);
#pragma unroll
            for (int i = 0; i < NQ; ++i) two_sum_acc(s[i], cc[i], q[i]);
        }
    }
    for (; t < nt; ++t) {
        float2 v[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p) v[p] = f[(static_cast<size_t>(t) * NP + p) * npix];
        float q[NQ];
        products<NP>(v, q);
#pragma unroll
        for (int i = 0; i < NQ; ++i) two_sum_acc(s[i], cc[i], q[i]);
    }
    store_products<NP>(acc_sum + abase, npix, k, s);
    store_products<NP>(acc_comp + abase, npix, k, cc);
    if (finalize) {
        float m[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) m[i] = (s[i] + cc[i]) * inv_n;
        store_products<NP>(image + abase, npix, k, m);
    }
}

epic_status launch_power(int n_pol, int npix, int n_chan, int nt, const float2 *field,
                         float2 *acc_sum, float2 *acc_comp, int finalize_n_time, float2 *image,
                         hipStream_t stream)
{
    const int64_t n = static_cast<int64_t>(n_chan) * npix;
    const dim3 blocks(static_cast<unsigned>((n + 255) / 256)), threads(256);
    const float inv = finalize_n_time > 0 ? static_cast<float>(1.0 / finalize_n_time) : 0.f;
    KernelTimer timer("square_accumulate", stream);
    const int fin = finalize_n_time > 0 ? 1 : 0;
    const bool batch4 = nt <= 64;                 // short per-thread loops
    if (n_pol == 2 && batch4)
        hipLaunchKernelGGL((k_power<2, 4>), blocks, threads, 0, stream, npix, n_chan, nt, field, acc_sum,
                           acc_comp, fin, inv, image);
    else if (n_pol == 2)
        hipLaunchKernelGGL((k_power<2, 1>), blocks, threads, 0, stream, npix, n_chan, nt, field, acc_sum,
                           acc_comp, fin, inv, image);
    else if (batch4)
        hipLaunchKernelGGL((k_power<1, 4>), blocks, threads, 0, stream, npix, n_chan, nt, field, acc_sum,
                           acc_comp, fin, inv, image);
    else
        hipLaunchKernelGGL((k_power<1, 1>), blocks, threads, 0, stream, npix, n_chan, nt, field, acc_sum,
                           acc_comp, fin, inv, image);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

__global__ __launch_bounds__(256) void k_queue_reset(int *__restrict__ counters, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) counters[i] = 0;
}

epic_status launch_queue_reset(int *counters, int n, hipStream_t stream)
{
    if (n <= 0) return EPIC_OK;
    hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(256), 0, stream, counters, n);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

__global__ __launch_bounds__(256) void k_zero(uint32_t *__restrict__ p, size_t n)
{
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<size_t>(gridDim.x) * blockDim.x)
        p[i] = 0u;
}

epic_status launch_zero(void *p, size_t bytes, hipStream_t stream)
{
    const size_t n = bytes / 4;
    if (n == 0) return EPIC_OK;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                       static_cast<uint32_t *>(p), n);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

}  // namespace epic
