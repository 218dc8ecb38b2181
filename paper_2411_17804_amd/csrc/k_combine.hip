// k_combine.hip -- incoherent combination of station images (Sec. 6.1,
// Eq. 7): per sky pixel, product and channel, the weighted mean of the
// stations' intensities,
//     I[c][q][k] = sum_m w[m][q][k] I_m[c][q][k] / sum_m w[m][q][k],
// for stations that share one sky pixel grid (same nx, ny and grid spacing in
// wavelengths).  The weights do not depend on the channel; they are re-read
// per channel from L2 (all of them together are a few MB).  The sums run over
// the stations in order, in FP32.
#include "internal.hpp"
#include "volts.hpp"

namespace epic {

namespace {

constexpr int kCombineBlock = 256;

}  // namespace

// One thread per output element (channel, product, pixel); grid.y = channel.
__global__ __launch_bounds__(kCombineBlock) void k_combine(StationImages imgs, int n_stations,
                                                           int plane, const float *__restrict__ w,
                                                           float2 *__restrict__ out)
{
    const int i = blockIdx.x * kCombineBlock + threadIdx.x;    // (product, pixel)
    if (i >= plane) return;
    const size_t off = static_cast<size_t>(blockIdx.y) * plane + i;
    float2 num = make_float2(0.f, 0.f);
    float den = 0.f;
#pragma unroll 8
    for (int m = 0; m < n_stations; ++m) {
        const float wm = w ? w[static_cast<size_t>(m) * plane + i] : 1.f;
        const float2 v = gload<float2>(imgs.p[m], off);
        num.x = fmaf(wm, v.x, num.x);
        num.y = fmaf(wm, v.y, num.y);
        den += wm;
    }
    const float inv = den != 0.f ? 1.f / den : 0.f;
    out[off] = make_float2(num.x * inv, num.y * inv);
}

epic_status launch_combine(const StationImages &imgs, int n_stations, int plane, int n_chan,
                           const float *weights, float2 *out, hipStream_t stream)
{
    const dim3 grid((plane + kCombineBlock - 1) / kCombineBlock, n_chan), threads(kCombineBlock);
    KernelTimer timer("combine_incoherent", stream);
    hipLaunchKernelGGL(k_combine, grid, threads, 0, stream, imgs, n_stations, plane, weights, out);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

}  // namespace epic
