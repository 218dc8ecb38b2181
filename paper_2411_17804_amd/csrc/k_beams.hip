// k_beams.hip -- the corner turn of coherent inter-station EPIC (Sec. 6.2,
// Eq. 10): the station-synthesised fields, one array per station laid out
// [c][t][p][beam pixel], become the voltages of array-scale imaging problems,
// one per (channel, selected beam pixel), laid out [problem][t][station][p]
// like any element voltages.
#include <algorithm>

#include "internal.hpp"
#include "volts.hpp"

namespace epic {

namespace {

constexpr int kGbBlock = 256;

// One thread per output value; problems item0 .. item0 + n_items - 1 of the
// (channel, pixel) order c * n_sel + s.
__global__ __launch_bounds__(kGbBlock) void k_gather_beams(StationImages beams, int n_st, int n_pol,
                                                           int n_time, int npix_b, int n_sel,
                                                           const int32_t *__restrict__ pix,
                                                           int64_t item0, int64_t n_items,
                                                           float2 *__restrict__ out)
{
    const int64_t total = n_items * n_time * n_st * n_pol;
    for (int64_t idx = static_cast<int64_t>(blockIdx.x) * kGbBlock + threadIdx.x; idx < total;
         idx += static_cast<int64_t>(gridDim.x) * kGbBlock) {
        int64_t r = idx;
        const int p = static_cast<int>(r % n_pol);
        r /= n_pol;
        const int m = static_cast<int>(r % n_st);
        r /= n_st;
        const int t = static_cast<int>(r % n_time);
        const int64_t item = item0 + r / n_time;
        const int c = static_cast<int>(item / n_sel), s = static_cast<int>(item % n_sel);
        const size_t off = ((static_cast<size_t>(c) * n_time + t) * n_pol + p) * npix_b + pix[s];
        out[idx] = gload<float2>(beams.p[m], off);
    }
}

}  // namespace

epic_status launch_gather_beams(const StationImages &beams, int n_st, int n_pol, int n_time,
                                int npix_b, int n_sel, const int32_t *pix, int64_t item0,
                                int64_t n_items, float2 *out, hipStream_t stream)
{
    const int64_t total = n_items * n_time * n_st * n_pol;
    const int64_t blocks = std::min<int64_t>((total + kGbBlock - 1) / kGbBlock, 1 << 20);
    KernelTimer timer("gather_beams", stream);
    hipLaunchKernelGGL(k_gather_beams, dim3(static_cast<unsigned>(blocks)), dim3(kGbBlock), 0, stream,
                       beams, n_st, n_pol, n_time, npix_b, n_sel, pix, item0, n_items, out);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

}  // namespace epic
