// k_grid.hip -- gridding of element voltages (Eq. 3, inner bracket) as a
// gather: each cell of the kernel-footprint box sums weight * voltage over
// the (element, weight) taps the plan lists for it, in ascending element
// order, so results are deterministic and no atomics are needed.
#include "internal.hpp"
#include "volts.hpp"

namespace epic {

// One work-group per (channel, block of TB samples): every cell's tap list is
// read once and applied to the TB samples, whose voltage loads are independent
// of each other.  Writes all n_pol planes of each sample's ny x nx grid (zero
// outside the footprint box).
template <int NP, int VT, int TB>
__global__ __launch_bounds__(256) void k_grid(StationDev sd, int n_time, int t0, int nt,
                                              float2 *__restrict__ grid)
{
    const int tb = blockIdx.x * TB;
    const int c = blockIdx.y;
    const int nts = min(TB, nt - tb);
    const ChanPlan cp = sd.chan[c];
    const int32_t *cs = sd.cell_start + cp.cell_off;
    const Tap *taps = sd.taps + cp.tap_off;
    const int nx = sd.nx, ny = sd.ny;
    const int npix = nx * ny;
    const size_t vrow0 = (static_cast<size_t>(c) * n_time + t0 + tb) * sd.n_elem;
    const size_t vstride = sd.n_elem;                      // elements per sample
    float2 *out = grid + (static_cast<size_t>(c) * nt + tb) * NP * npix;
    for (int i = threadIdx.x; i < npix; i += blockDim.x) {
        const int y = i / nx, x = i - y * nx;
        const int bx = x - cp.x0, by = y - cp.y0;
        float2 acc[TB][NP];
#pragma unroll
        for (int t = 0; t < TB; ++t)
#pragma unroll
            for (int p = 0; p < NP; ++p) acc[t][p] = make_float2(0.f, 0.f);
        if (bx >= 0 && bx < cp.bw && by >= 0 && by < cp.bh) {
            const int cell = by * cp.bw + bx;
            const int k1 = cs[cell + 1];
            for (int k = cs[cell]; k < k1; ++k) {
                const Tap tp = taps[k];
#pragma unroll
                for (int t = 0; t < TB; ++t) {
                    if (t < nts) {
                        float2 e[NP];
                        load_volt<NP, VT>(sd.volts, vrow0 + t * vstride + tp.elem, e);
#pragma unroll
                        for (int p = 0; p < NP; ++p) {
                            acc[t][p].x = fmaf(tp.w, e[p].x, acc[t][p].x);
                            acc[t][p].y = fmaf(tp.w, e[p].y, acc[t][p].y);
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int t = 0; t < TB; ++t)
            if (t < nts)
#pragma unroll
                for (int p = 0; p < NP; ++p)
                    out[(static_cast<size_t>(t) * NP + p) * npix + i] = acc[t][p];
    }
}

epic_status launch_grid(const StationDev &sd, int n_pol, int n_chan, int n_time, int volt_type,
                        int t0, int nt, float2 *grid, hipStream_t stream)
{
    constexpr int TB = 8;
    const dim3 blocks((nt + TB - 1) / TB, n_chan), threads(256);
    KernelTimer timer("grid_gather", stream);
    if (n_pol == 1 && volt_type == EPIC_CI8)
        hipLaunchKernelGGL((k_grid<1, EPIC_CI8, TB>), blocks, threads, 0, stream, sd, n_time, t0, nt, grid);
    else if (n_pol == 1)
        hipLaunchKernelGGL((k_grid<1, EPIC_CF32, TB>), blocks, threads, 0, stream, sd, n_time, t0, nt, grid);
    else if (volt_type == EPIC_CI8)
        hipLaunchKernelGGL((k_grid<2, EPIC_CI8, TB>), blocks, threads, 0, stream, sd, n_time, t0, nt, grid);
    else
        hipLaunchKernelGGL((k_grid<2, EPIC_CF32, TB>), blocks, threads, 0, stream, sd, n_time, t0, nt, grid);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

}  // namespace epic
