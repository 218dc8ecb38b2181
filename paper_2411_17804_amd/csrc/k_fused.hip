// k_fused.hip -- the whole FP32 cadence for square grids up to 64 x 64 in one
// kernel: for each sample of a time chunk, grid the voltages (Eq. 3 inner
// bracket) into LDS, transform rows then columns in LDS (Eq. 3 outer sum),
// and accumulate the polarisation products (Eq. 2) in registers.  One
// work-group owns one (channel, time chunk) and writes the chunk's plain FP32
// partial sums; k_reduce (k_power.hip) adds the chunks in time order with
// compensation and applies 1/n_time.
//
// Only rows inside the kernel-footprint box carry data, so the row transforms
// run on those rows alone and the first column pass treats the other rows as
// zero.
#include "fft_lds.hpp"
#include "internal.hpp"
#include "volts.hpp"

namespace epic {

template <int N> struct FusedShape;
template <> struct FusedShape<16> { static constexpr int BLOCK = 128; };
template <> struct FusedShape<32> { static constexpr int BLOCK = 256; };
template <> struct FusedShape<64> { static constexpr int BLOCK = 512; };

template <int N, int NP, int VT>
__global__ __launch_bounds__(FusedShape<N>::BLOCK) void k_fused_fft(StationDev sd, int n_time,
                                                                    int chunk,
                                                                    float *__restrict__ partials,
                                                                    const float2 *__restrict__ twg)
{
    constexpr int BLOCK = FusedShape<N>::BLOCK;
    constexpr int P = N + 1;                 // row pitch (float2) in LDS
    constexpr int PLANE = N * P;
    constexpr int NPIX = N * N;
    constexpr int NQ = NP == 2 ? 4 : 1;
    constexpr int PXT = (NPIX + BLOCK - 1) / BLOCK;   // pixels per thread
    extern __shared__ float2 lds[];
    float2 *buf = lds;                       // [NP][N][P]
    float2 *tw = lds + NP * PLANE;           // [N]

    const int ck = blockIdx.x, c = blockIdx.y;
    const int n_chunks = gridDim.x;
    const int t_begin = ck * chunk;
    const int t_end = min(n_time, t_begin + chunk);
    const ChanPlan cp = sd.chan[c];
    const int32_t *cs = sd.cell_start + cp.cell_off;
    const Tap *taps = sd.taps + cp.tap_off;

    for (int i = threadIdx.x; i < N; i += BLOCK) tw[i] = twg[i];

    float acc[PXT][NQ];
#pragma unroll
    for (int i = 0; i < PXT; ++i)
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[i][q] = 0.f;

    const int rows = cp.bh;
    const int row_cells = rows * N;
    for (int t = t_begin; t < t_end; ++t) {
        const size_t vrow = (static_cast<size_t>(c) * n_time + t) * sd.n_elem;
        // 1. gather the footprint rows (full width; zero outside the box)
        for (int i = threadIdx.x; i < row_cells; i += BLOCK) {
            const int ry = i / N, x = i - ry * N;
            const int bx = x - cp.x0;
            float2 a[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) a[p] = make_float2(0.f, 0.f);
            if (bx >= 0 && bx < cp.bw) {
                const int cell = ry * cp.bw + bx;
                const int k1 = cs[cell + 1];
                for (int k = cs[cell]; k < k1; ++k) {
                    const Tap tp = taps[k];
                    float2 e[NP];
                    load_volt<NP, VT>(sd.volts, vrow + tp.elem, e);
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        a[p].x = fmaf(tp.w, e[p].x, a[p].x);
                        a[p].y = fmaf(tp.w, e[p].y, a[p].y);
                    }
                }
            }
            const int y = cp.y0 + ry;
#pragma unroll
            for (int p = 0; p < NP; ++p) buf[p * PLANE + y * P + x] = a[p];
        }
        __syncthreads();
        // 2. rows inside the box, 3. all columns (rows outside the box are zero)
        fft_lines<N, BLOCK, NP * N, false>(buf, LineMap{rows, cp.y0, PLANE, P, 1}, NP * rows, tw);
        fft_lines<N, BLOCK, NP * N, true>(buf, LineMap{N, 0, PLANE, 1, P}, NP * N, tw, cp.y0,
                                          cp.y0 + rows);
        // 4. products of this sample, accumulated per owned pixel
#pragma unroll
        for (int i = 0; i < PXT; ++i) {
            const int k = threadIdx.x + i * BLOCK;
            if (NPIX % BLOCK == 0 || k < NPIX) {
                const int ky = k / N, kx = k - ky * N;
                const float2 fx = buf[ky * P + kx];
                acc[i][0] = fmaf(fx.x, fx.x, fmaf(fx.y, fx.y, acc[i][0]));
                if constexpr (NP == 2) {
                    const float2 fy = buf[PLANE + ky * P + kx];
                    acc[i][1] = fmaf(fx.x, fy.x, fmaf(fx.y, fy.y, acc[i][1]));
                    acc[i][2] = fmaf(fx.y, fy.x, fmaf(-fx.x, fy.y, acc[i][2]));
                    acc[i][3] = fmaf(fy.x, fy.x, fmaf(fy.y, fy.y, acc[i][3]));
                }
            }
        }
        __syncthreads();
    }
    float *out = partials + (static_cast<size_t>(c) * n_chunks + ck) * NQ * NPIX;
#pragma unroll
    for (int i = 0; i < PXT; ++i) {
        const int k = threadIdx.x + i * BLOCK;
        if (NPIX % BLOCK == 0 || k < NPIX)
#pragma unroll
            for (int q = 0; q < NQ; ++q) out[q * NPIX + k] = acc[i][q];
    }
}

namespace {

template <int N, int NP, int VT>
epic_status run_fused(const StationDev &sd, int n_chan, int n_time, int chunk, float *partials,
                      const float2 *tw, hipStream_t stream)
{
    constexpr int BLOCK = FusedShape<N>::BLOCK;
    const size_t bytes = sizeof(float2) * (NP * N * (N + 1) + N);
    auto k = k_fused_fft<N, NP, VT>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(bytes));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    const int n_chunks = (n_time + chunk - 1) / chunk;
    KernelTimer timer("fused_fft_cadence", stream);
    hipLaunchKernelGGL(k, dim3(n_chunks, n_chan), dim3(BLOCK), bytes, stream, sd, n_time, chunk,
                       partials, tw);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

template <int N>
epic_status dispatch(const StationDev &sd, int n_pol, int n_chan, int n_time, int volt_type,
                     int chunk, float *partials, const float2 *tw, hipStream_t stream)
{
    if (n_pol == 2 && volt_type == EPIC_CI8)
        return run_fused<N, 2, EPIC_CI8>(sd, n_chan, n_time, chunk, partials, tw, stream);
    if (n_pol == 2)
        return run_fused<N, 2, EPIC_CF32>(sd, n_chan, n_time, chunk, partials, tw, stream);
    if (volt_type == EPIC_CI8)
        return run_fused<N, 1, EPIC_CI8>(sd, n_chan, n_time, chunk, partials, tw, stream);
    return run_fused<N, 1, EPIC_CF32>(sd, n_chan, n_time, chunk, partials, tw, stream);
}

}  // namespace

epic_status launch_fused_fft_partials(const StationDev &sd, int n_pol, int n_chan, int n_time,
                                      int volt_type, int chunk, float *partials,
                                      const float2 *twiddles, hipStream_t stream)
{
    switch (sd.nx) {
    case 16: return dispatch<16>(sd, n_pol, n_chan, n_time, volt_type, chunk, partials, twiddles, stream);
    case 32: return dispatch<32>(sd, n_pol, n_chan, n_time, volt_type, chunk, partials, twiddles, stream);
    case 64: return dispatch<64>(sd, n_pol, n_chan, n_time, volt_type, chunk, partials, twiddles, stream);
    }
    return fail(EPIC_ERR_INTERNAL, "fused FFT path: unsupported grid");
}

}  // namespace epic
