// k_fused128.hip -- the FP32 cadence for 128 x 128 grids.  One 128 x 128
// complex plane takes 128 KB of the 160 KB of LDS, which leaves no room for a
// channel's gather taps, so the cadence runs per time block in two kernels:
//
//   k_grid_box      grids each sample of the block (Eq. 3 inner bracket) into
//                   its footprint box only, [pair][t][pol][max_bh][max_bw] in a
//                   device buffer (a fraction of the full grid's bytes);
//   k_fused_fft128  per (station, channel) pair and block: transforms each
//                   sample's boxes (Eq. 3 outer sum) and accumulates the
//                   polarisation products (Eq. 2) in registers, writing the
//                   block's plain FP32 partial sums; k_reduce (k_power.hip)
//                   adds the blocks in time order with compensation.
//
// The 128-point transforms use 128 = 16 x 8: with x = j + 8m and
// k = k1 + 16 k2,
//   X[k1 + 16 k2] = sum_j w128^(j k1) w8^(j k2) sum_m a[j + 8m] w16^(m k1),
// where wN = exp(+2 pi i / N).  Pass A is a 16-point DFT per (line, j) and
// stores its output k1 at position j + 8 k1; pass B reads the 8 positions
// [8 k1, 8 k1 + 8), twiddles, does an 8-point DFT and writes output k2 back to
// position 8 k1 + k2.  Both passes therefore read and write the same
// positions of their own task, so neither needs a barrier between its loads
// and stores, and after both passes position p holds frequency
// (p >> 3) + 16 (p & 7).  Rows use this along x, columns along y; the
// pixel's frequency order is undone when the partial sums are written.
#include "fft_lds.hpp"
#include "internal.hpp"
#include "volts.hpp"

namespace epic {

namespace {

constexpr int kGridBoxBlock = 512;
constexpr size_t kGridBoxLds = 64 * 1024;   // voltage staging of one gridding work-group
constexpr int kF128Block = 512;
constexpr size_t kF128Lds = sizeof(float2) * (128 * 128 + 8 * kF128Block);   // plane + pol X hold of CB task 3

// LDS position of (row y, column position p) in the 128 x 128 plane.  The XOR
// of the low 3 bits with bits 3-5 keeps the stride-8 reads of pass B on
// distinct banks; the XOR of bits 3-4 with the row spreads the 4 to 8 rows a
// wave touches in the row passes.  Both stay inside each aligned block of 64
// positions, so the column passes (one row, 64 consecutive positions per
// wave) are conflict-free as well.
__device__ __forceinline__ int pl(int y, int p)
{
    return y * 128 + (p ^ ((p >> 3) & 7) ^ ((y & 3) << 3));
}

}  // namespace

// items: (station index, channel, 0, box offset in float2) per pair; grid:
// 8 ceil(pairs / 8) ceil(chunk / TB) work-groups; block b covers samples
// [b chunk, min(n_time, (b + 1) chunk)).  The TB samples' voltages are first
// copied (coalesced, converted to FP32) into LDS; then every box cell, in
// natural order so that the tap lists and the box rows are read and written
// contiguously, sums weight * voltage over its taps for the TB samples.
template <int NP, int VT, int TB>
__global__ __launch_bounds__(kGridBoxBlock) void k_grid_box(const StationDev *__restrict__ sds,
                                                            const int4 *__restrict__ items, int n_items,
                                                            int n_time, int chunk, int block,
                                                            float2 *__restrict__ boxes)
{
    extern __shared__ float2 vl[];                        // [TB][n_elem][NP]
    // Work-groups are dealt to the 8 XCDs round-robin; pair x + 8 k runs all
    // its sub-blocks on XCD x, back to back, so its tap lists stay in that
    // XCD's L2 instead of every L2 streaming every channel's taps.
    const int nsub = (chunk + TB - 1) / TB;
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int pair = xcd + 8 * (slot / nsub);
    if (pair >= n_items) return;
    const int4 item = items[pair];
    const int sub = slot - (slot / nsub) * nsub;
    const StationDev sd = sds[item.x];
    const int c = item.y;
    const int tb0 = block * chunk;
    const int t_first = tb0 + sub * TB;
    const int t_stop = min(min(n_time, tb0 + chunk), t_first + TB);
    const int nts = t_stop - t_first;
    if (nts <= 0) return;
    const int ne = sd.n_elem;
    const size_t vrow0 = (static_cast<size_t>(c) * n_time + t_first) * ne;
    {
        // all loads first, then all LDS stores: the staging is one round trip
        // to memory, not one per iteration (nts * ne * NP * 8 B <= the 64 KB
        // staging bound, so MAXIT rounds of the work-group cover it)
        constexpr int MAXIT = kGridBoxLds / (sizeof(float2) * NP * kGridBoxBlock);
        float2 e[MAXIT][NP];
#pragma unroll
        for (int q = 0; q < MAXIT; ++q) {
            const int i = threadIdx.x + q * kGridBoxBlock;
            if (i < nts * ne) load_volt<NP, VT>(sd.volts, vrow0 + i, e[q]);
        }
#pragma unroll
        for (int q = 0; q < MAXIT; ++q) {
            const int i = threadIdx.x + q * kGridBoxBlock;
            if (i < nts * ne)
#pragma unroll
                for (int p = 0; p < NP; ++p) vl[i * NP + p] = e[q][p];
        }
    }
    __syncthreads();
    const ChanPlan cp = sd.chan[c];
    const int32_t *cs = sd.cell_start + cp.cell_off;
    const Tap *taps = sd.taps + cp.tap_off;
    const size_t plane = static_cast<size_t>(sd.max_bh) * sd.max_bw;
    float2 *out = boxes + item.w + static_cast<size_t>(t_first - tb0) * NP * plane;
    const int ncell = cp.bw * cp.bh;
    // two cells per thread at a time and taps in groups of four, so that
    // several independent tap loads are in flight (padding taps weigh 0)
    for (int i0 = threadIdx.x; i0 < ncell; i0 += 2 * kGridBoxBlock) {
        int kb[2], ke[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = i0 + u * kGridBoxBlock;
            kb[u] = i < ncell ? cs[i] : 0;
            ke[u] = i < ncell ? cs[i + 1] : 0;
        }
        float2 acc[2][TB][NP];
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int t = 0; t < TB; ++t)
#pragma unroll
                for (int p = 0; p < NP; ++p) acc[u][t][p] = make_float2(0.f, 0.f);
        const int rounds = max(ke[0] - kb[0], ke[1] - kb[1]);
        for (int k = 0; k < rounds; k += 4) {
            Tap tq[2][4];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int kk = kb[u] + k + q;
                    tq[u][q] = kk < ke[u] ? taps[kk] : Tap{0, 0.f};
                }
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int t = 0; t < TB; ++t) {
                        if (t < nts) {
#pragma unroll
                            for (int p = 0; p < NP; ++p) {
                                const float2 e = vl[(t * ne + tq[u][q].elem) * NP + p];
                                acc[u][t][p].x = fmaf(tq[u][q].w, e.x, acc[u][t][p].x);
                                acc[u][t][p].y = fmaf(tq[u][q].w, e.y, acc[u][t][p].y);
                            }
                        }
                    }
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = i0 + u * kGridBoxBlock;
            if (i < ncell) {
                const int by = i / cp.bw, bx = i - by * cp.bw;
                const size_t o = static_cast<size_t>(by) * sd.max_bw + bx;
#pragma unroll
                for (int t = 0; t < TB; ++t)
                    if (t < nts)
#pragma unroll
                        for (int p = 0; p < NP; ++p)
                            out[(static_cast<size_t>(t) * NP + p) * plane + o] = acc[u][t][p];
            }
        }
    }
}

// One work-group per (station, channel) pair of the block.  Per sample and
// pol: RA (16-point DFTs of the box rows, read straight from the box buffer),
// RB (8-point DFTs along x, in place), CA and CB (the same two passes along y
// for all 128 columns; rows outside the box are zero).  CB leaves 32 pixels
// per thread in registers: pol X's are held until pol Y's arrive and the
// products are accumulated.
template <int NP>
__global__ __launch_bounds__(kF128Block) void k_fused_fft128(const StationDev *__restrict__ sds,
                                                             const int4 *__restrict__ items,
                                                             int n_time, int chunk, int block,
                                                             const float2 *__restrict__ boxes,
                                                             float *__restrict__ partials,
                                                             const float2 *__restrict__ twg)
{
    constexpr int N = 128;
    constexpr int PLANE = N * N;
    constexpr int NQ = NP == 2 ? 4 : 1;
    extern __shared__ float2 lds[];
    const int tid = threadIdx.x;
    const int4 item = items[blockIdx.x];
    const StationDev sd = sds[item.x];
    const int c = item.y;
    const ChanPlan cp = sd.chan[c];
    const int n_chunks = (n_time + chunk - 1) / chunk;
    const int tb0 = block * chunk;
    const int t_end = min(n_time, tb0 + chunk);
    const size_t bplane = static_cast<size_t>(sd.max_bh) * sd.max_bw;
    const float2 *box = boxes + item.w;

    // column tasks: CA j' and CB k1' are (tid >> 7) + 4 r, the same across a wave
    const int cgrp = __builtin_amdgcn_readfirstlane(tid >> 7);

    float acc[4][8][NQ];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[r][k][q] = 0.f;
    [[maybe_unused]] float2 hold[3][8];   // pol X pixels of CB tasks 0-2 (two pols)

    for (int t = tb0; t < t_end; ++t) {
#pragma unroll 1
        for (int pol = 0; pol < NP; ++pol) {
            // Lane-dependent indices are re-derived from an opaque copy of the
            // thread index each pass, so the compiler recomputes addresses
            // instead of keeping dozens of them live across the sample loop.
            int lt;
            asm volatile("v_mov_b32 %0, %1" : "=v"(lt) : "v"(tid));
            // row tasks: RA (y_local = q >> 3, j = q & 7), RB (y_local = q >> 4,
            // k1 = q & 15) for q = lt + 512 r; column tasks: position p = lt & 127
            const int rb_k1 = lt & 15;
            const int p_col = lt & 127;
            const float2 *src = box + (static_cast<size_t>(t - tb0) * NP + pol) * bplane;
            // RA: 16-point DFTs of the box rows (box columns outside [0, bw) are zero)
#pragma unroll 1
            for (int r = 0; r < 2; ++r) {
                const int q = lt + kF128Block * r;
                const int yl = q >> 3, j = q & 7;
                if (yl < cp.bh) {
                    float2 v[16];
#pragma unroll
                    for (int m = 0; m < 16; ++m) {
                        const int bx = j + 8 * m - cp.x0;
                        v[m] = (bx >= 0 && bx < cp.bw) ? src[static_cast<size_t>(yl) * sd.max_bw + bx]
                                                       : make_float2(0.f, 0.f);
                    }
                    Dft<16>::run(v);
                    const int y = cp.y0 + yl;
#pragma unroll
                    for (int k1 = 0; k1 < 16; ++k1) lds[pl(y, j + 8 * k1)] = v[k1];
                }
            }
            __syncthreads();
            // RB: twiddle and 8-point DFTs along x, in place
#pragma unroll 1
            for (int r = 0; r < 4; ++r) {
                const int q = lt + kF128Block * r;
                const int yl = q >> 4;
                if (yl < cp.bh) {
                    const int y = cp.y0 + yl;
                    float2 v[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) v[j] = lds[pl(y, 8 * rb_k1 + j)];
#pragma unroll
                    for (int j = 1; j < 8; ++j) v[j] = cmul(v[j], twg[j * rb_k1]);
                    Dft<8>::run(v);
#pragma unroll
                    for (int k2 = 0; k2 < 8; ++k2) lds[pl(y, 8 * rb_k1 + k2)] = v[k2];
                }
            }
            __syncthreads();
            // CA: 16-point DFTs along y of column position p_col, rows j' + 8m
            // (zero outside the box), output k1' stored back at row j' + 8 k1'
#pragma unroll 1
            for (int r = 0; r < 2; ++r) {
                const int jc = cgrp + 4 * r;
                float2 v[16];
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    const int y = jc + 8 * m;
                    v[m] = static_cast<unsigned>(y - cp.y0) < static_cast<unsigned>(cp.bh)
                               ? lds[pl(y, p_col)] : make_float2(0.f, 0.f);
                }
                Dft<16>::run(v);
#pragma unroll
                for (int k1 = 0; k1 < 16; ++k1) lds[pl(jc + 8 * k1, p_col)] = v[k1];
            }
            __syncthreads();
            // CB: twiddle and 8-point DFTs along y; output k2' is pixel
            // (ky = k1' + 16 k2', kx = kx_of_p)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k1 = cgrp + 4 * r;
                float2 v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = lds[pl(8 * k1 + j, p_col)];
#pragma unroll
                for (int j = 1; j < 8; ++j) v[j] = cmul(v[j], twg[j * k1]);
                Dft<8>::run(v);
                if constexpr (NP == 1) {
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        acc[r][k][0] = fmaf(v[k].x, v[k].x, fmaf(v[k].y, v[k].y, acc[r][k][0]));
                } else {
                    // pol X pixels of CB task 3 wait in the LDS beyond the plane
                    float2 *hl = lds + PLANE + tid;
                    if (pol == 0) {
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
                            if (r < 3) hold[r][k] = v[k];
                            else hl[k * kF128Block] = v[k];
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < 8; ++k) {
                            const float2 fx = r < 3 ? hold[r][k] : hl[k * kF128Block], fy = v[k];
                            acc[r][k][0] = fmaf(fx.x, fx.x, fmaf(fx.y, fx.y, acc[r][k][0]));
                            acc[r][k][1] = fmaf(fx.x, fy.x, fmaf(fx.y, fy.y, acc[r][k][1]));
                            acc[r][k][2] = fmaf(fx.y, fy.x, fmaf(-fx.x, fy.y, acc[r][k][2]));
                            acc[r][k][3] = fmaf(fy.x, fy.x, fmaf(fy.y, fy.y, acc[r][k][3]));
                        }
                    }
                }
            }
            __syncthreads();
        }
    }
    const int p_col = tid & 127;
    const int kx_of_p = (p_col >> 3) + 16 * (p_col & 7);
    float *out = partials + sd.part_off + (static_cast<size_t>(c) * n_chunks + block) * NQ * PLANE;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int k1 = cgrp + 4 * r;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int pix = (k1 + 16 * k) * N + kx_of_p;
#pragma unroll
            for (int q = 0; q < NQ; ++q) out[q * PLANE + pix] = acc[r][k][q];
        }
    }
}

bool fused128_supported(int n, int max_bw, int max_bh, int n_elem, int n_pol)
{
    // one sample's voltages must fit the gridding kernel's LDS staging
    return n == 128 && max_bw <= 128 && max_bh <= 128 &&
           sizeof(float2) * static_cast<size_t>(n_elem) * n_pol <= kGridBoxLds;
}

// Samples per gridding work-group: as many (up to 8) as fit 64 KB of LDS.
int grid_box_tb(int max_elem, int n_pol)
{
    const size_t per = sizeof(float2) * static_cast<size_t>(max_elem) * n_pol;
    return per * 8 <= kGridBoxLds ? 8 : per * 4 <= kGridBoxLds ? 4 : per * 2 <= kGridBoxLds ? 2 : 1;
}

template <int NP, int VT>
epic_status launch_grid_box_tb(const FusedBatch &b, int tb, int n_time, int chunk, int block,
                               float2 *boxes, hipStream_t stream)
{
    auto pick = [&](auto k, int TB) -> epic_status {
        const int nsub = (chunk + TB - 1) / TB;
        const size_t lds = sizeof(float2) * static_cast<size_t>(TB) * b.max_elem * NP;
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(lds));
        if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
        const int per_xcd = (b.n_items + 7) / 8;
        hipLaunchKernelGGL(k, dim3(8 * per_xcd * nsub), dim3(kGridBoxBlock), lds, stream, b.sds, b.items,
                           b.n_items, n_time, chunk, block, boxes);
        EPIC_HIP_TRY(hipGetLastError());
        return EPIC_OK;
    };
    switch (tb) {
    case 8: return pick(k_grid_box<NP, VT, 8>, 8);
    case 4: return pick(k_grid_box<NP, VT, 4>, 4);
    case 2: return pick(k_grid_box<NP, VT, 2>, 2);
    default: return pick(k_grid_box<NP, VT, 1>, 1);
    }
}

epic_status launch_grid_box(const FusedBatch &b, int n_pol, int n_time, int volt_type, int chunk,
                            int block, float2 *boxes, hipStream_t stream)
{
    const int tb = grid_box_tb(b.max_elem, n_pol);
    KernelTimer timer("grid_box", stream);
    if (n_pol == 2 && volt_type == EPIC_CI8) return launch_grid_box_tb<2, EPIC_CI8>(b, tb, n_time, chunk, block, boxes, stream);
    if (n_pol == 2) return launch_grid_box_tb<2, EPIC_CF32>(b, tb, n_time, chunk, block, boxes, stream);
    if (volt_type == EPIC_CI8) return launch_grid_box_tb<1, EPIC_CI8>(b, tb, n_time, chunk, block, boxes, stream);
    return launch_grid_box_tb<1, EPIC_CF32>(b, tb, n_time, chunk, block, boxes, stream);
}

epic_status launch_fused_fft128_partials(const FusedBatch &b, int n_pol, int n_time, int chunk,
                                         int block, const float2 *boxes, float *partials,
                                         const float2 *twiddles, hipStream_t stream)
{
    auto k = n_pol == 2 ? k_fused_fft128<2> : k_fused_fft128<1>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(kF128Lds));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    KernelTimer timer("fused_fft128_cadence", stream);
    hipLaunchKernelGGL(k, dim3(b.n_items), dim3(kF128Block), kF128Lds, stream, b.sds, b.items,
                       n_time, chunk, block, boxes, partials, twiddles);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

}  // namespace epic
