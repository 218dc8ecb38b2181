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
#include "accum.hpp"
#include "fft_lds.hpp"
#include "internal.hpp"
#include "lds_sync.hpp"
#include "volts.hpp"

namespace epic {

namespace {

constexpr int kGridBoxBlock = 1024;
constexpr int kGridBoxCells = 12;   // box cells per gridding thread (boxes up to 12288 cells)
constexpr int kGridBoxPre = 8;      // raw voltage words per thread and sample
constexpr int kF128Block = 512;
constexpr size_t kF128Lds = sizeof(float2) * (128 * 128 + 8 * kF128Block);   // plane + pol X hold of CB task 3

// LDS position of (row y, column position p) in the 128 x 128 plane.  The LDS
// serves a 64-bit access a group of lanes at a time, and every group must
// touch distinct banks: the XOR of the low 3 bits with bits 3-5 spreads the
// stride-8 reads of pass B, the XOR of bit 0 with bit 6 separates positions
// 64 apart, and a row-dependent XOR (25 (y mod 4), low 6 bits) spreads the
// 2 to 8 rows a group touches in the row passes.  All of it stays inside
// each aligned block of 64 positions, so the column passes (one row, 64
// consecutive positions per wave) are conflict-free too; the choice was
// checked exhaustively against every access pattern of this kernel.
__device__ __forceinline__ int pl(int y, int p)
{
    return y * 128 + (p ^ ((p >> 3) & 7) ^ (((y & 3) * 25) & 63) ^ ((p >> 6) & 1));
}

// LDS slot of element e in the gridding kernel's voltage staging.
__host__ __device__ __forceinline__ int gb_slot(int e) { return e + (e >> 5); }

// LDS of the gridding kernel: one sample's voltages (FP32, padded slots) plus
// a zero element, and the channel's taps as FP32 weights and 16-bit slots.
size_t grid_box_lds(int max_elem, int max_ktaps, int n_pol)
{
    const size_t ntap = static_cast<size_t>(max_elem) * max_ktaps;
    return sizeof(float2) * static_cast<size_t>(gb_slot(max_elem) + 1) * n_pol +
           (sizeof(float) + sizeof(uint16_t)) * ntap;
}

}  // namespace

// One work-group per (station, channel) pair and time block (items: station
// index, channel, 0, box offset in float2); block b covers samples
// [b chunk, min(n_time, (b + 1) chunk)).  The channel's taps are compacted
// into LDS once (16-bit element index, FP32 weight) and each thread keeps its
// box cells' tap ranges in registers, so per sample the gather reads only
// LDS: the voltages of the sample, staged in LDS as FP32 while the next
// sample's are already on their way into registers.  Box cells are written in
// natural order, so the stores are contiguous along the box rows.
template <int NP, int VT>
__global__ __launch_bounds__(kGridBoxBlock) void k_grid_box(const StationDev *__restrict__ sds,
                                                            const int4 *__restrict__ items, int n_time,
                                                            int chunk, int block, int max_ntap,
                                                            float2 *__restrict__ boxes)
{
    constexpr int BLOCK = kGridBoxBlock;
    constexpr int VW = VT == EPIC_CI8 ? 1 : 2 * NP;          // 32-bit words per element
    extern __shared__ float2 lds[];
    const int4 item = items[blockIdx.x];
    const StationDev sd = sds[item.x];
    const int c = item.y;
    const int ne = sd.n_elem;
    // element e's voltages sit at slot e + e / 32 (one pad slot every 32
    // elements, so element strides that are multiples of 32, such as the
    // rows of a lattice, do not all land on one LDS bank); slot(ne) is zero
    float2 *vl = lds;                                          // [slot(ne) + 1][NP]
    float *wl = reinterpret_cast<float *>(vl + static_cast<size_t>(gb_slot(ne) + 1) * NP);   // [ntap]
    uint16_t *el = reinterpret_cast<uint16_t *>(wl + max_ntap);                 // [ntap]
    const ChanPlan cp = sd.chan[c];
    const gptr<int32_t> cs = global_ptr<int32_t>(sd.cell_start) + cp.cell_off;
    const Tap *taps = sd.taps + cp.tap_off;
    const int ncell = cp.bw * cp.bh;
    const int ntap = cs[ncell];
    for (int i = threadIdx.x; i < ntap; i += BLOCK) {
        const Tap tp = gload<Tap>(taps, i);
        wl[i] = tp.w;
        el[i] = static_cast<uint16_t>(gb_slot(tp.elem));
    }
    if (threadIdx.x < NP) vl[gb_slot(ne) * NP + threadIdx.x] = make_float2(0.f, 0.f);
    // this thread's cells i = tid + BLOCK q (q < nq): first tap << 5 | tap
    // count, and the cell's offset in the box plane, two 16-bit offsets a word
    const int nq = ncell > static_cast<int>(threadIdx.x) ? (ncell - 1 - static_cast<int>(threadIdx.x)) / BLOCK + 1 : 0;
    uint32_t job[kGridBoxCells];
    uint32_t boff[kGridBoxCells / 2];
#pragma unroll
    for (int q = 0; q < kGridBoxCells; ++q) {
        const int i = threadIdx.x + q * BLOCK;
        uint32_t off = 0;
        job[q] = 0;
        if (q < nq) {
            const int k0 = cs[i];
            job[q] = (static_cast<uint32_t>(k0) << 5) | static_cast<uint32_t>(cs[i + 1] - k0);
            const int by = i / cp.bw;
            off = static_cast<uint32_t>(by * sd.max_bw + (i - by * cp.bw));
        }
        if (q % 2 == 0) boff[q / 2] = off;
        else boff[q / 2] |= off << 16;
    }
    const int tb0 = block * chunk;
    const int t_end = min(n_time, tb0 + chunk);
    const int plane = sd.max_bh * sd.max_bw;
    const int vwords = ne * VW;
    const gptr<uint32_t> vbase = global_ptr<uint32_t>(sd.volts) +
                            (static_cast<size_t>(c) * n_time + tb0) * vwords;
    // the words of one sample are vwords <= kGridBoxPre * BLOCK
    uint32_t pre[kGridBoxPre];
    auto fetch = [&](int t, int tid) {
        const gptr<uint32_t> src = vbase + static_cast<size_t>(t - tb0) * vwords;
        // unconditional loads (clamped index): no branches between them, so
        // they all go out together
#pragma unroll
        for (int q = 0; q < kGridBoxPre; ++q) pre[q] = src[min(tid + q * BLOCK, vwords - 1)];
    };
    auto stash = [&](int tid) {
#pragma unroll
        for (int q = 0; q < kGridBoxPre; ++q) {
            const int i = tid + q * BLOCK;
            if (i < vwords) {
                const uint32_t w = pre[q];
                if constexpr (VT == EPIC_CI8) {
                    // one word = one element's two complex int8 values
                    const int d = 2 * gb_slot(i);
                    vl[d] = make_float2(static_cast<float>(static_cast<int8_t>(w & 0xff)),
                                        static_cast<float>(static_cast<int8_t>((w >> 8) & 0xff)));
                    vl[d + 1] = make_float2(static_cast<float>(static_cast<int8_t>((w >> 16) & 0xff)),
                                            static_cast<float>(static_cast<int8_t>((w >> 24) & 0xff)));
                } else {
                    // VW words per element
                    reinterpret_cast<uint32_t *>(vl)[gb_slot(i / VW) * VW + i % VW] = w;
                }
            }
        }
    };
    if (tb0 < t_end) fetch(tb0, threadIdx.x);
    for (int t = tb0; t < t_end; ++t) {
        // an opaque copy of the thread index keeps the compiler from holding
        // every unrolled address live across the sample loop
        int tid;
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(static_cast<int>(threadIdx.x)));
        lds_barrier();          // previous sample's gather done (and taps written)
        stash(tid);
        lds_barrier();
        if (t + 1 < t_end) fetch(t + 1, tid);
        float2 *out = boxes + item.w + static_cast<size_t>(t - tb0) * NP * plane;
        // cells in groups of G with the tap index outermost, so the G cells'
        // LDS reads are independent of each other and overlap
        constexpr int G = 4;
#pragma unroll
        for (int g0 = 0; g0 < kGridBoxCells; g0 += G) {
            if (g0 < nq) {
                int k0[G], kn[G], kmax = 0;
#pragma unroll
                for (int u = 0; u < G; ++u) {
                    k0[u] = static_cast<int>(job[g0 + u] >> 5);
                    kn[u] = g0 + u < nq ? static_cast<int>(job[g0 + u] & 31) : 0;
                    kmax = max(kmax, kn[u]);
                }
                float2 a[G][NP];
#pragma unroll
                for (int u = 0; u < G; ++u)
#pragma unroll
                    for (int p = 0; p < NP; ++p) a[u][p] = make_float2(0.f, 0.f);
                // branch-free: a cell past its last tap reads tap 0 and the
                // zero voltage slot (element ne), adding w * 0
                for (int s = 0; s < kmax; ++s) {
                    float w[G];
                    int e[G];
#pragma unroll
                    for (int u = 0; u < G; ++u) {
                        const bool ok = s < kn[u];
                        const int kk = ok ? k0[u] + s : 0;
                        w[u] = wl[kk];
                        e[u] = ok ? static_cast<int>(el[kk]) : gb_slot(ne);
                    }
#pragma unroll
                    for (int u = 0; u < G; ++u)
#pragma unroll
                        for (int p = 0; p < NP; ++p) {
                            const float2 v = vl[e[u] * NP + p];
                            a[u][p].x = fmaf(w[u], v.x, a[u][p].x);
                            a[u][p].y = fmaf(w[u], v.y, a[u][p].y);
                        }
                }
#pragma unroll
                for (int u = 0; u < G; ++u) {
                    if (g0 + u < nq) {
                        const int q = g0 + u;
                        const int o = static_cast<int>((boff[q / 2] >> (16 * (q % 2))) & 0xffff);
#pragma unroll
                        for (int p = 0; p < NP; ++p) out[p * plane + o] = a[u][p];
                    }
                }
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
                                                             int flush,
                                                             const float2 *__restrict__ boxes,
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
    const int tb0 = block * chunk;
    const int t_end = min(n_time, tb0 + chunk);
    const ItemSums sums = item_sums(sd.image, NP, PLANE, c);
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
            lds_barrier();
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
            lds_barrier();
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
            lds_barrier();
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
            lds_barrier();
        }
        // a block of samples ends (or this launch's time block does): its
        // sums go to the FP64 running sums, a few entries at a time
        if (block_ends(t, n_time, flush) || t + 1 == t_end) {
            int lt;
            asm volatile("v_mov_b32 %0, %1" : "=v"(lt) : "v"(tid));
            const int p_col = lt & 127;
            const int kx_of_p = (p_col >> 3) + 16 * (p_col & 7);
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int pix = (cgrp + 4 * r + 16 * k) * N + kx_of_p;
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        sums_add(sums, q, pix, acc[r][k][q], t < flush);
                        acc[r][k][q] = 0.f;
                    }
                    asm volatile("" ::: "memory");
                }
        }
    }
    // the last time block turns the running sums into the mean products
    if (t_end == n_time) {
        sums_settle();
        const int p_col = tid & 127;
        const int kx_of_p = (p_col >> 3) + 16 * (p_col & 7);
        const double inv = 1.0 / static_cast<double>(n_time);
#pragma unroll 1
        for (int r = 0; r < 4; ++r)
#pragma unroll 1
            for (int k = 0; k < 8; ++k) sums_finish<NP>(sums, (cgrp + 4 * r + 16 * k) * N + kx_of_p, inv);
    }
}

bool fused128_supported(int n, int max_bw, int max_bh, int n_elem, int n_pol, int volt_type,
                        int ktaps, int max_cell_taps)
{
    // the gridding kernel keeps a channel's taps and one sample's voltages in
    // LDS, each thread's cells in registers and one sample's raw voltage
    // words in registers
    const int vw = volt_type == EPIC_CI8 ? 1 : 2 * n_pol;
    const int64_t ntap = static_cast<int64_t>(n_elem) * ktaps;
    return n == 128 && max_bw <= 128 && max_bh <= 128 && gb_slot(n_elem) < 65535 &&
           max_bw * max_bh <= kGridBoxCells * kGridBoxBlock && max_cell_taps <= 31 &&
           ntap < (1 << 26) && static_cast<int64_t>(n_elem) * vw <= kGridBoxPre * kGridBoxBlock &&
           (volt_type != EPIC_CI8 || n_pol == 2) &&
           grid_box_lds(n_elem, ktaps, n_pol) <= 160 * 1024;
}

epic_status launch_grid_box(const FusedBatch &b, int n_pol, int n_time, int volt_type, int chunk,
                            int block, float2 *boxes, hipStream_t stream)
{
    const int max_ntap = b.max_elem * b.max_ktaps;
    const size_t lds = grid_box_lds(b.max_elem, b.max_ktaps, n_pol);
    auto go = [&](auto k) -> epic_status {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           static_cast<int>(lds));
        if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
        hipLaunchKernelGGL(k, dim3(b.n_items), dim3(kGridBoxBlock), lds, stream, b.sds, b.items,
                           n_time, chunk, block, max_ntap, boxes);
        EPIC_HIP_TRY(hipGetLastError());
        return EPIC_OK;
    };
    KernelTimer timer("grid_box", stream);
    if (n_pol == 2 && volt_type == EPIC_CI8) return go(k_grid_box<2, EPIC_CI8>);
    if (n_pol == 2) return go(k_grid_box<2, EPIC_CF32>);
    if (volt_type == EPIC_CI8) return go(k_grid_box<1, EPIC_CI8>);
    return go(k_grid_box<1, EPIC_CF32>);
}

epic_status launch_fused_fft128(const FusedBatch &b, int n_pol, int n_time, int chunk, int block,
                                int flush, const float2 *boxes,
                                         const float2 *twiddles, hipStream_t stream)
{
    auto k = n_pol == 2 ? k_fused_fft128<2> : k_fused_fft128<1>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(kF128Lds));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    KernelTimer timer("fused_fft128_cadence", stream);
    hipLaunchKernelGGL(k, dim3(b.n_items), dim3(kF128Block), kF128Lds, stream, b.sds, b.items,
                       n_time, chunk, block, flush, boxes, twiddles);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

}  // namespace epic
