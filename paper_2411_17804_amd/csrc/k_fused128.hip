// k_fused128.hip -- the FP32 cadence for 128 x 128 grids in one persistent
// kernel.  One 128 x 128 complex plane takes 128 KB of the 160 KB of LDS,
// which leaves no room for a channel's gather taps beside it, so a
// work-group runs its (station, channel) item in blocks of samples, each in
// two phases that take turns over the same LDS:
//
//   grid       the channel's taps and each sample's voltages in LDS, the
//              block's samples gridded (Eq. 3 inner bracket) into their
//              footprint boxes only, [t][pol][max_bh][max_bw], in the
//              work-group's own slice of a device buffer;
//   transform  each sample's boxes transformed (Eq. 3 outer sum) through the
//              LDS plane and the polarisation products (Eq. 2) accumulated in
//              registers; at the block's end its sums go to the FP64 running
//              sums (accum.hpp).
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

#include <algorithm>

namespace epic {

namespace {

constexpr int kF128Block = 512;
constexpr int kGridCells = 24;      // box cells per thread in the grid phase (boxes up to 12288 cells)
constexpr int kGridPre = 16;        // raw voltage words per thread and sample
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

// LDS of the grid phase: one sample's voltages (FP32, padded slots) plus a
// zero element, and the channel's taps as FP32 weights and 16-bit slots.
size_t grid_box_lds(int max_elem, int max_ktaps, int n_pol)
{
    const size_t ntap = static_cast<size_t>(max_elem) * max_ktaps;
    return sizeof(float2) * static_cast<size_t>(gb_slot(max_elem) + 1) * n_pol +
           (sizeof(float) + sizeof(uint16_t)) * ntap;
}

}  // namespace

// The grid phase of samples [t0, t1) of one (station, channel): the channel's
// taps are compacted into LDS (16-bit element slot, FP32 weight) and each
// thread keeps its box cells' tap ranges in registers, so per sample the
// gather reads only LDS: the sample's voltages, staged in LDS as FP32 while
// the next sample's are already on their way into registers.  Cells are
// taken in order of falling tap count (the plan's cell order), so the 64
// lanes of a wave hold cells with about the same number of taps and a group
// of cells needs about as many tap rounds as its cells have taps, not as
// many as the largest tap count among them.
template <int NP, int VT>
__device__ __forceinline__ void grid_phase(const StationDev &sd, const ChanPlan &cp, int c, int n_time, int t0,
                                           int t1, int max_ntap, float2 *lds, float2 *__restrict__ box)
{
    constexpr int BLOCK = kF128Block;
    constexpr int VW = VT == EPIC_CI8 ? 1 : 2 * NP;          // 32-bit words per element
    const int ne = sd.n_elem;
    // element e's voltages sit at slot e + e / 32 (one pad slot every 32
    // elements, so element strides that are multiples of 32, such as the
    // rows of a lattice, do not all land on one LDS bank); slot(ne) is zero
    float2 *vl = lds;                                          // [slot(ne) + 1][NP]
    float *wl = reinterpret_cast<float *>(vl + static_cast<size_t>(gb_slot(ne) + 1) * NP);   // [ntap]
    uint16_t *el = reinterpret_cast<uint16_t *>(wl + max_ntap);                 // [ntap]
    const gptr<int32_t> cs = global_ptr<int32_t>(sd.cell_start) + cp.cell_off;
    const gptr<int32_t> ord = global_ptr<int32_t>(sd.cell_order) + cp.cell_off;
    const Tap *taps = sd.taps + cp.tap_off;
    const int ncell = cp.bw * cp.bh;
    const int ntap = cs[ncell];
    // an opaque copy of the thread index: nothing below is hoisted out of
    // the caller's block loop (where it would hold registers through the
    // transform phase)
    int t_id;
    asm volatile("v_mov_b32 %0, %1" : "=v"(t_id) : "v"(static_cast<int>(threadIdx.x)));
    for (int i = t_id; i < ntap; i += BLOCK) {
        const Tap tp = gload<Tap>(taps, i);
        wl[i] = tp.w;
        el[i] = static_cast<uint16_t>(gb_slot(tp.elem));
    }
    if (t_id < NP) vl[gb_slot(ne) * NP + t_id] = make_float2(0.f, 0.f);
    // this thread's cells, the ones at positions i = tid + BLOCK q (q < nq)
    // of the cell order: first tap << 5 | tap count, and the cell's offset in
    // the box plane, two 16-bit offsets a word
    const int nq = ncell > t_id ? (ncell - 1 - t_id) / BLOCK + 1 : 0;
    uint32_t job[kGridCells];
    uint32_t boff[kGridCells / 2];
#pragma unroll
    for (int q = 0; q < kGridCells; ++q) {
        const int i = t_id + q * BLOCK;
        uint32_t off = 0;
        job[q] = 0;
        if (q < nq) {
            const int cell = ord[i];
            const int k0 = cs[cell];
            job[q] = (static_cast<uint32_t>(k0) << 5) | static_cast<uint32_t>(cs[cell + 1] - k0);
            const int by = cell / cp.bw;
            off = static_cast<uint32_t>(by * sd.max_bw + (cell - by * cp.bw));
        }
        if (q % 2 == 0) boff[q / 2] = off;
        else boff[q / 2] |= off << 16;
    }
    const int plane = sd.max_bh * sd.max_bw;
    const int vwords = ne * VW;
    const gptr<uint32_t> vbase = global_ptr<uint32_t>(sd.volts) + (static_cast<size_t>(c) * n_time + t0) * vwords;
    // the words of one sample are vwords <= kGridPre * BLOCK
    uint32_t pre[kGridPre];
    auto fetch = [&](int t, int tid) {
        const gptr<uint32_t> src = vbase + static_cast<size_t>(t - t0) * vwords;
        // unconditional loads (clamped index): no branches between them, so
        // they all go out together
#pragma unroll
        for (int q = 0; q < kGridPre; ++q) pre[q] = src[min(tid + q * BLOCK, vwords - 1)];
    };
    auto stash = [&](int tid) {
#pragma unroll
        for (int q = 0; q < kGridPre; ++q) {
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
    fetch(t0, t_id);
    for (int t = t0; t < t1; ++t) {
        // an opaque copy of the thread index keeps the compiler from holding
        // every unrolled address live across the sample loop
        int tid;
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(static_cast<int>(threadIdx.x)));
        // the same for the cell words: values derived from them (tap and box
        // addresses) are recomputed per sample instead of being held
#pragma unroll
        for (int q = 0; q < kGridCells; ++q) asm volatile("" : "+v"(job[q]));
#pragma unroll
        for (int q = 0; q < kGridCells / 2; ++q) asm volatile("" : "+v"(boff[q]));
        lds_barrier();          // previous sample's gather done (and taps written)
        stash(tid);
        lds_barrier();
        if (t + 1 < t1) fetch(t + 1, tid);
        float2 *out = box + static_cast<size_t>(t - t0) * NP * plane;
        // cells in groups of G with the tap index outermost, so the G cells'
        // LDS reads are independent of each other and overlap
        constexpr int G = 4;
#pragma unroll
        for (int g0 = 0; g0 < kGridCells; g0 += G) {
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

// One sample of the transform phase.  Per pol: RA (16-point DFTs of the box
// rows, read straight from the box buffer), RB (8-point DFTs along x, in
// place), CA and CB (the same two passes along y for all 128 columns; rows
// outside the box are zero).  CB leaves 32 pixels per thread in registers:
// pol X's are held until pol Y's arrive and the products are accumulated.
template <int NP>
__device__ __forceinline__ void transform_sample(const StationDev &sd, const ChanPlan &cp, const float2 *src0,
                                                 size_t bplane, float2 *lds, const float2 *__restrict__ twg,
                                                 int cgrp, float (&acc)[4][8][NP == 2 ? 4 : 1])
{
    constexpr int N = 128;
    constexpr int PLANE = N * N;
    [[maybe_unused]] float2 hold[3][8];   // pol X pixels of CB tasks 0-2 (two pols)
#pragma unroll 1
    for (int pol = 0; pol < NP; ++pol) {
        // Lane-dependent indices are re-derived from an opaque copy of the
        // thread index each pass, so the compiler recomputes addresses
        // instead of keeping dozens of them live across the sample loop.
        int lt;
        asm volatile("v_mov_b32 %0, %1" : "=v"(lt) : "v"(static_cast<int>(threadIdx.x)));
        // row tasks: RA (y_local = q >> 3, j = q & 7), RB (y_local = q >> 4,
        // k1 = q & 15) for q = lt + 512 r; column tasks: position p = lt & 127
        const int rb_k1 = lt & 15;
        const int p_col = lt & 127;
        const float2 *src = src0 + pol * bplane;
        // RA: 16-point DFTs of the box rows (box columns outside [0, bw) are zero)
#pragma unroll 1
        for (int r = 0; r < 2; ++r) {
            const int q = lt + kF128Block * r;
            const int yl = q >> 3, j = q & 7;
            if (yl < cp.bh) {
                float2 v[16];
                // 32-bit byte offsets from the uniform base: one register per load
                const char *srow = reinterpret_cast<const char *>(src);
#pragma unroll
                for (int m = 0; m < 16; ++m) {
                    const int bx = j + 8 * m - cp.x0;
                    const uint32_t off = static_cast<uint32_t>(yl * sd.max_bw + bx) * 8u;
                    v[m] = (bx >= 0 && bx < cp.bw) ? *reinterpret_cast<const float2 *>(srow + off)
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
                float2 *hl = lds + PLANE + lt;
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
}

// The persistent kernel: (station, channel) items from the work queue, each
// over the whole cadence in blocks of `flush` samples whose sums go to the
// FP64 running sums, each block gridded and transformed `gblock` samples at a
// time (grid phase, then transform phase); the work-group's boxes are its
// slice of `boxes` (wg_floats float2 each: gblock samples x pols x the
// class's largest box).  A small gblock keeps each work-group's boxes in the
// L2 between the two phases.
template <int NP, int VT>
__global__ __launch_bounds__(kF128Block) void k_cadence128(const StationDev *__restrict__ sds, ItemQueue q,
                                                          int n_time, int flush, int gblock, int max_ntap,
                                                          float2 *__restrict__ boxes, size_t wg_floats,
                                                          const float2 *__restrict__ twg)
{
    constexpr int N = 128;
    constexpr int PLANE = N * N;
    constexpr int NQ = NP == 2 ? 4 : 1;
    extern __shared__ __align__(16) float2 lds[];
    // the queue slot: the first word of the hold area, which no item uses
    // while the claim is read
    int *slot = reinterpret_cast<int *>(lds + PLANE);
    float2 *box = boxes + static_cast<size_t>(blockIdx.x) * wg_floats;
    for_each_item(q, slot, [&](const int4 item) {
        const StationDev sd = sds[item.x];
        const int c = item.y;
        const ChanPlan cp = sd.chan[c];
        const ItemSums sums = item_sums(sd.image, NP, PLANE, c);
        const size_t bplane = static_cast<size_t>(sd.max_bh) * sd.max_bw;
        // column tasks: CA j' and CB k1' are (tid >> 7) + 4 r, the same across a wave
        const int cgrp = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 7);
#pragma unroll 1
        for (int t0 = 0; t0 < n_time; t0 += flush) {
            const int t1 = min(n_time, t0 + flush);
            float acc[4][8][NQ];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int k = 0; k < 8; ++k)
#pragma unroll
                    for (int qq = 0; qq < NQ; ++qq) acc[r][k][qq] = 0.f;
#pragma unroll 1
            for (int g0 = t0; g0 < t1; g0 += gblock) {
                const int g1 = min(t1, g0 + gblock);
                grid_phase<NP, VT>(sd, cp, c, n_time, g0, g1, max_ntap, lds, box);
                // the boxes (global memory) are visible to the whole work-group
                // and the LDS is free for the plane
                __syncthreads();
#pragma unroll 1
                for (int t = g0; t < g1; ++t)
                    transform_sample<NP>(sd, cp, box + static_cast<size_t>(t - g0) * NP * bplane, bplane, lds,
                                         twg, cgrp, acc);
            }
            // the block's sums go to the FP64 running sums, a few entries at a time
            int lt;
            asm volatile("v_mov_b32 %0, %1" : "=v"(lt) : "v"(static_cast<int>(threadIdx.x)));
            const int p_col = lt & 127;
            const int kx_of_p = (p_col >> 3) + 16 * (p_col & 7);
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int pix = (cgrp + 4 * r + 16 * k) * N + kx_of_p;
#pragma unroll
                    for (int qq = 0; qq < NQ; ++qq) sums_add(sums, qq, pix, acc[r][k][qq], t0 == 0);
                    asm volatile("" ::: "memory");
                }
        }
        sums_settle();
        const int p_col = threadIdx.x & 127;
        const int kx_of_p = (p_col >> 3) + 16 * (p_col & 7);
        const double inv = 1.0 / static_cast<double>(n_time);
#pragma unroll 1
        for (int r = 0; r < 4; ++r)
#pragma unroll 1
            for (int k = 0; k < 8; ++k) sums_finish<NP>(sums, (cgrp + 4 * r + 16 * k) * N + kx_of_p, inv);
    });
}

bool fused128_supported(int n, int max_bw, int max_bh, int n_elem, int n_pol, int volt_type,
                        int ktaps, int max_cell_taps)
{
    // the grid phase keeps a channel's taps and one sample's voltages in LDS,
    // each thread's cells in registers and one sample's raw voltage words in
    // registers
    const int vw = volt_type == EPIC_CI8 ? 1 : 2 * n_pol;
    const int64_t ntap = static_cast<int64_t>(n_elem) * ktaps;
    return n == 128 && max_bw <= 128 && max_bh <= 128 && gb_slot(n_elem) < 65535 &&
           max_bw * max_bh <= kGridCells * kF128Block && max_cell_taps <= 31 &&
           ntap < (1 << 26) && static_cast<int64_t>(n_elem) * vw <= kGridPre * kF128Block &&
           (volt_type != EPIC_CI8 || n_pol == 2) && grid_box_lds(n_elem, ktaps, n_pol) <= kF128Lds;
}

namespace {

template <int NP, int VT>
const void *cadence128_kernel()
{
    return reinterpret_cast<const void *>(k_cadence128<NP, VT>);
}

const void *kernel_for(int n_pol, int volt_type)
{
    if (n_pol == 2 && volt_type == EPIC_CI8) return cadence128_kernel<2, EPIC_CI8>();
    if (n_pol == 2) return cadence128_kernel<2, EPIC_CF32>();
    if (volt_type == EPIC_CI8) return cadence128_kernel<1, EPIC_CI8>();
    return cadence128_kernel<1, EPIC_CF32>();
}

}  // namespace

int cadence128_grid(int n_pol, int volt_type, int n_items)
{
    return persistent_grid(kernel_for(n_pol, volt_type), kF128Block, kF128Lds, n_items);
}

epic_status launch_cadence128(const FusedBatch &b, int n_pol, int n_time, int volt_type, int flush, int gblock,
                              float2 *boxes, size_t wg_floats, const float2 *twiddles, hipStream_t stream)
{
    const void *k = kernel_for(n_pol, volt_type);
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kF128Lds));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    const int grid = std::min(b.grid, persistent_grid(k, kF128Block, kF128Lds, b.n_items));
    const int max_ntap = b.max_elem * b.max_ktaps;
    KernelTimer timer("fused_fft128_cadence", stream);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kF128Block), kF128Lds, stream, b.sds, b.q, n_time, flush,
                           gblock, max_ntap, boxes, wg_floats, twiddles);
    };
    if (n_pol == 2 && volt_type == EPIC_CI8) go(k_cadence128<2, EPIC_CI8>);
    else if (n_pol == 2) go(k_cadence128<2, EPIC_CF32>);
    else if (volt_type == EPIC_CI8) go(k_cadence128<1, EPIC_CI8>);
    else go(k_cadence128<1, EPIC_CF32>);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

}  // namespace epic
