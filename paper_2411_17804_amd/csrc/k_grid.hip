// k_grid.hip -- gridding of element voltages (Eq. 3, inner bracket) as a
// gather: each cell of the kernel-footprint box sums weight * voltage over
// the (element, weight) taps the plan lists for it, in ascending element
// order, so results are deterministic and no atomics are needed.
#include "fft_lds.hpp"
#include "internal.hpp"
#include "volts.hpp"

namespace epic {

constexpr int kGridCellBlock = 1024;   // grid cells per work-group (4 per thread)
constexpr int kGridTB = 8;             // samples per gridding work-group
constexpr size_t kBandLdsMax = 64 * 1024;  // LDS of one row band (one pass's words)

// One work-group per (channel, block of TB samples, block of CB cells): every
// cell's tap list is read once and applied to the TB samples, whose voltage
// loads are independent of each other.  Writes all n_pol planes of each
// sample's ny x nx grid (zero outside the footprint box).  The cell blocks
// keep the launch wide when a few samples of a large grid are gridded.  A
// thread owns two neighbouring cells of a row and writes them as one 16-byte
// streaming store (the grid is write-once data).
// Two neighbouring cells' values as one 16-byte streaming store.
__device__ __forceinline__ void store_pair(float2 *dst, float2 a, float2 b)
{
    typedef float f4 __attribute__((ext_vector_type(4)));
    __builtin_nontemporal_store(f4{a.x, a.y, b.x, b.y}, reinterpret_cast<f4 *>(dst));
}

template <int NP, int VT, int TB>
__device__ __forceinline__ void grid_cell(const StationDev &sd, const ChanPlan &cp,
                                          const gptr<int32_t> &cs, const Tap *taps, int x, int y,
                                          size_t vrow0, int nts, float2 (&acc)[TB][NP])
{
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
        for (int p = 0; p < NP; ++p) acc[t][p] = make_float2(0.f, 0.f);
    const int bx = x - cp.x0, by = y - cp.y0;
    if (bx < 0 || bx >= cp.bw || by < 0 || by >= cp.bh) return;
    const int cell = by * cp.bw + bx;
    const int k1 = cs[cell + 1];
    for (int k = cs[cell]; k < k1; ++k) {
        const Tap tp = gload<Tap>(taps, k);
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            if (t < nts) {
                float2 e[NP];
                load_volt<NP, VT>(sd.volts, vrow0 + t * static_cast<size_t>(sd.n_elem) + tp.elem, e);
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    acc[t][p].x = fmaf(tp.w, e[p].x, acc[t][p].x);
                    acc[t][p].y = fmaf(tp.w, e[p].y, acc[t][p].y);
                }
            }
        }
    }
}

template <int NP, int VT, int TB>
__global__ __launch_bounds__(256) void k_grid(StationDev sd, int n_time, int t0, int nt,
                                              float2 *__restrict__ grid, int region)
{
    constexpr int CB = kGridCellBlock;
    const int tb = blockIdx.x * TB;
    const int c = blockIdx.y;
    const int nts = min(TB, nt - tb);
    const ChanPlan cp = sd.chan[c];
    const gptr<int32_t> cs = global_ptr<int32_t>(sd.cell_start) + cp.cell_off;
    const Tap *taps = sd.taps + cp.tap_off;
    const int nx = sd.nx, ny = sd.ny;
    const int npix = nx * ny;
    const size_t vrow0 = (static_cast<size_t>(c) * n_time + t0 + tb) * sd.n_elem;
    float2 *out = grid + (static_cast<size_t>(c) * nt + tb) * NP * npix;
    if (region) {
        // the tile region (region 1) or the box's rows (region 2), one cell
        // per thread
        int rx0 = 0, rtx = nx / 16, ry0 = cp.y0, rh = cp.bh;
        if (region == 1) {
            int rty;
            tile_span(cp.x0, cp.bw, nx, rx0, rtx);
            tile_span(cp.y0, cp.bh, ny, ry0, rty);
            rh = 16 * rty;
        }
        const int rw = 16 * rtx, r_end = min(rw * rh, static_cast<int>(blockIdx.z + 1) * CB);
        for (int i = blockIdx.z * CB + threadIdx.x; i < r_end; i += blockDim.x) {
            const int x = rx0 + i % rw, y = ry0 + i / rw;
            float2 a[TB][NP];
            grid_cell<NP, VT, TB>(sd, cp, cs, taps, x, y, vrow0, nts, a);
#pragma unroll
            for (int t = 0; t < TB; ++t)
                if (t < nts)
#pragma unroll
                    for (int p = 0; p < NP; ++p)
                        out[(static_cast<size_t>(t) * NP + p) * npix + y * nx + x] = a[t][p];
        }
        return;
    }
    const int i_end = min(npix, static_cast<int>(blockIdx.z + 1) * CB);
    for (int i = blockIdx.z * CB + 2 * threadIdx.x; i < i_end; i += 2 * blockDim.x) {
        const int y = i / nx, x = i - y * nx;             // x even: x + 1 is on the same row
        float2 a0[TB][NP], a1[TB][NP];
        grid_cell<NP, VT, TB>(sd, cp, cs, taps, x, y, vrow0, nts, a0);
        grid_cell<NP, VT, TB>(sd, cp, cs, taps, x + 1, y, vrow0, nts, a1);
#pragma unroll
        for (int t = 0; t < TB; ++t)
            if (t < nts)
#pragma unroll
                for (int p = 0; p < NP; ++p)
                    store_pair(out + (static_cast<size_t>(t) * NP + p) * npix + i, a0[t][p], a1[t][p]);
    }
}

// Large stations: the TB samples of one element that a tap needs are first
// made contiguous.  k_volts_tb copies samples t0 .. t0+nt-1 into
// tv[c][block][elem][TB][NP] (FP32; samples past nt are 0), one thread per
// (channel, block, element), reading unit-stride rows and writing one
// contiguous run of TB * NP values; k_grid_tb then gathers each tap's TB
// samples from one or two cache lines instead of TB separate rows.
// With slot set (the row-band gather), element e's run goes to position
// slot[c][e] (the elements in order of their nearest row); the reads stay in
// element order, so they remain unit-stride.
template <int NP, int VT, int TB>
__global__ __launch_bounds__(256) void k_volts_tb(const void *__restrict__ volts, int n_elem,
                                                  int n_time, int t0, int nt, int nblk,
                                                  const int32_t *__restrict__ slot,
                                                  float2 *__restrict__ tv)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n_elem) return;
    const int blk = blockIdx.y, c = blockIdx.z;
    const int dst_e = slot ? gload<int32_t>(slot, static_cast<size_t>(c) * n_elem + e) : e;
    float2 v[TB][NP];
#pragma unroll
    for (int t = 0; t < TB; ++t) {
        const int tt = blk * TB + t;
        if (tt < nt) {
            load_volt<NP, VT>(volts, (static_cast<size_t>(c) * n_time + t0 + tt) * n_elem + e, v[t]);
        } else {
#pragma unroll
            for (int p = 0; p < NP; ++p) v[t][p] = make_float2(0.f, 0.f);
        }
    }
    float2 *dst = tv + ((static_cast<size_t>(c) * nblk + blk) * n_elem + dst_e) * TB * NP;
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
        for (int p = 0; p < NP; ++p) dst[t * NP + p] = v[t][p];
}

template <int NP, int TB>
__device__ __forceinline__ void grid_cell_tb(const ChanPlan &cp, const gptr<int32_t> &cs,
                                             const Tap *taps, const float2 *src, int x, int y,
                                             float2 (&acc)[TB][NP])
{
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
        for (int p = 0; p < NP; ++p) acc[t][p] = make_float2(0.f, 0.f);
    const int bx = x - cp.x0, by = y - cp.y0;
    if (bx < 0 || bx >= cp.bw || by < 0 || by >= cp.bh) return;
    const int cell = by * cp.bw + bx;
    const int k1 = cs[cell + 1];
    // taps two at a time: both taps' voltage loads are in flight together and
    // the next pair's tap entries load while this pair is summed; the sum
    // keeps the taps' order (same bits as one tap at a time)
    int k = cs[cell];
    Tap ta = k < k1 ? gload<Tap>(taps, k) : Tap{0, 0.f};
    Tap tb = k + 1 < k1 ? gload<Tap>(taps, k + 1) : Tap{0, 0.f};
    for (; k < k1; k += 2) {
        const bool two = k + 1 < k1;
        const float wa = ta.w, wb = tb.w;
        const float2 *ea = src + static_cast<size_t>(ta.elem) * TB * NP;
        const float2 *eb = src + static_cast<size_t>(tb.elem) * TB * NP;   // element 0 if no second tap
        float2 va[TB * NP], vb[TB * NP];
#pragma unroll
        for (int i = 0; i < TB * NP; ++i) {
            va[i] = gload<float2>(ea, i);
            vb[i] = gload<float2>(eb, i);
        }
        if (k + 2 < k1) ta = gload<Tap>(taps, k + 2);
        if (k + 3 < k1) tb = gload<Tap>(taps, k + 3);
#pragma unroll
        for (int t = 0; t < TB; ++t)
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const float2 v = va[t * NP + p];
                acc[t][p].x = fmaf(wa, v.x, acc[t][p].x);
                acc[t][p].y = fmaf(wa, v.y, acc[t][p].y);
            }
        if (two) {
#pragma unroll
            for (int t = 0; t < TB; ++t)
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    const float2 v = vb[t * NP + p];
                    acc[t][p].x = fmaf(wb, v.x, acc[t][p].x);
                    acc[t][p].y = fmaf(wb, v.y, acc[t][p].y);
                }
        }
    }
}

template <int NP, int TB>
//
// Work items (channel, sample block, cell block of CB cells) on a 1-D grid.
// By default the sample blocks run fastest (blk, channel, cell block).  With
// zfirst set (stations whose sample block of voltages is large next to an
// XCD's L2) the cell blocks run fastest and each XCD takes a contiguous range
// of items (work-group ids go to the 8 XCDs round-robin), so the work-groups
// that gather from one sample block run together on one XCD.
__global__ __launch_bounds__(256) void k_grid_tb(StationDev sd, int nt, int nblk, int n_chan, int nz,
                                                 int CB, int zfirst,
                                                 const float2 *__restrict__ tv,
                                                 float2 *__restrict__ grid, int region)
{
    const int64_t total = static_cast<int64_t>(nblk) * n_chan * nz;
    const int64_t id = blockIdx.x;
    int blk, c, zb;
    if (zfirst) {
        const int64_t item = total % 8 == 0 ? (id % 8) * (total / 8) + id / 8 : id;
        zb = static_cast<int>(item % nz);
        blk = static_cast<int>((item / nz) % nblk);
        c = static_cast<int>(item / nz / nblk);
    } else {
        blk = static_cast<int>(id % nblk);
        c = static_cast<int>((id / nblk) % n_chan);
        zb = static_cast<int>(id / nblk / n_chan);
    }
    const int tb = blk * TB;
    const int nts = min(TB, nt - tb);
    const ChanPlan cp = sd.chan[c];
    const gptr<int32_t> cs = global_ptr<int32_t>(sd.cell_start) + cp.cell_off;
    const Tap *taps = sd.taps + cp.tap_off;
    const int nx = sd.nx, ny = sd.ny;
    const int npix = nx * ny;
    const float2 *src = tv + (static_cast<size_t>(c) * nblk + blk) * sd.n_elem * TB * NP;
    float2 *out = grid + (static_cast<size_t>(c) * nt + tb) * NP * npix;
    // all cells, or the tile region (region 1), or the box's rows (region 2)
    int rx0 = 0, rw = nx, ry0 = 0, n_cells = npix;
    if (region == 1) {
        int rtx, rty;
        tile_span(cp.x0, cp.bw, nx, rx0, rtx);
        tile_span(cp.y0, cp.bh, ny, ry0, rty);
        rw = 16 * rtx;
        n_cells = rw * 16 * rty;
    } else if (region == 2) {
        ry0 = cp.y0;
        n_cells = nx * cp.bh;
    }
    const int i_end = min(n_cells, (zb + 1) * CB);
    // one cell per thread: large stations have many taps per cell, and the
    // wider launch hides their load latency better than paired stores save
    for (int i = zb * CB + threadIdx.x; i < i_end; i += blockDim.x) {
        const int y = ry0 + i / rw, x = rx0 + i % rw;
        float2 acc[TB][NP];
        grid_cell_tb<NP, TB>(cp, cs, taps, src, x, y, acc);
#pragma unroll
        for (int t = 0; t < TB; ++t)
            if (t < nts)
#pragma unroll
                for (int p = 0; p < NP; ++p)
                    out[(static_cast<size_t>(t) * NP + p) * npix + y * nx + x] = acc[t][p];
    }
}

// The row-band gather (stations with row-band tables): one work-group per
// (channel, grid row y) and every sample of the launch.  Every tap of a cell
// in row y comes from an element whose nearest row is within h of y, i.e. one
// of the slots [band_row[y - h], band_row[y + h + 1]); with the sample-blocked
// voltages in slot order (k_volts_tb with the slots) those are one contiguous
// range of runs per sample block.  The work-group takes the samples H at a
// time (a pass): it copies H samples of each of the band's runs into LDS with
// 16-byte loads (the 2h + 1 rows that share a run are neighbouring items on
// one XCD, so it leaves HBM about once), then gathers.  The pass length sets
// the LDS per work-group and so how many share a CU: measured on a 15.6k
// element station, one pass per 8-sample run (one work-group per CU) took
// 2.3x as long as passes of 2 samples (three per CU), and passes of 1 sample
// (eight per CU) drove the fetched bytes up 24x, the L2 no longer holding the
// band's lines between passes.  A thread owns one cell of the row (of each
// group of 256) and keeps its first BT taps in registers for the whole
// launch, so the tap lists are read once; it gathers from LDS, taps in list
// order (the same sums, in the same order, as k_grid_tb).  Cells outside the
// channel's box get zeros (region 0); region 2 launches only the box's rows.
// With NX > 0 (region 2, grids nx = NX <= 256 of the composed FP32 path) the
// work-group also does the row pass of the two-pass transform: the H NP rows
// of a pass go through the same Stockham passes in LDS as k_fft_rows does
// (fft_lds.hpp, the same twiddles, so the same bits) before they are
// written, and the column pass follows directly.
template <int NP, int TB, int H, int NX>
__global__ __launch_bounds__(256) void k_grid_band(StationDev sd, int nt, int nblk, int n_chan, int n_rows,
                                                   const float2 *__restrict__ tv, float2 *__restrict__ grid,
                                                   int region, const float2 *__restrict__ twx)
{
    constexpr int BT = 32;                           // taps per cell held in registers
    constexpr int RUN = TB * NP;                     // float2 per slot and sample block in tv
    constexpr int PART = H * NP;                     // float2 per slot and pass
    constexpr int PW = PART / 2;                     // 16-byte words per slot and pass
    constexpr int NQ = TB / H;                       // passes per sample block
    // a slot's part in LDS is padded by 16 bytes: neighbouring cells read
    // neighbouring slots, and at a stride of a power of two 16-byte words
    // lanes' reads would start on the same banks
    constexpr int SLOT = PART + 2;
    static_assert(PART % 2 == 0 && TB % H == 0, "whole 16-byte words per slot and pass");
    static_assert(NX == 0 || NX <= 256, "one row per work-group pass");
    constexpr int LP = NX + 1;                       // row pitch of the row-pass lines
    extern __shared__ __align__(16) float2 lds[];
    // [H NP][LP] lines of the row pass and NX twiddles, then [slots][SLOT]
    float2 *lines = lds;
    float2 *tw = lines + H * NP * LP;
    float2 *band = NX > 0 ? tw + NX : lds;
    if constexpr (NX > 0)
        for (int i = threadIdx.x; i < NX; i += blockDim.x) tw[i] = twx[i];
    const int64_t total = static_cast<int64_t>(n_chan) * n_rows;
    const int64_t id = blockIdx.x;
    // neighbouring rows of one channel back to back on one XCD (work-group
    // ids go to the 8 XCDs round-robin)
    const int64_t item = total % 8 == 0 ? (id % 8) * (total / 8) + id / 8 : id;
    const int r = static_cast<int>(item % n_rows);
    const int c = static_cast<int>(item / n_rows);
    const ChanPlan cp = sd.chan[c];
    int y = r;
    if (region == 2) {
        if (r >= cp.bh) return;
        y = cp.y0 + r;
    }
    const int nx = sd.nx, ny = sd.ny, h = sd.half_support;
    const int npix = nx * ny;
    const gptr<int32_t> rows = global_ptr<int32_t>(sd.band_row) + static_cast<size_t>(c) * (ny + 1);
    const int s0 = rows[max(0, y - h)], s1 = rows[min(ny, y + h + 1)];
    const gptr<int32_t> cs = global_ptr<int32_t>(sd.cell_start) + cp.cell_off;
    const Tap *taps = sd.band_taps + cp.tap_off;
    const int by = y - cp.y0;
    const int n4 = (s1 - s0) * PW;                   // 16-byte words per pass
    const int nq = nblk * NQ;
    const float2 *base = tv + (static_cast<size_t>(c) * nblk * sd.n_elem + s0) * RUN;
    for (int x0 = 0; x0 < nx; x0 += blockDim.x) {
        const int x = x0 + static_cast<int>(threadIdx.x);
        const int bx = x - cp.x0;
        int k0 = 0, kn = 0;
        if (x < nx && bx >= 0 && bx < cp.bw && by >= 0 && by < cp.bh) {
            const int cell = by * cp.bw + bx;
            k0 = cs[cell];
            kn = cs[cell + 1] - k0;
        }
        // this cell's first BT taps: LDS offset of the slot's part, weight
        int off[BT];
        float wt[BT];
#pragma unroll
        for (int k = 0; k < BT; ++k) {
            const Tap tp = k < kn ? gload<Tap>(taps, k0 + k) : Tap{s0, 0.f};
            off[k] = (tp.elem - s0) * SLOT;
            wt[k] = tp.w;
        }
        for (int q = 0; q < nq; ++q) {
            __syncthreads();   // the previous pass's reads of the LDS are done
            const float2 *src = base + static_cast<size_t>(q / NQ) * sd.n_elem * RUN + (q % NQ) * PART;
            float4 *dst = reinterpret_cast<float4 *>(band);
            for (int i = threadIdx.x; i < n4; i += blockDim.x) {
                const int sl = i / PW, w = i - sl * PW;
                dst[sl * (SLOT / 2) + w] = gload<float4>(src + static_cast<size_t>(sl) * RUN, w);
            }
            __syncthreads();
            float2 acc[H][NP];
#pragma unroll
            for (int t = 0; t < H; ++t)
#pragma unroll
                for (int p = 0; p < NP; ++p) acc[t][p] = make_float2(0.f, 0.f);
            auto add = [&](int o, float w) {
                const float2 *v = band + o;
#pragma unroll
                for (int t = 0; t < H; ++t)
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        const float2 e = v[t * NP + p];
                        acc[t][p].x = fmaf(w, e.x, acc[t][p].x);
                        acc[t][p].y = fmaf(w, e.y, acc[t][p].y);
                    }
            };
#pragma unroll
            for (int k = 0; k < BT; ++k)
                if (k < kn) add(off[k], wt[k]);
            for (int k = BT; k < kn; ++k) {
                const Tap tp = gload<Tap>(taps, k0 + k);
                add((tp.elem - s0) * SLOT, tp.w);
            }
            const int tb = q * H;   // the pass's first sample
            if constexpr (NX > 0) {
                // row pass: the pass's H NP rows through LDS (nx == NX, one
                // chunk of cells), then out
                if (x < NX) {
#pragma unroll
                    for (int t = 0; t < H; ++t)
#pragma unroll
                        for (int p = 0; p < NP; ++p) lines[(t * NP + p) * LP + x] = acc[t][p];
                }
                lds_barrier();
                fft_lines<NX, 256, H * NP, false>(lines, LineMap{H * NP, 0, 0, LP, 1}, H * NP, tw);
                if (x < NX) {
                    float2 *out = grid + (static_cast<size_t>(c) * nt + tb) * NP * npix + static_cast<size_t>(y) * NX + x;
#pragma unroll
                    for (int t = 0; t < H; ++t)
                        if (tb + t < nt)
#pragma unroll
                            for (int p = 0; p < NP; ++p)
                                out[(static_cast<size_t>(t) * NP + p) * npix] = lines[(t * NP + p) * LP + x];
                }
            } else if (x < nx) {
                float2 *out = grid + (static_cast<size_t>(c) * nt + tb) * NP * npix + static_cast<size_t>(y) * nx + x;
#pragma unroll
                for (int t = 0; t < H; ++t)
                    if (tb + t < nt)
#pragma unroll
                        for (int p = 0; p < NP; ++p) out[(static_cast<size_t>(t) * NP + p) * npix] = acc[t][p];
            }
        }
    }
}

template <int NP, int VT, int TB>
__device__ __forceinline__ void grid_cell_pol(const StationDev &sd, const ChanPlan &cp,
                                              const gptr<int32_t> &cs, const Tap *taps,
                                              const gptr<int32_t> &ecell, const float2 *kc, int K,
                                              int x, int y, size_t vrow0, int nts,
                                              float2 (&acc)[TB][NP])
{
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
        for (int p = 0; p < NP; ++p) acc[t][p] = make_float2(0.f, 0.f);
    const int bx = x - cp.x0, by = y - cp.y0;
    if (bx < 0 || bx >= cp.bw || by < 0 || by >= cp.bh) return;
    const int h = (K - 1) / 2, kk = K * K;
    const int cell = by * cp.bw + bx;
    const int k1 = cs[cell + 1];
    for (int k = cs[cell]; k < k1; ++k) {
        const Tap tp = gload<Tap>(taps, k);
        const int ec = ecell[tp.elem];
        const int dx = x - (ec & 0xffff) + h, dy = y - (ec >> 16) + h;
        const float2 *wk = kc + static_cast<size_t>(tp.elem) * NP * NP * kk + dy * K + dx;
        float2 w[NP][NP];
#pragma unroll
        for (int a = 0; a < NP; ++a)
#pragma unroll
            for (int p = 0; p < NP; ++p) w[a][p] = gload<float2>(wk, (a * NP + p) * kk);
#pragma unroll
        for (int t = 0; t < TB; ++t) {
            if (t < nts) {
                float2 e[NP];
                load_volt<NP, VT>(sd.volts, vrow0 + t * static_cast<size_t>(sd.n_elem) + tp.elem, e);
#pragma unroll
                for (int a = 0; a < NP; ++a)
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        // conj(w) e
                        acc[t][a].x = fmaf(w[a][p].x, e[p].x, fmaf(w[a][p].y, e[p].y, acc[t][a].x));
                        acc[t][a].y = fmaf(w[a][p].x, e[p].y, fmaf(-w[a][p].y, e[p].x, acc[t][a].y));
                    }
            }
        }
    }
}

// Full polarimetric gridding (Eq. 3 in general form): every cell sums, over
// its plan taps in order, conj(W_a^{ap}[dy][dx]) E_a^p for both output pols
// a and input pols p, with (dx, dy) the cell's offset in element a's K x K
// footprint.  Same work decomposition as k_grid.
template <int NP, int VT, int TB>
__global__ __launch_bounds__(256) void k_grid_pol(StationDev sd, const int32_t *__restrict__ elem_cell,
                                                  const float2 *__restrict__ kernels, int K,
                                                  int n_time, int t0, int nt,
                                                  float2 *__restrict__ grid)
{
    constexpr int CB = kGridCellBlock;
    const int tb = blockIdx.x * TB;
    const int c = blockIdx.y;
    const int nts = min(TB, nt - tb);
    const ChanPlan cp = sd.chan[c];
    const gptr<int32_t> cs = global_ptr<int32_t>(sd.cell_start) + cp.cell_off;
    const Tap *taps = sd.taps + cp.tap_off;
    const int nx = sd.nx, ny = sd.ny;
    const int npix = nx * ny;
    const gptr<int32_t> ecell = global_ptr<int32_t>(elem_cell) + static_cast<size_t>(c) * sd.n_elem;
    const float2 *kc = kernels + static_cast<size_t>(c) * sd.n_elem * NP * NP * K * K;
    const size_t vrow0 = (static_cast<size_t>(c) * n_time + t0 + tb) * sd.n_elem;
    float2 *out = grid + (static_cast<size_t>(c) * nt + tb) * NP * npix;
    const int i_end = min(npix, static_cast<int>(blockIdx.z + 1) * CB);
    for (int i = blockIdx.z * CB + 2 * threadIdx.x; i < i_end; i += 2 * blockDim.x) {
        const int y = i / nx, x = i - y * nx;             // x even: x + 1 is on the same row
        float2 a0[TB][NP], a1[TB][NP];
        grid_cell_pol<NP, VT, TB>(sd, cp, cs, taps, ecell, kc, K, x, y, vrow0, nts, a0);
        grid_cell_pol<NP, VT, TB>(sd, cp, cs, taps, ecell, kc, K, x + 1, y, vrow0, nts, a1);
#pragma unroll
        for (int t = 0; t < TB; ++t)
            if (t < nts)
#pragma unroll
                for (int p = 0; p < NP; ++p)
                    store_pair(out + (static_cast<size_t>(t) * NP + p) * npix + i, a0[t][p], a1[t][p]);
    }
}

// Cell blocks of cb cells per (channel, sample block): the whole plane, or the
// largest tile region over the channels (a box w cells wide spans
// ceil(w / 16) tiles), or the largest box's rows
static int grid_cell_blocks(const StationDev &sd, int region, int cb = kGridCellBlock)
{
    int cells = sd.nx * sd.ny;
    if (region == 1) {
        int r0, tx, ty;
        tile_span(0, sd.max_bw, sd.nx, r0, tx);
        tile_span(0, sd.max_bh, sd.ny, r0, ty);
        cells = 256 * tx * ty;
    } else if (region == 2) {
        cells = sd.nx * sd.max_bh;
    }
    return (cells + cb - 1) / cb;
}

epic_status launch_grid_pol(const StationDev &sd, const int32_t *elem_cell, const float2 *kernels,
                            int K, int n_pol, int n_chan, int n_time, int volt_type, int t0, int nt,
                            float2 *grid, hipStream_t stream)
{
    constexpr int TB = kGridTB;
    const int npix = sd.nx * sd.ny;
    const dim3 blocks((nt + TB - 1) / TB, n_chan, (npix + kGridCellBlock - 1) / kGridCellBlock),
        threads(256);
    KernelTimer timer("grid_pol", stream);
    if (n_pol == 1 && volt_type == EPIC_CI8)
        hipLaunchKernelGGL((k_grid_pol<1, EPIC_CI8, TB>), blocks, threads, 0, stream, sd, elem_cell, kernels, K, n_time, t0, nt, grid);
    else if (n_pol == 1)
        hipLaunchKernelGGL((k_grid_pol<1, EPIC_CF32, TB>), blocks, threads, 0, stream, sd, elem_cell, kernels, K, n_time, t0, nt, grid);
    else if (volt_type == EPIC_CI8)
        hipLaunchKernelGGL((k_grid_pol<2, EPIC_CI8, TB>), blocks, threads, 0, stream, sd, elem_cell, kernels, K, n_time, t0, nt, grid);
    else
        hipLaunchKernelGGL((k_grid_pol<2, EPIC_CF32, TB>), blocks, threads, 0, stream, sd, elem_cell, kernels, K, n_time, t0, nt, grid);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

epic_status launch_grid_tb(const StationDev &sd, int n_pol, int n_chan, int n_time, int volt_type,
                           int t0, int nt, float2 *tv, float2 *grid, hipStream_t stream, int region,
                           const float2 *row_twiddles, bool *rows_done)
{
    constexpr int TB = kGridTB;
    const int nblk = (nt + TB - 1) / TB;
    if (rows_done) *rows_done = false;
    // the row-band gather where the station has its tables, the gather writes
    // whole rows (the whole plane or the box's rows) and one band's words per
    // pass fit the LDS; with row twiddles (region 2, nx 128 or 256) it does
    // the row pass too
    constexpr int H = 2;   // samples per pass
    const bool rows = row_twiddles && region == 2 && (sd.nx == 128 || sd.nx == 256);
    const size_t rows_lds = rows ? sizeof(float2) * (static_cast<size_t>(H * n_pol) * (sd.nx + 1) + sd.nx) : 0;
    const size_t band_lds = sizeof(float2) * (H * n_pol + 2) * static_cast<size_t>(sd.max_band) + rows_lds;
    const bool banded = sd.band_taps && sd.max_band > 0 && region != 1 && band_lds <= kBandLdsMax;
    const int32_t *slot = banded ? sd.band_slot : nullptr;
    const dim3 tblocks((sd.n_elem + 255) / 256, nblk, n_chan), threads(256);
    {
        KernelTimer timer("volts_tb", stream);
        if (n_pol == 1 && volt_type == EPIC_CI8)
            hipLaunchKernelGGL((k_volts_tb<1, EPIC_CI8, TB>), tblocks, threads, 0, stream, sd.volts, sd.n_elem, n_time, t0, nt, nblk, slot, tv);
        else if (n_pol == 1)
            hipLaunchKernelGGL((k_volts_tb<1, EPIC_CF32, TB>), tblocks, threads, 0, stream, sd.volts, sd.n_elem, n_time, t0, nt, nblk, slot, tv);
        else if (volt_type == EPIC_CI8)
            hipLaunchKernelGGL((k_volts_tb<2, EPIC_CI8, TB>), tblocks, threads, 0, stream, sd.volts, sd.n_elem, n_time, t0, nt, nblk, slot, tv);
        else
            hipLaunchKernelGGL((k_volts_tb<2, EPIC_CF32, TB>), tblocks, threads, 0, stream, sd.volts, sd.n_elem, n_time, t0, nt, nblk, slot, tv);
        EPIC_HIP_TRY(hipGetLastError());
    }
    if (banded) {
        const int n_rows = region == 2 ? sd.max_bh : sd.ny;
        const int64_t n_wg = static_cast<int64_t>(n_chan) * n_rows;
        if (n_wg > 0x7fffffff) return fail(EPIC_ERR_UNSUPPORTED, "gridding launch too large");
        KernelTimer timer("grid_gather", stream);
        auto go = [&](auto kern) -> epic_status {
            EPIC_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             static_cast<int>(band_lds)));
            hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(n_wg)), threads, band_lds, stream, sd, nt, nblk,
                               n_chan, n_rows, tv, grid, region, row_twiddles);
            EPIC_HIP_TRY(hipGetLastError());
            if (rows_done) *rows_done = rows;
            return EPIC_OK;
        };
        if (rows && sd.nx == 256)
            return n_pol == 1 ? go(k_grid_band<1, TB, H, 256>) : go(k_grid_band<2, TB, H, 256>);
        if (rows)
            return n_pol == 1 ? go(k_grid_band<1, TB, H, 128>) : go(k_grid_band<2, TB, H, 128>);
        return n_pol == 1 ? go(k_grid_band<1, TB, H, 0>) : go(k_grid_band<2, TB, H, 0>);
    }
    // a sample block of voltages of 1 MB or more (a quarter of an XCD's L2):
    // one-row cell blocks, run block after block of one sample block per XCD
    const bool zfirst = static_cast<size_t>(sd.n_elem) * TB * n_pol * sizeof(float2) >= (size_t{1} << 20);
    const int cb = zfirst ? 256 : kGridCellBlock;
    const int nz = grid_cell_blocks(sd, region, cb);
    const int64_t n_wg = static_cast<int64_t>(nblk) * n_chan * nz;
    if (n_wg > 0x7fffffff) return fail(EPIC_ERR_UNSUPPORTED, "gridding launch too large");
    const dim3 blocks(static_cast<unsigned>(n_wg));
    KernelTimer timer("grid_gather", stream);
    if (n_pol == 1)
        hipLaunchKernelGGL((k_grid_tb<1, TB>), blocks, threads, 0, stream, sd, nt, nblk, n_chan, nz, cb,
                           zfirst ? 1 : 0, tv, grid, region);
    else
        hipLaunchKernelGGL((k_grid_tb<2, TB>), blocks, threads, 0, stream, sd, nt, nblk, n_chan, nz, cb,
                           zfirst ? 1 : 0, tv, grid, region);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

epic_status launch_grid(const StationDev &sd, int n_pol, int n_chan, int n_time, int volt_type,
                        int t0, int nt, float2 *grid, hipStream_t stream, int region)
{
    constexpr int TB = kGridTB;
    const dim3 blocks((nt + TB - 1) / TB, n_chan, grid_cell_blocks(sd, region)), threads(256);
    KernelTimer timer("grid_gather", stream);
    if (n_pol == 1 && volt_type == EPIC_CI8)
        hipLaunchKernelGGL((k_grid<1, EPIC_CI8, TB>), blocks, threads, 0, stream, sd, n_time, t0, nt, grid, region);
    else if (n_pol == 1)
        hipLaunchKernelGGL((k_grid<1, EPIC_CF32, TB>), blocks, threads, 0, stream, sd, n_time, t0, nt, grid, region);
    else if (volt_type == EPIC_CI8)
        hipLaunchKernelGGL((k_grid<2, EPIC_CI8, TB>), blocks, threads, 0, stream, sd, n_time, t0, nt, grid, region);
    else
        hipLaunchKernelGGL((k_grid<2, EPIC_CF32, TB>), blocks, threads, 0, stream, sd, n_time, t0, nt, grid, region);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

}  // namespace epic
