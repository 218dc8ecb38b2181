// k_fused.hip -- the whole FP32 cadence for square grids up to 64 x 64 in one
// kernel: for each sample, grid the voltages (Eq. 3 inner bracket) into LDS,
// transform rows then columns in LDS (Eq. 3 outer sum), and accumulate the
// polarisation products (Eq. 2) in registers.  One work-group images one
// (station, channel) over the whole cadence (items from the work queue),
// adding the products of blocks of samples to FP64 running sums kept in the
// image buffer, and finally writes the mean products (accum.hpp).
//
// Only rows inside the kernel-footprint box carry data, so the row transforms
// run on those rows alone and the first column pass treats the other rows as
// zero.
#include "accum.hpp"
#include "fft_lds.hpp"
#include "internal.hpp"
#include "lds_sync.hpp"
#include "volts.hpp"

namespace epic {

template <int N> struct FusedShape;
template <> struct FusedShape<16> { static constexpr int BLOCK = 128; };
template <> struct FusedShape<32> { static constexpr int BLOCK = 256; };
template <> struct FusedShape<64> { static constexpr int BLOCK = 512; };

template <int N, int NP, int VT>
__global__ __launch_bounds__(FusedShape<N>::BLOCK) void k_fused_fft(const StationDev *__restrict__ sds,
                                                                    ItemQueue q,
                                                                    int n_time, int flush,
                                                                    const float2 *__restrict__ twg)
{
    constexpr int BLOCK = FusedShape<N>::BLOCK;
    constexpr int P = N + 1;                 // row pitch (float2) in LDS
    constexpr int PLANE = N * P;
    constexpr int NPIX = N * N;
    constexpr int NQ = NP == 2 ? 4 : 1;
    constexpr int PXT = (NPIX + BLOCK - 1) / BLOCK;   // pixels per thread
    extern __shared__ __align__(16) float2 lds[];
    float2 *buf = lds;                       // [NP][N][P]
    float2 *tw = lds + NP * PLANE;           // [N]

    for_each_item(q, [&](const int4 item) {
        const StationDev sd = sds[item.x];
        const int c = item.y;
        const ChanPlan cp = sd.chan[c];
        const ItemSums sums = item_sums(sd.image, NP, NPIX, c);
        const gptr<int32_t> cs = global_ptr<int32_t>(sd.cell_start) + cp.cell_off;
        const Tap *taps = sd.taps + cp.tap_off;

        for (int i = threadIdx.x; i < N; i += BLOCK) tw[i] = twg[i];

        float acc[PXT][NQ];
#pragma unroll
        for (int i = 0; i < PXT; ++i)
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[i][q] = 0.f;

        const int rows = cp.bh;
        const int row_cells = rows * N;
        for (int t = 0; t < n_time; ++t) {
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
                        const Tap tp = gload<Tap>(taps, k);
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
            lds_barrier();
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
            // a block of samples ends: its sums go to the FP64 running sums
            if (block_ends(t, n_time, flush)) {
#pragma unroll
                for (int i = 0; i < PXT; ++i) {
                    const int k = threadIdx.x + i * BLOCK;
                    if (NPIX % BLOCK == 0 || k < NPIX)
#pragma unroll
                        for (int q = 0; q < NQ; ++q) {
                            sums_add(sums, q, k, acc[i][q], t < flush);
                            acc[i][q] = 0.f;
                        }
                }
            }
            lds_barrier();
        }
        // the mean products of the pixels this thread owns (all components)
        sums_settle();
        const double inv = 1.0 / static_cast<double>(n_time);
#pragma unroll
        for (int i = 0; i < PXT; ++i) {
            const int k = threadIdx.x + i * BLOCK;
            if (NPIX % BLOCK == 0 || k < NPIX) sums_finish<NP>(sums, k, inv);
        }
    });
}

// ---------------------------------------------------------------------------
// 64 x 64 grids: the 8 x 8 decomposition of each 64-point transform is kept in
// registers.  Per sample, in the Stockham notation of fft_lds.hpp:
//   R1  thread (row y, j) grids cells x = j + 8m straight into registers and
//       does the first radix-8 pass; outputs land at x = 8j + k1;
//   R2  the same thread reads x = j + 8r, twiddles by exp(+2 pi i r j / 64),
//       does the second pass in place (outputs at j + 8k);
//   C1, C2  the same two passes along y for column kx (rows outside the
//       footprint are zero), and C2 leaves pixel (ky = j + 8k, kx) of both
//       pols in the registers of one thread, which squares and accumulates.
// LDS holds one 64 x 64 plane per pol under an XOR swizzle of the low five bits
// of x that keys on y, chosen so that every access pattern above spreads a
// wave's 64 lanes evenly over the banks (row tasks of a wave are 8 rows
// apart).  The next sample's voltages are prefetched into registers and
// staged in a second LDS buffer while the current sample is transformed.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int sw64(int y, int x)
{
    const int t = (y ^ (y >> 3)) & 7;
    return y * 64 + (x ^ (t | ((t & 3) << 3)));
}

constexpr int kFused64Block = 512;
constexpr int kFused64Rounds = 8;     // gather rounds: box cells <= 8 * 512
constexpr int kFused64Prefetch = 4;   // raw voltage words per thread per sample (<= 8 KB/sample)
// dynamic LDS a work-group may take: 160 KB less room for the static LDS of
// the kernels (the work-queue slot, small reduction arrays)
constexpr size_t kLdsBytes = 160 * 1024 - 256;

// LDS of the 64 x 64 kernel: transform planes, the gathered footprint box,
// two voltage buffers (as float), the channel's gather taps.
inline size_t fused64_lds_bytes(int np, int max_elem, int ktaps, int max_cells)
{
    return sizeof(float2) * np * 64 * 64 + sizeof(float2) * np * max_cells +
           sizeof(float2) * 2 * np * static_cast<size_t>(max_elem) +
           sizeof(Tap) * static_cast<size_t>(max_elem) * ktaps;
}

template <int NP, int VT>
__global__ __launch_bounds__(kFused64Block) void k_fused_fft64(const StationDev *__restrict__ sds,
                                                               ItemQueue q,
                                                               int n_time, int flush,
                                                               const float2 *__restrict__ twg,
                                                               int max_elem, int max_cells)
{
    constexpr int PLANE = 64 * 64;
    constexpr int NQ = NP == 2 ? 4 : 1;
    constexpr int BLOCK = kFused64Block;
    extern __shared__ __align__(16) float2 lds[];
    float2 *buf = lds;                                   // [NP][PLANE], swizzled
    float2 *gb = buf + NP * PLANE;                       // [NP][max_cells] gathered box
    float2 *vf = gb + NP * max_cells;                    // [2][max_elem][NP] voltages
    Tap *taps_l = reinterpret_cast<Tap *>(vf + 2 * NP * max_elem);

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int j = lane & 7;                 // butterfly index in every pass
    const int yl = wv + 8 * (lane >> 3);    // row task (rows of a wave are 8 apart)
    const int kx = tid >> 3;                // column task
    for_each_item(q, [&](const int4 item) {
        const StationDev sd = sds[item.x];
        const int c = item.y;
        const int vwords = sd.n_elem * NP * (VT == EPIC_CI8 ? 2 : 8) / 4;
        const int t_begin = 0, t_end = n_time;
        const ItemSums sums = item_sums(sd.image, NP, PLANE, c);
        const ChanPlan cp = sd.chan[c];
        const bool row_active = yl < cp.bh;
        const int y = cp.y0 + yl;
        const int ncell = cp.bw * cp.bh;

        // gather jobs of this thread: box cells in descending tap-count order,
        // packed as cell << 20 | count << 16 | first tap
        uint32_t job[kFused64Rounds];
        {
            const gptr<int32_t> cs = global_ptr<int32_t>(sd.cell_start) + cp.cell_off;
            const gptr<int32_t> ord = global_ptr<int32_t>(sd.cell_order) + cp.cell_off;
            const Tap *taps = sd.taps + cp.tap_off;
            const int ntap = cs[ncell];
            for (int i = tid; i < ntap; i += BLOCK) taps_l[i] = gload<Tap>(taps, i);
#pragma unroll
            for (int q = 0; q < kFused64Rounds; ++q) {
                const int i = tid + q * BLOCK;
                job[q] = 0xffffffffu;
                if (i < ncell) {
                    const int cell = ord[i];
                    const int k0 = cs[cell];
                    job[q] = (static_cast<uint32_t>(cell) << 20) |
                             (static_cast<uint32_t>(cs[cell + 1] - k0) << 16) | static_cast<uint32_t>(k0);
                }
            }
        }

        float2 tw[8];
#pragma unroll
        for (int r = 1; r < 8; ++r) tw[r] = twg[r * j];

        // swizzled LDS addresses (see sw64): rows of this thread's row task ...
        const int tr = (y ^ (y >> 3)) & 7;
        const int sr = tr | ((tr & 3) << 3);
        const int bt = y * 64 + ((8 * j) ^ (sr & 0x18)) + tr;   // x = 8j + k  -> bt ^ k
        const int bj = y * 64 + (j ^ tr) + (sr & 0x18);          // x = j + 8r  -> bj ^ 8r
        // ... and of this thread's column task: rows j + 8m -> cm[m] + 512 m,
        // rows 8j + k -> cm[k] + 448 j + 64 k
        int cm[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int t = (j ^ m) & 7;
            cm[m] = j * 64 + (kx ^ (t | ((t & 3) << 3)));
        }
        const int dj = 448 * j;

        // voltages of sample t as float pairs in vf[buffer]
        auto stash = [&](int buffer, int i, uint32_t w) {
            float2 *dst = vf + buffer * NP * max_elem;
            if constexpr (VT == EPIC_CI8) {
                dst[2 * i] = make_float2(static_cast<float>(static_cast<int8_t>(w & 0xff)),
                                         static_cast<float>(static_cast<int8_t>((w >> 8) & 0xff)));
                dst[2 * i + 1] = make_float2(static_cast<float>(static_cast<int8_t>((w >> 16) & 0xff)),
                                             static_cast<float>(static_cast<int8_t>((w >> 24) & 0xff)));
            } else {
                reinterpret_cast<uint32_t *>(dst)[i] = w;
            }
        };
        const gptr<uint32_t> vsrc = global_ptr<uint32_t>(sd.volts) +
                               static_cast<size_t>(c) * n_time * vwords;
        for (int i = tid; i < vwords; i += BLOCK) stash(0, i, vsrc[static_cast<size_t>(t_begin) * vwords + i]);

        float acc[8][NQ];
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int q = 0; q < NQ; ++q) acc[k][q] = 0.f;
        lds_barrier();

        int cur = 0;
        for (int t = t_begin; t < t_end; ++t) {
            const bool has_next = t + 1 < t_end;
            uint32_t pre[kFused64Prefetch];
            if (has_next) {
#pragma unroll
                for (int q = 0; q < kFused64Prefetch; ++q) {
                    const int i = tid + q * BLOCK;
                    if (i < vwords) pre[q] = vsrc[static_cast<size_t>(t + 1) * vwords + i];
                }
            }
            // G: grid the footprint box (Eq. 3 inner bracket), one cell per job
            {
                const float2 *vcur = vf + cur * NP * max_elem;
#pragma unroll
                for (int q = 0; q < kFused64Rounds; ++q) {
                    if (job[q] != 0xffffffffu) {
                        const int cell = job[q] >> 20, kn = (job[q] >> 16) & 15, k0 = job[q] & 0xffff;
                        float2 a[NP];
#pragma unroll
                        for (int p = 0; p < NP; ++p) a[p] = make_float2(0.f, 0.f);
                        for (int s = 0; s < kn; ++s) {
                            const Tap tp = taps_l[k0 + s];
#pragma unroll
                            for (int p = 0; p < NP; ++p) {
                                const float2 e = vcur[tp.elem * NP + p];
                                a[p].x = fmaf(tp.w, e.x, a[p].x);
                                a[p].y = fmaf(tp.w, e.y, a[p].y);
                            }
                        }
#pragma unroll
                        for (int p = 0; p < NP; ++p) gb[p * max_cells + cell] = a[p];
                    }
                }
            }
            if (has_next) {
#pragma unroll
                for (int q = 0; q < kFused64Prefetch; ++q) {
                    const int i = tid + q * BLOCK;
                    if (i < vwords) stash(cur ^ 1, i, pre[q]);
                }
            }
            lds_barrier();
            // R1: first radix-8 pass along x on the box rows (cells outside the box are 0)
            if (row_active) {
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    float2 v[8];
#pragma unroll
                    for (int m = 0; m < 8; ++m) {
                        const int bx = j + 8 * m - cp.x0;
                        v[m] = (bx >= 0 && bx < cp.bw) ? gb[p * max_cells + yl * cp.bw + bx]
                                                       : make_float2(0.f, 0.f);
                    }
                    Dft<8>::run(v);
#pragma unroll
                    for (int k = 0; k < 8; ++k) buf[p * PLANE + (bt ^ k)] = v[k];
                }
            }
            lds_barrier();
            // R2: second radix-8 pass along x, in place
            if (row_active) {
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    float2 v[8];
#pragma unroll
                    for (int r = 0; r < 8; ++r) v[r] = buf[p * PLANE + (bj ^ (8 * r))];
#pragma unroll
                    for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], tw[r]);
                    Dft<8>::run(v);
#pragma unroll
                    for (int r = 0; r < 8; ++r) buf[p * PLANE + (bj ^ (8 * r))] = v[r];
                }
            }
            lds_barrier();
            // C1: first radix-8 pass along y for column kx (rows outside the box are 0)
            {
                float2 v[NP][8];
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int yy = j + 8 * m;
                    const bool in = yy >= cp.y0 && yy < cp.y0 + cp.bh;
#pragma unroll
                    for (int p = 0; p < NP; ++p)
                        v[p][m] = in ? buf[p * PLANE + cm[m] + 512 * m] : make_float2(0.f, 0.f);
                }
#pragma unroll
                for (int p = 0; p < NP; ++p) Dft<8>::run(v[p]);
                lds_barrier();
#pragma unroll
                for (int p = 0; p < NP; ++p)
#pragma unroll
                    for (int k = 0; k < 8; ++k) buf[p * PLANE + cm[k] + dj + 64 * k] = v[p][k];
            }
            lds_barrier();
            // C2: second pass along y; pixel (ky = j + 8k, kx) of both pols is here
            {
                float2 v[NP][8];
#pragma unroll
                for (int p = 0; p < NP; ++p) {
#pragma unroll
                    for (int r = 0; r < 8; ++r) v[p][r] = buf[p * PLANE + cm[r] + 512 * r];
#pragma unroll
                    for (int r = 1; r < 8; ++r) v[p][r] = cmul(v[p][r], tw[r]);
                    Dft<8>::run(v[p]);
                }
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const float2 fx = v[0][k];
                    acc[k][0] = fmaf(fx.x, fx.x, fmaf(fx.y, fx.y, acc[k][0]));
                    if constexpr (NP == 2) {
                        const float2 fy = v[1][k];
                        acc[k][1] = fmaf(fx.x, fy.x, fmaf(fx.y, fy.y, acc[k][1]));
                        acc[k][2] = fmaf(fx.y, fy.x, fmaf(-fx.x, fy.y, acc[k][2]));
                        acc[k][3] = fmaf(fy.x, fy.x, fmaf(fy.y, fy.y, acc[k][3]));
                    }
                }
                // a block of samples ends: its sums go to the FP64 running sums
                if (block_ends(t, n_time, flush)) {
                    int px0;   // opaque: keeps the addresses from being hoisted
                    asm volatile("v_mov_b32 %0, %1" : "=v"(px0) : "v"(j * 64 + kx));
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
#pragma unroll
                        for (int q = 0; q < NQ; ++q) {
                            sums_add(sums, q, px0 + 512 * k, acc[k][q], t < flush);
                            acc[k][q] = 0.f;
                        }
                        asm volatile("" ::: "memory");
                    }
                }
            }
            lds_barrier();
            cur ^= 1;
        }
        sums_settle();
        const double inv = 1.0 / static_cast<double>(n_time);
#pragma unroll
        for (int k = 0; k < 8; ++k) sums_finish<NP>(sums, (j + 8 * k) * 64 + kx, inv);
    });
}

// Two-pol form of the 64 x 64 kernel with 1024 threads: threads 0-511 carry
// pol X and threads 512-1023 pol Y through the same passes as above (one
// radix-8 butterfly of one pol per thread and pass).  That halves the
// registers of a thread and doubles the waves that hide LDS latency.  After
// the last column pass both halves leave their pixels in LDS and each picks up
// the other pol's, so that each forms and accumulates two of the four real
// product components.  A wave's row tasks are 8 adjacent rows aligned to 8 (the swizzle
// keeps those conflict-free too), so waves whose rows miss the footprint box
// skip the row passes.
//
// The gather writes each footprint cell straight into its pol's plane, at
// position x ^ 8 (y mod 8) of row y, so that the first row pass (lane j of
// a row reads x = j + 8m for m = 0..7, eight rows per wave) touches every
// bank pair once per read.  That pass then overwrites the same row in place:
// a row is read and written by the 8 lanes of one wave, whose LDS reads all
// complete before its first write (every output needs all eight inputs).
// Cells outside the box are never written; the row pass reads them as zero.
constexpr int kFused64x2Block = 1024;

__device__ __forceinline__ int gather_slot64(int y, int x) { return y * 64 + (x ^ ((y & 7) << 3)); }

template <int VT>
__global__ __launch_bounds__(kFused64x2Block) void k_fused_fft64x2(const StationDev *__restrict__ sds,
                                                                   ItemQueue q,
                                                                   int n_time, int flush,
                                                                   const float2 *__restrict__ twg,
                                                                   int max_elem, int max_cells)
{
    constexpr int NP = 2;
    constexpr int PLANE = 64 * 64;
    constexpr int BLOCK = kFused64x2Block;
    constexpr int ROUNDS = kFused64Rounds * kFused64Block / BLOCK;
    constexpr int PREFETCH = kFused64Prefetch * kFused64Block / BLOCK;
    extern __shared__ __align__(16) float2 lds[];
    float2 *buf = lds;                                   // [2][PLANE], swizzled
    float2 *vf = buf + NP * PLANE;                       // [2][max_elem][2] voltages
    Tap *taps_l = reinterpret_cast<Tap *>(vf + 2 * NP * max_elem);
    uint32_t *jobs = reinterpret_cast<uint32_t *>(taps_l + max_elem * 9);   // [max_cells]

    for_each_item(q, [&](const int4 item) {
        // thread indices from an opaque copy of the thread index, so that the
        // compiler derives them per item instead of keeping them (and values
        // built from them) live across the item loop
        int tid;
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(static_cast<int>(threadIdx.x)));
        // pol of this thread (the same across a wave, which the compiler learns
        // from readfirstlane: pol-dependent choices become scalar branches)
        const int pol = __builtin_amdgcn_readfirstlane(tid >> 9), tp5 = tid & 511;
        const int lane = tp5 & 63, wv = tp5 >> 6;
        const int j = lane & 7;
        const int y = 8 * wv + (lane >> 3);                  // row task: a wave owns 8 adjacent rows
        const int kx = tp5 >> 3;
        const StationDev sd = sds[item.x];
        const int c = item.y;
        const int vwords = sd.n_elem * NP * (VT == EPIC_CI8 ? 2 : 8) / 4;
        const int t_begin = 0, t_end = n_time;
        const ItemSums sums = item_sums(sd.image, NP, PLANE, c);
        const ChanPlan cp = sd.chan[c];
        const int yl = y - cp.y0;
        const bool row_active = yl >= 0 && yl < cp.bh;       // waves wholly outside the box skip R1, R2
        const int ncell = cp.bw * cp.bh;
        float2 *plane = buf + pol * PLANE;

        // gather jobs in LDS (box cells in descending tap-count order): all
        // 1024 threads grid both pols of one cell each round
        {
            const gptr<int32_t> cs = global_ptr<int32_t>(sd.cell_start) + cp.cell_off;
            const gptr<int32_t> ord = global_ptr<int32_t>(sd.cell_order) + cp.cell_off;
            const Tap *taps = sd.taps + cp.tap_off;
            const int ntap = cs[ncell];
            for (int i = tid; i < ntap; i += BLOCK) taps_l[i] = gload<Tap>(taps, i);
            for (int i = tid; i < ncell; i += BLOCK) {
                const int cell = ord[i];
                const int k0 = cs[cell];
                const int by = cell / cp.bw;
                const int slot = gather_slot64(cp.y0 + by, cp.x0 + (cell - by * cp.bw));   // 12 bits
                jobs[i] = (static_cast<uint32_t>(slot) << 20) |
                          (static_cast<uint32_t>(cs[cell + 1] - k0) << 16) | static_cast<uint32_t>(k0);
            }
        }

        float2 tw[8];
#pragma unroll
        for (int r = 1; r < 8; ++r) tw[r] = twg[r * j];
        const int tr = (y ^ (y >> 3)) & 7;
        const int sr = tr | ((tr & 3) << 3);
        const int bt = y * 64 + ((8 * j) ^ (sr & 0x18)) + tr;
        const int bj = y * 64 + (j ^ tr) + (sr & 0x18);
        int cm[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int t = (j ^ m) & 7;
            cm[m] = j * 64 + (kx ^ (t | ((t & 3) << 3)));
        }
        const int dj = 448 * j;

        auto stash = [&](int buffer, int i, uint32_t w) {
            float2 *dst = vf + buffer * NP * max_elem;
            if constexpr (VT == EPIC_CI8) {
                dst[2 * i] = make_float2(static_cast<float>(static_cast<int8_t>(w & 0xff)),
                                         static_cast<float>(static_cast<int8_t>((w >> 8) & 0xff)));
                dst[2 * i + 1] = make_float2(static_cast<float>(static_cast<int8_t>((w >> 16) & 0xff)),
                                             static_cast<float>(static_cast<int8_t>((w >> 24) & 0xff)));
            } else {
                reinterpret_cast<uint32_t *>(dst)[i] = w;
            }
        };
        const gptr<uint32_t> vsrc = global_ptr<uint32_t>(sd.volts) +
                               static_cast<size_t>(c) * n_time * vwords;
        for (int i = tid; i < vwords; i += BLOCK) stash(0, i, vsrc[static_cast<size_t>(t_begin) * vwords + i]);

        float acc[8][2];
#pragma unroll
        for (int k = 0; k < 8; ++k)
#pragma unroll
            for (int q = 0; q < 2; ++q) acc[k][q] = 0.f;

        int cur = 0;
        for (int t = t_begin; t < t_end; ++t) {
            const bool has_next = t + 1 < t_end;
            uint32_t pre[PREFETCH];
            if (has_next) {
#pragma unroll
                for (int q = 0; q < PREFETCH; ++q) {
                    const int i = tid + q * BLOCK;
                    if (i < vwords) pre[q] = vsrc[static_cast<size_t>(t + 1) * vwords + i];
                }
            }
            // the previous sample's products have read both planes (and, on the
            // first sample, the taps and voltages are in place)
            lds_barrier();
            // G: grid the footprint box (Eq. 3 inner bracket) into both planes; a
            // cell's taps serve both pols
            {
                const float2 *vcur = vf + cur * NP * max_elem;
#pragma unroll
                for (int q = 0; q < ROUNDS; ++q) {
                    const int i = tid + q * BLOCK;
                    if (i < ncell) {
                        const uint32_t job = jobs[i];
                        const int slot = job >> 20, kn = (job >> 16) & 15, k0 = job & 0xffff;
                        float2 a0 = make_float2(0.f, 0.f), a1 = a0;
                        for (int s = 0; s < kn; ++s) {
                            const Tap tp = taps_l[k0 + s];
                            const float2 e0 = vcur[tp.elem * 2], e1 = vcur[tp.elem * 2 + 1];
                            a0.x = fmaf(tp.w, e0.x, a0.x);
                            a0.y = fmaf(tp.w, e0.y, a0.y);
                            a1.x = fmaf(tp.w, e1.x, a1.x);
                            a1.y = fmaf(tp.w, e1.y, a1.y);
                        }
                        buf[slot] = a0;
                        buf[PLANE + slot] = a1;
                    }
                }
            }
            if (has_next) {
#pragma unroll
                for (int q = 0; q < PREFETCH; ++q) {
                    const int i = tid + q * BLOCK;
                    if (i < vwords) stash(cur ^ 1, i, pre[q]);
                }
            }
            lds_barrier();
            // R1: first radix-8 pass along x of this thread's pol, in place
            if (row_active) {
                float2 v[8];
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int x = j + 8 * m;
                    v[m] = static_cast<unsigned>(x - cp.x0) < static_cast<unsigned>(cp.bw)
                               ? plane[gather_slot64(y, x)] : make_float2(0.f, 0.f);
                }
                Dft<8>::run(v);
                // lanes j >= 4 store their outputs in the order k ^ 4, so that
                // the two lanes of a row whose positions differ by 32 never
                // share a bank in one store
                const bool hi = j >= 4;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const float2 a = v[k], b = v[k + 4];
                    v[k] = hi ? b : a;
                    v[k + 4] = hi ? a : b;
                }
                const int jr = hi ? 4 : 0;
#pragma unroll
                for (int k = 0; k < 8; ++k) plane[bt ^ (k ^ jr)] = v[k];
            }
            // a row is read and written by the 8 lanes of one wave in R1 and R2,
            // and a wave's LDS accesses are performed in order: no block barrier
            __builtin_amdgcn_wave_barrier();
            // R2: second pass along x, in place
            if (row_active) {
                float2 v[8];
#pragma unroll
                for (int r = 0; r < 8; ++r) v[r] = plane[bj ^ (8 * r)];
#pragma unroll
                for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], tw[r]);
                Dft<8>::run(v);
#pragma unroll
                for (int r = 0; r < 8; ++r) plane[bj ^ (8 * r)] = v[r];
            }
            lds_barrier();
            // C1: first pass along y for column kx
            {
                float2 v[8];
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int yy = j + 8 * m;
                    const bool in = yy >= cp.y0 && yy < cp.y0 + cp.bh;
                    v[m] = in ? plane[cm[m] + 512 * m] : make_float2(0.f, 0.f);
                }
                Dft<8>::run(v);
                // a column is read and rewritten only by its own 8 lanes (one
                // wave; the swizzle permutes columns within each row)
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int k = 0; k < 8; ++k) plane[cm[k] + dj + 64 * k] = v[k];
            }
            __builtin_amdgcn_wave_barrier();
            // C2: second pass along y; pixel (ky = j + 8k, kx) of this thread's pol.
            // A thread reads and rewrites only its own eight addresses, so the
            // result goes back in place without a barrier in between.  Pol X
            // stores -i F^X = (Im, -Re), pol Y stores F^Y as it is, so that one
            // formula, Re(F w*) with w the other pol's stored value, gives Re XY
            // on the pol-X threads and Im XY on the pol-Y threads.
            float2 v[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) v[r] = plane[cm[r] + 512 * r];
#pragma unroll
            for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], tw[r]);
            Dft<8>::run(v);
            if (pol == 0) {
#pragma unroll
                for (int k = 0; k < 8; ++k) plane[cm[k] + 512 * k] = make_float2(v[k].y, -v[k].x);
            } else {
#pragma unroll
                for (int k = 0; k < 8; ++k) plane[cm[k] + 512 * k] = v[k];
            }
            lds_barrier();
            // products (Eq. 2): |F|^2 (XX or YY) and the cross term (Re XY or
            // Im XY).  The next sample's gather writes the planes only after the
            // barrier at the top of the loop.
            {
                const float2 *other = buf + (pol ^ 1) * PLANE;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const float2 w = other[cm[k] + 512 * k];
                    acc[k][0] = fmaf(v[k].x, v[k].x, fmaf(v[k].y, v[k].y, acc[k][0]));
                    acc[k][1] = fmaf(v[k].x, w.x, fmaf(v[k].y, w.y, acc[k][1]));
                }
            }
            // a block of samples ends: its sums go to the FP64 running sums
            // (components XX, Re XY, Im XY, YY: pol X holds XX and Re XY, pol
            // Y holds YY and Im XY)
            if (block_ends(t, n_time, flush)) {
                const int q_sq = pol == 0 ? 0 : 3, q_x = pol == 0 ? 1 : 2;
                // addresses from an opaque copy of the pixel index, so that
                // the compiler does not keep all sixteen live across the loop
                int px0;
                asm volatile("v_mov_b32 %0, %1" : "=v"(px0) : "v"(j * 64 + kx));
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int pix = px0 + 512 * k;
                    sums_add(sums, q_sq, pix, acc[k][0], t < flush);
                    sums_add(sums, q_x, pix, acc[k][1], t < flush);
                    acc[k][0] = acc[k][1] = 0.f;
                    asm volatile("" ::: "memory");
                }
            }
            cur ^= 1;
        }
        // a pixel's components were summed by two threads: every sum is in
        // memory before any thread turns a pixel's sums into its products
        sums_settle();
        __syncthreads();
        const double inv = 1.0 / static_cast<double>(n_time);
        for (int pix = tid; pix < PLANE; pix += BLOCK) sums_finish<2>(sums, pix, inv);
    });
}

namespace {

// LDS of the two-pol 64 x 64 kernel: the planes (the gather writes into
// them), two voltage buffers, the channel's taps.
size_t fused64x2_lds_bytes(int max_elem, int max_cells)
{
    // the tap area is sized for supports up to 3 (9 taps per element)
    return sizeof(float2) * 2 * 64 * 64 + sizeof(float2) * 2 * 2 * static_cast<size_t>(max_elem) +
           sizeof(Tap) * static_cast<size_t>(max_elem) * 9 + sizeof(uint32_t) * static_cast<size_t>(max_cells);
}

}  // namespace

// Whether the register-resident 64 x 64 kernels cover a batch with these
// maxima (the generic k_fused_fft<64> runs otherwise).
bool fft64_fits(const FusedBatch &b, int n_pol, int volt_type, int variant)
{
    const int64_t vbytes = static_cast<int64_t>(b.max_elem) * n_pol * (volt_type == EPIC_CI8 ? 2 : 8);
    const bool common = b.n == 64 && vbytes % 4 == 0 && vbytes / 4 <= kFused64Prefetch * kFused64Block &&
                        b.max_cells <= kFused64Rounds * kFused64Block && b.max_cell_taps <= 15 &&
                        static_cast<int64_t>(b.max_elem) * b.max_ktaps <= 0xffff;
    if (!common) return false;
    if (n_pol == 2 && variant == 0)   // the two-pol kernel
        return b.max_side <= 64 && b.max_ktaps <= 9 &&
               fused64x2_lds_bytes(b.max_elem, b.max_cells) <= kLdsBytes;
    return fused64_lds_bytes(n_pol, b.max_elem, b.max_ktaps, b.max_cells) <= kLdsBytes;
}

namespace {

template <int NP, int VT>
epic_status run64(const FusedBatch &b, int n_time, int flush, const float2 *tw, hipStream_t stream)
{
    auto k = k_fused_fft64<NP, VT>;
    const size_t bytes = fused64_lds_bytes(NP, b.max_elem, b.max_ktaps, b.max_cells);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(bytes));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    const int grid = persistent_grid(reinterpret_cast<const void *>(k), kFused64Block, bytes, b.n_items);
    KernelTimer timer("fused_fft_cadence", stream);
    hipLaunchKernelGGL(k, dim3(grid), dim3(kFused64Block), bytes, stream, b.sds, b.q,
                       n_time, flush, tw, b.max_elem, b.max_cells);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

template <int VT>
epic_status run64x2(const FusedBatch &b, int n_time, int flush, const float2 *tw, hipStream_t stream)
{
    auto k = k_fused_fft64x2<VT>;
    const size_t bytes = fused64x2_lds_bytes(b.max_elem, b.max_cells);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(bytes));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    const int grid = persistent_grid(reinterpret_cast<const void *>(k), kFused64x2Block, bytes, b.n_items);
    KernelTimer timer("fused_fft_cadence", stream);
    hipLaunchKernelGGL(k, dim3(grid), dim3(kFused64x2Block), bytes, stream, b.sds, b.q,
                       n_time, flush, tw, b.max_elem, b.max_cells);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

template <int N, int NP, int VT>
epic_status run_small(const FusedBatch &b, int n_time, int flush, const float2 *tw,
                      hipStream_t stream)
{
    auto k = k_fused_fft<N, NP, VT>;
    const size_t bytes = sizeof(float2) * (NP * N * (N + 1) + N);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(bytes));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    const int grid = persistent_grid(reinterpret_cast<const void *>(k), FusedShape<N>::BLOCK, bytes,
                                     b.n_items);
    KernelTimer timer("fused_fft_cadence", stream);
    hipLaunchKernelGGL(k, dim3(grid), dim3(FusedShape<N>::BLOCK), bytes, stream, b.sds,
                       b.q, n_time, flush, tw);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

template <int N>
epic_status dispatch(const FusedBatch &b, int n_pol, int volt_type, int n_time, int flush,
                     const float2 *tw, hipStream_t stream)
{
    if constexpr (N == 64) {
        // variant 0: the two-pol kernel (1024 threads, one pol per thread);
        // variant 1: 512 threads carrying both pols (one pol: always this one)
        const int v = n_pol == 2 ? b.variant : 1;
        if (fft64_fits(b, n_pol, volt_type, v)) {
            const bool x2 = n_pol == 2 && v == 0;
            if (x2 && volt_type == EPIC_CI8) return run64x2<EPIC_CI8>(b, n_time, flush, tw, stream);
            if (x2) return run64x2<EPIC_CF32>(b, n_time, flush, tw, stream);
            if (n_pol == 2 && volt_type == EPIC_CI8) return run64<2, EPIC_CI8>(b, n_time, flush, tw, stream);
            if (n_pol == 2) return run64<2, EPIC_CF32>(b, n_time, flush, tw, stream);
            if (volt_type == EPIC_CI8) return run64<1, EPIC_CI8>(b, n_time, flush, tw, stream);
            return run64<1, EPIC_CF32>(b, n_time, flush, tw, stream);
        }
    }
    if (n_pol == 2 && volt_type == EPIC_CI8) return run_small<N, 2, EPIC_CI8>(b, n_time, flush, tw, stream);
    if (n_pol == 2) return run_small<N, 2, EPIC_CF32>(b, n_time, flush, tw, stream);
    if (volt_type == EPIC_CI8) return run_small<N, 1, EPIC_CI8>(b, n_time, flush, tw, stream);
    return run_small<N, 1, EPIC_CF32>(b, n_time, flush, tw, stream);
}

}  // namespace

bool fused_fft_supported(const FusedBatch &b, int, int)
{
    return b.n == 16 || b.n == 32 || b.n == 64;
}

epic_status launch_fused_fft(const FusedBatch &b, int n_pol, int n_time, int volt_type, int flush,
                             const float2 *twiddles,
                                      hipStream_t stream)
{
    switch (b.n) {
    case 16: return dispatch<16>(b, n_pol, volt_type, n_time, flush, twiddles, stream);
    case 32: return dispatch<32>(b, n_pol, volt_type, n_time, flush, twiddles, stream);
    case 64: return dispatch<64>(b, n_pol, volt_type, n_time, flush, twiddles, stream);
    }
    return fail(EPIC_ERR_INTERNAL, "fused FFT path: unsupported grid");
}

}  // namespace epic
