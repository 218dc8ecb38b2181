// k_fused_dft.hip -- the whole cadence for square grids up to 64 x 64 with the
// 2-D transform of Eq. 3 evaluated as split-precision DFT-matrix products on
// gfx950 matrix cores (EPIC_FP16_SPLIT / EPIC_BF16_SPLIT), fused with the
// gridding (Eq. 3 inner bracket) and the products and time average (Eq. 2).
//
// One work-group owns one (station, channel) and has N/16 waves; wave w
// owns output rows k_y in [16w, 16w + 16).  Per sample:
//   1. grid the kernel-footprint box (both pols), scale by a power of two s1
//      bounded from the sample's largest voltage component and the channel's
//      largest per-cell weight sum, split into hi/lo and store G^T in LDS;
//   2. stage 1 (transform along y, pruned to the footprint rows):
//        Y^T[x][k_y] = sum_y G^T[x][y] F[k_y][y0 + y]
//      with G^T as the A operand and the wave's 16 DFT rows as constant B
//      fragments held in registers for the whole cadence; steps 2-4 run for one
//      pol after the other, pol X's stage-2 tiles waiting in registers;
//   3. each wave scales its Y rows by a power of two s2 and re-splits them;
//      the stage-1 result tiles are already laid out as stage-2 A fragments
//      (the K index of stage 2 is ordered to match), so nothing goes back
//      through LDS;
//   4. stage 2 (transform along x, pruned to the footprint columns):
//        Z[k_y][k_x] = sum_x Y[k_y][x] F[k_x][x0 + x]
//      with B fragments from the channel's DFT rows in LDS; the 2x2 real
//      block of the complex product is formed in the A fragments (up to 3
//      footprint tiles) or, where registers are short, in the B fragments;
//   5. undo s1 s2 exactly, form XX, XY, YY and accumulate in registers.
// The work-group images one (station, channel) over the whole cadence; block
// sums go to FP64 running sums in the image buffer, as in the FP32 path
// (accum.hpp).
#include <algorithm>

#include "accum.hpp"
#include "internal.hpp"
#include "lds_sync.hpp"
#include "volts.hpp"
#include "mfma_split.hpp"

namespace epic {

template <int N, int T>
struct FusedDftShape {
    static constexpr int WAVES = N / 16;
    static constexpr int BLOCK = 64 * WAVES;
    static constexpr int PITCH = 16 * T + 4;      // LDS pitch of G^T rows and F_x rows (words)
    static constexpr int ROUNDS = (16 * T * 16 * T + BLOCK - 1) / BLOCK;   // gather rounds
};

inline size_t fused_dft_lds_bytes(int N, int T, int np, int vt, int n_elem, int max_cells)
{
    const int pitch = 16 * T + 4;
    return sizeof(uint32_t) * (2 * static_cast<size_t>(np) * 16 * T * pitch   // G^T hi, lo
                               + 2 * static_cast<size_t>(N) * pitch           // F_x rows hi, lo
                               + 2 * static_cast<size_t>(np) * n_elem * volt_words(vt)  // voltages x 2
                               + static_cast<size_t>(max_cells));             // gather jobs
}

// Footprints of up to 3 tiles leave room for two work-groups per compute unit
// (two waves per SIMD); with 4 tiles the LDS holds one work-group per CU, so
// each wave may take a SIMD's whole register file (no spills).
template <int T> struct FusedDftWaves { static constexpr int value = T >= 4 ? 1 : 2; };

template <int N, int T, int NP, int VT, int PREC>
__global__ __launch_bounds__(64 * (N / 16)) __attribute__((amdgpu_waves_per_eu(FusedDftWaves<T>::value))) void k_fused_dft(
    const StationDev *__restrict__ sds, ItemQueue q, int n_time, int flush,
    const uint32_t *__restrict__ rows, int max_elem)
{
    using Sh = FusedDftShape<N, T>;
    using S = Split<PREC>;
    using vec8 = typename S::vec8;
    using scalar = typename S::scalar;
    constexpr int WAVES = Sh::WAVES, BLOCK = Sh::BLOCK, PITCH = Sh::PITCH;
    constexpr int NQ = NP == 2 ? 4 : 1;
    constexpr int NT = N / 16;                      // k_x tiles
    constexpr int GPLANE = 16 * T * PITCH;          // words per pol of G^T
    extern __shared__ __align__(16) uint32_t lds[];
    uint32_t *gbh = lds;                            // [NP][16T][PITCH] G^T hi (re, im)
    uint32_t *gbl = gbh + NP * GPLANE;              // lo
    uint32_t *txh = gbl + NP * GPLANE;              // [N][PITCH] F[k_x][x0 + x] hi (re, im)
    uint32_t *txl = txh + N * PITCH;                // lo
    constexpr int VW = volt_words(VT);
    uint32_t *vf = txl + N * PITCH;                 // [2][max_elem][NP][VW] voltages
    uint32_t *jobs = vf + 2 * NP * VW * max_elem;   // [ncell] gather jobs
    __shared__ float vred[2][WAVES];

    for_each_item(q, [&](const int4 item) {
        // thread indices from an opaque copy of the thread index, so that the
        // compiler derives them per item instead of keeping values built from
        // them live across the item loop
        int tid;
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(static_cast<int>(threadIdx.x)));
        const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int g = lane >> 4, r16 = lane & 15;
        const StationDev sd = sds[item.x];
        const int c = item.y;
        const int vwords = sd.n_elem * NP * (VT == EPIC_CI8 ? 2 : 8) / 4;
        const int t_begin = 0, t_end = n_time;
        const ItemSums sums = item_sums(sd.image, NP, N * N, c);
        const ChanPlan cp = sd.chan[c];
        const int ncell = cp.bw * cp.bh;
        const int mx = (cp.bw + 15) >> 4, my = (cp.bh + 15) >> 4;   // footprint tiles (<= T)
        const uint32_t *rows_lo = rows + N * N;

        // ---- once per work-group -------------------------------------------
        for (int i = tid; i < 2 * NP * GPLANE; i += BLOCK) gbh[i] = 0u;     // padding stays 0
        for (int i = tid; i < N * 16 * T; i += BLOCK) {
            const int k = i / (16 * T), x = i - k * (16 * T);
            const int jj = (cp.x0 + x) & (N - 1);
            txh[k * PITCH + x] = rows[k * N + jj];
            txl[k * PITCH + x] = rows_lo[k * N + jj];
        }
        // gather jobs (cells in descending tap-count order): cell << 20 | count << 16 | first tap
        {
            const gptr<int32_t> cs = global_ptr<int32_t>(sd.cell_start) + cp.cell_off;
            const gptr<int32_t> ord = global_ptr<int32_t>(sd.cell_order) + cp.cell_off;
            for (int i = tid; i < ncell; i += BLOCK) {
                const int cell = ord[i];
                const int k0 = cs[cell];
                jobs[i] = (static_cast<uint32_t>(cell) << 20) |
                          (static_cast<uint32_t>(cs[cell + 1] - k0) << 16) | static_cast<uint32_t>(k0);
            }
        }
        const Tap *taps = sd.taps + cp.tap_off;
        // stage-1 B fragments: DFT rows k_y = 16 wave + r16 at y0 + 16 ks + 4 g + i,
        // held in registers for the whole cadence
        vec8 b1[T][4];   // [K-step][re hi, re lo, im hi, im lo]
        {
            const int ky_row = (16 * wave + r16) * N;
#pragma unroll
            for (int ks = 0; ks < T; ++ks) {
                u32x4_t wr_h, wr_l, wi_h, wi_l;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int jj = (cp.y0 + 16 * ks + 4 * g + i) & (N - 1);
                    const uint32_t h = rows[ky_row + jj], l = rows_lo[ky_row + jj];
                    wr_h[i] = neg_hi(h);
                    wr_l[i] = neg_hi(l);
                    wi_h[i] = swap_halves(h);
                    wi_l[i] = swap_halves(l);
                }
                b1[ks][0] = __builtin_bit_cast(vec8, wr_h);
                b1[ks][1] = __builtin_bit_cast(vec8, wr_l);
                b1[ks][2] = __builtin_bit_cast(vec8, wi_h);
                b1[ks][3] = __builtin_bit_cast(vec8, wi_l);
            }
        }

        // voltages of a sample as float pairs in vf[buffer]; returns the largest
        // |component| this thread stored
        const gptr<uint32_t> vsrc = global_ptr<uint32_t>(sd.volts) +
                               static_cast<size_t>(c) * n_time * vwords;
        auto stash = [&](int buffer, int i, uint32_t w) -> float {
            uint32_t *dst = vf + buffer * NP * VW * max_elem;
            if constexpr (VT == EPIC_CI8) {
                // four int8 components -> two exact FP16 pairs
                const int8_t a = static_cast<int8_t>(w & 0xff), b = static_cast<int8_t>((w >> 8) & 0xff);
                const int8_t cc = static_cast<int8_t>((w >> 16) & 0xff), d = static_cast<int8_t>((w >> 24) & 0xff);
                dst[2 * i] = pack2<EPIC_FP16_SPLIT>(static_cast<_Float16>(a), static_cast<_Float16>(b));
                dst[2 * i + 1] = pack2<EPIC_FP16_SPLIT>(static_cast<_Float16>(cc), static_cast<_Float16>(d));
                const int m = max(max(abs(static_cast<int>(a)), abs(static_cast<int>(b))),
                                  max(abs(static_cast<int>(cc)), abs(static_cast<int>(d))));
                return static_cast<float>(m);
            } else {
                dst[i] = w;
                return fabsf(__builtin_bit_cast(float, w));
            }
        };
        auto volt = [&](const uint32_t *vcur, int idx) -> float2 {
            if constexpr (VT == EPIC_CI8) {
                const uint32_t w = vcur[idx];
                return make_float2(static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(w & 0xffff))),
                                   static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(w >> 16))));
            } else {
                return reinterpret_cast<const float2 *>(vcur)[idx];
            }
        };
        auto reduce_max = [&](float m, int buffer) {
            for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
            if (lane == 0) vred[buffer][wave] = m;
        };
        {
            float m = 0.f;
            for (int i = tid; i < vwords; i += BLOCK)
                m = fmaxf(m, stash(0, i, vsrc[static_cast<size_t>(t_begin) * vwords + i]));
            reduce_max(m, 0);
        }

        lds_barrier();
        // the jobs with taps: the cell order puts the cells without taps last
        // (zero in G^T since the item began), so the gather stops before them
        int njob = 0;
        {
            int hi = ncell;
            while (njob < hi) {
                const int mid = (njob + hi) >> 1;
                if ((jobs[mid] >> 16) & 15) njob = mid + 1;
                else hi = mid;
            }
        }

        int cur = 0;
        // blocks of `flush` samples: their sums go to the FP64 running sums
        // after the block's loop, so that code stays out of the sample loop
#pragma unroll 1
        for (int t0 = t_begin; t0 < t_end; t0 += flush) {
        const int t1 = min(t_end, t0 + flush);
        float acc[NT][4][NQ];
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int q = 0; q < NQ; ++q) acc[a][i][q] = 0.f;
        for (int t = t0; t < t1; ++t) {
            const bool has_next = t + 1 < t_end;
            // ---- 1. grid the footprint box, scale, split -> G^T in LDS -------
            float vmax = 0.f;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) vmax = fmaxf(vmax, vred[cur][w]);
            const float s1 = pow2_scale(vmax * cp.wsum_max);
            {
                // G cells per thread at a time, tap index outermost, so that
                // the G cells' tap loads (from the L2) are in flight together
                // instead of one dependent chain per cell; each cell still
                // adds its taps in list order
                constexpr int G = 4;
                const uint32_t *vcur = vf + cur * NP * VW * max_elem;
                for (int i0 = tid; i0 < njob; i0 += G * BLOCK) {
                    int k0[G], kn[G], kmax = 0;
#pragma unroll
                    for (int u = 0; u < G; ++u) {
                        const int i = i0 + u * BLOCK;
                        const uint32_t job = i < njob ? jobs[i] : 0u;
                        k0[u] = static_cast<int>(job & 0xffff);
                        kn[u] = i < njob ? static_cast<int>((job >> 16) & 15) : 0;
                        kmax = max(kmax, kn[u]);
                    }
                    float2 a[G][NP];
#pragma unroll
                    for (int u = 0; u < G; ++u)
#pragma unroll
                        for (int p = 0; p < NP; ++p) a[u][p] = make_float2(0.f, 0.f);
#pragma unroll 2
                    for (int s = 0; s < kmax; ++s) {
                        Tap tp[G];
#pragma unroll
                        for (int u = 0; u < G; ++u) tp[u] = gload<Tap>(taps, s < kn[u] ? k0[u] + s : k0[u]);
#pragma unroll
                        for (int u = 0; u < G; ++u) {
                            if (s < kn[u]) {
#pragma unroll
                                for (int p = 0; p < NP; ++p) {
                                    const float2 e = volt(vcur, tp[u].elem * NP + p);
                                    a[u][p].x = fmaf(tp[u].w, e.x, a[u][p].x);
                                    a[u][p].y = fmaf(tp[u].w, e.y, a[u][p].y);
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < G; ++u) {
                        const int i = i0 + u * BLOCK;
                        if (i >= njob) break;
                        const int cell = static_cast<int>(jobs[i] >> 20);
                        const int by = cell / cp.bw, bx = cell - by * cp.bw;
#pragma unroll
                        for (int p = 0; p < NP; ++p) {
                            scalar hr, lr, hi_, li;
                            split<PREC>(a[u][p].x * s1, hr, lr);
                            split<PREC>(a[u][p].y * s1, hi_, li);
                            gbh[p * GPLANE + bx * PITCH + by] = pack2<PREC>(hr, hi_);
                            gbl[p * GPLANE + bx * PITCH + by] = pack2<PREC>(lr, li);
                        }
                    }
                }
            }
            if (has_next) {
                float m = 0.f;
                for (int i = tid; i < vwords; i += BLOCK)
                    m = fmaxf(m, stash(cur ^ 1, i, vsrc[static_cast<size_t>(t + 1) * vwords + i]));
                reduce_max(m, cur ^ 1);
            }
            lds_barrier();

            // ---- 2.-5. per pol: stage 1, rescale, stage 2; products once both
            // pols of a tile are known (pol X's stage-2 tiles wait in zx) ------
            floatx4_t zx[NT][2];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                // 2. stage 1: Y^T[x][k_y] for this wave's 16 k_y
                floatx4_t c1[T][2];   // [x tile][re, im]
#pragma unroll
                for (int mt = 0; mt < T; ++mt)
#pragma unroll
                    for (int o = 0; o < 2; ++o) c1[mt][o] = floatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < T; ++ks) {
                    if (ks >= my) break;
#pragma unroll
                    for (int mt = 0; mt < T; ++mt) {
                        if (mt >= mx) break;
                        const int off = p * GPLANE + (16 * mt + r16) * PITCH + 16 * ks + 4 * g;
                        const vec8 ah = __builtin_bit_cast(vec8, *reinterpret_cast<const u32x4_t *>(&gbh[off]));
                        const vec8 al = __builtin_bit_cast(vec8, *reinterpret_cast<const u32x4_t *>(&gbl[off]));
                        c1[mt][0] = mma3<PREC>(ah, al, b1[ks][0], b1[ks][1], c1[mt][0]);
                        c1[mt][1] = mma3<PREC>(ah, al, b1[ks][2], b1[ks][3], c1[mt][1]);
                    }
                }
                if (p == NP - 1) lds_barrier();   // G^T is free for the next sample

                // 3. per-wave power-of-two scale and re-split into stage-2 A fragments
                float ymax = 0.f;
#pragma unroll
                for (int mt = 0; mt < T; ++mt)
#pragma unroll
                    for (int o = 0; o < 2; ++o)
#pragma unroll
                        for (int i = 0; i < 4; ++i) ymax = fmaxf(ymax, fabsf(c1[mt][o][i]));
                for (int o = 32; o > 0; o >>= 1) ymax = fmaxf(ymax, __shfl_xor(ymax, o));
                const float s2 = pow2_scale(ymax);
                // The 2x2 real block of the complex product goes into whichever
                // operand is cheaper to rebuild.  Up to 3 footprint tiles it sits
                // in the A fragments (built once per sample and pol): with
                // B = (Re F, Im F) pairs as stored, A = (Re Y, -Im Y) gives the
                // real output and A = (Im Y, Re Y) the imaginary one.  With 4
                // tiles the extra A registers would spill, so the A fragments stay
                // (Re Y, Im Y) and each B fragment is turned into (Re F, -Im F)
                // and (Im F, Re F) as it is loaded.
                constexpr bool kBlockInA = T <= 3;
                constexpr int NA = kBlockInA ? 4 : 2;
                vec8 a2[T][NA];   // [x K-step][re hi, re lo(, im hi, im lo)]
#pragma unroll
                for (int mt = 0; mt < T; ++mt) {
                    u32x4_t rh, rl, ih, il;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        scalar hr, lr, hi_, li;
                        split<PREC>(c1[mt][0][i] * s2, hr, lr);
                        split<PREC>(c1[mt][1][i] * s2, hi_, li);
                        if constexpr (kBlockInA) {
                            rh[i] = pack2<PREC>(hr, -hi_);
                            rl[i] = pack2<PREC>(lr, -li);
                            ih[i] = pack2<PREC>(hi_, hr);
                            il[i] = pack2<PREC>(li, lr);
                        } else {
                            rh[i] = pack2<PREC>(hr, hi_);
                            rl[i] = pack2<PREC>(lr, li);
                        }
                    }
                    a2[mt][0] = __builtin_bit_cast(vec8, rh);
                    a2[mt][1] = __builtin_bit_cast(vec8, rl);
                    if constexpr (kBlockInA) {
                        a2[mt][NA > 2 ? 2 : 0] = __builtin_bit_cast(vec8, ih);
                        a2[mt][NA > 3 ? 3 : 1] = __builtin_bit_cast(vec8, il);
                    }
                }

                // 4. stage 2 per k_x tile; 5. products
                const float inv = 1.f / (s1 * s2);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    floatx4_t z0 = floatx4_t{0.f, 0.f, 0.f, 0.f}, z1 = z0;
#pragma unroll
                    for (int ks = 0; ks < T; ++ks) {
                        if (ks >= mx) break;
                        const int off = (16 * nt + r16) * PITCH + 16 * ks + 4 * g;
                        const u32x4_t wh = *reinterpret_cast<const u32x4_t *>(&txh[off]);
                        const u32x4_t wl = *reinterpret_cast<const u32x4_t *>(&txl[off]);
                        if constexpr (kBlockInA) {
                            const vec8 bh = __builtin_bit_cast(vec8, wh), bl = __builtin_bit_cast(vec8, wl);
                            z0 = mma3<PREC>(a2[ks][0], a2[ks][1], bh, bl, z0);
                            z1 = mma3<PREC>(a2[ks][NA > 2 ? 2 : 0], a2[ks][NA > 3 ? 3 : 1], bh, bl, z1);
                        } else {
                            u32x4_t rh, rl, ih, il;
#pragma unroll
                            for (int i = 0; i < 4; ++i) {
                                rh[i] = neg_hi(wh[i]);
                                rl[i] = neg_hi(wl[i]);
                                ih[i] = swap_halves(wh[i]);
                                il[i] = swap_halves(wl[i]);
                            }
                            z0 = mma3<PREC>(a2[ks][0], a2[ks][1], __builtin_bit_cast(vec8, rh),
                                            __builtin_bit_cast(vec8, rl), z0);
                            z1 = mma3<PREC>(a2[ks][0], a2[ks][1], __builtin_bit_cast(vec8, ih),
                                            __builtin_bit_cast(vec8, il), z1);
                        }
                    }
                    // lane holds pixels (k_y = 16 wave + 4 g + i, k_x = 16 nt + r16)
                    if (p == 0) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            z0[i] *= inv;
                            z1[i] *= inv;
                        }
                        if constexpr (NP == 1) {
#pragma unroll
                            for (int i = 0; i < 4; ++i)
                                acc[nt][i][0] = fmaf(z0[i], z0[i], fmaf(z1[i], z1[i], acc[nt][i][0]));
                        } else {
                            zx[nt][0] = z0;
                            zx[nt][1] = z1;
                        }
                    } else if constexpr (NP == 2) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const float xr = zx[nt][0][i], xi = zx[nt][1][i];
                            const float yr = z0[i] * inv, yi = z1[i] * inv;
                            acc[nt][i][0] = fmaf(xr, xr, fmaf(xi, xi, acc[nt][i][0]));
                            acc[nt][i][1] = fmaf(xr, yr, fmaf(xi, yi, acc[nt][i][1]));
                            acc[nt][i][2] = fmaf(xi, yr, fmaf(-xr, yi, acc[nt][i][2]));
                            acc[nt][i][3] = fmaf(yr, yr, fmaf(yi, yi, acc[nt][i][3]));
                        }
                    }
                }
            }
            cur ^= 1;
        }
        {
            int px0;   // opaque: keeps the addresses from being hoisted
            asm volatile("v_mov_b32 %0, %1" : "=v"(px0) : "v"((16 * wave + 4 * g) * N + r16));
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int pix = px0 + i * N + 16 * nt;
#pragma unroll
                    for (int q = 0; q < NQ; ++q) sums_add(sums, q, pix, acc[nt][i][q], t0 == t_begin);
                    asm volatile("" ::: "memory");
                }
        }
        }
        sums_settle();
        const double inv_n = 1.0 / static_cast<double>(n_time);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) sums_finish<NP>(sums, (16 * wave + 4 * g + i) * N + 16 * nt + r16, inv_n);
    });
}

namespace {

template <int N, int T, int NP, int VT, int PREC>
epic_status run(const FusedBatch &b, int n_time, int flush, const uint32_t *rows,
                hipStream_t stream)
{
    using Sh = FusedDftShape<N, T>;
    const size_t bytes = fused_dft_lds_bytes(N, T, NP, VT, b.max_elem, b.max_cells);
    auto k = k_fused_dft<N, T, NP, VT, PREC>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(bytes));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    const int grid = persistent_grid(reinterpret_cast<const void *>(k), Sh::BLOCK, bytes, b.n_items);
    KernelTimer timer("fused_dft_cadence", stream);
    hipLaunchKernelGGL(k, dim3(grid), dim3(Sh::BLOCK), bytes, stream, b.sds, b.q, n_time,
                       flush, rows, b.max_elem);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

template <int N, int T, int PREC>
epic_status by_type(const FusedBatch &b, int n_pol, int volt_type, int n_time, int flush,
                    const uint32_t *rows, hipStream_t stream)
{
    if (n_pol == 2 && volt_type == EPIC_CI8) return run<N, T, 2, EPIC_CI8, PREC>(b, n_time, flush, rows, stream);
    if (n_pol == 2) return run<N, T, 2, EPIC_CF32, PREC>(b, n_time, flush, rows, stream);
    if (volt_type == EPIC_CI8) return run<N, T, 1, EPIC_CI8, PREC>(b, n_time, flush, rows, stream);
    return run<N, T, 1, EPIC_CF32, PREC>(b, n_time, flush, rows, stream);
}

// footprint tiles of a batch: its largest box side, at least the smallest
// template size for the grid
int tiles_of(const FusedBatch &b) { return std::max((b.max_side + 15) / 16, b.n == 64 ? 2 : 1); }

template <int PREC>
epic_status by_size(const FusedBatch &b, int n_pol, int volt_type, int n_time, int flush,
                    const uint32_t *rows, hipStream_t stream)
{
    switch (b.n * 8 + tiles_of(b)) {
    case 16 * 8 + 1: return by_type<16, 1, PREC>(b, n_pol, volt_type, n_time, flush, rows, stream);
    case 32 * 8 + 1: return by_type<32, 1, PREC>(b, n_pol, volt_type, n_time, flush, rows, stream);
    case 32 * 8 + 2: return by_type<32, 2, PREC>(b, n_pol, volt_type, n_time, flush, rows, stream);
    case 64 * 8 + 2: return by_type<64, 2, PREC>(b, n_pol, volt_type, n_time, flush, rows, stream);
    case 64 * 8 + 3: return by_type<64, 3, PREC>(b, n_pol, volt_type, n_time, flush, rows, stream);
    case 64 * 8 + 4: return by_type<64, 4, PREC>(b, n_pol, volt_type, n_time, flush, rows, stream);
    }
    return fail(EPIC_ERR_INTERNAL, "fused split path: unsupported grid/footprint");
}

}  // namespace

epic_status launch_fused_dft(const FusedBatch &b, int n_pol, int n_time, int volt_type,
                            int precision, int flush, const uint32_t *rows, hipStream_t stream)
{
    if (b.n == 128) return launch_fused_dft128(b, n_pol, n_time, volt_type, precision, flush, rows, stream);
    if (precision == EPIC_FP16_SPLIT)
        return by_size<EPIC_FP16_SPLIT>(b, n_pol, volt_type, n_time, flush, rows, stream);
    return by_size<EPIC_BF16_SPLIT>(b, n_pol, volt_type, n_time, flush, rows, stream);
}

bool fused_dft_supported(const FusedBatch &b, int n_pol, int volt_type)
{
    if (b.n == 128) return fused_dft128_supported(b, n_pol, volt_type);
    if (b.n != 16 && b.n != 32 && b.n != 64) return false;
    const int64_t vbytes = static_cast<int64_t>(b.max_elem) * n_pol * (volt_type == EPIC_CI8 ? 2 : 8);
    if (vbytes % 4 != 0) return false;
    if (b.max_cell_taps > 15 || static_cast<int64_t>(b.max_elem) * b.max_ktaps > 0xffff) return false;
    const int t = tiles_of(b);
    if (t > b.n / 16) return false;
    // 256 bytes stay free for the kernel's static LDS
    return fused_dft_lds_bytes(b.n, t, n_pol, volt_type, b.max_elem, b.max_cells) <= 160 * 1024 - 256;
}

}  // namespace epic
