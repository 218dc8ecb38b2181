// k_fused_dft128.hip -- the whole cadence for 128 x 128 grids with the 2-D
// transform of Eq. 3 evaluated as split-precision DFT-matrix products on
// gfx950 matrix cores (EPIC_FP16_SPLIT / EPIC_BF16_SPLIT), fused with the
// gridding (Eq. 3 inner bracket) and the products and time average (Eq. 2).
//
// Work items are (station, channel, half): a work-group of four waves images
// output rows k_y in [64 half, 64 half + 64) over the whole cadence, wave w
// owning the 16 rows from 64 half + 16 w.  Both halves grid the same
// footprint box (the gridding is a small part of the work); the rest is split
// without overlap.  Per sample:
//   1. grid the footprint box (both pols), scale by a power of two s1, split
//      into hi/lo and store G^T in LDS;
//   2. stage 1 (along y, pruned to the box rows), for each pol:
//        Y^T[x][k_y] = sum_y G^T[x][y] F[k_y][y]
//      G^T is the A operand, the wave's 16 DFT rows the B operand, read per
//      K-step from the 32-row table in LDS and turned (below); each wave
//      rescales its result by a power of two s2 and splits it again.  The result tiles are laid out as the A
//      fragments of stage 2, so both pols' tiles stay in registers;
//   3. stage 2 (along x, pruned to the box columns), 16 k_x at a time:
//        Z[k_y][k_x] = sum_x Y[k_y][x] F[k_x][x]
//      with one set of B fragments for both pols;
//   4. undo s1 s2 exactly, form XX, XY, YY and add them to registers; block
//      sums go to FP64 running sums in the image buffer (accum.hpp).
//
// The transform runs on box coordinates (x, y counted from the box corner
// x0, y0).  The true transform differs by the factor w^(k_x x0 + k_y y0) of
// unit modulus, the same for both pols, so every product F^a conj(F^b) is
// unchanged, and one DFT table serves every channel.  Rows k >= 32 of that
// table are rows k mod 32 times i^(x (k div 32)) (w^32 = i for
// w = exp(2 pi i / 128)), an exact change of signs and halves in FP16 or
// BF16, so LDS holds only rows 0-31 for both stages; within one B fragment
// the column (x or y) mod 4 is the word index, so the change is fixed per
// word.
#include <algorithm>
#include <type_traits>

#include "accum.hpp"
#include "internal.hpp"
#include "lds_sync.hpp"
#include "mfma_split.hpp"
#include "volts.hpp"

namespace epic {

namespace {

constexpr int kD128Block = 256;
constexpr int kD128Tiles = 5;          // footprint boxes up to 80 cells on a side
constexpr int kD128Rows = 32;          // DFT rows held in LDS
constexpr size_t kD128Lds = 160 * 1024 - 256;   // 256 bytes stay free for static LDS

// Raw voltage words per thread and sample that the next sample's prefetch holds.
template <int VT> struct VoltPre { static constexpr int value = VT == EPIC_CI8 ? 8 : 32; };

struct Dft128Dims {
    int gx;      // G^T rows (16 x tiles)
    int pg;      // G^T row pitch in words (16 y tiles + 4)
    int pf;      // DFT table row pitch in words (16 x or y tiles, the larger, + 4)
};

Dft128Dims dims_of(int max_bw, int max_bh)
{
    const int tx = (max_bw + 15) / 16, ty = (max_bh + 15) / 16;
    // the table serves both stages: columns up to the larger box side
    return Dft128Dims{16 * tx, 16 * ty + 4, 16 * std::max(tx, ty) + 4};
}

size_t dft128_lds_bytes(const Dft128Dims &d, int np, int vt, int max_elem, int max_cells)
{
    return sizeof(uint32_t) * (2 * static_cast<size_t>(np) * d.gx * d.pg        // G^T hi, lo
                               + 2 * static_cast<size_t>(kD128Rows) * d.pf      // DFT rows hi, lo
                               + static_cast<size_t>(np) * max_elem * volt_words(vt)   // voltages
                               + static_cast<size_t>(max_cells));               // gather jobs
}

// The 2x2 block columns of B fragment words w of DFT row k0 + 32 M (the
// table holds row k0): the real-output column (Re F, -Im F) and the
// imaginary-output column (Im F, Re F) of the row, which is row k0 times
// i^(M i) in word i.  With P = (Re, -Im) and Q = (Im, Re) of the stored word,
// a turn by i maps (P, Q) to (-Q, P).
template <int J>
__device__ __forceinline__ void turned_word(uint32_t w, uint32_t &re_col, uint32_t &im_col)
{
    const uint32_t p = neg_hi(w), q = swap_halves(w);
    if constexpr (J == 0) { re_col = p; im_col = q; }
    else if constexpr (J == 1) { re_col = neg_both(q); im_col = p; }
    else if constexpr (J == 2) { re_col = neg_both(p); im_col = neg_both(q); }
    else { re_col = q; im_col = neg_both(p); }
}

template <int M>
__device__ __forceinline__ void turned_block(const u32x4_t &w, u32x4_t &re_col, u32x4_t &im_col)
{
    uint32_t r[4], m[4];
    turned_word<(M * 0) & 3>(w[0], r[0], m[0]);
    turned_word<(M * 1) & 3>(w[1], r[1], m[1]);
    turned_word<(M * 2) & 3>(w[2], r[2], m[2]);
    turned_word<(M * 3) & 3>(w[3], r[3], m[3]);
    re_col = u32x4_t{r[0], r[1], r[2], r[3]};
    im_col = u32x4_t{m[0], m[1], m[2], m[3]};
}

}  // namespace

template <int NP, int VT, int PREC>
__global__ __launch_bounds__(kD128Block) __attribute__((amdgpu_waves_per_eu(1))) void k_fused_dft128(
    const StationDev *__restrict__ sds, ItemQueue q, int n_time, int flush, const uint32_t *__restrict__ rows,
    int max_elem, Dft128Dims d)
{
    using S = Split<PREC>;
    using vec8 = typename S::vec8;
    using scalar = typename S::scalar;
    constexpr int N = 128, T = kD128Tiles, NT = N / 16, WAVES = kD128Block / 64, BLOCK = kD128Block;
    constexpr int NQ = NP == 2 ? 4 : 1;
    constexpr int VW = volt_words(VT);
    constexpr int VPRE = VoltPre<VT>::value;
    extern __shared__ __align__(16) uint32_t lds[];
    const int gplane = d.gx * d.pg;
    uint32_t *gbh = lds;                               // [NP][gx][pg] G^T hi (re, im)
    uint32_t *gbl = gbh + NP * gplane;                 // lo
    uint32_t *fh = gbl + NP * gplane;                  // [32][pf] DFT rows hi (re, im)
    uint32_t *fl = fh + kD128Rows * d.pf;              // lo
    uint32_t *vf = fl + kD128Rows * d.pf;              // [max_elem][NP][VW] voltages
    uint32_t *jobs = vf + NP * VW * max_elem;          // [ncell] gather jobs (see below)
    __shared__ float vred[WAVES];
    const uint32_t *rows_lo = rows + N * N;

    // DFT rows 0-31 over the box columns, once per work-group (the item
    // loop's first barrier orders them before any read)
    for (int i = threadIdx.x; i < kD128Rows * d.pf; i += BLOCK) {
        const int k = i / d.pf, x = i - k * d.pf;
        const bool in = x < d.pf - 4;
        fh[i] = in ? rows[k * N + x] : 0u;
        fl[i] = in ? rows_lo[k * N + x] : 0u;
    }

    for_each_item(q, [&](const int4 item) {
        // thread indices from an opaque copy of the thread index (see k_fused_dft)
        int tid;
        asm volatile("v_mov_b32 %0, %1" : "=v"(tid) : "v"(static_cast<int>(threadIdx.x)));
        const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
        const int g = lane >> 4, r16 = lane & 15;
        const StationDev sd = sds[item.x];
        const int c = item.y;
        const int ky0 = 64 * item.z + 16 * wave;       // this wave's first output row
        const int vwords = sd.n_elem * NP * (VT == EPIC_CI8 ? 2 : 8) / 4;
        const ItemSums sums = item_sums(sd.image, NP, N * N, c);
        const ChanPlan cp = sd.chan[c];
        const int ncell = cp.bw * cp.bh;
        const int mx = (cp.bw + 15) >> 4, my = (cp.bh + 15) >> 4;   // footprint tiles (<= T)
        const float inv_bw = 1.f / static_cast<float>(cp.bw);

        // ---- once per item --------------------------------------------------
        // Gather jobs.  A wave grids 256 cells at a time and runs as many tap
        // rounds as the largest tap count among them, several times the mean
        // on a random layout.  Where the channel's tap indices fit the bits
        // that a cell index and a count leave (kbits below), the jobs are the
        // cells with taps in order of falling tap count (stable: equal counts
        // in box order), cell << (kbits + 5) | count << kbits | first tap,
        // so a wave's cells have about equal counts and cells
        // without taps (zero in G^T from the start) are skipped; otherwise
        // every cell in box order, first tap << 5 | count.  Either way each
        // cell adds its own taps in list order.
        const gptr<int32_t> cs = global_ptr<int32_t>(sd.cell_start) + cp.cell_off;
        // field widths: cell index (cbits, enough for ncell), count (5), first
        // tap (the remaining kbits)
        const int cbits = 32 - __builtin_clz(static_cast<unsigned>(max(ncell - 1, 1)));
        const int kbits = 27 - cbits;
        const bool sorted = cs[ncell] <= (1 << kbits);
        int njob = ncell;
        {
            uint32_t *box_jobs = sorted ? gbh : jobs;   // G^T is free until it is cleared below
            for (int i = tid; i < ncell; i += BLOCK) {
                const int k0 = cs[i];
                box_jobs[i] = (static_cast<uint32_t>(k0) << 5) | static_cast<uint32_t>(cs[i + 1] - k0);
            }
            if (sorted) {
                // counting sort by falling count, one count at a time: thread
                // tid ranks the cells of its own run [r0, r1) in box order
                int *wsum = reinterpret_cast<int *>(gbh + ncell);   // 4 wave totals
                const int per = (ncell + BLOCK - 1) / BLOCK;
                const int r0 = min(ncell, tid * per), r1 = min(ncell, r0 + per);
                lds_barrier();
                int base = 0;
                for (int b = 31; b >= 1; --b) {
                    int cnt = 0;
                    for (int i = r0; i < r1; ++i) cnt += (box_jobs[i] & 31u) == static_cast<uint32_t>(b);
                    // exclusive scan of cnt over the work-group
                    int inc = cnt;
                    for (int o = 1; o < 64; o <<= 1) {
                        const int v = __shfl_up(inc, o);
                        if (lane >= o) inc += v;
                    }
                    if (lane == 63) wsum[wave] = inc;
                    lds_barrier();
                    int before = 0, total = 0;
#pragma unroll
                    for (int w = 0; w < WAVES; ++w) {
                        const int v = wsum[w];
                        before += w < wave ? v : 0;
                        total += v;
                    }
                    int pos = base + before + inc - cnt;
                    for (int i = r0; i < r1 && cnt > 0; ++i) {
                        const uint32_t j = box_jobs[i];
                        if ((j & 31u) == static_cast<uint32_t>(b)) {
                            jobs[pos++] = (static_cast<uint32_t>(i) << (kbits + 5)) | (static_cast<uint32_t>(b) << kbits) |
                                          (j >> 5);
                            --cnt;
                        }
                    }
                    base += total;
                    lds_barrier();   // wsum is read before the next count's totals
                }
                njob = base;
            }
        }
        for (int i = tid; i < 2 * NP * gplane; i += BLOCK) gbh[i] = 0u;     // padding stays 0
        const Tap *taps = sd.taps + cp.tap_off;
        // stage-1 B fragments: DFT row k_y = ky0 + r16 at y = 16 ks + 4 g + i,
        // read per K-step from the table in LDS: row k_y is table row
        // k_y mod 32 times i^(M y), M = k_y div 32 (the same for the whole
        // wave), and y mod 4 is the word index i, so word i is turned by
        // J = M i mod 4 quarter turns: (P, Q) -> (P, Q), (-Q, P), (-P, -Q),
        // (Q, -P) for J = 0, 1, 2, 3, with P = (Re, -Im), Q = (Im, Re)
        const int m1 = __builtin_amdgcn_readfirstlane(ky0 >> 5);
        const int f1row = (16 * (wave & 1) + r16) * d.pf + 4 * g;
        auto b1frag = [&](int ks, vec8 &brh, vec8 &brl, vec8 &bih, vec8 &bil) {
            const u32x4_t wh = *reinterpret_cast<const u32x4_t *>(&fh[f1row + 16 * ks]);
            const u32x4_t wl = *reinterpret_cast<const u32x4_t *>(&fl[f1row + 16 * ks]);
            u32x4_t rh, rl, ih, il;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = (m1 * i) & 3;
                const bool sw = j & 1;
                const uint32_t mre = (j == 1 || j == 2) ? 0x80008000u : 0u, mim = j >= 2 ? 0x80008000u : 0u;
                const uint32_t ph = neg_hi(wh[i]), qh = swap_halves(wh[i]);
                const uint32_t pl = neg_hi(wl[i]), ql = swap_halves(wl[i]);
                rh[i] = (sw ? qh : ph) ^ mre;
                ih[i] = (sw ? ph : qh) ^ mim;
                rl[i] = (sw ? ql : pl) ^ mre;
                il[i] = (sw ? pl : ql) ^ mim;
            }
            brh = __builtin_bit_cast(vec8, rh);
            brl = __builtin_bit_cast(vec8, rl);
            bih = __builtin_bit_cast(vec8, ih);
            bil = __builtin_bit_cast(vec8, il);
        };

        // a sample's voltages: raw words into registers (fetch), then into LDS
        // as FP16 pairs (int8) or float pairs with the largest |component|
        // reduced into vred (stash)
        const gptr<uint32_t> vsrc = global_ptr<uint32_t>(sd.volts) + static_cast<size_t>(c) * n_time * vwords;
        uint32_t pre[VPRE];
        auto fetch = [&](int t) {
            // 32-bit byte offsets from the sample's (uniform) base address
            const gptr<char> src = (gptr<char>)(vsrc + static_cast<size_t>(t) * vwords);
#pragma unroll
            for (int k = 0; k < VPRE; ++k) {
                const uint32_t off = static_cast<uint32_t>(min(tid + k * BLOCK, vwords - 1)) * 4u;
                pre[k] = *(gptr<uint32_t>)(src + off);
            }
        };
        auto stash = [&]() {
            float m = 0.f;
#pragma unroll
            for (int k = 0; k < VPRE; ++k) {
                const int i = tid + k * BLOCK;
                if (i < vwords) {
                    const uint32_t w = pre[k];
                    if constexpr (VT == EPIC_CI8) {
                        // four int8 components -> two exact FP16 pairs
                        const int8_t a = static_cast<int8_t>(w & 0xff), b = static_cast<int8_t>((w >> 8) & 0xff);
                        const int8_t cc = static_cast<int8_t>((w >> 16) & 0xff), dd = static_cast<int8_t>((w >> 24) & 0xff);
                        vf[2 * i] = pack2<EPIC_FP16_SPLIT>(static_cast<_Float16>(a), static_cast<_Float16>(b));
                        vf[2 * i + 1] = pack2<EPIC_FP16_SPLIT>(static_cast<_Float16>(cc), static_cast<_Float16>(dd));
                        const int mm = max(max(abs(static_cast<int>(a)), abs(static_cast<int>(b))),
                                           max(abs(static_cast<int>(cc)), abs(static_cast<int>(dd))));
                        m = fmaxf(m, static_cast<float>(mm));
                    } else {
                        vf[i] = w;
                        m = fmaxf(m, fabsf(__builtin_bit_cast(float, w)));
                    }
                }
            }
            for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
            if (lane == 0) vred[wave] = m;
        };
        auto volt = [&](int idx) -> float2 {
            if constexpr (VT == EPIC_CI8) {
                const uint32_t w = vf[idx];
                return make_float2(static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(w & 0xffff))),
                                   static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(w >> 16))));
            } else {
                return reinterpret_cast<const float2 *>(vf)[idx];
            }
        };
        fetch(0);
        stash();

        float acc[NT][4][NQ];
#pragma unroll
        for (int a = 0; a < NT; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int qq = 0; qq < NQ; ++qq) acc[a][i][qq] = 0.f;
        lds_barrier();

        for (int t = 0; t < n_time; ++t) {
            const bool has_next = t + 1 < n_time;
            if (has_next) fetch(t + 1);   // in flight during the gridding
            // ---- 1. grid the footprint box, scale, split -> G^T in LDS -------
            float vmax = 0.f;
#pragma unroll
            for (int w = 0; w < WAVES; ++w) vmax = fmaxf(vmax, vred[w]);
            const float s1 = pow2_scale(vmax * cp.wsum_max);
            {
                // G cells per thread at a time, tap index outermost, so that
                // the G cells' tap loads are in flight together; each cell
                // still adds its taps in list order
                constexpr int G = 4;
                // wave w takes the runs of 256 jobs w, w + 4, ...; lane l
                // the jobs 64 u + l of a run
                for (int j0 = 256 * wave + lane; j0 < njob; j0 += G * BLOCK) {
                    int k0[G], kn[G], cell[G], kmax = 0;
#pragma unroll
                    for (int u = 0; u < G; ++u) {
                        const int j = j0 + 64 * u;
                        const uint32_t job = j < njob ? jobs[j] : 0u;
                        if (sorted) {
                            cell[u] = static_cast<int>(job >> (kbits + 5));
                            kn[u] = static_cast<int>((job >> kbits) & 31u);
                            k0[u] = static_cast<int>(job & ((1u << kbits) - 1u));
                        } else {
                            cell[u] = j;
                            kn[u] = static_cast<int>(job & 31u);
                            k0[u] = static_cast<int>(job >> 5);
                        }
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
                                    const float2 e = volt(tp[u].elem * NP + p);
                                    a[u][p].x = fmaf(tp[u].w, e.x, a[u][p].x);
                                    a[u][p].y = fmaf(tp[u].w, e.y, a[u][p].y);
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < G; ++u) {
                        if (j0 + 64 * u >= njob) break;
                        const int i = cell[u];
                        // box row of cell i: (i + 1/2) / bw is at least 1/(2 bw)
                        // away from an integer, far more than its FP32 error
                        const int by = static_cast<int>((static_cast<float>(i) + 0.5f) * inv_bw);
                        const int bx = i - by * cp.bw;
#pragma unroll
                        for (int p = 0; p < NP; ++p) {
                            scalar hr, lr, hi_, li;
                            split<PREC>(a[u][p].x * s1, hr, lr);
                            split<PREC>(a[u][p].y * s1, hi_, li);
                            gbh[p * gplane + bx * d.pg + by] = pack2<PREC>(hr, hi_);
                            gbl[p * gplane + bx * d.pg + by] = pack2<PREC>(lr, li);
                        }
                    }
                }
            }
            lds_barrier();   // G^T complete; the sample's voltages and vred are free
            if (has_next) stash();

            // ---- 2. stage 1 per pol -> stage-2 A fragments --------------------
            vec8 a2[NP][T][2];   // [pol][x K-step][hi, lo] of (Re Y, Im Y) s2
            float inv[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                floatx4_t c1[T][2];   // [x tile][re, im]
#pragma unroll
                for (int mt = 0; mt < T; ++mt)
#pragma unroll
                    for (int o = 0; o < 2; ++o) c1[mt][o] = floatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < T; ++ks) {
                    if (ks >= my) break;
                    vec8 b1[4];
                    b1frag(ks, b1[0], b1[1], b1[2], b1[3]);
#pragma unroll
                    for (int mt = 0; mt < T; ++mt) {
                        if (mt >= mx) break;
                        const int off = p * gplane + (16 * mt + r16) * d.pg + 16 * ks + 4 * g;
                        const vec8 ah = __builtin_bit_cast(vec8, *reinterpret_cast<const u32x4_t *>(&gbh[off]));
                        const vec8 al = __builtin_bit_cast(vec8, *reinterpret_cast<const u32x4_t *>(&gbl[off]));
                        c1[mt][0] = mma3<PREC>(ah, al, b1[0], b1[1], c1[mt][0]);
                        c1[mt][1] = mma3<PREC>(ah, al, b1[2], b1[3], c1[mt][1]);
                    }
                }
                float ymax = 0.f;
#pragma unroll
                for (int mt = 0; mt < T; ++mt)
#pragma unroll
                    for (int o = 0; o < 2; ++o)
#pragma unroll
                        for (int i = 0; i < 4; ++i) ymax = fmaxf(ymax, fabsf(c1[mt][o][i]));
                for (int o = 32; o > 0; o >>= 1) ymax = fmaxf(ymax, __shfl_xor(ymax, o));
                const float s2 = pow2_scale(ymax);
                inv[p] = 1.f / (s1 * s2);
#pragma unroll
                for (int mt = 0; mt < T; ++mt) {
                    u32x4_t rh, rl;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        scalar hr, lr, hi_, li;
                        split<PREC>(c1[mt][0][i] * s2, hr, lr);
                        split<PREC>(c1[mt][1][i] * s2, hi_, li);
                        rh[i] = pack2<PREC>(hr, hi_);
                        rl[i] = pack2<PREC>(lr, li);
                    }
                    a2[p][mt][0] = __builtin_bit_cast(vec8, rh);
                    a2[p][mt][1] = __builtin_bit_cast(vec8, rl);
                }
            }
            lds_barrier();   // G^T is free for the next sample; its voltages are in LDS

            // ---- 3. stage 2 per 16 k_x, one set of B fragments for both pols;
            // 4. products ---------------------------------------------------------
            // a tile's DFT-row words at K-step ks; tile nt reads rows
            // 16 (nt & 1) + r16 of the table.  The row offset is opaque:
            // tiles 2m and 2m + 2 read the same rows, and sharing those loads
            // would hold them in registers across the tiles in between
            auto row_off = [&](int nt) {
                int f;
                asm volatile("v_mov_b32 %0, %1" : "=v"(f) : "v"((16 * (nt & 1) + r16) * d.pf + 4 * g));
                return f;
            };
            // wh, wl: on entry the words of this tile's first K-step, on exit
            // those of the next tile's (each K-step's successor is loaded
            // before its products, so the LDS latency overlaps them)
            auto tile = [&](auto m_tag, int nt, u32x4_t &wh, u32x4_t &wl) {
                constexpr int M = decltype(m_tag)::value;
                const int frow = row_off(nt), fnext = row_off(nt + 1);
                floatx4_t z[NP][2];
#pragma unroll
                for (int p = 0; p < NP; ++p) z[p][0] = z[p][1] = floatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < T; ++ks) {
                    if (ks >= mx) break;
                    const int o = ks + 1 < mx ? frow + 16 * (ks + 1) : fnext;
                    const u32x4_t nh = *reinterpret_cast<const u32x4_t *>(&fh[o]);
                    const u32x4_t nl = *reinterpret_cast<const u32x4_t *>(&fl[o]);
                    u32x4_t rh, ih, rl, il;
                    turned_block<M>(wh, rh, ih);
                    turned_block<M>(wl, rl, il);
                    const vec8 brh = __builtin_bit_cast(vec8, rh), brl = __builtin_bit_cast(vec8, rl);
                    const vec8 bih = __builtin_bit_cast(vec8, ih), bil = __builtin_bit_cast(vec8, il);
#pragma unroll
                    for (int p = 0; p < NP; ++p) {
                        z[p][0] = mma3<PREC>(a2[p][ks][0], a2[p][ks][1], brh, brl, z[p][0]);
                        z[p][1] = mma3<PREC>(a2[p][ks][0], a2[p][ks][1], bih, bil, z[p][1]);
                    }
                    wh = nh;
                    wl = nl;
                }
                // lane holds pixels (k_y = ky0 + 4 g + i, k_x = 16 nt + r16)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float xr = z[0][0][i] * inv[0], xi = z[0][1][i] * inv[0];
                    if constexpr (NP == 1) {
                        acc[nt][i][0] = fmaf(xr, xr, fmaf(xi, xi, acc[nt][i][0]));
                    } else {
                        const float yr = z[NP - 1][0][i] * inv[NP - 1], yi = z[NP - 1][1][i] * inv[NP - 1];
                        acc[nt][i][0] = fmaf(xr, xr, fmaf(xi, xi, acc[nt][i][0]));
                        acc[nt][i][1] = fmaf(xr, yr, fmaf(xi, yi, acc[nt][i][1]));
                        acc[nt][i][2] = fmaf(xi, yr, fmaf(-xr, yi, acc[nt][i][2]));
                        acc[nt][i][3] = fmaf(yr, yr, fmaf(yi, yi, acc[nt][i][3]));
                    }
                }
            };
            // scheduling barriers keep each tile's fragment loads with its
            // products instead of all eight tiles' loads up front
            u32x4_t wh, wl;
            {
                const int f0 = row_off(0);
                wh = *reinterpret_cast<const u32x4_t *>(&fh[f0]);
                wl = *reinterpret_cast<const u32x4_t *>(&fl[f0]);
            }
            __builtin_amdgcn_sched_barrier(0);
            tile(std::integral_constant<int, 0>{}, 0, wh, wl);
            __builtin_amdgcn_sched_barrier(0);
            tile(std::integral_constant<int, 0>{}, 1, wh, wl);
            __builtin_amdgcn_sched_barrier(0);
            tile(std::integral_constant<int, 1>{}, 2, wh, wl);
            __builtin_amdgcn_sched_barrier(0);
            tile(std::integral_constant<int, 1>{}, 3, wh, wl);
            __builtin_amdgcn_sched_barrier(0);
            tile(std::integral_constant<int, 2>{}, 4, wh, wl);
            __builtin_amdgcn_sched_barrier(0);
            tile(std::integral_constant<int, 2>{}, 5, wh, wl);
            __builtin_amdgcn_sched_barrier(0);
            tile(std::integral_constant<int, 3>{}, 6, wh, wl);
            __builtin_amdgcn_sched_barrier(0);
            tile(std::integral_constant<int, 3>{}, 7, wh, wl);
            __builtin_amdgcn_sched_barrier(0);

            // a block of samples ends: its sums go to the FP64 running sums
            if (block_ends(t, n_time, flush)) {
                int px0;   // opaque: keeps the addresses from being hoisted
                asm volatile("v_mov_b32 %0, %1" : "=v"(px0) : "v"((ky0 + 4 * g) * N + r16));
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int pix = px0 + i * N + 16 * nt;
#pragma unroll
                        for (int qq = 0; qq < NQ; ++qq) {
                            sums_add(sums, qq, pix, acc[nt][i][qq], t < flush);
                            acc[nt][i][qq] = 0.f;
                        }
                        asm volatile("" ::: "memory");
                    }
            }
        }
        sums_settle();
        const double inv_n = 1.0 / static_cast<double>(n_time);
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) sums_finish<NP>(sums, (ky0 + 4 * g + i) * N + 16 * nt + r16, inv_n);
    });
}

namespace {

template <int NP, int VT, int PREC>
epic_status run128(const FusedBatch &b, int n_time, int flush, const uint32_t *rows, hipStream_t stream)
{
    const Dft128Dims d = dims_of(b.max_bw, b.max_bh);
    const size_t bytes = dft128_lds_bytes(d, NP, VT, b.max_elem, b.max_cells);
    auto k = k_fused_dft128<NP, VT, PREC>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    const int grid = persistent_grid(reinterpret_cast<const void *>(k), kD128Block, bytes, b.n_items);
    KernelTimer timer("fused_dft128_cadence", stream);
    hipLaunchKernelGGL(k, dim3(grid), dim3(kD128Block), bytes, stream, b.sds, b.q, n_time, flush, rows,
                       b.max_elem, d);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

template <int PREC>
epic_status by_type128(const FusedBatch &b, int n_pol, int volt_type, int n_time, int flush,
                       const uint32_t *rows, hipStream_t stream)
{
    if (n_pol == 2 && volt_type == EPIC_CI8) return run128<2, EPIC_CI8, PREC>(b, n_time, flush, rows, stream);
    if (n_pol == 2) return run128<2, EPIC_CF32, PREC>(b, n_time, flush, rows, stream);
    if (volt_type == EPIC_CI8) return run128<1, EPIC_CI8, PREC>(b, n_time, flush, rows, stream);
    return run128<1, EPIC_CF32, PREC>(b, n_time, flush, rows, stream);
}

}  // namespace

epic_status launch_fused_dft128(const FusedBatch &b, int n_pol, int n_time, int volt_type, int precision,
                                int flush, const uint32_t *rows, hipStream_t stream)
{
    if (precision == EPIC_FP16_SPLIT)
        return by_type128<EPIC_FP16_SPLIT>(b, n_pol, volt_type, n_time, flush, rows, stream);
    return by_type128<EPIC_BF16_SPLIT>(b, n_pol, volt_type, n_time, flush, rows, stream);
}

bool fused_dft128_supported(const FusedBatch &b, int n_pol, int volt_type)
{
    if (b.n != 128) return false;
    if (b.max_bw > 16 * kD128Tiles || b.max_bh > 16 * kD128Tiles || b.max_bw < 1 || b.max_bh < 1) return false;
    const int64_t vbytes = static_cast<int64_t>(b.max_elem) * n_pol * (volt_type == EPIC_CI8 ? 2 : 8);
    if (vbytes % 4 != 0) return false;
    const int vpre = volt_type == EPIC_CI8 ? VoltPre<EPIC_CI8>::value : VoltPre<EPIC_CF32>::value;
    if (vbytes / 4 > static_cast<int64_t>(vpre) * kD128Block) return false;
    if (b.max_cell_taps > 31 || static_cast<int64_t>(b.max_elem) * b.max_ktaps >= (int64_t(1) << 27)) return false;
    return dft128_lds_bytes(dims_of(b.max_bw, b.max_bh), n_pol, volt_type, b.max_elem, b.max_cells) <= kD128Lds;
}

}  // namespace epic
