// k_dft.hip -- the 2-D transform of Eq. 3 (outer sum) as dense DFT-matrix
// products on gfx950 matrix cores, in split precision (EPIC_FP16_SPLIT /
// EPIC_BF16_SPLIT): Z = F_y . X . F_x^T with F_n[k][j] = exp(+2 pi i k j / n).
//
// One pass computes, for every batch item, P = F_n . X (X: [n][m] complex,
// transform along the first axis) and stores P transposed ([m][n]).  Two
// passes, the second on the first's output, give the 2-D transform in natural
// layout.  The DFT matrix is generated on the host in FP64 (angle reduced as
// the integer (k j mod n) / n), split into hi + lo parts and stored in MFMA
// A-fragment order.  Each work-group scales its block of input columns by a
// power of two so the FP16 parts cannot overflow (exact, undone on store).
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"
#include "mfma_split.hpp"

namespace epic {

epic_status cache_dft_table(int n, int precision, int device, size_t bytes,
                            void (*fill)(int, int, void *), const void **out);

namespace {

// Host: complex DFT matrix of size n as the real 2x2-block A operand.
// Row m of an M-tile holds output k = 8 mt + m/2, part m%2 (re, im); K entry
// kk of a K-step holds input j = 16 ks + kk/2, part kk%2.
template <typename T>
void fill_tables(int n, void *dst)
{
    const int MT = 2 * n / 16, KS = n / 16;
    T *hi = static_cast<T *>(dst);
    T *lo = hi + static_cast<size_t>(MT) * KS * 64 * 8;
    const double two_pi = 6.283185307179586476925286766559;
    for (int mt = 0; mt < MT; ++mt)
        for (int ks = 0; ks < KS; ++ks)
            for (int lane = 0; lane < 64; ++lane)
                for (int r = 0; r < 8; ++r) {
                    const int m = lane % 16, kk = 8 * (lane / 16) + r;
                    const long k = 8 * mt + m / 2, j = 16 * ks + kk / 2;
                    const double ang = two_pi * static_cast<double>((k * j) % n) / n;
                    const double fr = std::cos(ang), fi = std::sin(ang);
                    const bool out_im = (m % 2) == 1, in_im = (kk % 2) == 1;
                    const double v = !out_im ? (!in_im ? fr : -fi) : (!in_im ? fi : fr);
                    const T h = static_cast<T>(v);
                    const T l = static_cast<T>(v - static_cast<double>(h));
                    const size_t idx = ((static_cast<size_t>(mt) * KS + ks) * 64 + lane) * 8 + r;
                    hi[idx] = h;
                    lo[idx] = l;
                }
}

void fill_any(int n, int precision, void *dst)
{
    if (precision == EPIC_FP16_SPLIT)
        fill_tables<_Float16>(n, dst);
    else
        fill_tables<__bf16>(n, dst);
}

}  // namespace

// Host: rows of the DFT matrix as (re, im) pairs, [k][j] = exp(+2 pi i k j / n),
// hi parts then lo parts, each pair packed into 32 bits (re low, im high).
template <typename T>
void fill_rows(int n, void *dst)
{
    T *hi = static_cast<T *>(dst);
    T *lo = hi + static_cast<size_t>(n) * n * 2;
    const double two_pi = 6.283185307179586476925286766559;
    for (long k = 0; k < n; ++k)
        for (long j = 0; j < n; ++j) {
            const double ang = two_pi * static_cast<double>((k * j) % n) / n;
            const double v[2] = {std::cos(ang), std::sin(ang)};
            for (int part = 0; part < 2; ++part) {
                const T h = static_cast<T>(v[part]);
                const T l = static_cast<T>(v[part] - static_cast<double>(h));
                hi[(k * n + j) * 2 + part] = h;
                lo[(k * n + j) * 2 + part] = l;
            }
        }
}

void fill_rows_any(int n, int precision, void *dst)
{
    if ((precision & 0xf) == EPIC_FP16_SPLIT)
        fill_rows<_Float16>(n, dst);
    else
        fill_rows<__bf16>(n, dst);
}

epic_status get_dft_rows(int n, int precision, int device, const uint32_t **out)
{
    const size_t bytes = static_cast<size_t>(n) * n * 4 * 2;
    const void *p = nullptr;
    epic_status s = cache_dft_table(n, precision | 0x10, device, bytes, fill_rows_any, &p);
    *out = static_cast<const uint32_t *>(p);
    return s;
}

epic_status get_dft_tables(int n, int precision, int device, const void **out)
{
    const size_t bytes = static_cast<size_t>(2 * n / 16) * (n / 16) * 64 * 8 * 2 * 2;
    return cache_dft_table(n, precision, device, bytes, fill_any, out);
}

// With chan set (the composed cadence), item item0 + b belongs to channel
// (item0 + b) / items_per_chan and only the K-steps that cover the channel's footprint
// along the transformed axis are summed (the rest of the input is zero); on
// the first axis (axis 0, along y) work-groups whose columns miss the
// footprint write nothing, since the second pass sums only footprint rows.
template <int N, int NTW, int PREC>
__global__ __launch_bounds__(256) void k_dft_pass(const float2 *__restrict__ in,
                                                  float2 *__restrict__ out, int M,
                                                  const typename Split<PREC>::vec8 *__restrict__ tab,
                                                  const ChanPlan *__restrict__ chan,
                                                  int64_t item0, int items_per_chan, int axis)
{
    using S = Split<PREC>;
    using vec8 = typename S::vec8;
    using scalar = typename S::scalar;
    constexpr int CB = 16 * NTW;          // input columns per work-group
    constexpr int MT = 2 * N / 16;        // real M-tiles of P
    constexpr int KS = N / 16;            // K-steps
    constexpr int MTW = (MT + 3) / 4;     // M-tiles per wave
    constexpr int JP = N + 4;             // LDS pitch (packed complex) per column
    extern __shared__ __align__(16) uint32_t lds[];
    uint32_t *lhi = lds;                  // [CB][JP] (re, im) hi parts
    uint32_t *llo = lds + CB * JP;        // [CB][JP] lo parts
    __shared__ float red[4];

    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int g = lane / 16, r = lane % 16;
    const size_t b = blockIdx.y;
    const int c0 = blockIdx.x * CB;
    const float2 *src = in + b * N * M;
    int ks_lo = 0, ks_hi = KS - 1;
    if (chan) {
        const ChanPlan cp = chan[(item0 + static_cast<int64_t>(b)) / items_per_chan];
        const int lo = axis == 0 ? cp.y0 : cp.x0, len = axis == 0 ? cp.bh : cp.bw;
        ks_lo = lo >> 4;
        ks_hi = (lo + len - 1) >> 4;
        if (axis == 0 && (c0 + CB <= cp.x0 || c0 >= cp.x0 + cp.bw)) return;
    }
    const int j_lo = 16 * ks_lo, nrows = 16 * (ks_hi - ks_lo + 1);

    // the block's input, read once into registers (rows past the pruned
    // range read as zero)
    constexpr int PER = N * CB / 256;
    float2 xin[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = threadIdx.x + 256 * q;
        xin[q] = i < nrows * CB ? src[(j_lo + i / CB) * M + c0 + i % CB] : make_float2(0.f, 0.f);
    }
    float s = 1.f;
    if constexpr (S::needs_scale) {
        float mx = 0.f;
#pragma unroll
        for (int q = 0; q < PER; ++q) mx = fmaxf(mx, fmaxf(fabsf(xin[q].x), fabsf(xin[q].y)));
        for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
        if (lane == 0) red[wave] = mx;
        __syncthreads();
        mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        s = pow2_scale(mx);
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = threadIdx.x + 256 * q;
        if (i >= nrows * CB) break;
        const int j = j_lo + i / CB, c = i % CB;
        scalar hr, lr, hi_, li;
        split<PREC>(xin[q].x * s, hr, lr);
        split<PREC>(xin[q].y * s, hi_, li);
        const uint32_t ph = static_cast<uint32_t>(__builtin_bit_cast(uint16_t, hr)) |
                            (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, hi_)) << 16);
        const uint32_t pl = static_cast<uint32_t>(__builtin_bit_cast(uint16_t, lr)) |
                            (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, li)) << 16);
        lhi[c * JP + j] = ph;
        llo[c * JP + j] = pl;
    }
    __syncthreads();

    floatx4_t acc[MTW][NTW];
#pragma unroll
    for (int w = 0; w < MTW; ++w)
#pragma unroll
        for (int t = 0; t < NTW; ++t) acc[w][t] = floatx4_t{0.f, 0.f, 0.f, 0.f};

    // DFT-table fragments double-buffered: step ks + 1's loads are in flight
    // while step ks's products run
    const vec8 *tab_lo = tab + static_cast<size_t>(MT) * KS * 64;
    auto load_a = [&](int ks, vec8 *ah, vec8 *al) {
#pragma unroll
        for (int w = 0; w < MTW; ++w) {
            const int mt = wave + 4 * w;
            if (mt < MT) {
                ah[w] = tab[(mt * KS + ks) * 64 + lane];
                al[w] = tab_lo[(mt * KS + ks) * 64 + lane];
            }
        }
    };
    auto step = [&](int ks, const vec8 *ah, const vec8 *al) {
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            const int c = t * 16 + r, j0 = ks * 16 + 4 * g;
            const vec8 bh = *reinterpret_cast<const vec8 *>(&lhi[c * JP + j0]);
            const vec8 bl = *reinterpret_cast<const vec8 *>(&llo[c * JP + j0]);
#pragma unroll
            for (int w = 0; w < MTW; ++w)
                if (wave + 4 * w < MT) acc[w][t] = mma3<PREC>(ah[w], al[w], bh, bl, acc[w][t]);
        }
    };
    vec8 ah0[MTW], al0[MTW], ah1[MTW], al1[MTW];
    load_a(ks_lo, ah0, al0);
    for (int ks = ks_lo; ks <= ks_hi; ks += 2) {
        if (ks + 1 <= ks_hi) load_a(ks + 1, ah1, al1);
        step(ks, ah0, al0);
        if (ks + 1 > ks_hi) break;
        if (ks + 2 <= ks_hi) load_a(ks + 2, ah0, al0);
        step(ks + 1, ah1, al1);
    }

    const float inv = 1.f / s;
#pragma unroll
    for (int w = 0; w < MTW; ++w) {
        const int mt = wave + 4 * w;
        if (mt >= MT) continue;
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            const int c = c0 + t * 16 + r;
            const int k = mt * 8 + 2 * g;
            const floatx4_t a = acc[w][t];
            float4 v = make_float4(a[0] * inv, a[1] * inv, a[2] * inv, a[3] * inv);
            *reinterpret_cast<float4 *>(&out[(b * M + c) * N + k]) = v;
        }
    }
}

// The whole 2-D transform of one N x N plane (N <= 64) in one work-group:
// the pass along y leaves its result in LDS, rescaled by a new power of two
// and re-split, as the operand of the pass along x, so HBM sees the plane
// once in and once out (the two-launch form writes and re-reads the
// intermediate).  Same fragments, tables and arithmetic as k_dft_pass.
template <int N, int PREC>
__global__ __launch_bounds__(256) void k_dft2_plane(const float2 *__restrict__ in,
                                                    float2 *__restrict__ out,
                                                    const typename Split<PREC>::vec8 *__restrict__ tab)
{
    using S = Split<PREC>;
    using vec8 = typename S::vec8;
    using scalar = typename S::scalar;
    constexpr int NTW = N / 16;           // column tiles: the whole plane
    constexpr int MT = 2 * N / 16;        // real M-tiles
    constexpr int KS = N / 16;            // K-steps
    constexpr int MTW = (MT + 3) / 4;     // M-tiles per wave
    constexpr int JP = N + 4;             // LDS pitch (packed complex) per column
    constexpr int PER = N * N / 256;      // plane values per thread
    extern __shared__ __align__(16) uint32_t lds[];
    uint32_t *lhi = lds;                  // [N][JP]: column c, transform index j
    uint32_t *llo = lds + N * JP;
    __shared__ float red[4];

    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int g = lane / 16, r = lane % 16;
    const size_t b = blockIdx.x;
    const float2 *src = in + b * N * N;
    const vec8 *tab_lo = tab + static_cast<size_t>(MT) * KS * 64;

    auto block_max = [&](float mx) {
        for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
        __syncthreads();                  // red[] of an earlier use has been read
        if (lane == 0) red[wave] = mx;
        __syncthreads();
        return fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    };
    auto put = [&](int c, int j, float re, float im) {
        scalar hr, lr, hi_, li;
        split<PREC>(re, hr, lr);
        split<PREC>(im, hi_, li);
        lhi[c * JP + j] = static_cast<uint32_t>(__builtin_bit_cast(uint16_t, hr)) |
                          (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, hi_)) << 16);
        llo[c * JP + j] = static_cast<uint32_t>(__builtin_bit_cast(uint16_t, lr)) |
                          (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, li)) << 16);
    };
    floatx4_t acc[MTW][NTW];
    auto transform = [&]() {              // acc = F . (LDS operand), both split parts
#pragma unroll
        for (int w = 0; w < MTW; ++w)
#pragma unroll
            for (int t = 0; t < NTW; ++t) acc[w][t] = floatx4_t{0.f, 0.f, 0.f, 0.f};
        // every K step's table fragments are loaded before the first product
        vec8 ah[KS][MTW], al[KS][MTW];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int w = 0; w < MTW; ++w) {
                const int mt = wave + 4 * w;
                if (mt < MT) {
                    ah[ks][w] = tab[(mt * KS + ks) * 64 + lane];
                    al[ks][w] = tab_lo[(mt * KS + ks) * 64 + lane];
                }
            }
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
            for (int t = 0; t < NTW; ++t) {
                const int c = t * 16 + r, j0 = ks * 16 + 4 * g;
                const vec8 bh = *reinterpret_cast<const vec8 *>(&lhi[c * JP + j0]);
                const vec8 bl = *reinterpret_cast<const vec8 *>(&llo[c * JP + j0]);
#pragma unroll
                for (int w = 0; w < MTW; ++w)
                    if (wave + 4 * w < MT) acc[w][t] = mma3<PREC>(ah[ks][w], al[ks][w], bh, bl, acc[w][t]);
            }
        }
    };

    // pass along y: operand column x, index y
    float2 xin[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) xin[q] = src[threadIdx.x + 256 * q];
    float s1 = 1.f;
    if constexpr (S::needs_scale) {
        float mx = 0.f;
#pragma unroll
        for (int q = 0; q < PER; ++q) mx = fmaxf(mx, fmaxf(fabsf(xin[q].x), fabsf(xin[q].y)));
        s1 = pow2_scale(block_max(mx));
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = threadIdx.x + 256 * q;          // i = y * N + x
        put(i % N, i / N, xin[q].x * s1, xin[q].y * s1);
    }
    __syncthreads();
    transform();                                      // acc: P[k_y][x] * s1

    // pass along x: operand column k_y, index x, rescaled for the split
    float s2 = 1.f / s1;
    if constexpr (S::needs_scale) {
        float mx = 0.f;
#pragma unroll
        for (int w = 0; w < MTW; ++w)
#pragma unroll
            for (int t = 0; t < NTW; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) mx = fmaxf(mx, fabsf(acc[w][t][e]));
        const float m = block_max(mx) / s1;           // largest |P| component
        s2 = pow2_scale(m) / s1;                      // exact: powers of two
    }
    __syncthreads();                                  // every pass-1 operand read
#pragma unroll
    for (int w = 0; w < MTW; ++w) {
        const int mt = wave + 4 * w;
        if (mt >= MT) continue;
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            const int x = t * 16 + r, k = mt * 8 + 2 * g;
            const floatx4_t a = acc[w][t];
            put(k, x, a[0] * s2, a[1] * s2);
            put(k + 1, x, a[2] * s2, a[3] * s2);
        }
    }
    __syncthreads();
    transform();                                      // acc: Z[k_y][k_x] * (s1 s2)
    const float inv = 1.f / (s1 * s2);
#pragma unroll
    for (int w = 0; w < MTW; ++w) {
        const int mt = wave + 4 * w;
        if (mt >= MT) continue;
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
            const int ky = t * 16 + r, kx = mt * 8 + 2 * g;
            const floatx4_t a = acc[w][t];
            *reinterpret_cast<float4 *>(&out[(b * N + ky) * N + kx]) =
                make_float4(a[0] * inv, a[1] * inv, a[2] * inv, a[3] * inv);
        }
    }
}

// acc[w][t] = sum over K tiles 0 .. nks - 1 of the 128-point DFT table's
// M-tile mt0 + mt_step w times the LDS operand's column tile col0 + t
// (t < ncols <= TMAX; operand pitch jp words per column), both split parts.
// The table fragments are double-buffered: step s + 1's loads are in flight
// while step s's products run.
template <int PREC, int MTW, int TMAX>
__device__ __forceinline__ void tile_products128(floatx4_t (&acc)[MTW][TMAX],
                                                 const typename Split<PREC>::vec8 *__restrict__ tab,
                                                 const uint32_t *lhi, const uint32_t *llo, int mt0,
                                                 int mt_step, int nks, int col0, int ncols, int jp)
{
    using vec8 = typename Split<PREC>::vec8;
    constexpr int MT = 16, KS = 8;
    const int lane = threadIdx.x % 64, g = lane / 16, r = lane % 16;
    const vec8 *tab_lo = tab + MT * KS * 64;
#pragma unroll
    for (int w = 0; w < MTW; ++w)
#pragma unroll
        for (int t = 0; t < TMAX; ++t) acc[w][t] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    auto load_a = [&](int ks, vec8 *ah, vec8 *al) {
#pragma unroll
        for (int w = 0; w < MTW; ++w) {
            const int i = ((mt0 + mt_step * w) * KS + ks) * 64 + lane;
            ah[w] = tab[i];
            al[w] = tab_lo[i];
        }
    };
    auto step = [&](int s, const vec8 *ah, const vec8 *al) {
#pragma unroll
        for (int t = 0; t < TMAX; ++t) {
            if (t >= ncols) break;
            const int o = ((col0 + t) * 16 + r) * jp + s * 16 + 4 * g;
            const vec8 bh = *reinterpret_cast<const vec8 *>(&lhi[o]);
            const vec8 bl = *reinterpret_cast<const vec8 *>(&llo[o]);
#pragma unroll
            for (int w = 0; w < MTW; ++w) acc[w][t] = mma3<PREC>(ah[w], al[w], bh, bl, acc[w][t]);
        }
    };
    vec8 ah0[MTW], al0[MTW], ah1[MTW], al1[MTW];
    load_a(0, ah0, al0);
    for (int s = 0; s < nks; s += 2) {
        if (s + 1 < nks) load_a(s + 1, ah1, al1);
        step(s, ah0, al0);
        if (s + 1 >= nks) break;
        if (s + 2 < nks) load_a(s + 2, ah0, al0);
        step(s + 1, ah1, al1);
    }
}

// The 2-D transform of one 128 x 128 plane in one work-group, summing over the
// box of its non-zero cells only.  The box comes from the channel's footprint
// (chan set: only the box is read) or, for a dense call, from the plane itself
// (every cell is read).  The sums run over 16-cell tiles counted from the
// box's first cell (x0, y0), moved back where the tiles would pass the
// plane's edge, so a box w cells wide takes ceil(w / 16) tiles; by the
// shift theorem the transform of the shifted operand times
// exp(+2 pi i (kx x0 + ky y0) / 128) is the transform of the plane (the
// factors from an FP64 table).  The longer side (ka tiles) is transformed
// first over the cb <= ka tile columns of the other side; the second pass
// then sums cb tiles for all 128 outputs of the first, so the LDS holds at
// most 2 x max(16 cb (16 ka + 4), 128 (16 cb + 4)) words (the operands of the
// two passes, hi and lo parts, one after the other).  Cells outside the box
// add exact zeros, so the result depends only on the box.  Fragments,
// tables, scaling and split as in k_dft2_plane.
//
// Every wave multiplies a pair of M-tiles (p, p + 8) by up to 4 column tiles,
// so each operand fragment read from LDS feeds six products.  NW = 16 waves
// (any box): pair wave % 8, column tiles 4 (wave / 8) .. + 3 in both passes.
// NW = 8 waves (footprint boxes with cb <= 4, which need at most 68 KB of
// LDS, so two work-groups share a compute unit): pair wave, all cb column
// tiles in the first pass, and the two column halves in two rounds in the
// second, each stored as it ends.
template <int PREC, int NW>
__global__ __launch_bounds__(64 * NW, NW == 8 ? 4 : 1)
void k_dft2_tiles128(const float2 *__restrict__ in, float2 *__restrict__ out,
                     const typename Split<PREC>::vec8 *__restrict__ tab,
                     const float2 *__restrict__ phase, const ChanPlan *__restrict__ chan,
                     int64_t item0, int items_per_chan, int lds_words)
{
    static_assert(NW == 16 || NW == 8, "16 or 8 waves");
    using S = Split<PREC>;
    using scalar = typename S::scalar;
    constexpr int N = 128, KS = 8, NT = 64 * NW;
    constexpr int SLOTS = NT / 256;       // tiles read at once (256 threads per tile)
    constexpr int MAX_TILES = NW == 16 ? 64 : 32;
    constexpr int PER = MAX_TILES / SLOTS;
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ float red[NW];
    __shared__ int redi[4][NW];
    __shared__ float2 ph[N];              // the shift-theorem factors

    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int g = lane / 16, r = lane % 16;
    const int tid = threadIdx.x;
    const size_t b = blockIdx.x;
    const float2 *src = in + b * N * N;
    float2 *dst = out + b * N * N;
    if (tid < N) ph[tid] = phase[tid];    // read after the barriers below

    // block-wide max; each use is separated from the previous one's reads of
    // red[] by a barrier of the caller's (the one before the first pass)
    auto block_max = [&](float mx) {
        for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
        if (lane == 0) red[wave] = mx;
        __syncthreads();
        float m = red[0];
#pragma unroll
        for (int w = 1; w < NW; ++w) m = fmaxf(m, red[w]);
        return m;
    };

    // the region read (first cell x0, y0; sx x sy tiles): the footprint
    // box's tiles, or the whole plane
    int x0 = 0, y0 = 0, sx = KS, sy = KS;
    if (chan) {
        const ChanPlan cp = chan[(item0 + static_cast<int64_t>(b)) / items_per_chan];
        tile_span(cp.x0, cp.bw, N, x0, sx);
        tile_span(cp.y0, cp.bh, N, y0, sy);
    }
    if (sx * sy > MAX_TILES || (NW == 8 && min(sx, sy) > 4)) return;   // the host dispatches by box size
    // thread: cell (tid % 16, (tid / 16) % 16) of tiles tid / 256, + SLOTS,
    // + 2 SLOTS, ... of the region in raster order; tt / sx by multiply-shift
    // (exact for tile indices below 64 and sx <= 8)
    const uint32_t inv_sx = (65536u + sx - 1) / sx;
    const int cx = tid % 16, cy = (tid / 16) % 16, slot = tid / 256;
    const int rsx = sx, rx0 = x0, ry0 = y0, n_tiles = sx * sy;   // the region read
    float2 xin[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int tt = slot + SLOTS * q;
        xin[q] = make_float2(0.f, 0.f);
        if (tt < n_tiles) {
            const int tr = static_cast<int>((static_cast<uint32_t>(tt) * inv_sx) >> 16), tc = tt - tr * sx;
            xin[q] = src[(y0 + tr * 16 + cy) * N + x0 + tc * 16 + cx];
        }
    }
    if (!chan) {
        // dense call: the box of the non-zero cells
        int lo_x = N, hi_x = -1, lo_y = N, hi_y = -1;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int tt = slot + SLOTS * q;
            if (xin[q].x != 0.f || xin[q].y != 0.f) {
                const int x = (tt % KS) * 16 + cx, y = (tt / KS) * 16 + cy;
                lo_x = min(lo_x, x);
                hi_x = max(hi_x, x);
                lo_y = min(lo_y, y);
                hi_y = max(hi_y, y);
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            lo_x = min(lo_x, __shfl_xor(lo_x, o));
            hi_x = max(hi_x, __shfl_xor(hi_x, o));
            lo_y = min(lo_y, __shfl_xor(lo_y, o));
            hi_y = max(hi_y, __shfl_xor(hi_y, o));
        }
        if (lane == 0) {
            redi[0][wave] = lo_x;
            redi[1][wave] = hi_x;
            redi[2][wave] = lo_y;
            redi[3][wave] = hi_y;
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            lo_x = min(lo_x, redi[0][w]);
            hi_x = max(hi_x, redi[1][w]);
            lo_y = min(lo_y, redi[2][w]);
            hi_y = max(hi_y, redi[3][w]);
        }
        if (hi_x < 0) {                   // an all-zero plane
            for (int i = tid; i < N * N; i += NT) dst[i] = make_float2(0.f, 0.f);
            return;
        }
        tile_span(lo_x, hi_x - lo_x + 1, N, x0, sx);
        tile_span(lo_y, hi_y - lo_y + 1, N, y0, sy);
    }
    const bool x_first = sx > sy;         // the longer side first
    const int ka = x_first ? sx : sy, cb = x_first ? sy : sx;
    const int jp1 = 16 * ka + 4, jp2 = 16 * cb + 4;   // LDS pitches (words per column)
    const int half = max(16 * cb * jp1, N * jp2);
    if (2 * half > lds_words) return;     // cannot happen: the host sizes the LDS for the box
    uint32_t *lhi = lds, *llo = lds + half;

    auto put = [&](int o, float re, float im) {     // o: word offset in the operand
        scalar hr, lr, hi_, li;
        split<PREC>(re, hr, lr);
        split<PREC>(im, hi_, li);
        lhi[o] = static_cast<uint32_t>(__builtin_bit_cast(uint16_t, hr)) |
                 (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, hi_)) << 16);
        llo[o] = static_cast<uint32_t>(__builtin_bit_cast(uint16_t, lr)) |
                 (static_cast<uint32_t>(__builtin_bit_cast(uint16_t, li)) << 16);
    };

    // pass 1 along the longer side: operand column = position along the
    // shorter side, index = position along the longer side (box-relative)
    float s1 = 1.f;
    if constexpr (S::needs_scale) {
        float mx = 0.f;
#pragma unroll
        for (int q = 0; q < PER; ++q) mx = fmaxf(mx, fmaxf(fabsf(xin[q].x), fabsf(xin[q].y)));
        s1 = pow2_scale(block_max(mx));
    }
    {
        const uint32_t inv_r = (65536u + rsx - 1) / rsx;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int tt = slot + SLOTS * q;
            if (tt >= n_tiles) break;
            const int tr = static_cast<int>((static_cast<uint32_t>(tt) * inv_r) >> 16), tc = tt - tr * rsx;
            const int dx = rx0 + tc * 16 + cx - x0, dy = ry0 + tr * 16 + cy - y0;  // box-relative
            if (dx < 0 || dx >= 16 * sx || dy < 0 || dy >= 16 * sy) continue;
            const int c = x_first ? dy : dx, j = x_first ? dx : dy;
            put(c * jp1 + j, xin[q].x * s1, xin[q].y * s1);
        }
    }
    __syncthreads();
    const int pair = wave % 8, col1 = NW == 16 ? 4 * (wave / 8) : 0;
    const int n1 = min(4, max(0, cb - col1));         // this wave's pass-1 column tiles
    floatx4_t acc1[2][4];                 // P[k1][c] * s1, k1 along the longer side
    tile_products128<PREC, 2, 4>(acc1, tab, lhi, llo, pair, 8, ka, col1, n1, jp1);

    // pass 2 along the shorter side: operand column k1, index c
    float s2 = 1.f / s1;
    if constexpr (S::needs_scale) {
        float mx = 0.f;
#pragma unroll
        for (int w = 0; w < 2; ++w)
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) mx = fmaxf(mx, fabsf(acc1[w][t][e]));
        // its barrier also comes after every pass-1 operand read
        const float m = block_max(mx) / s1;           // largest |P| component
        s2 = pow2_scale(m) / s1;                      // exact: powers of two
    } else {
        __syncthreads();                              // every pass-1 operand read
    }
#pragma unroll
    for (int w = 0; w < 2; ++w) {
        const int k1 = (pair + 8 * w) * 8 + 2 * g;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t >= n1) break;
            const int c = (col1 + t) * 16 + r;
            const floatx4_t a = acc1[w][t];
            put(k1 * jp2 + c, a[0] * s2, a[1] * s2);
            put((k1 + 1) * jp2 + c, a[2] * s2, a[3] * s2);
        }
    }
    __syncthreads();
    const float inv = 1.f / (s1 * s2);
    // the shift back: output (kx, ky) times phase[(kx x0 + ky y0) mod 128]
    const int s1x = x_first ? x0 : y0, s2x = x_first ? y0 : x0;   // shifts along k1, k2
    auto rot = [&](float re, float im, int m) {
        const float2 w = ph[m & (N - 1)];
        return make_float2((re * w.x - im * w.y) * inv, (re * w.y + im * w.x) * inv);
    };
#pragma unroll
    for (int round = 0; round < 16 / NW; ++round) {
        const int col2 = NW == 16 ? 4 * (wave / 8) : 4 * round;
        floatx4_t acc[2][4];              // Z[k2][k1] * (s1 s2), k2 along the shorter side
        tile_products128<PREC, 2, 4>(acc, tab, lhi, llo, pair, 8, cb, col2, 4, jp2);
#pragma unroll
        for (int w = 0; w < 2; ++w) {
            const int k2 = (pair + 8 * w) * 8 + 2 * g;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int k1 = (col2 + t) * 16 + r;
                const floatx4_t a = acc[w][t];
                const int m = k1 * s1x + k2 * s2x;
                const float2 v0 = rot(a[0], a[1], m), v1 = rot(a[2], a[3], m + s2x);
                if (x_first) {            // k1 = kx, k2 = ky
                    dst[k2 * N + k1] = v0;
                    dst[(k2 + 1) * N + k1] = v1;
                } else {                  // k1 = ky, k2 = kx
                    *reinterpret_cast<float4 *>(&dst[k1 * N + k2]) = make_float4(v0.x, v0.y, v1.x, v1.y);
                }
            }
        }
    }
}

namespace {

struct Prune {
    const ChanPlan *chan;   // null: dense
    int items_per_chan;
    int axis;
};

template <int N, int NTW, int PREC>
epic_status run_pass(int64_t batch, int m, const float2 *in, float2 *out, const void *tab,
                     const Prune &pr, hipStream_t stream)
{
    constexpr int CB = 16 * NTW;
    const size_t bytes = sizeof(uint32_t) * 2 * CB * (N + 4);
    auto k = k_dft_pass<N, NTW, PREC>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(bytes));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    KernelTimer timer("dft_gemm_pass", stream);
    for (int64_t b0 = 0; b0 < batch; b0 += 65535) {
        const int64_t nb = std::min<int64_t>(65535, batch - b0);
        hipLaunchKernelGGL(k, dim3(m / CB, static_cast<unsigned>(nb)), dim3(256), bytes, stream,
                           in + b0 * N * m, out + b0 * N * m, m,
                           static_cast<const typename Split<PREC>::vec8 *>(tab), pr.chan, b0,
                           pr.items_per_chan, pr.axis);
        EPIC_HIP_TRY(hipGetLastError());
    }
    return EPIC_OK;
}

template <int N, int PREC>
epic_status pass_n(int64_t batch, int m, const float2 *in, float2 *out, const void *tab,
                   const Prune &pr, hipStream_t stream)
{
    // columns per work-group: as many as the accumulators allow
    constexpr int MAX_NTW = N >= 128 ? 2 : 4;
    if (m >= 16 * MAX_NTW) return run_pass<N, MAX_NTW, PREC>(batch, m, in, out, tab, pr, stream);
    if (m >= 32) return run_pass<N, 2, PREC>(batch, m, in, out, tab, pr, stream);
    return run_pass<N, 1, PREC>(batch, m, in, out, tab, pr, stream);
}

template <int PREC>
epic_status pass_any(int n, int64_t batch, int m, const float2 *in, float2 *out, const void *tab,
                     const Prune &pr, hipStream_t stream)
{
    switch (n) {
    case 16: return pass_n<16, PREC>(batch, m, in, out, tab, pr, stream);
    case 32: return pass_n<32, PREC>(batch, m, in, out, tab, pr, stream);
    case 64: return pass_n<64, PREC>(batch, m, in, out, tab, pr, stream);
    case 128: return pass_n<128, PREC>(batch, m, in, out, tab, pr, stream);
    case 256: return pass_n<256, PREC>(batch, m, in, out, tab, pr, stream);
    }
    return fail(EPIC_ERR_INTERNAL, "dft pass: unexpected size");
}

template <int N, int PREC>
epic_status dft2_plane(int64_t batch, const float2 *in, float2 *out, const void *tab, hipStream_t stream)
{
    const size_t bytes = sizeof(uint32_t) * 2 * N * (N + 4);
    auto k = k_dft2_plane<N, PREC>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(bytes));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    KernelTimer timer("dft2_plane", stream);
    for (int64_t b0 = 0; b0 < batch; b0 += (int64_t{1} << 30)) {
        const int64_t nb = std::min<int64_t>(int64_t{1} << 30, batch - b0);
        hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(nb)), dim3(256), bytes, stream,
                           in + b0 * N * N, out + b0 * N * N,
                           static_cast<const typename Split<PREC>::vec8 *>(tab));
        EPIC_HIP_TRY(hipGetLastError());
    }
    return EPIC_OK;
}

epic_status dft2_plane_any(int n, int64_t batch, int precision, const float2 *in, float2 *out,
                           int device, hipStream_t stream)
{
    const void *tab = nullptr;
    epic_status s = get_dft_tables(n, precision, device, &tab);
    if (s != EPIC_OK) return s;
    const bool f16 = precision == EPIC_FP16_SPLIT;
    switch (n) {
    case 16: return f16 ? dft2_plane<16, EPIC_FP16_SPLIT>(batch, in, out, tab, stream)
                        : dft2_plane<16, EPIC_BF16_SPLIT>(batch, in, out, tab, stream);
    case 32: return f16 ? dft2_plane<32, EPIC_FP16_SPLIT>(batch, in, out, tab, stream)
                        : dft2_plane<32, EPIC_BF16_SPLIT>(batch, in, out, tab, stream);
    case 64: return f16 ? dft2_plane<64, EPIC_FP16_SPLIT>(batch, in, out, tab, stream)
                        : dft2_plane<64, EPIC_BF16_SPLIT>(batch, in, out, tab, stream);
    }
    return fail(EPIC_ERR_INTERNAL, "dft2 plane: unexpected size");
}

// exp(+2 pi i m / 128), m = 0 .. 127, as FP32 pairs from FP64
void fill_phase128(int n, int, void *dst)
{
    float2 *p = static_cast<float2 *>(dst);
    const double two_pi = 6.283185307179586476925286766559;
    for (int m = 0; m < n; ++m)
        p[m] = make_float2(static_cast<float>(std::cos(two_pi * m / n)),
                           static_cast<float>(std::sin(two_pi * m / n)));
}

epic_status get_phase128(int device, const void **out)
{
    return cache_dft_table(128, 0x20, device, sizeof(float2) * 128, fill_phase128, out);
}

template <int PREC>
epic_status dft2_tiles128(int64_t batch, const float2 *in, float2 *out, const void *tab,
                          const ChanPlan *chan, int items_per_chan, int max_bw, int max_bh,
                          hipStream_t stream, int device)
{
    // LDS for the largest box: w cells take ceil(w / 16) tiles; the longer
    // side is transformed first
    int sx = 8, sy = 8;
    if (chan) {
        sx = std::min(8, (max_bw + 15) / 16);
        sy = std::min(8, (max_bh + 15) / 16);
    }
    const void *phase = nullptr;
    epic_status s = get_phase128(device, &phase);
    if (s != EPIC_OK) return s;
    const int ka = std::max(sx, sy), cb = std::min(sx, sy);
    const int words = 2 * std::max(16 * cb * (16 * ka + 4), 128 * (16 * cb + 4));
    const size_t bytes = sizeof(uint32_t) * words;
    // footprint boxes no more than 4 tiles on their shorter side: 8 waves,
    // two work-groups per compute unit
    const bool small = chan && cb <= 4;
    auto k = small ? k_dft2_tiles128<PREC, 8> : k_dft2_tiles128<PREC, 16>;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(bytes));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    KernelTimer timer("dft2_tiles128", stream);
    for (int64_t b0 = 0; b0 < batch; b0 += (int64_t{1} << 30)) {
        const int64_t nb = std::min<int64_t>(int64_t{1} << 30, batch - b0);
        hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(nb)), dim3(small ? 512 : 1024), bytes, stream,
                           in + b0 * 128 * 128, out + b0 * 128 * 128,
                           static_cast<const typename Split<PREC>::vec8 *>(tab),
                           static_cast<const float2 *>(phase), chan, b0, items_per_chan, words);
        EPIC_HIP_TRY(hipGetLastError());
    }
    return EPIC_OK;
}

}  // namespace

bool split_reads_tile_region(int nx, int ny) { return nx == 128 && ny == 128; }

epic_status launch_dft2_split(int nx, int ny, int64_t batch, int precision, const float2 *in,
                              float2 *out, int device, hipStream_t stream, const ChanPlan *chan,
                              int items_per_chan, int max_bw, int max_bh)
{
    const Prune p1{chan, items_per_chan, 0}, p2{chan, items_per_chan, 1};
    if (split_reads_tile_region(nx, ny)) {
        if (chan && (max_bw <= 0 || max_bh <= 0))
            return fail(EPIC_ERR_INTERNAL, "dft2 split: footprint mode without box bounds");
        const void *tab = nullptr;
        epic_status s = get_dft_tables(128, precision, device, &tab);
        if (s != EPIC_OK) return s;
        return precision == EPIC_FP16_SPLIT
                   ? dft2_tiles128<EPIC_FP16_SPLIT>(batch, in, out, tab, chan, items_per_chan, max_bw,
                                                    max_bh, stream, device)
                   : dft2_tiles128<EPIC_BF16_SPLIT>(batch, in, out, tab, chan, items_per_chan, max_bw,
                                                    max_bh, stream, device);
    }
    if (!chan && nx == ny && nx <= 64) return dft2_plane_any(nx, batch, precision, in, out, device, stream);
    const void *tab_y = nullptr, *tab_x = nullptr;
    epic_status s = get_dft_tables(ny, precision, device, &tab_y);
    if (s != EPIC_OK) return s;
    s = get_dft_tables(nx, precision, device, &tab_x);
    if (s != EPIC_OK) return s;
    void *ws = nullptr;
    s = get_workspace(device, stream, 3, sizeof(float2) * static_cast<size_t>(batch) * nx * ny, &ws);
    if (s != EPIC_OK) return s;
    float2 *mid = static_cast<float2 *>(ws);
    // pass 1: along y (input [ny][nx]) -> [nx][ny]; pass 2: along x -> [ny][nx]
    if (precision == EPIC_FP16_SPLIT) {
        s = pass_any<EPIC_FP16_SPLIT>(ny, batch, nx, in, mid, tab_y, p1, stream);
        if (s != EPIC_OK) return s;
        return pass_any<EPIC_FP16_SPLIT>(nx, batch, ny, mid, out, tab_x, p2, stream);
    }
    s = pass_any<EPIC_BF16_SPLIT>(ny, batch, nx, in, mid, tab_y, p1, stream);
    if (s != EPIC_OK) return s;
    return pass_any<EPIC_BF16_SPLIT>(nx, batch, ny, mid, out, tab_x, p2, stream);
}

}  // namespace epic
