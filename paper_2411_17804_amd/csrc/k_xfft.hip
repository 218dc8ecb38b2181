// k_xfft.hip -- the XFFT route of Sec. 5.4 (Eq. 4 then Eq. 6): the
// correlator on matrix cores and the gridding of its visibilities with the
// cross-correlated element kernels.  The transform that follows is
// k_fft.hip's forward FP32 transform.
//
// Correlator: per channel, with rows r = a * n_pol + p (the order of the
// voltage layout) and X[r][t] the voltage of row r at sample t,
//     V[r][s] = (1/n_time) sum_t X[r][t] conj(X[s][t]),
// a Hermitian R x R product (R = n_elem * n_pol).  Work-groups own 64 x 64
// blocks (I, J) with J >= I; the block (J, I) is written as the conjugate
// transpose.  Complex products are four real ones,
//     Re V = Xr Xr^T + Xi Xi^T,   Im V = Xi Xr^T - Xr Xi^T,
// so no operand is negated (an int8 -128 has no negation).  ci8 voltages run
// on v_mfma_i32_16x16x64_i8 with exact 32-bit sums; cf32 on
// v_mfma_f32_16x16x4f32.
#include <algorithm>
#include <type_traits>

#include "internal.hpp"
#include "volts.hpp"

namespace epic {

namespace {

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kXB = 64;            // output rows (and columns) of a block
constexpr int kXThreads = 256;
constexpr int kP8 = 144;           // bytes per row of an int8 plane: 128 samples + 16 pad
constexpr int kKT8 = 128;          // samples per chunk (ci8): two MFMA K steps of 64
constexpr int kKT32 = 32;          // samples per chunk (cf32): eight MFMA K steps of 4
constexpr int kP32 = 80;           // floats per sample row of an FP32 plane: 64 rows + 16 pad
// Largest sample count whose int8 products cannot overflow a 32-bit sum:
// |re re + im im| <= 2 * 128^2 per sample, 65535 * 32768 < 2^31.
constexpr int kMaxSeg8 = 65535 / kKT8 * kKT8;

__device__ __forceinline__ uint32_t byte_perm(uint32_t hi, uint32_t lo, uint32_t sel)
{
    return __builtin_amdgcn_perm(hi, lo, sel);
}

// Block pair (I, J), J >= I, of upper-triangle index p in row-major order.
__device__ __forceinline__ void block_pair(int p, int nb, int &I, int &J)
{
    int i = 0;
    while (p >= nb - i) {
        p -= nb - i;
        ++i;
    }
    I = i;
    J = i + p;
}

// ci8: a thread stages 4 samples x 8 rows of each block (one 16-byte load per
// sample and block) and writes, per row, the 4 samples' real and imaginary
// bytes as one 32-bit word of the re and im planes ([row][sample], kP8 bytes
// per row).  32 sample quads x 8 row octets cover a block; with the 144-byte
// pitch a wave's stores and the 16-lane fragment reads are bank-conflict free.
struct Stage8 {
    uint32_t d[2][4][4];

    __device__ __forceinline__ void load(const int8_t *v, int R, int n_time, size_t cbase, int t,
                                         const int *row0, int nside, bool vec)
    {
#pragma unroll
        for (int sd = 0; sd < 2; ++sd)
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
                for (int w = 0; w < 4; ++w) d[sd][u][w] = 0u;
                const int tt = t + u;
                if (sd >= nside || tt >= n_time) continue;
                const size_t off = (cbase + static_cast<size_t>(tt) * R + row0[sd]) * 2;
                if (vec) {
                    if (row0[sd] < R) {
                        const i32x4 q = gload<i32x4>(v + off, 0);
#pragma unroll
                        for (int w = 0; w < 4; ++w) d[sd][u][w] = static_cast<uint32_t>(q[w]);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < 8; ++k)
                        if (row0[sd] + k < R) {
                            const uint32_t h = gload<uint16_t>(v + off + 2 * k, 0);
                            d[sd][u][k >> 1] |= h << (16 * (k & 1));
                        }
                }
            }
    }

    __device__ __forceinline__ void store(uint8_t *const *re, uint8_t *const *im, int nside,
                                          int row_l, int col) const
    {
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            if (sd >= nside) break;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int w = k >> 1;
                const uint32_t sel = (k & 1) ? 0x07030602u : 0x05010400u;
                const uint32_t p01 = byte_perm(d[sd][1][w], d[sd][0][w], sel);   // re0 re1 im0 im1
                const uint32_t p23 = byte_perm(d[sd][3][w], d[sd][2][w], sel);   // re2 re3 im2 im3
                *reinterpret_cast<uint32_t *>(re[sd] + (row_l + k) * kP8 + col) = byte_perm(p23, p01, 0x05040100u);
                *reinterpret_cast<uint32_t *>(im[sd] + (row_l + k) * kP8 + col) = byte_perm(p23, p01, 0x07060302u);
            }
        }
    }
};

// cf32: a thread stages 8 (sample, row pair) slots (16 bytes each) and writes
// float2 pairs into the re and im planes ([sample][row], kP32 floats per
// sample).
struct Stage32 {
    float4 d[8];

    __device__ __forceinline__ void load(const float2 *v, int R, int n_time, size_t cbase, int t0,
                                         int blk0, int i, bool vec)
    {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int slot = i + 128 * s;          // 32 samples x 32 row pairs
            const int tt = t0 + (slot >> 5), r = blk0 + 2 * (slot & 31);
            d[s] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (tt >= n_time) continue;
            const size_t off = cbase + static_cast<size_t>(tt) * R + r;
            if (vec) {
                if (r < R) d[s] = gload<float4>(v + off, 0);
            } else {
                if (r < R) {
                    const float2 a = gload<float2>(v + off, 0);
                    d[s].x = a.x;
                    d[s].y = a.y;
                }
                if (r + 1 < R) {
                    const float2 b = gload<float2>(v + off + 1, 0);
                    d[s].z = b.x;
                    d[s].w = b.y;
                }
            }
        }
    }

    __device__ __forceinline__ void store(float *re, float *im, int i) const
    {
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int slot = i + 128 * s;
            const int tl = slot >> 5, rl = 2 * (slot & 31);
            *reinterpret_cast<float2 *>(re + tl * kP32 + rl) = make_float2(d[s].x, d[s].z);
            *reinterpret_cast<float2 *>(im + tl * kP32 + rl) = make_float2(d[s].y, d[s].w);
        }
    }
};

template <int VT>
__global__ __launch_bounds__(kXThreads) void k_xcorr(const void *__restrict__ volts, int R,
                                                     int n_time, int t_beg, int t_cnt, int nb,
                                                     int64_t n_items, float inv_nt, int accumulate,
                                                     float2 *__restrict__ vis)
{
    // XCD-aware order: consecutive items (blocks of one channel) go to the
    // work-groups one XCD runs, so a channel's voltages stay in one L2
    const int64_t q = (n_items + 7) / 8;
    const int64_t item = (blockIdx.x % 8) * q + blockIdx.x / 8;
    if (item >= n_items) return;
    const int npair = nb * (nb + 1) / 2;
    const int c = static_cast<int>(item / npair);
    int I, J;
    block_pair(static_cast<int>(item % npair), nb, I, J);
    const bool diag = I == J;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const bool stager = tid < 128 || !diag;
    const int side = tid >> 7, i = tid & 127;
    const int blk0 = (side == 0 ? I : J) * kXB;
    const size_t cbase = static_cast<size_t>(c) * n_time * R;
    const int mi = (wave >> 1) * 32, nj = (wave & 1) * 32;

    constexpr bool I8 = VT == EPIC_CI8;
    using Acc = typename std::conditional<I8, i32x4, f32x4>::type;
    Acc rr[2][2], ir[2][2], ri[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) rr[a][b] = ir[a][b] = ri[a][b] = Acc{0, 0, 0, 0};

    const int t_end = t_beg + t_cnt;
    if constexpr (I8) {
        __shared__ __attribute__((aligned(16))) uint8_t lds[4][kXB * kP8];
        uint8_t *are = lds[0], *aim = lds[1];
        uint8_t *bre = diag ? lds[0] : lds[2], *bim = diag ? lds[1] : lds[3];
        uint8_t *const sre[2] = {lds[0], lds[2]}, *const sim[2] = {lds[1], lds[3]};
        const int nside = diag ? 1 : 2;
        const bool vec = (R & 7) == 0;
        const int8_t *v = static_cast<const int8_t *>(volts);
        const int tq = tid & 31, ro = tid >> 5;
        const int row0[2] = {I * kXB + 8 * ro, J * kXB + 8 * ro};
        Stage8 st;
        st.load(v, R, t_end, cbase, t_beg + 4 * tq, row0, nside, vec);
        for (int t0 = t_beg; t0 < t_end; t0 += kKT8) {
            __syncthreads();
            st.store(sre, sim, nside, 8 * ro, 4 * tq);
            __syncthreads();
            if (t0 + kKT8 < t_end) st.load(v, R, t_end, cbase, t0 + kKT8 + 4 * tq, row0, nside, vec);
#pragma unroll
            for (int ks = 0; ks < kKT8 / 64; ++ks) {
                const int fo = (lane & 15) * kP8 + 64 * ks + 16 * (lane >> 4);
                i32x4 xr[2], xi[2], yr[2], yi[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    xr[a] = *reinterpret_cast<const i32x4 *>(are + (mi + 16 * a) * kP8 + fo);
                    xi[a] = *reinterpret_cast<const i32x4 *>(aim + (mi + 16 * a) * kP8 + fo);
                    yr[a] = *reinterpret_cast<const i32x4 *>(bre + (nj + 16 * a) * kP8 + fo);
                    yi[a] = *reinterpret_cast<const i32x4 *>(bim + (nj + 16 * a) * kP8 + fo);
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        rr[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(xr[a], yr[b], rr[a][b], 0, 0, 0);
                        rr[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(xi[a], yi[b], rr[a][b], 0, 0, 0);
                        ir[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(xi[a], yr[b], ir[a][b], 0, 0, 0);
                        ri[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(xr[a], yi[b], ri[a][b], 0, 0, 0);
                    }
            }
        }
    } else {
        __shared__ __attribute__((aligned(16))) float lds[4][kKT32 * kP32];
        float *are = lds[0], *aim = lds[1];
        float *bre = diag ? lds[0] : lds[2], *bim = diag ? lds[1] : lds[3];
        float *sre = lds[2 * side], *sim = lds[2 * side + 1];
        const bool vec = (R & 1) == 0;
        const float2 *v = static_cast<const float2 *>(volts);
        Stage32 st;
        if (stager) st.load(v, R, t_end, cbase, t_beg, blk0, i, vec);
        for (int t0 = t_beg; t0 < t_end; t0 += kKT32) {
            __syncthreads();
            if (stager) st.store(sre, sim, i);
            __syncthreads();
            if (t0 + kKT32 < t_end && stager) st.load(v, R, t_end, cbase, t0 + kKT32, blk0, i, vec);
#pragma unroll 2
            for (int ks = 0; ks < kKT32 / 4; ++ks) {
                const int fo = (4 * ks + (lane >> 4)) * kP32 + (lane & 15);
                float xr[2], xi[2], yr[2], yi[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    xr[a] = are[fo + mi + 16 * a];
                    xi[a] = aim[fo + mi + 16 * a];
                    yr[a] = bre[fo + nj + 16 * a];
                    yi[a] = bim[fo + nj + 16 * a];
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        rr[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr[a], yr[b], rr[a][b], 0, 0, 0);
                        rr[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi[a], yi[b], rr[a][b], 0, 0, 0);
                        ir[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi[a], yr[b], ir[a][b], 0, 0, 0);
                        ri[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr[a], yi[b], ri[a][b], 0, 0, 0);
                    }
            }
        }
    }

    // C fragment: lane holds rows 4 (lane / 16) + e, column lane % 16
    float2 *out = vis + static_cast<size_t>(c) * R * R;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int r = I * kXB + mi + 16 * a + 4 * (lane >> 4) + e;
                const int s = J * kXB + nj + 16 * b + (lane & 15);
                if (r >= R || s >= R) continue;
                float2 val;
                if constexpr (I8) {
                    val = make_float2(static_cast<float>(rr[a][b][e]) * inv_nt,
                                      static_cast<float>(ir[a][b][e] - ri[a][b][e]) * inv_nt);
                } else {
                    val = make_float2(rr[a][b][e] * inv_nt, (ir[a][b][e] - ri[a][b][e]) * inv_nt);
                }
                float2 *p1 = out + static_cast<size_t>(r) * R + s;
                if (accumulate) {
                    const float2 o = *p1;
                    val = make_float2(o.x + val.x, o.y + val.y);
                }
                *p1 = val;
                if (!diag) out[static_cast<size_t>(s) * R + r] = make_float2(val.x, -val.y);
            }
}

// Eq. 6 gridding of visibilities in two passes.
//
// k_vis_centres: a centre (a non-empty baseline cell e = c_a - c_b) is served
// by n_pol^2 * S lanes, one per (product, block of OYB row offsets); each lane
// sums, over the centre's pairs in order,
//     V_ab^{pq} Ky_ab(oy) Kx_ab(ox)   for its row offsets oy and every ox,
// where Kx_ab(o) = sum_i wx_a[i] wx_b[i - o] is the cross-correlation of the
// two elements' weights (the same for y), and stores the sums in
// part[c][oy][product][ox][e].  Kx and Ky are formed once per pair and lane;
// the channel's element weights sit in LDS; pairs go in batches whose id and
// visibility loads are all in flight together.
//
// k_vis_gather: every (channel, product, cell d) sums part[..][d - offset]
// over the (2K-1)^2 offsets in a fixed order (deterministic); each partial
// is read once, by one cell, and neighbouring cells read neighbouring words.
constexpr int kVcThreads = 256;
constexpr int kVcLdsMax = 64 * 1024;
constexpr int kVcBatch = 8;            // pairs per lane whose loads are in flight together

// Weights (wx[0..K), wy[0..K)) of element a into w[0..2K): from the LDS copy
// (ES floats per element, 16-byte aligned) with float4 reads, or from the
// plan in global memory (2K floats per element).
template <int K, int ES, bool ELDS>
__device__ __forceinline__ void load_weights(const float *lds, const float *glob, int a, float *w)
{
    if constexpr (ELDS) {
#pragma unroll
        for (int i = 0; i < ES / 4; ++i) {
            const float4 q = *reinterpret_cast<const float4 *>(lds + a * ES + 4 * i);
            w[4 * i] = q.x;
            w[4 * i + 1] = q.y;
            w[4 * i + 2] = q.z;
            w[4 * i + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 2 * K; ++i) w[i] = gload<float>(glob, static_cast<size_t>(a) * 2 * K + i);
    }
}

// Cross-correlation of two K-tap weight rows at every offset o - (K - 1).
template <int K>
__device__ __forceinline__ void xcorr_taps(const float *u, const float *v, float *out)
{
#pragma unroll
    for (int o = 0; o < 2 * K - 1; ++o) {
        const int oo = o - (K - 1);
        float t = 0.f;
#pragma unroll
        for (int i = 0; i < K; ++i)
            if (i - oo >= 0 && i - oo < K) t = fmaf(u[i], v[i - oo], t);
        out[o] = t;
    }
}

template <int K> struct VcSplit { static constexpr int S = K <= 3 ? 1 : (K == 5 ? 3 : 7); };

template <int NP, int K, bool ELDS>
__global__ __launch_bounds__(kVcThreads) void k_vis_centres(const float2 *__restrict__ vis,
                                                            XfftPlanHandle pl, int n_elem, int nx,
                                                            int ny, int n_chan, int bpc,
                                                            float2 *__restrict__ part)
{
    constexpr int W = 2 * K - 1, NQ = NP * NP, G = W * NQ;
    constexpr int S = VcSplit<K>::S, OYB = (W + S - 1) / S;   // row-offset blocks, rows per block
    constexpr int L = NQ * S, CPW = 64 / L;                   // lanes per centre, centres per wave
    constexpr int CPB = (kVcThreads / 64) * CPW;              // centres per block
    constexpr int ES = (2 * K + 3) & ~3;                       // LDS floats per element
    extern __shared__ float4 vc_lds4[];
    float *vc_lds = reinterpret_cast<float *>(vc_lds4);
    // XCD-aware order: the blocks of one channel run on one XCD, so the
    // channel's visibilities stay in one L2
    const int64_t total = static_cast<int64_t>(n_chan) * bpc, q8 = (total + 7) / 8;
    const int64_t item = (blockIdx.x % 8) * q8 + blockIdx.x / 8;
    if (item >= total) return;
    const int c = static_cast<int>(item / bpc), blk = static_cast<int>(item % bpc);
    const int npix = nx * ny;
    const int n_cent = static_cast<int>(pl.cent_base[c + 1] - pl.cent_base[c]);
    if (blk * CPB >= n_cent) return;                             // block-uniform
    const float *ew_g = pl.elem_w + static_cast<size_t>(c) * n_elem * 2 * K;
    if constexpr (ELDS) {
        // repacked at a 16-byte stride: (wx[0..K), wy[0..K), 0...) per element
        for (int i = threadIdx.x; i < n_elem * ES; i += kVcThreads) {
            const int a = i / ES, r = i - a * ES;
            vc_lds[i] = r < 2 * K ? ew_g[a * 2 * K + r] : 0.f;
        }
        __syncthreads();
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int cl = lane / L, li = lane % L;
    const int k = blk * CPB + wave * CPW + cl;                   // centre of this lane
    if (cl >= CPW || k >= n_cent) return;
    const int R = n_elem * NP;
    const int qd = li % NQ, sb = li / NQ;                        // product, row-offset block
    const int al = qd / NP, be = qd % NP;
    const int32_t *cs = pl.cent_start + static_cast<size_t>(c) * (npix + 1);
    const uint32_t *pr = pl.pairs + static_cast<size_t>(c) * n_elem * n_elem;
    const float2 *vc = vis + static_cast<size_t>(c) * R * R + al * R + be;

    float2 acc[OYB][W];
#pragma unroll
    for (int r = 0; r < OYB; ++r)
#pragma unroll
        for (int o = 0; o < W; ++o) acc[r][o] = make_float2(0.f, 0.f);
    const int e_beg = cs[k], e_end = cs[k + 1];
    for (int e0 = e_beg; e0 < e_end; e0 += kVcBatch) {
        // a batch of pairs: ids, then visibilities, all loads in flight together
        uint32_t ab[kVcBatch];
        float2 v[kVcBatch];
#pragma unroll
        for (int u = 0; u < kVcBatch; ++u) ab[u] = e0 + u < e_end ? gload<uint32_t>(pr, e0 + u) : 0u;
#pragma unroll
        for (int u = 0; u < kVcBatch; ++u)
            v[u] = gload<float2>(vc, static_cast<size_t>(ab[u] & 0xffff) * NP * R + (ab[u] >> 16) * NP);
#pragma unroll
        for (int u = 0; u < kVcBatch; ++u) {
            if (e0 + u >= e_end) break;
            const int a = ab[u] & 0xffff, b = ab[u] >> 16;
            float wa[ES], wb[ES];
            load_weights<K, ES, ELDS>(vc_lds, ew_g, a, wa);
            load_weights<K, ES, ELDS>(vc_lds, ew_g, b, wb);
            float kx[W], ky[W];
            xcorr_taps<K>(wa, wb, kx);
            xcorr_taps<K>(wa + K, wb + K, ky);
#pragma unroll
            for (int r = 0; r < OYB; ++r) {
                float t = 0.f;                                    // Ky of row sb * OYB + r
#pragma unroll
                for (int s2 = 0; s2 < S; ++s2)
                    if (s2 * OYB + r < W) t = sb == s2 ? ky[s2 * OYB + r] : t;
                const float vx = v[u].x * t, vy = v[u].y * t;
#pragma unroll
                for (int o = 0; o < W; ++o) {
                    acc[r][o].x = fmaf(vx, kx[o], acc[r][o].x);
                    acc[r][o].y = fmaf(vy, kx[o], acc[r][o].y);
                }
            }
        }
    }
    const int32_t cell = pl.cent_cell[static_cast<size_t>(c) * npix + k];
    const int ec = (cell >> 16) * nx + (cell & 0xffff);
#pragma unroll
    for (int r = 0; r < OYB; ++r) {
        const int oyi = sb * OYB + r;
        if (oyi >= W) break;
        float2 *dst = part + (static_cast<size_t>(c) * G + oyi * NQ + qd) * W * npix + ec;
#pragma unroll
        for (int o = 0; o < W; ++o) dst[static_cast<size_t>(o) * npix] = acc[r][o];
    }
}

template <int NP, int K>
__global__ __launch_bounds__(256) void k_vis_gather(XfftPlanHandle pl, int nx, int ny,
                                                    const float2 *__restrict__ part,
                                                    float2 *__restrict__ grid)
{
    constexpr int W = 2 * K - 1, NQ = NP * NP, G = W * NQ;
    const int npix = nx * ny;
    const int d = blockIdx.x * 256 + threadIdx.x;
    if (d >= npix) return;
    const int qd = blockIdx.y, c = blockIdx.z;
    const int y = d / nx, x = d - y * nx;
    const int32_t *cm = pl.cell_cent + static_cast<size_t>(c) * npix;
    const float2 *pc = part + static_cast<size_t>(c) * G * W * npix;
    float2 s = make_float2(0.f, 0.f);
    for (int o_y = 0; o_y < W; ++o_y) {
        int ey = y - (o_y - (K - 1));
        ey = ey < 0 ? ey + ny : (ey >= ny ? ey - ny : ey);
        const float2 *prow = pc + static_cast<size_t>(o_y * NQ + qd) * W * npix;
#pragma unroll
        for (int o_x = 0; o_x < W; ++o_x) {
            int ex = x - (o_x - (K - 1));
            ex = ex < 0 ? ex + nx : (ex >= nx ? ex - nx : ex);
            const int e = ey * nx + ex;
            if (cm[e] >= 0) {
                const float2 v = gload<float2>(prow, static_cast<size_t>(o_x) * npix + e);
                s.x += v.x;
                s.y += v.y;
            }
        }
    }
    grid[(static_cast<size_t>(c) * NQ + qd) * npix + d] = s;
}

template <int NP, int K>
epic_status vg_launch(const float2 *vis, const XfftPlanHandle &pl, int n_elem, int n_chan, int nx,
                      int ny, float2 *part, float2 *grid, hipStream_t stream)
{
    constexpr int NQ = NP * NP;
    constexpr int L = NQ * VcSplit<K>::S, CPB = (kVcThreads / 64) * (64 / L);
    const int npix = nx * ny;
    const size_t ew_bytes = sizeof(float) * static_cast<size_t>(n_elem) * ((2 * K + 3) & ~3);
    const bool elds = ew_bytes <= static_cast<size_t>(kVcLdsMax);
    {
        auto kern = elds ? k_vis_centres<NP, K, true> : k_vis_centres<NP, K, false>;
        const size_t bytes = elds ? ew_bytes : 0;
        if (elds) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               kVcLdsMax);
            if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
        }
        const int bpc = (npix + CPB - 1) / CPB;
        const int64_t total = static_cast<int64_t>(n_chan) * bpc;
        const dim3 blocks(static_cast<unsigned>(8 * ((total + 7) / 8))), threads(kVcThreads);
        KernelTimer timer("vis_centres", stream);
        hipLaunchKernelGGL(kern, blocks, threads, bytes, stream, vis, pl, n_elem, nx, ny, n_chan,
                           bpc, part);
        EPIC_HIP_TRY(hipGetLastError());
    }
    const dim3 blocks((npix + 255) / 256, NQ, n_chan), threads(256);
    KernelTimer timer("vis_gather", stream);
    hipLaunchKernelGGL((k_vis_gather<NP, K>), blocks, threads, 0, stream, pl, nx, ny, part, grid);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

template <int NP>
epic_status vg_k(int K, const float2 *vis, const XfftPlanHandle &pl, int n_elem, int n_chan, int nx,
                 int ny, float2 *part, float2 *grid, hipStream_t stream)
{
    switch (K) {
    case 1: return vg_launch<NP, 1>(vis, pl, n_elem, n_chan, nx, ny, part, grid, stream);
    case 3: return vg_launch<NP, 3>(vis, pl, n_elem, n_chan, nx, ny, part, grid, stream);
    case 5: return vg_launch<NP, 5>(vis, pl, n_elem, n_chan, nx, ny, part, grid, stream);
    case 7: return vg_launch<NP, 7>(vis, pl, n_elem, n_chan, nx, ny, part, grid, stream);
    }
    return fail(EPIC_ERR_INTERNAL, "visibility gridding: unexpected support");
}

}  // namespace

epic_status launch_xcorr(const void *volts, int volt_type, int R, int n_chan, int n_time,
                         float2 *vis, hipStream_t stream)
{
    const int nb = (R + kXB - 1) / kXB;
    const int64_t n_items = static_cast<int64_t>(n_chan) * nb * (nb + 1) / 2;
    const int64_t q = (n_items + 7) / 8;
    if (8 * q > 0x7fffffffLL) return fail(EPIC_ERR_UNSUPPORTED, "correlator: too many blocks");
    const dim3 blocks(static_cast<unsigned>(8 * q)), threads(kXThreads);
    const float inv = static_cast<float>(1.0 / static_cast<double>(n_time));
    KernelTimer timer("xcorr", stream);
    const int seg = volt_type == EPIC_CI8 ? kMaxSeg8 : n_time;
    for (int t0 = 0; t0 < n_time; t0 += seg) {
        const int cnt = std::min(seg, n_time - t0);
        if (volt_type == EPIC_CI8)
            hipLaunchKernelGGL(k_xcorr<EPIC_CI8>, blocks, threads, 0, stream, volts, R, n_time, t0,
                               cnt, nb, n_items, inv, t0 > 0 ? 1 : 0, vis);
        else
            hipLaunchKernelGGL(k_xcorr<EPIC_CF32>, blocks, threads, 0, stream, volts, R, n_time, t0,
                               cnt, nb, n_items, inv, t0 > 0 ? 1 : 0, vis);
        EPIC_HIP_TRY(hipGetLastError());
    }
    return EPIC_OK;
}

epic_status launch_vis_grid(const float2 *vis, const XfftPlanHandle &pl, int n_pol, int n_elem,
                            int n_chan, int nx, int ny, float2 *part, float2 *grid,
                            hipStream_t stream)
{
    if (n_pol == 1) return vg_k<1>(pl.K, vis, pl, n_elem, n_chan, nx, ny, part, grid, stream);
    return vg_k<2>(pl.K, vis, pl, n_elem, n_chan, nx, ny, part, grid, stream);
}

}  // namespace epic
