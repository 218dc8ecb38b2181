// k_fft.hip -- batched FP32 2-D transform of Eq. 3 (outer sum): + sign,
// unnormalised, natural order.  Grids up to 16384 cells are transformed in
// one pass through LDS (one work-group per batch item); larger grids take a
// row pass and a column pass through global memory.
//
// With INV the kernels compute the inverse, (1/(nx ny)) sum_k x[k]
// exp(-2 pi i k.j / N), as conj(F(conj(x))) / (nx ny): the input is
// conjugated as it is loaded and the result conjugated and scaled as it is
// stored, so the inverse costs no extra pass.
#include <type_traits>

#include "fft_lds.hpp"
#include "internal.hpp"

namespace epic {

// Load a 2-D item into LDS (row pitch P), transform rows then columns, store.
__device__ __forceinline__ float2 conj_scaled(float2 v, float s) { return make_float2(v.x * s, -v.y * s); }

template <int NX, int NY, int BLOCK, bool INV>
__global__ __launch_bounds__(BLOCK) void k_fft2_lds(const float2 *__restrict__ in,
                                                    float2 *__restrict__ out,
                                                    const float2 *__restrict__ twx,
                                                    const float2 *__restrict__ twy)
{
    constexpr int P = NX + 1;
    extern __shared__ __align__(16) float2 lds[];
    float2 *buf = lds;
    float2 *tx = lds + NY * P;
    float2 *ty = tx + NX;
    const size_t item = blockIdx.x;
    const float2 *src = in + item * (NX * NY);
    for (int i = threadIdx.x; i < NX; i += BLOCK) tx[i] = twx[i];
    for (int i = threadIdx.x; i < NY; i += BLOCK) ty[i] = twy[i];
    // every load of the plane in flight before the LDS writes
    constexpr int PER = NX * NY / BLOCK;
    static_assert(PER * BLOCK == NX * NY, "plane must split evenly over the block");
    float2 v[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) v[r] = src[threadIdx.x + r * BLOCK];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int i = threadIdx.x + r * BLOCK;
        buf[(i / NX) * P + (i % NX)] = INV ? conj_scaled(v[r], 1.f) : v[r];
    }
    __syncthreads();
    constexpr int MAXL = NX > NY ? NX : NY;
    fft_lines<NX, BLOCK, MAXL, false>(buf, LineMap{NY, 0, 0, P, 1}, NY, tx);
    fft_lines<NY, BLOCK, MAXL, false>(buf, LineMap{NX, 0, 0, 1, P}, NX, ty);
    float2 *dst = out + item * (NX * NY);
    constexpr float kInv = 1.f / static_cast<float>(NX * NY);   // a power of two: exact
    for (int i = threadIdx.x; i < NX * NY; i += BLOCK) {
        const float2 v = buf[(i / NX) * P + (i % NX)];
        dst[i] = INV ? conj_scaled(v, kInv) : v;
    }
}

// Row pass for large grids: ROWS consecutive rows of length NX per block.
template <int NX, int ROWS, int BLOCK, bool INV>
//
// With chan set (the composed cadence), the rows of plane b outside channel
// (b / items_per_chan)'s footprint box are zero: they are neither read nor
// written (the column pass takes them as zero).
__global__ __launch_bounds__(BLOCK) void k_fft_rows(const float2 *__restrict__ in,
                                                    float2 *__restrict__ out,
                                                    const float2 *__restrict__ tw, int64_t n_rows,
                                                    const ChanPlan *__restrict__ chan,
                                                    int items_per_chan, int ny)
{
    constexpr int P = NX + 1;
    extern __shared__ __align__(16) float2 lds[];
    float2 *buf = lds;
    float2 *t = lds + ROWS * P;
    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * ROWS;
    const int nr = static_cast<int>(min<int64_t>(ROWS, n_rows - row0));
    int ylo = 0, yhi = ROWS;                      // block rows inside the box
    if (chan) {
        const ChanPlan cp = chan[(row0 / ny) / items_per_chan];
        const int yb = static_cast<int>(row0 % ny);
        ylo = max(0, cp.y0 - yb);
        yhi = min(ROWS, cp.y0 + cp.bh - yb);
        if (ylo >= yhi) return;
    }
    for (int i = threadIdx.x; i < NX; i += BLOCK) t[i] = tw[i];
    // every load of the rows in flight before the LDS writes
    constexpr int PER = (ROWS * NX + BLOCK - 1) / BLOCK;
    float2 v[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int i = threadIdx.x + r * BLOCK;
        const int y = i / NX;
        v[r] = i < nr * NX && y >= ylo && y < yhi ? in[row0 * NX + i] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int i = threadIdx.x + r * BLOCK;
        if (i < nr * NX) buf[(i / NX) * P + (i % NX)] = INV ? conj_scaled(v[r], 1.f) : v[r];
    }
    __syncthreads();
    fft_lines<NX, BLOCK, ROWS, false>(buf, LineMap{ROWS, 0, 0, P, 1}, nr, t);
    for (int i = threadIdx.x; i < nr * NX; i += BLOCK) {
        const int y = i / NX;
        if (y >= ylo && y < yhi) out[row0 * NX + i] = buf[y * P + (i % NX)];
    }
}

// Column pass for large grids: COLS adjacent columns (length NY) per block.
// With chan set, the rows outside the channel's footprint box are taken as
// zero (not read); every row is written.
template <int NX, int NY, int COLS, int BLOCK, bool INV>
__global__ __launch_bounds__(BLOCK) void k_fft_cols(float2 *__restrict__ data,
                                                    const float2 *__restrict__ tw,
                                                    const ChanPlan *__restrict__ chan,
                                                    int items_per_chan)
{
    constexpr int P = COLS + 1;   // LDS holds the tile transposed-free: [y][col]
    extern __shared__ __align__(16) float2 lds[];
    float2 *buf = lds;
    float2 *t = lds + NY * P;
    constexpr int TILES = NX / COLS;
    const int64_t item = blockIdx.x / TILES;
    const int c0 = (blockIdx.x % TILES) * COLS;
    float2 *base = data + item * (NX * NY) + c0;
    int ylo = 0, yhi = NY;
    if (chan) {
        const ChanPlan cp = chan[item / items_per_chan];
        ylo = cp.y0;
        yhi = cp.y0 + cp.bh;
    }
    for (int i = threadIdx.x; i < NY; i += BLOCK) t[i] = tw[i];
    // every load of the tile in flight before the LDS writes
    constexpr int PER = NY * COLS / BLOCK;
    static_assert(PER * BLOCK == NY * COLS, "tile must split evenly over the block");
    float2 v[PER];
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int i = threadIdx.x + r * BLOCK;
        const int y = i / COLS;
        v[r] = y >= ylo && y < yhi ? base[y * NX + (i % COLS)] : make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int r = 0; r < PER; ++r) {
        const int i = threadIdx.x + r * BLOCK;
        buf[(i / COLS) * P + (i % COLS)] = v[r];
    }
    __syncthreads();
    fft_lines<NY, BLOCK, COLS, false>(buf, LineMap{COLS, 0, 0, 1, P}, COLS, t);
    constexpr float kInv = 1.f / static_cast<float>(NX * NY);
    for (int i = threadIdx.x; i < NY * COLS; i += BLOCK) {
        const float2 v = buf[(i / COLS) * P + (i % COLS)];
        base[(i / COLS) * NX + (i % COLS)] = INV ? conj_scaled(v, kInv) : v;
    }
}

namespace {

struct RowBox {               // footprint rows of the composed cadence (chan null: none)
    const ChanPlan *chan;
    int items_per_chan;
};

template <typename K>
epic_status set_lds(K kernel, size_t bytes)
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(bytes));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    return EPIC_OK;
}

template <int NX, int NY, bool INV>
epic_status run_lds(int64_t batch, const float2 *in, float2 *out, const float2 *twx,
                    const float2 *twy, hipStream_t stream)
{
    constexpr int BLOCK = NX * NY >= 8192 ? 512 : 256;
    const size_t bytes = sizeof(float2) * (NY * (NX + 1) + NX + NY);
    auto k = k_fft2_lds<NX, NY, BLOCK, INV>;
    epic_status s = set_lds(k, bytes);
    if (s != EPIC_OK) return s;
    // gridDim.x is limited to 2^31-1; batches beyond that are split
    KernelTimer timer("fft2_lds", stream);
    for (int64_t b0 = 0; b0 < batch; b0 += (1LL << 30)) {
        const int64_t nb = std::min<int64_t>(batch - b0, 1LL << 30);
        hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(nb)), dim3(BLOCK), bytes, stream,
                           in + b0 * NX * NY, out + b0 * NX * NY, twx, twy);
        EPIC_HIP_TRY(hipGetLastError());
    }
    return EPIC_OK;
}

template <int NX, bool INV>
epic_status run_rows(int64_t n_rows, const float2 *in, float2 *out, const float2 *tw,
                     hipStream_t stream, const RowBox &rb, int ny)
{
    constexpr int ROWS = 16, BLOCK = 256;
    const size_t bytes = sizeof(float2) * (ROWS * (NX + 1) + NX);
    auto k = k_fft_rows<NX, ROWS, BLOCK, INV>;
    epic_status s = set_lds(k, bytes);
    if (s != EPIC_OK) return s;
    const int64_t blocks = (n_rows + ROWS - 1) / ROWS;
    KernelTimer timer("fft_rows", stream);
    hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(blocks)), dim3(BLOCK), bytes, stream, in, out,
                       tw, n_rows, rb.chan, rb.items_per_chan, ny);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

template <int NX, int NY, bool INV>
epic_status run_cols(int64_t batch, float2 *data, const float2 *tw, hipStream_t stream,
                     const RowBox &rb)
{
    constexpr int COLS = 16, BLOCK = 256;
    const size_t bytes = sizeof(float2) * (NY * (COLS + 1) + NY);
    auto k = k_fft_cols<NX, NY, COLS, BLOCK, INV>;
    epic_status s = set_lds(k, bytes);
    if (s != EPIC_OK) return s;
    const int64_t blocks = batch * (NX / COLS);
    KernelTimer timer("fft_cols", stream);
    hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(blocks)), dim3(BLOCK), bytes, stream, data, tw,
                       rb.chan, rb.items_per_chan);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

template <int NX, bool INV>
epic_status dispatch_ny(int ny, int64_t batch, const float2 *in, float2 *out, const float2 *twx,
                        const float2 *twy, hipStream_t stream, const RowBox &rb)
{
    if constexpr (NX <= 128) {
        switch (ny) {
        case 16: return run_lds<NX, 16, INV>(batch, in, out, twx, twy, stream);
        case 32: return run_lds<NX, 32, INV>(batch, in, out, twx, twy, stream);
        case 64: return run_lds<NX, 64, INV>(batch, in, out, twx, twy, stream);
        case 128:
            if constexpr (NX <= 64) return run_lds<NX, 128, INV>(batch, in, out, twx, twy, stream);
            break;
        default: break;
        }
    }
    if constexpr (NX == 256) {
        if (ny == 16) return run_lds<NX, 16, INV>(batch, in, out, twx, twy, stream);
        if (ny == 32) return run_lds<NX, 32, INV>(batch, in, out, twx, twy, stream);
        if (ny == 64) return run_lds<NX, 64, INV>(batch, in, out, twx, twy, stream);
    }
    // two passes through global memory
    epic_status s = run_rows<NX, INV>(batch * ny, in, out, twx, stream, rb, ny);
    if (s != EPIC_OK) return s;
    switch (ny) {
    case 16: return run_cols<NX, 16, INV>(batch, out, twy, stream, rb);
    case 32: return run_cols<NX, 32, INV>(batch, out, twy, stream, rb);
    case 64: return run_cols<NX, 64, INV>(batch, out, twy, stream, rb);
    case 128: return run_cols<NX, 128, INV>(batch, out, twy, stream, rb);
    case 256: return run_cols<NX, 256, INV>(batch, out, twy, stream, rb);
    }
    return fail(EPIC_ERR_INTERNAL, "fft2: unexpected ny");
}

}  // namespace

bool fft_f32_two_pass(int nx, int ny) { return ny == 256 || (ny == 128 && nx >= 128); }

epic_status launch_fft2_f32_cols(int nx, int ny, int64_t batch, float2 *data, int device,
                                 hipStream_t stream, const ChanPlan *chan, int items_per_chan)
{
    if (!chan || !fft_f32_two_pass(nx, ny) || (nx != 128 && nx != 256))
        return fail(EPIC_ERR_INTERNAL, "fft2: column pass alone on an unexpected grid");
    const RowBox rb{chan, items_per_chan};
    const float2 *twy = nullptr;
    epic_status s = get_twiddles(ny, device, &twy);
    if (s != EPIC_OK) return s;
    auto by_ny = [&](auto nx_c) -> epic_status {
        constexpr int NX = decltype(nx_c)::value;
        switch (ny) {
        case 128: return run_cols<NX, 128, false>(batch, data, twy, stream, rb);
        case 256: return run_cols<NX, 256, false>(batch, data, twy, stream, rb);
        }
        return fail(EPIC_ERR_INTERNAL, "fft2: unexpected ny");
    };
    return nx == 256 ? by_ny(std::integral_constant<int, 256>{}) : by_ny(std::integral_constant<int, 128>{});
}

epic_status launch_fft2_f32(int nx, int ny, int64_t batch, const float2 *in, float2 *out,
                            int device, hipStream_t stream, bool inverse, const ChanPlan *chan,
                            int items_per_chan)
{
    if (chan && !fft_f32_two_pass(nx, ny))
        return fail(EPIC_ERR_INTERNAL, "fft2: footprint rows on a one-pass grid");
    const RowBox rb{chan, items_per_chan};
    const float2 *twx = nullptr, *twy = nullptr;
    epic_status s = get_twiddles(nx, device, &twx);
    if (s != EPIC_OK) return s;
    s = get_twiddles(ny, device, &twy);
    if (s != EPIC_OK) return s;
    auto go = [&](auto inv) -> epic_status {
        constexpr bool INV = decltype(inv)::value;
        switch (nx) {
        case 16: return dispatch_ny<16, INV>(ny, batch, in, out, twx, twy, stream, rb);
        case 32: return dispatch_ny<32, INV>(ny, batch, in, out, twx, twy, stream, rb);
        case 64: return dispatch_ny<64, INV>(ny, batch, in, out, twx, twy, stream, rb);
        case 128: return dispatch_ny<128, INV>(ny, batch, in, out, twx, twy, stream, rb);
        case 256: return dispatch_ny<256, INV>(ny, batch, in, out, twx, twy, stream, rb);
        }
        return fail(EPIC_ERR_INTERNAL, "fft2: unexpected nx");
    };
    return inverse ? go(std::true_type{}) : go(std::false_type{});
}

}  // namespace epic
