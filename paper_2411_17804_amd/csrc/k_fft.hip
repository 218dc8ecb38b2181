// k_fft.hip -- batched FP32 2-D transform of Eq. 3 (outer sum): + sign,
// unnormalised, natural order.  Grids up to 16384 cells are transformed in
// one pass through LDS (one work-group per batch item); larger grids take a
// row pass and a column pass through global memory.
#include "fft_lds.hpp"
#include "internal.hpp"

namespace epic {

// Load a 2-D item into LDS (row pitch P), transform rows then columns, store.
template <int NX, int NY, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_fft2_lds(const float2 *__restrict__ in,
                                                    float2 *__restrict__ out,
                                                    const float2 *__restrict__ twx,
                                                    const float2 *__restrict__ twy)
{
    constexpr int P = NX + 1;
    extern __shared__ float2 lds[];
    float2 *buf = lds;
    float2 *tx = lds + NY * P;
    float2 *ty = tx + NX;
    const size_t item = blockIdx.x;
    const float2 *src = in + item * (NX * NY);
    for (int i = threadIdx.x; i < NX; i += BLOCK) tx[i] = twx[i];
    for (int i = threadIdx.x; i < NY; i += BLOCK) ty[i] = twy[i];
    for (int i = threadIdx.x; i < NX * NY; i += BLOCK) buf[(i / NX) * P + (i % NX)] = src[i];
    __syncthreads();
    constexpr int MAXL = NX > NY ? NX : NY;
    fft_lines<NX, BLOCK, MAXL, false>(buf, LineMap{NY, 0, 0, P, 1}, NY, tx);
    fft_lines<NY, BLOCK, MAXL, false>(buf, LineMap{NX, 0, 0, 1, P}, NX, ty);
    float2 *dst = out + item * (NX * NY);
    for (int i = threadIdx.x; i < NX * NY; i += BLOCK) dst[i] = buf[(i / NX) * P + (i % NX)];
}

// Row pass for large grids: ROWS consecutive rows of length NX per block.
template <int NX, int ROWS, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_fft_rows(const float2 *__restrict__ in,
                                                    float2 *__restrict__ out,
                                                    const float2 *__restrict__ tw, int64_t n_rows)
{
    constexpr int P = NX + 1;
    extern __shared__ float2 lds[];
    float2 *buf = lds;
    float2 *t = lds + ROWS * P;
    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * ROWS;
    const int nr = static_cast<int>(min<int64_t>(ROWS, n_rows - row0));
    for (int i = threadIdx.x; i < NX; i += BLOCK) t[i] = tw[i];
    for (int i = threadIdx.x; i < nr * NX; i += BLOCK) buf[(i / NX) * P + (i % NX)] = in[row0 * NX + i];
    __syncthreads();
    fft_lines<NX, BLOCK, ROWS, false>(buf, LineMap{ROWS, 0, 0, P, 1}, nr, t);
    for (int i = threadIdx.x; i < nr * NX; i += BLOCK) out[row0 * NX + i] = buf[(i / NX) * P + (i % NX)];
}

// Column pass for large grids: COLS adjacent columns (length NY) per block.
template <int NX, int NY, int COLS, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_fft_cols(float2 *__restrict__ data,
                                                    const float2 *__restrict__ tw)
{
    constexpr int P = COLS + 1;   // LDS holds the tile transposed-free: [y][col]
    extern __shared__ float2 lds[];
    float2 *buf = lds;
    float2 *t = lds + NY * P;
    constexpr int TILES = NX / COLS;
    const int64_t item = blockIdx.x / TILES;
    const int c0 = (blockIdx.x % TILES) * COLS;
    float2 *base = data + item * (NX * NY) + c0;
    for (int i = threadIdx.x; i < NY; i += BLOCK) t[i] = tw[i];
    for (int i = threadIdx.x; i < NY * COLS; i += BLOCK) buf[(i / COLS) * P + (i % COLS)] = base[(i / COLS) * NX + (i % COLS)];
    __syncthreads();
    fft_lines<NY, BLOCK, COLS, false>(buf, LineMap{COLS, 0, 0, 1, P}, COLS, t);
    for (int i = threadIdx.x; i < NY * COLS; i += BLOCK) base[(i / COLS) * NX + (i % COLS)] = buf[(i / COLS) * P + (i % COLS)];
}

namespace {

template <typename K>
epic_status set_lds(K kernel, size_t bytes)
{
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                       static_cast<int>(bytes));
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    return EPIC_OK;
}

template <int NX, int NY>
epic_status run_lds(int64_t batch, const float2 *in, float2 *out, const float2 *twx,
                    const float2 *twy, hipStream_t stream)
{
    constexpr int BLOCK = NX * NY >= 8192 ? 512 : 256;
    const size_t bytes = sizeof(float2) * (NY * (NX + 1) + NX + NY);
    auto k = k_fft2_lds<NX, NY, BLOCK>;
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

template <int NX>
epic_status run_rows(int64_t n_rows, const float2 *in, float2 *out, const float2 *tw,
                     hipStream_t stream)
{
    constexpr int ROWS = 16, BLOCK = 256;
    const size_t bytes = sizeof(float2) * (ROWS * (NX + 1) + NX);
    auto k = k_fft_rows<NX, ROWS, BLOCK>;
    epic_status s = set_lds(k, bytes);
    if (s != EPIC_OK) return s;
    const int64_t blocks = (n_rows + ROWS - 1) / ROWS;
    KernelTimer timer("fft_rows", stream);
    hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(blocks)), dim3(BLOCK), bytes, stream, in, out,
                       tw, n_rows);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

template <int NX, int NY>
epic_status run_cols(int64_t batch, float2 *data, const float2 *tw, hipStream_t stream)
{
    constexpr int COLS = 16, BLOCK = 256;
    const size_t bytes = sizeof(float2) * (NY * (COLS + 1) + NY);
    auto k = k_fft_cols<NX, NY, COLS, BLOCK>;
    epic_status s = set_lds(k, bytes);
    if (s != EPIC_OK) return s;
    const int64_t blocks = batch * (NX / COLS);
    KernelTimer timer("fft_cols", stream);
    hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(blocks)), dim3(BLOCK), bytes, stream, data, tw);
    EPIC_HIP_TRY(hipGetLastError());
    return EPIC_OK;
}

template <int NX>
epic_status dispatch_ny(int ny, int64_t batch, const float2 *in, float2 *out, const float2 *twx,
                        const float2 *twy, hipStream_t stream)
{
    if constexpr (NX <= 128) {
        switch (ny) {
        case 16: return run_lds<NX, 16>(batch, in, out, twx, twy, stream);
        case 32: return run_lds<NX, 32>(batch, in, out, twx, twy, stream);
        case 64: return run_lds<NX, 64>(batch, in, out, twx, twy, stream);
        case 128:
            if constexpr (NX <= 64) return run_lds<NX, 128>(batch, in, out, twx, twy, stream);
            break;
        default: break;
        }
    }
    if constexpr (NX == 256) {
        if (ny == 16) return run_lds<NX, 16>(batch, in, out, twx, twy, stream);
        if (ny == 32) return run_lds<NX, 32>(batch, in, out, twx, twy, stream);
        if (ny == 64) return run_lds<NX, 64>(batch, in, out, twx, twy, stream);
    }
    // two passes through global memory
    epic_status s = run_rows<NX>(batch * ny, in, out, twx, stream);
    if (s != EPIC_OK) return s;
    switch (ny) {
    case 16: return run_cols<NX, 16>(batch, out, twy, stream);
    case 32: return run_cols<NX, 32>(batch, out, twy, stream);
    case 64: return run_cols<NX, 64>(batch, out, twy, stream);
    case 128: return run_cols<NX, 128>(batch, out, twy, stream);
    case 256: return run_cols<NX, 256>(batch, out, twy, stream);
    }
    return fail(EPIC_ERR_INTERNAL, "fft2: unexpected ny");
}

}  // namespace

epic_status launch_fft2_f32(int nx, int ny, int64_t batch, const float2 *in, float2 *out,
                            int device, hipStream_t stream)
{
    const float2 *twx = nullptr, *twy = nullptr;
    epic_status s = get_twiddles(nx, device, &twx);
    if (s != EPIC_OK) return s;
    s = get_twiddles(ny, device, &twy);
    if (s != EPIC_OK) return s;
    switch (nx) {
    case 16: return dispatch_ny<16>(ny, batch, in, out, twx, twy, stream);
    case 32: return dispatch_ny<32>(ny, batch, in, out, twx, twy, stream);
    case 64: return dispatch_ny<64>(ny, batch, in, out, twx, twy, stream);
    case 128: return dispatch_ny<128>(ny, batch, in, out, twx, twy, stream);
    case 256: return dispatch_ny<256>(ny, batch, in, out, twx, twy, stream);
    }
    return fail(EPIC_ERR_INTERNAL, "fft2: unexpected nx");
}

}  // namespace epic
