// internal.hpp -- declarations shared by the host code and the HIP kernels of
// the EPIC imager library.  Nothing here is part of the public ABI (epic.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "epic.h"
#include "plan_host.hpp"
#include "queue.hpp"

namespace epic {

// ---------------------------------------------------------------------------
// Plan tables (built on the host in FP64, stored in FP32 on the device).
//
// For one (station, channel) the kernel footprints of all elements cover the
// cell box [x0, x0+bw) x [y0, y0+bh).  Gridding is a gather: every box cell
// owns the list of (element, weight) taps that land on it, in ascending
// element order, so each cell's sum has a fixed order and needs no atomics.
// ---------------------------------------------------------------------------
// Tap and ChanPlan: plan_host.hpp.

// The cells along one axis (n cells) that the 128 x 128 split-precision
// transform reads of a plane whose non-zero cells lie in [lo, lo + len): the
// ceil(len / 16) tiles of 16 cells from lo, moved back where they would pass
// the plane's edge.
__host__ __device__ __forceinline__ void tile_span(int lo, int len, int n, int &r0, int &tiles)
{
    tiles = (len + 15) >> 4;
    r0 = lo < n - 16 * tiles ? lo : n - 16 * tiles;
}

// Device-side view of one station's plan and buffers (kernel argument).
struct StationDev {
    const ChanPlan *chan;     // [n_chan]
    const int32_t *cell_start;// per channel: [bw*bh + 1] offsets relative to tap_off
    const Tap *taps;          // per channel: taps in cell order
    const int32_t *cell_order;// per channel: box cells by descending tap count (cell_off based)
    const void *volts;        // [n_chan][n_time][n_elem][n_pol]
    float2 *image;            // [n_chan][n_pol^2][ny][nx]
    int32_t n_elem;
    int32_t nx, ny;
    int32_t log2n;            // log2(nx) (square grids in the fused kernels)
    int32_t ktaps;            // taps per element (support^2): n_elem*ktaps taps per channel
    int32_t max_cells;        // max footprint-box cells over channels
    int32_t max_cell_taps;    // max taps landing on one cell over channels
    int32_t max_bw, max_bh;   // largest footprint box sides over channels
    const Tap *band_taps;     // row-band gather (stations of >= kBandMinElem elements), else null:
    const int32_t *band_row;  //   taps by element slot, first slot of each row [n_chan][ny + 1],
    const int32_t *band_slot; //   element -> slot [n_chan][n_elem]
    int32_t max_band;         //   most slots reaching one row
    int32_t half_support;     // (kernel support - 1) / 2
};

// A batch of fused work: items (station index, channel, time chunk, band or
// 0) over a device table of stations, plus the class-wide maxima the LDS
// layout uses.  Persistent kernels take their items from the queue q with
// `grid` work-groups.
struct FusedBatch {
    const StationDev *sds = nullptr;   // device [n_stations]
    const int4 *items = nullptr;       // device [n_items]
    ItemQueue q{};
    int grid = 0;
    int variant = 0;                   // tile choice of the class (autotuned)
    int n_items = 0;
    int max_elem = 0;                  // max n_elem over the batch's stations
    int max_cells = 0;                 // max footprint-box cells
    int max_cell_taps = 0;
    int max_ktaps = 0;                 // max kernel taps per element (support^2)
    int max_side = 0;                  // max footprint-box side
    int max_bw = 0, max_bh = 0;        // max footprint-box width, height
    int n = 0;                         // grid size (square) shared by the batch
};

// ---------------------------------------------------------------------------
// Error reporting (thread-local detail string).
// ---------------------------------------------------------------------------
epic_status hip_fail(hipError_t e, const char *what);

// Every library-owned device allocation goes through here.  Test hook: with
// EPIC_TEST_FAIL_ALLOC=1 in the environment every one of them fails with
// EPIC_ERR_OUT_OF_MEMORY (and nothing is allocated).
epic_status dev_alloc(void **p, size_t bytes);

#define EPIC_HIP_TRY(call)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return ::epic::hip_fail(e_, #call); \
    } while (0)

// Brackets one kernel launch with HIP events on its stream while timing is
// enabled (timing.cpp); a no-op otherwise.
class KernelTimer {
  public:
    KernelTimer(const char *name, hipStream_t stream);
    ~KernelTimer();
    KernelTimer(const KernelTimer &) = delete;
    KernelTimer &operator=(const KernelTimer &) = delete;

  private:
    const char *name_;
    hipStream_t stream_;
    hipEvent_t start_ = nullptr, stop_ = nullptr;
    bool active_ = false;
};

// ---------------------------------------------------------------------------
// Plan cache (plan.cpp).
// ---------------------------------------------------------------------------
struct PlanHandle {
    const ChanPlan *chan = nullptr;
    const int32_t *cell_start = nullptr;
    const Tap *taps = nullptr;
    const int32_t *cell_order = nullptr;
    const int32_t *elem_cell = nullptr;   // [n_chan][n_elem]: nearest cell ci | cj << 16
    int32_t max_box = 0;       // max bw*bh over channels
    int32_t max_bw = 0, max_bh = 0;
    int32_t max_cell_taps = 0; // max taps landing on one cell over channels
    int64_t n_taps_total = 0;
    const Tap *band_taps = nullptr;      // row-band gather tables (see HostPlan), or null
    const int32_t *band_row = nullptr;
    const int32_t *band_slot = nullptr;
    int32_t max_band = 0;
};

// Plan of the XFFT route (Eq. 6 gridding of visibilities) of one station.
// Per channel c (fixed strides): elem_w[c][a][2K] = (wx[0..K), wy[0..K)) of
// element a; the non-empty baseline cells ("centres") cent_cell[c][i]
// (x | y << 16) in raster order, their pair ranges
// cent_start[c][i..i+1] (offsets into pairs[c][n_elem^2]); pairs are
// (a | b << 16) with ascending (a, b) inside a centre.  cell_cent[c][cell] is
// the centre index of a cell (-1 if no pair lands there) and cent_base[c] the
// number of centres of the channels before c (cent_base[n_chan] =
// n_cent_total).
struct XfftPlanHandle {
    const float *elem_w = nullptr;
    const int32_t *cent_cell = nullptr;
    const int32_t *cent_start = nullptr;
    const uint32_t *pairs = nullptr;
    const int32_t *cell_cent = nullptr;
    const int64_t *cent_base = nullptr;
    int64_t n_cent_total = 0;
    int32_t K = 0;
};

epic_status get_xfft_plan(const epic_common *common, const epic_station *st, int device,
                          XfftPlanHandle *out);

// Validates the geometry and returns the (cached) device plan of one station.
epic_status get_plan(const epic_common *common, const epic_station *st, int device,
                     PlanHandle *out);

// Device table of exp(+2 pi i k / n), k < n (FP64-generated, FP32 stored),
// and its host form.
epic_status get_twiddles(int n, int device, const float2 **out);
void fill_twiddles(int n, float2 *dst);

// Split-precision DFT tables in MFMA fragment order (k_dft.hip).
epic_status get_dft_tables(int n, int precision, int device, const void **out);

// DFT matrix rows [n][n] as packed (re, im) hi parts, then lo parts (k_dft.hip),
// and its host form (n * n * 8 bytes).
epic_status get_dft_rows(int n, int precision, int device, const uint32_t **out);
void fill_rows_any(int n, int precision, void *dst);

// Fused split-precision cadence for square grids n in {16, 32, 64, 128}: one
// work-group per (station, channel) item over the whole cadence, block sums of
// `flush` samples added to FP64 running sums in the image buffer (accum.hpp),
// which finally receives the mean products.
epic_status launch_fused_dft(const FusedBatch &b, int n_pol, int n_time, int volt_type,
                             int precision, int flush, const uint32_t *dft_rows, hipStream_t stream);

// Whether launch_fused_dft covers a batch with these maxima.
bool fused_dft_supported(const FusedBatch &b, int n_pol, int volt_type);
// The same for 128 x 128 grids (k_fused_dft128.hip; items carry the half of
// the output rows in z), reached through the two calls above.
epic_status launch_fused_dft128(const FusedBatch &b, int n_pol, int n_time, int volt_type, int precision,
                                int flush, const uint32_t *rows, hipStream_t stream);
bool fused_dft128_supported(const FusedBatch &b, int n_pol, int volt_type);

// Library-owned device workspace, per (device, stream, slot); grows on demand.
epic_status get_workspace(int device, hipStream_t stream, int slot, size_t bytes, void **out);

void clear_all_caches();

// The cadence driver (cadence.cpp): groups stations into fused kernel classes,
// launches one kernel per class plus the ordered reductions, replays the whole
// cadence as a hipGraph when it can, and tunes the time-chunk length.
epic_status run_cadence(const epic_common *c, const epic_station *st, int n, const PlanHandle *plans,
                        int device, hipStream_t stream);
epic_status tune_cadence(const epic_common *c, const epic_station *st, int n,
                         const PlanHandle *plans, int device, hipStream_t stream);
void clear_cadence_cache();

// The cadence of stations that the persistent fused kernels cover, with every
// table in a fixed file-scope device array (no allocation; cadence.cpp).
epic_status run_cadence_noalloc(const epic_common *c, const epic_station *st, int n, int device,
                                hipStream_t stream);
size_t noalloc_scratch_bytes();
bool timing_on();

// ---------------------------------------------------------------------------
// Kernel launchers (each .hip file).  All validate nothing: the ABI layer has
// already checked every argument against what the kernel assumes.
// ---------------------------------------------------------------------------
// With region 1, only each channel's tile region (tile_span of its footprint
// box along x and y) is written: the planes are for the split transform's
// footprint mode, which reads nothing else (split_reads_tile_region).  With
// region 2, only the box's rows (all columns) are written, for the two-pass
// FP32 transform's footprint mode.
epic_status launch_grid(const StationDev &sd, int n_pol, int n_chan, int n_time, int volt_type,
                        int t0, int nt, float2 *grid, hipStream_t stream, int region = 0);

// Gridding with full polarimetric complex kernels (k_grid.hip): kernels
// [n_chan][n_elem][n_pol][n_pol][K][K] cf32 applied conjugated at the K x K
// cells around each element's nearest cell elem_cell[c][a].
epic_status launch_grid_pol(const StationDev &sd, const int32_t *elem_cell, const float2 *kernels,
                            int K, int n_pol, int n_chan, int n_time, int volt_type, int t0, int nt,
                            float2 *grid, hipStream_t stream);

// XFFT route (k_xfft.hip).  Correlator (Eq. 4): vis[c][R][R] (R = n_elem *
// n_pol rows in voltage order) = mean over n_time of X X^H.
epic_status launch_xcorr(const void *volts, int volt_type, int R, int n_chan, int n_time,
                         float2 *vis, hipStream_t stream);
// Eq. 6 gridding of vis into grid[c][n_pol^2][ny][nx] (no transform);
// part is a device buffer of n_chan * (2K-1)^2 * n_pol^2 * nx * ny float2.
epic_status launch_vis_grid(const float2 *vis, const XfftPlanHandle &pl, int n_pol, int n_elem,
                            int n_chan, int nx, int ny, float2 *part, float2 *grid,
                            hipStream_t stream);

// Gridding of large stations through a sample-blocked copy of the voltages:
// tv is a device buffer of n_chan * ceil(nt / 8) * n_elem * 8 * n_pol float2.
// With row_twiddles (the nx-point twiddles of get_twiddles) and region 2,
// the row-band gather may also do the row pass of the two-pass FP32
// transform (grids 128 or 256 wide); *rows_done then says whether it did.
epic_status launch_grid_tb(const StationDev &sd, int n_pol, int n_chan, int n_time, int volt_type,
                           int t0, int nt, float2 *tv, float2 *grid, hipStream_t stream,
                           int region = 0, const float2 *row_twiddles = nullptr,
                           bool *rows_done = nullptr);
constexpr int kGridTbMinElem = 1024;   // stations at least this large take that route

// inverse: (1/(nx ny)) sum_k x[k] exp(-2 pi i k.j / N) instead of the + sign
// transform.  With chan set (two-pass grids only, fft_f32_two_pass), batch
// item b is a plane of channel b / items_per_chan whose rows outside that
// channel's footprint box are zero and are never read (nor written by the
// row pass); the output is complete.
bool fft_f32_two_pass(int nx, int ny);
epic_status launch_fft2_f32(int nx, int ny, int64_t batch, const float2 *in, float2 *out,
                            int device, hipStream_t stream, bool inverse = false,
                            const ChanPlan *chan = nullptr, int items_per_chan = 1);
// The column pass alone (forward, in place), after a row pass done by the
// gridding (launch_grid_tb's rows_done): two-pass grids with chan set.
epic_status launch_fft2_f32_cols(int nx, int ny, int64_t batch, float2 *data, int device,
                                 hipStream_t stream, const ChanPlan *chan, int items_per_chan);

epic_status launch_power(int n_pol, int npix, int n_chan, int nt, const float2 *field,
                         float2 *acc_sum, float2 *acc_comp, int finalize_n_time, float2 *image,
                         hipStream_t stream);

// With chan set, batch item b is a plane of channel b / items_per_chan whose
// input is zero outside that channel's footprint box; the transform then sums
// only the footprint's 16-row/16-column tiles (same result).  max_bw / max_bh
// bound the boxes' sides over the channels (they size the LDS of the 128 x 128
// plane kernel).
// Whether launch_dft2_split with a ChanPlan reads only each plane's tile
// region (tile_span of the footprint box) for this grid size.
bool split_reads_tile_region(int nx, int ny);
epic_status launch_dft2_split(int nx, int ny, int64_t batch, int precision, const float2 *in,
                              float2 *out, int device, hipStream_t stream,
                              const ChanPlan *chan = nullptr, int items_per_chan = 1,
                              int max_bw = 0, int max_bh = 0);

// Work-groups of a persistent launch of `kernel` (block threads, lds bytes of
// dynamic LDS): as many as the GPU holds at once, at most n_items.
int persistent_grid(const void *kernel, int block, size_t lds, int n_items);

// Queue counters of a cadence: k_queue_reset clears n ints before the class
// kernels of every cadence run (a kernel, so that a captured graph holds no
// memset node).
epic_status launch_queue_reset(int *counters, int n, hipStream_t stream);
// Zero fill of n bytes (multiple of 4) by a kernel, for the same reason.
epic_status launch_zero(void *p, size_t bytes, hipStream_t stream);

// Whether a register-resident 64 x 64 FP32 kernel covers a batch: variant 0
// the two-pol kernel (n_pol 2), variant 1 the one with both pols per thread
// (any n_pol); the generic kernel runs where neither does.
bool fft64_fits(const FusedBatch &b, int n_pol, int volt_type, int variant);

// Fused FP32 cadence for square grids n in {16, 32, 64}, items and sums as
// launch_fused_dft.
epic_status launch_fused_fft(const FusedBatch &b, int n_pol, int n_time, int volt_type, int flush,
                             const float2 *twiddles, hipStream_t stream);
// Whether the fused FP32 kernels cover a batch with these maxima.
bool fused_fft_supported(const FusedBatch &b, int n_pol, int volt_type);

// The FP32 cadence for 128 x 128 grids (k_fused128.hip): a persistent
// kernel over the batch's (station, channel) items, each over the whole
// cadence; `gblock` samples at a time are gridded into the work-group's
// footprint boxes (boxes + blockIdx * wg_floats; [gblock][pol][max_bh][max_bw]
// float2) and then transformed and squared, and block sums of `flush`
// samples go to FP64 running sums in the image buffer.  b.grid work-groups at
// most (cadence128_grid, which sizes the box buffer).
bool fused128_supported(int n, int max_bw, int max_bh, int n_elem, int n_pol, int volt_type,
                        int ktaps, int max_cell_taps);
int cadence128_grid(int n_pol, int volt_type, int n_items);
epic_status launch_cadence128(const FusedBatch &b, int n_pol, int n_time, int volt_type, int flush, int gblock,
                              float2 *boxes, size_t wg_floats, const float2 *twiddles, hipStream_t stream);

// Incoherent combination of station images (k_combine.hip): device pointers
// of up to kMaxCombine station images, passed by value as a kernel argument.
constexpr int kMaxCombine = 128;
struct StationImages {
    const float2 *p[kMaxCombine];
};
epic_status launch_combine(const StationImages &imgs, int n_stations, int plane, int n_chan,
                           const float *weights, float2 *out, hipStream_t stream);

// Corner turn of coherent inter-station EPIC (k_beams.hip): station fields
// beams.p[m] [n_chan][n_time][n_pol][npix_b] (up to kMaxCombine stations) ->
// out[i][t][m][p] for problems i = item0 .. item0 + n_items - 1 of the order
// c * n_sel + s, beam pixel pix[s] (device array).
epic_status launch_gather_beams(const StationImages &beams, int n_st, int n_pol, int n_time,
                                int npix_b, int n_sel, const int32_t *pix, int64_t item0,
                                int64_t n_items, float2 *out, hipStream_t stream);

}  // namespace epic
