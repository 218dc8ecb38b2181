// abi.cpp -- the C ABI of include/epic.h: argument validation, plan lookup
// and dispatch to the HIP kernels.  No device work happens before every
// argument has been checked.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace epic;

namespace epic {
StationDev make_station_dev(const epic_station *s, const PlanHandle &p);
epic_status cadence_composed(const epic_common *c, const epic_station *s, const PlanHandle &p,
                             int device, hipStream_t stream, const float2 *pol_kernels = nullptr);
epic_status xfft_image_run(const epic_common *common, const epic_station *station,
                           const float2 *vis, float2 *gridded, int dev, hipStream_t stream);
epic_status array_run(const epic_common *common, const epic_station *array,
                      const void *const *beams, int32_t beam_nx, int32_t beam_ny, int32_t n_sel,
                      const int32_t *pixels, bool xfft, hipStream_t stream);
}

namespace {

int ilog2(int n)
{
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

epic_status current_device(int *dev)
{
    hipError_t e = hipGetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    return EPIC_OK;
}

}  // namespace

StationDev epic::make_station_dev(const epic_station *s, const PlanHandle &p)
{
    StationDev d{};
    d.chan = p.chan;
    d.cell_start = p.cell_start;
    d.taps = p.taps;
    d.cell_order = p.cell_order;
    d.volts = s->volts;
    d.image = static_cast<float2 *>(s->image);
    d.n_elem = s->n_elem;
    d.nx = s->nx;
    d.ny = s->ny;
    d.log2n = ilog2(s->nx);
    d.ktaps = s->kernel.support * s->kernel.support;
    d.max_cells = p.max_box;
    d.max_cell_taps = p.max_cell_taps;
    d.max_bw = p.max_bw;
    d.max_bh = p.max_bh;
    d.band_taps = p.band_taps;
    d.band_row = p.band_row;
    d.band_slot = p.band_slot;
    d.max_band = p.max_band;
    d.half_support = (s->kernel.support - 1) / 2;
    return d;
}

// The composed cadence path: grid -> transform -> square/accumulate through a
// library-owned workspace, in time chunks.  Used for the grids and precisions
// that the fused kernel does not cover, and for gridding with full
// polarimetric kernels (pol_kernels non-null).
epic_status epic::cadence_composed(const epic_common *c, const epic_station *s,
                                   const PlanHandle &p, int device, hipStream_t stream,
                                   const float2 *pol_kernels)
{
    const int n_pol = c->n_pol, n_chan = c->n_chan;
    const int64_t npix = static_cast<int64_t>(s->nx) * s->ny;
    const int64_t per_sample = static_cast<int64_t>(n_chan) * n_pol * npix * 8;  // bytes
    // chunk so that the field workspace stays near 4 GiB (EPIC_FIELD_BUDGET_MB
    // overrides): each chunk reads and writes the accumulators once, so longer
    // chunks save that traffic
    int64_t budget = 4LL << 30;
    if (const char *e = std::getenv("EPIC_FIELD_BUDGET_MB")) budget = std::max<int64_t>(1, std::atoll(e)) << 20;
    int chunk = static_cast<int>(std::max<int64_t>(1, budget / per_sample));
    chunk = std::min(chunk, c->n_time);
    const size_t acc_bytes = static_cast<size_t>(n_chan) * n_pol * n_pol * npix * 8;
    void *ws_field = nullptr, *ws_acc = nullptr;
    epic_status st = get_workspace(device, stream, 0, static_cast<size_t>(per_sample) * chunk, &ws_field);
    if (st != EPIC_OK) return st;
    st = get_workspace(device, stream, 1, 2 * acc_bytes, &ws_acc);
    if (st != EPIC_OK) return st;
    float2 *acc_sum = static_cast<float2 *>(ws_acc);
    float2 *acc_comp = acc_sum + acc_bytes / 8;
    // a fill kernel, not a memset: the cadence may be captured into a graph
    st = launch_zero(ws_acc, 2 * acc_bytes, stream);
    if (st != EPIC_OK) return st;
    const StationDev sd = make_station_dev(s, p);
    float2 *field = static_cast<float2 *>(ws_field);
    // the transform's footprint mode reads only each plane's tile region
    // (split precision, 128 x 128) or the box's rows (FP32, two-pass grids):
    // the gridding writes nothing else
    const bool f32 = c->precision == EPIC_FP32_FFT;
    const int region = pol_kernels ? 0
                       : !f32 && split_reads_tile_region(s->nx, s->ny) ? 1
                       : f32 && fft_f32_two_pass(s->nx, s->ny) ? 2 : 0;
    // large stations, and every station gridded by region: sample-blocked
    // voltage copy for the gather (k_grid.hip)
    float2 *tv = nullptr;
    if ((s->n_elem >= kGridTbMinElem || region == 1) && !pol_kernels) {
        void *ws_tv = nullptr;
        const size_t tv_bytes = sizeof(float2) * static_cast<size_t>(n_chan) * ((chunk + 7) / 8) * 8 *
                                s->n_elem * n_pol;
        st = get_workspace(device, stream, 2, tv_bytes, &ws_tv);
        if (st != EPIC_OK) return st;
        tv = static_cast<float2 *>(ws_tv);
    }
    for (int t0 = 0; t0 < c->n_time; t0 += chunk) {
        const int nt = std::min(chunk, c->n_time - t0);
        bool rows_done = false;
        if (pol_kernels)
            st = launch_grid_pol(sd, p.elem_cell, pol_kernels, s->kernel.support, n_pol, n_chan,
                                 c->n_time, c->volt_type, t0, nt, field, stream);
        else if (tv) {
            // FP32 two-pass grids: the row-band gather may do the row pass too
            const float2 *twx = nullptr;
            if (region == 2) {
                st = get_twiddles(s->nx, device, &twx);
                if (st != EPIC_OK) return st;
            }
            st = launch_grid_tb(sd, n_pol, n_chan, c->n_time, c->volt_type, t0, nt, tv, field, stream,
                                region, twx, &rows_done);
        } else {
            st = launch_grid(sd, n_pol, n_chan, c->n_time, c->volt_type, t0, nt, field, stream, region);
        }
        if (st != EPIC_OK) return st;
        const int64_t batch = static_cast<int64_t>(n_chan) * nt * n_pol;
        if (f32 && rows_done)
            st = launch_fft2_f32_cols(s->nx, s->ny, batch, field, device, stream, sd.chan, nt * n_pol);
        else if (f32)
            st = launch_fft2_f32(s->nx, s->ny, batch, field, field, device, stream, false,
                                 region == 2 ? sd.chan : nullptr, nt * n_pol);
        else
            // the planes are zero outside each channel's footprint box: the
            // transform sums over the box's tiles only
            st = launch_dft2_split(s->nx, s->ny, batch, c->precision, field, field, device, stream,
                                   sd.chan, nt * n_pol, p.max_bw, p.max_bh);
        if (st != EPIC_OK) return st;
        const bool last = t0 + nt >= c->n_time;
        st = launch_power(n_pol, static_cast<int>(npix), n_chan, nt, field, acc_sum, acc_comp,
                          last ? c->n_time : 0, static_cast<float2 *>(s->image), stream);
        if (st != EPIC_OK) return st;
    }
    return EPIC_OK;
}

// Eq. 6 gridding of visibilities and the transform into station->image, for
// arguments already checked (xfft_image, array_xfft).
epic_status epic::xfft_image_run(const epic_common *common, const epic_station *station,
                                 const float2 *vis, float2 *gridded, int dev, hipStream_t stream)
{
    XfftPlanHandle pl;
    epic_status st = get_xfft_plan(common, station, dev, &pl);
    if (st != EPIC_OK) return st;
    const int n_pol = common->n_pol, nx = station->nx, ny = station->ny;
    const int64_t batch = static_cast<int64_t>(common->n_chan) * n_pol * n_pol;
    float2 *g = gridded;
    if (!g) {
        void *ws = nullptr;
        st = get_workspace(dev, stream, 4, sizeof(float2) * static_cast<size_t>(batch) * nx * ny, &ws);
        if (st != EPIC_OK) return st;
        g = static_cast<float2 *>(ws);
    }
    const int W = 2 * station->kernel.support - 1;
    void *part = nullptr;
    st = get_workspace(dev, stream, 5, sizeof(float2) * static_cast<size_t>(batch) * W * W * nx * ny,
                       &part);
    if (st != EPIC_OK) return st;
    st = launch_vis_grid(vis, pl, n_pol, station->n_elem, common->n_chan, nx, ny,
                         static_cast<float2 *>(part), g, stream);
    if (st != EPIC_OK) return st;
    return launch_fft2_f32(nx, ny, batch, g, static_cast<float2 *>(station->image), dev, stream);
}

// Coherent inter-station imaging over station fields (Sec. 6.2): the corner
// turn of every chunk of (channel, beam pixel) problems, then either the
// EPIC cadence (Eq. 10, 9) or the XFFT route (Eq. 11, 13) at array scale.
epic_status epic::array_run(const epic_common *common, const epic_station *array,
                            const void *const *beams, int32_t beam_nx, int32_t beam_ny,
                            int32_t n_sel, const int32_t *pixels, bool xfft, hipStream_t stream)
{
    set_error("");
    epic_status st = check_common(common);
    if (st != EPIC_OK) return st;
    if (!array) return fail(EPIC_ERR_INVALID_ARG, "array is NULL");
    st = check_station(array, 0, false);
    if (st != EPIC_OK) return st;
    if (!array->image) return fail(EPIC_ERR_INVALID_ARG, "array image is NULL");
    const int n_st = array->n_elem;
    if (n_st > kMaxCombine) return fail(EPIC_ERR_INVALID_ARG, "at most 128 stations");
    if (!beams) return fail(EPIC_ERR_INVALID_ARG, "beams is NULL");
    StationImages bt{};
    for (int m = 0; m < n_st; ++m) {
        if (!beams[m]) return fail(EPIC_ERR_INVALID_ARG, "a station beam pointer is NULL");
        bt.p[m] = static_cast<const float2 *>(beams[m]);
    }
    if (!is_pow2_grid(beam_nx) || !is_pow2_grid(beam_ny))
        return fail(EPIC_ERR_INVALID_ARG, "beam_nx, beam_ny must be powers of two in 16..256");
    if (n_sel < 1 || !pixels) return fail(EPIC_ERR_INVALID_ARG, "need n_sel >= 1 selected pixels");
    const int npix_b = beam_nx * beam_ny;
    for (int s = 0; s < n_sel; ++s)
        if (pixels[s] < 0 || pixels[s] >= npix_b)
            return fail(EPIC_ERR_INVALID_ARG, "selected pixel " + std::to_string(s) + " is off the beam grid");
    if (xfft && 2 * array->kernel.support - 1 > std::min(array->nx, array->ny))
        return fail(EPIC_ERR_UNSUPPORTED, "visibility kernel wider than the array grid");
    st = check_geometry(common, array);
    if (st != EPIC_OK) return fail(st, std::string("array: ") + last_error_cstr());
    int dev = 0;
    st = current_device(&dev);
    if (st != EPIC_OK) return st;
    void *ws_pix = nullptr, *ws_v = nullptr, *ws_vis = nullptr;
    st = get_workspace(dev, stream, 7, sizeof(int32_t) * static_cast<size_t>(n_sel), &ws_pix);
    if (st != EPIC_OK) return st;
    EPIC_HIP_TRY(hipMemcpyAsync(ws_pix, pixels, sizeof(int32_t) * n_sel, hipMemcpyHostToDevice, stream));
    // the (channel, pixel) problems in chunks whose array-scale voltages fit 1 GiB
    const int n_pol = common->n_pol;
    const int R = n_st * n_pol;
    const int64_t per_item = static_cast<int64_t>(common->n_time) * n_st * n_pol * 8;
    const int64_t total = static_cast<int64_t>(common->n_chan) * n_sel;
    int64_t budget = int64_t{1} << 30;
    if (const char *e = std::getenv("EPIC_ARRAY_BUDGET_KB")) budget = std::max<int64_t>(1, std::atoll(e)) << 10;
    int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(total, budget / per_item));
    if (xfft)   // the XFFT plan holds n_st^2 pairs per problem
        chunk = std::min<int64_t>(chunk, std::max<int64_t>(1, (int64_t{1} << 31) / (int64_t{n_st} * n_st)));
    st = get_workspace(dev, stream, 6, static_cast<size_t>(chunk * per_item), &ws_v);
    if (st != EPIC_OK) return st;
    if (xfft) {
        st = get_workspace(dev, stream, 8, sizeof(float2) * static_cast<size_t>(chunk) * R * R, &ws_vis);
        if (st != EPIC_OK) return st;
    }
    const size_t plane = static_cast<size_t>(n_pol) * n_pol * array->nx * array->ny;
    for (int64_t i0 = 0; i0 < total; i0 += chunk) {
        const int n = static_cast<int>(std::min(chunk, total - i0));
        st = launch_gather_beams(bt, n_st, n_pol, common->n_time, npix_b, n_sel,
                                 static_cast<const int32_t *>(ws_pix), i0, n,
                                 static_cast<float2 *>(ws_v), stream);
        if (st != EPIC_OK) return st;
        std::vector<double> lam(n);
        for (int k = 0; k < n; ++k) lam[k] = common->wavelength_m[(i0 + k) / n_sel];
        epic_common c2 = *common;
        c2.n_chan = n;
        c2.wavelength_m = lam.data();
        c2.volt_type = EPIC_CF32;
        epic_station s2 = *array;
        s2.volts = ws_v;
        s2.image = static_cast<float2 *>(array->image) + static_cast<size_t>(i0) * plane;
        if (xfft) {
            st = launch_xcorr(ws_v, EPIC_CF32, R, n, common->n_time, static_cast<float2 *>(ws_vis), stream);
            if (st != EPIC_OK) return st;
            st = xfft_image_run(&c2, &s2, static_cast<const float2 *>(ws_vis), nullptr, dev, stream);
        } else {
            PlanHandle p;
            st = get_plan(&c2, &s2, dev, &p);
            if (st != EPIC_OK) return st;
            st = run_cadence(&c2, &s2, 1, &p, dev, stream);
        }
        if (st != EPIC_OK) return st;
    }
    return EPIC_OK;
}

extern "C" {

const char *epic_status_string(epic_status status)
{
    switch (status) {
    case EPIC_OK: return "EPIC_OK";
    case EPIC_ERR_INVALID_ARG: return "EPIC_ERR_INVALID_ARG";
    case EPIC_ERR_UNSUPPORTED: return "EPIC_ERR_UNSUPPORTED";
    case EPIC_ERR_OUT_OF_MEMORY: return "EPIC_ERR_OUT_OF_MEMORY";
    case EPIC_ERR_DEVICE: return "EPIC_ERR_DEVICE";
    case EPIC_ERR_INTERNAL: return "EPIC_ERR_INTERNAL";
    }
    return "EPIC_ERR_UNKNOWN";
}

const char *epic_last_error(void) { return last_error_cstr(); }

void epic_cache_clear(void)
{
    clear_cadence_cache();
    clear_all_caches();
}

epic_status epic_validate(const epic_common *common, const epic_station *stations,
                          int32_t n_stations)
{
    set_error("");
    epic_status st = check_common(common);
    if (st != EPIC_OK) return st;
    if (!stations || n_stations < 1) return fail(EPIC_ERR_INVALID_ARG, "need >= 1 station");
    for (int i = 0; i < n_stations; ++i) {
        st = check_station(&stations[i], i);
        if (st != EPIC_OK) return st;
        st = check_geometry(common, &stations[i]);
        if (st != EPIC_OK) return fail(st, "station " + std::to_string(i) + ": " + last_error_cstr());
    }
    return EPIC_OK;
}

epic_status grid_voltages(const epic_common *common, const epic_station *station, int32_t t0,
                          int32_t nt, void *grid, hipStream_t stream)
{
    set_error("");
    epic_status st = check_common(common);
    if (st != EPIC_OK) return st;
    if (!station) return fail(EPIC_ERR_INVALID_ARG, "station is NULL");
    st = check_station(station, 0);
    if (st != EPIC_OK) return st;
    if (t0 < 0 || nt < 1 || static_cast<int64_t>(t0) + nt > common->n_time)
        return fail(EPIC_ERR_INVALID_ARG, "need 0 <= t0, nt >= 1, t0 + nt <= n_time");
    if (!grid) return fail(EPIC_ERR_INVALID_ARG, "grid is NULL");
    int dev = 0;
    st = current_device(&dev);
    if (st != EPIC_OK) return st;
    PlanHandle p;
    st = get_plan(common, station, dev, &p);
    if (st != EPIC_OK) return st;
    const StationDev sd = make_station_dev(station, p);
    if (station->n_elem >= kGridTbMinElem) {
        // large stations: the samples are first made contiguous per element
        // (same taps, same order, same bits)
        void *ws_tv = nullptr;
        const size_t tv_bytes = sizeof(float2) * static_cast<size_t>(common->n_chan) * ((nt + 7) / 8) * 8 *
                                station->n_elem * common->n_pol;
        st = get_workspace(dev, stream, 2, tv_bytes, &ws_tv);
        if (st != EPIC_OK) return st;
        return launch_grid_tb(sd, common->n_pol, common->n_chan, common->n_time, common->volt_type, t0, nt,
                              static_cast<float2 *>(ws_tv), static_cast<float2 *>(grid), stream);
    }
    return launch_grid(sd, common->n_pol, common->n_chan, common->n_time, common->volt_type, t0, nt,
                       static_cast<float2 *>(grid), stream);
}

epic_status grid_voltages_pol(const epic_common *common, const epic_station *station,
                              const void *kernels, int32_t t0, int32_t nt, void *grid,
                              hipStream_t stream)
{
    set_error("");
    epic_status st = check_common(common);
    if (st != EPIC_OK) return st;
    if (!station) return fail(EPIC_ERR_INVALID_ARG, "station is NULL");
    st = check_station(station, 0);
    if (st != EPIC_OK) return st;
    if (!kernels) return fail(EPIC_ERR_INVALID_ARG, "kernels is NULL");
    if (t0 < 0 || nt < 1 || static_cast<int64_t>(t0) + nt > common->n_time)
        return fail(EPIC_ERR_INVALID_ARG, "need 0 <= t0, nt >= 1, t0 + nt <= n_time");
    if (!grid) return fail(EPIC_ERR_INVALID_ARG, "grid is NULL");
    int dev = 0;
    st = current_device(&dev);
    if (st != EPIC_OK) return st;
    PlanHandle p;
    st = get_plan(common, station, dev, &p);
    if (st != EPIC_OK) return st;
    return launch_grid_pol(make_station_dev(station, p), p.elem_cell,
                           static_cast<const float2 *>(kernels), station->kernel.support,
                           common->n_pol, common->n_chan, common->n_time, common->volt_type, t0, nt,
                           static_cast<float2 *>(grid), stream);
}

epic_status image_cadence_pol(const epic_common *common, const epic_station *station,
                              const void *kernels, hipStream_t stream)
{
    set_error("");
    epic_status st = check_common(common);
    if (st != EPIC_OK) return st;
    if (!station) return fail(EPIC_ERR_INVALID_ARG, "station is NULL");
    st = check_station(station, 0);
    if (st != EPIC_OK) return st;
    if (!kernels) return fail(EPIC_ERR_INVALID_ARG, "kernels is NULL");
    if (!station->image) return fail(EPIC_ERR_INVALID_ARG, "station image is NULL");
    int dev = 0;
    st = current_device(&dev);
    if (st != EPIC_OK) return st;
    PlanHandle p;
    st = get_plan(common, station, dev, &p);
    if (st != EPIC_OK) return st;
    return cadence_composed(common, station, p, dev, stream, static_cast<const float2 *>(kernels));
}

epic_status fft2_batched(int32_t nx, int32_t ny, int64_t batch, int32_t precision, const void *in,
                         void *out, hipStream_t stream)
{
    set_error("");
    if (!is_pow2_grid(nx) || !is_pow2_grid(ny))
        return fail(EPIC_ERR_INVALID_ARG, "nx, ny must be powers of two in 16..256");
    if (batch < 1) return fail(EPIC_ERR_INVALID_ARG, "batch must be >= 1");
    if (!in || !out) return fail(EPIC_ERR_INVALID_ARG, "in/out is NULL");
    if (precision != EPIC_FP32_FFT && precision != EPIC_FP16_SPLIT && precision != EPIC_BF16_SPLIT)
        return fail(EPIC_ERR_INVALID_ARG, "unknown precision");
    int dev = 0;
    epic_status st = current_device(&dev);
    if (st != EPIC_OK) return st;
    if (precision == EPIC_FP32_FFT)
        return launch_fft2_f32(nx, ny, batch, static_cast<const float2 *>(in),
                               static_cast<float2 *>(out), dev, stream);
    return launch_dft2_split(nx, ny, batch, precision, static_cast<const float2 *>(in),
                             static_cast<float2 *>(out), dev, stream);
}

epic_status accumulate_power(int32_t n_pol, int32_t nx, int32_t ny, int32_t n_chan, int32_t nt,
                             const void *field, void *acc_sum, void *acc_comp,
                             int32_t finalize_n_time, void *image, hipStream_t stream)
{
    set_error("");
    if (n_pol != 1 && n_pol != 2) return fail(EPIC_ERR_INVALID_ARG, "n_pol must be 1 or 2");
    if (!is_pow2_grid(nx) || !is_pow2_grid(ny))
        return fail(EPIC_ERR_INVALID_ARG, "nx, ny must be powers of two in 16..256");
    if (n_chan < 1 || nt < 1) return fail(EPIC_ERR_INVALID_ARG, "n_chan and nt must be >= 1");
    if (!field || !acc_sum || !acc_comp) return fail(EPIC_ERR_INVALID_ARG, "NULL buffer");
    if (finalize_n_time < 0) return fail(EPIC_ERR_INVALID_ARG, "finalize_n_time must be >= 0");
    if (finalize_n_time > 0 && !image) return fail(EPIC_ERR_INVALID_ARG, "image is NULL");
    return launch_power(n_pol, nx * ny, n_chan, nt, static_cast<const float2 *>(field),
                        static_cast<float2 *>(acc_sum), static_cast<float2 *>(acc_comp),
                        finalize_n_time, static_cast<float2 *>(image), stream);
}

epic_status image_to_visibilities(int32_t n_pol, int32_t nx, int32_t ny, int32_t n_chan,
                                  const void *image, void *vis, hipStream_t stream)
{
    set_error("");
    if (n_pol != 1 && n_pol != 2) return fail(EPIC_ERR_INVALID_ARG, "n_pol must be 1 or 2");
    if (!is_pow2_grid(nx) || !is_pow2_grid(ny))
        return fail(EPIC_ERR_INVALID_ARG, "nx, ny must be powers of two in 16..256");
    if (n_chan < 1) return fail(EPIC_ERR_INVALID_ARG, "n_chan must be >= 1");
    if (!image || !vis) return fail(EPIC_ERR_INVALID_ARG, "image/vis is NULL");
    int dev = 0;
    epic_status st = current_device(&dev);
    if (st != EPIC_OK) return st;
    const int64_t batch = static_cast<int64_t>(n_chan) * n_pol * n_pol;
    return launch_fft2_f32(nx, ny, batch, static_cast<const float2 *>(image), static_cast<float2 *>(vis),
                           dev, stream, true);
}

epic_status combine_incoherent(int32_t n_pol, int32_t nx, int32_t ny, int32_t n_chan,
                               int32_t n_stations, const void *const *images,
                               const float *weights, void *out, hipStream_t stream)
{
    set_error("");
    if (n_pol != 1 && n_pol != 2) return fail(EPIC_ERR_INVALID_ARG, "n_pol must be 1 or 2");
    if (!is_pow2_grid(nx) || !is_pow2_grid(ny))
        return fail(EPIC_ERR_INVALID_ARG, "nx, ny must be powers of two in 16..256");
    if (n_chan < 1 || n_chan > 65535) return fail(EPIC_ERR_INVALID_ARG, "n_chan must be in 1..65535");
    if (n_stations < 1 || n_stations > kMaxCombine)
        return fail(EPIC_ERR_INVALID_ARG, "n_stations must be in 1..128");
    if (!images || !out) return fail(EPIC_ERR_INVALID_ARG, "images/out is NULL");
    StationImages imgs{};
    for (int m = 0; m < n_stations; ++m) {
        if (!images[m]) return fail(EPIC_ERR_INVALID_ARG, "a station image pointer is NULL");
        imgs.p[m] = static_cast<const float2 *>(images[m]);
    }
    return launch_combine(imgs, n_stations, n_pol * n_pol * nx * ny, n_chan, weights,
                          static_cast<float2 *>(out), stream);
}

epic_status xfft_correlate(const epic_common *common, const epic_station *station, void *vis,
                           hipStream_t stream)
{
    set_error("");
    epic_status st = check_common(common);
    if (st != EPIC_OK) return st;
    if (!station) return fail(EPIC_ERR_INVALID_ARG, "station is NULL");
    st = check_station(station, 0);
    if (st != EPIC_OK) return st;
    if (!vis) return fail(EPIC_ERR_INVALID_ARG, "vis is NULL");
    if (station->n_elem > 65535) return fail(EPIC_ERR_UNSUPPORTED, "correlator: more than 65535 elements");
    int dev = 0;
    st = current_device(&dev);
    if (st != EPIC_OK) return st;
    return launch_xcorr(station->volts, common->volt_type, station->n_elem * common->n_pol,
                        common->n_chan, common->n_time, static_cast<float2 *>(vis), stream);
}

epic_status xfft_image(const epic_common *common, const epic_station *station, const void *vis,
                       void *gridded, hipStream_t stream)
{
    set_error("");
    epic_status st = check_common(common);
    if (st != EPIC_OK) return st;
    if (!station) return fail(EPIC_ERR_INVALID_ARG, "station is NULL");
    st = check_station(station, 0, false);
    if (st != EPIC_OK) return st;
    if (!vis) return fail(EPIC_ERR_INVALID_ARG, "vis is NULL");
    if (!station->image) return fail(EPIC_ERR_INVALID_ARG, "station image is NULL");
    if (2 * station->kernel.support - 1 > std::min(station->nx, station->ny))
        return fail(EPIC_ERR_UNSUPPORTED, "visibility kernel wider than the grid");
    int dev = 0;
    st = current_device(&dev);
    if (st != EPIC_OK) return st;
    return xfft_image_run(common, station, static_cast<const float2 *>(vis),
                          static_cast<float2 *>(gridded), dev, stream);
}

epic_status array_cadence(const epic_common *common, const epic_station *array,
                          const void *const *beams, int32_t beam_nx, int32_t beam_ny,
                          int32_t n_sel, const int32_t *pixels, hipStream_t stream)
{
    return array_run(common, array, beams, beam_nx, beam_ny, n_sel, pixels, false, stream);
}

epic_status array_xfft(const epic_common *common, const epic_station *array,
                       const void *const *beams, int32_t beam_nx, int32_t beam_ny, int32_t n_sel,
                       const int32_t *pixels, hipStream_t stream)
{
    return array_run(common, array, beams, beam_nx, beam_ny, n_sel, pixels, true, stream);
}

epic_status image_cadence(const epic_common *common, const epic_station *stations,
                          int32_t n_stations, hipStream_t stream)
{
    set_error("");
    epic_status st = check_common(common);
    if (st != EPIC_OK) return st;
    if (!stations || n_stations < 1) return fail(EPIC_ERR_INVALID_ARG, "need >= 1 station");
    for (int i = 0; i < n_stations; ++i) {
        st = check_station(&stations[i], i);
        if (st != EPIC_OK) return st;
        if (!stations[i].image) return fail(EPIC_ERR_INVALID_ARG, "station image is NULL");
    }
    int dev = 0;
    st = current_device(&dev);
    if (st != EPIC_OK) return st;
    // every plan first: geometry errors surface before any launch
    std::vector<PlanHandle> plans(n_stations);
    for (int i = 0; i < n_stations; ++i) {
        st = get_plan(common, &stations[i], dev, &plans[i]);
        if (st != EPIC_OK) return fail(st, "station " + std::to_string(i) + ": " + last_error_cstr());
    }
    return run_cadence(common, stations, n_stations, plans.data(), dev, stream);
}

epic_status image_cadence_noalloc(const epic_common *common, const epic_station *stations,
                                  int32_t n_stations, hipStream_t stream)
{
    set_error("");
    epic_status st = check_common(common);
    if (st != EPIC_OK) return st;
    if (!stations || n_stations < 1) return fail(EPIC_ERR_INVALID_ARG, "need >= 1 station");
    for (int i = 0; i < n_stations; ++i) {
        st = check_station(&stations[i], i);
        if (st != EPIC_OK) return st;
        if (!stations[i].image) return fail(EPIC_ERR_INVALID_ARG, "station image is NULL");
    }
    int dev = 0;
    st = current_device(&dev);
    if (st != EPIC_OK) return st;
    return run_cadence_noalloc(common, stations, n_stations, dev, stream);
}

epic_status epic_autotune(const epic_common *common, const epic_station *stations,
                          int32_t n_stations, hipStream_t stream)
{
    set_error("");
    epic_status st = check_common(common);
    if (st != EPIC_OK) return st;
    if (!stations || n_stations < 1) return fail(EPIC_ERR_INVALID_ARG, "need >= 1 station");
    for (int i = 0; i < n_stations; ++i) {
        st = check_station(&stations[i], i);
        if (st != EPIC_OK) return st;
        if (!stations[i].image) return fail(EPIC_ERR_INVALID_ARG, "station image is NULL");
    }
    int dev = 0;
    st = current_device(&dev);
    if (st != EPIC_OK) return st;
    std::vector<PlanHandle> plans(n_stations);
    for (int i = 0; i < n_stations; ++i) {
        st = get_plan(common, &stations[i], dev, &plans[i]);
        if (st != EPIC_OK) return fail(st, "station " + std::to_string(i) + ": " + last_error_cstr());
    }
    return tune_cadence(common, stations, n_stations, plans.data(), dev, stream);
}

}  // extern "C"
