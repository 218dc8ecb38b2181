/*
 * epic.h -- C ABI of the EPIC direct-imager hot path on gfx950 (MI355X).
 *
 * The imager (Thyagarajan, "Comparison of Fast, Hybrid Imaging Architectures
 * for Multi-scale, Hierarchical Aperture Arrays", Sec. 5.2) forms, for every
 * channel and time sample, the gridded aperture field
 *
 *     G^p[j] = sum_a W~_a(r_j - r_a) E^p_a                        (Eq. 3, inner)
 *
 * transforms it to the sky,
 *
 *     F^p[k] = sum_j exp(+2 pi i k.j / N) G^p[j]                   (Eq. 3, outer)
 *
 * and averages the polarisation outer products over the cadence t_acc,
 *
 *     I^{ab}[k] = < F^a[k] conj(F^b[k]) >                           (Eq. 2).
 *
 * Conventions used by every call (the paper leaves them open):
 *   - Channels are independent (Sec. 5.1).  The grid spacing is fixed in
 *     wavelengths: channel c uses Delta_c = grid_spacing_wl * wavelength_m[c]
 *     metres per cell, so sky pixels are the same directions in every channel.
 *   - Element a sits at u = x/Delta_c + nx/2, v = y/Delta_c + ny/2 (cells),
 *     nearest cell (floor(u+1/2), floor(v+1/2)).  The kernel covers the
 *     support x support cells around the nearest cell.  NEAREST: support 1,
 *     weight 1.  GAUSSIAN: separable exp(-d^2 / (2 sigma^2)) of the distance d
 *     (cells) from the element's true position, normalised to unit sum.  The
 *     kernel is real, so the conjugate of Eq. 3 changes nothing.  A footprint
 *     that leaves the grid at any channel is an error (never wrapped).
 *   - The transform has the + sign, no area factor (delta^2 r = 1) and
 *     natural (unshifted) pixel order: pixel k <-> direction cosine
 *     l = k'/(nx * grid_spacing_wl), k' = k - nx*[k >= nx/2]; same for m.
 *   - Products are stored alpha-major: XX, XY, YX, YY (n_pol = 2) or XX
 *     (n_pol = 1).  YX is written as the exact conjugate of XY; Im XX and
 *     Im YY are exactly 0.
 *   - Complex numbers are interleaved (re, im) pairs: "cf32" = 2 x float,
 *     "ci8" = 2 x int8.
 *
 * Memory: device pointers are HIP device memory on the current device; host
 * pointers are ordinary host memory, read during the call only.  The caller
 * owns every buffer it passes.  The library owns its plan tables (kernel cells
 * and weights per station and channel, uploaded once and cached by content),
 * its transform tables and its workspaces; epic_cache_clear() frees them.
 *
 * Errors: every call validates all arguments before it launches anything and
 * returns a status; 0 is success.  Launches are asynchronous on `stream`
 * (NULL = the null stream); a fault inside a kernel surfaces at the caller's
 * next synchronisation.  epic_last_error() gives a human-readable detail of
 * the last failure on the calling thread.  Calls on different streams may run
 * concurrently; the caches are internally locked.
 */
#ifndef EPIC_H
#define EPIC_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EPIC_OK = 0,
    EPIC_ERR_INVALID_ARG = -1,   /* bad pointer, shape, enum or geometry */
    EPIC_ERR_UNSUPPORTED = -2,   /* valid but not implemented here */
    EPIC_ERR_OUT_OF_MEMORY = -3, /* a library-owned allocation failed */
    EPIC_ERR_DEVICE = -4,        /* a HIP runtime call failed */
    EPIC_ERR_INTERNAL = -5
} epic_status;

typedef enum { EPIC_CI8 = 0, EPIC_CF32 = 1 } epic_volt_type;

/* How the 2-D transform is evaluated.
 *   EPIC_FP32_FFT   : mixed-radix FFT in FP32 (adds and multiplies in FP32).
 *   EPIC_FP16_SPLIT : dense DFT-matrix products F_y . X . F_x^T on FP16 matrix
 *                     cores with FP32 accumulation; each operand is split into
 *                     hi + lo FP16 parts and three products (hi.hi, hi.lo,
 *                     lo.hi) are summed.  The DFT tables are generated in FP64.
 *   EPIC_BF16_SPLIT : the same with BF16 parts. */
typedef enum { EPIC_FP32_FFT = 0, EPIC_FP16_SPLIT = 1, EPIC_BF16_SPLIT = 2 } epic_precision;

typedef enum { EPIC_KERNEL_NEAREST = 0, EPIC_KERNEL_GAUSSIAN = 1 } epic_kernel_type;

/* Element gridding kernel W~ of Eq. 3.  support: odd, 1..7 (NEAREST: 1).
 * sigma_cells: Gaussian width in cells (> 0; ignored for NEAREST). */
typedef struct {
    int32_t type;
    int32_t support;
    double sigma_cells;
} epic_kernel;

/* Parameters shared by all stations of one call. */
typedef struct {
    int32_t n_pol;                /* 1 or 2 */
    int32_t n_chan;               /* >= 1 */
    const double *wavelength_m;   /* host [n_chan], finite, > 0 */
    double grid_spacing_wl;       /* cell size in wavelengths, > 0 (0.5 = lambda/2) */
    int32_t n_time;               /* samples per cadence (t_acc / delta_t), >= 1 */
    int32_t volt_type;            /* epic_volt_type */
    int32_t precision;            /* epic_precision (image_cadence only) */
} epic_common;

/* One station: one independent imaging problem. */
typedef struct {
    int32_t n_elem;               /* >= 1 */
    const double *pos_m;          /* host [n_elem][2]: x, y metres from the station phase centre */
    int32_t nx, ny;               /* grid = image size; powers of two, 16..256 */
    epic_kernel kernel;
    const void *volts;            /* device [n_chan][n_time][n_elem][n_pol] of volt_type */
    void *image;                  /* device out: cf32 [n_chan][n_pol*n_pol][ny][nx],
                                     the mean over n_time (image_cadence only) */
} epic_station;

/*
 * Gridding (Eq. 3, inner bracket) of samples t0 .. t0+nt-1 of every channel
 * of one station.  Writes every cell of
 *     grid: device cf32 [n_chan][nt][n_pol][ny][nx]
 * (cells outside the kernel footprints are written as 0).  The gridded value
 * of a cell is the FP32 sum of weight * voltage over the element taps that
 * land on it, in ascending element order (deterministic; no atomics).
 * Stations of 1024 elements or more first copy the samples, per element and
 * block of 8 samples, into a library-owned workspace (same values).
 * station->image is not used.  0 <= t0, nt >= 1, t0 + nt <= common->n_time.
 */
epic_status grid_voltages(const epic_common *common, const epic_station *station,
                          int32_t t0, int32_t nt, void *grid, hipStream_t stream);

/*
 * Batched 2-D transform of Eq. 3 (outer sum):
 *     out[b][ky][kx] = sum_{y,x} in[b][y][x] exp(+2 pi i (kx x/nx + ky y/ny))
 * in, out: device cf32 [batch][ny][nx]; nx, ny powers of two in 16..256;
 * batch >= 1.  Unnormalised, natural order.  in == out is allowed for every
 * precision (the split paths stage through a library-owned workspace).
 */
epic_status fft2_batched(int32_t nx, int32_t ny, int64_t batch, int32_t precision,
                         const void *in, void *out, hipStream_t stream);

/*
 * Squaring and accumulation (Eq. 2) of nt samples of a per-sample field:
 *     field: device cf32 [n_chan][nt][n_pol][ny][nx]
 *     acc_sum, acc_comp: device cf32 [n_chan][n_pol*n_pol][ny][nx], the running
 *         compensated sum (sum + comp) of F^a conj(F^b).  Zero them before the
 *         first call of a cadence; keep them across calls to split a cadence.
 * Each sample is added with an error-free two-sum, so a cadence split over
 * several calls gives bit-identical results to one call over the same samples
 * in the same order.  If finalize_n_time > 0 the mean
 *     image = (acc_sum + acc_comp) * (1 / finalize_n_time)
 * is also written to image (device cf32, same shape as acc_sum); otherwise
 * image is not touched and may be NULL.
 */
epic_status accumulate_power(int32_t n_pol, int32_t nx, int32_t ny, int32_t n_chan, int32_t nt,
                             const void *field, void *acc_sum, void *acc_comp,
                             int32_t finalize_n_time, void *image, hipStream_t stream);

/*
 * The whole cadence, all steps fused (Eq. 3 then Eq. 2): for every station
 * and channel, grid each sample, transform it with common->precision, form the
 * products and average them over common->n_time samples into station->image.
 * Stations may differ in element count, layout, grid size and kernel; all of
 * them run in one pass.  Plan tables are built on the host in FP64 on the first
 * call for a geometry and reused afterwards.
 */
epic_status image_cadence(const epic_common *common, const epic_station *stations,
                          int32_t n_stations, hipStream_t stream);

/*
 * image_cadence for callers that cannot allocate device memory: code under
 * hipGraph stream capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, layouts and results as image_cadence (the same
 * persistent kernels run; where the autotuner chose the composed path for a
 * class, this call runs the class's persistent kernel instead, so its images
 * then agree with image_cadence's within the tolerances rather than bit for
 * bit), but the call allocates nothing: every table it needs (the
 * stations' kernel cells and weights, the transform tables, the work lists
 * and queue counters) is written into one fixed device array of 64 MiB that
 * the library holds on each GPU until the process ends, and the images
 * themselves carry the running sums.  Covered: stations with square grids up
 * to 64 x 64 at FP32 and up to 128 x 128 in split precision (the persistent
 * kernels); anything else, or a call whose tables exceed the 64 MiB (a
 * 256-element station with a 3 x 3 kernel on a 64 x 64 grid needs about 37 KB
 * per channel), returns EPIC_ERR_UNSUPPORTED before any launch.  The tables are
 * rebuilt on the host and copied on every call (nothing is cached).  The call
 * first waits for the earlier work on `stream`, which may still read the
 * array; calls on one GPU share the array, so calls that overlap on one GPU
 * (different streams or threads) race and must not be made.
 */
epic_status image_cadence_noalloc(const epic_common *common, const epic_station *stations,
                                  int32_t n_stations, hipStream_t stream);

/*
 * FFT-correlator output (Sec. 6.2: an FFT correlator obtains the visibilities
 * by one more, inverse, transform of the polarised intensities; Eq. 4 defines
 * the visibilities and Eq. 6 their gridding with the cross-correlated element
 * kernels).  For every channel and product of an image_cadence output:
 *     vis[c][q][y][x] = 1/(nx ny) sum_{ky,kx} image[c][q][ky][kx]
 *                                            exp(-2 pi i (kx x/nx + ky y/ny)),
 * the inverse of the transform of Eq. 3, which returns the time-averaged
 * visibilities (autocorrelations included) gridded at the baseline cells with
 * the kernels' cross-correlation, on the circular grid.
 * image, vis: device cf32 [n_chan][n_pol*n_pol][ny][nx] (image == vis is
 * allowed); n_pol 1 or 2; nx, ny powers of two in 16..256; n_chan >= 1.
 * FP32.  Errors: EPIC_ERR_INVALID_ARG for shapes or NULL pointers.
 */
epic_status image_to_visibilities(int32_t n_pol, int32_t nx, int32_t ny, int32_t n_chan,
                                  const void *image, void *vis, hipStream_t stream);

/*
 * Incoherent combination of station images (Sec. 6.1, Eq. 7): the weighted
 * mean of the stations' polarised intensities per sky pixel,
 *     out[c][q][k] = sum_m w[m][q][k] images[m][c][q][k] / sum_m w[m][q][k],
 * for stations imaged on one sky pixel grid (same nx, ny and grid spacing in
 * wavelengths, hence the same directions per pixel).
 * images: host array of n_stations device pointers, each cf32
 *         [n_chan][n_pol*n_pol][ny][nx] (image_cadence outputs);
 * weights: device float [n_stations][n_pol*n_pol][ny][nx], the same for every
 *         channel (a station's beam weight towards each pixel), or NULL for
 *         equal weights; pixels whose weights sum to 0 are written as 0;
 * out: device cf32 [n_chan][n_pol*n_pol][ny][nx] (may be one of the images).
 * 1 <= n_stations <= 128.  FP32 sums over the stations in order.
 * Errors: EPIC_ERR_INVALID_ARG for shapes, counts or NULL pointers.
 */
epic_status combine_incoherent(int32_t n_pol, int32_t nx, int32_t ny, int32_t n_chan,
                               int32_t n_stations, const void *const *images,
                               const float *weights, void *out, hipStream_t stream);

/*
 * Gridding with full polarimetric complex kernels (Sec. 5.2, Eq. 3 in its
 * general form): every output pol a collects every input pol p of every
 * element through that element's own complex kernel, applied conjugated,
 *     grid[c][t - t0][a][j] = sum_elem sum_p conj(W[c][elem][a][p][dy][dx]) E_elem^p(t),
 * over the K x K cells j = (c_x - h + dx, c_y - h + dy) around the element's
 * nearest cell c (the cells of grid_voltages; h = (K - 1) / 2, K =
 * station->kernel.support).  This carries an antenna's holographic
 * illumination pattern with its pol leakage and w-projection phase screens
 * (a larger K for non-coplanar elements).
 * kernels: device cf32 [n_chan][n_elem][n_pol (a)][n_pol (p)][K (dy)][K (dx)],
 *          the kernel values at those cells (the caller evaluates them at the
 *          element's true position); station->kernel.type and sigma_cells are
 *          not used;
 * grid:    as for grid_voltages.  FP32 sums over the cell's taps in element
 *          order (deterministic).
 * Errors: as grid_voltages, plus EPIC_ERR_INVALID_ARG for kernels NULL.
 */
epic_status grid_voltages_pol(const epic_common *common, const epic_station *station,
                              const void *kernels, int32_t t0, int32_t nt, void *grid,
                              hipStream_t stream);

/*
 * The whole cadence of one station (Eq. 3 with grid_voltages_pol's kernels,
 * then Eq. 2) into station->image [n_chan][n_pol^2][ny][nx]: gridding,
 * transform (common->precision: the FP32 FFT or a split-precision DFT-matrix
 * product), products and compensated time average, in time chunks through a
 * library workspace.  kernels as for grid_voltages_pol.
 * Errors: as image_cadence, plus EPIC_ERR_INVALID_ARG for kernels NULL.
 */
epic_status image_cadence_pol(const epic_common *common, const epic_station *station,
                              const void *kernels, hipStream_t stream);

/*
 * Correlator of the XFFT architecture (Sec. 5.4, Eq. 4): the visibilities of
 * one station, for every channel c, ordered element pair (a, b)
 * (autocorrelations included) and pol pair (p, q),
 *     vis[c][a][p][b][q] = (1/n_time) sum_t E_a^p(t) conj(E_b^q(t)),
 * i.e. per channel the R x R matrix X X^H / n_time of the rows r = a*n_pol + p
 * (R = n_elem*n_pol; Hermitian, both triangles written).
 * common, station: as for image_cadence (station->volts is read; positions,
 *         grid and image are not used);
 * vis:    device, cf32 [n_chan][n_elem][n_pol][n_elem][n_pol], caller-owned.
 * ci8 voltages are summed exactly in 32-bit integers on the int8 matrix cores
 * (n_time of any length: longer cadences are summed in segments of 65472
 * samples) and scaled by 1/n_time in FP32; cf32 voltages are summed in FP32
 * on the FP32 matrix cores.  Deterministic.
 * Errors: EPIC_ERR_INVALID_ARG for arguments as image_cadence (plus vis
 * NULL); EPIC_ERR_UNSUPPORTED for n_elem > 65535.
 */
epic_status xfft_correlate(const epic_common *common, const epic_station *station, void *vis,
                           hipStream_t stream);

/*
 * Imaging stage of the XFFT architecture (Sec. 5.4, Eq. 6): grids the
 * visibilities of xfft_correlate at their baseline cells c_a - c_b with the
 * cross-correlation of the two elements' kernels,
 *     G[c][p*n_pol+q][j] = sum_{a,b} sum_{i,m} w_a(i) w_b(m) vis[c][a][p][b][q]
 *                          over j = (c_a + i) - (c_b + m) mod (nx, ny),
 * and transforms G as Eq. 3 does (+ sign, unnormalised, natural order) into
 * station->image [n_chan][n_pol^2][ny][nx]: the same polarised intensities
 * image_cadence returns (Wiener-Khinchin on the circular grid), up to FP32
 * rounding.  Cells and weights are those of Eq. 3's gridding (the station's
 * positions, kernel and grid, per channel's wavelength).
 * vis:     device cf32 as xfft_correlate writes it;
 * gridded: device cf32 [n_chan][n_pol^2][ny][nx] that receives G (the
 *          gridded visibilities), or NULL (a library workspace is used);
 * station->volts may be NULL.  The per-station plan (every element pair
 * sorted by baseline cell, n_elem^2 * n_chan entries of 4 bytes) is built on
 * the host once per geometry and cached like image_cadence's.  FP32 sums in a
 * fixed order (deterministic).
 * Errors: EPIC_ERR_INVALID_ARG as image_cadence (footprint off the grid
 * included); EPIC_ERR_UNSUPPORTED for n_elem > 65535, n_elem^2 * n_chan >
 * 2^31, or a visibility kernel (2K - 1 cells) wider than the grid.
 */
epic_status xfft_image(const epic_common *common, const epic_station *station, const void *vis,
                       void *gridded, hipStream_t stream);

/*
 * Coherent inter-station EPIC (Sec. 6.2, Eq. 10 then Eq. 9): the M stations
 * of an array act as the elements of an array-scale EPIC imager.  Each
 * station's synthesised field towards the directions of its sky grid (the
 * per-sample Eq. 3 transform before squaring, e.g. grid_voltages then
 * fft2_batched of that station) is the input; for every channel c and every
 * selected beam pixel k (one direction s_k of the stations' common sky grid),
 * the M fields are gridded at the station positions on the array grid,
 * transformed, squared and averaged over the cadence, as image_cadence does
 * for elements:
 *     image[c][s][p*n_pol+q][y][x],  s = index into pixels.
 * common: n_pol, channels, n_time, precision as for image_cadence;
 *         grid_spacing_wl is the ARRAY grid spacing; volt_type is ignored
 *         (the fields are cf32);
 * array:  the array geometry as a station: n_elem = M (1..128) station
 *         positions pos_m in metres in the array frame, the array grid
 *         (nx, ny) and kernel; volts is ignored; image is the device output,
 *         cf32 [n_chan][n_sel][n_pol^2][ny][nx];
 * beams:  host array of M device pointers, station m's fields cf32
 *         [n_chan][n_time][n_pol][beam_ny][beam_nx] (the stations must share
 *         one sky grid: the same beam_nx, beam_ny and grid spacing in
 *         wavelengths; each field is phase-referenced to its own station's
 *         grid, and the common per-pixel phase this leaves cancels in the
 *         products);
 * pixels: host int32 [n_sel], flat beam pixels ky * beam_nx + kx (natural
 *         order, as the transform writes them).
 * The (channel, pixel) problems are processed in chunks whose array-scale
 * voltages fit 1 GiB of library workspace (EPIC_ARRAY_BUDGET_KB overrides);
 * each chunk runs image_cadence's kernels (plans and graphs are cached per
 * chunk); the chunking never changes the result.
 * Errors: EPIC_ERR_INVALID_ARG for arguments as image_cadence, NULL beams,
 * more than 128 stations, beam grids that are not powers of two in 16..256,
 * or a selected pixel off the beam grid.
 */
epic_status array_cadence(const epic_common *common, const epic_station *array,
                          const void *const *beams, int32_t beam_nx, int32_t beam_ny,
                          int32_t n_sel, const int32_t *pixels, hipStream_t stream);

/*
 * Coherent inter-station imaging by the XFFT route (Sec. 6.2, Eq. 11 then
 * Eq. 13): the same arguments, chunking and output as array_cadence, but each
 * (channel, beam pixel) problem correlates the M station fields over the
 * cadence (the inter-station visibilities phased towards s_k, as
 * xfft_correlate does for elements) and grids them at the station
 * separations with the cross-correlated array kernels before one transform
 * (as xfft_image).  The image equals array_cadence's up to FP32 rounding
 * (Wiener-Khinchin on the circular array grid); the work per problem scales
 * with M^2 instead of the array grid size.
 * Errors: as array_cadence, plus EPIC_ERR_UNSUPPORTED for an array visibility
 * kernel (2K - 1 cells) wider than the array grid.
 */
epic_status array_xfft(const epic_common *common, const epic_station *array,
                       const void *const *beams, int32_t beam_nx, int32_t beam_ny, int32_t n_sel,
                       const int32_t *pixels, hipStream_t stream);

/*
 * Tile tuning (auxiliary).  image_cadence sorts the stations into kernel
 * classes (grid size, footprint tiles, pols, voltage type, precision) and
 * runs each class as one persistent kernel over (station, channel) items.
 * A class's tile is the flush interval (8 or 16 samples summed in FP32
 * before the FP64 running sums) and, where it has several, the kernel shape:
 * the 64 x 64 FP32 kernel with one pol per half of 1024 threads or both pols
 * on 512, the 128 x 128 FP32 kernel's gridding block (1, 2, 4 or 16
 * samples), and for every split-precision class and every FP32 class up to
 * 64 x 64 the composed path (separate gridding, transform and squaring
 * kernels) instead of the persistent kernel.  epic_autotune runs each class
 * of this call with each candidate on the caller's buffers (it overwrites
 * station images), keeps the fastest for later image_cadence calls of the
 * same class and, if the environment variable EPIC_TUNE_CACHE names a file,
 * stores the choices there and reads them back in later processes;
 * epic_cache_clear forgets the choices held in memory.  Synchronises the
 * stream.  The flush interval changes only the grouping of the time
 * average's sums, never the set of samples summed.
 */
epic_status epic_autotune(const epic_common *common, const epic_station *stations,
                          int32_t n_stations, hipStream_t stream);

/*
 * Host-only check of everything image_cadence would check (arguments and
 * geometry: every element's kernel footprint inside its grid at every
 * channel), without touching a device.  Returns EPIC_OK or the error
 * image_cadence would return; the volts and image pointers are not checked.
 */
epic_status epic_validate(const epic_common *common, const epic_station *stations,
                          int32_t n_stations);

/*
 * Kernel timing (auxiliary instrumentation, off by default).  While enabled,
 * every kernel the library launches is bracketed by a pair of HIP events
 * recorded on the kernel's own stream.  epic_timing_report() waits for the
 * recorded events and writes one line per kernel name, "name count total_ms",
 * into buf (NUL-terminated, truncated to len); it returns the number of
 * kernel names.  epic_timing_reset() drops the records.
 */
void epic_timing_enable(int32_t enable);
int32_t epic_timing_report(char *buf, int32_t len);
void epic_timing_reset(void);

/* Static name of a status code. */
const char *epic_status_string(epic_status status);

/* Detail of the last failure on the calling thread ("" if none). */
const char *epic_last_error(void);

/* Free every library-owned device table, workspace and graph, and forget the
 * autotuner's choices (read again from EPIC_TUNE_CACHE when it names a file).
 * Must not race with calls in flight on any stream. */
void epic_cache_clear(void);

#ifdef __cplusplus
}
#endif

#endif /* EPIC_H */
