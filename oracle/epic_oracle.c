/*
 * epic_oracle.c -- plain FP64 CPU oracle for the EPIC direct imager.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this code.  It shares no code, header,
 * table or helper with the GPU library; it recomputes every cell index, weight
 * and twiddle itself, in double precision.
 *
 * What it computes (Thyagarajan, "Comparison of Fast, Hybrid Imaging
 * Architectures ...", Sec. 5.2, Eq. 3 followed by Eq. 2):
 *
 *   G^p[j]      = sum_a  W~_a(r_j - r_a) E^p_a               (gridding, inner
 *                                                            bracket of Eq. 3)
 *   F^p[k]      = sum_j  exp(+2 pi i k.j / N) G^p[j]         (outer sum of Eq. 3,
 *                                                            area factor = 1)
 *   I^{ab}[k]   = < F^a[k] conj(F^b[k]) >_t                   (Eq. 2: pol outer
 *                                                            product, time mean)
 *
 * for every channel independently (Sec. 5.1: each spectral channel is processed
 * on its own).  Readings of points the paper leaves open:
 *   - grid spacing is fixed in wavelengths: Delta_c = grid_spacing_wl * lambda_c;
 *   - element a sits at u = x/Delta_c + nx/2 (integer nx/2), nearest cell
 *     i = floor(u + 1/2), sub-cell offset du = u - i in [-1/2, 1/2);
 *   - kernel: NEAREST (K = 1, weight 1) or a separable Gaussian of width sigma
 *     cells on the K x K cells centred on the nearest cell, evaluated at the
 *     true sub-cell offset and normalised to unit sum.  The kernel is real, so
 *     the conjugate in Eq. 3 changes nothing;
 *   - transform sign +, unnormalised, natural (unshifted) pixel order;
 *   - products in alpha-major order (XX, XY, YX, YY); mean = sum / n_time;
 *   - a kernel footprint that leaves the grid is an error (never wrapped).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define EO_OK 0
#define EO_ERR_ARG -1
#define EO_ERR_OFFGRID -2
#define EO_ERR_NOMEM -3

#define EO_KERNEL_NEAREST 0
#define EO_KERNEL_GAUSSIAN 1
#define EO_VOLT_CI8 0
#define EO_VOLT_CF32 1
#define EO_VOLT_CF64 2

static const double EO_TWO_PI = 6.283185307179586476925286766559;

/*
 * Element kernel taps (Sec. 5.2, Eq. 3; the kernel is centred on the element
 * position r_a).  Writes the nearest cell (ix, iy) and the K separable weights
 * wx[0..K-1], wy[0..K-1] for offsets d = -h..h, h = (K-1)/2.  The 2-D weight of
 * cell (ix+dx, iy+dy) is wx[dx+h]*wy[dy+h].
 */
int eo_element_taps(double x_m, double y_m, double delta_m, int nx, int ny,
                    int kernel_type, int K, double sigma_cells,
                    int *ix, int *iy, double *wx, double *wy)
{
    if (!(delta_m > 0.0) || K < 1 || (K % 2) == 0) return EO_ERR_ARG;
    if (kernel_type == EO_KERNEL_NEAREST && K != 1) return EO_ERR_ARG;
    if (kernel_type == EO_KERNEL_GAUSSIAN && !(sigma_cells > 0.0)) return EO_ERR_ARG;
    const double u = x_m / delta_m + (double)(nx / 2);
    const double v = y_m / delta_m + (double)(ny / 2);
    const double ci = floor(u + 0.5);
    const double cj = floor(v + 0.5);
    const double du = u - ci;
    const double dv = v - cj;
    const int h = (K - 1) / 2;
    if (ci - h < 0 || ci + h > nx - 1 || cj - h < 0 || cj + h > ny - 1)
        return EO_ERR_OFFGRID;
    *ix = (int)ci;
    *iy = (int)cj;
    if (kernel_type == EO_KERNEL_NEAREST) {
        wx[0] = 1.0;
        wy[0] = 1.0;
        return EO_OK;
    }
    double sx = 0.0, sy = 0.0;
    for (int d = -h; d <= h; ++d) {
        const double ex = ((double)d - du) / sigma_cells;
        const double ey = ((double)d - dv) / sigma_cells;
        wx[d + h] = exp(-0.5 * ex * ex);
        wy[d + h] = exp(-0.5 * ey * ey);
        sx += wx[d + h];
        sy += wy[d + h];
    }
    for (int d = 0; d < K; ++d) {
        wx[d] /= sx;
        wy[d] /= sy;
    }
    return EO_OK;
}

/* All elements of one station at one wavelength.  ix, iy: [n_elem];
 * wx, wy: [n_elem][K].  Returns the first error met. */
int eo_plan(int n_elem, const double *pos_m, double lambda_m, double grid_spacing_wl,
            int nx, int ny, int kernel_type, int K, double sigma_cells,
            int *ix, int *iy, double *wx, double *wy)
{
    if (n_elem < 1 || !(lambda_m > 0.0) || !(grid_spacing_wl > 0.0)) return EO_ERR_ARG;
    const double delta = grid_spacing_wl * lambda_m;
    for (int a = 0; a < n_elem; ++a) {
        int rc = eo_element_taps(pos_m[2 * a], pos_m[2 * a + 1], delta, nx, ny, kernel_type,
                                 K, sigma_cells, &ix[a], &iy[a], &wx[(size_t)a * K],
                                 &wy[(size_t)a * K]);
        if (rc != EO_OK) return rc;
    }
    return EO_OK;
}

/* Gridding of one time sample (inner bracket of Eq. 3), as a scatter over
 * elements and taps.  E: [n_elem][n_pol]; G: [n_pol][ny][nx], overwritten. */
void eo_grid_sample(int n_elem, int n_pol, int K, const int *ix, const int *iy,
                    const double *wx, const double *wy, const double complex *E,
                    int nx, int ny, double complex *G)
{
    const int h = (K - 1) / 2;
    memset(G, 0, sizeof(double complex) * (size_t)n_pol * nx * ny);
    for (int a = 0; a < n_elem; ++a) {
        for (int dy = -h; dy <= h; ++dy) {
            for (int dx = -h; dx <= h; ++dx) {
                const double w = wx[(size_t)a * K + dx + h] * wy[(size_t)a * K + dy + h];
                const size_t cell = (size_t)(iy[a] + dy) * nx + (ix[a] + dx);
                for (int p = 0; p < n_pol; ++p)
                    G[(size_t)p * nx * ny + cell] += w * E[(size_t)a * n_pol + p];
            }
        }
    }
}

/* exp(+2 pi i m / n) with the angle reduced to an integer fraction first. */
static double complex eo_root(long m, long n)
{
    long r = m % n;
    if (r < 0) r += n;
    const double ang = EO_TWO_PI * (double)r / (double)n;
    return cos(ang) + I * sin(ang);
}

/* In-place radix-2 decimation-in-time FFT of n points spaced by `stride`,
 * with the + sign of Eq. 3 and no normalisation.  n must be a power of two. */
void eo_fft1(double complex *a, int n, int stride)
{
    /* bit-reversal permutation */
    for (int i = 1, j = 0; i < n; ++i) {
        int bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double complex t = a[(size_t)i * stride];
            a[(size_t)i * stride] = a[(size_t)j * stride];
            a[(size_t)j * stride] = t;
        }
    }
    for (int len = 2; len <= n; len <<= 1) {
        const int half = len / 2;
        for (int i = 0; i < n; i += len) {
            for (int k = 0; k < half; ++k) {
                const double complex w = eo_root(k, len);
                const double complex u = a[(size_t)(i + k) * stride];
                const double complex v = a[(size_t)(i + k + half) * stride] * w;
                a[(size_t)(i + k) * stride] = u + v;
                a[(size_t)(i + k + half) * stride] = u - v;
            }
        }
    }
}

/* 2-D transform of Eq. 3 (outer sum): rows (x) then columns (y), in place. */
void eo_fft2(double complex *g, int nx, int ny)
{
    for (int y = 0; y < ny; ++y) eo_fft1(g + (size_t)y * nx, nx, 1);
    for (int x = 0; x < nx; ++x) eo_fft1(g + x, ny, nx);
}

/* The same transform as a direct O(N^4) sum, for small grids. */
void eo_dft2(const double complex *g, double complex *out, int nx, int ny)
{
    for (int ky = 0; ky < ny; ++ky)
        for (int kx = 0; kx < nx; ++kx) {
            double complex s = 0.0;
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    const double complex e = eo_root((long)kx * x, nx) * eo_root((long)ky * y, ny);
                    s += e * g[(size_t)y * nx + x];
                }
            out[(size_t)ky * nx + kx] = s;
        }
}

/* Batched 2-D transform of cf64 data [batch][ny][nx] (in place). */
void eo_fft2_batched(double *data, long batch, int nx, int ny)
{
    double complex *g = (double complex *)data;
    for (long b = 0; b < batch; ++b) eo_fft2(g + (size_t)b * nx * ny, nx, ny);
}

/* Exact conversion of one voltage sample to complex128. */
static double complex eo_volt(int volt_type, const void *volts, size_t idx)
{
    if (volt_type == EO_VOLT_CI8) {
        const int8_t *v = (const int8_t *)volts;
        return (double)v[2 * idx] + I * (double)v[2 * idx + 1];
    }
    if (volt_type == EO_VOLT_CF32) {
        const float *v = (const float *)volts;
        return (double)v[2 * idx] + I * (double)v[2 * idx + 1];
    }
    const double *v = (const double *)volts;
    return v[2 * idx] + I * v[2 * idx + 1];
}

/*
 * Time-averaged polarisation products (Eq. 2) of a per-sample field.
 * field: cf64 [nt][n_pol][ny][nx]; out: cf64 [n_pol*n_pol][ny][nx],
 * out[a*n_pol+b] = (1/n_div) sum_t F^a conj(F^b).  n_div = 0 means nt.
 */
void eo_power_mean(int n_pol, int nx, int ny, int nt, const double *field, int n_div,
                   double *out)
{
    const size_t npix = (size_t)nx * ny;
    const double complex *f = (const double complex *)field;
    double complex *o = (double complex *)out;
    memset(o, 0, sizeof(double complex) * npix * n_pol * n_pol);
    for (int t = 0; t < nt; ++t)
        for (int a = 0; a < n_pol; ++a)
            for (int b = 0; b < n_pol; ++b)
                for (size_t k = 0; k < npix; ++k) {
                    const double complex fa = f[((size_t)t * n_pol + a) * npix + k];
                    const double complex fb = f[((size_t)t * n_pol + b) * npix + k];
                    o[(size_t)(a * n_pol + b) * npix + k] += fa * conj(fb);
                }
    const double d = (double)(n_div > 0 ? n_div : nt);
    for (size_t k = 0; k < npix * n_pol * n_pol; ++k) o[k] /= d;
}

/*
 * Gridded field of a run of samples of one station and channel.
 * volts: [n_time_total][n_elem][n_pol] of volt_type for THIS channel;
 * out G: cf64 [nt][n_pol][ny][nx] for samples t0..t0+nt-1.
 */
int eo_grid(int n_elem, const double *pos_m, double lambda_m, double grid_spacing_wl,
            int nx, int ny, int kernel_type, int K, double sigma_cells, int n_pol,
            int volt_type, const void *volts, int t0, int nt, double *out)
{
    int *ix = malloc(sizeof(int) * n_elem), *iy = malloc(sizeof(int) * n_elem);
    double *wx = malloc(sizeof(double) * n_elem * K), *wy = malloc(sizeof(double) * n_elem * K);
    double complex *E = malloc(sizeof(double complex) * n_elem * n_pol);
    int rc = EO_ERR_NOMEM;
    if (!ix || !iy || !wx || !wy || !E) goto done;
    rc = eo_plan(n_elem, pos_m, lambda_m, grid_spacing_wl, nx, ny, kernel_type, K,
                 sigma_cells, ix, iy, wx, wy);
    if (rc != EO_OK) goto done;
    for (int t = 0; t < nt; ++t) {
        for (size_t e = 0; e < (size_t)n_elem * n_pol; ++e)
            E[e] = eo_volt(volt_type, volts, (size_t)(t0 + t) * n_elem * n_pol + e);
        eo_grid_sample(n_elem, n_pol, K, ix, iy, wx, wy, E, nx, ny,
                       (double complex *)out + (size_t)t * n_pol * nx * ny);
    }
done:
    free(ix); free(iy); free(wx); free(wy); free(E);
    return rc;
}

/*
 * The full EPIC image of one station (Eq. 3 then Eq. 2) for every channel.
 * volts: [n_chan][n_time][n_elem][n_pol] of volt_type.
 * image: cf64 [n_chan][n_pol*n_pol][ny][nx] = mean over n_time.
 * use_dft != 0 evaluates the transform as the direct sum (small grids).
 * n_threads > 0 bounds the OpenMP threads over channels.
 */
int eo_image(int n_elem, const double *pos_m, int n_chan, const double *lambda_m,
             double grid_spacing_wl, int n_time, int n_pol, int nx, int ny,
             int kernel_type, int K, double sigma_cells, int volt_type, const void *volts,
             int use_dft, int n_threads, double *image)
{
    if (n_chan < 1 || n_time < 1 || (n_pol != 1 && n_pol != 2) || nx < 1 || ny < 1)
        return EO_ERR_ARG;
    for (int n = nx; n > 1; n >>= 1) if (n & 1) return EO_ERR_ARG;
    for (int n = ny; n > 1; n >>= 1) if (n & 1) return EO_ERR_ARG;
    const size_t npix = (size_t)nx * ny;
    int status = EO_OK;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int c = 0; c < n_chan; ++c) {
        int *ix = malloc(sizeof(int) * n_elem), *iy = malloc(sizeof(int) * n_elem);
        double *wx = malloc(sizeof(double) * n_elem * K);
        double *wy = malloc(sizeof(double) * n_elem * K);
        double complex *E = malloc(sizeof(double complex) * n_elem * n_pol);
        double complex *G = malloc(sizeof(double complex) * n_pol * npix);
        double complex *F = malloc(sizeof(double complex) * n_pol * npix);
        double complex *S = calloc(npix * n_pol * n_pol, sizeof(double complex));
        int rc = EO_ERR_NOMEM;
        if (ix && iy && wx && wy && E && G && F && S) {
            rc = eo_plan(n_elem, pos_m, lambda_m[c], grid_spacing_wl, nx, ny, kernel_type,
                         K, sigma_cells, ix, iy, wx, wy);
        }
        if (rc == EO_OK) {
            const size_t chan_off = (size_t)c * n_time * n_elem * n_pol;
            for (int t = 0; t < n_time; ++t) {
                for (size_t e = 0; e < (size_t)n_elem * n_pol; ++e)
                    E[e] = eo_volt(volt_type, volts, chan_off + (size_t)t * n_elem * n_pol + e);
                eo_grid_sample(n_elem, n_pol, K, ix, iy, wx, wy, E, nx, ny, G);
                for (int p = 0; p < n_pol; ++p) {
                    if (use_dft) {
                        eo_dft2(G + p * npix, F + p * npix, nx, ny);
                    } else {
                        memcpy(F + p * npix, G + p * npix, sizeof(double complex) * npix);
                        eo_fft2(F + p * npix, nx, ny);
                    }
                }
                for (int a = 0; a < n_pol; ++a)
                    for (int b = 0; b < n_pol; ++b) {
                        double complex *s = S + (size_t)(a * n_pol + b) * npix;
                        const double complex *fa = F + (size_t)a * npix;
                        const double complex *fb = F + (size_t)b * npix;
                        for (size_t k = 0; k < npix; ++k) s[k] += fa[k] * conj(fb[k]);
                    }
            }
            double complex *out = (double complex *)image + (size_t)c * n_pol * n_pol * npix;
            for (size_t k = 0; k < npix * n_pol * n_pol; ++k) out[k] = S[k] / (double)n_time;
        }
        if (rc != EO_OK) {
#ifdef _OPENMP
#pragma omp critical
#endif
            status = rc;
        }
        free(ix); free(iy); free(wx); free(wy); free(E); free(G); free(F); free(S);
    }
    return status;
}

/* Number of OpenMP threads a parallel region would use (1 without OpenMP). */
int eo_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
