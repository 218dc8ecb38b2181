// host.cpp -- argument validation and the FP64 plan builder (plan_host.hpp):
// no device code and no HIP calls, so that the host side of the library can
// also be built and exercised with a plain host compiler and sanitizers.
//
// For every (station, channel) the plan holds the kernel taps of Eq. 3's
// gridding: each element a lands on the K x K cells around its nearest cell
// with separable weights evaluated at its true sub-cell position (Sec. 5.2:
// the kernel W~ is centred on r_a; the grid r_j is fixed in wavelengths so
// the geometry is recomputed per channel).  Everything is computed in double
// precision and rounded once to FP32 when stored.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "plan_host.hpp"

namespace epic {

// ----------------------------------------------------------------- errors --
static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

epic_status fail(epic_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

const char *last_error_cstr() { return g_last_error.c_str(); }

// ------------------------------------------------------------- arguments --
bool is_pow2_grid(int n) { return n >= 16 && n <= 256 && (n & (n - 1)) == 0; }

epic_status check_common(const epic_common *c)
{
    if (!c) return fail(EPIC_ERR_INVALID_ARG, "common is NULL");
    if (c->n_pol != 1 && c->n_pol != 2) return fail(EPIC_ERR_INVALID_ARG, "n_pol must be 1 or 2");
    if (c->n_chan < 1) return fail(EPIC_ERR_INVALID_ARG, "n_chan must be >= 1");
    if (!c->wavelength_m) return fail(EPIC_ERR_INVALID_ARG, "wavelength_m is NULL");
    for (int i = 0; i < c->n_chan; ++i)
        if (!std::isfinite(c->wavelength_m[i]) || !(c->wavelength_m[i] > 0.0))
            return fail(EPIC_ERR_INVALID_ARG, "wavelength_m[" + std::to_string(i) + "] must be finite and > 0");
    if (!std::isfinite(c->grid_spacing_wl) || !(c->grid_spacing_wl > 0.0))
        return fail(EPIC_ERR_INVALID_ARG, "grid_spacing_wl must be finite and > 0");
    if (c->n_time < 1) return fail(EPIC_ERR_INVALID_ARG, "n_time must be >= 1");
    if (c->volt_type != EPIC_CI8 && c->volt_type != EPIC_CF32)
        return fail(EPIC_ERR_INVALID_ARG, "unknown volt_type");
    if (c->precision != EPIC_FP32_FFT && c->precision != EPIC_FP16_SPLIT &&
        c->precision != EPIC_BF16_SPLIT)
        return fail(EPIC_ERR_INVALID_ARG, "unknown precision");
    return EPIC_OK;
}

epic_status check_station(const epic_station *s, int idx, bool need_volts)
{
    const std::string who = "station " + std::to_string(idx) + ": ";
    if (s->n_elem < 1) return fail(EPIC_ERR_INVALID_ARG, who + "n_elem must be >= 1");
    if (!s->pos_m) return fail(EPIC_ERR_INVALID_ARG, who + "pos_m is NULL");
    for (int64_t i = 0; i < 2LL * s->n_elem; ++i)
        if (!std::isfinite(s->pos_m[i])) return fail(EPIC_ERR_INVALID_ARG, who + "non-finite position");
    if (!is_pow2_grid(s->nx) || !is_pow2_grid(s->ny))
        return fail(EPIC_ERR_INVALID_ARG, who + "nx, ny must be powers of two in 16..256");
    const epic_kernel &k = s->kernel;
    if (k.type != EPIC_KERNEL_NEAREST && k.type != EPIC_KERNEL_GAUSSIAN)
        return fail(EPIC_ERR_INVALID_ARG, who + "unknown kernel type");
    if (k.support < 1 || k.support > 7 || (k.support % 2) == 0)
        return fail(EPIC_ERR_INVALID_ARG, who + "kernel support must be odd, 1..7");
    if (k.type == EPIC_KERNEL_NEAREST && k.support != 1)
        return fail(EPIC_ERR_INVALID_ARG, who + "NEAREST kernel needs support 1");
    if (k.type == EPIC_KERNEL_GAUSSIAN && (!std::isfinite(k.sigma_cells) || !(k.sigma_cells > 0.0)))
        return fail(EPIC_ERR_INVALID_ARG, who + "Gaussian sigma_cells must be finite and > 0");
    if (need_volts && !s->volts) return fail(EPIC_ERR_INVALID_ARG, who + "volts is NULL");
    return EPIC_OK;
}

// ----------------------------------------------------------------- plans --
// Geometry of one element at one channel: nearest cell and separable weights.
// Returns false if the footprint leaves the grid.
bool element_taps(double x, double y, double delta, int nx, int ny, const epic_kernel &kn,
                         int *ci, int *cj, double *wx, double *wy)
{
    const double u = x / delta + static_cast<double>(nx / 2);
    const double v = y / delta + static_cast<double>(ny / 2);
    const double fi = std::floor(u + 0.5);
    const double fj = std::floor(v + 0.5);
    const int K = kn.support;
    const int h = (K - 1) / 2;
    if (fi - h < 0 || fi + h > nx - 1 || fj - h < 0 || fj + h > ny - 1) return false;
    *ci = static_cast<int>(fi);
    *cj = static_cast<int>(fj);
    if (kn.type == EPIC_KERNEL_NEAREST) {
        wx[0] = wy[0] = 1.0;
        return true;
    }
    const double du = u - fi, dv = v - fj;
    double sx = 0.0, sy = 0.0;
    for (int d = -h; d <= h; ++d) {
        const double ex = (static_cast<double>(d) - du) / kn.sigma_cells;
        const double ey = (static_cast<double>(d) - dv) / kn.sigma_cells;
        wx[d + h] = std::exp(-0.5 * ex * ex);
        wy[d + h] = std::exp(-0.5 * ey * ey);
        sx += wx[d + h];
        sy += wy[d + h];
    }
    for (int d = 0; d < K; ++d) {
        wx[d] /= sx;
        wy[d] /= sy;
    }
    return true;
}

epic_status check_geometry(const epic_common *common, const epic_station *st)
{
    const int K = st->kernel.support;
    std::vector<double> wx(K), wy(K);
    for (int c = 0; c < common->n_chan; ++c) {
        const double delta = common->grid_spacing_wl * common->wavelength_m[c];
        for (int a = 0; a < st->n_elem; ++a) {
            int ci = 0, cj = 0;
            if (!element_taps(st->pos_m[2 * a], st->pos_m[2 * a + 1], delta, st->nx, st->ny,
                              st->kernel, &ci, &cj, wx.data(), wy.data()))
                return fail(EPIC_ERR_INVALID_ARG,
                            "element " + std::to_string(a) + " kernel footprint leaves the " +
                                std::to_string(st->nx) + "x" + std::to_string(st->ny) +
                                " grid at channel " + std::to_string(c));
        }
    }
    return EPIC_OK;
}

epic_status build_host_plan(const epic_common *common, const epic_station *st, HostPlan *out)
{
    const int n_chan = common->n_chan;
    const int n_elem = st->n_elem;
    const int K = st->kernel.support;
    const int nx = st->nx, ny = st->ny, h = (K - 1) / 2;
    HostPlan &hd = *out;
    hd = HostPlan();
    std::vector<ChanPlan> &chans = hd.chans;
    chans.resize(n_chan);
    std::vector<int32_t> &cell_start = hd.cell_start;
    std::vector<int32_t> &cell_order = hd.cell_order;   // per channel: box cells by descending tap count
    std::vector<int32_t> &elem_cell = hd.elem_cell;     // ci | cj << 16
    elem_cell.assign(static_cast<size_t>(n_chan) * n_elem, 0);
    std::vector<Tap> &taps = hd.taps;
    std::vector<int> ci(n_elem), cj(n_elem);
    std::vector<double> wx(static_cast<size_t>(n_elem) * K), wy(static_cast<size_t>(n_elem) * K);
    for (int c = 0; c < n_chan; ++c) {
        const double delta = common->grid_spacing_wl * common->wavelength_m[c];
        int x_lo = nx, x_hi = -1, y_lo = ny, y_hi = -1;
        for (int a = 0; a < n_elem; ++a) {
            if (!element_taps(st->pos_m[2 * a], st->pos_m[2 * a + 1], delta, nx, ny, st->kernel,
                              &ci[a], &cj[a], &wx[static_cast<size_t>(a) * K],
                              &wy[static_cast<size_t>(a) * K])) {
                return fail(EPIC_ERR_INVALID_ARG,
                            "element " + std::to_string(a) + " kernel footprint leaves the " +
                                std::to_string(nx) + "x" + std::to_string(ny) +
                                " grid at channel " + std::to_string(c));
            }
            x_lo = std::min(x_lo, ci[a] - h);
            x_hi = std::max(x_hi, ci[a] + h);
            y_lo = std::min(y_lo, cj[a] - h);
            y_hi = std::max(y_hi, cj[a] + h);
        }
        for (int a = 0; a < n_elem; ++a)
            elem_cell[static_cast<size_t>(c) * n_elem + a] = ci[a] | (cj[a] << 16);
        ChanPlan &cp = chans[c];
        cp.x0 = x_lo;
        cp.y0 = y_lo;
        cp.bw = x_hi - x_lo + 1;
        cp.bh = y_hi - y_lo + 1;
        cp.cell_off = static_cast<int64_t>(cell_start.size());
        cp.tap_off = static_cast<int64_t>(taps.size());
        const int ncell = cp.bw * cp.bh;
        hd.max_box = std::max(hd.max_box, ncell);
        hd.max_bw = std::max(hd.max_bw, cp.bw);
        hd.max_bh = std::max(hd.max_bh, cp.bh);
        // counting sort of taps by cell; elements visited in ascending order
        std::vector<int32_t> count(static_cast<size_t>(ncell) + 1, 0);
        for (int a = 0; a < n_elem; ++a)
            for (int dy = -h; dy <= h; ++dy)
                for (int dx = -h; dx <= h; ++dx)
                    ++count[static_cast<size_t>(cj[a] + dy - y_lo) * cp.bw + (ci[a] + dx - x_lo) + 1];
        for (int i = 0; i < ncell; ++i) count[i + 1] += count[i];
        const size_t base = taps.size();
        taps.resize(base + static_cast<size_t>(count[ncell]));
        std::vector<int32_t> fillp(count.begin(), count.end() - 1);
        for (int a = 0; a < n_elem; ++a)
            for (int dy = -h; dy <= h; ++dy)
                for (int dx = -h; dx <= h; ++dx) {
                    const size_t cell = static_cast<size_t>(cj[a] + dy - y_lo) * cp.bw + (ci[a] + dx - x_lo);
                    const double w = wx[static_cast<size_t>(a) * K + dx + h] * wy[static_cast<size_t>(a) * K + dy + h];
                    taps[base + fillp[cell]++] = Tap{a, static_cast<float>(w)};
                }
        for (int i = 0; i < ncell; ++i) hd.max_cell_taps = std::max(hd.max_cell_taps, count[i + 1] - count[i]);
        {
            std::vector<double> wsum(ncell, 0.0);
            for (int a = 0; a < n_elem; ++a)
                for (int dy = -h; dy <= h; ++dy)
                    for (int dx = -h; dx <= h; ++dx)
                        wsum[static_cast<size_t>(cj[a] + dy - y_lo) * cp.bw + (ci[a] + dx - x_lo)] +=
                            std::fabs(wx[static_cast<size_t>(a) * K + dx + h] * wy[static_cast<size_t>(a) * K + dy + h]);
            double m = 0.0;
            for (double v : wsum) m = std::max(m, v);
            cp.wsum_max = static_cast<float>(m * (1.0 + 1e-6));   // rounded up
            cp.pad_ = 0;
        }
        cell_start.insert(cell_start.end(), count.begin(), count.end());
        // cells sorted by tap count (ties by index) so that neighbouring lanes of a
        // gathering wave walk lists of about the same length
        std::vector<int32_t> order(ncell);
        for (int i = 0; i < ncell; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            return count[a + 1] - count[a] > count[b + 1] - count[b];
        });
        cell_order.insert(cell_order.end(), order.begin(), order.end());
        cell_order.push_back(-1);
        if (n_elem >= kBandMinElem) {
            // row-band tables: counting sort of the elements by nearest row
            std::vector<int32_t> row(static_cast<size_t>(ny) + 1, 0);
            for (int a = 0; a < n_elem; ++a) ++row[static_cast<size_t>(cj[a]) + 1];
            for (int y = 0; y < ny; ++y) row[y + 1] += row[y];
            std::vector<int32_t> slot(n_elem), next(row.begin(), row.end() - 1);
            for (int a = 0; a < n_elem; ++a) slot[a] = next[cj[a]]++;
            hd.band_slot.insert(hd.band_slot.end(), slot.begin(), slot.end());
            for (int y = 0; y < ny; ++y)
                hd.max_band = std::max(hd.max_band, row[std::min(ny, y + h + 1)] - row[std::max(0, y - h)]);
            hd.band_row.insert(hd.band_row.end(), row.begin(), row.end());
            hd.band_taps.resize(taps.size());
            for (size_t k = base; k < taps.size(); ++k) hd.band_taps[k] = Tap{slot[taps[k].elem], taps[k].w};
        }
    }
    return EPIC_OK;
}

}  // namespace epic
