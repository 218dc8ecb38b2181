// host_sanitize_driver.cpp -- exercises the library's host side (argument
// validation and the FP64 plan builder of host.cpp) in a build with
// AddressSanitizer and UndefinedBehaviorSanitizer, no GPU involved.  Test
// infrastructure: built and run by tests/test_host_sanitize.py.
//
// Layouts are drawn with a small fixed-seed generator here; the checks are
// structural (statuses of valid and invalid calls, and per channel: the
// gather lists cover every element's K x K taps exactly once, the weights of
// an element sum to 1, offsets are monotone and in range, the cell order is
// a permutation of the box cells).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "plan_host.hpp"

using namespace epic;

namespace {

int g_fail = 0;

void expect(bool ok, const char *what)
{
    if (!ok) {
        std::printf("FAIL: %s (%s)\n", what, last_error_cstr());
        ++g_fail;
    }
}

struct Lcg {
    uint64_t s;
    double next() { s = s * 6364136223846793005ULL + 1442695040888963407ULL; return ((s >> 11) & ((1ULL << 53) - 1)) / 9007199254740992.0; }
};

std::vector<double> circle(int n, double diameter, uint64_t seed)
{
    Lcg g{seed};
    std::vector<double> p(2 * n);
    for (int a = 0; a < n; ++a) {
        const double r = 0.5 * diameter * std::sqrt(g.next()), t = 6.283185307179586 * g.next();
        p[2 * a] = r * std::cos(t);
        p[2 * a + 1] = r * std::sin(t);
    }
    return p;
}

std::vector<double> lattice(int side, double step, int drop_every)
{
    std::vector<double> p;
    for (int i = 0; i < side; ++i)
        for (int j = 0; j < side; ++j) {
            if (drop_every && (i * side + j) % drop_every == 0) continue;
            p.push_back((i - side / 2) * step);
            p.push_back((j - side / 2) * step);
        }
    return p;
}

std::vector<double> wavelengths(int n, double lam0)
{
    std::vector<double> l(n);
    for (int c = 0; c < n; ++c) l[c] = lam0 * (1.0 + 2e-4 * (c - n / 2));
    return l;
}

void check_plan(const epic_common &c, const epic_station &s, const char *name)
{
    HostPlan hp;
    const epic_status st = build_host_plan(&c, &s, &hp);
    expect(st == EPIC_OK, name);
    if (st != EPIC_OK) return;
    const int K = s.kernel.support, ne = s.n_elem;
    expect(static_cast<int>(hp.chans.size()) == c.n_chan, "one ChanPlan per channel");
    expect(hp.taps.size() == static_cast<size_t>(c.n_chan) * ne * K * K, "K^2 taps per element and channel");
    expect(hp.elem_cell.size() == static_cast<size_t>(c.n_chan) * ne, "one nearest cell per element and channel");
    for (int ch = 0; ch < c.n_chan; ++ch) {
        const ChanPlan &cp = hp.chans[ch];
        const int ncell = cp.bw * cp.bh;
        expect(cp.x0 >= 0 && cp.y0 >= 0 && cp.x0 + cp.bw <= s.nx && cp.y0 + cp.bh <= s.ny, "box on the grid");
        expect(cp.cell_off >= 0 && cp.cell_off + ncell + 1 <= static_cast<int64_t>(hp.cell_start.size()), "cell range");
        const int32_t *cs = hp.cell_start.data() + cp.cell_off;
        expect(cs[0] == 0 && cs[ncell] == ne * K * K, "cell offsets span the channel's taps");
        std::vector<int> seen(ne, 0);
        std::vector<double> wsum(ne, 0.0);
        bool mono = true, in_range = true;
        for (int cell = 0; cell < ncell; ++cell) {
            mono = mono && cs[cell] <= cs[cell + 1];
            for (int k = cs[cell]; k < cs[cell + 1]; ++k) {
                const Tap t = hp.taps[cp.tap_off + k];
                if (t.elem < 0 || t.elem >= ne || !(t.w >= 0.f)) { in_range = false; continue; }
                ++seen[t.elem];
                wsum[t.elem] += t.w;
            }
        }
        expect(mono, "cell offsets monotone");
        expect(in_range, "tap elements in range, weights non-negative");
        bool once = true, unit = true;
        for (int a = 0; a < ne; ++a) {
            once = once && seen[a] == K * K;
            unit = unit && std::fabs(wsum[a] - 1.0) < 1e-5;
        }
        expect(once, "every element's K^2 taps once");
        expect(unit, "an element's weights sum to 1");
        const int32_t *ord = hp.cell_order.data() + cp.cell_off;
        std::vector<int> hit(ncell, 0);
        bool perm = true;
        for (int i = 0; i < ncell; ++i) {
            if (ord[i] < 0 || ord[i] >= ncell) { perm = false; break; }
            ++hit[ord[i]];
        }
        for (int i = 0; perm && i < ncell; ++i) perm = hit[i] == 1;
        expect(perm && ord[ncell] == -1, "cell order is a permutation of the box cells");
        if (ne < kBandMinElem) continue;
        // row-band tables: slot order by nearest row, rows' first slots, and
        // every tap of a row-y cell inside the slots of rows y - h .. y + h
        const int h = (K - 1) / 2;
        const int32_t *bs = hp.band_slot.data() + static_cast<size_t>(ch) * ne;
        const int32_t *br = hp.band_row.data() + static_cast<size_t>(ch) * (s.ny + 1);
        std::vector<int> slot_of(bs, bs + ne), owner(ne, -1);
        bool bperm = true;
        for (int a = 0; a < ne; ++a) {
            if (bs[a] < 0 || bs[a] >= ne || owner[bs[a]] >= 0) { bperm = false; break; }
            owner[bs[a]] = a;
        }
        expect(bperm, "band slots are a permutation of the elements");
        for (int a = 0; bperm && a < ne; ++a) {
            const int row_a = hp.elem_cell[static_cast<size_t>(ch) * ne + a] >> 16;
            expect(bs[a] >= br[row_a] && bs[a] < br[row_a + 1], "an element's slot lies in its row's range");
            if (bs[a] < br[row_a] || bs[a] >= br[row_a + 1]) break;
        }
        bool rows_ok = br[0] == 0 && br[s.ny] == ne;
        for (int y = 0; y < s.ny; ++y) rows_ok = rows_ok && br[y] <= br[y + 1];
        expect(rows_ok, "band rows monotone, spanning the elements");
        bool bt_ok = bperm, within = true;
        for (int cell = 0; bperm && cell < ncell; ++cell) {
            const int y = cp.y0 + cell / cp.bw;
            const int lo = br[std::max(0, y - h)], hi = br[std::min(s.ny, y + h + 1)];
            expect(hi - lo <= hp.max_band, "band within max_band");
            for (int k = cs[cell]; k < cs[cell + 1]; ++k) {
                const Tap t = hp.taps[cp.tap_off + k], b = hp.band_taps[cp.tap_off + k];
                bt_ok = bt_ok && t.elem >= 0 && t.elem < ne && b.elem == slot_of[t.elem] && b.w == t.w;
                within = within && b.elem >= lo && b.elem < hi;
            }
        }
        expect(bt_ok, "band taps are the taps with elements replaced by their slots");
        expect(within, "every tap of a row's cells lies in the row's band");
    }
    expect((ne >= kBandMinElem) == (hp.max_band > 0), "band tables exactly for large stations");
}

}  // namespace

int main()
{
    // a station-scale layout: 256 elements in a 38 m circle, 64 x 64, K = 3
    std::vector<double> pos = circle(256, 38.0, 17804), lam = wavelengths(64, 2.0);
    epic_common c{2, 64, lam.data(), 0.5, 32, EPIC_CI8, EPIC_FP32_FFT};
    epic_station s{256, pos.data(), 64, 64, {EPIC_KERNEL_GAUSSIAN, 3, 0.5}, reinterpret_cast<void *>(0x1000), nullptr};
    expect(check_common(&c) == EPIC_OK, "valid common");
    expect(check_station(&s, 0) == EPIC_OK, "valid station");
    expect(check_geometry(&c, &s) == EPIC_OK, "station fits its grid");
    check_plan(c, s, "station-scale plan");

    // a large lattice on 256 x 256 with a 5 x 5 kernel (every 20th site dropped)
    std::vector<double> lat = lattice(128, 0.75, 20), lam5 = wavelengths(4, 1.5);
    epic_common c5{2, 4, lam5.data(), 0.5, 8, EPIC_CF32, EPIC_FP16_SPLIT};
    epic_station s5{static_cast<int32_t>(lat.size() / 2), lat.data(), 256, 256, {EPIC_KERNEL_GAUSSIAN, 5, 5.0 / 6.0},
                    reinterpret_cast<void *>(0x1000), nullptr};
    check_plan(c5, s5, "large lattice plan");

    // nearest-cell kernel on a small grid, one pol
    std::vector<double> sq = circle(64, 14.0, 3), lam1 = wavelengths(4, 2.0);
    epic_common c1{1, 4, lam1.data(), 0.5, 16, EPIC_CF32, EPIC_FP32_FFT};
    epic_station s1{64, sq.data(), 32, 32, {EPIC_KERNEL_NEAREST, 1, 0.0}, reinterpret_cast<void *>(0x1000), nullptr};
    check_plan(c1, s1, "nearest-cell plan");

    // invalid arguments: every one is refused with EPIC_ERR_INVALID_ARG
    auto bad_common = [&](epic_common b, const char *what) { expect(check_common(&b) == EPIC_ERR_INVALID_ARG, what); };
    epic_common b = c;
    b.n_pol = 3; bad_common(b, "n_pol 3");
    b = c; b.n_time = 0; bad_common(b, "n_time 0");
    b = c; b.grid_spacing_wl = std::nan(""); bad_common(b, "NaN grid spacing");
    b = c; b.wavelength_m = nullptr; bad_common(b, "NULL wavelengths");
    std::vector<double> lam_bad = lam;
    lam_bad[7] = -1.0;
    b = c; b.wavelength_m = lam_bad.data(); bad_common(b, "negative wavelength");
    b = c; b.volt_type = 9; bad_common(b, "volt type");
    b = c; b.precision = -1; bad_common(b, "precision");
    expect(check_common(nullptr) == EPIC_ERR_INVALID_ARG, "NULL common");
    auto bad_station = [&](epic_station t, const char *what) { expect(check_station(&t, 0) == EPIC_ERR_INVALID_ARG, what); };
    epic_station t = s;
    t.nx = 48; bad_station(t, "grid 48");
    t = s; t.ny = 512; bad_station(t, "grid 512");
    t = s; t.kernel.support = 4; bad_station(t, "even support");
    t = s; t.kernel.sigma_cells = 0.0; bad_station(t, "sigma 0");
    t = s; t.kernel.type = EPIC_KERNEL_NEAREST; bad_station(t, "nearest with support 3");
    t = s; t.volts = nullptr; bad_station(t, "NULL volts");
    t = s; t.n_elem = 0; bad_station(t, "no elements");
    std::vector<double> pos_nan = pos;
    pos_nan[11] = std::nan("");
    t = s; t.pos_m = pos_nan.data(); bad_station(t, "NaN position");
    // a footprint off the grid at the highest channel only
    std::vector<double> edge = {14.0, 0.0};
    std::vector<double> lam_e = {2.2, 2.0, 1.8};
    epic_common ce{1, 3, lam_e.data(), 0.5, 4, EPIC_CF32, EPIC_FP32_FFT};
    epic_station se{1, edge.data(), 32, 32, {EPIC_KERNEL_GAUSSIAN, 3, 0.5}, reinterpret_cast<void *>(0x1000), nullptr};
    expect(check_geometry(&ce, &se) == EPIC_ERR_INVALID_ARG, "footprint off the grid at one channel");
    HostPlan hp;
    expect(build_host_plan(&ce, &se, &hp) == EPIC_ERR_INVALID_ARG, "plan of an off-grid footprint");

    if (g_fail == 0) std::printf("host checks OK\n");
    return g_fail == 0 ? 0 : 1;
}
