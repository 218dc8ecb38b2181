// plan.cpp -- the library's device caches: station plans (built on the host
// by host.cpp, uploaded once per geometry), transform tables, workspaces and
// the XFFT route's plans, and the one device allocator they all use.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <unordered_map>

#include "internal.hpp"

namespace epic {

// ----------------------------------------------------------------- errors --
epic_status hip_fail(hipError_t e, const char *what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? EPIC_ERR_OUT_OF_MEMORY : EPIC_ERR_DEVICE;
}

// Test hook: EPIC_TEST_FAIL_ALLOC=1 makes every library-owned allocation fail.
static bool alloc_fail_forced()
{
    const char *e = std::getenv("EPIC_TEST_FAIL_ALLOC");
    return e && e[0] == '1';
}

epic_status dev_alloc(void **p, size_t bytes)
{
    if (alloc_fail_forced()) return fail(EPIC_ERR_OUT_OF_MEMORY, "allocation refused (EPIC_TEST_FAIL_ALLOC)");
    hipError_t e = hipMalloc(p, bytes == 0 ? 16 : bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_fail(e, "hipMalloc");
    }
    return EPIC_OK;
}

// ------------------------------------------------------------------ plans --
struct PlanEntry {
    void *dev = nullptr;
    PlanHandle h;
};

static std::mutex g_mu;
static std::unordered_map<std::string, PlanEntry> g_plans;
static std::map<std::pair<int, int>, void *> g_twiddles;
static std::map<std::tuple<int, int, int>, void *> g_dft_tables;
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
};
static std::map<std::tuple<int, uintptr_t, int>, Workspace> g_ws;
struct XfftEntry {
    void *dev = nullptr;
    XfftPlanHandle h;
};
static std::unordered_map<std::string, XfftEntry> g_xplans;

static void append(std::string &k, const void *p, size_t n)
{
    k.append(static_cast<const char *>(p), n);
}

// Cache key of a station's geometry on one device (everything a plan depends on).
static std::string geometry_key(const epic_common *common, const epic_station *st, int device)
{
    const int n_chan = common->n_chan;
    const int n_elem = st->n_elem;
    const int K = st->kernel.support;
    std::string key;
    key.reserve(64 + sizeof(double) * (2 * n_elem + n_chan));
    append(key, &device, sizeof device);
    append(key, &n_elem, sizeof n_elem);
    append(key, &st->nx, sizeof st->nx);
    append(key, &st->ny, sizeof st->ny);
    append(key, &st->kernel.type, sizeof st->kernel.type);
    append(key, &K, sizeof K);
    append(key, &st->kernel.sigma_cells, sizeof st->kernel.sigma_cells);
    append(key, &common->grid_spacing_wl, sizeof common->grid_spacing_wl);
    append(key, &n_chan, sizeof n_chan);
    append(key, common->wavelength_m, sizeof(double) * n_chan);
    append(key, st->pos_m, sizeof(double) * 2 * n_elem);
    return key;
}

epic_status get_plan(const epic_common *common, const epic_station *st, int device,
                     PlanHandle *out)
{
    std::string key = geometry_key(common, st, device);

    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
        *out = it->second.h;
        return EPIC_OK;
    }

    HostPlan hp;
    epic_status bs = build_host_plan(common, st, &hp);
    if (bs != EPIC_OK) return bs;
    const std::vector<ChanPlan> &chans = hp.chans;
    const std::vector<int32_t> &cell_start = hp.cell_start, &cell_order = hp.cell_order,
                               &elem_cell = hp.elem_cell;
    const std::vector<Tap> &taps = hp.taps;
    PlanHandle hd;
    hd.max_box = hp.max_box;
    hd.max_bw = hp.max_bw;
    hd.max_bh = hp.max_bh;
    hd.max_cell_taps = hp.max_cell_taps;
    hd.n_taps_total = static_cast<int64_t>(taps.size());

    // Upload: one allocation, three 256-byte aligned sections.
    auto up = [](size_t b) { return (b + 255) & ~static_cast<size_t>(255); };
    const size_t b_chan = up(sizeof(ChanPlan) * chans.size());
    const size_t b_cell = up(sizeof(int32_t) * cell_start.size());
    const size_t b_taps = up(sizeof(Tap) * taps.size());
    const size_t b_order = up(sizeof(int32_t) * cell_order.size());
    const size_t b_ec = up(sizeof(int32_t) * elem_cell.size());
    const size_t b_bt = up(sizeof(Tap) * hp.band_taps.size());
    const size_t b_br = up(sizeof(int32_t) * hp.band_row.size());
    const size_t b_bp = up(sizeof(int32_t) * hp.band_slot.size());
    void *dev = nullptr;
    epic_status s = dev_alloc(&dev, b_chan + b_cell + b_taps + b_order + b_ec + b_bt + b_br + b_bp);
    if (s != EPIC_OK) return s;
    char *p = static_cast<char *>(dev);
    hipError_t e = hipMemcpy(p, chans.data(), sizeof(ChanPlan) * chans.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p + b_chan, cell_start.data(), sizeof(int32_t) * cell_start.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !taps.empty())
        e = hipMemcpy(p + b_chan + b_cell, taps.data(), sizeof(Tap) * taps.size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p + b_chan + b_cell + b_taps, cell_order.data(),
                      sizeof(int32_t) * cell_order.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p + b_chan + b_cell + b_taps + b_order, elem_cell.data(),
                      sizeof(int32_t) * elem_cell.size(), hipMemcpyHostToDevice);
    char *pb = p + b_chan + b_cell + b_taps + b_order + b_ec;
    if (e == hipSuccess && hp.max_band > 0) {
        e = hipMemcpy(pb, hp.band_taps.data(), sizeof(Tap) * hp.band_taps.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(pb + b_bt, hp.band_row.data(), sizeof(int32_t) * hp.band_row.size(),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(pb + b_bt + b_br, hp.band_slot.data(), sizeof(int32_t) * hp.band_slot.size(),
                          hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return hip_fail(e, "plan upload");
    }
    hd.chan = reinterpret_cast<const ChanPlan *>(p);
    hd.cell_start = reinterpret_cast<const int32_t *>(p + b_chan);
    hd.taps = reinterpret_cast<const Tap *>(p + b_chan + b_cell);
    hd.cell_order = reinterpret_cast<const int32_t *>(p + b_chan + b_cell + b_taps);
    hd.elem_cell = reinterpret_cast<const int32_t *>(p + b_chan + b_cell + b_taps + b_order);
    if (hp.max_band > 0) {
        hd.band_taps = reinterpret_cast<const Tap *>(pb);
        hd.band_row = reinterpret_cast<const int32_t *>(pb + b_bt);
        hd.band_slot = reinterpret_cast<const int32_t *>(pb + b_bt + b_br);
        hd.max_band = hp.max_band;
    }
    g_plans.emplace(std::move(key), PlanEntry{dev, hd});
    *out = hd;
    return EPIC_OK;
}

void fill_twiddles(int n, float2 *dst)
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int k = 0; k < n; ++k) {
        const double a = two_pi * static_cast<double>(k) / static_cast<double>(n);
        dst[k] = make_float2(static_cast<float>(std::cos(a)), static_cast<float>(std::sin(a)));
    }
}

epic_status get_twiddles(int n, int device, const float2 **out)
{
    std::lock_guard<std::mutex> lock(g_mu);
    auto key = std::make_pair(device, n);
    auto it = g_twiddles.find(key);
    if (it != g_twiddles.end()) {
        *out = static_cast<const float2 *>(it->second);
        return EPIC_OK;
    }
    std::vector<float2> tw(n);
    fill_twiddles(n, tw.data());
    void *dev = nullptr;
    epic_status s = dev_alloc(&dev, sizeof(float2) * n);
    if (s != EPIC_OK) return s;
    hipError_t e = hipMemcpy(dev, tw.data(), sizeof(float2) * n, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return hip_fail(e, "twiddle upload");
    }
    g_twiddles[key] = dev;
    *out = static_cast<const float2 *>(dev);
    return EPIC_OK;
}

// Registry used by k_dft.hip: the table is built by the caller-supplied
// function the first time (under the cache lock).
epic_status cache_dft_table(int n, int precision, int device, size_t bytes,
                            void (*fill)(int, int, void *), const void **out)
{
    std::lock_guard<std::mutex> lock(g_mu);
    auto key = std::make_tuple(device, n, precision);
    auto it = g_dft_tables.find(key);
    if (it != g_dft_tables.end()) {
        *out = it->second;
        return EPIC_OK;
    }
    std::vector<char> host(bytes);
    fill(n, precision, host.data());
    void *dev = nullptr;
    epic_status s = dev_alloc(&dev, bytes);
    if (s != EPIC_OK) return s;
    hipError_t e = hipMemcpy(dev, host.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return hip_fail(e, "DFT table upload");
    }
    g_dft_tables[key] = dev;
    *out = dev;
    return EPIC_OK;
}

epic_status get_workspace(int device, hipStream_t stream, int slot, size_t bytes, void **out)
{
    std::lock_guard<std::mutex> lock(g_mu);
    Workspace &w = g_ws[std::make_tuple(device, reinterpret_cast<uintptr_t>(stream), slot)];
    if (w.bytes >= bytes && w.ptr) {
        *out = w.ptr;
        return EPIC_OK;
    }
    if (w.ptr) {
        // the old buffer may still be read by work queued on this stream
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
        (void)hipFree(w.ptr);
        w.ptr = nullptr;
        w.bytes = 0;
    }
    const size_t want = bytes + bytes / 8;   // some headroom for growing workloads
    epic_status s = dev_alloc(&w.ptr, want);
    if (s != EPIC_OK) return s;
    w.bytes = want;
    *out = w.ptr;
    return EPIC_OK;
}

// ------------------------------------------------------------- XFFT plans --
// Eq. 6 gridding of visibilities.  Per channel: every element's nearest cell
// and separable weights (as for Eq. 3), and every ordered element pair (a, b)
// sorted by its baseline cell c_a - c_b (mod the grid), the "centre" of the
// pair's (2K-1)^2 footprint.  Centres (cells that hold at least one pair)
// are kept in raster order: neighbouring cells have similar pair counts, and
// the per-centre partial sums of a channel then lie in cell order.
epic_status get_xfft_plan(const epic_common *common, const epic_station *st, int device,
                          XfftPlanHandle *out)
{
    const int n_chan = common->n_chan;
    const int n_elem = st->n_elem;
    const int K = st->kernel.support;
    const int nx = st->nx, ny = st->ny, npix = nx * ny;
    const int64_t n_pairs = static_cast<int64_t>(n_elem) * n_elem;
    if (n_elem > 65535)
        return fail(EPIC_ERR_UNSUPPORTED, "XFFT plan: more than 65535 elements");
    if (n_pairs * n_chan > (int64_t{1} << 31))
        return fail(EPIC_ERR_UNSUPPORTED,
                    "XFFT plan: n_elem^2 * n_chan exceeds 2^31 element pairs; call with fewer "
                    "channels at a time");
    std::string key = geometry_key(common, st, device);
    key.push_back('X');

    std::lock_guard<std::mutex> lock(g_mu);
    auto it = g_xplans.find(key);
    if (it != g_xplans.end()) {
        *out = it->second.h;
        return EPIC_OK;
    }
    std::vector<float> elem_w(static_cast<size_t>(n_chan) * n_elem * 2 * K);
    std::vector<int32_t> cent_cell(static_cast<size_t>(n_chan) * npix, 0);
    std::vector<int32_t> cent_start(static_cast<size_t>(n_chan) * (npix + 1), 0);
    std::vector<int32_t> cell_cent(static_cast<size_t>(n_chan) * npix, -1);
    std::vector<int64_t> cent_base(static_cast<size_t>(n_chan) + 1, 0);
    std::vector<uint32_t> pairs(static_cast<size_t>(n_pairs) * n_chan);
    std::vector<int> ci(n_elem), cj(n_elem);
    std::vector<double> wx(K), wy(K);
    std::vector<int32_t> count(npix), slot(npix), order;
    order.reserve(npix);
    for (int c = 0; c < n_chan; ++c) {
        const double delta = common->grid_spacing_wl * common->wavelength_m[c];
        float *ew = elem_w.data() + static_cast<size_t>(c) * n_elem * 2 * K;
        for (int a = 0; a < n_elem; ++a) {
            if (!element_taps(st->pos_m[2 * a], st->pos_m[2 * a + 1], delta, nx, ny, st->kernel,
                              &ci[a], &cj[a], wx.data(), wy.data()))
                return fail(EPIC_ERR_INVALID_ARG,
                            "element " + std::to_string(a) + " kernel footprint leaves the grid at channel " +
                                std::to_string(c));
            for (int d = 0; d < K; ++d) {
                ew[static_cast<size_t>(a) * 2 * K + d] = static_cast<float>(wx[d]);
                ew[static_cast<size_t>(a) * 2 * K + K + d] = static_cast<float>(wy[d]);
            }
        }
        auto centre = [&](int a, int b) {
            const int dx = ((ci[a] - ci[b]) % nx + nx) % nx;
            const int dy = ((cj[a] - cj[b]) % ny + ny) % ny;
            return dy * nx + dx;
        };
        std::fill(count.begin(), count.end(), 0);
        for (int a = 0; a < n_elem; ++a)
            for (int b = 0; b < n_elem; ++b) ++count[centre(a, b)];
        order.clear();
        for (int i = 0; i < npix; ++i)
            if (count[i] > 0) order.push_back(i);
        int32_t *cc = cent_cell.data() + static_cast<size_t>(c) * npix;
        int32_t *cs = cent_start.data() + static_cast<size_t>(c) * (npix + 1);
        int32_t run = 0;
        for (size_t k = 0; k < order.size(); ++k) {
            const int cell = order[k];
            cc[k] = (cell % nx) | ((cell / nx) << 16);
            cs[k] = run;
            slot[cell] = run;
            run += count[cell];
        }
        cs[order.size()] = run;
        int32_t *cm = cell_cent.data() + static_cast<size_t>(c) * npix;
        for (size_t k = 0; k < order.size(); ++k) cm[order[k]] = static_cast<int32_t>(k);
        cent_base[c + 1] = cent_base[c] + static_cast<int64_t>(order.size());
        uint32_t *pr = pairs.data() + static_cast<size_t>(c) * n_pairs;
        for (int a = 0; a < n_elem; ++a)
            for (int b = 0; b < n_elem; ++b)
                pr[slot[centre(a, b)]++] = static_cast<uint32_t>(a) | (static_cast<uint32_t>(b) << 16);
    }

    auto up = [](size_t b) { return (b + 255) & ~static_cast<size_t>(255); };
    const size_t b_w = up(sizeof(float) * elem_w.size());
    const size_t b_cc = up(sizeof(int32_t) * cent_cell.size());
    const size_t b_cs = up(sizeof(int32_t) * cent_start.size());
    const size_t b_pr = up(sizeof(uint32_t) * pairs.size());
    const size_t b_cm = up(sizeof(int32_t) * cell_cent.size());
    const size_t b_cb = up(sizeof(int64_t) * cent_base.size());
    void *dev = nullptr;
    epic_status s = dev_alloc(&dev, b_w + b_cc + b_cs + b_pr + b_cm + b_cb);
    if (s != EPIC_OK) return s;
    char *p = static_cast<char *>(dev);
    size_t off = 0;
    hipError_t e = hipSuccess;
    auto put = [&](const void *src, size_t bytes, size_t span) {
        if (e == hipSuccess && bytes) e = hipMemcpy(p + off, src, bytes, hipMemcpyHostToDevice);
        const char *where = p + off;
        off += span;
        return where;
    };
    XfftPlanHandle hd;
    hd.elem_w = reinterpret_cast<const float *>(put(elem_w.data(), sizeof(float) * elem_w.size(), b_w));
    hd.cent_cell = reinterpret_cast<const int32_t *>(put(cent_cell.data(), sizeof(int32_t) * cent_cell.size(), b_cc));
    hd.cent_start = reinterpret_cast<const int32_t *>(put(cent_start.data(), sizeof(int32_t) * cent_start.size(), b_cs));
    hd.pairs = reinterpret_cast<const uint32_t *>(put(pairs.data(), sizeof(uint32_t) * pairs.size(), b_pr));
    hd.cell_cent = reinterpret_cast<const int32_t *>(put(cell_cent.data(), sizeof(int32_t) * cell_cent.size(), b_cm));
    hd.cent_base = reinterpret_cast<const int64_t *>(put(cent_base.data(), sizeof(int64_t) * cent_base.size(), b_cb));
    hd.n_cent_total = cent_base[n_chan];
    if (e != hipSuccess) {
        (void)hipFree(dev);
        return hip_fail(e, "XFFT plan upload");
    }
    hd.K = K;
    g_xplans.emplace(std::move(key), XfftEntry{dev, hd});
    *out = hd;
    return EPIC_OK;
}

void clear_all_caches()
{
    std::lock_guard<std::mutex> lock(g_mu);
    (void)hipDeviceSynchronize();
    for (auto &kv : g_plans) (void)hipFree(kv.second.dev);
    g_plans.clear();
    for (auto &kv : g_xplans) (void)hipFree(kv.second.dev);
    g_xplans.clear();
    for (auto &kv : g_twiddles) (void)hipFree(kv.second);
    g_twiddles.clear();
    for (auto &kv : g_dft_tables) (void)hipFree(kv.second);
    g_dft_tables.clear();
    for (auto &kv : g_ws) (void)hipFree(kv.second.ptr);
    g_ws.clear();
}

}  // namespace epic
