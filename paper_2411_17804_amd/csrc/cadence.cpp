// cadence.cpp -- the image_cadence driver.
//
// Stations of one call are sorted into kernel classes: the fused FP32 kernels
// (square grids up to 64, one class per grid size, split where the LDS of
// the class's largest station would not fit the fast kernel), the fused
// split-precision kernel (square grids up to 64, per grid size and footprint
// tile count, split where the LDS would overflow) and the FP32 kernel for
// 128 x 128 grids.  All are persistent kernels: one launch per class takes
// its (station, channel) items from a work queue (queue.hpp) whose lists are
// balanced over the XCDs and ordered longest first, and each item images its
// pair over the whole cadence, keeping FP64 running sums in the caller's
// image buffer until it writes the mean products (accum.hpp).  The
// 128 x 128 kernel grids each block of samples into footprint boxes in its
// work-group's slice of a box buffer before transforming them.  Stations
// outside every class take the composed path (grid -> transform -> square
// and accumulate, in time chunks).
//
// The class tables, item lists and queue counters are built once per distinct
// call (same geometry, buffers and stream) and kept.  The first call runs
// eagerly (kernel attributes are set and every library buffer is allocated);
// later calls replay the whole cadence, the queue reset included, from a
// captured hipGraph.
//
// Each class has tile parameters: the number of samples summed in FP32
// before they go to the FP64 running sums (8 or 16; both keep the error of
// the mean within 16 units in the last place of FP32) and, where the class
// has more than one kernel shape, the shape (for the 64 x 64 FP32 class the
// 1024-thread kernel with one pol per thread or the 512-thread kernel with
// both).  epic_autotune times every candidate on the caller's data and keeps
// the fastest, in memory and, if EPIC_TUNE_CACHE names a file, on disk
// ("key variant flush" lines).
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "internal.hpp"

namespace epic {

StationDev make_station_dev(const epic_station *s, const PlanHandle &p);
epic_status cadence_composed(const epic_common *c, const epic_station *s, const PlanHandle &p,
                             int device, hipStream_t stream, const float2 *pol_kernels = nullptr);

int persistent_grid(const void *kernel, int block, size_t lds, int n_items)
{
    static int n_cu = 0;
    if (n_cu == 0) {
        int dev = 0;
        hipDeviceProp_t prop{};
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            n_cu = prop.multiProcessorCount;
        if (n_cu <= 0) n_cu = 256;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, lds) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return std::max(1, std::min(n_items, per_cu * n_cu));
}

namespace {

constexpr int kPathFft = 0, kPathDft = 1, kPathFft128 = 2;
// Samples summed in FP32 before the FP64 running sums (the bound of the
// plain block sum, (B - 1) units in the last place, is what limits the error
// of the mean).
constexpr int kDefaultFlush = 16;
const int kFlushCandidates[] = {8, 16};
// Samples the 128 x 128 FP32 kernel grids at a time (its variants): each
// work-group's boxes for one sample take about 100 KB on the largest
// stations, so blocks of a few samples stay in the L2 between gridding and
// transform, while larger blocks stage the channel's taps into LDS less
// often; the autotuner measures which wins.
const int kGridBlocks128[] = {2, 4, 1, 16};

struct Tile {
    int variant = 0;
    int flush = kDefaultFlush;
};

struct Group {
    int path = kPathFft;
    int n = 0;
    int tiles = 0;
    Tile tile;
    std::vector<int> members;     // station indices of the call
    FusedBatch batch;             // device pointers set after upload
    size_t wg_box_floats = 0;     // 128 x 128 class: footprint boxes per work-group
    std::vector<StationDev> host_sds;
    std::vector<int4> host_items;
    int queue_slot = 0;           // first of this group's kXcds counters
};

struct CadencePlan {
    std::vector<Group> groups;
    std::vector<int> composed;
    void *dev_tables = nullptr;
    float2 *boxes = nullptr;         // footprint boxes of the 128 x 128 classes' work-groups
    int *counters = nullptr;         // queue counters, kXcds per persistent group
    int n_counters = 0;
    const float2 *twiddles[257] = {};
    const uint32_t *rows[257] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_failed = false;
    int runs = 0;
};

std::mutex g_mu;
std::map<std::string, CadencePlan *> g_plans;
std::map<std::string, Tile> g_tuned;   // class key -> tile
int g_tune_generation = 0;
bool g_tune_loaded = false;

int tiles_for_side(int side, int n) { return std::max((side + 15) / 16, n == 64 ? 2 : 1); }

std::string class_key(const Group &g, const epic_common *c)
{
    std::ostringstream o;
    o << (g.path == kPathFft ? "fft" : g.path == kPathDft ? "dft" : "fft128") << "_n" << g.n << "_t"
      << g.tiles << "_p" << c->n_pol << "_v" << c->volt_type << "_q" << c->precision;
    return o.str();
}

int grid_block128(const Group &g) { return kGridBlocks128[g.tile.variant & 3]; }

// Every split-precision class runs either its persistent kernel (variant 0)
// or, per station, the composed path (variant 1), and the FP32 classes up to
// 64 x 64 have the composed path as variant kComposedFft: the autotuner
// measures both.  At 128 x 128 the composed path's separate gridding,
// transform and squaring kernels can be the faster on gfx950; smaller, a
// persistent work-group images a (station, channel) over the whole cadence,
// so a call with few channels keeps few work-groups busy, while the composed
// kernels spread every (channel, sample) over the GPU.
constexpr int kComposedFft = 2;
bool runs_composed(const Group &g)
{
    return (g.path == kPathDft && g.tile.variant == 1) || (g.path == kPathFft && g.tile.variant == kComposedFft);
}

// Kernel shapes a class can run (variant numbers the launcher understands).
std::vector<int> variants_of(const Group &g, const epic_common *c)
{
    if (g.path == kPathDft) return {0, 1};
    if (g.path == kPathFft128) return {0, 1, 2, 3};
    if (g.path == kPathFft && g.n == 64 && c->n_pol == 2) {
        std::vector<int> v;
        for (int k = 0; k < 2; ++k)
            if (fft64_fits(g.batch, c->n_pol, c->volt_type, k)) v.push_back(k);
        if (!v.empty()) {
            v.push_back(kComposedFft);
            return v;
        }
    }
    if (g.path == kPathFft) return {0, kComposedFft};
    return {0};
}

void load_tune_file()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("EPIC_TUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string key;
        Tile t;
        if (!(in >> key >> t.variant >> t.flush)) continue;
        if (std::find(std::begin(kFlushCandidates), std::end(kFlushCandidates), t.flush) !=
                std::end(kFlushCandidates) && t.variant >= 0 && t.variant < 4)
            g_tuned[key] = t;
    }
}

void save_tune_file()
{
    const char *path = std::getenv("EPIC_TUNE_CACHE");
    if (!path) return;
    std::ofstream f(path, std::ios::trunc);
    for (auto &kv : g_tuned) f << kv.first << " " << kv.second.variant << " " << kv.second.flush << "\n";
}

void free_plan(CadencePlan *p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->dev_tables) (void)hipFree(p->dev_tables);
    if (p->boxes) (void)hipFree(p->boxes);
    delete p;
}

std::string call_key(const epic_common *c, const epic_station *st, int n, const PlanHandle *plans,
                     int device, hipStream_t stream, const std::vector<Tile> &tiles_override)
{
    std::string k;
    auto put = [&k](const void *p, size_t b) { k.append(static_cast<const char *>(p), b); };
    put(&device, sizeof device);
    put(&stream, sizeof stream);
    put(&g_tune_generation, sizeof g_tune_generation);
    put(&c->n_pol, sizeof c->n_pol);
    put(&c->n_chan, sizeof c->n_chan);
    put(&c->n_time, sizeof c->n_time);
    put(&c->volt_type, sizeof c->volt_type);
    put(&c->precision, sizeof c->precision);
    for (int i = 0; i < n; ++i) {
        put(&plans[i].chan, sizeof plans[i].chan);   // plans are cached by content
        put(&st[i].volts, sizeof st[i].volts);
        put(&st[i].image, sizeof st[i].image);
    }
    for (const Tile &t : tiles_override) {
        put(&t.variant, sizeof t.variant);
        put(&t.flush, sizeof t.flush);
    }
    return k;
}

// The batch maxima of one station.
FusedBatch station_batch(const StationDev &sd, int n)
{
    FusedBatch b;
    b.n = n;
    b.max_elem = sd.n_elem;
    b.max_cells = sd.max_cells;
    b.max_cell_taps = sd.max_cell_taps;
    b.max_ktaps = sd.ktaps;
    b.max_side = std::max(sd.max_bw, sd.max_bh);
    b.max_bw = sd.max_bw;
    b.max_bh = sd.max_bh;
    return b;
}

FusedBatch merged(const FusedBatch &a, const FusedBatch &b)
{
    FusedBatch m = a;
    m.max_elem = std::max(a.max_elem, b.max_elem);
    m.max_cells = std::max(a.max_cells, b.max_cells);
    m.max_cell_taps = std::max(a.max_cell_taps, b.max_cell_taps);
    m.max_ktaps = std::max(a.max_ktaps, b.max_ktaps);
    m.max_side = std::max(a.max_side, b.max_side);
    m.max_bw = std::max(a.max_bw, b.max_bw);
    m.max_bh = std::max(a.max_bh, b.max_bh);
    return m;
}

// Whether one launch of the group's kernel covers stations with these
// combined maxima (the LDS and register layouts are sized by the maxima).
bool group_fits(int path, const FusedBatch &b, int max_bw, int max_bh, const epic_common *c)
{
    if (path == kPathDft) return fused_dft_supported(b, c->n_pol, c->volt_type);
    if (path == kPathFft128)
        return fused128_supported(128, max_bw, max_bh, b.max_elem, c->n_pol, c->volt_type, b.max_ktaps,
                                  b.max_cell_taps);
    return true;   // the generic FP32 kernel takes any batch; see below for 64
}

// Sort the call's stations into groups (no device work).
void classify(const epic_common *c, const epic_station *st, int n, const PlanHandle *plans,
              std::vector<Group> &groups, std::vector<int> &composed)
{
    std::map<std::string, int> index;
    for (int i = 0; i < n; ++i) {
        const StationDev sd = make_station_dev(&st[i], plans[i]);
        const bool square = st[i].nx == st[i].ny && st[i].nx <= 64;
        // the split-precision kernels also take 128 x 128 grids
        const bool split_square = square || (st[i].nx == 128 && st[i].ny == 128);
        int path = -1, tiles = 0;
        if (st[i].nx == st[i].ny && c->precision == EPIC_FP32_FFT &&
            fused128_supported(st[i].nx, sd.max_bw, sd.max_bh, sd.n_elem, c->n_pol, c->volt_type,
                               sd.ktaps, sd.max_cell_taps)) {
            path = kPathFft128;
        } else if (square && c->precision == EPIC_FP32_FFT) {
            path = kPathFft;
        } else if (split_square && c->precision != EPIC_FP32_FFT) {
            const FusedBatch one = station_batch(sd, st[i].nx);
            const int64_t vbytes = static_cast<int64_t>(sd.n_elem) * c->n_pol * (c->volt_type == EPIC_CI8 ? 2 : 8);
            if (vbytes % 4 == 0 && fused_dft_supported(one, c->n_pol, c->volt_type)) {
                path = kPathDft;
                // one class for 128 x 128 (its kernel takes any footprint up
                // to its limit); by footprint tiles below that
                tiles = one.n == 128 ? 0 : tiles_for_side(one.max_side, one.n);
            }
        }
        if (path < 0) {
            composed.push_back(i);
            continue;
        }
        Group probe;
        probe.path = path;
        probe.n = st[i].nx;
        probe.tiles = tiles;
        const std::string key = class_key(probe, c);
        auto it = index.find(key);
        if (it == index.end()) {
            index[key] = static_cast<int>(groups.size());
            groups.push_back(probe);
            it = index.find(key);
        }
        groups[it->second].members.push_back(i);
    }
    // largest stations first inside each group; split groups whose combined
    // maxima would overflow the kernel's LDS (or, for the 64 x 64 FP32 class,
    // push the fast kernels' LDS over the limit: the stations that break it
    // start a group of their own)
    std::vector<Group> out;
    for (auto &g : groups) {
        std::sort(g.members.begin(), g.members.end(),
                  [&](int a, int b) { return st[a].n_elem > st[b].n_elem; });
        Group cur = g;
        cur.members.clear();
        FusedBatch acc;
        acc.n = g.n;
        int bw = 0, bh = 0;
        for (int i : g.members) {
            const StationDev sd = make_station_dev(&st[i], plans[i]);
            const FusedBatch one = station_batch(sd, g.n);
            const FusedBatch next = cur.members.empty() ? one : merged(acc, one);
            const int nbw = std::max(bw, sd.max_bw), nbh = std::max(bh, sd.max_bh);
            bool fits = group_fits(g.path, next, nbw, nbh, c);
            if (g.path == kPathFft && g.n == 64 && !cur.members.empty()) {
                // a group either fits the fastest kernel (the two-pol one for
                // two pols) or runs the next one that does
                const int v0 = c->n_pol == 2 ? 0 : 1;
                const bool f_acc = fft64_fits(acc, c->n_pol, c->volt_type, v0);
                const bool f_one = fft64_fits(one, c->n_pol, c->volt_type, v0);
                fits = f_acc ? fft64_fits(next, c->n_pol, c->volt_type, v0) : !f_one;
            }
            if (!fits && !cur.members.empty()) {
                cur.batch = acc;
                out.push_back(cur);
                cur.members.clear();
                acc = one;
                bw = sd.max_bw;
                bh = sd.max_bh;
            } else {
                acc = next;
                bw = nbw;
                bh = nbh;
            }
            cur.members.push_back(i);
        }
        cur.batch = acc;
        out.push_back(cur);
    }
    groups.swap(out);
    for (Group &g : groups) {
        auto it = g_tuned.find(class_key(g, c));
        g.tile = it == g_tuned.end() ? Tile{} : it->second;
        const std::vector<int> vs = variants_of(g, c);
        if (std::find(vs.begin(), vs.end(), g.tile.variant) == vs.end()) g.tile.variant = 0;
    }
}

// Relative cost of an item of `nt` samples of one station (for ordering).
double item_cost(const StationDev &sd, int n_pol, int nt)
{
    const double npix = static_cast<double>(sd.nx) * sd.ny;
    return nt * (npix * sd.log2n * 2.0 * n_pol + 4.0 * sd.n_elem * sd.ktaps * n_pol);
}

// Work items per (station, channel): the 128 x 128 split-precision kernel
// takes each half of the output rows as an item of its own.
int parts_of(const Group &g) { return g.path == kPathDft && g.n == 128 ? 2 : 1; }

// The persistent group's (station, channel) items in kXcds lists: longest
// first onto the least loaded list, and each list ordered longest first.
void build_queue_lists(Group &g, int n_chan, int n_time, int n_pol)
{
    struct Item {
        double cost;
        int4 it;
    };
    std::vector<Item> all;
    const int parts = parts_of(g);
    for (size_t k = 0; k < g.host_sds.size(); ++k)
        for (int ch = 0; ch < n_chan; ++ch)
            for (int part = 0; part < parts; ++part)
                all.push_back({item_cost(g.host_sds[k], n_pol, n_time) / parts,
                               make_int4(static_cast<int>(k), ch, part, 0)});
    std::stable_sort(all.begin(), all.end(), [](const Item &a, const Item &b) { return a.cost > b.cost; });
    double load[kXcds] = {};
    std::vector<int4> lists[kXcds];
    for (const Item &i : all) {
        const int x = static_cast<int>(std::min_element(load, load + kXcds) - load);
        load[x] += i.cost;
        lists[x].push_back(i.it);
    }
    g.host_items.clear();
    for (int x = 0; x < kXcds; ++x) {
        g.batch.q.start[x] = static_cast<int>(g.host_items.size());
        g.host_items.insert(g.host_items.end(), lists[x].begin(), lists[x].end());
    }
    g.batch.q.start[kXcds] = static_cast<int>(g.host_items.size());
}

epic_status build_plan(const epic_common *c, const epic_station *st, int n, const PlanHandle *plans,
                       int device, const std::vector<Tile> &tiles_override, CadencePlan *p)
{
    classify(c, st, n, plans, p->groups, p->composed);
    size_t n_sds = 0, n_items = 0, box_floats = 0;
    int n_counters = 0;
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        Group &g = p->groups[gi];
        if (gi < tiles_override.size() && tiles_override[gi].flush > 0) g.tile = tiles_override[gi];
        g.batch.variant = g.tile.variant;
        for (int i : g.members) g.host_sds.push_back(make_station_dev(&st[i], plans[i]));
        build_queue_lists(g, c->n_chan, c->n_time, c->n_pol);
        g.queue_slot = n_counters;
        n_counters += kXcds;
        g.batch.n_items = static_cast<int>(g.host_items.size());
        if (g.path == kPathFft128) {
            // each work-group grids a block of samples at a time into its own
            // boxes; the classes run one after another, so one buffer serves
            // them all
            const int block = std::min(grid_block128(g), c->n_time);
            size_t wg = 0;
            for (const StationDev &sd : g.host_sds)
                wg = std::max(wg, static_cast<size_t>(block) * c->n_pol * sd.max_bw * sd.max_bh);
            g.wg_box_floats = (wg + 31) & ~static_cast<size_t>(31);   // 256-byte slices
            g.batch.grid = cadence128_grid(c->n_pol, c->volt_type, g.batch.n_items);
            box_floats = std::max(box_floats, g.wg_box_floats * g.batch.grid);
        }
        n_sds += g.host_sds.size();
        n_items += g.host_items.size();
        if (g.path != kPathDft && !p->twiddles[g.n]) {
            epic_status s = get_twiddles(g.n, device, &p->twiddles[g.n]);
            if (s != EPIC_OK) return s;
        }
        if (g.path == kPathDft && !p->rows[g.n]) {
            epic_status s = get_dft_rows(g.n, c->precision, device, &p->rows[g.n]);
            if (s != EPIC_OK) return s;
        }
    }
    if (p->groups.empty()) return EPIC_OK;
    auto up = [](size_t b) { return (b + 255) & ~static_cast<size_t>(255); };
    const size_t b_sds = up(sizeof(StationDev) * n_sds);
    const size_t b_items = up(sizeof(int4) * n_items);
    const size_t b_cnt = up(sizeof(int) * std::max(1, n_counters));
    epic_status as = dev_alloc(&p->dev_tables, b_sds + b_items + b_cnt);
    if (as != EPIC_OK) return as;
    if (box_floats) {
        as = dev_alloc(reinterpret_cast<void **>(&p->boxes), sizeof(float2) * box_floats);
        if (as != EPIC_OK) return as;
    }
    char *base = static_cast<char *>(p->dev_tables);
    StationDev *dsds = reinterpret_cast<StationDev *>(base);
    int4 *ditems = reinterpret_cast<int4 *>(base + b_sds);
    p->counters = reinterpret_cast<int *>(base + b_sds + b_items);
    p->n_counters = n_counters;
    for (auto &g : p->groups) {
        EPIC_HIP_TRY(hipMemcpy(dsds, g.host_sds.data(), sizeof(StationDev) * g.host_sds.size(),
                               hipMemcpyHostToDevice));
        EPIC_HIP_TRY(hipMemcpy(ditems, g.host_items.data(), sizeof(int4) * g.host_items.size(),
                               hipMemcpyHostToDevice));
        g.batch.sds = dsds;
        g.batch.items = ditems;
        g.batch.q.items = ditems;
        g.batch.q.counters = p->counters + g.queue_slot;
        dsds += g.host_sds.size();
        ditems += g.host_items.size();
        g.host_items.clear();
        g.host_items.shrink_to_fit();
    }
    return EPIC_OK;
}

epic_status launch_group(const epic_common *c, const epic_station *st, const PlanHandle *plans, int device,
                         const CadencePlan *p, const Group &g, hipStream_t stream)
{
    const int flush = g.tile.flush;
    if (runs_composed(g)) {
        for (int i : g.members) {
            epic_status s = cadence_composed(c, &st[i], plans[i], device, stream);
            if (s != EPIC_OK) return s;
        }
        return EPIC_OK;
    }
    if (g.path == kPathFft)
        return launch_fused_fft(g.batch, c->n_pol, c->n_time, c->volt_type, flush, p->twiddles[g.n], stream);
    if (g.path == kPathFft128)
        return launch_cadence128(g.batch, c->n_pol, c->n_time, c->volt_type, flush, grid_block128(g), p->boxes,
                                 g.wg_box_floats, p->twiddles[g.n], stream);
    return launch_fused_dft(g.batch, c->n_pol, c->n_time, c->volt_type, c->precision, flush,
                            p->rows[g.n], stream);
}

// The whole cadence: queue reset, the class kernels (which write the fused
// stations' images), then the composed stations.
epic_status enqueue_all(const epic_common *c, const epic_station *st, const PlanHandle *plans,
                        const CadencePlan *p, int device, hipStream_t stream)
{
    epic_status s = launch_queue_reset(p->counters, p->n_counters, stream);
    if (s != EPIC_OK) return s;
    for (const Group &g : p->groups) {
        s = launch_group(c, st, plans, device, p, g, stream);
        if (s != EPIC_OK) return s;
    }
    for (int i : p->composed) {
        s = cadence_composed(c, &st[i], plans[i], device, stream);
        if (s != EPIC_OK) return s;
    }
    return EPIC_OK;
}

bool graphs_enabled()
{
    const char *e = std::getenv("EPIC_NO_GRAPH");
    return !(e && e[0] == '1') && !timing_on();
}

epic_status get_or_build(const epic_common *c, const epic_station *st, int n, const PlanHandle *plans,
                         int device, hipStream_t stream, const std::vector<Tile> &tiles_override,
                         CadencePlan **out)
{
    const std::string key = call_key(c, st, n, plans, device, stream, tiles_override);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
        *out = it->second;
        return EPIC_OK;
    }
    if (g_plans.size() >= 32) {   // keep the cache bounded
        (void)hipStreamSynchronize(stream);
        (void)hipDeviceSynchronize();
        for (auto &kv : g_plans) free_plan(kv.second);
        g_plans.clear();
    }
    CadencePlan *p = new CadencePlan();
    epic_status s = build_plan(c, st, n, plans, device, tiles_override, p);
    if (s != EPIC_OK) {
        free_plan(p);
        return s;
    }
    g_plans[key] = p;
    *out = p;
    return EPIC_OK;
}

void drop_plan(CadencePlan *p)
{
    for (auto it = g_plans.begin(); it != g_plans.end(); ++it)
        if (it->second == p) {
            free_plan(p);
            g_plans.erase(it);
            return;
        }
}

}  // namespace

epic_status run_cadence(const epic_common *c, const epic_station *st, int n, const PlanHandle *plans,
                        int device, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(g_mu);
    load_tune_file();
    CadencePlan *p = nullptr;
    epic_status s = get_or_build(c, st, n, plans, device, stream, {}, &p);
    if (s != EPIC_OK) return s;
    // first call eager (sets kernel attributes, allocates the composed path's
    // workspaces, checks launches); afterwards the captured graph
    if (graphs_enabled() && !p->graph_failed && p->runs > 0) {
        if (!p->exec) {
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed);
            epic_status es = e == hipSuccess ? enqueue_all(c, st, plans, p, device, stream) : EPIC_ERR_DEVICE;
            hipError_t e2 = hipStreamEndCapture(stream, &graph);
            hipGraphExec_t exec = nullptr;
            if (e == hipSuccess && es == EPIC_OK && e2 == hipSuccess && graph &&
                hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess) {
                p->graph = graph;
                p->exec = exec;
            } else {
                if (graph) (void)hipGraphDestroy(graph);
                (void)hipGetLastError();
                p->graph_failed = true;
            }
        }
        if (p->exec) {
            ++p->runs;
            EPIC_HIP_TRY(hipGraphLaunch(p->exec, stream));
            return EPIC_OK;
        }
    }
    ++p->runs;
    return enqueue_all(c, st, plans, p, device, stream);
}

epic_status tune_cadence(const epic_common *c, const epic_station *st, int n,
                         const PlanHandle *plans, int device, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(g_mu);
    load_tune_file();
    // the group layout does not depend on the tiles: classify once
    std::vector<Group> groups;
    std::vector<int> composed;
    classify(c, st, n, plans, groups, composed);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    EPIC_HIP_TRY(hipEventCreate(&e0));
    EPIC_HIP_TRY(hipEventCreate(&e1));
    std::vector<Tile> best(groups.size());
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        float best_ms = 1e30f;
        for (int variant : variants_of(groups[gi], c))
            for (int flush : kFlushCandidates) {
                std::vector<Tile> over(groups.size(), Tile{0, 0});
                over[gi] = Tile{variant, flush};
                CadencePlan *p = nullptr;
                epic_status s = get_or_build(c, st, n, plans, device, stream, over, &p);
                if (s != EPIC_OK) return s;
                // one untimed launch, then the better of two timed ones
                s = launch_queue_reset(p->counters, p->n_counters, stream);
                if (s == EPIC_OK) s = launch_group(c, st, plans, device, p, p->groups[gi], stream);
                if (s != EPIC_OK) return s;
                float ms = 1e30f;
                for (int rep = 0; rep < 2; ++rep) {
                    s = launch_queue_reset(p->counters, p->n_counters, stream);
                    if (s != EPIC_OK) return s;
                    EPIC_HIP_TRY(hipEventRecord(e0, stream));
                    s = launch_group(c, st, plans, device, p, p->groups[gi], stream);
                    if (s != EPIC_OK) return s;
                    EPIC_HIP_TRY(hipEventRecord(e1, stream));
                    EPIC_HIP_TRY(hipEventSynchronize(e1));
                    float t = 0.f;
                    EPIC_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
                    ms = std::min(ms, t);
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    best[gi] = Tile{variant, flush};
                }
                // free each trial plan at once
                EPIC_HIP_TRY(hipStreamSynchronize(stream));
                drop_plan(p);
            }
        g_tuned[class_key(groups[gi], c)] = best[gi];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // drop the trial plans; the next image_cadence builds with the tuned tiles
    EPIC_HIP_TRY(hipStreamSynchronize(stream));
    for (auto &kv : g_plans) free_plan(kv.second);
    g_plans.clear();
    ++g_tune_generation;
    save_tune_file();
    return EPIC_OK;
}

// ------------------------------------------------------------------------
// The cadence without allocating: every table a call needs (the stations'
// plans, the transform tables, the class tables, item lists and queue
// counters) goes into one file-scope device array instead of library
// allocations.  The image buffers carry the running sums as in run_cadence.
// Each GPU holds its own copy of the array (its address, taken once per
// device with hipGetSymbolAddress, is kept per device); calls on one GPU
// share it, so calls that overlap on one GPU race (the call waits for its own
// stream's earlier work before it overwrites the array).
// ------------------------------------------------------------------------
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch;   // device -> address of its scratch

epic_status scratch_of(int device, unsigned char **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch.find(device);
    if (it != g_scratch.end()) {
        *out = it->second;
        return EPIC_OK;
    }
    void *ptr = nullptr;
    EPIC_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch[device] = static_cast<unsigned char *>(ptr);
    *out = static_cast<unsigned char *>(ptr);
    return EPIC_OK;
}

// Sub-ranges of the scratch array, 256-byte aligned, with their host sources.
struct ScratchLayout {
    size_t used = 0;
    std::vector<std::pair<size_t, std::pair<const void *, size_t>>> copies;
    size_t put(const void *src, size_t bytes)
    {
        const size_t off = used;
        used = (used + bytes + 255) & ~static_cast<size_t>(255);
        if (src && bytes) copies.push_back({off, {src, bytes}});
        return off;
    }
};

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

epic_status run_cadence_noalloc(const epic_common *c, const epic_station *st, int n, int device,
                                hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(g_mu);
    load_tune_file();
    unsigned char *base = nullptr;
    epic_status s = scratch_of(device, &base);
    if (s != EPIC_OK) return s;

    // host tables of every station
    std::vector<HostPlan> hps(n);
    for (int i = 0; i < n; ++i) {
        s = build_host_plan(c, &st[i], &hps[i]);
        if (s != EPIC_OK) return fail(s, "station " + std::to_string(i) + ": " + last_error_cstr());
    }
    ScratchLayout lay;
    std::vector<PlanHandle> plans(n);
    for (int i = 0; i < n; ++i) {
        const HostPlan &h = hps[i];
        PlanHandle &ph = plans[i];
        ph.chan = reinterpret_cast<const ChanPlan *>(base + lay.put(h.chans.data(), sizeof(ChanPlan) * h.chans.size()));
        ph.cell_start = reinterpret_cast<const int32_t *>(base + lay.put(h.cell_start.data(), sizeof(int32_t) * h.cell_start.size()));
        ph.taps = reinterpret_cast<const Tap *>(base + lay.put(h.taps.data(), sizeof(Tap) * h.taps.size()));
        ph.cell_order = reinterpret_cast<const int32_t *>(base + lay.put(h.cell_order.data(), sizeof(int32_t) * h.cell_order.size()));
        ph.elem_cell = nullptr;   // the fused kernels do not read it
        ph.max_box = h.max_box;
        ph.max_bw = h.max_bw;
        ph.max_bh = h.max_bh;
        ph.max_cell_taps = h.max_cell_taps;
        ph.n_taps_total = static_cast<int64_t>(h.taps.size());
    }
    CadencePlan p;
    classify(c, st, n, plans.data(), p.groups, p.composed);
    if (!p.composed.empty())
        return fail(EPIC_ERR_UNSUPPORTED, "image_cadence_noalloc: station " + std::to_string(p.composed.front()) +
                                              " needs the composed path's workspaces; square grids up to 64 (FP32) "
                                              "or 128 (split precision) run without allocating");
    std::vector<std::vector<float2>> tw_host;
    std::vector<std::vector<unsigned char>> rows_host;
    for (Group &g : p.groups) {
        if (g.path == kPathFft128)
            return fail(EPIC_ERR_UNSUPPORTED, "image_cadence_noalloc: 128 x 128 FP32 stations need the footprint-box "
                                              "buffer; FP32 runs without allocating on square grids up to 64");
        if (runs_composed(g)) g.tile.variant = 0;   // the persistent kernel allocates nothing
        g.batch.variant = g.tile.variant;
        for (int i : g.members) g.host_sds.push_back(make_station_dev(&st[i], plans[i]));
        build_queue_lists(g, c->n_chan, c->n_time, c->n_pol);
        g.batch.n_items = static_cast<int>(g.host_items.size());
        if (g.path == kPathFft && !p.twiddles[g.n]) {
            tw_host.emplace_back(g.n);
            fill_twiddles(g.n, tw_host.back().data());
            p.twiddles[g.n] = reinterpret_cast<const float2 *>(base + lay.put(tw_host.back().data(), sizeof(float2) * g.n));
        }
        if (g.path == kPathDft && !p.rows[g.n]) {
            rows_host.emplace_back(static_cast<size_t>(g.n) * g.n * 8);
            fill_rows_any(g.n, c->precision, rows_host.back().data());
            p.rows[g.n] = reinterpret_cast<const uint32_t *>(base + lay.put(rows_host.back().data(), rows_host.back().size()));
        }
    }
    int n_counters = 0;
    for (Group &g : p.groups) {
        g.batch.sds = reinterpret_cast<const StationDev *>(base + lay.put(g.host_sds.data(), sizeof(StationDev) * g.host_sds.size()));
        g.batch.items = reinterpret_cast<const int4 *>(base + lay.put(g.host_items.data(), sizeof(int4) * g.host_items.size()));
        g.batch.q.items = g.batch.items;
        g.queue_slot = n_counters;
        n_counters += kXcds;
    }
    p.counters = reinterpret_cast<int *>(base + lay.put(nullptr, sizeof(int) * std::max(1, n_counters)));
    p.n_counters = n_counters;
    for (Group &g : p.groups) g.batch.q.counters = p.counters + g.queue_slot;
    if (lay.used > kScratchBytes)
        return fail(EPIC_ERR_UNSUPPORTED, "image_cadence_noalloc: the call needs " + std::to_string(lay.used) +
                                              " bytes of tables, the allocation-free scratch holds " +
                                              std::to_string(kScratchBytes) + " (fewer channels or stations per call)");
    // the previous call on this stream may still read the scratch
    EPIC_HIP_TRY(hipStreamSynchronize(stream));
    for (const auto &cp : lay.copies)
        EPIC_HIP_TRY(hipMemcpy(base + cp.first, cp.second.first, cp.second.second, hipMemcpyHostToDevice));
    s = launch_queue_reset(p.counters, p.n_counters, stream);
    if (s != EPIC_OK) return s;
    for (const Group &g : p.groups) {
        s = launch_group(c, st, plans.data(), device, &p, g, stream);
        if (s != EPIC_OK) return s;
    }
    return EPIC_OK;
}

void clear_cadence_cache()
{
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto &kv : g_plans) free_plan(kv.second);
    g_plans.clear();
    // the tuner's choices too: the next plan reads EPIC_TUNE_CACHE again
    g_tuned.clear();
    g_tune_loaded = false;
}

}  // namespace epic
