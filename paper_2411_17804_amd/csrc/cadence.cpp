// cadence.cpp -- the image_cadence driver.
//
// Stations of one call are sorted into kernel classes: the fused FP32 kernel
// (square grids up to 64, one class per grid size), the fused split-precision
// kernel (square grids up to 64, one class per grid size and footprint tile
// count, split further if the LDS would overflow) and the FP32 path for
// 128 x 128 grids.  Each of the first two runs as ONE launch over its work
// items (station, channel, time chunk), ordered largest station first so the
// longest items start first.  The 128 x 128 class runs per time block: a
// gridding launch into footprint boxes, then the fused transform-and-square
// launch, for each batch of (station, channel) pairs whose boxes fit the box
// buffer.  Each fused station then gets its ordered, compensated chunk
// reduction.  Stations outside every class take the composed path (grid ->
// transform -> square and accumulate, in time chunks).
//
// The class tables, item lists and partial-sum buffers are built once per
// distinct call (same geometry, buffers and stream) and kept; when every
// station is fused the whole cadence is captured into a hipGraph on first use
// and replayed afterwards.
//
// The time-chunk length of each class (16, 32, 64 or 128 samples) is a tile
// parameter: epic_autotune times the candidates on the caller's data and keeps
// the fastest, in memory and, if EPIC_TUNE_CACHE names a file, on disk
// ("key chunk" lines).
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

namespace {

constexpr int kPathFft = 0, kPathDft = 1, kPathFft128 = 2;
// Bytes of footprint boxes per batch of the 128 x 128 class: 2 GiB, or
// EPIC_BOX_BUDGET_MB megabytes (a smaller buffer means more, smaller batches).
size_t box_budget()
{
    const char *e = std::getenv("EPIC_BOX_BUDGET_MB");
    const long mb = e ? std::atol(e) : 0;
    return mb > 0 ? static_cast<size_t>(mb) << 20 : size_t(2) << 30;
}
constexpr int kDefaultChunk = 32;
// Chunk lengths the autotuner tries.  Each chunk is a plain FP32 sum (its
// rounding error grows at most linearly, 128 * 2^-24 < 1e-5 relative), and
// the chunks are then added with compensation.
const int kChunkCandidates[] = {16, 32, 64, 128};

struct Group {
    int path = kPathFft;
    int n = 0;
    int tiles = 0;
    int chunk = kDefaultChunk;
    std::vector<int> members;     // station indices of the call
    FusedBatch batch;             // device pointers set after upload
    std::vector<std::pair<int, int>> pair_batches;   // 128 x 128 class: (first item, count)
    std::vector<StationDev> host_sds;
    std::vector<int4> host_items;
};

struct CadencePlan {
    std::vector<Group> groups;
    std::vector<int> composed;
    std::vector<int64_t> part_off;   // per station, floats (fused stations)
    std::vector<int> chunk;          // per station chunk length (fused stations)
    void *dev_tables = nullptr;
    float *partials = nullptr;
    float2 *boxes = nullptr;         // footprint boxes of one batch (128 x 128 class)
    const float2 *twiddles[257] = {};
    const uint32_t *rows[257] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_failed = false;
    int runs = 0;
};

std::mutex g_mu;
std::map<std::string, CadencePlan *> g_plans;
std::map<std::string, int> g_tuned;   // class key -> chunk
int g_tune_generation = 0;
bool g_tune_loaded = false;

int tiles_for_side(int side, int n) { return std::max((side + 15) / 16, n == 64 ? 2 : 1); }

std::string class_key(int path, int n, int tiles, const epic_common *c)
{
    std::ostringstream o;
    o << (path == kPathFft ? "fft" : path == kPathDft ? "dft" : "fft128") << "_n" << n << "_t" << tiles << "_p" << c->n_pol << "_v"
      << c->volt_type << "_q" << c->precision;
    return o.str();
}

void load_tune_file()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("EPIC_TUNE_CACHE");
    if (!path) return;
    std::ifstream f(path);
    std::string key;
    int chunk = 0;
    while (f >> key >> chunk)
        if (chunk == 16 || chunk == 32 || chunk == 64 || chunk == 128) g_tuned[key] = chunk;
}

void save_tune_file()
{
    const char *path = std::getenv("EPIC_TUNE_CACHE");
    if (!path) return;
    std::ofstream f(path, std::ios::trunc);
    for (auto &kv : g_tuned) f << kv.first << " " << kv.second << "\n";
}

int tuned_chunk(const std::string &key)
{
    auto it = g_tuned.find(key);
    return it == g_tuned.end() ? kDefaultChunk : it->second;
}

void free_plan(CadencePlan *p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->dev_tables) (void)hipFree(p->dev_tables);
    if (p->partials) (void)hipFree(p->partials);
    if (p->boxes) (void)hipFree(p->boxes);
    delete p;
}

std::string call_key(const epic_common *c, const epic_station *st, int n, const PlanHandle *plans,
                     int device, hipStream_t stream, const std::vector<int> &chunks_override)
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
    for (int v : chunks_override) put(&v, sizeof v);
    return k;
}

// Sort the call's stations into groups (no device work).
void classify(const epic_common *c, const epic_station *st, int n, const PlanHandle *plans,
              std::vector<Group> &groups, std::vector<int> &composed)
{
    std::map<std::string, int> index;
    for (int i = 0; i < n; ++i) {
        const StationDev sd = make_station_dev(&st[i], plans[i]);
        const bool square = st[i].nx == st[i].ny && st[i].nx <= 64;
        int path = -1, tiles = 0;
        if (st[i].nx == st[i].ny && c->precision == EPIC_FP32_FFT &&
            fused128_supported(st[i].nx, sd.max_bw, sd.max_bh, sd.n_elem, c->n_pol, c->volt_type,
                               sd.ktaps, sd.max_cell_taps)) {
            path = kPathFft128;
        } else if (square && c->precision == EPIC_FP32_FFT) {
            path = kPathFft;
        } else if (square) {
            FusedBatch one;
            one.n = st[i].nx;
            one.max_elem = sd.n_elem;
            one.max_cells = sd.max_cells;
            one.max_cell_taps = sd.max_cell_taps;
            one.max_ktaps = sd.ktaps;
            one.max_side = std::max(sd.max_bw, sd.max_bh);
            const int64_t vbytes = static_cast<int64_t>(sd.n_elem) * c->n_pol * (c->volt_type == EPIC_CI8 ? 2 : 8);
            if (vbytes % 4 == 0 && fused_dft_supported(one, c->n_pol, c->volt_type)) {
                path = kPathDft;
                tiles = tiles_for_side(one.max_side, one.n);
            }
        }
        if (path < 0) {
            composed.push_back(i);
            continue;
        }
        const std::string key = class_key(path, st[i].nx, tiles, c);
        auto it = index.find(key);
        if (it == index.end()) {
            Group g;
            g.path = path;
            g.n = st[i].nx;
            g.tiles = tiles;
            g.chunk = tuned_chunk(key);
            index[key] = static_cast<int>(groups.size());
            groups.push_back(g);
            it = index.find(key);
        }
        groups[it->second].members.push_back(i);
    }
    // largest stations first inside each group; split split-precision groups
    // whose combined maxima would overflow the LDS
    std::vector<Group> out;
    for (auto &g : groups) {
        std::sort(g.members.begin(), g.members.end(),
                  [&](int a, int b) { return st[a].n_elem > st[b].n_elem; });
        Group cur = g;
        cur.members.clear();
        FusedBatch acc;
        acc.n = g.n;
        for (int i : g.members) {
            const StationDev sd = make_station_dev(&st[i], plans[i]);
            FusedBatch next = acc;
            next.max_elem = std::max(next.max_elem, sd.n_elem);
            next.max_cells = std::max(next.max_cells, sd.max_cells);
            next.max_cell_taps = std::max(next.max_cell_taps, sd.max_cell_taps);
            next.max_ktaps = std::max(next.max_ktaps, sd.ktaps);
            next.max_side = std::max(next.max_side, std::max(sd.max_bw, sd.max_bh));
            const bool fits = g.path != kPathDft || fused_dft_supported(next, c->n_pol, c->volt_type);
            if (!fits && !cur.members.empty()) {
                out.push_back(cur);
                cur.members.clear();
                next = FusedBatch();
                next.n = g.n;
                next.max_elem = sd.n_elem;
                next.max_cells = sd.max_cells;
                next.max_cell_taps = sd.max_cell_taps;
                next.max_ktaps = sd.ktaps;
                next.max_side = std::max(sd.max_bw, sd.max_bh);
            }
            cur.members.push_back(i);
            acc = next;
        }
        cur.batch = acc;
        out.push_back(cur);
    }
    groups.swap(out);
}

epic_status build_plan(const epic_common *c, const epic_station *st, int n, const PlanHandle *plans,
                       int device, const std::vector<int> &chunks_override, CadencePlan *p)
{
    classify(c, st, n, plans, p->groups, p->composed);
    p->part_off.assign(n, -1);
    p->chunk.assign(n, 0);
    const int nq = c->n_pol == 2 ? 4 : 1;
    int64_t part = 0;
    size_t n_sds = 0, n_items = 0, box_floats = 0;
    for (size_t gi = 0; gi < p->groups.size(); ++gi) {
        Group &g = p->groups[gi];
        if (gi < chunks_override.size() && chunks_override[gi] > 0) g.chunk = chunks_override[gi];
        const int n_chunks = (c->n_time + g.chunk - 1) / g.chunk;
        for (size_t k = 0; k < g.members.size(); ++k) {
            const int i = g.members[k];
            StationDev sd = make_station_dev(&st[i], plans[i]);
            sd.part_off = part;
            p->part_off[i] = part;
            p->chunk[i] = g.chunk;
            part += static_cast<int64_t>(c->n_chan) * n_chunks * nq * sd.nx * sd.ny;
            g.host_sds.push_back(sd);
            if (g.path == kPathFft128) {
                for (int ch = 0; ch < c->n_chan; ++ch) g.host_items.push_back(make_int4(static_cast<int>(k), ch, 0, 0));
            } else {
                for (int ch = 0; ch < c->n_chan; ++ch)
                    for (int ck = 0; ck < n_chunks; ++ck)
                        g.host_items.push_back(make_int4(static_cast<int>(k), ch, ck, 0));
            }
        }
        g.batch.n_items = static_cast<int>(g.host_items.size());
        if (g.path == kPathFft128) {
            // batches of pairs whose boxes for one time block fit the budget;
            // box offsets restart at 0 in every batch (one buffer serves all)
            size_t pair_floats = 0;
            for (const StationDev &sd : g.host_sds)
                pair_floats = std::max(pair_floats, static_cast<size_t>(g.chunk) * c->n_pol * sd.max_bw * sd.max_bh);
            const int n_pairs = static_cast<int>(g.host_items.size());
            int per = static_cast<int>(std::max<size_t>(1, box_budget() / (sizeof(float2) * pair_floats)));
            if (per > 256 && per < n_pairs) per = per / 256 * 256;   // whole waves of work-groups
            per = std::min(per, n_pairs);
            for (int first = 0; first < n_pairs; first += per) {
                const int cnt = std::min(per, n_pairs - first);
                for (int q = 0; q < cnt; ++q)
                    g.host_items[first + q].w = static_cast<int>(static_cast<size_t>(q) * pair_floats);
                g.pair_batches.emplace_back(first, cnt);
            }
            box_floats = std::max(box_floats, static_cast<size_t>(per) * pair_floats);
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
    const size_t sds_bytes = (sizeof(StationDev) * n_sds + 255) & ~static_cast<size_t>(255);
    hipError_t e = hipMalloc(&p->dev_tables, sds_bytes + sizeof(int4) * n_items);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc (cadence tables)");
    e = hipMalloc(reinterpret_cast<void **>(&p->partials), sizeof(float) * std::max<int64_t>(part, 1));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc (chunk partial sums)");
    if (box_floats) {
        e = hipMalloc(reinterpret_cast<void **>(&p->boxes), sizeof(float2) * box_floats);
        if (e != hipSuccess) return hip_fail(e, "hipMalloc (footprint boxes)");
    }
    char *base = static_cast<char *>(p->dev_tables);
    StationDev *dsds = reinterpret_cast<StationDev *>(base);
    int4 *ditems = reinterpret_cast<int4 *>(base + sds_bytes);
    for (auto &g : p->groups) {
        EPIC_HIP_TRY(hipMemcpy(dsds, g.host_sds.data(), sizeof(StationDev) * g.host_sds.size(),
                               hipMemcpyHostToDevice));
        EPIC_HIP_TRY(hipMemcpy(ditems, g.host_items.data(), sizeof(int4) * g.host_items.size(),
                               hipMemcpyHostToDevice));
        g.batch.sds = dsds;
        g.batch.items = ditems;
        dsds += g.host_sds.size();
        ditems += g.host_items.size();
        g.host_items.clear();
        g.host_items.shrink_to_fit();
    }
    return EPIC_OK;
}

epic_status launch_group(const epic_common *c, const CadencePlan *p, const Group &g, hipStream_t stream)
{
    if (g.path == kPathFft)
        return launch_fused_fft_partials(g.batch, c->n_pol, c->n_time, c->volt_type, g.chunk,
                                         p->partials, p->twiddles[g.n], stream);
    if (g.path == kPathFft128) {
        const int n_blocks = (c->n_time + g.chunk - 1) / g.chunk;
        for (int blk = 0; blk < n_blocks; ++blk)
            for (const auto &pb : g.pair_batches) {
                FusedBatch sub = g.batch;
                sub.items = g.batch.items + pb.first;
                sub.n_items = pb.second;
                epic_status s = launch_grid_box(sub, c->n_pol, c->n_time, c->volt_type, g.chunk, blk,
                                                p->boxes, stream);
                if (s != EPIC_OK) return s;
                s = launch_fused_fft128_partials(sub, c->n_pol, c->n_time, g.chunk, blk, p->boxes,
                                                 p->partials, p->twiddles[g.n], stream);
                if (s != EPIC_OK) return s;
            }
        return EPIC_OK;
    }
    return launch_fused_dft_partials(g.batch, c->n_pol, c->n_time, c->volt_type, c->precision,
                                     g.chunk, p->partials, p->rows[g.n], stream);
}

epic_status enqueue_fused(const epic_common *c, const epic_station *st, const CadencePlan *p,
                          hipStream_t stream)
{
    for (const Group &g : p->groups) {
        epic_status s = launch_group(c, p, g, stream);
        if (s != EPIC_OK) return s;
    }
    const float inv = static_cast<float>(1.0 / static_cast<double>(c->n_time));
    for (const Group &g : p->groups)
        for (int i : g.members) {
            const int n_chunks = (c->n_time + p->chunk[i] - 1) / p->chunk[i];
            epic_status s = launch_reduce_partials(c->n_pol, st[i].nx * st[i].ny, c->n_chan, n_chunks,
                                                   p->partials + p->part_off[i], inv,
                                                   static_cast<float2 *>(st[i].image), stream);
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
                         int device, hipStream_t stream, const std::vector<int> &chunks_override,
                         CadencePlan **out)
{
    const std::string key = call_key(c, st, n, plans, device, stream, chunks_override);
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
    epic_status s = build_plan(c, st, n, plans, device, chunks_override, p);
    if (s != EPIC_OK) {
        free_plan(p);
        return s;
    }
    g_plans[key] = p;
    *out = p;
    return EPIC_OK;
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
    const bool all_fused = p->composed.empty() && !p->groups.empty();
    // first call eager (sets kernel attributes, checks launches); afterwards a
    // captured graph when every station is fused
    if (all_fused && graphs_enabled() && !p->graph_failed && p->runs > 0) {
        if (!p->exec) {
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed);
            epic_status es = e == hipSuccess ? enqueue_fused(c, st, p, stream) : EPIC_ERR_DEVICE;
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
    s = enqueue_fused(c, st, p, stream);
    if (s != EPIC_OK) return s;
    for (int i : p->composed) {
        s = cadence_composed(c, &st[i], plans[i], device, stream);
        if (s != EPIC_OK) return s;
    }
    return EPIC_OK;
}

epic_status tune_cadence(const epic_common *c, const epic_station *st, int n,
                         const PlanHandle *plans, int device, hipStream_t stream)
{
    std::lock_guard<std::mutex> lock(g_mu);
    load_tune_file();
    // the group layout does not depend on the chunk: classify once
    std::vector<Group> groups;
    std::vector<int> composed;
    classify(c, st, n, plans, groups, composed);
    std::vector<int> best(groups.size(), kDefaultChunk);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    EPIC_HIP_TRY(hipEventCreate(&e0));
    EPIC_HIP_TRY(hipEventCreate(&e1));
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        float best_ms = 1e30f;
        for (int chunk : kChunkCandidates) {
            std::vector<int> over(groups.size(), 0);
            over[gi] = chunk;
            CadencePlan *p = nullptr;
            epic_status s = get_or_build(c, st, n, plans, device, stream, over, &p);
            if (s != EPIC_OK) return s;
            // one untimed launch, then the better of two timed ones
            s = launch_group(c, p, p->groups[gi], stream);
            if (s != EPIC_OK) return s;
            float ms = 1e30f;
            for (int rep = 0; rep < 2; ++rep) {
                EPIC_HIP_TRY(hipEventRecord(e0, stream));
                s = launch_group(c, p, p->groups[gi], stream);
                if (s != EPIC_OK) return s;
                EPIC_HIP_TRY(hipEventRecord(e1, stream));
                EPIC_HIP_TRY(hipEventSynchronize(e1));
                float t = 0.f;
                EPIC_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
                ms = std::min(ms, t);
            }
            if (ms < best_ms) {
                best_ms = ms;
                best[gi] = chunk;
            }
            // trial plans can be large (chunk partial sums): free each at once
            EPIC_HIP_TRY(hipStreamSynchronize(stream));
            for (auto it = g_plans.begin(); it != g_plans.end(); ++it)
                if (it->second == p) {
                    free_plan(p);
                    g_plans.erase(it);
                    break;
                }
        }
        g_tuned[class_key(groups[gi].path, groups[gi].n, groups[gi].tiles, c)] = best[gi];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // drop the trial plans; the next image_cadence builds with the tuned chunks
    EPIC_HIP_TRY(hipStreamSynchronize(stream));
    for (auto &kv : g_plans) free_plan(kv.second);
    g_plans.clear();
    ++g_tune_generation;
    save_tune_file();
    return EPIC_OK;
}

void clear_cadence_cache()
{
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto &kv : g_plans) free_plan(kv.second);
    g_plans.clear();
}

}  // namespace epic
