// timing.cpp -- optional per-kernel timing with HIP events on each launch's
// own stream (see epic_timing_enable in epic.h).
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"

namespace epic {

namespace {
struct Rec {
    const char *name;
    hipEvent_t start, stop;
};
std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Rec> g_recs;
}  // namespace

bool timing_on() { return g_on.load(std::memory_order_relaxed); }

KernelTimer::KernelTimer(const char *name, hipStream_t stream) : name_(name), stream_(stream)
{
    if (!timing_on()) return;
    if (hipEventCreate(&start_) != hipSuccess || hipEventCreate(&stop_) != hipSuccess) return;
    active_ = hipEventRecord(start_, stream_) == hipSuccess;
}

KernelTimer::~KernelTimer()
{
    if (!active_) return;
    if (hipEventRecord(stop_, stream_) != hipSuccess) return;
    std::lock_guard<std::mutex> lock(g_mu);
    g_recs.push_back(Rec{name_, start_, stop_});
}

}  // namespace epic

using namespace epic;

extern "C" {

void epic_timing_enable(int32_t enable) { g_on.store(enable != 0); }

void epic_timing_reset(void)
{
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto &r : g_recs) {
        (void)hipEventSynchronize(r.stop);
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    g_recs.clear();
}

int32_t epic_timing_report(char *buf, int32_t len)
{
    std::lock_guard<std::mutex> lock(g_mu);
    std::map<std::string, std::pair<long, double>> agg;
    for (auto &r : g_recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.stop) == hipSuccess && hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
            auto &a = agg[r.name];
            a.first += 1;
            a.second += ms;
        }
    }
    std::string out;
    for (auto &kv : agg)
        out += kv.first + " " + std::to_string(kv.second.first) + " " + std::to_string(kv.second.second) + "\n";
    if (buf && len > 0) {
        const size_t n = std::min(out.size(), static_cast<size_t>(len - 1));
        out.copy(buf, n);
        buf[n] = '\0';
    }
    return static_cast<int32_t>(agg.size());
}

}  // extern "C"
