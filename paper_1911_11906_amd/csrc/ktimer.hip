// Optional per-kernel timing: HIP events recorded on the launching stream
// immediately before and after selected kernel launches, accumulated by name.
// Off by default (no events are created); used to time the dominant kernel
// of a run live, beside an external profiler.  Launches queued while their
// stream is being captured into a graph are not timed (the events would
// belong to the graph).  Disabling the timer destroys every pending event.
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>
#include "internal.h"

namespace {
struct Registry {
    std::mutex mu;
    bool enabled = false;
    std::map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> ev;
};
Registry& reg() {
    static Registry r;
    return r;
}
}  // namespace

KScope::KScope(const char* name, hipStream_t s) : name_(name), s_(s) {
    if (!name) return;
    Registry& r = reg();
    std::lock_guard<std::mutex> g(r.mu);
    if (!r.enabled) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s && hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return;
    if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess || hipEventRecord(a_, s_) != hipSuccess) {
        if (a_) (void)hipEventDestroy(a_);
        if (b_) (void)hipEventDestroy(b_);
        a_ = b_ = nullptr;
        return;
    }
    on_ = true;
}

KScope::~KScope() {
    if (!on_) return;
    Registry& r = reg();
    std::lock_guard<std::mutex> g(r.mu);
    if (hipEventRecord(b_, s_) == hipSuccess) {
        r.ev[name_].push_back({a_, b_});
    } else {
        (void)hipEventDestroy(a_);
        (void)hipEventDestroy(b_);
    }
}

extern "C" {

int fl_kernel_timing(int enable) {
    Registry& r = reg();
    std::lock_guard<std::mutex> g(r.mu);
    r.enabled = enable != 0;
    if (!r.enabled) {
        for (auto& kv : r.ev)
            for (auto& p : kv.second) {
                (void)hipEventSynchronize(p.second);
                (void)hipEventDestroy(p.first);
                (void)hipEventDestroy(p.second);
            }
        r.ev.clear();
    }
    return FL_OK;
}

int fl_kernel_time(const char* name, int64_t* count, double* total_ms) {
    if (!name || !count || !total_ms) return FL_EINVAL;
    Registry& r = reg();
    std::vector<std::pair<hipEvent_t, hipEvent_t>> v;
    {
        std::lock_guard<std::mutex> g(r.mu);
        auto it = r.ev.find(name);
        if (it != r.ev.end()) {
            v.swap(it->second);
            r.ev.erase(it);
        }
    }
    double tot = 0.0;
    for (auto& p : v) {
        float ms = 0.f;
        if (hipEventSynchronize(p.second) == hipSuccess && hipEventElapsedTime(&ms, p.first, p.second) == hipSuccess)
            tot += ms;
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    *count = (int64_t)v.size();
    *total_ms = tot;
    return FL_OK;
}

}  // extern "C"
