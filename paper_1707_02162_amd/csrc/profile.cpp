// Launch timing of the batched GEMM kernels: when enabled, every product
// launch is bracketed by HIP events recorded on the launch's own stream, so
// a benchmark can divide the algorithmic work of a launch by its measured
// duration.  Diagnostics only: no effect on results.
#include <mutex>
#include <vector>

#include "redo_internal.h"

namespace redo {
namespace {
struct Prof {
    std::mutex mu;
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> open;
    std::vector<hipEvent_t> pool;
    double ms = 0.0;
    long long launches = 0;
};
Prof& prof() {
    static Prof p;
    return p;
}
hipEvent_t take_event(Prof& p) {
    if (!p.pool.empty()) {
        hipEvent_t e = p.pool.back();
        p.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

bool profiling_on() { return prof().on; }

void profile_begin(hipStream_t st, void** token) {
    Prof& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    hipEvent_t a = take_event(p), b = take_event(p);
    if (!a || !b) {
        *token = nullptr;
        return;
    }
    (void)hipEventRecord(a, st);
    p.open.emplace_back(a, b);
    *token = reinterpret_cast<void*>(p.open.size());
}

void profile_end(hipStream_t st, void* token) {
    if (!token) return;
    Prof& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    const size_t i = reinterpret_cast<size_t>(token) - 1;
    if (i < p.open.size()) (void)hipEventRecord(p.open[i].second, st);
}

}  // namespace redo

extern "C" {

redo_status redo_profile_enable(int32_t enable) {
    redo::Prof& p = redo::prof();
    std::lock_guard<std::mutex> g(p.mu);
    p.on = enable != 0;
    return REDO_OK;
}

redo_status redo_profile_read(double* gemm_ms, int64_t* gemm_launches, int32_t reset) {
    redo::Prof& p = redo::prof();
    std::lock_guard<std::mutex> g(p.mu);
    for (auto& ev : p.open) {
        if (hipEventSynchronize(ev.second) != hipSuccess) return redo::fail(REDO_ERR_HIP, "event synchronize failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev.first, ev.second) == hipSuccess) p.ms += ms;
        p.launches += 1;
        p.pool.push_back(ev.first);
        p.pool.push_back(ev.second);
    }
    p.open.clear();
    if (gemm_ms) *gemm_ms = p.ms;
    if (gemm_launches) *gemm_launches = p.launches;
    if (reset) {
        p.ms = 0.0;
        p.launches = 0;
    }
    return REDO_OK;
}

}  // extern "C"
