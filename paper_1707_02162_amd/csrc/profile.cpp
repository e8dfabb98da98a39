// Launch timing of the batched GEMM kernels (kind 0), of the structure-aware
// step kernel (kind 1) and of the re-projection GEMMs (kind 2): when enabled, every such launch is bracketed by HIP
// events recorded on the launch's own stream, so a benchmark can divide the
// algorithmic work of a launch by its measured duration.  Diagnostics only: no
// effect on results.
#include <mutex>
#include <vector>

#include "redo_internal.h"

namespace redo {
namespace {
struct Prof {
    std::mutex mu;
    bool on = false;
    struct Open {
        hipEvent_t a, b;
        int kind;
    };
    std::vector<Open> open;
    std::vector<hipEvent_t> pool;
    double ms[PROFILE_KINDS] = {};
    long long launches[PROFILE_KINDS] = {};
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

void profile_begin(hipStream_t st, void** token, int kind) {
    Prof& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    hipEvent_t a = take_event(p), b = take_event(p);
    if (!a || !b) {
        *token = nullptr;
        return;
    }
    (void)hipEventRecord(a, st);
    p.open.push_back({a, b, kind});
    *token = reinterpret_cast<void*>(p.open.size());
}

void profile_end(hipStream_t st, void* token) {
    if (!token) return;
    Prof& p = prof();
    std::lock_guard<std::mutex> g(p.mu);
    const size_t i = reinterpret_cast<size_t>(token) - 1;
    if (i < p.open.size()) (void)hipEventRecord(p.open[i].b, st);
}

}  // namespace redo

extern "C" {

redo_status redo_profile_enable(int32_t enable) {
    redo::Prof& p = redo::prof();
    std::lock_guard<std::mutex> g(p.mu);
    p.on = enable != 0;
    return REDO_OK;
}

redo_status redo_profile_read_kind(int32_t kind, double* ms, int64_t* launches, int32_t reset) {
    if (kind < 0 || kind >= redo::PROFILE_KINDS) return redo::fail(REDO_ERR_ARG, "unknown launch kind");
    redo::Prof& p = redo::prof();
    std::lock_guard<std::mutex> g(p.mu);
    for (auto& ev : p.open) {
        if (hipEventSynchronize(ev.b) != hipSuccess) return redo::fail(REDO_ERR_HIP, "event synchronize failed");
        float t = 0.f;
        if (hipEventElapsedTime(&t, ev.a, ev.b) == hipSuccess) p.ms[ev.kind] += t;
        p.launches[ev.kind] += 1;
        p.pool.push_back(ev.a);
        p.pool.push_back(ev.b);
    }
    p.open.clear();
    if (ms) *ms = p.ms[kind];
    if (launches) *launches = p.launches[kind];
    if (reset) {
        p.ms[kind] = 0.0;
        p.launches[kind] = 0;
    }
    return REDO_OK;
}

redo_status redo_profile_read(double* gemm_ms, int64_t* gemm_launches, int32_t reset) {
    return redo_profile_read_kind(0, gemm_ms, gemm_launches, reset);
}

}  // extern "C"
