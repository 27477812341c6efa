// Optional kernel timing for benchmarks: when enabled, every launch of the
// library's kernels carries a start and a stop hipEvent of its own
// (hipExtLaunchKernelGGL records them at the kernel's start and end), and
// bs_timing_read sums the elapsed times per kernel.  Disabled by default; when
// disabled the hook costs one relaxed atomic load.
#include "bs_internal.h"

#include <atomic>
#include <mutex>
#include <vector>

namespace bs {

static const char* const kKernelNames[K_COUNT] = {
    "level_count", "level_scan", "level_write", "neighbour_table", "bist_step", "bist_other",
    "splat", "init", "pcg_start", "pcg_matvec", "pcg_update", "pcg_reduce", "slice",
    "grad_scatter", "dt_rows", "dt_cols", "dt_other"};

namespace {
struct Pending {
    int id;
    hipEvent_t start, stop;
};
struct Timing {
    std::mutex mu;
    std::atomic<bool> on{false};
    std::vector<hipEvent_t> pool;
    std::vector<Pending> pending;
    double total_ms[K_COUNT] = {};
    int64_t launches[K_COUNT] = {};
};
Timing& T() {
    static Timing t;
    return t;
}
hipEvent_t take_event(Timing& t) {
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
bs_status drain(Timing& t) {
    for (const Pending& p : t.pending) {
        BS_TRY_HIP(hipEventSynchronize(p.stop));
        float ms = 0.0f;
        BS_TRY_HIP(hipEventElapsedTime(&ms, p.start, p.stop));
        t.total_ms[p.id] += ms;
        t.launches[p.id] += 1;
        t.pool.push_back(p.start);
        t.pool.push_back(p.stop);
    }
    t.pending.clear();
    return BS_OK;
}
}  // namespace

bool timing_enabled() { return T().on.load(std::memory_order_relaxed); }

void timing_pair(int id, hipEvent_t* start, hipEvent_t* stop) {
    *start = *stop = nullptr;
    Timing& t = T();
    if (!t.on.load(std::memory_order_relaxed)) return;
    std::lock_guard<std::mutex> g(t.mu);
    hipEvent_t a = take_event(t), b = take_event(t);
    if (!a || !b) {
        if (a) t.pool.push_back(a);
        if (b) t.pool.push_back(b);
        return;
    }
    t.pending.push_back({id, a, b});
    *start = a;
    *stop = b;
}

}  // namespace bs

using namespace bs;

extern "C" bs_status bs_timing_enable(int32_t on) {
    T().on.store(on != 0);
    return BS_OK;
}

extern "C" bs_status bs_timing_reset(void) {
    Timing& t = T();
    std::lock_guard<std::mutex> g(t.mu);
    bs_status st = drain(t);
    for (int i = 0; i < K_COUNT; ++i) {
        t.total_ms[i] = 0.0;
        t.launches[i] = 0;
    }
    return st;
}

extern "C" bs_status bs_timing_read(const char* kernel, double* total_ms, int64_t* launches) {
    if (!kernel || !total_ms || !launches) return fail(BS_EINVAL, "NULL pointer argument");
    Timing& t = T();
    std::lock_guard<std::mutex> g(t.mu);
    bs_status st = drain(t);
    if (st != BS_OK) return st;
    for (int i = 0; i < K_COUNT; ++i) {
        if (std::strcmp(kernel, kKernelNames[i]) == 0) {
            *total_ms = t.total_ms[i];
            *launches = t.launches[i];
            return BS_OK;
        }
    }
    return fail(BS_EINVAL, std::string("unknown kernel name ") + kernel);
}
