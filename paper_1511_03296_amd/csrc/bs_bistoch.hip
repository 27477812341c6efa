// Bistochastization of the grid blur (supplement Algorithm 1, Eq. equiv), in
// float64:  n <- sqrt(n o m / (B n)),  n = 1 initially, with B = 10 I + N.
//
// Launch s reads n_s from ping-pong buffer s % 2, writes n_{s+1} to the other
// buffer and publishes per-block maxima of the invariant residual
// max_v |n_v (B n_s)_v - m_v| / m_v.  Launch s+1 first reduces those maxima
// (the order of a max does not matter) and decides whether n_s is the answer:
// stop when the residual is <= tol or s >= max_iters.  Once stopped, later
// launches return at once, so the host may enqueue them without waiting.
#include "bs_bist_ops.h"

#include <mutex>
#include <vector>

namespace bs {

namespace {
constexpr int kSideStreams = 8;
struct SideStreams {
    std::mutex mu;
    std::vector<std::vector<hipStream_t>> per_device;
};
SideStreams& sides() {
    static SideStreams s;
    return s;
}
}  // namespace

bs_status side_stream(hipStream_t s, hipStream_t* out) {
    int dev = 0;
    BS_TRY_HIP(hipGetDevice(&dev));
    SideStreams& ss = sides();
    std::lock_guard<std::mutex> lock(ss.mu);
    if ((int)ss.per_device.size() <= dev) ss.per_device.resize(dev + 1);
    std::vector<hipStream_t>& v = ss.per_device[dev];
    if (v.empty()) {
        for (int i = 0; i < kSideStreams; ++i) {
            hipStream_t h;
            BS_TRY_HIP(hipStreamCreateWithFlags(&h, hipStreamNonBlocking));
            v.push_back(h);
        }
    }
    const uintptr_t key = (uintptr_t)s;
    *out = v[(key >> 8 ^ key >> 4) % kSideStreams];
    return BS_OK;
}

bs_status library_stream(int index, hipStream_t* out) {
    hipStream_t any;
    const bs_status st = side_stream(nullptr, &any);   // creates the device's streams once
    if (st != BS_OK) return st;
    int dev = 0;
    BS_TRY_HIP(hipGetDevice(&dev));
    SideStreams& ss = sides();
    std::lock_guard<std::mutex> lock(ss.mu);
    *out = ss.per_device[dev][index % kSideStreams];
    return BS_OK;
}

}  // namespace bs

using namespace bs;

extern "C" bs_status bs_bistochastize(bs_grid* grid, const bs_bistoch_params* params,
                                      void* stream) {
    if (!grid || impl(grid)->magic != kGridMagic) return fail(BS_EINVAL, "grid was not built");
    bs_bistoch_params p{200, 8, 1e-10};
    if (params) p = *params;
    if (p.max_iters < 0 || p.check_every < 0 || !(p.tol >= 0.0))
        return fail(BS_EINVAL, "bistochastization parameters out of range");
    GridImpl& g = *impl(grid);
    hipStream_t s = (hipStream_t)stream;
    // The pyramid levels k >= 1 and the bistochastization both read level 0
    // only: the pyramid is built on a side stream meanwhile and joined below.
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    if (!g.pyramid_built) {
        BS_TRY_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        BS_TRY_HIP(hipEventCreateWithFlags(&join, hipEventDisableTiming));
        bs_status st = side_stream(s, &side);
        if (st != BS_OK) return st;
        BS_TRY_HIP(hipEventRecord(fork, s));
        BS_TRY_HIP(hipStreamWaitEvent(side, fork, 0));
        st = build_pyramid(g, side);
        if (st != BS_OK) return st;
        BS_TRY_HIP(hipEventRecord(join, side));
        g.pyramid_built = 1;
    }
    const int blocks = grid_blocks(ceil_div(g.vcap, kBlock));
    BS_LAUNCH(s, K_BIST_OTHER, "bist_init", one_launch<BistInit>, dim3(blocks), dim3(kBlock), 0, s,
              bist_init_args(g), 0);
    const int G = red_grid(g.vcap);
    const BistStep::Args sa = bist_step_args(g, p);
    int last = 0;
    {
        // updates after the fixed point return at once: the polls lag behind
        StopPoller poller(g.counts + CNT_BIST_DONE, 1, s, false);
        for (int step = 0; step <= p.max_iters; ++step) {
            BS_LAUNCH(s, K_BIST_STEP, "bist_step", one_launch<BistStep>, dim3(G), dim3(kRedBlock),
                      0, s, sa, step);
            last = step;
            if (p.check_every > 0 && (step + 1) % p.check_every == 0 && step < p.max_iters) {
                bool done = false;
                const bs_status st = poller.check(done);
                if (st != BS_OK) return st;
                if (done) break;
            }
        }
    }
    BS_LAUNCH(s, K_BIST_OTHER, "bist_decide", one_launch<BistDecide>, dim3(1), dim3(kRedBlock), 0,
              s, bist_decide_args(g, G, nullptr), last);
    BS_LAUNCH(s, K_BIST_OTHER, "bist_finalize", one_launch<BistFinalize>, dim3(blocks),
              dim3(kBlock), 0, s, bist_finalize_args(g), 0);
    if (join) {
        BS_TRY_HIP(hipStreamWaitEvent(s, join, 0));
        BS_TRY_HIP(hipEventDestroy(fork));
        BS_TRY_HIP(hipEventDestroy(join));
    }
    g.bistochastized = 1;
    return BS_OK;
}
