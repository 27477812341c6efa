// Batch engine: many images of uneven size and channel count solved
// concurrently.  A small pool of host threads, each owning one HIP stream,
// takes images from a shared queue (largest first) and runs the per-image
// path on its stream: grid build, bistochastization, solve, slice (forward)
// or splat, adjoint solve, gradient scatter (backward).  The single-image
// kernels are latency-bound below ~10^5 vertices, so images on different
// streams overlap on the device; each thread's convergence polls only block
// its own stream.  The batch is ordered after the caller's stream and the
// caller's stream waits for it, so the calls compose with stream-ordered work.
#include "bs_internal.h"

#include <algorithm>
#include <atomic>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

namespace bs {

namespace {

constexpr int kMaxStreams = 16;

struct StreamPool {
    std::mutex mu;
    int device = -1;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> done;
    hipEvent_t start = nullptr;
};

StreamPool& pool() {
    static StreamPool p;
    return p;
}

// Streams and events of the current device, created once (default priority).
bs_status ensure_pool(int n, int device) {
    StreamPool& p = pool();
    if (p.device != device) {
        if (p.device >= 0) return fail(BS_EUNSUPPORTED, "batch engine bound to another device");
        p.device = device;
        BS_TRY_HIP(hipEventCreateWithFlags(&p.start, hipEventDisableTiming));
    }
    while ((int)p.streams.size() < n) {
        hipStream_t s;
        hipEvent_t e;
        BS_TRY_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        BS_TRY_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        p.streams.push_back(s);
        p.done.push_back(e);
    }
    return BS_OK;
}

size_t item_solve_bytes(const bs_batch_item& it) {
    GridImpl g;
    layout_grid(g, it.H, it.W, it.sigma, nullptr);
    bs_grid tmp;
    std::memcpy(tmp.opaque, &g, sizeof(g));
    return bs_solve_workspace_bytes(&tmp, it.C);
}

bs_status validate_items(const bs_batch_item* items, int n, int n_streams, bool backward) {
    if (!items || n < 1) return fail(BS_EINVAL, "empty batch");
    if (n_streams < 1 || n_streams > kMaxStreams)
        return fail(BS_EINVAL, "stream count must be in 1..16");
    for (int i = 0; i < n; ++i) {
        const bs_batch_item& it = items[i];
        const std::string tag = "item " + std::to_string(i) + ": ";
        if (it.C < 1 || it.C > BS_MAX_CHANNELS) return fail(BS_EINVAL, tag + "bad channel count");
        const size_t need = bs_grid_workspace_bytes(it.H, it.W, &it.sigma);
        if (need == 0) return fail(BS_EINVAL, tag + bs_last_error());
        if (!it.grid_ws || it.grid_ws_bytes < need)
            return fail(BS_EWORKSPACE, tag + "grid workspace needs " + std::to_string(need));
        if (!it.ref || !it.target || !it.conf || !it.y) return fail(BS_EINVAL, tag + "NULL input");
        if (backward && (!it.grad_x || !it.grad_t || !it.grad_c))
            return fail(BS_EINVAL, tag + "NULL gradient buffer");
    }
    return BS_OK;
}

// Runs `work(item, stream, ws)` for every item on n_streams worker threads.
template <class Work>
bs_status run_pool(const bs_batch_item* items, int n, int n_streams, void* ws, size_t ws_bytes,
                   size_t per_stream, void* caller_stream, Work work) {
    int device = 0;
    BS_TRY_HIP(hipGetDevice(&device));
    StreamPool& p = pool();
    std::lock_guard<std::mutex> lock(p.mu);
    bs_status st = ensure_pool(n_streams, device);
    if (st != BS_OK) return st;
    if (((uintptr_t)ws & 255) != 0) return fail(BS_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < per_stream * n_streams)
        return fail(BS_EWORKSPACE,
                    "batch workspace needs " + std::to_string(per_stream * n_streams) + " bytes");
    hipStream_t cs = (hipStream_t)caller_stream;
    BS_TRY_HIP(hipEventRecord(p.start, cs));
    for (int s = 0; s < n_streams; ++s) BS_TRY_HIP(hipStreamWaitEvent(p.streams[s], p.start, 0));

    // largest images first
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (int64_t)items[a].H * items[a].W * items[a].C >
               (int64_t)items[b].H * items[b].W * items[b].C;
    });
    std::atomic<int> next{0};
    std::atomic<int> failed{0};
    std::mutex err_mu;
    bs_status first_err = BS_OK;
    std::string first_msg;
    auto worker = [&](int s) {
        hipSetDevice(device);
        void* mine = (char*)ws + per_stream * s;
        for (;;) {
            if (failed.load()) return;
            const int k = next.fetch_add(1);
            if (k >= n) return;
            const int i = order[k];
            const bs_status r = work(i, p.streams[s], mine, per_stream);
            if (r != BS_OK) {
                std::lock_guard<std::mutex> g(err_mu);
                if (first_err == BS_OK) {
                    first_err = r;
                    first_msg = "item " + std::to_string(i) + ": " + bs_last_error();
                }
                failed.store(1);
                return;
            }
        }
    };
    std::vector<std::thread> threads;
    for (int s = 1; s < n_streams; ++s) threads.emplace_back(worker, s);
    worker(0);
    for (auto& t : threads) t.join();
    for (int s = 0; s < n_streams; ++s) {
        BS_TRY_HIP(hipEventRecord(p.done[s], p.streams[s]));
        BS_TRY_HIP(hipStreamWaitEvent(cs, p.done[s], 0));
    }
    if (first_err != BS_OK) return fail(first_err, first_msg);
    return BS_OK;
}

size_t per_stream_bytes(const bs_batch_item* items, int n) {
    size_t m = 0;
    for (int i = 0; i < n; ++i) m = std::max(m, item_solve_bytes(items[i]));
    return align_up(m, 256);
}

}  // namespace
}  // namespace bs

using namespace bs;

extern "C" size_t bs_batch_workspace_bytes(const bs_batch_item* items, int32_t n,
                                           int32_t n_streams) {
    if (!items || n < 1 || n_streams < 1 || n_streams > kMaxStreams) return 0;
    for (int i = 0; i < n; ++i)
        if (items[i].C < 1 || items[i].C > BS_MAX_CHANNELS ||
            bs_grid_workspace_bytes(items[i].H, items[i].W, &items[i].sigma) == 0)
            return 0;
    return per_stream_bytes(items, n) * n_streams;
}

extern "C" bs_status bs_batch_forward(const bs_batch_item* items, int32_t n,
                                      const bs_solve_params* params,
                                      const bs_bistoch_params* bist, bs_grid* grids,
                                      int32_t n_streams, void* ws, size_t ws_bytes,
                                      void* stream) {
    bs_status st = validate_items(items, n, n_streams, false);
    if (st != BS_OK) return st;
    if (!params || !grids) return fail(BS_EINVAL, "NULL params or grid array");
    const size_t per = per_stream_bytes(items, n);
    return run_pool(items, n, n_streams, ws, ws_bytes, per, stream,
                    [&](int i, hipStream_t s, void* mine, size_t mine_bytes) -> bs_status {
                        const bs_batch_item& it = items[i];
                        bs_status r = bs_build_grid(it.ref, it.H, it.W, &it.sigma, it.grid_ws,
                                                    it.grid_ws_bytes, s, &grids[i]);
                        if (r != BS_OK) return r;
                        r = bs_bistochastize(&grids[i], bist, s);
                        if (r != BS_OK) return r;
                        r = bs_solve(&grids[i], it.target, it.conf, it.C, params, it.y, mine,
                                     mine_bytes, it.stats, s);
                        if (r != BS_OK) return r;
                        if (it.x) r = bs_slice(&grids[i], it.y, it.C, it.x, s);
                        return r;
                    });
}

extern "C" bs_status bs_batch_backward(const bs_batch_item* items, int32_t n,
                                       const bs_grid* grids, const bs_solve_params* params,
                                       int32_t n_streams, void* ws, size_t ws_bytes,
                                       void* stream) {
    bs_status st = validate_items(items, n, n_streams, true);
    if (st != BS_OK) return st;
    if (!params || !grids) return fail(BS_EINVAL, "NULL params or grid array");
    const size_t per = per_stream_bytes(items, n);
    return run_pool(items, n, n_streams, ws, ws_bytes, per, stream,
                    [&](int i, hipStream_t s, void* mine, size_t mine_bytes) -> bs_status {
                        const bs_batch_item& it = items[i];
                        return bs_solve_backward(&grids[i], it.target, it.conf, it.y, it.grad_x,
                                                 it.C, params, it.grad_t, it.grad_c, nullptr,
                                                 mine, mine_bytes, it.stats, s);
                    });
}
