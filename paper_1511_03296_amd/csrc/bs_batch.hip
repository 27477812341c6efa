// Batch engine: many images of uneven size and channel count solved together.
//
// Per-image set-up runs concurrently: a small pool of host threads, each owning
// one HIP stream, takes images from a shared queue (largest first) and builds
// the grid, bistochastizes it, splats the right-hand side and computes the
// initial state.  The PCG then runs over all images at once: images that share
// a lane width (1 to 4 channels per lane) form a group whose every PCG
// phase is ONE launch, each block working on one image through a block-to-image
// table, each image with its own channel state, partials and stopping rule;
// blocks of stopped images return at once.  Small images, which alone are
// latency-bound, thus share launches with large ones.  Finally each image's
// solution is sliced (forward) or its gradients scattered (backward).
//
// The batch is ordered after the caller's stream and the caller's stream
// waits for it, so the calls compose with stream-ordered work.
#include "bs_solve_impl.h"

#include <algorithm>
#include <atomic>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

namespace bs {

namespace {

constexpr int kMaxStreams = 16;
constexpr int kMaxTilesPerBlock = 64;
// PCG tiles per block of a batched launch, per lane width (index K; 0: the
// default, where fewer, longer-running blocks measured faster: 16 tiles for
// 3- and 4-channel lanes, 8 otherwise).  Set by bs_batch_set_tiles_per_block.
std::atomic<int> g_tiles[5] = {{0}, {0}, {0}, {0}, {0}};
inline int default_tiles_per_block(int K) { return K >= 3 ? 16 : 8; }
inline int tiles_per_block(int K) {
    const int t = g_tiles[K].load(std::memory_order_relaxed);
    return t > 0 ? t : default_tiles_per_block(K);
}

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

// Grid of an item as laid out (sizes only), for workspace sizing.
GridImpl sized_grid(const bs_batch_item& it) {
    GridImpl g;
    std::memset(&g, 0, sizeof(g));
    layout_grid(g, it.H, it.W, it.sigma, nullptr);
    return g;
}

size_t item_solve_bytes(const bs_batch_item& it) {
    const GridImpl g = sized_grid(it);
    SolveWs w;
    return align_up(layout_solve(g, it.C, kRedGridMax, nullptr, w), 256);
}

// Device tables of the batched PCG: images (grouped), block-to-image map and
// active counters.
size_t table_bytes(int n) {
    return align_up((size_t)n * sizeof(PcgImage), 256) +
           align_up((size_t)n * kRedGridMax * sizeof(int32_t), 256) +
           align_up((size_t)n * sizeof(int32_t), 256);
}

size_t batch_bytes(const bs_batch_item* items, int n) {
    size_t total = table_bytes(n);
    for (int i = 0; i < n; ++i) total += item_solve_bytes(items[i]);
    return total;
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
        if (((uintptr_t)it.target | (uintptr_t)it.conf | (uintptr_t)it.y) & 3)
            return fail(BS_EINVAL, tag + "misaligned buffer");
        if (backward && (!it.grad_x || !it.grad_t || !it.grad_c))
            return fail(BS_EINVAL, tag + "NULL gradient buffer");
    }
    return BS_OK;
}

// Runs `work(item, stream)` for every item on n_streams worker threads, each
// with its own stream, ordered after `cs` and joined back into it.
template <class Work>
bs_status for_each_item(const bs_batch_item* items, int n, int n_streams, hipStream_t cs,
                        Work work) {
    int device = 0;
    BS_TRY_HIP(hipGetDevice(&device));
    StreamPool& p = pool();
    std::lock_guard<std::mutex> lock(p.mu);
    bs_status st = ensure_pool(n_streams, device);
    if (st != BS_OK) return st;
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
        if (hipSetDevice(device) != hipSuccess) {
            std::lock_guard<std::mutex> g(err_mu);
            if (first_err == BS_OK) {
                first_err = BS_EDEVICE;
                first_msg = "hipSetDevice failed on a worker thread";
            }
            failed.store(1);
            return;
        }
        for (;;) {
            if (failed.load()) return;
            const int k = next.fetch_add(1);
            if (k >= n) return;
            const int i = order[k];
            const bs_status r = work(i, p.streams[s]);
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

// Per-image solve state of a batch call.
struct Plan {
    SolveWs w;
    float* yw;   // solution (forward) or adjoint solution (backward), stride Cp
};

// Carves every image's solve workspace after the tables (the layout depends
// only on the image size, grid scales and channel count).
bs_status carve(const bs_batch_item* items, int n, void* ws, size_t ws_bytes,
                std::vector<Plan>& plans) {
    if (((uintptr_t)ws & 255) != 0) return fail(BS_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = batch_bytes(items, n);
    if (!ws || ws_bytes < need)
        return fail(BS_EWORKSPACE, "batch workspace needs " + std::to_string(need) + " bytes");
    plans.assign(n, Plan{});
    size_t off = table_bytes(n);
    for (int i = 0; i < n; ++i) {
        const GridImpl g = sized_grid(items[i]);
        off += align_up(layout_solve(g, items[i].C, kRedGridMax, (char*)ws + off, plans[i].w), 256);
        plans[i].yw = nullptr;
    }
    return BS_OK;
}

// The batched PCG over every image: groups by lane width, one launch per
// phase and group; groups run one after another on `cs`.
bs_status batched_pcg(const bs_batch_item* items, int n, const bs_grid* grids,
                      std::vector<Plan>& plans, const bs_solve_params& p, void* ws,
                      hipStream_t cs) {
    // vertex counts decide each image's share of blocks
    std::vector<int32_t> V(n);
    for (int i = 0; i < n; ++i)
        BS_TRY_HIP(hipMemcpyAsync(&V[i], impl(&grids[i])->counts + CNT_V, sizeof(int32_t),
                                  hipMemcpyDeviceToHost, cs));
    BS_TRY_HIP(hipStreamSynchronize(cs));

    char* base = (char*)ws;
    PcgImage* d_imgs = (PcgImage*)base;
    int32_t* d_blk = (int32_t*)(base + align_up((size_t)n * sizeof(PcgImage), 256));
    int32_t* d_act = (int32_t*)((char*)d_blk + align_up((size_t)n * kRedGridMax * sizeof(int32_t), 256));

    struct Group {
        int K, first, count, G, max_cp;
        size_t blk_first;
    };
    std::vector<PcgImage> imgs;
    std::vector<int32_t> blk;
    std::vector<Group> groups;
    for (int K : {4, 3, 2, 1}) {
        Group gr{K, (int)imgs.size(), 0, 0, 0, blk.size()};
        for (int i = 0; i < n; ++i) {
            Plan& pl = plans[i];
            if (pl.w.K != K) continue;
            const GridImpl& g = *impl(&grids[i]);
            const int Lv = pl.w.Cp / K, vpb = kRedBlock / Lv;
            const int64_t tiles = ceil_div(std::max<int32_t>(V[i], 1), vpb);
            int nb = (int)ceil_div(ceil_div(tiles, tiles_per_block(K)), kXcds) * kXcds;
            nb = std::min(std::max(nb, kXcds), kRedGridMax);
            pl.w.nb = nb;
            PcgImage I = make_image(g, pl.w, p.lambda, pl.yw, items[i].stats);
            I.active = d_act + imgs.size();
            I.block0 = gr.G;
            for (int b = 0; b < nb; ++b) blk.push_back(gr.count);
            gr.G += nb;
            gr.max_cp = std::max(gr.max_cp, pl.w.Cp);
            gr.count += 1;
            imgs.push_back(I);
        }
        if (gr.count > 0) groups.push_back(gr);
    }
    // the block map holds each group's local image indices
    BS_TRY_HIP(hipMemcpyAsync(d_imgs, imgs.data(), imgs.size() * sizeof(PcgImage),
                              hipMemcpyHostToDevice, cs));
    BS_TRY_HIP(hipMemcpyAsync(d_blk, blk.data(), blk.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, cs));
    // the host vectors must outlive the copies
    BS_TRY_HIP(hipStreamSynchronize(cs));
    // The groups are independent: each runs on its own library stream and host
    // thread, so the small images' latency-bound launches overlap the large
    // images' bandwidth-bound ones.  With kernel timing enabled they run one
    // after another, so that each timed launch has the device to itself.
    const int ng = (int)groups.size();
    if (ng == 1 || timing_enabled()) {
        for (const Group& gr : groups) {
            const bs_status st =
                run_pcg(gr.K, imgs.data() + gr.first, gr.count, d_imgs + gr.first,
                        d_blk + gr.blk_first, gr.G, gr.max_cp, p, d_act + gr.first, cs);
            if (st != BS_OK) return st;
        }
        return BS_OK;
    }
    int device = 0;
    BS_TRY_HIP(hipGetDevice(&device));
    StreamPool& sp = pool();
    std::lock_guard<std::mutex> lock(sp.mu);
    bs_status st = ensure_pool(ng, device);
    if (st != BS_OK) return st;
    BS_TRY_HIP(hipEventRecord(sp.start, cs));
    for (int g = 0; g < ng; ++g) BS_TRY_HIP(hipStreamWaitEvent(sp.streams[g], sp.start, 0));
    std::vector<bs_status> res(ng, BS_OK);
    std::vector<std::string> msg(ng);
    auto work = [&](int g) {
        if (hipSetDevice(device) != hipSuccess) {
            res[g] = BS_EDEVICE;
            msg[g] = "hipSetDevice failed on a group thread";
            return;
        }
        const Group& gr = groups[g];
        res[g] = run_pcg(gr.K, imgs.data() + gr.first, gr.count, d_imgs + gr.first,
                         d_blk + gr.blk_first, gr.G, gr.max_cp, p, d_act + gr.first,
                         sp.streams[g]);
        if (res[g] != BS_OK) msg[g] = bs_last_error();
    };
    std::vector<std::thread> threads;
    for (int g = 1; g < ng; ++g) threads.emplace_back(work, g);
    work(0);
    for (auto& t : threads) t.join();
    for (int g = 0; g < ng; ++g) {
        BS_TRY_HIP(hipEventRecord(sp.done[g], sp.streams[g]));
        BS_TRY_HIP(hipStreamWaitEvent(cs, sp.done[g], 0));
    }
    for (int g = 0; g < ng; ++g)
        if (res[g] != BS_OK) return fail(res[g], msg[g]);
    return BS_OK;
}

bs_status check_params(const bs_solve_params* p) {
    if (!p) return fail(BS_EINVAL, "NULL params");
    if (!(p->lambda >= 0.0f) || !std::isfinite(p->lambda))
        return fail(BS_EINVAL, "lambda must be finite and >= 0");
    if (p->init != BS_INIT_FLAT && p->init != BS_INIT_HIER) return fail(BS_EINVAL, "unknown init");
    if (p->max_iters < 0 || p->check_every < 0) return fail(BS_EINVAL, "negative iteration count");
    if (!(p->rel_tol >= 0.0)) return fail(BS_EINVAL, "rel_tol must be >= 0");
    if (p->init == BS_INIT_HIER && !(p->init_alpha > 0.0f && std::isfinite(p->init_alpha)))
        return fail(BS_EINVAL, "init_alpha must be positive");
    if (p->init == BS_INIT_HIER && !std::isfinite(p->init_beta))
        return fail(BS_EINVAL, "init_beta must be finite");
    return BS_OK;
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
    return batch_bytes(items, n);
}

extern "C" bs_status bs_batch_forward(const bs_batch_item* items, int32_t n,
                                      const bs_solve_params* params,
                                      const bs_bistoch_params* bist, bs_grid* grids,
                                      int32_t n_streams, void* ws, size_t ws_bytes,
                                      void* stream) {
    bs_status st = validate_items(items, n, n_streams, false);
    if (st != BS_OK) return st;
    st = check_params(params);
    if (st != BS_OK) return st;
    if (!grids) return fail(BS_EINVAL, "NULL grid array");
    const bs_solve_params& p = *params;
    hipStream_t cs = (hipStream_t)stream;
    std::vector<Plan> plans;
    st = carve(items, n, ws, ws_bytes, plans);
    if (st != BS_OK) return st;
    // set-up per image: grid, bistochastization, splat and initial state
    st = for_each_item(items, n, n_streams, cs, [&](int i, hipStream_t s) -> bs_status {
        const bs_batch_item& it = items[i];
        bs_status r = bs_build_grid(it.ref, it.H, it.W, &it.sigma, it.grid_ws, it.grid_ws_bytes, s,
                                    &grids[i]);
        if (r != BS_OK) return r;
        r = bs_bistochastize(&grids[i], bist, s);
        if (r != BS_OK) return r;
        const GridImpl& g = *impl(&grids[i]);
        Plan& pl = plans[i];
        pl.yw = (pl.w.Cp == it.C && ((uintptr_t)it.y & 15) == 0) ? it.y : pl.w.yi;
        return solve_setup(g, pl.w, it.conf, it.target, true, p, pl.yw, s);
    });
    if (st != BS_OK) return st;
    st = batched_pcg(items, n, grids, plans, p, ws, cs);
    if (st != BS_OK) return st;
    for (int i = 0; i < n; ++i) {
        const bs_batch_item& it = items[i];
        const GridImpl& g = *impl(&grids[i]);
        if (plans[i].yw != it.y) {
            st = copy_unpadded(g, plans[i].yw, it.C, plans[i].w.Cp, it.y, cs);
            if (st != BS_OK) return st;
        }
        if (it.x) {
            st = bs_slice(&grids[i], it.y, it.C, it.x, cs);
            if (st != BS_OK) return st;
        }
    }
    return BS_OK;
}

extern "C" bs_status bs_batch_backward(const bs_batch_item* items, int32_t n,
                                       const bs_grid* grids, const bs_solve_params* params,
                                       int32_t n_streams, void* ws, size_t ws_bytes,
                                       void* stream) {
    bs_status st = validate_items(items, n, n_streams, true);
    if (st != BS_OK) return st;
    st = check_params(params);
    if (st != BS_OK) return st;
    if (!grids) return fail(BS_EINVAL, "NULL grid array");
    for (int i = 0; i < n; ++i)
        if (impl(&grids[i])->magic != kGridMagic || !impl(&grids[i])->bistochastized)
            return fail(BS_EINVAL, "item " + std::to_string(i) + ": grid was not built");
    const bs_solve_params& p = *params;
    hipStream_t cs = (hipStream_t)stream;
    std::vector<Plan> plans;
    st = carve(items, n, ws, ws_bytes, plans);
    if (st != BS_OK) return st;
    // set-up per image: splat of dL/dx and initial state of the adjoint solve
    st = for_each_item(items, n, n_streams, cs, [&](int i, hipStream_t s) -> bs_status {
        const bs_batch_item& it = items[i];
        Plan& pl = plans[i];
        pl.yw = pl.w.yi;
        return solve_setup(*impl(&grids[i]), pl.w, it.conf, it.grad_x, false, p, pl.yw, s);
    });
    if (st != BS_OK) return st;
    st = batched_pcg(items, n, grids, plans, p, ws, cs);
    if (st != BS_OK) return st;
    for (int i = 0; i < n; ++i) {
        const bs_batch_item& it = items[i];
        st = grad_scatter_launch(*impl(&grids[i]), plans[i].yw, plans[i].w.Cp, it.y, it.target,
                                 it.conf, it.C, it.grad_t, it.grad_c, cs);
        if (st != BS_OK) return st;
    }
    return BS_OK;
}

// Bytes of one image's part of a low-rank batch: its solve workspace, then
// the reduced system, Gram partials and factors.
static size_t lowrank_item_bytes(const bs_batch_item& it) {
    const GridImpl g = sized_grid(it);
    return item_solve_bytes(it) + align_up(lowrank_extra_bytes(g, it.C, kRedGridMax), 256);
}

extern "C" size_t bs_batch_lowrank_workspace_bytes(const bs_batch_item* items, int32_t n,
                                                   int32_t n_streams) {
    if (validate_items(items, n, n_streams, false) != BS_OK) return 0;
    size_t total = table_bytes(n);
    for (int i = 0; i < n; ++i) total += lowrank_item_bytes(items[i]);
    return total;
}

extern "C" bs_status bs_batch_forward_lowrank(const bs_batch_item* items, int32_t n,
                                              const bs_solve_params* params,
                                              const bs_bistoch_params* bist, bs_grid* grids,
                                              int32_t n_streams, double eps, int32_t* ranks,
                                              void* ws, size_t ws_bytes, void* stream) {
    bs_status st = validate_items(items, n, n_streams, false);
    if (st != BS_OK) return st;
    st = check_params(params);
    if (st != BS_OK) return st;
    if (!grids || !ranks) return fail(BS_EINVAL, "NULL grid or rank array");
    if (!(eps >= 0.0 && eps < 1.0)) return fail(BS_EINVAL, "eps must be in [0, 1)");
    if (((uintptr_t)ws & 255) != 0) return fail(BS_EINVAL, "workspace must be 256-byte aligned");
    const size_t need = bs_batch_lowrank_workspace_bytes(items, n, n_streams);
    if (!ws || ws_bytes < need)
        return fail(BS_EWORKSPACE, "batch workspace needs " + std::to_string(need) + " bytes");
    const bs_solve_params& p = *params;
    hipStream_t cs = (hipStream_t)stream;
    // every image: its full-channel solve workspace, then its reduced system
    std::vector<SolveWs> full(n);
    std::vector<char*> extra(n);
    std::vector<LowRankPlan> lr(n);
    size_t off = table_bytes(n);
    for (int i = 0; i < n; ++i) {
        const GridImpl g = sized_grid(items[i]);
        layout_solve(g, items[i].C, kRedGridMax, (char*)ws + off, full[i]);
        extra[i] = (char*)ws + off + item_solve_bytes(items[i]);
        off += lowrank_item_bytes(items[i]);
    }
    // set-up per image: grid, bistochastization, splat, reduction (the host
    // factorisation synchronises the image's library stream) and the reduced
    // system's initial state
    st = for_each_item(items, n, n_streams, cs, [&](int i, hipStream_t s) -> bs_status {
        const bs_batch_item& it = items[i];
        bs_status r = bs_build_grid(it.ref, it.H, it.W, &it.sigma, it.grid_ws, it.grid_ws_bytes, s,
                                    &grids[i]);
        if (r != BS_OK) return r;
        r = bs_bistochastize(&grids[i], bist, s);
        if (r != BS_OK) return r;
        const GridImpl& g = *impl(&grids[i]);
        r = splat_setup(g, full[i], it.conf, it.target, true, (double)p.lambda, s);
        if (r != BS_OK) return r;
        return lowrank_prepare(g, full[i], extra[i], kRedGridMax, eps, p, s, lr[i]);
    });
    if (st != BS_OK) return st;
    // the reduced systems of rank > 0 through the batched PCG
    std::vector<bs_batch_item> items_c;
    std::vector<bs_grid> grids_c;
    std::vector<Plan> plans_c;
    for (int i = 0; i < n; ++i) {
        ranks[i] = lr[i].t;
        if (lr[i].t == 0) continue;
        items_c.push_back(items[i]);
        grids_c.push_back(grids[i]);
        plans_c.push_back(Plan{lr[i].w, lr[i].w.yi});
    }
    if (!plans_c.empty()) {
        st = batched_pcg(items_c.data(), (int)items_c.size(), grids_c.data(), plans_c, p, ws, cs);
        if (st != BS_OK) return st;
    }
    for (int i = 0; i < n; ++i) {
        const bs_batch_item& it = items[i];
        const GridImpl& g = *impl(&grids[i]);
        st = lowrank_finish(g, lr[i], it.C, it.y, cs);
        if (st != BS_OK) return st;
        if (it.x) {
            st = bs_slice(&grids[i], it.y, it.C, it.x, cs);
            if (st != BS_OK) return st;
        }
    }
    return BS_OK;
}

extern "C" bs_status bs_batch_set_tiles_per_block(int32_t K, int32_t tiles) {
    if (K < 1 || K > 4) return fail(BS_EINVAL, "lane width must be in 1..4");
    if (tiles < 0 || tiles > kMaxTilesPerBlock)
        return fail(BS_EINVAL, "tiles per block must be in 0..64");
    g_tiles[K].store(tiles, std::memory_order_relaxed);
    return BS_OK;
}

extern "C" int32_t bs_batch_tiles_per_block(int32_t K) {
    return (K < 1 || K > 4) ? 0 : tiles_per_block(K);
}

extern "C" int32_t bs_lane_width(int32_t C) {
    return (C < 1 || C > BS_MAX_CHANNELS) ? 0 : lane_width(C);
}
