// Batch engine: many images of uneven size and channel count solved together
// (Section 3: the solver inside a learned pipeline runs forward and backward
// over minibatches).
//
// A plan is made once on the host from the images' sizes, scales and
// channel counts alone: it lays out every image's grid and solve workspace
// (capacities from Vcap, the vertex bound known without building the grid)
// and the device tables of every launch, and uploads the tables.  A run then
// only enqueues kernels on one stream, with no host synchronisation and no
// host threads, so that a forward and a backward run can be captured into
// one HIP graph and replayed:
//   - every stage is ONE launch over all images (multi_launch): grid level 0,
//     the neighbour table, each pyramid level, every bistochastization
//     update, the splat, each level of the initial state, the slice and the
//     gradient scatter;
//   - the PCG runs one launch per phase for each lane width (1 to 4 channels
//     per lane), each image with its own channel state, partials and
//     stopping rule; blocks of stopped images return at once;
//   - launches over the images' vertices are scheduled on the device: right
//     after level 0 a schedule kernel reads every image's vertex count and
//     gives each image a share of the launch's fixed block count in
//     proportion to its work (a multiple of 8, so each image's blocks keep
//     the die-aware tile mapping).  Launches over pixels and grid cells have
//     schedules fixed at plan time.
// Iteration counts are then fixed at enqueue time (max_iters PCG iterations,
// max_iters + 1 bistochastization updates); updates after a stop do nothing.
// With check_every > 0 a run instead polls the stop flags and returns early
// (not capturable).
#include "bs_bist_ops.h"
#include "bs_grid_ops.h"
#include "bs_setup_ops.h"
#include "bs_solve_impl.h"

#include <algorithm>
#include <atomic>
#include <numeric>
#include <vector>

namespace bs {

namespace {

constexpr int kMaxBatch = 4096;
constexpr int kMaxTilesPerBlock = 64;
// PCG tiles per block of a batched launch, per lane width (index K; 0: the
// default, 16 tiles for 3- and 4-channel lanes, 8 otherwise).  Set by
// bs_batch_set_tiles_per_block.
std::atomic<int> g_tiles[5] = {{0}, {0}, {0}, {0}, {0}};
inline int default_tiles_per_block(int K) { return K >= 3 ? 16 : 8; }
inline int tiles_per_block(int K) {
    const int t = g_tiles[K].load(std::memory_order_relaxed);
    return t > 0 ? t : default_tiles_per_block(K);
}

// ---------------------------------------------------------------------------
// Device-side schedules.
// ---------------------------------------------------------------------------

// One schedule: n images share G blocks in proportion to their work
// max(V, 1) * mul; each gets 8 blocks plus a floor share of the other G - 8n
// in units of 8, at most cap, rounded down to a multiple of align once it
// reaches it.  Writes the Sched arrays and, when given, the nb and block0
// fields of PCG image descriptors.
struct SchedDesc {
    const int32_t* const* counts;   // [n] each image's counter array
    const int32_t* mul;             // [n] work per vertex
    const int32_t* cap;             // [n] most blocks (a multiple of 8)
    const int32_t* align;           // [n] block-count multiple (a power of two >= 8)
    int32_t* blk2img;               // [G]
    int32_t* block0;                // [n]
    int32_t* nb;                    // [n]
    PcgImage* imgs0;                // [n] or nullptr
    PcgImage* imgs1;                // [n] or nullptr
    int32_t n, G;
};

constexpr int kSchedThreads = 1024;

// Exclusive block-wide scan of one int per thread (1024 threads).
__device__ inline int block_exclusive_scan(int v, int* total) {
    __shared__ int wsum[kSchedThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    __syncthreads();
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int before = incl - v, tot = 0;
    for (int w = 0; w < kSchedThreads / 64; ++w) {
        if (w < wave) before += wsum[w];
        tot += wsum[w];
    }
    *total = tot;
    return before;
}

__global__ void __launch_bounds__(kSchedThreads) sched_build(const SchedDesc* __restrict__ descs) {
    const SchedDesc& d = descs[blockIdx.x];
    __shared__ int32_t s_nb[kMaxBatch];
    __shared__ int32_t s_b0[kMaxBatch];
    const int t = threadIdx.x, n = d.n;
    double wsum = 0.0;
    for (int i = t; i < n; i += kSchedThreads)
        wsum += (double)max(d.counts[i][CNT_V], 1) * (double)d.mul[i];
    const double total = block_sum<kSchedThreads>(wsum);
    const int units = d.G / 8 - n;
    for (int i = t; i < n; i += kSchedThreads) {
        const double w = (double)max(d.counts[i][CNT_V], 1) * (double)d.mul[i];
        const double share = floor((double)units * (w / total));
        int nb = 8 * (1 + (int)share);
        nb = min(nb, d.cap[i]);
        const int al = d.align[i];
        if (nb >= al) nb -= nb % al;
        s_nb[i] = nb;
    }
    __syncthreads();
    // block0: exclusive prefix of the block counts, a chunk of images per thread
    const int chunk = (n + kSchedThreads - 1) / kSchedThreads;
    const int s = min(t * chunk, n), e = min(s + chunk, n);
    int local = 0;
    for (int i = s; i < e; ++i) local += s_nb[i];
    int used = 0;
    int pre = block_exclusive_scan(local, &used);
    for (int i = s; i < e; ++i) {
        s_b0[i] = pre;
        d.block0[i] = pre;
        d.nb[i] = s_nb[i];
        if (d.imgs0) {
            d.imgs0[i].nb = s_nb[i];
            d.imgs0[i].block0 = pre;
        }
        if (d.imgs1) {
            d.imgs1[i].nb = s_nb[i];
            d.imgs1[i].block0 = pre;
        }
        pre += s_nb[i];
    }
    __syncthreads();
    for (int b = t; b < d.G; b += kSchedThreads) {
        int img = -1;
        if (b < used) {
            int lo = 0, hi = n - 1;   // last image whose block0 <= b
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_b0[mid] <= b) lo = mid;
                else hi = mid - 1;
            }
            img = lo;
        }
        d.blk2img[b] = img;
    }
}

// flag[0] = 1 when every image's bistochastization has stopped.
__global__ void __launch_bounds__(kBlock) all_bist_done(const int32_t* const* __restrict__ counts,
                                                        int n, int32_t* __restrict__ flag) {
    __shared__ int pending;
    if (threadIdx.x == 0) pending = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kBlock)
        if (counts[i][CNT_BIST_DONE] == 0) atomicOr(&pending, 1);
    __syncthreads();
    if (threadIdx.x == 0) flag[0] = pending ? 0 : 1;
}

// ---------------------------------------------------------------------------
// Plan tables: one host byte image, uploaded once.
// ---------------------------------------------------------------------------
struct Blob {
    std::vector<char> host;
    uintptr_t dev = 0;   // device address of byte 0 (0 while sizing)
    template <class T>
    T* put(const T* data, size_t n) {
        const size_t off = align_up(host.size(), 256);
        host.resize(off + n * sizeof(T));
        if (n) std::memcpy(host.data() + off, data, n * sizeof(T));
        return reinterpret_cast<T*>(dev + off);
    }
    template <class T>
    T* put(const std::vector<T>& v) {
        return put(v.data(), v.size());
    }
    template <class T>
    T* reserve(size_t n) {
        const size_t off = align_up(host.size(), 256);
        host.resize(off + n * sizeof(T), 0);
        return reinterpret_cast<T*>(dev + off);
    }
};

// One launch over an image table: the table, its schedule and the grid.
struct ML {
    const void* tab = nullptr;
    Sched s{};
    int G = 0;
};

template <class Op>
bs_status go(const ML& L, hipStream_t st, int id, const char* name, int arg = 0) {
    if (L.G <= 0) return BS_OK;
    BS_LAUNCH(st, id, name, (multi_launch<Op>), dim3(L.G), dim3(Op::kThreads), 0, st,
              (const typename Op::Args*)L.tab, L.s, arg);
    return BS_OK;
}

// A launch whose schedule is fixed at plan time: blocks[i] blocks for table
// entry i, in table order.
// (The block map is padded to `map_reserve` entries, so that a table's size
// can be made independent of which entries have blocks.)
template <class Op>
ML fixed_launch(Blob& b, const std::vector<typename Op::Args>& args, const std::vector<int>& blocks,
                size_t map_reserve = 0) {
    ML L;
    if (args.empty()) return L;
    std::vector<int32_t> b0(args.size()), nb(args.size()), map;
    for (size_t i = 0; i < args.size(); ++i) {
        b0[i] = (int32_t)map.size();
        nb[i] = blocks[i];
        map.insert(map.end(), (size_t)blocks[i], (int32_t)i);
    }
    L.G = (int)map.size();
    if (map.size() < map_reserve) map.resize(map_reserve, -1);
    L.tab = b.put(args);
    L.s = Sched{b.put(map), b.put(b0), b.put(nb)};
    return L;
}

// A launch over every image with a device-computed schedule.
struct DevSched {
    Sched s{};
    int G = 0;
};

// A launch with the same images, in the same order, and schedule as `like`.
template <class Op>
ML same_launch(Blob& b, const std::vector<typename Op::Args>& args, const ML& like) {
    ML L = like;
    L.tab = args.empty() ? nullptr : b.put(args);
    if (args.empty()) L.G = 0;
    return L;
}

template <class Op>
ML sched_launch(Blob& b, const std::vector<typename Op::Args>& args, const DevSched& ds) {
    ML L;
    L.tab = b.put(args);
    L.s = ds.s;
    L.G = ds.G;
    return L;
}

// Level-0 and splat kinds by items per cell (sigma_xy^2): 64, 256, 1024 or
// more pixels.
inline int level0_kind(int sigma_xy) {
    const int items = sigma_xy * sigma_xy;
    return items <= 64 ? 0 : (items <= 256 ? 1 : (items <= 1024 ? 2 : 3));
}

// Vertices an image is expected to have, for sizing launches: the splat
// cells of Vcap, with about 32 colour vertices per 8 x 8 cell (the schedules
// redistribute the blocks by the true counts).
inline int64_t vertex_estimate(const GridImpl& g) {
    const int64_t s2 = (int64_t)g.sg.sigma_xy * g.sg.sigma_xy;
    return std::max<int64_t>(1, std::min<int64_t>(g.vcap, (int64_t)g.P * 32 / s2 + 1));
}

struct Img {
    bs_batch_item it;
    GridImpl g;
    SolveWs w;
    float* yf;       // forward working solution: the caller's y, or w.yi when padded
    int kind0;       // level-0 kind
    int k0;          // first pyramid level of the initial state done in one block
};

struct Group {
    int K = 0, G = 0, max_cp = 0;
    std::vector<int> members;
    std::vector<PcgImage> himg[2];   // host copies (fields read on the host)
    PcgImage* dimg[2] = {nullptr, nullptr};
    int32_t* act = nullptr;
    const int32_t* blk2img = nullptr;
};

}  // namespace

struct PlanImpl {
    uint32_t magic = 0;
    int n = 0;
    bs_solve_params prm[2];          // forward, backward
    bs_bistoch_params bist;
    std::vector<Img> im;
    char* ws = nullptr;
    size_t img_bytes = 0, blob_bytes = 0;
    int Lmax = 0;
    // grid
    ML clear, scan0, nbt, cnt0[4], wr0[4];
    std::vector<ML> cntk, scank, wrk;
    // bistochastization
    ML binit, bstep, bdecide, bfin;
    const int32_t* const* counts_tab = nullptr;
    int32_t* done_flag = nullptr;
    // solve, per direction
    ML spl[2][4], flat[2], hfin[2], small[2];
    std::vector<ML> up[2], down[2];
    ML unpad, slice, scatter;
    // schedules
    const SchedDesc* descs = nullptr;
    int ndesc = 0;
    std::vector<Group> groups;
    // the lane-width groups' PCGs run concurrently: group g > 0 on library
    // stream g, forked from and joined back into the run's stream by events
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    std::vector<hipStream_t> gstream;

    ~PlanImpl() {
        if (fork) (void)hipEventDestroy(fork);
        for (hipEvent_t e : join)
            if (e) (void)hipEventDestroy(e);
    }
};

namespace {

constexpr uint32_t kPlanMagic = 0xB5A7B001u;

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
    if (p->precond != BS_PRECOND_JACOBI)
        return fail(BS_EUNSUPPORTED, "batches use the Jacobi preconditioner");
    return BS_OK;
}

bs_status validate_items(const bs_batch_item* items, int n, bool backward) {
    if (!items || n < 1) return fail(BS_EINVAL, "empty batch");
    if (n > kMaxBatch) return fail(BS_EUNSUPPORTED, "more than 4096 images in a batch");
    for (int i = 0; i < n; ++i) {
        const bs_batch_item& it = items[i];
        const std::string tag = "item " + std::to_string(i) + ": ";
        if (it.C < 1 || it.C > BS_MAX_CHANNELS) return fail(BS_EINVAL, tag + "bad channel count");
        const size_t need = bs_grid_workspace_bytes(it.H, it.W, &it.sigma);
        if (need == 0) return fail(BS_EINVAL, tag + bs_last_error());
        {
            GridImpl g;
            layout_grid(g, it.H, it.W, it.sigma, nullptr);
            if (!solve_fits(g.vcap, it.C))
                return fail(BS_EUNSUPPORTED, tag + "grid too large for 32-bit vector offsets");
        }
        if (it.grid_ws && it.grid_ws_bytes < need)
            return fail(BS_EWORKSPACE, tag + "grid workspace needs " + std::to_string(need));
        if (((uintptr_t)it.grid_ws & 255) != 0)
            return fail(BS_EINVAL, tag + "grid workspace must be 256-byte aligned");
        if (!it.ref || !it.target || !it.conf || !it.y) return fail(BS_EINVAL, tag + "NULL input");
        if (((uintptr_t)it.ref | (uintptr_t)it.target | (uintptr_t)it.conf | (uintptr_t)it.y |
             (uintptr_t)it.x) & 3)
            return fail(BS_EINVAL, tag + "misaligned buffer");
        if (backward && (!it.grad_x || !it.grad_t || !it.grad_c))
            return fail(BS_EINVAL, tag + "NULL gradient buffer");
        if (backward && (((uintptr_t)it.grad_x | (uintptr_t)it.grad_t | (uintptr_t)it.grad_c) & 3))
            return fail(BS_EINVAL, tag + "misaligned gradient buffer");
    }
    return BS_OK;
}

// Block cap and alignment of an image's PCG partials: the most blocks whose
// partials the consumers sum in registers when the estimated need fits under
// it, else kRedGridMax blocks with the partials reduced by pcg_reduce.
void pcg_caps(int Cp, int64_t need, int& cap, int& align, bool& sep) {
    int q = 64;
    while (q > 8 && q * 3 * Cp > kRedBlock) q >>= 1;
    const int fit_cap = 16 * q;
    if (q * 3 * Cp <= kRedBlock && need <= fit_cap && pcg_partials_fit(Cp, fit_cap)) {
        cap = fit_cap;
        align = q;
        sep = false;
    } else {
        cap = kRedGridMax;
        align = 8;
        sep = true;
    }
}

// Fills the plan's tables for workspace base `ws` (0 while sizing).
void build_tables(PlanImpl& P, uintptr_t ws, Blob& b) {
    const int n = P.n;
    b.host.clear();
    b.dev = 0;
    // per-image regions first, so that their addresses do not depend on the
    // size of the tables that follow them
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        Img& I = P.im[i];
        const bs_batch_item& it = I.it;
        void* gbase = it.grid_ws;
        if (!gbase) {
            GridImpl tmp;
            gbase = ws ? (void*)(ws + off) : nullptr;
            off += align_up(layout_grid(tmp, it.H, it.W, it.sigma, nullptr), 256);
        }
        layout_grid(I.g, it.H, it.W, it.sigma, gbase);   // sizes only while sizing
        void* sbase = ws ? (void*)(ws + off) : nullptr;
        off += align_up(layout_solve(I.g, it.C, kRedGridMax, sbase, I.w), 256);
        I.yf = (I.w.Cp == it.C && ((uintptr_t)it.y & 15) == 0) ? it.y : I.w.yi;
        I.kind0 = level0_kind(it.sigma.sigma_xy);
        I.k0 = small_pyr_level(I.g, I.w.Cp);
    }
    P.img_bytes = align_up(off, 256);
    b.dev = ws ? ws + P.img_bytes : 0;
    P.Lmax = 0;
    for (const Img& I : P.im) P.Lmax = std::max(P.Lmax, I.g.levels);

    // counters of every image
    std::vector<const int32_t*> counts(n);
    for (int i = 0; i < n; ++i) counts[i] = P.im[i].g.counts;
    P.counts_tab = b.put(counts);
    P.done_flag = b.reserve<int32_t>(64);

    // ---- schedules over the images' vertices (computed on the device) ----
    std::vector<SchedDesc> descs;
    auto add_desc = [&](const std::vector<int>& members, const std::vector<int32_t>& mul,
                        const std::vector<int32_t>& cap, const std::vector<int32_t>& align,
                        int G, int G_reserve, PcgImage* i0, PcgImage* i1) -> DevSched {
        const int m = (int)members.size();
        std::vector<const int32_t*> cnt(m);
        for (int j = 0; j < m; ++j) cnt[j] = P.im[members[j]].g.counts;
        SchedDesc d;
        d.counts = b.put(cnt);
        d.mul = b.put(mul);
        d.cap = b.put(cap);
        d.align = b.put(align);
        d.blk2img = b.reserve<int32_t>(G_reserve);
        d.block0 = b.reserve<int32_t>(m);
        d.nb = b.reserve<int32_t>(m);
        d.imgs0 = i0;
        d.imgs1 = i1;
        d.n = m;
        d.G = G;
        descs.push_back(d);
        DevSched ds;
        ds.s = Sched{d.blk2img, d.block0, d.nb};
        ds.G = G;
        return ds;
    };

    std::vector<int> all(n);
    std::iota(all.begin(), all.end(), 0);
    DevSched vs;
    {
        int64_t vsum = 0;
        for (const Img& I : P.im) vsum += vertex_estimate(I.g);
        const int64_t G = std::min<int64_t>(std::max<int64_t>(8 * (int64_t)n,
                                                              ceil_div(vsum, kRedBlock * 8) / 8 * 8),
                                            std::max<int64_t>(8 * (int64_t)n, 8192));
        vs = add_desc(all, std::vector<int32_t>(n, 1), std::vector<int32_t>(n, kRedGridMax),
                      std::vector<int32_t>(n, 8), (int)G, (int)G, nullptr, nullptr);
    }

    // ---- PCG groups by lane width ----
    P.groups.clear();
    for (int K : {4, 3, 2, 1}) {
        Group gr;
        gr.K = K;
        for (int i = 0; i < n; ++i)
            if (P.im[i].w.K == K) gr.members.push_back(i);
        if (gr.members.empty()) continue;
        const int m = (int)gr.members.size();
        gr.act = b.reserve<int32_t>(m);
        std::vector<int32_t> mul(m), cap(m), align(m);
        int64_t Gsum = 0;
        for (int j = 0; j < m; ++j) {
            Img& I = P.im[gr.members[j]];
            const int Lv = I.w.Cp / K;
            const int64_t tiles = ceil_div(vertex_estimate(I.g) * Lv, kRedBlock);
            const int64_t need = ceil_div(ceil_div(tiles, tiles_per_block(K)), 8) * 8;
            bool sep = false;
            pcg_caps(I.w.Cp, need, cap[j], align[j], sep);
            mul[j] = Lv;
            Gsum += std::max<int64_t>(8, std::min<int64_t>(need, cap[j]));
            gr.max_cp = std::max(gr.max_cp, I.w.Cp);
            for (int dir = 0; dir < 2; ++dir) {
                float* yw = dir == 0 ? I.yf : I.w.yi;
                PcgImage pi = make_image(I.g, I.w, P.prm[dir].lambda, yw, I.it.stats);
                pi.sums[0] = sep ? I.w.sums[0] : nullptr;
                pi.sums[1] = sep ? I.w.sums[1] : nullptr;
                pi.active = gr.act + j;
                pi.nb = 8;        // set by the schedule
                pi.block0 = 0;
                gr.himg[dir].push_back(pi);
            }
        }
        gr.G = (int)std::min<int64_t>(Gsum, (int64_t)m * kRedGridMax);
        gr.G = std::max(gr.G, 8 * m);
        gr.dimg[0] = b.put(gr.himg[0]);
        gr.dimg[1] = b.put(gr.himg[1]);
        // (the map is reserved for the largest G, so the workspace size does
        // not depend on the tiles per block in effect)
        const DevSched ds = add_desc(gr.members, mul, cap, align, gr.G, m * kRedGridMax,
                                     gr.dimg[0], gr.dimg[1]);
        gr.blk2img = ds.s.blk2img;
        P.groups.push_back(std::move(gr));
    }
    P.descs = b.put(descs);
    P.ndesc = (int)descs.size();

    // ---- grid level 0 ----
    {
        std::vector<ClearCounts::Args> a(n);
        for (int i = 0; i < n; ++i) a[i] = {P.im[i].g.counts};
        P.clear = fixed_launch<ClearCounts>(b, a, std::vector<int>(n, 1));
    }
    std::vector<int> kind_members[4];
    for (int i = 0; i < n; ++i) kind_members[P.im[i].kind0].push_back(i);
    auto pixel_source = [](const Img& I) {
        return PixelSource{I.it.ref, I.g.H, I.g.W, I.g.P, I.g.sg.sigma_xy, I.g.sg.sigma_l,
                           I.g.sg.sigma_uv, I.g.lv[0].ncx};
    };
    // the cell schedule of each kind, shared by the level-0 passes and the splat
    std::vector<int> cells0[4];
    for (int k = 0; k < 4; ++k)
        for (int i : kind_members[k]) cells0[k].push_back(P.im[i].g.lv[0].ncx * P.im[i].g.lv[0].ncy);
#define BS_LEVEL0(KIND, B, CAP)                                                                 \
    {                                                                                           \
        std::vector<typename LevelCount<B, CAP, PixelSource>::Args> ca;                         \
        std::vector<typename LevelWrite<B, CAP, PixelSource>::Args> wa;                         \
        for (int i : kind_members[KIND]) {                                                      \
            const PixelSource ps = pixel_source(P.im[i]);                                       \
            ca.push_back(level_count_args<B, CAP>(ps, P.im[i].g));                              \
            wa.push_back(level_write_args<B, CAP>(ps, P.im[i].g, 0));                           \
        }                                                                                       \
        P.cnt0[KIND] = fixed_launch<LevelCount<B, CAP, PixelSource>>(b, ca, cells0[KIND]);     \
        P.wr0[KIND] = same_launch<LevelWrite<B, CAP, PixelSource>>(b, wa, P.cnt0[KIND]);       \
    }
    BS_LEVEL0(0, 64, 64)
    BS_LEVEL0(1, 256, 256)
    BS_LEVEL0(2, 256, 1024)
    BS_LEVEL0(3, 256, 2048)
#undef BS_LEVEL0
    {
        std::vector<LevelScan::Args> a(n);
        for (int i = 0; i < n; ++i) a[i] = level_scan_args(P.im[i].g, 0);
        P.scan0 = fixed_launch<LevelScan>(b, a, std::vector<int>(n, 1));
    }
    {
        std::vector<NeighbourTable::Args> a(n);
        for (int i = 0; i < n; ++i) a[i] = neighbour_args(P.im[i].g);
        P.nbt = sched_launch<NeighbourTable>(b, a, vs);
    }
    // ---- pyramid levels k >= 1 ----
    P.cntk.assign(P.Lmax, ML{});
    P.scank.assign(P.Lmax, ML{});
    P.wrk.assign(P.Lmax, ML{});
    for (int k = 1; k < P.Lmax; ++k) {
        using LC = LevelCount<128, 1024, VertexSource>;
        using LW = LevelWrite<128, 1024, VertexSource>;
        std::vector<LC::Args> ca;
        std::vector<LW::Args> wa;
        std::vector<LevelScan::Args> sa;
        std::vector<int> cells;
        for (int i = 0; i < n; ++i) {
            const GridImpl& g = P.im[i].g;
            if (k >= g.levels) continue;
            const Level& C = g.lv[k - 1];
            const VertexSource vsrc{C.key, C.cell_vbase, g.counts, C.ncx, C.ncy, g.lv[k].ncx, k};
            ca.push_back(level_count_args<128, 1024>(vsrc, g));
            wa.push_back(level_write_args<128, 1024>(vsrc, g, k));
            sa.push_back(level_scan_args(g, k));
            cells.push_back(g.lv[k].ncx * g.lv[k].ncy);
        }
        P.cntk[k] = fixed_launch<LC>(b, ca, cells);
        P.wrk[k] = same_launch<LW>(b, wa, P.cntk[k]);
        P.scank[k] = fixed_launch<LevelScan>(b, sa, std::vector<int>(sa.size(), 1));
    }
    // ---- bistochastization ----
    {
        std::vector<BistInit::Args> ia(n);
        std::vector<BistStep::Args> sa(n);
        std::vector<BistDecide::Args> da(n);
        std::vector<BistFinalize::Args> fa(n);
        for (int i = 0; i < n; ++i) {
            const GridImpl& g = P.im[i].g;
            ia[i] = bist_init_args(g);
            sa[i] = bist_step_args(g, P.bist);
            da[i] = bist_decide_args(g, 0, vs.s.nb + i);
            fa[i] = bist_finalize_args(g);
        }
        P.binit = sched_launch<BistInit>(b, ia, vs);
        P.bstep = sched_launch<BistStep>(b, sa, vs);
        P.bdecide = fixed_launch<BistDecide>(b, da, std::vector<int>(n, 1));
        P.bfin = sched_launch<BistFinalize>(b, fa, vs);
    }
    // ---- splat and initial state, per direction ----
    for (int dir = 0; dir < 2; ++dir) {
        const bool wgt = dir == 0;
#define BS_SPLAT(KIND, B, CAP)                                                                  \
    {                                                                                           \
        if (wgt) {                                                                              \
            std::vector<typename SplatCells<B, CAP, true>::Args> a;                             \
            for (int i : kind_members[KIND])                                                    \
                a.push_back(splat_cells_args<B, CAP, true>(P.im[i].g, P.im[i].w, P.im[i].it.conf, \
                                                           P.im[i].it.target,                   \
                                                           (double)P.prm[0].lambda));           \
            P.spl[dir][KIND] = same_launch<SplatCells<B, CAP, true>>(b, a, P.cnt0[KIND]);      \
        } else {                                                                                \
            std::vector<typename SplatCells<B, CAP, false>::Args> a;                            \
            for (int i : kind_members[KIND])                                                    \
                a.push_back(splat_cells_args<B, CAP, false>(P.im[i].g, P.im[i].w,               \
                                                            P.im[i].it.conf, P.im[i].it.grad_x, \
                                                            (double)P.prm[1].lambda));          \
            P.spl[dir][KIND] = same_launch<SplatCells<B, CAP, false>>(b, a, P.cnt0[KIND]);     \
        }                                                                                       \
    }
        BS_SPLAT(0, 64, 64)
        BS_SPLAT(1, 256, 256)
        BS_SPLAT(2, 256, 1024)
#undef BS_SPLAT
        // kind 3: per vertex, over the kind's images only (a fixed schedule)
        if (!kind_members[3].empty()) {
            std::vector<int> blocks;
            for (int i : kind_members[3]) blocks.push_back(grid_blocks(ceil_div(P.im[i].g.vcap, kBlock)));
            if (wgt) {
                std::vector<SplatVertex<true>::Args> a;
                for (int i : kind_members[3])
                    a.push_back(splat_vertex_args<true>(P.im[i].g, P.im[i].w, P.im[i].it.conf,
                                                        P.im[i].it.target, (double)P.prm[0].lambda));
                P.spl[dir][3] = fixed_launch<SplatVertex<true>>(b, a, blocks);
            } else {
                std::vector<SplatVertex<false>::Args> a;
                for (int i : kind_members[3])
                    a.push_back(splat_vertex_args<false>(P.im[i].g, P.im[i].w, P.im[i].it.conf,
                                                         P.im[i].it.grad_x, (double)P.prm[1].lambda));
                P.spl[dir][3] = fixed_launch<SplatVertex<false>>(b, a, blocks);
            }
        }
        const bs_solve_params& p = P.prm[dir];
        std::vector<FlatInit::Args> fa(n);
        std::vector<HierFinal::Args> ha(n);
        for (int i = 0; i < n; ++i) {
            float* y = dir == 0 ? P.im[i].yf : P.im[i].w.yi;
            fa[i] = flat_init_args(P.im[i].g, P.im[i].w, y);
            ha[i] = hier_final_args(P.im[i].g, P.im[i].w, y);
        }
        P.flat[dir] = sched_launch<FlatInit>(b, fa, vs);
        P.hfin[dir] = sched_launch<HierFinal>(b, ha, vs);
        P.up[dir].assign(P.Lmax, ML{});
        P.down[dir].assign(P.Lmax, ML{});
        for (int k = 1; k < P.Lmax; ++k) {
            std::vector<PyrUp::Args> ua;
            std::vector<PyrDown::Args> da;
            std::vector<int> blocks;
            for (int i = 0; i < n; ++i) {
                const Img& I = P.im[i];
                if (k >= I.k0) continue;
                ua.push_back(pyr_up_args(I.g, I.w, k));
                da.push_back(pyr_down_args(I.g, I.w, p, k));
                blocks.push_back(grid_blocks(ceil_div(I.g.lv[k].cap * (I.w.Cp + 1), kBlock)));
            }
            P.up[dir][k] = fixed_launch<PyrUp>(b, ua, blocks);
            P.down[dir][k] = same_launch<PyrDown>(b, da, P.up[dir][k]);
        }
        std::vector<PyrSmall::Args> sa;
        for (int i = 0; i < n; ++i) {
            const Img& I = P.im[i];
            if (I.k0 < I.g.levels) sa.push_back(pyr_small_args(I.g, I.w, p, I.k0));
        }
        P.small[dir] = fixed_launch<PyrSmall>(b, sa, std::vector<int>(sa.size(), 1));
    }
    // ---- output ----
    {
        std::vector<Unpad::Args> ua;
        std::vector<int> ub;
        std::vector<Slice::Args> sa;
        std::vector<int> sb;
        std::vector<GradScatter::Args> ga;
        // every image has an entry (no blocks where there is nothing to do),
        // so the tables' size does not depend on the output pointers
        for (int i = 0; i < n; ++i) {
            const Img& I = P.im[i];
            const bs_batch_item& it = I.it;
            ua.push_back(Unpad::Args{I.yf, I.g.counts, it.y, I.w.Cp, it.C});
            ub.push_back(I.yf != it.y ? grid_blocks(ceil_div(I.g.vcap * it.C, kBlock)) : 0);
            sa.push_back(Slice::Args{I.g.lv[0].item_parent, it.y, it.x, it.C, I.g.P});
            sb.push_back(it.x ? grid_blocks(ceil_div(I.g.P, kBlock)) : 0);
            ga.push_back(GradScatter::Args{I.g.lv[0].item_parent, I.w.yi, it.y, it.target, it.conf,
                                           it.grad_t, it.grad_c, I.w.Cp, it.C, I.g.P});
        }
        size_t ur = 0, sr = 0;
        for (int i = 0; i < n; ++i) {
            ur += grid_blocks(ceil_div(P.im[i].g.vcap * P.im[i].it.C, kBlock));
            sr += grid_blocks(ceil_div(P.im[i].g.P, kBlock));
        }
        P.unpad = fixed_launch<Unpad>(b, ua, ub, ur);
        P.slice = fixed_launch<Slice>(b, sa, sb, sr);
        std::vector<int> gb;
        for (int i = 0; i < n; ++i) gb.push_back(grid_blocks(ceil_div(P.im[i].g.P, kBlock)));
        P.scatter = fixed_launch<GradScatter>(b, ga, gb);
    }
    P.blob_bytes = align_up(b.host.size(), 256);
}

// ---------------------------------------------------------------------------
// Runs.
// ---------------------------------------------------------------------------
// The kernel instances of the batch's launches.
using LC0 = LevelCount<64, 64, PixelSource>;
using LC1 = LevelCount<256, 256, PixelSource>;
using LC2 = LevelCount<256, 1024, PixelSource>;
using LC3 = LevelCount<256, 2048, PixelSource>;
using LW0 = LevelWrite<64, 64, PixelSource>;
using LW1 = LevelWrite<256, 256, PixelSource>;
using LW2 = LevelWrite<256, 1024, PixelSource>;
using LW3 = LevelWrite<256, 2048, PixelSource>;
using LCk = LevelCount<128, 1024, VertexSource>;
using LWk = LevelWrite<128, 1024, VertexSource>;
using SCw0 = SplatCells<64, 64, true>;
using SCw1 = SplatCells<256, 256, true>;
using SCw2 = SplatCells<256, 1024, true>;
using SCu0 = SplatCells<64, 64, false>;
using SCu1 = SplatCells<256, 256, false>;
using SCu2 = SplatCells<256, 1024, false>;

bs_status run_sched(const PlanImpl& P, hipStream_t s) {
    BS_LAUNCH(s, K_INIT, "sched_build", sched_build, dim3(P.ndesc), dim3(kSchedThreads), 0, s,
              P.descs);
    return BS_OK;
}

bs_status run_grids(const PlanImpl& P, hipStream_t s) {
    bs_status st = go<ClearCounts>(P.clear, s, K_BIST_OTHER, "clear_counts");
    if (st != BS_OK) return st;
#define BS_GO(OP, L, ID, NAME)                  \
    do {                                        \
        st = go<OP>(L, s, ID, NAME);            \
        if (st != BS_OK) return st;             \
    } while (0)
    BS_GO(LC0, P.cnt0[0], K_LEVEL_COUNT, "level_count");
    BS_GO(LC1, P.cnt0[1], K_LEVEL_COUNT, "level_count");
    BS_GO(LC2, P.cnt0[2], K_LEVEL_COUNT, "level_count");
    BS_GO(LC3, P.cnt0[3], K_LEVEL_COUNT, "level_count");
    BS_GO(LevelScan, P.scan0, K_LEVEL_SCAN, "level_scan");
    BS_GO(LW0, P.wr0[0], K_LEVEL_WRITE, "level_write");
    BS_GO(LW1, P.wr0[1], K_LEVEL_WRITE, "level_write");
    BS_GO(LW2, P.wr0[2], K_LEVEL_WRITE, "level_write");
    BS_GO(LW3, P.wr0[3], K_LEVEL_WRITE, "level_write");
    st = run_sched(P, s);
    if (st != BS_OK) return st;
    BS_GO(NeighbourTable, P.nbt, K_NEIGHBOURS, "neighbour_table");
    for (int k = 1; k < P.Lmax; ++k) {
        BS_GO(LCk, P.cntk[k], K_LEVEL_COUNT, "level_count");
        BS_GO(LevelScan, P.scank[k], K_LEVEL_SCAN, "level_scan");
        BS_GO(LWk, P.wrk[k], K_LEVEL_WRITE, "level_write");
    }
    return BS_OK;
}

bs_status run_bist(const PlanImpl& P, hipStream_t s) {
    bs_status st;
    BS_GO(BistInit, P.binit, K_BIST_OTHER, "bist_init");
    int last = 0;
    {
        // updates after every image's fixed point return at once: the polls lag
        StopPoller poller(P.done_flag, 1, s, false);
        for (int step = 0; step <= P.bist.max_iters; ++step) {
            st = go<BistStep>(P.bstep, s, K_BIST_STEP, "bist_step", step);
            if (st != BS_OK) return st;
            last = step;
            const int ce = P.bist.check_every;
            if (ce > 0 && (step + 1) % ce == 0 && step < P.bist.max_iters) {
                BS_LAUNCH(s, K_BIST_OTHER, "all_bist_done", all_bist_done, dim3(1), dim3(kBlock), 0,
                          s, P.counts_tab, P.n, P.done_flag);
                bool done = false;
                st = poller.check(done);
                if (st != BS_OK) return st;
                if (done) break;
            }
        }
    }
    st = go<BistDecide>(P.bdecide, s, K_BIST_OTHER, "bist_decide", last);
    if (st != BS_OK) return st;
    BS_GO(BistFinalize, P.bfin, K_BIST_OTHER, "bist_finalize");
    return BS_OK;
}

bs_status run_setup(const PlanImpl& P, int dir, hipStream_t s) {
    bs_status st;
    if (dir == 0) {
        BS_GO(SCw0, P.spl[0][0], K_SPLAT, "splat_cells");
        BS_GO(SCw1, P.spl[0][1], K_SPLAT, "splat_cells");
        BS_GO(SCw2, P.spl[0][2], K_SPLAT, "splat_cells");
        BS_GO(SplatVertex<true>, P.spl[0][3], K_SPLAT, "splat");
    } else {
        BS_GO(SCu0, P.spl[1][0], K_SPLAT, "splat_cells");
        BS_GO(SCu1, P.spl[1][1], K_SPLAT, "splat_cells");
        BS_GO(SCu2, P.spl[1][2], K_SPLAT, "splat_cells");
        BS_GO(SplatVertex<false>, P.spl[1][3], K_SPLAT, "splat");
    }
    if (P.prm[dir].init == BS_INIT_FLAT) {
        BS_GO(FlatInit, P.flat[dir], K_INIT, "flat_init");
        return BS_OK;
    }
    for (int k = 1; k < P.Lmax; ++k) BS_GO(PyrUp, P.up[dir][k], K_INIT, "pyr_up");
    BS_GO(PyrSmall, P.small[dir], K_INIT, "pyr_small");
    for (int k = P.Lmax - 1; k >= 1; --k) BS_GO(PyrDown, P.down[dir][k], K_INIT, "pyr_down");
    BS_GO(HierFinal, P.hfin[dir], K_INIT, "hier_final");
    return BS_OK;
}

// The PCG of every lane-width group.  The groups are independent: the
// smaller groups' launches (latency-bound for one- and two-channel images)
// run on their own streams beside the largest group's.  With convergence
// polls or kernel timing they run one after another on `s` (a poll
// synchronises its stream; a timed launch should have the device to itself).
bs_status run_pcg_groups(const PlanImpl& P, int dir, hipStream_t s) {
    const int ng = (int)P.groups.size();
    const bool concurrent = ng > 1 && P.prm[dir].check_every == 0 && !timing_enabled() &&
                            (int)P.gstream.size() >= ng && P.fork;
    auto group = [&](int g, hipStream_t st) {
        const Group& gr = P.groups[g];
        return run_pcg(gr.K, gr.himg[dir].data(), (int)gr.members.size(), gr.dimg[dir],
                       gr.blk2img, gr.G, gr.max_cp, P.prm[dir], gr.act, st);
    };
    if (!concurrent) {
        for (int g = 0; g < ng; ++g) {
            const bs_status st = group(g, s);
            if (st != BS_OK) return st;
        }
        return BS_OK;
    }
    BS_TRY_HIP(hipEventRecord(P.fork, s));
    for (int g = 1; g < ng; ++g) {
        BS_TRY_HIP(hipStreamWaitEvent(P.gstream[g], P.fork, 0));
        const bs_status st = group(g, P.gstream[g]);
        if (st != BS_OK) return st;
        BS_TRY_HIP(hipEventRecord(P.join[g], P.gstream[g]));
    }
    bs_status st = group(0, s);
    if (st != BS_OK) return st;
    for (int g = 1; g < ng; ++g) BS_TRY_HIP(hipStreamWaitEvent(s, P.join[g], 0));
    return BS_OK;
}

bs_status run_forward(const PlanImpl& P, hipStream_t s) {
    bs_status st = run_grids(P, s);
    if (st != BS_OK) return st;
    st = run_bist(P, s);
    if (st != BS_OK) return st;
    st = run_setup(P, 0, s);
    if (st != BS_OK) return st;
    st = run_pcg_groups(P, 0, s);
    if (st != BS_OK) return st;
    BS_GO(Unpad, P.unpad, K_INIT, "unpad");
    BS_GO(Slice, P.slice, K_SLICE, "slice");
    return BS_OK;
}

bs_status run_backward(const PlanImpl& P, hipStream_t s) {
    bs_status st = run_sched(P, s);
    if (st != BS_OK) return st;
    st = run_setup(P, 1, s);
    if (st != BS_OK) return st;
    st = run_pcg_groups(P, 1, s);
    if (st != BS_OK) return st;
    BS_GO(GradScatter, P.scatter, K_GRAD_SCATTER, "grad_scatter");
    return BS_OK;
}
#undef BS_GO

// Makes a plan over `items` in `ws` (uploading its tables on `stream`, which
// is synchronised).  `bwd` may equal `fwd`.
bs_status make_plan(const bs_batch_item* items, int n, const bs_solve_params* fwd,
                    const bs_solve_params* bwd, const bs_bistoch_params* bist, bool backward,
                    void* ws, size_t ws_bytes, hipStream_t stream, PlanImpl& P) {
    bs_status st = validate_items(items, n, backward);
    if (st != BS_OK) return st;
    st = check_params(fwd);
    if (st != BS_OK) return st;
    st = check_params(bwd);
    if (st != BS_OK) return st;
    bs_bistoch_params bp{200, 0, 1e-10};
    if (bist) bp = *bist;
    if (bp.max_iters < 0 || bp.check_every < 0 || !(bp.tol >= 0.0))
        return fail(BS_EINVAL, "bistochastization parameters out of range");
    if (!ws || ((uintptr_t)ws & 255) != 0)
        return fail(BS_EINVAL, "workspace must be a 256-byte aligned device pointer");
    P.n = n;
    P.prm[0] = *fwd;
    P.prm[1] = *bwd;
    P.bist = bp;
    P.im.assign(n, Img{});
    for (int i = 0; i < n; ++i) P.im[i].it = items[i];
    Blob b;
    build_tables(P, 0, b);   // sizes
    const size_t need = P.img_bytes + P.blob_bytes;
    if (ws_bytes < need)
        return fail(BS_EWORKSPACE, "batch workspace needs " + std::to_string(need) + " bytes");
    build_tables(P, (uintptr_t)ws, b);
    P.ws = (char*)ws;
    BS_TRY_HIP(hipMemcpyAsync((char*)ws + P.img_bytes, b.host.data(), b.host.size(),
                              hipMemcpyHostToDevice, stream));
    BS_TRY_HIP(hipStreamSynchronize(stream));
    const int ng = (int)P.groups.size();
    if (ng > 1) {
        BS_TRY_HIP(hipEventCreateWithFlags(&P.fork, hipEventDisableTiming));
        P.join.assign(ng, nullptr);
        P.gstream.assign(ng, nullptr);
        for (int g = 1; g < ng; ++g) {
            BS_TRY_HIP(hipEventCreateWithFlags(&P.join[g], hipEventDisableTiming));
            st = library_stream(g, &P.gstream[g]);
            if (st != BS_OK) return st;
        }
    }
    P.magic = kPlanMagic;
    return BS_OK;
}

size_t plan_bytes(const bs_batch_item* items, int n) {
    if (!items || n < 1 || n > kMaxBatch) return 0;
    for (int i = 0; i < n; ++i)
        if (items[i].C < 1 || items[i].C > BS_MAX_CHANNELS ||
            bs_grid_workspace_bytes(items[i].H, items[i].W, &items[i].sigma) == 0)
            return 0;
    PlanImpl P;
    P.n = n;
    bs_solve_params p{};
    p.init = BS_INIT_HIER;
    p.init_alpha = 4.0f;
    P.prm[0] = P.prm[1] = p;
    P.bist = bs_bistoch_params{200, 0, 1e-10};
    P.im.assign(n, Img{});
    for (int i = 0; i < n; ++i) P.im[i].it = items[i];
    Blob b;
    build_tables(P, 0, b);
    return P.img_bytes + P.blob_bytes;
}

void grid_handle(const PlanImpl& P, int i, bs_grid* out) {
    GridImpl g = P.im[i].g;
    g.bistochastized = 1;
    g.pyramid_built = 1;
    std::memset(out->opaque, 0, sizeof(out->opaque));
    std::memcpy(out->opaque, &g, sizeof(g));
}

// ---------------------------------------------------------------------------
// The low-rank batch: set-up through a plan, then the reduced systems through
// the PCG over an image table laid out from the vertex counts read back (the
// host factorisation synchronises anyway).
// ---------------------------------------------------------------------------
struct LowPlan {
    SolveWs w;
    float* yw;
};

bs_status lowrank_pcg(const std::vector<const GridImpl*>& grids, std::vector<LowPlan>& plans,
                      const std::vector<bs_chan_stats*>& stats, const bs_solve_params& p,
                      char* tables, hipStream_t cs) {
    const int n = (int)grids.size();
    std::vector<int32_t> V(n);
    for (int i = 0; i < n; ++i)
        BS_TRY_HIP(hipMemcpyAsync(&V[i], grids[i]->counts + CNT_V, sizeof(int32_t),
                                  hipMemcpyDeviceToHost, cs));
    BS_TRY_HIP(hipStreamSynchronize(cs));
    PcgImage* d_imgs = (PcgImage*)tables;
    int32_t* d_blk = (int32_t*)(tables + align_up((size_t)n * sizeof(PcgImage), 256));
    int32_t* d_act =
        (int32_t*)((char*)d_blk + align_up((size_t)n * kRedGridMax * sizeof(int32_t), 256));
    struct G {
        int K, first, count, G, max_cp;
        size_t blk_first;
    };
    std::vector<PcgImage> imgs;
    std::vector<int32_t> blk;
    std::vector<G> groups;
    for (int K : {4, 3, 2, 1}) {
        G gr{K, (int)imgs.size(), 0, 0, 0, blk.size()};
        for (int i = 0; i < n; ++i) {
            LowPlan& pl = plans[i];
            if (pl.w.K != K) continue;
            const int Lv = pl.w.Cp / K, vpb = kRedBlock / Lv;
            const int64_t tiles = ceil_div(std::max<int32_t>(V[i], 1), vpb);
            int nb = (int)ceil_div(ceil_div(tiles, tiles_per_block(K)), kXcds) * kXcds;
            nb = std::min(std::max(nb, kXcds), kRedGridMax);
            pl.w.nb = nb;
            PcgImage I = make_image(*grids[i], pl.w, p.lambda, pl.yw, stats[i]);
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
    BS_TRY_HIP(hipMemcpyAsync(d_imgs, imgs.data(), imgs.size() * sizeof(PcgImage),
                              hipMemcpyHostToDevice, cs));
    BS_TRY_HIP(hipMemcpyAsync(d_blk, blk.data(), blk.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, cs));
    // the host vectors must outlive the copies
    BS_TRY_HIP(hipStreamSynchronize(cs));
    for (const G& gr : groups) {
        const bs_status st = run_pcg(gr.K, imgs.data() + gr.first, gr.count, d_imgs + gr.first,
                                     d_blk + gr.blk_first, gr.G, gr.max_cp, p, d_act + gr.first, cs);
        if (st != BS_OK) return st;
    }
    return BS_OK;
}

size_t lowrank_table_bytes(int n) {
    return align_up((size_t)n * sizeof(PcgImage), 256) +
           align_up((size_t)n * kRedGridMax * sizeof(int32_t), 256) +
           align_up((size_t)n * sizeof(int32_t), 256);
}

}  // namespace
}  // namespace bs

using namespace bs;

struct bs_batch_plan {
    PlanImpl impl;
};

extern "C" size_t bs_batch_plan_workspace_bytes(const bs_batch_item* items, int32_t n) {
    return plan_bytes(items, n);
}

extern "C" bs_status bs_batch_plan_create(const bs_batch_item* items, int32_t n,
                                          const bs_solve_params* fwd, const bs_solve_params* bwd,
                                          const bs_bistoch_params* bist, void* ws, size_t ws_bytes,
                                          void* stream, bs_batch_plan** out) {
    if (!out) return fail(BS_EINVAL, "NULL plan pointer");
    *out = nullptr;
    bs_batch_plan* pl = new (std::nothrow) bs_batch_plan;
    if (!pl) return fail(BS_EINVAL, "out of host memory");
    const bs_status st = make_plan(items, n, fwd, bwd ? bwd : fwd, bist, bwd != nullptr, ws,
                                   ws_bytes, (hipStream_t)stream, pl->impl);
    if (st != BS_OK) {
        delete pl;
        return st;
    }
    *out = pl;
    return BS_OK;
}

static bs_status check_plan(const bs_batch_plan* plan) {
    if (!plan || plan->impl.magic != kPlanMagic) return fail(BS_EINVAL, "not a batch plan");
    return BS_OK;
}

extern "C" bs_status bs_batch_run_forward(bs_batch_plan* plan, void* stream) {
    bs_status st = check_plan(plan);
    if (st != BS_OK) return st;
    return run_forward(plan->impl, (hipStream_t)stream);
}

extern "C" bs_status bs_batch_run_backward(bs_batch_plan* plan, void* stream) {
    bs_status st = check_plan(plan);
    if (st != BS_OK) return st;
    for (int i = 0; i < plan->impl.n; ++i) {
        const bs_batch_item& it = plan->impl.im[i].it;
        if (!it.grad_x || !it.grad_t || !it.grad_c)
            return fail(BS_EINVAL, "plan was made without gradient buffers");
    }
    return run_backward(plan->impl, (hipStream_t)stream);
}

extern "C" bs_status bs_batch_plan_grid(const bs_batch_plan* plan, int32_t i, bs_grid* out) {
    bs_status st = check_plan(plan);
    if (st != BS_OK) return st;
    if (i < 0 || i >= plan->impl.n || !out) return fail(BS_EINVAL, "bad image index");
    grid_handle(plan->impl, i, out);
    return BS_OK;
}

extern "C" void bs_batch_plan_destroy(bs_batch_plan* plan) {
    if (plan && plan->impl.magic == kPlanMagic) {
        plan->impl.magic = 0;
        delete plan;
    }
}

// ---- the synchronous batch calls, on a plan made per call ----

extern "C" size_t bs_batch_workspace_bytes(const bs_batch_item* items, int32_t n,
                                           int32_t n_streams) {
    if (n_streams < 1 || n_streams > 16) return 0;
    return plan_bytes(items, n);
}

extern "C" bs_status bs_batch_forward(const bs_batch_item* items, int32_t n,
                                      const bs_solve_params* params,
                                      const bs_bistoch_params* bist, bs_grid* grids,
                                      int32_t n_streams, void* ws, size_t ws_bytes,
                                      void* stream) {
    if (n_streams < 1 || n_streams > 16) return fail(BS_EINVAL, "stream count must be in 1..16");
    if (!grids) return fail(BS_EINVAL, "NULL grid array");
    if (items)
        for (int i = 0; i < n; ++i)
            if (!items[i].grid_ws)
                return fail(BS_EINVAL, "item " + std::to_string(i) + ": NULL grid workspace");
    PlanImpl P;
    hipStream_t s = (hipStream_t)stream;
    bs_status st = make_plan(items, n, params, params, bist, false, ws, ws_bytes, s, P);
    if (st != BS_OK) return st;
    st = run_forward(P, s);
    if (st != BS_OK) return st;
    for (int i = 0; i < n; ++i) grid_handle(P, i, &grids[i]);
    return BS_OK;
}

extern "C" bs_status bs_batch_backward(const bs_batch_item* items, int32_t n,
                                       const bs_grid* grids, const bs_solve_params* params,
                                       int32_t n_streams, void* ws, size_t ws_bytes,
                                       void* stream) {
    if (n_streams < 1 || n_streams > 16) return fail(BS_EINVAL, "stream count must be in 1..16");
    if (!grids) return fail(BS_EINVAL, "NULL grid array");
    bs_status st = validate_items(items, n, true);
    if (st != BS_OK) return st;
    for (int i = 0; i < n; ++i) {
        const GridImpl& g = *impl(&grids[i]);
        if (g.magic != kGridMagic || !g.bistochastized)
            return fail(BS_EINVAL, "item " + std::to_string(i) + ": grid was not built");
        if (g.ws != items[i].grid_ws)
            return fail(BS_EINVAL, "item " + std::to_string(i) + ": grid is not in its grid_ws");
    }
    PlanImpl P;
    hipStream_t s = (hipStream_t)stream;
    st = make_plan(items, n, params, params, nullptr, true, ws, ws_bytes, s, P);
    if (st != BS_OK) return st;
    return run_backward(P, s);
}

// Bytes of one image's part of a low-rank batch: its reduced system, Gram
// partials and factors (after the plan's own workspace).
static size_t lowrank_item_bytes(const bs_batch_item& it) {
    GridImpl g;
    std::memset(&g, 0, sizeof(g));
    layout_grid(g, it.H, it.W, it.sigma, nullptr);
    return align_up(lowrank_extra_bytes(g, it.C, kRedGridMax), 256);
}

extern "C" size_t bs_batch_lowrank_workspace_bytes(const bs_batch_item* items, int32_t n,
                                                   int32_t n_streams) {
    if (n_streams < 1 || n_streams > 16) return 0;
    const size_t base = plan_bytes(items, n);
    if (base == 0) return 0;
    size_t total = align_up(base, 256) + lowrank_table_bytes(n);
    for (int i = 0; i < n; ++i) total += lowrank_item_bytes(items[i]);
    return total;
}

extern "C" bs_status bs_batch_forward_lowrank(const bs_batch_item* items, int32_t n,
                                              const bs_solve_params* params,
                                              const bs_bistoch_params* bist, bs_grid* grids,
                                              int32_t n_streams, double eps, int32_t* ranks,
                                              void* ws, size_t ws_bytes, void* stream) {
    if (n_streams < 1 || n_streams > 16) return fail(BS_EINVAL, "stream count must be in 1..16");
    if (!grids || !ranks) return fail(BS_EINVAL, "NULL grid or rank array");
    if (!(eps >= 0.0 && eps < 1.0)) return fail(BS_EINVAL, "eps must be in [0, 1)");
    if (items)
        for (int i = 0; i < n; ++i)
            if (!items[i].grid_ws)
                return fail(BS_EINVAL, "item " + std::to_string(i) + ": NULL grid workspace");
    const size_t need = bs_batch_lowrank_workspace_bytes(items, n, n_streams);
    if (need == 0) {
        bs_status st = validate_items(items, n, false);
        return st != BS_OK ? st : check_params(params);
    }
    if (!ws || ws_bytes < need)
        return fail(BS_EWORKSPACE, "batch workspace needs " + std::to_string(need) + " bytes");
    hipStream_t s = (hipStream_t)stream;
    PlanImpl P;
    const size_t base = plan_bytes(items, n);
    bs_status st = make_plan(items, n, params, params, bist, false, ws, base, s, P);
    if (st != BS_OK) return st;
    const bs_solve_params& p = *params;
    // grid, pyramid, bistochastization and the splat of every image
    st = run_grids(P, s);
    if (st != BS_OK) return st;
    st = run_bist(P, s);
    if (st != BS_OK) return st;
    for (int i = 0; i < n; ++i) {
        const Img& I = P.im[i];
        st = splat_setup(I.g, I.w, I.it.conf, I.it.target, true, (double)p.lambda, s);
        if (st != BS_OK) return st;
    }
    // the reductions (each factorisation synchronises the stream)
    char* tables = (char*)ws + align_up(base, 256);
    char* extra = tables + lowrank_table_bytes(n);
    std::vector<LowRankPlan> lr(n);
    for (int i = 0; i < n; ++i) {
        const Img& I = P.im[i];
        st = lowrank_prepare(I.g, I.w, extra, kRedGridMax, eps, p, s, lr[i]);
        if (st != BS_OK) return fail(st, "item " + std::to_string(i) + ": " + bs_last_error());
        extra += lowrank_item_bytes(items[i]);
    }
    // the reduced systems of rank > 0 through the batched PCG
    std::vector<const GridImpl*> gsub;
    std::vector<LowPlan> psub;
    std::vector<bs_chan_stats*> ssub;
    for (int i = 0; i < n; ++i) {
        ranks[i] = lr[i].t;
        if (lr[i].t == 0) continue;
        gsub.push_back(&P.im[i].g);
        psub.push_back(LowPlan{lr[i].w, lr[i].w.yi});
        ssub.push_back(items[i].stats);
    }
    if (!gsub.empty()) {
        st = lowrank_pcg(gsub, psub, ssub, p, tables, s);
        if (st != BS_OK) return st;
    }
    for (int i = 0; i < n; ++i) {
        const bs_batch_item& it = items[i];
        const GridImpl& g = P.im[i].g;
        st = lowrank_finish(g, lr[i], it.C, it.y, s);
        if (st != BS_OK) return st;
        if (it.x) {
            grid_handle(P, i, &grids[i]);
            st = bs_slice(&grids[i], it.y, it.C, it.x, s);
            if (st != BS_OK) return st;
        }
    }
    for (int i = 0; i < n; ++i) grid_handle(P, i, &grids[i]);
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
