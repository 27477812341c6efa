// Internal definitions of the bilateral-solver HIP library: the grid layout
// carved from the caller's workspace, launch helpers, error reporting and the
// device-side reduction helpers shared by the kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <unordered_map>

#include "bsolve.h"

namespace bs {

// ---------------------------------------------------------------------------
// Error reporting (thread-local text behind bs_last_error).
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
bs_status fail(bs_status st, const std::string& msg);
bs_status check_hip(hipError_t e, const char* what);

#define BS_TRY_HIP(expr)                                        \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) return ::bs::check_hip(e_, #expr); \
    } while (0)

// Checks the launch that was just enqueued.
#define BS_CHECK_LAUNCH(name)                                        \
    do {                                                             \
        hipError_t e_ = hipGetLastError();                           \
        if (e_ != hipSuccess) return ::bs::check_hip(e_, name);      \
    } while (0)

// ---------------------------------------------------------------------------
// Stop-flag polls.
// ---------------------------------------------------------------------------
// Convergence polls that do not idle the device.  check() enqueues a copy of
// the device's stop flags into pinned host memory behind the launches made so
// far, then waits only for the copy kLag check points back: the device always
// has that many check periods of launches queued while the host reads flags.
// The iterative kernels return at once after convergence, so the lag costs a
// few microseconds per launch after it instead of a stream drain at every
// check point.  The buffers and events belong to the calling thread (one set
// per device, a few bytes per image, kept until the process ends: freeing
// them from thread-exit destructors could run after the runtime's own
// teardown); the destructor waits for the last copy, so that the next call
// can reuse them.  A lag of one check point measured best: 2 % on the stereo
// image and 15 % on the 64x48 one over a lag of two, whose extra launches
// after convergence cost more than the host's wait saves.
class StopPoller {
  public:
    static constexpr int kLag = 1;

    // all_zero: stop once every flag reads 0 (per-image active counts); else
    // once flag 0 reads nonzero (a done flag)
    StopPoller(const int32_t* flags, int n, hipStream_t s, bool all_zero = true)
        : flags_(flags), n_(n), s_(s), all_zero_(all_zero) {}
    StopPoller(const StopPoller&) = delete;
    StopPoller& operator=(const StopPoller&) = delete;
    ~StopPoller() {
        if (count_ > 0) (void)hipEventSynchronize(pool_->ev[(count_ - 1) % kSlots]);
    }

    // stop: an earlier check point found the stop condition
    bs_status check(bool& stop) {
        stop = false;
        if (!pool_) {
            int dev = 0;
            BS_TRY_HIP(hipGetDevice(&dev));
            static thread_local std::unordered_map<int, Pool> pools;
            pool_ = &pools[dev];
            if (!pool_->ev[0])
                for (hipEvent_t& e : pool_->ev)
                    BS_TRY_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            if (pool_->cap < n_) {   // every earlier copy has completed (destructor)
                if (pool_->host) BS_TRY_HIP(hipHostFree(pool_->host));
                pool_->host = nullptr;
                pool_->cap = 0;
                BS_TRY_HIP(hipHostMalloc((void**)&pool_->host, sizeof(int32_t) * kSlots * n_,
                                         hipHostMallocDefault));
                pool_->cap = n_;
            }
        }
        const int slot = count_ % kSlots;
        BS_TRY_HIP(hipMemcpyAsync(pool_->host + (size_t)slot * n_, flags_, sizeof(int32_t) * n_,
                                  hipMemcpyDeviceToHost, s_));
        BS_TRY_HIP(hipEventRecord(pool_->ev[slot], s_));
        ++count_;
        if (count_ > kLag) {
            const int old = (count_ - 1 - kLag) % kSlots;
            BS_TRY_HIP(hipEventSynchronize(pool_->ev[old]));
            const int32_t* f = pool_->host + (size_t)old * n_;
            bool any = false;
            for (int i = 0; i < n_; ++i) any = any || f[i] != 0;
            stop = all_zero_ ? !any : f[0] != 0;
        }
        return BS_OK;
    }

  private:
    static constexpr int kSlots = kLag + 1;
    struct Pool {
        int32_t* host = nullptr;   // pinned, [kSlots][cap]
        int cap = 0;
        hipEvent_t ev[kSlots] = {};
    };
    const int32_t* flags_;
    int n_;
    hipStream_t s_;
    bool all_zero_;
    Pool* pool_ = nullptr;
    int count_ = 0;
};


// ---------------------------------------------------------------------------
// Kernel timing hooks (see bs_timing.hip).
// ---------------------------------------------------------------------------
enum KernelId : int {
    K_LEVEL_COUNT, K_LEVEL_SCAN, K_LEVEL_WRITE, K_NEIGHBOURS, K_BIST_STEP, K_BIST_OTHER,
    K_SPLAT, K_INIT, K_PCG_START, K_PCG_MATVEC, K_PCG_UPDATE, K_PCG_REDUCE, K_SLICE,
    K_GRAD_SCATTER, K_DT_ROWS, K_DT_COLS, K_DT_OTHER,
    K_COUNT
};
bool timing_enabled();
// The start and stop events of one timed launch of kernel `id` (both null
// while timing is disabled).  The launch takes them itself
// (hipExtLaunchKernelGGL), so they bracket the kernel's execution alone,
// without the cost of separate event records on the stream.
void timing_pair(int id, hipEvent_t* start, hipEvent_t* stop);

// Enqueues `kernel` on `lstream` (the launch's stream, the same as `stream`),
// timed when timing is enabled, and checks it.
#define BS_LAUNCH(stream, id, name, kernel, grid, block, shmem, lstream, ...)                \
    do {                                                                                    \
        hipEvent_t e0_ = nullptr, e1_ = nullptr;                                            \
        ::bs::timing_pair(id, &e0_, &e1_);                                                  \
        if (e0_)                                                                            \
            hipExtLaunchKernelGGL(kernel, grid, block, shmem, lstream, e0_, e1_, 0,         \
                                  __VA_ARGS__);                                             \
        else                                                                                \
            hipLaunchKernelGGL(kernel, grid, block, shmem, lstream, __VA_ARGS__);           \
        BS_CHECK_LAUNCH(name);                                                              \
    } while (0)

// ---------------------------------------------------------------------------
// Sizes and constants.
// ---------------------------------------------------------------------------
constexpr int kBlock = 256;          // threads per block of streaming kernels
constexpr int kXcds = 8;             // MI355X: 8 accelerator dies, one L2 each
constexpr int kMaxGrid = 2048;       // blocks of a grid-stride launch
// Reducing kernels (bistochastization, PCG) run G blocks of kRedBlock threads
// (G from red_grid): small blocks spread even small grids over every compute
// unit, whose address units bound the neighbour gathers.  Each writes one
// partial per block; the next kernel reduces them in its prologue (the kernel
// boundary is the only grid-wide synchronisation).
constexpr int kRedBlock = 256;
constexpr int kRedGridSmall = 256;    // one block per compute unit
constexpr int kRedGridLarge = 1024;   // four: more waves in flight for large grids
constexpr int kRedGridMax = kRedGridLarge;
static_assert(kRedGridMax % kRedBlock == 0, "partials per thread");

// Grid of the reducing kernels for `elements` (vertex, channel) elements (an
// upper bound known on the host): small grids are latency-bound and favour
// cheap prologue reductions, large ones bandwidth-bound and favour occupancy.
inline int red_grid(int64_t elements) {
    return elements >= (int64_t)1 << 21 ? kRedGridLarge : kRedGridSmall;
}

// Slots of the device counter array.
enum Counter : int {
    CNT_V = 0,            // level-0 vertex count
    CNT_K = 1,            // pyramid top level K (first level with one vertex)
    CNT_BIST_ITERS = 2,   // bistochastization updates applied
    CNT_BIST_DONE = 3,    // 1 once bistochastization has stopped
    CNT_BIST_SRC = 4,     // ping-pong buffer holding the final n
    CNT_NB_WIDE = 5,      // 1 when some neighbour lies more than 32767 ids away
                          // (a diagnostic: nb_packed grids never set it)
    CNT_LEVEL0 = 8,       // V_k at CNT_LEVEL0 + k
    CNT_SIZE = 64
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Round-half-up grid coordinate in integers: floor((2v + s) / 2s).
__host__ __device__ inline int grid_coord(int v, int s) { return (2 * v + s) / (2 * s); }

// First index p >= 0 whose coordinate is g: ceil((2 g s - s) / 2), clamped at 0.
__host__ __device__ inline int cell_lo(int g, int s) {
    int t = 2 * g * s - s;
    return t <= 0 ? 0 : (t + 1) / 2;
}

inline int bit_length(int v) {
    int b = 0;
    while (v > 0) { ++b; v >>= 1; }
    return b;
}

// Number of grid-stride blocks for `units` work units, a multiple of kXcds.
inline int grid_blocks(int64_t units) {
    int64_t g = ceil_div(units < 1 ? 1 : units, 1);
    g = ceil_div(g, kXcds) * kXcds;
    if (g > kMaxGrid) g = kMaxGrid;
    return (int)g;
}

// ---------------------------------------------------------------------------
// Workspace carving.
// ---------------------------------------------------------------------------
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base((char*)b) {}
    template <class T>
    T* take(int64_t count) {
        off = align_up(off, 256);
        T* p = base ? (T*)(base + off) : nullptr;
        off += (size_t)(count < 0 ? 0 : count) * sizeof(T);
        return p;
    }
};

// One level of the grid pyramid.  Level 0 is the grid itself: its items are
// pixels.  The items of level k >= 1 are the vertices of level k-1.
struct Level {
    int64_t cap;             // vertex capacity
    int64_t item_cap;        // item capacity (P at level 0, cap of level k-1 above)
    int32_t ncx, ncy;        // spatial cells
    uint64_t* key;           // [cap] packed keys, ascending
    int32_t* mult;           // [cap] items per vertex (level 0: m)
    int32_t* ones;           // [cap] level-0 vertices below each vertex (level >= 1)
    int32_t* cell_vbase;     // [ncells + 1] first vertex of each cell
    int32_t* cell_ibase;     // [ncells + 1] first CSR slot of each cell
    int32_t* ptr;            // [cap + 1] CSR of items per vertex
    int32_t* list;           // [item_cap] item ids
    int32_t* item_parent;    // [item_cap] vertex of each item (level 0: idx)
};

struct GridImpl {
    uint32_t magic;
    int32_t H, W, P;
    bs_grid_params sg;
    int32_t levels;          // allocated levels, K <= levels - 1
    int32_t bistochastized;  // set by bs_bistochastize
    int32_t pyramid_built;   // levels k >= 1 enqueued (by the first bs_bistochastize)
    int64_t vcap;
    size_t ws_bytes;
    void* ws;
    int32_t max_cells;
    Level lv[BS_MAX_LEVELS];
    int32_t* nbr;            // [10][vcap]
    uint32_t* nb16;          // [5][vcap] the same table as signed 16-bit offsets u - v
                             // (0: no neighbour), slots 2i and 2i+1 in word i
    int32_t nb_packed;       // 1 when every offset provably fits 16 bits (the stencil
                             // passes read nb16), else they read nbr
    double* nbuf[2];         // bistochastization ping-pong
    double* n64;             // [vcap] final n
    float* nf;               // [vcap]
    double* nn;              // [vcap] n o N n
    int32_t* counts;         // [CNT_SIZE]
    double* bist_res;        // [1]
    double* bist_part;       // [2][kRedGridMax] ping-pong partial maxima
    int32_t* cell_cnt;       // [max_cells] scratch
    int32_t* cell_items;     // [max_cells] scratch
    uint32_t* ikey;          // [P] item keys with first-occurrence flag, scratch
};
static_assert(sizeof(GridImpl) <= BS_GRID_BYTES, "bs_grid too small");

constexpr uint32_t kGridMagic = 0xB5A7E001u;

inline GridImpl* impl(bs_grid* g) { return reinterpret_cast<GridImpl*>(g->opaque); }
inline const GridImpl* impl(const bs_grid* g) { return reinterpret_cast<const GridImpl*>(g->opaque); }

// Enqueues the pyramid levels k >= 1 of a grid whose level 0 is built.
bs_status build_pyramid(const GridImpl& g, hipStream_t s);

// A library-owned stream of the current device paired with `s` (default
// priority, created once), for work that may overlap work on `s`.
bs_status side_stream(hipStream_t s, hipStream_t* out);
// Library-owned stream `index` (of 8) of the current device.
bs_status library_stream(int index, hipStream_t* out);

// Lays out (or sizes, with base == nullptr) a grid for an H x W image.
// Returns the bytes used; fills `g` when base != nullptr.
size_t layout_grid(GridImpl& g, int H, int W, const bs_grid_params& sp, void* base);

// ---------------------------------------------------------------------------
// Device helpers.
// ---------------------------------------------------------------------------

// XCD-aware tile mapping for grid-stride loops.  Workgroups are dispatched to
// the dies round-robin, so block b runs on die b % 8.  Tiles [0, T) are split
// into 8 contiguous chunks, one per die, so that neighbouring tiles (and the
// vertices their stencils gather) share one L2.
struct XcdTiles {
    int64_t first, step, end;
    __device__ XcdTiles(int64_t T) : XcdTiles(T, blockIdx.x, gridDim.x) {}
    // Block j of nb blocks working on one image (j % 8 is the block's die:
    // the image's first block and nb are multiples of 8).
    __device__ XcdTiles(int64_t T, int j, int nb) {
        const int xcd = j % kXcds;
        const int local = j / kXcds;
        const int per = nb / kXcds;
        const int64_t chunk = (T + kXcds - 1) / kXcds;
        first = (int64_t)xcd * chunk + local;
        int64_t e = (int64_t)(xcd + 1) * chunk;
        end = e < T ? e : T;
        step = per;
    }
};

// Slot of block j's partial result among nb: blocks of one die get
// consecutive slots, so a cache line of partials is written from one die only.
__device__ inline int partial_slot(int j, int nb) {
    return (j % kXcds) * (nb / kXcds) + j / kXcds;
}
__device__ inline int partial_slot() { return partial_slot(blockIdx.x, gridDim.x); }

// ---------------------------------------------------------------------------
// Launches over one image or over a table of images.
//
// A kernel body is an Op: a struct with its per-image arguments Args, its
// block size kThreads and run(args, j, nb, arg), which does block j of the
// nb blocks working on one image (`arg`: a scalar of the launch, the same for
// every image, e.g. an iteration number).  one_launch runs an Op over one
// image (j = blockIdx.x, nb = gridDim.x); multi_launch runs it over a table
// of images, every block finding its image and its place among that image's
// blocks in a schedule.  So the single-image calls and the batch engine run
// the same code.
// ---------------------------------------------------------------------------
struct Sched {
    const int32_t* blk2img;   // [G] table index of each block's image, -1: idle block
    const int32_t* block0;    // [n] first block of each image
    const int32_t* nb;        // [n] blocks of each image
};

template <class Op>
__global__ void __launch_bounds__(Op::kThreads) one_launch(typename Op::Args a, int arg) {
    Op::run(a, (int)blockIdx.x, (int)gridDim.x, arg);
}

template <class Op>
__global__ void __launch_bounds__(Op::kThreads)
    multi_launch(const typename Op::Args* __restrict__ tab, Sched s, int arg) {
    const int i = s.blk2img[blockIdx.x];
    if (i < 0) return;
    Op::run(tab[i], (int)blockIdx.x - s.block0[i], s.nb[i], arg);
}

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide sum of one double per thread, deterministic (fixed shuffle and
// LDS trees); the result is returned to every thread.
template <int B>
__device__ inline double block_sum(double v) {
    __shared__ double red[B / 64];
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < B / 64; ++w) s += red[w];
    return s;
}

template <int B>
__device__ inline double block_max(double v) {
    __shared__ double red[B / 64];
    v = wave_max(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = red[0];
#pragma unroll
    for (int w = 1; w < B / 64; ++w) s = fmax(s, red[w]);
    return s;
}

// Packed neighbour table: signed 16-bit offsets u - v, 0 for a missing
// neighbour (a vertex is never its own neighbour), slots 2i and 2i+1 in word
// i.  Vertices are ordered by (cell row, cell column, colour), so a neighbour
// is at most one row of cells plus one cell away: |u - v| < (ncx + 1) * the
// most vertices a cell can hold.  Grids where that bound exceeds 32767 keep
// the 32-bit table for the stencil passes.
constexpr int kNbOffsetMax = 32767;

inline bool packed_table_fits(int64_t ncx, int64_t cell_max) {
    return (ncx + 1) * cell_max <= (int64_t)kNbOffsetMax + 1;
}

__host__ __device__ inline uint32_t pack_offsets(int v, int lo, int hi) {
    const uint32_t a = lo < 0 ? 0u : (uint32_t)(lo - v) & 0xffffu;
    const uint32_t b = hi < 0 ? 0u : (uint32_t)(hi - v) & 0xffffu;
    return a | (b << 16);
}

__device__ inline int unpack_offset(int v, uint32_t half) {
    const int o = (int)(int16_t)(uint16_t)half;
    return o != 0 ? v + o : -1;
}

// The ten neighbour ids of vertex v (slot 2d: -1 step, 2d+1: +1 step along
// dim d of (y, x, l, u, v); -1 if absent): five packed words, or ten 32-bit
// ids.  `packed` is uniform over the launch.
template <class P32, class P16>
__device__ inline void load_neighbours(int (&nb)[10], int v, int64_t vcap, bool packed, P32 nbr,
                                       P16 nb16) {
    if (packed) {
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const uint32_t p = nb16[i * vcap + v];
            nb[2 * i] = unpack_offset(v, p & 0xffffu);
            nb[2 * i + 1] = unpack_offset(v, p >> 16);
        }
    } else {
#pragma unroll
        for (int j = 0; j < 10; ++j) nb[j] = nbr[j * vcap + v];
    }
}

}  // namespace bs
