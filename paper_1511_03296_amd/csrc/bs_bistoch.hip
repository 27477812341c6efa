// Bistochastization of the grid blur (supplement Algorithm 1, Eq. equiv), in
// float64:  n <- sqrt(n o m / (B n)),  n = 1 initially, with B = 10 I + N.
//
// Launch s reads n_s from ping-pong buffer s % 2, writes n_{s+1} to the other
// buffer and publishes per-block maxima of the invariant residual
// max_v |n_v (B n_s)_v - m_v| / m_v.  Launch s+1 first reduces those maxima
// (the order of a max does not matter) and decides whether n_s is the answer:
// stop when the residual is <= tol or s >= max_iters.  Once stopped, later
// launches return at once, so the host may enqueue them without waiting.
#include "bs_internal.h"

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

__global__ void __launch_bounds__(kBlock) bist_init(double* __restrict__ n0,
                                                     const int32_t* __restrict__ counts) {
    const int V = counts[CNT_V];
    const XcdTiles tl((V + kBlock - 1) / kBlock);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int v = (int)(tile * kBlock) + threadIdx.x;
        if (v < V) n0[v] = 1.0;
    }
}

// Stop rule for the residual R of n_s.
__device__ inline bool bist_stop(double R, int s, int max_iters, double tol) {
    return R <= tol || s >= max_iters;
}

__global__ void __launch_bounds__(kRedBlock) bist_step(const int32_t* __restrict__ nbr,
                                                        const uint32_t* __restrict__ nb16,
                                                        const int32_t* __restrict__ m,
                                                        const double* __restrict__ src,
                                                        double* __restrict__ dst, int64_t vcap,
                                                        int32_t* __restrict__ counts,
                                                        double* __restrict__ part,
                                                        double* __restrict__ res_out, int step,
                                                        int max_iters, double tol, int packed) {
#pragma clang fp contract(off)
    const int G = gridDim.x;
    if (counts[CNT_BIST_DONE]) return;
    const int V = counts[CNT_V];
    const XcdTiles tl((V + kRedBlock - 1) / kRedBlock);
    // The previous launch's maxima, then the first tile's operands, are loaded
    // before the stop decision: loads complete in issue order, so waiting for
    // the maxima leaves the operand loads in flight during the reduction.
    double prevmax = 0.0;
    if (step >= 1) {
        const double* prev = part + ((step - 1) & 1) * kRedGridMax;
        for (int i = threadIdx.x; i < G; i += kRedBlock) prevmax = fmax(prevmax, prev[i]);
    }
    int v = (int)(tl.first * kRedBlock) + threadIdx.x;
    bool have = tl.first < tl.end && v < V;
    double n = 0.0, nbv[10];
    int mv = 1, nbi[10];
    if (have) {
        n = src[v];
        mv = m[v];
        load_neighbours(nbi, v, vcap, packed, nbr, nb16);
#pragma unroll
        for (int j = 0; j < 10; ++j) nbv[j] = (nbi[j] >= 0) ? src[nbi[j]] : 0.0;
    }
    if (step >= 1) {
        const double R = block_max<kRedBlock>(prevmax);
        if (bist_stop(R, step - 1, max_iters, tol)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                counts[CNT_BIST_ITERS] = step - 1;
                counts[CNT_BIST_SRC] = (step - 1) & 1;
                *res_out = R;
                counts[CNT_BIST_DONE] = 1;
            }
            return;
        }
    }
    double lmax = 0.0;
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        if (tile != tl.first) {
            v = (int)(tile * kRedBlock) + threadIdx.x;
            have = v < V;
            if (have) {
                n = src[v];
                mv = m[v];
                load_neighbours(nbi, v, vcap, packed, nbr, nb16);
#pragma unroll
                for (int j = 0; j < 10; ++j) nbv[j] = (nbi[j] >= 0) ? src[nbi[j]] : 0.0;
            }
        }
        if (!have) continue;
        double ns = 0.0;
#pragma unroll
        for (int j = 0; j < 10; ++j) ns += nbv[j];
        const double bn = 10.0 * n + ns;
        const double md = (double)mv;
        const double prod = n * bn;
        const double r = fabs(prod - md) / md;
        lmax = fmax(lmax, r);
        const double q = (n * md) / bn;
        dst[v] = sqrt(q);
    }
    lmax = block_max<kRedBlock>(lmax);
    if (threadIdx.x == 0) part[(step & 1) * kRedGridMax + partial_slot()] = lmax;
}

// After the last enqueued launch `last`: decide on its residual if no launch
// has stopped the iteration yet (single block).
__global__ void __launch_bounds__(kRedBlock) bist_decide(int32_t* __restrict__ counts,
                                                          const double* __restrict__ part,
                                                          double* __restrict__ res_out, int last,
                                                          int G) {
    if (counts[CNT_BIST_DONE]) return;
    const double* prev = part + (last & 1) * kRedGridMax;
    double r = 0.0;
    for (int i = threadIdx.x; i < G; i += kRedBlock) r = fmax(r, prev[i]);
    const double R = block_max<kRedBlock>(r);
    if (threadIdx.x == 0) {
        counts[CNT_BIST_ITERS] = last;
        counts[CNT_BIST_SRC] = last & 1;
        *res_out = R;
        counts[CNT_BIST_DONE] = 1;
    }
}

// Copies the final n, its float rounding and n o (N n) (the smoothness
// diagonal divided by lambda at the fixed point) into the grid.
__global__ void __launch_bounds__(kBlock) bist_finalize(const int32_t* __restrict__ nbr,
                                                         const uint32_t* __restrict__ nb16,
                                                         const double* __restrict__ b0,
                                                         const double* __restrict__ b1,
                                                         int64_t vcap, double* __restrict__ n64,
                                                         float* __restrict__ nf,
                                                         double* __restrict__ nn,
                                                         const int32_t* __restrict__ counts,
                                                         int packed) {
#pragma clang fp contract(off)
    const int V = counts[CNT_V];
    const double* src = counts[CNT_BIST_SRC] ? b1 : b0;
    const XcdTiles tl((V + kBlock - 1) / kBlock);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int v = (int)(tile * kBlock) + threadIdx.x;
        if (v >= V) continue;
        const double n = src[v];
        int nbi[10];
        load_neighbours(nbi, v, vcap, packed, nbr, nb16);
        double ns = 0.0;
#pragma unroll
        for (int j = 0; j < 10; ++j) ns += (nbi[j] >= 0) ? src[nbi[j]] : 0.0;
        n64[v] = n;
        nf[v] = (float)n;
        nn[v] = n * ns;
    }
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
    BS_LAUNCH(s, K_BIST_OTHER, "bist_init", bist_init, dim3(blocks), dim3(kBlock), 0, s,
              g.nbuf[0], g.counts);
    const int G = red_grid(g.vcap);
    int last = 0;
    for (int step = 0; step <= p.max_iters; ++step) {
        BS_LAUNCH(s, K_BIST_STEP, "bist_step", bist_step, dim3(G), dim3(kRedBlock), 0, s,
                  g.nbr, g.nb16, g.lv[0].mult, g.nbuf[step & 1], g.nbuf[(step + 1) & 1], g.vcap,
                  g.counts, g.bist_part, g.bist_res, step, p.max_iters, p.tol,
                  g.nb_packed);
        last = step;
        if (p.check_every > 0 && (step + 1) % p.check_every == 0 && step < p.max_iters) {
            int32_t done = 0;
            BS_TRY_HIP(hipMemcpyAsync(&done, g.counts + CNT_BIST_DONE, sizeof(int32_t),
                                      hipMemcpyDeviceToHost, s));
            BS_TRY_HIP(hipStreamSynchronize(s));
            if (done) break;
        }
    }
    BS_LAUNCH(s, K_BIST_OTHER, "bist_decide", bist_decide, dim3(1), dim3(kRedBlock), 0, s,
              g.counts, g.bist_part, g.bist_res, last, G);
    BS_LAUNCH(s, K_BIST_OTHER, "bist_finalize", bist_finalize, dim3(blocks), dim3(kBlock), 0, s,
              g.nbr, g.nb16, g.nbuf[0], g.nbuf[1], g.vcap, g.n64, g.nf, g.nn, g.counts,
              g.nb_packed);
    if (join) {
        BS_TRY_HIP(hipStreamWaitEvent(s, join, 0));
        BS_TRY_HIP(hipEventDestroy(fork));
        BS_TRY_HIP(hipEventDestroy(join));
    }
    g.bistochastized = 1;
    return BS_OK;
}
