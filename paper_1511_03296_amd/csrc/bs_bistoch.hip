// Bistochastization of the grid blur (supplement Algorithm 1, Eq. equiv), in
// float64:  n <- sqrt(n o m / (B n)),  n = 1 initially, with B = 10 I + N.
// Each launch applies one Jacobi-style update to every vertex (reading the
// previous n from one ping-pong buffer and writing the other) and reduces the
// invariant residual max_v |n_v (B n)_v - m_v| / m_v of the n it read.  The
// last block to finish decides, on the device, whether to stop; later
// launches then return at once, so the host may enqueue them blindly.
#include "bs_internal.h"

namespace bs {

__global__ void __launch_bounds__(kBlock) bist_init(double* __restrict__ n0,
                                                     const int32_t* __restrict__ counts) {
    const int V = counts[CNT_V];
    const XcdTiles tl((V + kBlock - 1) / kBlock);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int v = (int)(tile * kBlock) + threadIdx.x;
        if (v < V) n0[v] = 1.0;
    }
}

__global__ void __launch_bounds__(kBlock) bist_step(const int32_t* __restrict__ nbr,
                                                     const int32_t* __restrict__ m,
                                                     const double* __restrict__ src,
                                                     double* __restrict__ dst, int64_t vcap,
                                                     int32_t* __restrict__ counts,
                                                     double* __restrict__ part,
                                                     double* __restrict__ res_out,
                                                     uint32_t* __restrict__ ticket, int step,
                                                     int max_iters, double tol) {
#pragma clang fp contract(off)
    // Uniform across the grid: written by the previous launch's last block.
    if (counts[CNT_BIST_DONE]) return;
    const int V = counts[CNT_V];
    double lmax = 0.0;
    const XcdTiles tl((V + kBlock - 1) / kBlock);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int v = (int)(tile * kBlock) + threadIdx.x;
        if (v >= V) continue;
        const double n = src[v];
        double ns = 0.0;
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            const int u = nbr[j * vcap + v];
            ns += (u >= 0) ? src[u] : 0.0;
        }
        const double bn = 10.0 * n + ns;
        const double mv = (double)m[v];
        const double prod = n * bn;
        const double r = fabs(prod - mv) / mv;
        lmax = fmax(lmax, r);
        const double q = (n * mv) / bn;
        dst[v] = sqrt(q);
    }
    __shared__ double red[kBlock / 64];
    lmax = wave_max(lmax);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = red[0];
        for (int w = 1; w < kBlock / 64; ++w) b = fmax(b, red[w]);
        part[blockIdx.x] = b;
    }
    if (last_block(ticket)) {
        double b = 0.0;
        for (int i = threadIdx.x; i < (int)gridDim.x; i += kBlock) b = fmax(b, part[i]);
        b = wave_max(b);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
        __syncthreads();
        if (threadIdx.x == 0) {
            double R = red[0];
            for (int w = 1; w < kBlock / 64; ++w) R = fmax(R, red[w]);
            if (R <= tol || step >= max_iters) {
                counts[CNT_BIST_DONE] = 1;
                counts[CNT_BIST_ITERS] = step;
                counts[CNT_BIST_SRC] = step & 1;
                *res_out = R;
            }
            atomicExch(ticket, 0u);
        }
    }
}

// Copies the final n, its float rounding and n o (N n) (the smoothness
// diagonal divided by lambda at the fixed point) into the grid.
__global__ void __launch_bounds__(kBlock) bist_finalize(const int32_t* __restrict__ nbr,
                                                         const double* __restrict__ b0,
                                                         const double* __restrict__ b1,
                                                         int64_t vcap, double* __restrict__ n64,
                                                         float* __restrict__ nf,
                                                         double* __restrict__ nn,
                                                         const int32_t* __restrict__ counts) {
#pragma clang fp contract(off)
    const int V = counts[CNT_V];
    const double* src = counts[CNT_BIST_SRC] ? b1 : b0;
    const XcdTiles tl((V + kBlock - 1) / kBlock);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int v = (int)(tile * kBlock) + threadIdx.x;
        if (v >= V) continue;
        const double n = src[v];
        double ns = 0.0;
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            const int u = nbr[j * vcap + v];
            ns += (u >= 0) ? src[u] : 0.0;
        }
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
    const int blocks = grid_blocks(ceil_div(g.vcap, kBlock));
    hipLaunchKernelGGL(bist_init, dim3(blocks), dim3(kBlock), 0, s, g.nbuf[0], g.counts);
    BS_CHECK_LAUNCH("bist_init");
    for (int step = 0; step <= p.max_iters; ++step) {
        hipLaunchKernelGGL(bist_step, dim3(blocks), dim3(kBlock), 0, s, g.nbr, g.lv[0].mult,
                           g.nbuf[step & 1], g.nbuf[(step + 1) & 1], g.vcap, g.counts,
                           g.bist_part, g.bist_res, g.ticket, step, p.max_iters, p.tol);
        BS_CHECK_LAUNCH("bist_step");
        if (p.check_every > 0 && (step + 1) % p.check_every == 0 && step < p.max_iters) {
            int32_t done = 0;
            BS_TRY_HIP(hipMemcpyAsync(&done, g.counts + CNT_BIST_DONE, sizeof(int32_t),
                                      hipMemcpyDeviceToHost, s));
            BS_TRY_HIP(hipStreamSynchronize(s));
            if (done) break;
        }
    }
    hipLaunchKernelGGL(bist_finalize, dim3(blocks), dim3(kBlock), 0, s, g.nbr, g.nbuf[0],
                       g.nbuf[1], g.vcap, g.n64, g.nf, g.nn, g.counts);
    BS_CHECK_LAUNCH("bist_finalize");
    g.bistochastized = 1;
    return BS_OK;
}
