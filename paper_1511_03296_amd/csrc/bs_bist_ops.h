// Kernel bodies of the bistochastization (supplement Algorithm 1, Eq. equiv),
// in float64:  n <- sqrt(n o m / (B n)),  n = 1 initially, with B = 10 I + N,
// as Ops run by the single-image entry point (one_launch) and by the batch
// engine (multi_launch).
#pragma once

#include "bs_internal.h"

namespace bs {

struct BistInit {
    static constexpr int kThreads = kBlock;
    struct Args {
        double* n0;
        const int32_t* counts;
    };
    __device__ static void run(const Args& a, int jb, int nb, int) {
        const int V = a.counts[CNT_V];
        const XcdTiles tl((V + kBlock - 1) / kBlock, jb, nb);
        for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
            const int v = (int)(tile * kBlock) + threadIdx.x;
            if (v < V) a.n0[v] = 1.0;
        }
    }
};

// Stop rule for the residual R of n_s.
__device__ inline bool bist_stop(double R, int s, int max_iters, double tol) {
    return R <= tol || s >= max_iters;
}

// Update `step` (the launch argument): n_{s+1} from n_s, with the stop
// decision on n_{s-1}'s residual first.  The image's nb blocks publish their
// maxima in slots partial_slot(j, nb) of the step's half of `part`.
struct BistStep {
    static constexpr int kThreads = kRedBlock;
    struct Args {
        const int32_t* nbr;
        const uint32_t* nb16;
        const int32_t* m;
        double* nbuf[2];
        int32_t* counts;
        double* part;
        double* res_out;
        int64_t vcap;
        int max_iters, packed;
        double tol;
    };
    __device__ static void run(const Args& a, int jb, int nb, int step);
};

__device__ inline void BistStep::run(const Args& a, int jb, int G, int step) {
#pragma clang fp contract(off)
    const int32_t* __restrict__ nbr = a.nbr;
    const uint32_t* __restrict__ nb16 = a.nb16;
    const int32_t* __restrict__ m = a.m;
    const double* __restrict__ src = a.nbuf[step & 1];
    double* __restrict__ dst = a.nbuf[(step + 1) & 1];
    int32_t* __restrict__ counts = a.counts;
    double* __restrict__ part = a.part;
    const int64_t vcap = a.vcap;
    const bool packed = a.packed != 0;
    if (counts[CNT_BIST_DONE]) return;
    const int V = counts[CNT_V];
    const XcdTiles tl((V + kRedBlock - 1) / kRedBlock, jb, G);
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
        if (bist_stop(R, step - 1, a.max_iters, a.tol)) {
            if (jb == 0 && threadIdx.x == 0) {
                counts[CNT_BIST_ITERS] = step - 1;
                counts[CNT_BIST_SRC] = (step - 1) & 1;
                *a.res_out = R;
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
    if (threadIdx.x == 0) part[(step & 1) * kRedGridMax + partial_slot(jb, G)] = lmax;
}

// After the last enqueued update `last` (the launch argument): decide on its
// residual if no update has stopped the iteration yet (one block per image).
// The image's updates ran on G blocks: `G`, or *Gp when Gp is set (a
// schedule's block count).
struct BistDecide {
    static constexpr int kThreads = kRedBlock;
    struct Args {
        int32_t* counts;
        const double* part;
        double* res_out;
        const int32_t* Gp;
        int G;
    };
    __device__ static void run(const Args& a, int, int, int last) {
        int32_t* __restrict__ counts = a.counts;
        if (counts[CNT_BIST_DONE]) return;
        const int G = a.Gp ? *a.Gp : a.G;
        const double* prev = a.part + (last & 1) * kRedGridMax;
        double r = 0.0;
        for (int i = threadIdx.x; i < G; i += kRedBlock) r = fmax(r, prev[i]);
        const double R = block_max<kRedBlock>(r);
        if (threadIdx.x == 0) {
            counts[CNT_BIST_ITERS] = last;
            counts[CNT_BIST_SRC] = last & 1;
            *a.res_out = R;
            counts[CNT_BIST_DONE] = 1;
        }
    }
};

// Copies the final n, its float rounding and n o (N n) (the smoothness
// diagonal divided by lambda at the fixed point) into the grid.
struct BistFinalize {
    static constexpr int kThreads = kBlock;
    struct Args {
        const int32_t* nbr;
        const uint32_t* nb16;
        const double* nbuf[2];
        double* n64;
        float* nf;
        double* nn;
        const int32_t* counts;
        int64_t vcap;
        int packed;
    };
    __device__ static void run(const Args& a, int jb, int nb, int) {
#pragma clang fp contract(off)
        const int V = a.counts[CNT_V];
        const double* __restrict__ src = a.counts[CNT_BIST_SRC] ? a.nbuf[1] : a.nbuf[0];
        const XcdTiles tl((V + kBlock - 1) / kBlock, jb, nb);
        for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
            const int v = (int)(tile * kBlock) + threadIdx.x;
            if (v >= V) continue;
            const double n = src[v];
            int nbi[10];
            load_neighbours(nbi, v, a.vcap, a.packed != 0, a.nbr, a.nb16);
            double ns = 0.0;
#pragma unroll
            for (int j = 0; j < 10; ++j) ns += (nbi[j] >= 0) ? src[nbi[j]] : 0.0;
            a.n64[v] = n;
            a.nf[v] = (float)n;
            a.nn[v] = n * ns;
        }
    }
};

inline BistInit::Args bist_init_args(const GridImpl& g) { return {g.nbuf[0], g.counts}; }

inline BistStep::Args bist_step_args(const GridImpl& g, const bs_bistoch_params& p) {
    BistStep::Args a;
    a.nbr = g.nbr;
    a.nb16 = g.nb16;
    a.m = g.lv[0].mult;
    a.nbuf[0] = g.nbuf[0];
    a.nbuf[1] = g.nbuf[1];
    a.counts = g.counts;
    a.part = g.bist_part;
    a.res_out = g.bist_res;
    a.vcap = g.vcap;
    a.max_iters = p.max_iters;
    a.packed = g.nb_packed;
    a.tol = p.tol;
    return a;
}

inline BistDecide::Args bist_decide_args(const GridImpl& g, int G, const int32_t* Gp) {
    return {g.counts, g.bist_part, g.bist_res, Gp, G};
}

inline BistFinalize::Args bist_finalize_args(const GridImpl& g) {
    BistFinalize::Args a;
    a.nbr = g.nbr;
    a.nb16 = g.nb16;
    a.nbuf[0] = g.nbuf[0];
    a.nbuf[1] = g.nbuf[1];
    a.n64 = g.n64;
    a.nf = g.nf;
    a.nn = g.nn;
    a.counts = g.counts;
    a.vcap = g.vcap;
    a.packed = g.nb_packed;
    return a;
}

}  // namespace bs
