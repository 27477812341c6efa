// The bilateral-space solve (paper Eq. quad_min and Eq. solution, supplement
// Algorithm 2, Section 4 initialisation) and its backward pass (Section 3).
//
// Layouts: pixel planes [C][P] float32; bilateral-space vectors [V][C]
// float32, channels contiguous per vertex.  A thread of the vertex kernels
// owns one (vertex, channel) element: a block covers vpb = 256 / C vertices of
// all C channels, so the neighbour table is read once per vertex and the
// channel gathers of one neighbour are contiguous.
//
// PCG (supplement Algorithm 2) runs one independent PCG per channel.  One
// iteration is two kernels, each with one grid-wide reduction:
//   pcg_matvec:  d = M^-1 r + beta d  (fused: the neighbours' new d values are
//                recomputed from their gathered r and old d),  q = A d, d^T q;
//   pcg_update:  y += alpha d,  r -= alpha q,  r^T r,  r^T M^-1 r.
// A z is evaluated in Laplacian form,
//   (A z)_v = (S c)_v z_v + lam n_v sum_u n_u (z_v - z_u),
// which equals diag(A) z - lam n o N(n o z) with diag(A) = lam n o N n + S c,
// but cancels constants exactly and keeps float32 rounding relative to the
// result rather than to lam m z (the difference matters where confidence is
// sparse).  Dot products accumulate in float64; the next kernel reduces the
// per-block partials in its prologue in a fixed order, so results are
// deterministic and no host synchronisation is needed.
#include "bs_internal.h"

namespace bs {

// One record per 128-byte cache line: each block reads back its own record,
// written by the block of the same index (same die) in the previous launch.
// With 48- or 64-byte records a line held records of blocks on two dies and
// that read cost ~12 us per launch on MI355X.
struct alignas(128) ChanState {
    double rho, alpha, beta, bnorm, res;
    int32_t active, iters, reason, phase;   // phase 0: initial residual not yet reduced
};
static_assert(sizeof(ChanState) == 128, "one record per cache line");

enum Ctl : int { CTL_ACTIVE = 0, CTL_SIZE = 8 };

// Partials of the reducing kernels: [2 slots][3 values][C][G].
//   slot 0 -- pcg_start (r^T r, b^T b, r^T M^-1 r), pcg_update (r^T r, 0, r^T M^-1 r);
//   slot 1 -- pcg_matvec (d^T q).
// Per-channel state, double-buffered the same way: pcg_matvec reads state 0
// and writes state 1, pcg_update reads state 1 and writes state 0.  Every
// block computes the same state from the same partials and keeps its own copy
// (slot [block][C]): block b always runs on die b % 8, so its copy stays in
// that die's L2, whereas reading one copy written by another die's block cost
// ~12 us per launch.
struct SolveWs {
    int C, vpb, G;
    float* sc;
    float* diag;
    float* minv;
    float* b;
    float* r;
    float* d[2];
    float* q;
    float* g;
    float* up[BS_MAX_LEVELS];
    ChanState* cs[2];
    double* part[2];
    double* sums[2];     // [3][C] reduced partials when pcg_reduce is used
    int32_t* ctl;
    size_t bytes;
};

static size_t layout_solve(const GridImpl& g, int C, void* base, SolveWs& w) {
    w.C = C;
    w.vpb = kRedBlock / C;
    w.G = red_grid(g.vcap * C);
    Carver c(base);
    const int64_t n = g.vcap * C;
    w.sc = c.take<float>(g.vcap);
    w.diag = c.take<float>(g.vcap);
    w.minv = c.take<float>(g.vcap);
    w.b = c.take<float>(n);
    w.r = c.take<float>(n);
    w.d[0] = c.take<float>(n);
    w.d[1] = c.take<float>(n);
    w.q = c.take<float>(n);
    w.g = c.take<float>(n);
    w.up[0] = nullptr;
    for (int k = 1; k < BS_MAX_LEVELS; ++k)
        w.up[k] = (k < g.levels) ? c.take<float>(g.lv[k].cap * (C + 1)) : nullptr;
    w.cs[0] = c.take<ChanState>((int64_t)kRedGridMax * C);
    w.cs[1] = c.take<ChanState>((int64_t)kRedGridMax * C);
    w.part[0] = c.take<double>((int64_t)3 * C * kRedGridMax);
    w.part[1] = c.take<double>((int64_t)3 * C * kRedGridMax);
    w.sums[0] = c.take<double>(3 * C);
    w.sums[1] = c.take<double>(3 * C);
    w.ctl = c.take<int32_t>(CTL_SIZE);
    w.bytes = align_up(c.off, 256);
    return w.bytes;
}

// ---------------------------------------------------------------------------
// Reductions over (vertex, channel) blocks.
// ---------------------------------------------------------------------------

// Sums NV per-thread values over the vertices of the block, per channel, with
// a fixed tree, and writes the block's partials to part[(k C + ch) G + block]
// (G = gridDim.x).
template <int NV>
__device__ inline void block_channel_partials(const double (&acc)[NV], int C, int vpb,
                                              double* __restrict__ part) {
    const int t = threadIdx.x;
    if (C == 1) {
        // one channel: shuffle trees per wave, then one pass over the waves
        __shared__ double red[NV][kRedBlock / 64];
        double v[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = wave_sum(acc[k]);
        __syncthreads();
        if ((t & 63) == 0) {
#pragma unroll
            for (int k = 0; k < NV; ++k) red[k][t >> 6] = v[k];
        }
        __syncthreads();
        if (t < NV) {
            double s = 0.0;
            for (int w = 0; w < kRedBlock / 64; ++w) s += red[t][w];
            part[(int64_t)t * gridDim.x + partial_slot()] = s;
        }
        return;
    }
    __shared__ double s[NV][kRedBlock];
#pragma unroll
    for (int k = 0; k < NV; ++k) s[k][t] = acc[k];
    __syncthreads();
    int n = vpb;
    while (n > 1) {
        const int h = (n + 1) >> 1;
        if (t < (n - h) * C) {
#pragma unroll
            for (int k = 0; k < NV; ++k) s[k][t] += s[k][t + h * C];
        }
        __syncthreads();
        n = h;
    }
    if (t < C) {
#pragma unroll
        for (int k = 0; k < NV; ++k) part[((int64_t)k * C + t) * gridDim.x + partial_slot()] = s[k][t];
    }
}

// out[k C + ch] = sum over the G blocks of the producer's partials,
// computed identically by every block.  The NV C sums are spread over the
// block: q lanes (a power of two <= 64, so a group lies in one wave) share a
// sum, each adding every q-th partial, then a shuffle tree over the group.
// Loading (load) and summing (sum) are split so that callers can issue other
// loads in between; loads complete in issue order, so waiting for these does
// not wait for loads issued after them.
struct PartialSums {
    static constexpr int kMax = 16;   // partials per thread held in registers
    double v[kMax];
    int pairs, q, pair, seg, G;
    bool held;
    const double* pre;   // sums already reduced by pcg_reduce, or nullptr

    // Lanes per pair for `pairs` sums over G partials, and whether each lane's
    // share fits in registers (the host uses the same rule to decide when to
    // run pcg_reduce instead).
    __host__ __device__ static int lanes(int pairs) {
        int q = 64;
        while (q > 1 && q * pairs > kRedBlock) q >>= 1;
        return q;
    }
    __host__ __device__ static bool fits(int pairs, int G) {
        const int q = lanes(pairs);
        return pairs * q <= kRedBlock && G / q <= kMax;
    }

    __device__ void load(const double* __restrict__ part, int nv_c, int grid,
                         const double* __restrict__ sums = nullptr) {
        pre = sums;
        pairs = nv_c;
        G = grid;
        if (pre) {
            if ((int)threadIdx.x < pairs) v[0] = pre[threadIdx.x];
            return;
        }
        q = lanes(pairs);
        pair = threadIdx.x / q;
        seg = threadIdx.x - pair * q;
        held = fits(pairs, G);
        if (held && pair < pairs) {
#pragma unroll
            for (int i = 0; i < kMax; ++i)
                if (i < G / q) v[i] = part[(int64_t)pair * G + seg + q * i];
        }
    }

    __device__ void sum(const double* __restrict__ part, double* out) {
        if (pre) {
            if ((int)threadIdx.x < pairs) out[threadIdx.x] = v[0];
        } else if (held) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < kMax; ++i)
                if (i < G / q && pair < pairs) s += v[i];
            for (int o = q >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
            if (seg == 0 && pair < pairs) out[pair] = s;
        } else {
            for (int base = 0; base < pairs; base += kRedBlock / q) {
                const int pr = base + pair;
                double s = 0.0;
                if (pr < pairs)
                    for (int b = seg; b < G; b += q) s += part[(int64_t)pr * G + b];
                for (int o = q >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
                if (seg == 0 && pr < pairs) out[pr] = s;
            }
        }
        __syncthreads();
    }
};

template <int NV>
__device__ inline void reduce_partials(const double* __restrict__ part, int C, int G,
                                       double* out, const double* __restrict__ sums = nullptr) {
    PartialSums ps;
    ps.load(part, NV * C, G, sums);
    ps.sum(part, out);
}

// With many channels the per-block partials are reduced once, by one block per
// (value, channel) pair, rather than redundantly in every consumer block.
__global__ void __launch_bounds__(kRedBlock) pcg_reduce(const double* __restrict__ part,
                                                         double* __restrict__ sums, int G) {
    double v = 0.0;
    for (int i = threadIdx.x; i < G; i += kRedBlock) v += part[(int64_t)blockIdx.x * G + i];
    const double s = block_sum<kRedBlock>(v);
    if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

// Completes the previous PCG step of one channel from the reduced slot-0
// partials: the initial residual (phase 0) or the end of an iteration, with
// the stopping rule and the next beta.
__device__ inline void advance_state(ChanState& st, double rr, double bb, double rho_new,
                                     int max_iters, double tol) {
    int reason = 0;
    if (st.phase == 0) {
        st.phase = 1;
        st.bnorm = sqrt(bb);
        st.rho = rho_new;
        st.beta = 0.0;
        st.iters = 0;
        if (bb == 0.0) {
            st.res = 0.0;
            reason = 5;
        } else {
            st.res = sqrt(rr) / st.bnorm;
            if (st.res <= tol) reason = 1;
            else if (max_iters <= 0) reason = 2;
            else if (rho_new == 0.0) reason = 3;
        }
    } else {
        if (!st.active) return;
        st.beta = rho_new / st.rho;
        st.rho = rho_new;
        st.iters += 1;
        st.res = sqrt(rr) / st.bnorm;
        if (st.res <= tol) reason = 1;
        else if (st.iters >= max_iters) reason = 2;
        else if (rho_new == 0.0) reason = 3;
    }
    st.active = reason == 0;
    if (reason) st.reason = reason;
}

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------

__global__ void solve_prologue(ChanState* cs0, ChanState* cs1, int n, int32_t* ctl) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < CTL_SIZE) ctl[t] = 0;
    if (t < n) {
        ChanState z;
        z.rho = z.alpha = z.beta = z.bnorm = z.res = 0.0;
        z.active = z.iters = z.reason = z.phase = 0;
        cs0[t] = z;
        cs1[t] = z;
    }
}

// S c, b = S (v o t) (or S t when `weighted` is false) as ascending-pixel sums
// in float64, and diag(A) = lam n o (N n) + S c with its Jacobi inverse.
template <bool WEIGHTED>
__global__ void __launch_bounds__(kBlock) splat_kernel(
    const int32_t* __restrict__ ptr, const int32_t* __restrict__ list,
    const float* __restrict__ conf, const float* __restrict__ vals, int C, int P,
    const double* __restrict__ nn, double lam, const int32_t* __restrict__ counts,
    float* __restrict__ sc_out, float* __restrict__ diag_out, float* __restrict__ minv_out,
    float* __restrict__ b) {
    const int V = counts[CNT_V];
    const XcdTiles tl((V + kBlock - 1) / kBlock);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int v = (int)(tile * kBlock) + threadIdx.x;
        if (v >= V) continue;
        const int s = ptr[v], e = ptr[v + 1];
        double sc = 0.0;
        for (int j = s; j < e; ++j) sc += (double)conf[list[j]];
        for (int c0 = 0; c0 < C; c0 += 8) {
            double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            const int cn = min(8, C - c0);
            for (int j = s; j < e; ++j) {
                const int p = list[j];
                const double w = WEIGHTED ? (double)conf[p] : 1.0;
#pragma unroll
                for (int k = 0; k < 8; ++k)
                    if (k < cn) acc[k] += w * (double)vals[(int64_t)(c0 + k) * P + p];
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (k < cn) b[(int64_t)v * C + c0 + k] = (float)acc[k];
        }
        const double d = lam * nn[v] + sc;
        sc_out[v] = (float)sc;
        diag_out[v] = (float)d;
        minv_out[v] = d > 0.0 ? (float)(1.0 / d) : 0.0f;
    }
}

// The same sums computed per spatial cell of the grid: every pixel of a cell
// lies on one of the cell's vertices, so a block stages the cell's pixels in
// LDS with coalesced row loads and each (vertex, channel) thread sums its own
// pixels, in ascending pixel order, from LDS.  CAP bounds the cell's pixels.
constexpr int kSplatVals = 4096;   // floats of staged values per channel chunk

template <int B, int CAP, bool WEIGHTED>
__global__ void __launch_bounds__(B) splat_cells(
    int H, int W, int sxy, int ncx, const int32_t* __restrict__ cell_vbase,
    const int32_t* __restrict__ cell_ibase, const int32_t* __restrict__ ptr,
    const int32_t* __restrict__ list, const float* __restrict__ conf,
    const float* __restrict__ vals, int C, int P, const double* __restrict__ nn, double lam,
    float* __restrict__ sc_out, float* __restrict__ diag_out, float* __restrict__ minv_out,
    float* __restrict__ b) {
    __shared__ float cv[CAP];
    __shared__ int32_t lst[CAP];
    __shared__ float tv[kSplatVals];
    const int c = blockIdx.x;
    const int cy = c / ncx, cx = c - cy * ncx;
    const int y0 = cell_lo(cy, sxy), y1 = min(cell_lo(cy + 1, sxy), H);
    const int x0 = cell_lo(cx, sxy), x1 = min(cell_lo(cx + 1, sxy), W);
    const int wx = x1 - x0, n = (y1 - y0) * wx;
    const int vbase = cell_vbase[c], cnt = cell_vbase[c + 1] - vbase, ibase = cell_ibase[c];
    for (int j = threadIdx.x; j < n; j += B) {
        const int r = j / wx;
        cv[j] = conf[(y0 + r) * W + x0 + (j - r * wx)];
        const int pq = list[ibase + j];
        const int py = pq / W;
        lst[j] = (py - y0) * wx + (pq - py * W - x0);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < cnt; k += B) {
        const int s0 = ptr[vbase + k] - ibase, s1 = ptr[vbase + k + 1] - ibase;
        double sc = 0.0;
        for (int q = s0; q < s1; ++q) sc += (double)cv[lst[q]];
        const double d = lam * nn[vbase + k] + sc;
        sc_out[vbase + k] = (float)sc;
        diag_out[vbase + k] = (float)d;
        minv_out[vbase + k] = d > 0.0 ? (float)(1.0 / d) : 0.0f;
    }
    const int CH = max(1, min(C, kSplatVals / max(n, 1)));
    for (int c0 = 0; c0 < C; c0 += CH) {
        const int cn = min(CH, C - c0);
        __syncthreads();
        for (int e = threadIdx.x; e < cn * n; e += B) {
            const int cc = e / n, j = e - cc * n;
            const int r = j / wx;
            tv[cc * n + j] = vals[(int64_t)(c0 + cc) * P + (y0 + r) * W + x0 + (j - r * wx)];
        }
        __syncthreads();
        for (int e = threadIdx.x; e < cnt * cn; e += B) {
            const int k = e / cn, cc = e - k * cn;
            const int s0 = ptr[vbase + k] - ibase, s1 = ptr[vbase + k + 1] - ibase;
            double acc = 0.0;
            for (int q = s0; q < s1; ++q) {
                const int jl = lst[q];
                acc += WEIGHTED ? (double)cv[jl] * (double)tv[cc * n + jl] : (double)tv[cc * n + jl];
            }
            b[(int64_t)(vbase + k) * C + c0 + cc] = (float)acc;
        }
    }
}

// Launches the splat: per cell when a cell's pixels fit the LDS staging,
// otherwise per vertex.
template <bool WEIGHTED>
static bs_status launch_splat(const GridImpl& g, const float* conf, const float* vals, int C,
                              double lam, float* sc, float* diag, float* minv, float* b,
                              hipStream_t s) {
    const Level& L = g.lv[0];
    const int items = g.sg.sigma_xy * g.sg.sigma_xy;
    const int ncells = L.ncx * L.ncy;
#define BS_SPLAT_CELLS(B, CAP)                                                                  \
    BS_LAUNCH(s, K_SPLAT, "splat_cells", (splat_cells<B, CAP, WEIGHTED>), dim3(ncells), dim3(B), \
              0, s, g.H, g.W, g.sg.sigma_xy, L.ncx, L.cell_vbase, L.cell_ibase, L.ptr, L.list,   \
              conf, vals, C, g.P, g.nn, lam, sc, diag, minv, b)
    if (items <= 64) BS_SPLAT_CELLS(64, 64);
    else if (items <= 256) BS_SPLAT_CELLS(256, 256);
    else if (items <= 1024) BS_SPLAT_CELLS(256, 1024);
    else {
        const int vblocks = grid_blocks(ceil_div(g.vcap, kBlock));
        BS_LAUNCH(s, K_SPLAT, "splat", splat_kernel<WEIGHTED>, dim3(vblocks), dim3(kBlock), 0, s,
                  L.ptr, L.list, conf, vals, C, g.P, g.nn, lam, g.counts, sc, diag, minv, b);
    }
#undef BS_SPLAT_CELLS
    return BS_OK;
}

// Flat init: y = b / S c, 0 where S c = 0.
__global__ void __launch_bounds__(kBlock) flat_init_kernel(const float* __restrict__ b,
                                                            const float* __restrict__ sc, int C,
                                                            const int32_t* __restrict__ counts,
                                                            float* __restrict__ y) {
    const int64_t n = (int64_t)counts[CNT_V] * C;
    const XcdTiles tl((n + kBlock - 1) / kBlock);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int64_t e = tile * kBlock + threadIdx.x;
        if (e >= n) continue;
        const float s = sc[e / C];
        y[e] = s > 0.0f ? b[e] / s : 0.0f;
    }
}

// Pyramid lift, level k >= 1: child sums of level k-1 for C channels of b and
// S c (channel C).  up_k[u][ch] = sum over children of the child's value.
__global__ void __launch_bounds__(kBlock) pyr_up(const int32_t* __restrict__ cptr,
                                                  const int32_t* __restrict__ clist,
                                                  const float* __restrict__ b,
                                                  const float* __restrict__ sc,
                                                  const float* __restrict__ prev, float* __restrict__ up,
                                                  int C, int level, const int32_t* __restrict__ counts) {
    if (counts[CNT_K] < level) return;
    const int Vk = counts[CNT_LEVEL0 + level];
    const int C1 = C + 1;
    const int64_t n = (int64_t)Vk * C1;
    const XcdTiles tl((n + kBlock - 1) / kBlock);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int64_t e = tile * kBlock + threadIdx.x;
        if (e >= n) continue;
        const int u = (int)(e / C1), ch = (int)(e - (int64_t)u * C1);
        double s = 0.0;
        for (int j = cptr[u]; j < cptr[u + 1]; ++j) {
            const int c = clist[j];
            if (prev) s += (double)prev[(int64_t)c * C1 + ch];
            else s += (double)(ch < C ? b[(int64_t)c * C + ch] : sc[c]);
        }
        up[e] = (float)s;
    }
}

// Pyramid collapse, level k >= 1 (top-down): acc_k = w_k P_k / P(1)_k + acc_{k+1}[parent].
__global__ void __launch_bounds__(kBlock) pyr_down(float* __restrict__ up,
                                                    const float* __restrict__ up_parent,
                                                    const int32_t* __restrict__ parent,
                                                    const int32_t* __restrict__ ones, float wk,
                                                    int C, int level,
                                                    const int32_t* __restrict__ counts) {
    const int K = counts[CNT_K];
    if (K < level) return;
    const int Vk = counts[CNT_LEVEL0 + level];
    const int C1 = C + 1;
    const int64_t n = (int64_t)Vk * C1;
    const XcdTiles tl((n + kBlock - 1) / kBlock);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int64_t e = tile * kBlock + threadIdx.x;
        if (e >= n) continue;
        const int u = (int)(e / C1), ch = (int)(e - (int64_t)u * C1);
        float v = wk * up[e] / (float)ones[u];
        if (level < K) v += up_parent[(int64_t)parent[u] * C1 + ch];
        up[e] = v;
    }
}

// Level 0 of the collapse and the ratio of the two push-pull filters:
// y0 = (b + acc_1[parent]) / (S c + acc_1[parent][C]), 0 where the
// denominator is 0 (zero total confidence).
__global__ void __launch_bounds__(kBlock) hier_final(const float* __restrict__ b,
                                                      const float* __restrict__ sc,
                                                      const float* __restrict__ up1,
                                                      const int32_t* __restrict__ parent0, int C,
                                                      const int32_t* __restrict__ counts,
                                                      float* __restrict__ y) {
    const int K = counts[CNT_K];
    const int64_t n = (int64_t)counts[CNT_V] * C;
    const int C1 = C + 1;
    const XcdTiles tl((n + kBlock - 1) / kBlock);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int64_t e = tile * kBlock + threadIdx.x;
        if (e >= n) continue;
        const int v = (int)(e / C), ch = (int)(e - (int64_t)v * C);
        float num = b[e], den = sc[v];
        if (K >= 1) {
            const int64_t p = (int64_t)parent0[v] * C1;
            num += up1[p + ch];
            den += up1[p + C];
        }
        y[e] = den > 0.0f ? num / den : 0.0f;
    }
}

// r = b - A y0, one (vertex, channel) element per thread; partials r^T r,
// b^T b, r^T M^-1 r.
__global__ void __launch_bounds__(kRedBlock) pcg_start(
    const int32_t* __restrict__ nbr, int64_t vcap, const float* __restrict__ nf,
    const float* __restrict__ sc, const float* __restrict__ minv, const float* __restrict__ b,
    const float* __restrict__ y, float* __restrict__ r, float lam, int C, int vpb,
    const int32_t* __restrict__ counts, double* __restrict__ part) {
    const int V = counts[CNT_V];
    const int t = threadIdx.x;
    const int vl = t / C, ch = t - vl * C;
    const bool lane_ok = vl < vpb;
    double acc[3] = {0.0, 0.0, 0.0};
    const XcdTiles tl((V + vpb - 1) / vpb);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int v = (int)(tile * vpb) + vl;
        if (!lane_ok || v >= V) continue;
        const int64_t e = (int64_t)v * C + ch;
        const float yv = y[e];
        float ns = 0.0f;
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            const int u = nbr[j * vcap + v];
            if (u >= 0) ns += nf[u] * (yv - y[(int64_t)u * C + ch]);
        }
        const float ay = sc[v] * yv + lam * nf[v] * ns;
        const float bv = b[e];
        const float rv = bv - ay;
        r[e] = rv;
        acc[0] += (double)rv * (double)rv;
        acc[1] += (double)bv * (double)bv;
        acc[2] += (double)rv * (double)(minv[v] * rv);
    }
    block_channel_partials<3>(acc, C, vpb, part);
}

// Operands of one (vertex, channel) element of pcg_matvec.  Loading them does
// not depend on the iteration's scalars, so the first tile's loads are issued
// before the prologue and overlap its reduction.
struct MatvecOperands {
    int v;
    int nb[10];
    float r[10], d[10], mi[10], nf[10];
    float rv, dv, miv, scv, nfv;
};

__device__ inline bool load_matvec(MatvecOperands& o, int64_t tile, int vpb, int vl, int ch,
                                   int C, int V, int64_t vcap, const int32_t* __restrict__ nbr,
                                   const float* __restrict__ nf, const float* __restrict__ sc,
                                   const float* __restrict__ minv, const float* __restrict__ r,
                                   const float* __restrict__ dold) {
    o.v = (int)(tile * vpb) + vl;
    if (o.v >= V) return false;
#pragma unroll
    for (int j = 0; j < 10; ++j) o.nb[j] = nbr[j * vcap + o.v];
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        const int u = o.nb[j] >= 0 ? o.nb[j] : o.v;
        const int64_t eu = (int64_t)u * C + ch;
        o.r[j] = r[eu];
        o.d[j] = dold[eu];
        o.mi[j] = minv[u];
        o.nf[j] = nf[u];
    }
    const int64_t e = (int64_t)o.v * C + ch;
    o.rv = r[e];
    o.dv = dold[e];
    o.miv = minv[o.v];
    o.scv = sc[o.v];
    o.nfv = nf[o.v];
    return true;
}

// New search direction of one element: M^-1 r + beta d_old (M^-1 r first).
__device__ inline float pcg_dir(float r, float d_old, float mi, float beta, bool first) {
    const float s = mi * r;
    return first ? s : fmaf(beta, d_old, s);
}

// Prologue: finish the previous step (stopping rule, beta) from the slot-0
// partials.  Then d = M^-1 r + beta d_old, q = A d and partials of d^T q.
__global__ void __launch_bounds__(kRedBlock) pcg_matvec(
    const int32_t* __restrict__ nbr, int64_t vcap, const float* __restrict__ nf,
    const float* __restrict__ sc, const float* __restrict__ minv, const float* __restrict__ r,
    const float* __restrict__ dold, float* __restrict__ dnew, float* __restrict__ q, float lam,
    int C, int vpb, const int32_t* __restrict__ counts, const ChanState* __restrict__ cs_in,
    ChanState* __restrict__ cs_out, const double* __restrict__ part_in,
    const double* __restrict__ sums_in, double* __restrict__ part_out,
    int32_t* __restrict__ ctl, int max_iters, double tol) {
    __shared__ ChanState S[BS_MAX_CHANNELS];
    __shared__ double fin[3 * BS_MAX_CHANNELS];
    __shared__ int n_active;
    const int t = threadIdx.x;
    const int V = counts[CNT_V];
    const int vl = t / C, ch = t - vl * C;
    const bool lane_ok = vl < vpb;
    const XcdTiles tl((V + vpb - 1) / vpb);
    // Loads complete in issue order: partials and state first, then the first
    // tile's operands, which stay in flight during the reduction.
    PartialSums ps;
    ps.load(part_in, 3 * C, gridDim.x, sums_in);
    ChanState st0;
    if (t < C) st0 = cs_in[(int64_t)blockIdx.x * C + t];
    MatvecOperands o;
    bool have = lane_ok && tl.first < tl.end &&
                load_matvec(o, tl.first, vpb, vl, ch, C, V, vcap, nbr, nf, sc, minv, r, dold);
    ps.sum(part_in, fin);
    if (t == 0) n_active = 0;
    __syncthreads();
    if (t < C) {
        advance_state(st0, fin[t], fin[C + t], fin[2 * C + t], max_iters, tol);
        S[t] = st0;
        if (st0.active) atomicAdd(&n_active, 1);
        cs_out[(int64_t)blockIdx.x * C + t] = st0;
    }
    __syncthreads();
    if (blockIdx.x == 0 && t == 0) ctl[CTL_ACTIVE] = n_active;
    if (n_active == 0) return;
    const ChanState st = S[lane_ok ? ch : 0];
    const bool act = lane_ok && st.active;
    const bool first = st.iters == 0;
    const float beta = (float)st.beta;
    double acc[1] = {0.0};
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        if (tile != tl.first)
            have = lane_ok &&
                   load_matvec(o, tile, vpb, vl, ch, C, V, vcap, nbr, nf, sc, minv, r, dold);
        if (!act || !have) continue;
        const float dv = pcg_dir(o.rv, o.dv, o.miv, beta, first);
        float ns = 0.0f;
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            if (o.nb[j] >= 0) ns += o.nf[j] * (dv - pcg_dir(o.r[j], o.d[j], o.mi[j], beta, first));
        }
        const float qv = o.scv * dv + lam * o.nfv * ns;
        const int64_t e = (int64_t)o.v * C + ch;
        dnew[e] = dv;
        q[e] = qv;
        acc[0] += (double)dv * (double)qv;
    }
    block_channel_partials<1>(acc, C, vpb, part_out);
}

// Prologue: alpha = r^T M^-1 r / d^T q from the slot-1 partials (a channel
// with d^T q <= 0 stops).  Then y += alpha d, r -= alpha q and partials of
// r^T r and r^T M^-1 r.
__global__ void __launch_bounds__(kRedBlock) pcg_update(
    const float* __restrict__ minv, const float* __restrict__ d, const float* __restrict__ q,
    float* __restrict__ y, float* __restrict__ r, int C, int vpb,
    const int32_t* __restrict__ counts, const ChanState* __restrict__ cs_in,
    ChanState* __restrict__ cs_out, const double* __restrict__ part_in,
    const double* __restrict__ sums_in, double* __restrict__ part_out,
    int32_t* __restrict__ ctl) {
    __shared__ ChanState S[BS_MAX_CHANNELS];
    __shared__ double fin[BS_MAX_CHANNELS];
    __shared__ int n_active;
    const int t = threadIdx.x;
    const int V = counts[CNT_V];
    const int vl = t / C, ch = t - vl * C;
    const bool lane_ok = vl < vpb;
    const XcdTiles tl((V + vpb - 1) / vpb);
    PartialSums ps;
    ps.load(part_in, C, gridDim.x, sums_in);
    ChanState st0;
    if (t < C) st0 = cs_in[(int64_t)blockIdx.x * C + t];
    // first tile's operands in flight during the reduction
    int v = (int)(tl.first * vpb) + vl;
    bool have = lane_ok && tl.first < tl.end && v < V;
    float yv = 0.0f, dv = 0.0f, rv = 0.0f, qv = 0.0f, miv = 0.0f;
    if (have) {
        const int64_t e = (int64_t)v * C + ch;
        yv = y[e];
        dv = d[e];
        rv = r[e];
        qv = q[e];
        miv = minv[v];
    }
    ps.sum(part_in, fin);
    if (t == 0) n_active = 0;
    __syncthreads();
    if (t < C) {
        if (st0.active) {
            const double dq = fin[t];
            if (!(dq > 0.0)) {
                st0.active = 0;
                st0.reason = 4;
            } else {
                st0.alpha = st0.rho / dq;
            }
        }
        S[t] = st0;
        if (st0.active) atomicAdd(&n_active, 1);
        cs_out[(int64_t)blockIdx.x * C + t] = st0;
    }
    __syncthreads();
    if (blockIdx.x == 0 && t == 0) ctl[CTL_ACTIVE] = n_active;
    if (n_active == 0) return;
    const ChanState st = S[lane_ok ? ch : 0];
    const bool act = lane_ok && st.active;
    const float alpha = (float)st.alpha;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        if (tile != tl.first) {
            v = (int)(tile * vpb) + vl;
            have = lane_ok && v < V;
            if (have) {
                const int64_t e = (int64_t)v * C + ch;
                yv = y[e];
                dv = d[e];
                rv = r[e];
                qv = q[e];
                miv = minv[v];
            }
        }
        if (!act || !have) continue;
        const int64_t e = (int64_t)v * C + ch;
        y[e] = fmaf(alpha, dv, yv);
        const float r1 = fmaf(-alpha, qv, rv);
        r[e] = r1;
        acc[0] += (double)r1 * (double)r1;
        acc[2] += (double)r1 * (double)(miv * r1);
    }
    block_channel_partials<3>(acc, C, vpb, part_out);
}

// After the last enqueued iteration (single block): completes the pending
// step and writes the per-channel stats.
__global__ void __launch_bounds__(kRedBlock) pcg_finish(const ChanState* __restrict__ cs_in,
                                                         ChanState* __restrict__ cs_out,
                                                         const double* __restrict__ part,
                                                         const double* __restrict__ sums, int C,
                                                         int G, int max_iters, double tol,
                                                         bs_chan_stats* __restrict__ out) {
    __shared__ double fin[3 * BS_MAX_CHANNELS];
    const int t = threadIdx.x;
    reduce_partials<3>(part, C, G, fin, sums);
    if (t < C) {
        ChanState st = cs_in[t];
        advance_state(st, fin[t], fin[C + t], fin[2 * C + t], max_iters, tol);
        cs_out[t] = st;
        if (out) {
            bs_chan_stats o;
            o.iters = st.iters;
            o.reason = st.reason;
            o.rel_residual = st.res;
            o.bnorm = st.bnorm;
            out[t] = o;
        }
    }
}

// x[c][p] = y[idx[p]][c].
__global__ void __launch_bounds__(kBlock) slice_kernel(const int32_t* __restrict__ idx,
                                                        const float* __restrict__ y, int C, int P,
                                                        float* __restrict__ x) {
    const XcdTiles tl((P + kBlock - 1) / kBlock);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int p = (int)(tile * kBlock) + threadIdx.x;
        if (p >= P) continue;
        const int64_t v = idx[p];
        for (int c = 0; c < C; ++c) x[(int64_t)c * P + p] = y[v * C + c];
    }
}

// dL/dt[c][p] = conf[p] g[idx[p]][c];  dL/dconf[p] = sum_c g[idx][c] (t[c][p] - y[idx][c]).
__global__ void __launch_bounds__(kBlock) grad_scatter(const int32_t* __restrict__ idx,
                                                        const float* __restrict__ g,
                                                        const float* __restrict__ yhat,
                                                        const float* __restrict__ target,
                                                        const float* __restrict__ conf, int C,
                                                        int P, float* __restrict__ gt,
                                                        float* __restrict__ gc) {
    const XcdTiles tl((P + kBlock - 1) / kBlock);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int p = (int)(tile * kBlock) + threadIdx.x;
        if (p >= P) continue;
        const int64_t v = idx[p];
        const float cp = conf[p];
        float s = 0.0f;
        for (int c = 0; c < C; ++c) {
            const float gv = g[v * C + c];
            gt[(int64_t)c * P + p] = cp * gv;
            s += gv * (target[(int64_t)c * P + p] - yhat[v * C + c]);
        }
        gc[p] = s;
    }
}

// ---------------------------------------------------------------------------
// Host sequencing.
// ---------------------------------------------------------------------------
static bs_status validate_solve(const bs_grid* grid, int C, const bs_solve_params* p) {
    if (!grid || impl(grid)->magic != kGridMagic) return fail(BS_EINVAL, "grid was not built");
    if (!impl(grid)->bistochastized) return fail(BS_EINVAL, "grid was not bistochastized");
    if (C < 1 || C > BS_MAX_CHANNELS) return fail(BS_EINVAL, "channel count must be in 1..64");
    if (!p) return fail(BS_EINVAL, "solve params is NULL");
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

static bool misaligned(const void* p) { return ((uintptr_t)p & 3) != 0; }

// Initial state into `y` from the right-hand side already splatted into w.b.
static bs_status run_init(const GridImpl& g, const SolveWs& w, const bs_solve_params& p,
                          float* y, hipStream_t s) {
    const int C = w.C;
    const int blocks = grid_blocks(ceil_div(g.vcap * C, kBlock));
    if (p.init == BS_INIT_FLAT) {
        BS_LAUNCH(s, K_INIT, "flat_init", flat_init_kernel, dim3(blocks), dim3(kBlock), 0, s, w.b, w.sc, C,
                           g.counts, y);
        return BS_OK;
    }
    for (int k = 1; k < g.levels; ++k) {
        const int bk = grid_blocks(ceil_div(g.lv[k].cap * (C + 1), kBlock));
        BS_LAUNCH(s, K_INIT, "pyr_up", pyr_up, dim3(bk), dim3(kBlock), 0, s, g.lv[k].ptr, g.lv[k].list, w.b,
                           w.sc, (const float*)(k >= 2 ? w.up[k - 1] : nullptr), w.up[k], C, k,
                           g.counts);
    }
    for (int k = g.levels - 1; k >= 1; --k) {
        const int bk = grid_blocks(ceil_div(g.lv[k].cap * (C + 1), kBlock));
        const float wk = (float)std::pow((double)p.init_alpha, -((double)p.init_beta + k));
        const float* upp = (k + 1 < g.levels) ? w.up[k + 1] : nullptr;
        const int32_t* par = (k + 1 < g.levels) ? g.lv[k + 1].item_parent : nullptr;
        BS_LAUNCH(s, K_INIT, "pyr_down", pyr_down, dim3(bk), dim3(kBlock), 0, s, w.up[k], upp, par,
                           g.lv[k].ones, wk, C, k, g.counts);
    }
    const int32_t* par0 = g.levels > 1 ? g.lv[1].item_parent : nullptr;
    const float* up1 = g.levels > 1 ? w.up[1] : nullptr;
    BS_LAUNCH(s, K_INIT, "hier_final", hier_final, dim3(blocks), dim3(kBlock), 0, s, w.b, w.sc, up1, par0, C,
                       g.counts, y);
    return BS_OK;
}

// PCG on A y = w.b from the state already in y.
static bs_status run_pcg(const GridImpl& g, const SolveWs& w, const bs_solve_params& p,
                         float* y, bs_chan_stats* stats, hipStream_t s) {
    const int C = w.C;
    // Consumers reduce up to 8 (value, channel) partial rows themselves; above
    // that a pcg_reduce launch does it once.
    const bool sep = !PartialSums::fits(3 * C, w.G);
    const double* s0 = sep ? w.sums[0] : nullptr;
    const double* s1 = sep ? w.sums[1] : nullptr;
    const int nstate = w.G * C;
    BS_LAUNCH(s, K_INIT, "solve_prologue", solve_prologue, dim3((nstate + 255) / 256),
              dim3(256), 0, s, w.cs[0], w.cs[1], nstate, w.ctl);
    BS_LAUNCH(s, K_PCG_START, "pcg_start", pcg_start, dim3(w.G), dim3(kRedBlock), 0, s,
              g.nbr, g.vcap, g.nf, w.sc, w.minv, w.b, y, w.r, p.lambda, C, w.vpb, g.counts,
              w.part[0]);
    if (sep)
        BS_LAUNCH(s, K_PCG_REDUCE, "pcg_reduce", pcg_reduce, dim3(3 * C), dim3(kRedBlock), 0, s,
                  w.part[0], w.sums[0], w.G);
    for (int it = 0; it < p.max_iters; ++it) {
        float* dn = w.d[it & 1];
        const float* dold = w.d[(it + 1) & 1];
        BS_LAUNCH(s, K_PCG_MATVEC, "pcg_matvec", pcg_matvec, dim3(w.G), dim3(kRedBlock), 0,
                  s, g.nbr, g.vcap, g.nf, w.sc, w.minv, w.r, dold, dn, w.q, p.lambda, C, w.vpb,
                  g.counts, w.cs[0], w.cs[1], w.part[0], s0, w.part[1], w.ctl, p.max_iters,
                  p.rel_tol);
        if (sep)
            BS_LAUNCH(s, K_PCG_REDUCE, "pcg_reduce", pcg_reduce, dim3(C), dim3(kRedBlock), 0, s,
                      w.part[1], w.sums[1], w.G);
        BS_LAUNCH(s, K_PCG_UPDATE, "pcg_update", pcg_update, dim3(w.G), dim3(kRedBlock), 0,
                  s, w.minv, dn, w.q, y, w.r, C, w.vpb, g.counts, w.cs[1], w.cs[0], w.part[1], s1,
                  w.part[0], w.ctl);
        if (sep)
            BS_LAUNCH(s, K_PCG_REDUCE, "pcg_reduce", pcg_reduce, dim3(3 * C), dim3(kRedBlock), 0,
                      s, w.part[0], w.sums[0], w.G);
        if (p.check_every > 0 && (it + 1) % p.check_every == 0 && it + 1 < p.max_iters) {
            int32_t active = 0;
            BS_TRY_HIP(hipMemcpyAsync(&active, w.ctl + CTL_ACTIVE, sizeof(int32_t),
                                      hipMemcpyDeviceToHost, s));
            BS_TRY_HIP(hipStreamSynchronize(s));
            if (active == 0) break;
        }
    }
    BS_LAUNCH(s, K_INIT, "pcg_finish", pcg_finish, dim3(1), dim3(kRedBlock), 0, s, w.cs[0],
              w.cs[1], w.part[0], s0, C, w.G, p.max_iters, p.rel_tol, stats);
    return BS_OK;
}

}  // namespace bs

using namespace bs;

extern "C" size_t bs_solve_workspace_bytes(const bs_grid* grid, int32_t C) {
    if (!grid || impl(grid)->magic != kGridMagic || C < 1 || C > BS_MAX_CHANNELS) return 0;
    SolveWs w;
    return layout_solve(*impl(grid), C, nullptr, w);
}

extern "C" bs_status bs_solve_ws_view(const bs_grid* grid, int32_t C, void* ws, size_t ws_bytes,
                                      const float** b, const float** sc, const float** diag,
                                      const float** minv) {
    if (!grid || impl(grid)->magic != kGridMagic || C < 1 || C > BS_MAX_CHANNELS)
        return fail(BS_EINVAL, "bad grid or channel count");
    SolveWs w;
    if (ws_bytes < layout_solve(*impl(grid), C, nullptr, w)) return fail(BS_EWORKSPACE, "workspace too small");
    layout_solve(*impl(grid), C, ws, w);
    if (b) *b = w.b;
    if (sc) *sc = w.sc;
    if (diag) *diag = w.diag;
    if (minv) *minv = w.minv;
    return BS_OK;
}

extern "C" bs_status bs_solve(const bs_grid* grid, const float* target, const float* conf,
                              int32_t C, const bs_solve_params* params, float* y, void* ws,
                              size_t ws_bytes, bs_chan_stats* stats, void* stream) {
    bs_status st = validate_solve(grid, C, params);
    if (st != BS_OK) return st;
    if (!target || !conf || !y || !ws) return fail(BS_EINVAL, "NULL pointer argument");
    if (misaligned(target) || misaligned(conf) || misaligned(y) || ((uintptr_t)ws & 255))
        return fail(BS_EINVAL, "misaligned buffer");
    const GridImpl& g = *impl(grid);
    SolveWs w;
    const size_t need = layout_solve(g, C, nullptr, w);
    if (ws_bytes < need)
        return fail(BS_EWORKSPACE, "solve workspace needs " + std::to_string(need) + " bytes");
    layout_solve(g, C, ws, w);
    hipStream_t s = (hipStream_t)stream;
    const bs_solve_params& p = *params;

    st = launch_splat<true>(g, conf, target, C, (double)p.lambda, w.sc, w.diag, w.minv, w.b, s);
    if (st != BS_OK) return st;
    st = run_init(g, w, p, y, s);
    if (st != BS_OK) return st;
    st = run_pcg(g, w, p, y, stats, s);
    if (st != BS_OK) return st;
    return BS_OK;
}

extern "C" bs_status bs_slice(const bs_grid* grid, const float* y, int32_t C, float* x,
                              void* stream) {
    if (!grid || impl(grid)->magic != kGridMagic) return fail(BS_EINVAL, "grid was not built");
    if (C < 1 || C > BS_MAX_CHANNELS) return fail(BS_EINVAL, "channel count must be in 1..64");
    if (!y || !x) return fail(BS_EINVAL, "NULL pointer argument");
    if (misaligned(y) || misaligned(x)) return fail(BS_EINVAL, "misaligned buffer");
    const GridImpl& g = *impl(grid);
    hipStream_t s = (hipStream_t)stream;
    const int blocks = grid_blocks(ceil_div(g.P, kBlock));
    BS_LAUNCH(s, K_SLICE, "slice", slice_kernel, dim3(blocks), dim3(kBlock), 0, s, g.lv[0].item_parent, y, C,
                       g.P, x);
    return BS_OK;
}

extern "C" bs_status bs_solve_backward(const bs_grid* grid, const float* target, const float* conf,
                                       const float* y_hat, const float* grad_x, int32_t C,
                                       const bs_solve_params* params, float* grad_t,
                                       float* grad_c, float* g_out, void* ws, size_t ws_bytes,
                                       bs_chan_stats* stats, void* stream) {
    bs_status st = validate_solve(grid, C, params);
    if (st != BS_OK) return st;
    if (!target || !conf || !y_hat || !grad_x || !grad_t || !grad_c || !ws)
        return fail(BS_EINVAL, "NULL pointer argument");
    if (misaligned(target) || misaligned(conf) || misaligned(y_hat) || misaligned(grad_x) ||
        misaligned(grad_t) || misaligned(grad_c) || (g_out && misaligned(g_out)) ||
        ((uintptr_t)ws & 255))
        return fail(BS_EINVAL, "misaligned buffer");
    const GridImpl& g = *impl(grid);
    SolveWs w;
    const size_t need = layout_solve(g, C, nullptr, w);
    if (ws_bytes < need)
        return fail(BS_EWORKSPACE, "solve workspace needs " + std::to_string(need) + " bytes");
    layout_solve(g, C, ws, w);
    hipStream_t s = (hipStream_t)stream;
    const bs_solve_params& p = *params;
    float* gb = g_out ? g_out : w.g;

    st = launch_splat<false>(g, conf, grad_x, C, (double)p.lambda, w.sc, w.diag, w.minv, w.b,
                             s);
    if (st != BS_OK) return st;
    st = run_init(g, w, p, gb, s);
    if (st != BS_OK) return st;
    st = run_pcg(g, w, p, gb, stats, s);
    if (st != BS_OK) return st;
    const int pblocks = grid_blocks(ceil_div(g.P, kBlock));
    BS_LAUNCH(s, K_GRAD_SCATTER, "grad_scatter", grad_scatter, dim3(pblocks), dim3(kBlock), 0, s, g.lv[0].item_parent, gb,
                       y_hat, target, conf, C, g.P, grad_t, grad_c);
    return BS_OK;
}
