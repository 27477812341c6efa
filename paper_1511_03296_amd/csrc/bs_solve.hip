// The bilateral-space solve (paper Eq. quad_min and Eq. solution, supplement
// Algorithm 2, Section 4 initialisation) and its backward pass (Section 3).
//
// Layouts: pixel planes [C][P] float32; bilateral-space vectors [V][C]
// float32, channels contiguous per vertex.  A thread of the vertex kernels
// owns one (vertex, channel) element: a block covers vpb = 256 / C vertices of
// all C channels, so the neighbour table is read once per vertex and the
// channel gathers of one neighbour are contiguous.
//
// PCG runs one independent PCG per channel.  One iteration is two kernels:
//   dir_matvec:  d = M^-1 r + beta d  (fused; the neighbours' new d values are
//                recomputed from r and the previous d, so no separate
//                direction pass is needed),  q = A d,  partial d^T q;
//   update:      y += alpha d,  r -= alpha q,  partial r^T M^-1 r and r^T r.
// Dot products accumulate in float64; each kernel's last block reduces the
// per-block partials in a fixed order and updates the per-channel scalars,
// so results are deterministic and no host synchronisation is needed.
#include "bs_internal.h"

namespace bs {

struct ChanState {
    double rho, alpha, beta, bnorm, res;
    int32_t active, iters, reason, phase;   // phase 0: initial residual not yet reduced
};

enum Ctl : int { CTL_ACTIVE = 0, CTL_SIZE = 8 };

// Partials of the reducing kernels: [2 slots][3 values][C][kRedGrid].
//   slot 0 -- written by pcg_start (r^T r, b^T b, r^T M^-1 r) and by
//             pcg_update (r^T r, 0, r^T M^-1 r);
//   slot 1 -- written by pcg_dir_matvec (d^T q).
// Per-channel state, double-buffered the same way: pcg_dir_matvec reads
// state 0 and writes state 1, pcg_update reads state 1 and writes state 0.
struct SolveWs {
    int C, vpb;
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
    int32_t* ctl;
    size_t bytes;
};

static size_t layout_solve(const GridImpl& g, int C, void* base, SolveWs& w) {
    w.C = C;
    w.vpb = kRedBlock / C;
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
    w.cs[0] = c.take<ChanState>(C);
    w.cs[1] = c.take<ChanState>(C);
    w.part[0] = c.take<double>((int64_t)3 * C * kRedGrid);
    w.part[1] = c.take<double>((int64_t)3 * C * kRedGrid);
    w.ctl = c.take<int32_t>(CTL_SIZE);
    w.bytes = align_up(c.off, 256);
    return w.bytes;
}

// ---------------------------------------------------------------------------
// Reductions over (vertex, channel) blocks.
// ---------------------------------------------------------------------------

// Sums NV per-thread values over the vertices of the block, per channel, with
// a fixed tree, and writes the block's partials to part[(k C + ch) G + block].
template <int NV>
__device__ inline void block_channel_partials(const double (&acc)[NV], int C, int vpb,
                                              double* __restrict__ part) {
    const int t = threadIdx.x;
    if (C == 1) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            const double v = block_sum<kRedBlock>(acc[k]);
            if (t == 0) part[(int64_t)k * kRedGrid + blockIdx.x] = v;
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
        for (int k = 0; k < NV; ++k) part[((int64_t)k * C + t) * kRedGrid + blockIdx.x] = s[k][t];
    }
}

// out[k C + ch] = sum over the kRedGrid blocks of the producer's partials,
// computed identically by every block: one wave per (k, ch) pair, lanes
// striding over blocks, then a shuffle tree.
template <int NV>
__device__ inline void reduce_partials(const double* __restrict__ part, int C, double* out) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int pair = wave; pair < NV * C; pair += kRedBlock / 64) {
        double s = 0.0;
        for (int b = lane; b < kRedGrid; b += 64) s += part[(int64_t)pair * kRedGrid + b];
        s = wave_sum(s);
        if (lane == 0) out[pair] = s;
    }
    __syncthreads();
}

// Completes the previous PCG step for every channel from the slot-0 partials:
// the initial residual (phase 0) or the end of an iteration (stopping rule).
__device__ inline void advance_state(ChanState& st, double rr, double bb, double rho_new,
                                     int max_iters, double tol) {
    if (st.phase == 0) {
        st.phase = 1;
        st.bnorm = sqrt(bb);
        st.rho = rho_new;
        st.beta = 0.0;
        st.iters = 0;
        st.active = 0;
        if (bb == 0.0) {
            st.reason = 5;
            st.res = 0.0;
        } else {
            st.res = sqrt(rr) / st.bnorm;
            if (st.res <= tol) st.reason = 1;
            else if (max_iters <= 0) st.reason = 2;
            else if (rho_new == 0.0) st.reason = 3;
            else {
                st.active = 1;
                st.reason = 0;
            }
        }
        return;
    }
    if (!st.active) return;
    st.beta = rho_new / st.rho;
    st.rho = rho_new;
    st.iters += 1;
    st.res = sqrt(rr) / st.bnorm;
    int reason = 0;
    if (st.res <= tol) reason = 1;
    else if (st.iters >= max_iters) reason = 2;
    else if (rho_new == 0.0) reason = 3;
    if (reason) {
        st.active = 0;
        st.reason = reason;
    }
}

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------

__global__ void solve_prologue(ChanState* cs0, ChanState* cs1, int C, int32_t* ctl) {
    const int t = threadIdx.x;
    if (t < CTL_SIZE) ctl[t] = 0;
    for (int c = t; c < C; c += blockDim.x) {
        ChanState z;
        z.rho = z.alpha = z.beta = z.bnorm = z.res = 0.0;
        z.active = z.iters = z.reason = z.phase = 0;
        cs0[c] = z;
        cs1[c] = z;
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

// r = b - A y0 for one (vertex, channel) element per thread, with
// A z = diag(A) z_v - lam n_v sum_j n_j z_j; partials r^T r, b^T b, r^T M^-1 r.
__global__ void __launch_bounds__(kRedBlock) pcg_start(
    const int32_t* __restrict__ nbr, int64_t vcap, const float* __restrict__ nf,
    const float* __restrict__ diag, const float* __restrict__ minv, const float* __restrict__ b,
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
        float ns = 0.0f;
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            const int u = nbr[j * vcap + v];
            if (u >= 0) ns += nf[u] * y[(int64_t)u * C + ch];
        }
        const int64_t e = (int64_t)v * C + ch;
        const float ay = diag[v] * y[e] - lam * nf[v] * ns;
        const float bv = b[e];
        const float rv = bv - ay;
        r[e] = rv;
        acc[0] += (double)rv * (double)rv;
        acc[1] += (double)bv * (double)bv;
        acc[2] += (double)rv * (double)(minv[v] * rv);
    }
    block_channel_partials<3>(acc, C, vpb, part);
}

// Prologue: finish the previous step from the slot-0 partials (stopping rule,
// beta).  Then  d = M^-1 r + beta d_old  (beta = 0 on the first iteration),
// q = A d  and partials of d^T q.
__global__ void __launch_bounds__(kRedBlock) pcg_dir_matvec(
    const int32_t* __restrict__ nbr, int64_t vcap, const float* __restrict__ nf,
    const float* __restrict__ diag, const float* __restrict__ minv, const float* __restrict__ r,
    const float* __restrict__ dold, float* __restrict__ dnew, float* __restrict__ q, float lam,
    int C, int vpb, const int32_t* __restrict__ counts, const ChanState* __restrict__ cs_in,
    ChanState* __restrict__ cs_out, const double* __restrict__ part_in,
    double* __restrict__ part_out, int32_t* __restrict__ ctl, int max_iters, double tol) {
    __shared__ ChanState S[BS_MAX_CHANNELS];
    __shared__ double fin[3 * BS_MAX_CHANNELS];
    __shared__ int n_active;
    const int t = threadIdx.x;
    reduce_partials<3>(part_in, C, fin);
    if (t == 0) n_active = 0;
    __syncthreads();
    if (t < C) {
        ChanState st = cs_in[t];
        advance_state(st, fin[t], fin[C + t], fin[2 * C + t], max_iters, tol);
        S[t] = st;
        if (st.active) atomicAdd(&n_active, 1);
        if (blockIdx.x == 0) cs_out[t] = st;
    }
    __syncthreads();
    if (blockIdx.x == 0 && t == 0) ctl[CTL_ACTIVE] = n_active;
    if (n_active == 0) return;
    const int V = counts[CNT_V];
    const int vl = t / C, ch = t - vl * C;
    const bool lane_ok = vl < vpb;
    const ChanState st = S[lane_ok ? ch : 0];
    const bool act = lane_ok && st.active;
    const bool first = st.iters == 0;
    const float beta = (float)st.beta;
    double acc[1] = {0.0};
    const XcdTiles tl((V + vpb - 1) / vpb);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int v = (int)(tile * vpb) + vl;
        if (!act || v >= V) continue;
        float ns = 0.0f;
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            const int u = nbr[j * vcap + v];
            if (u >= 0) {
                const int64_t eu = (int64_t)u * C + ch;
                float du = minv[u] * r[eu];
                if (!first) du += beta * dold[eu];
                ns += nf[u] * du;
            }
        }
        const int64_t e = (int64_t)v * C + ch;
        float dv = minv[v] * r[e];
        if (!first) dv += beta * dold[e];
        const float qv = diag[v] * dv - lam * nf[v] * ns;
        dnew[e] = dv;
        q[e] = qv;
        acc[0] += (double)dv * (double)qv;
    }
    block_channel_partials<1>(acc, C, vpb, part_out);
}

// Prologue: alpha = r^T M^-1 r / d^T q from the slot-1 partials (a channel
// with d^T q <= 0 stops).  Then  y += alpha d,  r -= alpha q  and partials of
// r^T r and r^T M^-1 r.
__global__ void __launch_bounds__(kRedBlock) pcg_update(
    const float* __restrict__ minv, const float* __restrict__ d, const float* __restrict__ q,
    float* __restrict__ y, float* __restrict__ r, int C, int vpb,
    const int32_t* __restrict__ counts, const ChanState* __restrict__ cs_in,
    ChanState* __restrict__ cs_out, const double* __restrict__ part_in,
    double* __restrict__ part_out, int32_t* __restrict__ ctl) {
    __shared__ ChanState S[BS_MAX_CHANNELS];
    __shared__ double fin[BS_MAX_CHANNELS];
    __shared__ int n_active;
    const int t = threadIdx.x;
    reduce_partials<1>(part_in, C, fin);
    if (t == 0) n_active = 0;
    __syncthreads();
    if (t < C) {
        ChanState st = cs_in[t];
        if (st.active) {
            const double dq = fin[t];
            if (!(dq > 0.0)) {
                st.active = 0;
                st.reason = 4;
            } else {
                st.alpha = st.rho / dq;
            }
        }
        S[t] = st;
        if (st.active) atomicAdd(&n_active, 1);
        if (blockIdx.x == 0) cs_out[t] = st;
    }
    __syncthreads();
    if (blockIdx.x == 0 && t == 0) ctl[CTL_ACTIVE] = n_active;
    if (n_active == 0) return;
    const int V = counts[CNT_V];
    const int vl = t / C, ch = t - vl * C;
    const bool lane_ok = vl < vpb;
    const ChanState st = S[lane_ok ? ch : 0];
    const bool act = lane_ok && st.active;
    const float alpha = (float)st.alpha;
    double acc[3] = {0.0, 0.0, 0.0};
    const XcdTiles tl((V + vpb - 1) / vpb);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int v = (int)(tile * vpb) + vl;
        if (!act || v >= V) continue;
        const int64_t e = (int64_t)v * C + ch;
        y[e] += alpha * d[e];
        const float rv = r[e] - alpha * q[e];
        r[e] = rv;
        acc[0] += (double)rv * (double)rv;
        acc[2] += (double)rv * (double)(minv[v] * rv);
    }
    block_channel_partials<3>(acc, C, vpb, part_out);
}

// After the last enqueued iteration (single block): completes the pending
// step from the slot-0 partials and writes the per-channel stats.
__global__ void __launch_bounds__(kRedBlock) pcg_finish(ChanState* __restrict__ cs,
                                                         const double* __restrict__ part, int C,
                                                         int max_iters, double tol,
                                                         bs_chan_stats* __restrict__ out) {
    __shared__ double fin[3 * BS_MAX_CHANNELS];
    const int t = threadIdx.x;
    reduce_partials<3>(part, C, fin);
    if (t < C) {
        ChanState st = cs[t];
        advance_state(st, fin[t], fin[C + t], fin[2 * C + t], max_iters, tol);
        cs[t] = st;
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
    BS_LAUNCH(s, K_INIT, "solve_prologue", solve_prologue, dim3(1), dim3(64), 0, s, w.cs[0],
              w.cs[1], C, w.ctl);
    BS_LAUNCH(s, K_PCG_START, "pcg_start", pcg_start, dim3(kRedGrid), dim3(kRedBlock), 0, s,
              g.nbr, g.vcap, g.nf, w.diag, w.minv, w.b, y, w.r, p.lambda, C, w.vpb, g.counts,
              w.part[0]);
    for (int it = 0; it < p.max_iters; ++it) {
        float* dn = w.d[it & 1];
        const float* dold = w.d[(it + 1) & 1];
        BS_LAUNCH(s, K_PCG_DIR_MATVEC, "pcg_dir_matvec", pcg_dir_matvec, dim3(kRedGrid),
                  dim3(kRedBlock), 0, s, g.nbr, g.vcap, g.nf, w.diag, w.minv, w.r, dold, dn, w.q,
                  p.lambda, C, w.vpb, g.counts, w.cs[0], w.cs[1], w.part[0], w.part[1], w.ctl,
                  p.max_iters, p.rel_tol);
        BS_LAUNCH(s, K_PCG_UPDATE, "pcg_update", pcg_update, dim3(kRedGrid), dim3(kRedBlock), 0,
                  s, w.minv, dn, w.q, y, w.r, C, w.vpb, g.counts, w.cs[1], w.cs[0], w.part[1],
                  w.part[0], w.ctl);
        if (p.check_every > 0 && (it + 1) % p.check_every == 0 && it + 1 < p.max_iters) {
            int32_t active = 0;
            BS_TRY_HIP(hipMemcpyAsync(&active, w.ctl + CTL_ACTIVE, sizeof(int32_t),
                                      hipMemcpyDeviceToHost, s));
            BS_TRY_HIP(hipStreamSynchronize(s));
            if (active == 0) break;
        }
    }
    BS_LAUNCH(s, K_INIT, "pcg_finish", pcg_finish, dim3(1), dim3(kRedBlock), 0, s, w.cs[0],
              w.part[0], C, p.max_iters, p.rel_tol, stats);
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

    const int vblocks = grid_blocks(ceil_div(g.vcap, kBlock));
    BS_LAUNCH(s, K_SPLAT, "splat", splat_kernel<true>, dim3(vblocks), dim3(kBlock), 0, s, g.lv[0].ptr,
                       g.lv[0].list, conf, target, C, g.P, g.nn, (double)p.lambda, g.counts,
                       w.sc, w.diag, w.minv, w.b);
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

    const int vblocks = grid_blocks(ceil_div(g.vcap, kBlock));
    BS_LAUNCH(s, K_SPLAT, "splat_grad", splat_kernel<false>, dim3(vblocks), dim3(kBlock), 0, s, g.lv[0].ptr,
                       g.lv[0].list, conf, grad_x, C, g.P, g.nn, (double)p.lambda, g.counts,
                       w.sc, w.diag, w.minv, w.b);
    st = run_init(g, w, p, gb, s);
    if (st != BS_OK) return st;
    st = run_pcg(g, w, p, gb, stats, s);
    if (st != BS_OK) return st;
    const int pblocks = grid_blocks(ceil_div(g.P, kBlock));
    BS_LAUNCH(s, K_GRAD_SCATTER, "grad_scatter", grad_scatter, dim3(pblocks), dim3(kBlock), 0, s, g.lv[0].item_parent, gb,
                       y_hat, target, conf, C, g.P, grad_t, grad_c);
    return BS_OK;
}
