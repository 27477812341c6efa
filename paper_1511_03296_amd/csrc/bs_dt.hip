// The domain-transform post-process of the solver's output (Section 4, the
// post-processing paragraph: spatial and range bandwidths sigma'_xy and
// sigma'_rgb) and the edge-aware variance that sets the robust solver's
// initial confidence (supplement Section Robustness, the equations for V and
// c_init).  The filter is the recursive formulation of Gastal and Oliveira's
// domain transform:
//   - neighbouring samples of a line lie d = 1 + (s_s / s_r) sum_c |dI_c| apart
//     in the transformed domain, dI the difference of the guide's 8-bit RGB
//     codes across the edge between them;
//   - a pass runs J[x] = (1 - w) I[x] + w J[x-1], w = a^d, a = exp(-sqrt2 / sigma),
//     along the line, then the same recursion backwards on its output; the
//     first sample in each direction passes unchanged;
//   - N iterations each run a horizontal then a vertical pass, iteration i
//     (1-based) with sigma_i = s_s sqrt(3) 2^(N-i) / sqrt(4^N - 1).
//
// A recursion is a chain of affine maps y -> w y + (1 - w) I, so runs of it
// compose into one map (A, B) and a line is filtered by a scan of maps:
//   - horizontal pass: one wave per image row and channel; a chunk of 64 x M
//     samples gives each lane M consecutive samples, whose composed map the
//     wave scans (six shuffle steps), and every lane then replays its samples
//     from the value entering its run;
//   - vertical pass: a block per 16 columns of a channel, its 64 segments of
//     rows one thread row each; segment maps meet in LDS, every thread composes
//     the maps of the segments before its own (after its own, backwards) and
//     replays its segment.  Lanes run along rows, so every load and store of a
//     wave covers four 64-byte row pieces (with 32 columns per block, whole
//     128-byte lines, the pass was 20 % slower for lack of blocks).
// The domain distances are computed once per call: 16-bit sums of absolute
// code differences (at most 765) to the left and upper neighbour, one 32-bit
// word per pixel.  A sample reads its own word (the distance of the edge
// behind it) or the next sample's (the edge ahead of it).  Every pass reads
// and writes a sample in the same thread, forwards and backwards, so passes
// need no synchronisation beyond the kernel boundary and the LDS exchange.
#include "bs_grid_ops.h"

namespace bs {

constexpr int kDtRowM = 16;         // samples per lane and chunk of a row (1024 per chunk)
constexpr int kDtRowBlock = 256;    // 4 waves, one row each
constexpr int kDtColW = 16;         // columns per block of the vertical pass
constexpr int kDtColBlock = 1024;   // threads per block of the vertical pass
constexpr int kDtSegs = kDtColBlock / kDtColW;   // row segments per block
constexpr int kDtMaxIters = 16;

// Feedback coefficient a^d of an edge whose colour distance is `dist`:
// exp2(k d), k = -sqrt(2) log2(e) / sigma, d = 1 + ratio dist.
__device__ inline float dt_weight(uint32_t dist, float k, float ratio) {
    return exp2f(k * fmaf(ratio, (float)dist, 1.0f));
}

// Domain distances of every pixel: low half the edge to the left neighbour,
// high half the edge to the upper one (0 where there is none).
__global__ void __launch_bounds__(kBlock) dt_steps(const float* __restrict__ ref, int H, int W,
                                                   uint32_t* __restrict__ dist) {
    const int64_t P = (int64_t)H * W;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < P;
         p += (int64_t)gridDim.x * kBlock) {
        const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
        uint32_t dh = 0, dv = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float* ch = ref + c * P;
            const int q = quantise8(ch[p]);
            if (x > 0) dh += (uint32_t)abs(q - quantise8(ch[p - 1]));
            if (y > 0) dv += (uint32_t)abs(q - quantise8(ch[p - W]));
        }
        dist[p] = dh | (dv << 16);
    }
}

// Composition: `m` applied after (A, B).
__device__ inline void dt_after(float& A, float& B, float mA, float mB) {
    B = fmaf(mA, B, mB);
    A = mA * A;
}

// Horizontal pass of one iteration over every row of every channel:
// src -> dst (src == dst allowed).
__global__ void __launch_bounds__(kDtRowBlock) dt_rows(const float* src, float* dst,
                                                       const uint32_t* __restrict__ dist,
                                                       int H, int W, int C, float k,
                                                       float ratio) {
    constexpr int M = kDtRowM;
    const int lane = threadIdx.x & 63;
    const int64_t lines = (int64_t)C * H;
    const int64_t chunk = 64 * M;
    const int nchunks = (int)((W + chunk - 1) / chunk);
    for (int64_t line = (int64_t)blockIdx.x * (kDtRowBlock / 64) + (threadIdx.x >> 6);
         line < lines; line += (int64_t)gridDim.x * (kDtRowBlock / 64)) {
        const int y = (int)(line % H);
        const float* in = src + line * W;
        float* out = dst + line * W;
        const uint32_t* drow = dist + (int64_t)y * W;
        // left to right
        float carry = 0.0f;
        float v[M], w[M];
        for (int ci = 0; ci < nchunks; ++ci) {
            const int e0 = ci * (int)chunk + lane * M;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const int e = e0 + j;
                // beyond the row: the identity map; the first sample: w = 0
                v[j] = e < W ? in[e] : 0.0f;
                w[j] = e >= W ? 1.0f : (e == 0 ? 0.0f : dt_weight(drow[e] & 0xffffu, k, ratio));
            }
            float A = 1.0f, B = 0.0f;
#pragma unroll
            for (int j = 0; j < M; ++j) dt_after(A, B, w[j], (1.0f - w[j]) * v[j]);
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const float pA = __shfl_up(A, o), pB = __shfl_up(B, o);
                if (lane >= o) {
                    B = fmaf(A, pB, B);
                    A = A * pA;
                }
            }
            float eA = __shfl_up(A, 1), eB = __shfl_up(B, 1);
            if (lane == 0) {
                eA = 1.0f;
                eB = 0.0f;
            }
            float yv = fmaf(eA, carry, eB);
#pragma unroll
            for (int j = 0; j < M; ++j) {
                yv = fmaf(w[j], yv, (1.0f - w[j]) * v[j]);
                v[j] = yv;
                // the last chunk's outputs stay in v for the backward recursion
                if (ci + 1 < nchunks && e0 + j < W) out[e0 + j] = yv;
            }
            carry = __shfl(yv, 63);
        }
        // right to left over the forward pass's output: the last chunk is still
        // in registers (outputs in v, forward weights in w), earlier chunks are
        // read back (written by this lane)
        carry = 0.0f;
        for (int ci = nchunks - 1; ci >= 0; --ci) {
            const int e0 = ci * (int)chunk + lane * M;
            float wb[M];
            if (ci == nchunks - 1) {
                // the edge ahead of a sample is the forward weight of the next
                const float next0 = __shfl_down(w[0], 1);
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    const int e = e0 + j;
                    wb[j] = e >= W ? 1.0f : (e + 1 == W ? 0.0f : (j + 1 < M ? w[j + 1] : next0));
                }
            } else {
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    const int e = e0 + j;
                    // the edge ahead (e, e+1); the last sample: w = 0
                    v[j] = e < W ? out[e] : 0.0f;
                    wb[j] = e >= W ? 1.0f
                                   : (e + 1 == W ? 0.0f
                                                 : dt_weight(drow[e + 1] & 0xffffu, k, ratio));
                }
            }
            float A = 1.0f, B = 0.0f;
#pragma unroll
            for (int j = M - 1; j >= 0; --j) dt_after(A, B, wb[j], (1.0f - wb[j]) * v[j]);
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const float pA = __shfl_down(A, o), pB = __shfl_down(B, o);
                if (lane + o < 64) {
                    B = fmaf(A, pB, B);
                    A = A * pA;
                }
            }
            float eA = __shfl_down(A, 1), eB = __shfl_down(B, 1);
            if (lane == 63) {
                eA = 1.0f;
                eB = 0.0f;
            }
            float yv = fmaf(eA, carry, eB);
#pragma unroll
            for (int j = M - 1; j >= 0; --j) {
                yv = fmaf(wb[j], yv, (1.0f - wb[j]) * v[j]);
                if (e0 + j < W) out[e0 + j] = yv;
            }
            carry = __shfl(yv, 0);
        }
    }
}

// Rows of a column segment are taken kDtBatch at a time: the loads of a batch
// are issued together, so a segment waits for memory once per batch rather
// than once per row.
constexpr int kDtBatch = 8;

// One column's segment [r0, r1), downwards.  STORE false: compose its map
// into (A, B); STORE true: replay it from `yv`, writing the outputs.
template <bool STORE>
__device__ inline void col_down(float* xc, const uint32_t* dc, int W, int r0, int r1, float k,
                                float ratio, float& A, float& B, float& yv) {
    for (int rb = r0; rb < r1; rb += kDtBatch) {
        float* xb = xc + (int64_t)rb * W;
        const uint32_t* db = dc + (int64_t)rb * W;
        float xv[kDtBatch];
        uint32_t dv[kDtBatch];
#pragma unroll
        for (int j = 0; j < kDtBatch; ++j) {
            const bool ok = rb + j < r1;
            xv[j] = ok ? xb[j * W] : 0.0f;
            dv[j] = ok && rb + j > 0 ? db[j * W] >> 16 : 0u;
        }
#pragma unroll
        for (int j = 0; j < kDtBatch; ++j) {
            if (rb + j < r1) {
                const float w = rb + j == 0 ? 0.0f : dt_weight(dv[j], k, ratio);
                if constexpr (STORE) {
                    yv = fmaf(w, yv, (1.0f - w) * xv[j]);
                    xb[j * W] = yv;
                } else {
                    dt_after(A, B, w, (1.0f - w) * xv[j]);
                }
            }
        }
    }
}

// The same upwards: row r takes the edge (r, r+1); the last row passes.
template <bool STORE>
__device__ inline void col_up(float* xc, const uint32_t* dc, int W, int H, int r0, int r1,
                              float k, float ratio, float& A, float& B, float& yv) {
    for (int rt = r1 - 1; rt >= r0; rt -= kDtBatch) {
        float* xb = xc + (int64_t)rt * W;
        const uint32_t* db = dc + (int64_t)(rt + 1) * W;
        float xv[kDtBatch];
        uint32_t dv[kDtBatch];
#pragma unroll
        for (int j = 0; j < kDtBatch; ++j) {
            const bool ok = rt - j >= r0;
            xv[j] = ok ? xb[-j * W] : 0.0f;
            dv[j] = ok && rt - j + 1 < H ? db[-j * W] >> 16 : 0u;
        }
#pragma unroll
        for (int j = 0; j < kDtBatch; ++j) {
            if (rt - j >= r0) {
                const float w = rt - j + 1 == H ? 0.0f : dt_weight(dv[j], k, ratio);
                if constexpr (STORE) {
                    yv = fmaf(w, yv, (1.0f - w) * xv[j]);
                    xb[-j * W] = yv;
                } else {
                    dt_after(A, B, w, (1.0f - w) * xv[j]);
                }
            }
        }
    }
}

// Vertical pass of one iteration, in place: block (channel, 32-column strip),
// kDtSegs segments of rows per column.
__global__ void __launch_bounds__(kDtColBlock) dt_cols(float* x, const uint32_t* __restrict__ dist,
                                                       int H, int W, int strips, float k,
                                                       float ratio) {
    __shared__ float sA[kDtSegs][kDtColW], sB[kDtSegs][kDtColW];
    const int col_in = threadIdx.x % kDtColW, seg = threadIdx.x / kDtColW;
    const int c = blockIdx.x / strips;
    const int col = (blockIdx.x - c * strips) * kDtColW + col_in;
    const bool live = col < W;
    const int L = (H + kDtSegs - 1) / kDtSegs;
    const int r0 = min(H, seg * L), r1 = min(H, r0 + L);
    float* xc = x + (int64_t)c * H * W + col;
    const uint32_t* dc = dist + col;
    // downwards: the segment's map, then the maps of the segments above it
    float A = 1.0f, B = 0.0f, yv = 0.0f;
    if (live) col_down<false>(xc, dc, W, r0, r1, k, ratio, A, B, yv);
    sA[seg][col_in] = A;
    sB[seg][col_in] = B;
    __syncthreads();
    {
        float cA = 1.0f, cB = 0.0f;
        for (int s = 0; s < seg; ++s) dt_after(cA, cB, sA[s][col_in], sB[s][col_in]);
        yv = cB;   // segment 0 starts with w = 0: the entering value is cB
    }
    if (live) col_down<true>(xc, dc, W, r0, r1, k, ratio, A, B, yv);
    __syncthreads();   // every thread has read the maps
    // upwards over the downward pass's output (written by this thread)
    A = 1.0f;
    B = 0.0f;
    if (live) col_up<false>(xc, dc, W, H, r0, r1, k, ratio, A, B, yv);
    sA[seg][col_in] = A;
    sB[seg][col_in] = B;
    __syncthreads();
    {
        float cA = 1.0f, cB = 0.0f;
        for (int s = kDtSegs - 1; s > seg; --s) dt_after(cA, cB, sA[s][col_in], sB[s][col_in]);
        yv = cB;   // the last segment ends with w = 0
    }
    if (live) col_up<true>(xc, dc, W, H, r0, r1, k, ratio, A, B, yv);
}

constexpr int kDtSumBlocks = 256;

// Per-block float64 partial sums of z [P] (kDtSumBlocks blocks).
__global__ void __launch_bounds__(kBlock) dt_partial_sums(const float* __restrict__ z,
                                                          int64_t P,
                                                          double* __restrict__ part) {
    __shared__ double red[kBlock];
    double s = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < P;
         p += (int64_t)kDtSumBlocks * kBlock)
        s += (double)z[p];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// The two signals of the variance, about the mean mu of z (every block sums
// the partials in the same order): s[0] = z - mu, s[1] = (z - mu)^2.  V is the
// same for every shift mu; the shift keeps the float32 rounding relative to
// the spread of z instead of its offset.
__global__ void __launch_bounds__(kBlock) dt_moments(const float* __restrict__ z, int64_t P,
                                                     const double* __restrict__ part,
                                                     float* __restrict__ s) {
    static_assert(kDtSumBlocks == kBlock, "one partial per thread");
    __shared__ double red[kBlock];
    red[threadIdx.x] = part[threadIdx.x];
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const float mu = (float)(red[0] / (double)P);
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < P;
         p += (int64_t)gridDim.x * kBlock) {
        const float d = z[p] - mu;
        s[p] = d;
        s[P + p] = d * d;
    }
}

// c = exp(-max(DT(s1) - DT(s0)^2, 0) / (2 sigma_dt^2)), 0 in the leftmost
// zero_cols columns.
__global__ void __launch_bounds__(kBlock) dt_conf(const float* __restrict__ s, int H, int W,
                                                  float inv2s2, int zero_cols,
                                                  float* __restrict__ c) {
    const int64_t P = (int64_t)H * W;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < P;
         p += (int64_t)gridDim.x * kBlock) {
        const int x = (int)(p % W);
        const float m1 = s[p];
        const float V = fmaxf(s[P + p] - m1 * m1, 0.0f);
        c[p] = x < zero_cols ? 0.0f : expf(-V * inv2s2);
    }
}

namespace {

struct DtWs {
    uint32_t* dist;
    float* sig;      // [2][P]
    double* part;    // [kDtSumBlocks] partial sums of z
    size_t bytes;
};

DtWs layout_dt(int64_t P, void* base) {
    Carver c(base);
    DtWs w;
    w.dist = c.take<uint32_t>(P);
    w.sig = c.take<float>(2 * P);
    w.part = c.take<double>(kDtSumBlocks);
    w.bytes = align_up(c.off, 256);
    return w;
}

bs_status check_image(const float* ref, int32_t H, int32_t W) {
    if (H < 1 || W < 1) return fail(BS_EINVAL, "image sides must be positive");
    if (H > 65535 || W > 65535) return fail(BS_EUNSUPPORTED, "image side above 65535");
    if ((int64_t)H * W > (int64_t)1 << 30) return fail(BS_EUNSUPPORTED, "image above 2^30 pixels");
    if (!ref) return fail(BS_EINVAL, "NULL pointer argument");
    if (((uintptr_t)ref & 3) != 0) return fail(BS_EINVAL, "misaligned buffer");
    return BS_OK;
}

bs_status check_params(const bs_dt_params* p) {
    if (!p) return fail(BS_EINVAL, "NULL params");
    if (!(p->sigma_s > 0.0f) || !std::isfinite(p->sigma_s) || !(p->sigma_r > 0.0f) ||
        !std::isfinite(p->sigma_r))
        return fail(BS_EINVAL, "sigma_s and sigma_r must be positive and finite");
    if (p->iters < 1 || p->iters > kDtMaxIters)
        return fail(BS_EINVAL, "iters must be in 1.." + std::to_string(kDtMaxIters));
    return BS_OK;
}

bs_status check_ws(void* ws, size_t ws_bytes, int32_t H, int32_t W) {
    const size_t need = bs_dt_workspace_bytes(H, W);
    if (!ws) return fail(BS_EINVAL, "NULL workspace");
    if (((uintptr_t)ws & 255) != 0) return fail(BS_EINVAL, "workspace not 256-byte aligned");
    if (ws_bytes < need)
        return fail(BS_EWORKSPACE, "domain-transform workspace needs " + std::to_string(need) +
                                       " bytes");
    return BS_OK;
}

// The N iterations on `C` planes: src -> dst for the first pass, then in place.
bs_status run_dt(const float* src, float* dst, const uint32_t* dist, int H, int W, int C,
                 const bs_dt_params& p, hipStream_t s) {
    const int N = p.iters;
    const double ratio = (double)p.sigma_s / (double)p.sigma_r;
    const int64_t lines = (int64_t)C * H;
    const int row_blocks =
        (int)std::min<int64_t>(ceil_div(lines, kDtRowBlock / 64), (int64_t)1 << 16);
    const int strips = (int)ceil_div(W, kDtColW);
    for (int i = 1; i <= N; ++i) {
        const double sig = (double)p.sigma_s * std::sqrt(3.0) * std::ldexp(1.0, N - i) /
                           std::sqrt(std::ldexp(1.0, 2 * N) - 1.0);
        const float k = (float)(-std::sqrt(2.0) / sig / std::log(2.0));
        BS_LAUNCH(s, K_DT_ROWS, "dt_rows", dt_rows, dim3(row_blocks), dim3(kDtRowBlock), 0, s,
                  i == 1 ? src : dst, dst, dist, H, W, C, k, (float)ratio);
        BS_LAUNCH(s, K_DT_COLS, "dt_cols", dt_cols, dim3(C * strips), dim3(kDtColBlock), 0, s,
                  dst, dist, H, W, strips, k, (float)ratio);
    }
    return BS_OK;
}

}  // namespace
}  // namespace bs

using namespace bs;

extern "C" size_t bs_dt_workspace_bytes(int32_t H, int32_t W) {
    if (H < 1 || W < 1 || H > 65535 || W > 65535 || (int64_t)H * W > (int64_t)1 << 30) return 0;
    return layout_dt((int64_t)H * W, nullptr).bytes;
}

extern "C" bs_status bs_domain_transform(const float* ref, int32_t H, int32_t W, const float* x,
                                         int32_t C, const bs_dt_params* params, float* out,
                                         void* ws, size_t ws_bytes, void* stream) {
    bs_status st = check_image(ref, H, W);
    if (st != BS_OK) return st;
    if ((st = check_params(params)) != BS_OK) return st;
    if (C < 1 || C > BS_MAX_CHANNELS) return fail(BS_EINVAL, "channel count out of range");
    if (!x || !out) return fail(BS_EINVAL, "NULL pointer argument");
    if ((((uintptr_t)x | (uintptr_t)out) & 3) != 0) return fail(BS_EINVAL, "misaligned buffer");
    const int64_t P = (int64_t)H * W;
    const size_t bytes = (size_t)C * P * sizeof(float);
    const char *xb = (const char*)x, *ob = (const char*)out;
    if (x != out && xb < ob + bytes && ob < xb + bytes)
        return fail(BS_EINVAL, "x and out overlap without being the same buffer");
    if ((st = check_ws(ws, ws_bytes, H, W)) != BS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const DtWs w = layout_dt(P, ws);
    BS_LAUNCH(s, K_DT_OTHER, "dt_steps", dt_steps, dim3(grid_blocks(ceil_div(P, kBlock))),
              dim3(kBlock), 0, s, ref, H, W, w.dist);
    return run_dt(x, out, w.dist, H, W, C, *params, s);
}

extern "C" bs_status bs_dt_confidence(const float* ref, int32_t H, int32_t W, const float* z,
                                      const bs_dt_params* params, float sigma_dt,
                                      int32_t zero_cols, float* conf, void* ws, size_t ws_bytes,
                                      void* stream) {
    bs_status st = check_image(ref, H, W);
    if (st != BS_OK) return st;
    if ((st = check_params(params)) != BS_OK) return st;
    if (!(sigma_dt > 0.0f) || !std::isfinite(sigma_dt))
        return fail(BS_EINVAL, "sigma_dt must be positive and finite");
    if (zero_cols < 0) return fail(BS_EINVAL, "zero_cols must be >= 0");
    if (!z || !conf) return fail(BS_EINVAL, "NULL pointer argument");
    if ((((uintptr_t)z | (uintptr_t)conf) & 3) != 0) return fail(BS_EINVAL, "misaligned buffer");
    if ((st = check_ws(ws, ws_bytes, H, W)) != BS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const int64_t P = (int64_t)H * W;
    const DtWs w = layout_dt(P, ws);
    const dim3 pg(grid_blocks(ceil_div(P, kBlock)));
    BS_LAUNCH(s, K_DT_OTHER, "dt_steps", dt_steps, pg, dim3(kBlock), 0, s, ref, H, W, w.dist);
    BS_LAUNCH(s, K_DT_OTHER, "dt_partial_sums", dt_partial_sums, dim3(kDtSumBlocks),
              dim3(kBlock), 0, s, z, P, w.part);
    BS_LAUNCH(s, K_DT_OTHER, "dt_moments", dt_moments, pg, dim3(kBlock), 0, s, z, P, w.part,
              w.sig);
    if ((st = run_dt(w.sig, w.sig, w.dist, H, W, 2, *params, s)) != BS_OK) return st;
    const float inv2s2 = (float)(1.0 / (2.0 * (double)sigma_dt * (double)sigma_dt));
    BS_LAUNCH(s, K_DT_OTHER, "dt_conf", dt_conf, pg, dim3(kBlock), 0, s, w.sig, H, W, inv2s2,
              zero_cols, conf);
    return BS_OK;
}
