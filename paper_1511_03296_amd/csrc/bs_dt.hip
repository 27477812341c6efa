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
//   - vertical pass: a block per 8 columns of a channel, 64 segments of rows
//     per column, a thread per segment holding its samples in registers (up
//     to 2048 rows); the segment maps are scanned in LDS by one wave per
//     column, and every thread replays its segment from the value entering it.
//     Lanes run along rows, so every load and store of a wave covers eight
//     32-byte row pieces.  Taller images stream their segments (dt_cols: a
//     block per 16 columns, maps composed serially from LDS).
//   - rows are read and written with 16-byte vector accesses when every row
//     starts 16-byte aligned.
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

// M consecutive samples of a row from e0 (0 beyond the row): 16-byte vector
// loads when the row is 16-byte aligned (VEC: W a multiple of 4, so a group
// of four lies wholly inside the row or wholly past it), else one by one.
// Every load is issued unconditionally from an address clamped into the row
// and a select zeroes what lies past it: a load under a branch is waited for
// where the branches join, which would serialise the loads.
template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<uint32_t> { using type = uint4; };

template <bool VEC, int M, typename T>
__device__ inline void load_run(const T* p, int e0, int W, T (&v)[M]) {
    if constexpr (VEC) {
#pragma unroll
        for (int j = 0; j < M; j += 4) {
            const typename Vec4<T>::type t =
                *reinterpret_cast<const typename Vec4<T>::type*>(p + min(e0 + j, W - 4));
            const bool in = e0 + j < W;
            v[j] = in ? t.x : T(0);
            v[j + 1] = in ? t.y : T(0);
            v[j + 2] = in ? t.z : T(0);
            v[j + 3] = in ? t.w : T(0);
        }
    } else {
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const T t = p[min(e0 + j, W - 1)];
            v[j] = e0 + j < W ? t : T(0);
        }
    }
}

// The guide values of four consecutive pixels (x0 .. x0+3) of row y in the
// three channels (0 beyond the row), as load_run reads them.
template <bool VEC>
__device__ inline void load4(const float* __restrict__ ref, int64_t P, int W, int y, int x0,
                             float (&v)[3][4]) {
    const int64_t row = (int64_t)y * W;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) load_run<VEC, 4>(ref + ch * P + row, x0, W, v[ch]);
}

// The 8-bit codes of the three channels packed into the low three bytes.
__device__ inline uint32_t pack_codes(float r, float g, float b) {
    return (uint32_t)quantise8(r) | ((uint32_t)quantise8(g) << 8) | ((uint32_t)quantise8(b) << 16);
}

// Sum over the three packed channels of |a_c - b_c|.
__device__ inline uint32_t code_dist(uint32_t a, uint32_t b) {
    uint32_t d = 0;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const int u = (int)((a >> (8 * ch)) & 255u), v = (int)((b >> (8 * ch)) & 255u);
        d += (uint32_t)abs(u - v);
    }
    return d;
}

// Domain distances of every pixel: low half the edge to the left neighbour,
// high half the edge to the upper one (0 where there is none).  A lane takes
// four consecutive pixels of kDtStepRows rows (grid: 256-column pieces by
// groups of 4 x kDtStepRows rows, a wave per row group): every code is
// computed once per row plus once for the row above the group, and the left
// neighbour comes from the lane before (lane 0 reads it).  Every load of the
// lane is issued before the first code is computed (rows past the image are
// clamped to its last row and not stored; the pixel left of the row's first
// to itself).  One row per wave measured best: the pass is latency-bound, and
// four rows per wave (the row above computed once per four) were 7 % slower
// for a quarter of the waves.
constexpr int kDtStepRows = 1;

template <bool VEC>
__global__ void __launch_bounds__(kBlock) dt_steps(const float* __restrict__ ref, int H, int W,
                                                   uint32_t* __restrict__ dist) {
    const int lane = threadIdx.x & 63;
    const int x0 = blockIdx.x * 256 + lane * 4;
    const int y0 = (blockIdx.y * (kBlock / 64) + (threadIdx.x >> 6)) * kDtStepRows;
    if (y0 >= H) return;   // the whole wave
    const int64_t P = (int64_t)H * W;
    float v[kDtStepRows + 1][3][4];   // row y0 - 1 (clamped to 0), then the group's rows
    float lv[kDtStepRows][3];         // the pixel left of x0 in each row
#pragma unroll
    for (int r = 0; r <= kDtStepRows; ++r)
        load4<VEC>(ref, P, W, min(max(y0 + r - 1, 0), H - 1), x0, v[r]);
    const int xl = x0 > 0 ? x0 - 1 : 0;
#pragma unroll
    for (int r = 0; r < kDtStepRows; ++r) {
        const int64_t q = (int64_t)min(y0 + r, H - 1) * W + min(xl, W - 1);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) lv[r][ch] = ref[ch * P + q];
    }
    uint32_t up[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) up[j] = pack_codes(v[0][0][j], v[0][1][j], v[0][2][j]);
#pragma unroll
    for (int r = 0; r < kDtStepRows; ++r) {
        const int y = y0 + r;
        uint32_t c[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) c[j] = pack_codes(v[r + 1][0][j], v[r + 1][1][j], v[r + 1][2][j]);
        const uint32_t from_lane = __shfl_up(c[3], 1);
        const uint32_t left = lane == 0 ? pack_codes(lv[r][0], lv[r][1], lv[r][2]) : from_lane;
        uint32_t o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t dh = x0 + j > 0 ? code_dist(c[j], j ? c[j - 1] : left) : 0u;
            const uint32_t dv = y > 0 ? code_dist(c[j], up[j]) : 0u;
            o[j] = dh | (dv << 16);
            up[j] = c[j];
        }
        if (y < H) {
            uint32_t* d = dist + (int64_t)y * W;
            if (VEC && x0 + 4 <= W) {
                *reinterpret_cast<uint4*>(d + x0) = make_uint4(o[0], o[1], o[2], o[3]);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (x0 + j < W) d[x0 + j] = o[j];
            }
        }
    }
}

// Composition: `m` applied after (A, B).
__device__ inline void dt_after(float& A, float& B, float mA, float mB) {
    B = fmaf(mA, B, mB);
    A = mA * A;
}

template <bool VEC, int M>
__device__ inline void store_run(float* p, int e0, int W, const float (&v)[M]) {
    if (VEC && e0 + M <= W) {
#pragma unroll
        for (int j = 0; j < M; j += 4)
            *reinterpret_cast<float4*>(p + e0 + j) = make_float4(v[j], v[j + 1], v[j + 2], v[j + 3]);
    } else {
#pragma unroll
        for (int j = 0; j < M; ++j)
            if (e0 + j < W) p[e0 + j] = v[j];
    }
}

// Horizontal pass of one iteration over every row of every channel:
// src -> dst (src == dst allowed).  VEC: rows are 16-byte aligned (W a
// multiple of 4 and 16-byte aligned planes).
template <bool VEC>
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
            uint32_t dw[M];
            load_run<VEC, M>(in, e0, W, v);
            load_run<VEC, M>(drow, e0, W, dw);
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const int e = e0 + j;
                // beyond the row: the identity map; the first sample: w = 0
                w[j] = e >= W ? 1.0f : (e == 0 ? 0.0f : dt_weight(dw[j] & 0xffffu, k, ratio));
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
            }
            // the last chunk's outputs stay in v for the backward recursion
            if (ci + 1 < nchunks) store_run<VEC, M>(out, e0, W, v);
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
                // a chunk before the last lies inside the row
                uint32_t dw[M];
                load_run<VEC, M>(out, e0, W, v);
                load_run<VEC, M>(drow, e0, W, dw);
                // the edge ahead of the lane's last sample opens the next lane's
                // run; lane 63's lies in the next chunk
                // (the shuffle runs on every lane: one under a branch would read
                // 0 from the lanes the branch leaves out)
                const uint32_t ahead = drow[min(e0 + M, W - 1)];
                const uint32_t from_next = __shfl_down(dw[0], 1);
                const uint32_t next = lane == 63 ? ahead : from_next;
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    const int e = e0 + j;
                    // the edge ahead (e, e+1); the last sample: w = 0
                    const uint32_t da = j + 1 < M ? dw[j + 1] : next;
                    wb[j] = e >= W ? 1.0f
                                   : (e + 1 == W ? 0.0f : dt_weight(da & 0xffffu, k, ratio));
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
                v[j] = yv;
            }
            store_run<VEC, M>(out, e0, W, v);
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
        for (int j = 0; j < kDtBatch; ++j) {   // rows past the segment: clamped, zeroed
            const int jj = min(j, r1 - 1 - rb);
            const float xl = xb[(int64_t)jj * W];
            const uint32_t dl = db[(int64_t)jj * W];
            const bool ok = rb + j < r1;
            xv[j] = ok ? xl : 0.0f;
            dv[j] = ok && rb + j > 0 ? dl >> 16 : 0u;
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
        for (int j = 0; j < kDtBatch; ++j) {   // rows before the segment: clamped, zeroed
            const int jj = min(j, rt - r0);
            const float xl = xb[-(int64_t)jj * W];
            // the edge ahead of the image's last row does not exist: row H - 1
            const uint32_t dl = db[-(int64_t)(rt + 1 == H ? max(jj, 1) : jj) * W];
            const bool ok = rt - j >= r0;
            xv[j] = ok ? xl : 0.0f;
            dv[j] = ok && rt - j + 1 < H ? dl >> 16 : 0u;
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

// Vertical pass of one iteration for images of any height, in place: block
// (channel, 16-column strip), kDtSegs segments of rows per column streamed
// from memory (compose, replay, both ways).
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

// Vertical pass with every column segment held in registers, for images of
// at most 64 * LMAX rows: a block takes CW columns of a channel (CW waves),
// 64 segments of L = ceil(H / 64) <= LMAX rows each per column, so every
// sample and distance is read once and every output written once.  The
// segment maps are scanned by one wave per column (lane = segment, six
// shuffle steps), downwards and then upwards.  Blocks are dealt to the dies in
// contiguous runs of column strips, so a die's L2 holds whole cache lines of
// the rows.  Eight columns (32-byte row pieces) measured best on the 1024x768
// stereo image: 4 % ahead of 16 columns, level with 4.  Taller images (more
// than 64 * 32 rows) take the streaming pass dt_cols.
constexpr int kDtRegSegs = 64;
constexpr int kDtRegCW = 8;

// The exclusive scan of the segment maps of column `col` held in LDS
// (sA[seg][col], sB[seg][col]), in place: DOWN composes the maps above a
// segment, !DOWN those below it.
template <bool DOWN, int CWP>
__device__ inline void scan_segment_maps(float (*sA)[CWP], float (*sB)[CWP], int col) {
    const int lane = threadIdx.x & 63;
    float A = sA[lane][col], B = sB[lane][col];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const float pA = DOWN ? __shfl_up(A, o) : __shfl_down(A, o);
        const float pB = DOWN ? __shfl_up(B, o) : __shfl_down(B, o);
        if (DOWN ? lane >= o : lane + o < 64) {
            B = fmaf(A, pB, B);
            A = A * pA;
        }
    }
    float eA = DOWN ? __shfl_up(A, 1) : __shfl_down(A, 1);
    float eB = DOWN ? __shfl_up(B, 1) : __shfl_down(B, 1);
    if (lane == (DOWN ? 0 : 63)) {
        eA = 1.0f;
        eB = 0.0f;
    }
    sA[lane][col] = eA;
    sB[lane][col] = eB;
}

template <int CW, int LMAX>
__global__ void __launch_bounds__(CW * 64) dt_cols_reg(float* x, const uint32_t* __restrict__ dist,
                                                       int H, int W, int strips, int tiles,
                                                       float k, float ratio) {
    static_assert(CW * 64 / kDtRegSegs == CW, "one wave per column of the block");
    __shared__ float sA[kDtRegSegs][CW + 1], sB[kDtRegSegs][CW + 1];
    const int nb = gridDim.x;
    const int tile = nb % kXcds == 0 ? partial_slot(blockIdx.x, nb) : blockIdx.x;
    if (tile >= tiles) return;   // the whole block: the grid is rounded up to the dies
    const int col_in = threadIdx.x % CW, seg = threadIdx.x / CW;
    const int c = tile / strips;
    const int col = (tile - c * strips) * CW + col_in;
    const bool live = col < W;
    const int L = (H + kDtRegSegs - 1) / kDtRegSegs;
    const int r0 = min(H, seg * L), n = min(H, r0 + L) - r0;
    float* xc = x + ((int64_t)c * H + r0) * W + col;
    // loads from addresses clamped into the image (column, then row), the
    // samples outside the segment zeroed by a select: no load under a branch
    const int colc = min(col, W - 1);
    const float* xp = x + (int64_t)c * H * W + colc;
    const uint32_t* dp = dist + colc;
    float v[LMAX], w[LMAX];
    uint32_t dw[LMAX];
#pragma unroll
    for (int j = 0; j < LMAX; ++j) {
        const int64_t at = (int64_t)min(r0 + j, H - 1) * W;
        const float xv = xp[at];
        const uint32_t dv = dp[at];
        const bool ok = live && j < n;
        v[j] = ok ? xv : 0.0f;
        dw[j] = ok ? dv >> 16 : 0u;
    }
    // the edge below the segment's last row opens the next segment
    const uint32_t dl = dp[(int64_t)min(r0 + n, H - 1) * W];
    const bool below = live && n > 0 && r0 + n < H;
    const float wlast = below ? dt_weight(dl >> 16, k, ratio) : 0.0f;
    // edge (r-1, r) of row r = r0 + j; the image's first row: 0; beyond the
    // segment: the identity map (w = 1 with v = 0)
#pragma unroll
    for (int j = 0; j < LMAX; ++j)
        w[j] = j < n ? (r0 + j == 0 ? 0.0f : dt_weight(dw[j], k, ratio)) : 1.0f;
    // downwards
    float A = 1.0f, B = 0.0f;
#pragma unroll
    for (int j = 0; j < LMAX; ++j) dt_after(A, B, w[j], (1.0f - w[j]) * v[j]);
    sA[seg][col_in] = A;
    sB[seg][col_in] = B;
    __syncthreads();
    scan_segment_maps<true, CW + 1>(sA, sB, threadIdx.x >> 6);
    __syncthreads();
    float yv = sB[seg][col_in];   // the image's first row has w = 0: the map at 0
#pragma unroll
    for (int j = 0; j < LMAX; ++j) {
        yv = fmaf(w[j], yv, (1.0f - w[j]) * v[j]);
        v[j] = yv;
    }
    __syncthreads();   // every thread has read its prefix
    // upwards over the downward output: row r takes the edge (r, r+1), the
    // image's last row 0
    A = 1.0f;
    B = 0.0f;
#pragma unroll
    for (int j = LMAX - 1; j >= 0; --j) {
        const float u = j + 1 < n ? w[j + 1 < LMAX ? j + 1 : LMAX - 1]
                                    : (j + 1 == n ? wlast : 1.0f);
        dt_after(A, B, u, (1.0f - u) * v[j]);
    }
    sA[seg][col_in] = A;
    sB[seg][col_in] = B;
    __syncthreads();
    scan_segment_maps<false, CW + 1>(sA, sB, threadIdx.x >> 6);
    __syncthreads();
    yv = sB[seg][col_in];   // the image's last row has w = 0
#pragma unroll
    for (int j = LMAX - 1; j >= 0; --j) {
        const float u = j + 1 < n ? w[j + 1 < LMAX ? j + 1 : LMAX - 1]
                                    : (j + 1 == n ? wlast : 1.0f);
        yv = fmaf(u, yv, (1.0f - u) * v[j]);
        if (live && j < n) xc[(int64_t)j * W] = yv;
    }
}

constexpr int kDtSumBlocks = 256;

// Sum of a float64 over the block (kBlock threads), the same order in every
// block: the waves' shuffle trees, then the four wave sums in turn.
__device__ inline double block_sum(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();   // `red` may still be read from an earlier call
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) t += red[w];
    return t;
}

// Per-block float64 partial sums of z [P] (kDtSumBlocks blocks); four loads
// in flight per thread.
__global__ void __launch_bounds__(kBlock) dt_partial_sums(const float* __restrict__ z,
                                                          int64_t P,
                                                          double* __restrict__ part) {
    __shared__ double red[kBlock / 64];
    constexpr int64_t stride = (int64_t)kDtSumBlocks * kBlock;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (; p + 3 * stride < P; p += 4 * stride) {
        s0 += (double)z[p];
        s1 += (double)z[p + stride];
        s2 += (double)z[p + 2 * stride];
        s3 += (double)z[p + 3 * stride];
    }
    for (; p < P; p += stride) s0 += (double)z[p];
    const double t = block_sum((s0 + s1) + (s2 + s3), red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// The two signals of the variance, about the mean mu of z (every block sums
// the partials in the same order): s[0] = z - mu, s[1] = (z - mu)^2.  V is the
// same for every shift mu; the shift keeps the float32 rounding relative to
// the spread of z instead of its offset.
__global__ void __launch_bounds__(kBlock) dt_moments(const float* __restrict__ z, int64_t P,
                                                     const double* __restrict__ part,
                                                     float* __restrict__ s) {
    static_assert(kDtSumBlocks == kBlock, "one partial per thread");
    __shared__ double red[kBlock / 64];
    int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const float z0 = p < P ? z[p] : 0.0f;   // in flight during the sum of the partials
    const float mu = (float)(block_sum(part[threadIdx.x], red) / (double)P);
    for (float zv = z0; p < P; p += (int64_t)gridDim.x * kBlock) {
        if (p != (int64_t)blockIdx.x * kBlock + threadIdx.x) zv = z[p];
        const float d = zv - mu;
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
        const int x = (int)((uint32_t)p % (uint32_t)W);   // P < 2^30
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

// The domain distances of the guide into `dist`.
bs_status launch_steps(const float* ref, int H, int W, uint32_t* dist, hipStream_t s) {
    const dim3 grid((unsigned)ceil_div(W, 256), (unsigned)ceil_div(H, (kBlock / 64) * kDtStepRows));
    // 16-byte accesses: every plane and row starts 16-byte aligned
    const bool vec = W % 4 == 0 && ((uintptr_t)ref & 15) == 0 && ((uintptr_t)dist & 15) == 0;
    if (vec)
        BS_LAUNCH(s, K_DT_OTHER, "dt_steps", dt_steps<true>, grid, dim3(kBlock), 0, s, ref, H, W,
                  dist);
    else
        BS_LAUNCH(s, K_DT_OTHER, "dt_steps", dt_steps<false>, grid, dim3(kBlock), 0, s, ref, H,
                  W, dist);
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
    // segments in registers: rows per segment, column strips, tiles and the
    // grid rounded up to whole dies
    const int reg_rows = (int)ceil_div(H, kDtRegSegs);
    const int reg_strips = (int)ceil_div(W, kDtRegCW);
    const int reg_tiles = C * reg_strips;
    const int reg_grid = (int)ceil_div(reg_tiles, kXcds) * kXcds;
    // 16-byte row accesses: every row starts on a 16-byte boundary
    const bool vec = W % 4 == 0 && ((uintptr_t)src & 15) == 0 && ((uintptr_t)dst & 15) == 0 &&
                     ((uintptr_t)dist & 15) == 0;
    for (int i = 1; i <= N; ++i) {
        const double sig = (double)p.sigma_s * std::sqrt(3.0) * std::ldexp(1.0, N - i) /
                           std::sqrt(std::ldexp(1.0, 2 * N) - 1.0);
        const float k = (float)(-std::sqrt(2.0) / sig / std::log(2.0));
        const float* in = i == 1 ? src : dst;
        if (vec)
            BS_LAUNCH(s, K_DT_ROWS, "dt_rows", dt_rows<true>, dim3(row_blocks),
                      dim3(kDtRowBlock), 0, s, in, dst, dist, H, W, C, k, (float)ratio);
        else
            BS_LAUNCH(s, K_DT_ROWS, "dt_rows", dt_rows<false>, dim3(row_blocks),
                      dim3(kDtRowBlock), 0, s, in, dst, dist, H, W, C, k, (float)ratio);
        if (reg_rows <= 8)
            BS_LAUNCH(s, K_DT_COLS, "dt_cols", (dt_cols_reg<kDtRegCW, 8>), dim3(reg_grid),
                      dim3(kDtRegCW * 64), 0, s, dst, dist, H, W, reg_strips, reg_tiles, k,
                      (float)ratio);
        else if (reg_rows <= 16)
            BS_LAUNCH(s, K_DT_COLS, "dt_cols", (dt_cols_reg<kDtRegCW, 16>), dim3(reg_grid),
                      dim3(kDtRegCW * 64), 0, s, dst, dist, H, W, reg_strips, reg_tiles, k,
                      (float)ratio);
        else if (reg_rows <= 32)
            BS_LAUNCH(s, K_DT_COLS, "dt_cols", (dt_cols_reg<kDtRegCW, 32>), dim3(reg_grid),
                      dim3(kDtRegCW * 64), 0, s, dst, dist, H, W, reg_strips, reg_tiles, k,
                      (float)ratio);
        else
            BS_LAUNCH(s, K_DT_COLS, "dt_cols", dt_cols, dim3(C * strips), dim3(kDtColBlock), 0,
                      s, dst, dist, H, W, strips, k, (float)ratio);
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
    if ((st = launch_steps(ref, H, W, w.dist, s)) != BS_OK) return st;
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
    if ((st = launch_steps(ref, H, W, w.dist, s)) != BS_OK) return st;
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
