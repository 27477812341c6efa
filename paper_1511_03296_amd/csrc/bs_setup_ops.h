// Kernel bodies of the per-image stages around the PCG: the splat of the
// right-hand side with diag(A) and its Jacobi inverse (Eq. quad_min, the
// Jacobi preconditioner of Section 4), the flat and hierarchical initial
// states (Section 4, supplement Section 2), the slice (Eq. solution) and the
// gradient scatter (Section 3).  They are Ops: the single-image entry points
// run them through one_launch, the batch engine through multi_launch.
#pragma once

#include "bs_solve_impl.h"

namespace bs {

// ---------------------------------------------------------------------------
// Splat.
// ---------------------------------------------------------------------------

// Output arrays of the splat of one image.
struct SplatOut {
    float* sc;       // [V] S c
    float* diag;     // [V] diag(A)
    float* minv;     // [V] 1 / diag(A), 0 where diag(A) <= 0
    float2* nfm;     // [V] {n, 1 / diag(A)}
    float* b;        // [V][Cp] right-hand side
};

// S c, b = S (c o t) (or S t when `weighted` is false) as ascending-pixel sums
// in float64, diag(A) = lam n o (N n) + S c with its Jacobi inverse, and the
// packed per-vertex scalars {n, 1 / diag(A)} of the PCG kernels.  b has
// stride Cp; channels C..Cp-1 are zero.  One thread per vertex.
template <bool WEIGHTED>
struct SplatVertex {
    static constexpr int kThreads = kBlock;
    struct Args {
        const int32_t* ptr;
        const int32_t* list;
        const float* conf;
        const float* vals;
        const double* nn;
        const float* nf;
        const int32_t* counts;
        SplatOut o;
        double lam;
        int C, Cp, P;
    };
    __device__ static void run(const Args& a, int jb, int nb, int) {
        const int32_t* __restrict__ ptr = a.ptr;
        const int32_t* __restrict__ list = a.list;
        const float* __restrict__ conf = a.conf;
        const float* __restrict__ vals = a.vals;
        float* __restrict__ b = a.o.b;
        const int C = a.C, Cp = a.Cp, P = a.P;
        const int V = a.counts[CNT_V];
        const XcdTiles tl((V + kBlock - 1) / kBlock, jb, nb);
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
                    if (k < cn) b[(int64_t)v * Cp + c0 + k] = (float)acc[k];
            }
            for (int c = C; c < Cp; ++c) b[(int64_t)v * Cp + c] = 0.0f;
            const double d = a.lam * a.nn[v] + sc;
            const float mi = d > 0.0 ? (float)(1.0 / d) : 0.0f;
            a.o.sc[v] = (float)sc;
            a.o.diag[v] = (float)d;
            a.o.minv[v] = mi;
            a.o.nfm[v] = make_float2(a.nf[v], mi);
        }
    }
};

// The same sums computed per spatial cell of the grid (block c: cell c):
// every pixel of a cell lies on one of the cell's vertices, so a block stages
// the cell's pixels in LDS with coalesced row loads and each (vertex,
// channel) thread sums its own pixels, in ascending pixel order, from LDS.
// CAP bounds the cell's pixels.
constexpr int kSplatVals = 4096;   // floats of staged values per channel chunk

template <int B, int CAP, bool WEIGHTED>
struct SplatCells {
    static constexpr int kThreads = B;
    struct Args {
        const int32_t* cell_vbase;
        const int32_t* cell_ibase;
        const int32_t* ptr;
        const int32_t* list;
        const float* conf;
        const float* vals;
        const double* nn;
        const float* nf;
        SplatOut o;
        double lam;
        int H, W, sxy, ncx, C, Cp, P;
    };
    __device__ static void run(const Args& a, int c, int, int) {
        __shared__ float cv[CAP];
        __shared__ int32_t lst[CAP];
        __shared__ int32_t sp[CAP + 1];   // the cell's vertex CSR, relative to ibase
        __shared__ float tv[kSplatVals];
        const int32_t* __restrict__ ptr = a.ptr;
        const float* __restrict__ vals = a.vals;
        float* __restrict__ b = a.o.b;
        const int H = a.H, W = a.W, sxy = a.sxy, ncx = a.ncx, C = a.C, Cp = a.Cp, P = a.P;
        const int cy = c / ncx, cx = c - cy * ncx;
        const int y0 = cell_lo(cy, sxy), y1 = min(cell_lo(cy + 1, sxy), H);
        const int x0 = cell_lo(cx, sxy), x1 = min(cell_lo(cx + 1, sxy), W);
        const int wx = x1 - x0, n = (y1 - y0) * wx;
        const int vbase = a.cell_vbase[c], cnt = a.cell_vbase[c + 1] - vbase;
        const int ibase = a.cell_ibase[c];
        for (int j = threadIdx.x; j < n; j += B) {
            const int r = j / wx;
            cv[j] = a.conf[(y0 + r) * W + x0 + (j - r * wx)];
            const int pq = a.list[ibase + j];
            const int py = pq / W;
            lst[j] = (py - y0) * wx + (pq - py * W - x0);
        }
        for (int k = threadIdx.x; k <= cnt; k += B) sp[k] = ptr[vbase + k] - ibase;
        __syncthreads();
        for (int k = threadIdx.x; k < cnt; k += B) {
            const int s0 = sp[k], s1 = sp[k + 1];
            double sc = 0.0;
            int q = s0;
            // four pixels' LDS reads issued together, summed in ascending order
            for (; q + 4 <= s1; q += 4) {
                const int j0 = lst[q], j1 = lst[q + 1], j2 = lst[q + 2], j3 = lst[q + 3];
                const float c0 = cv[j0], c1 = cv[j1], c2 = cv[j2], c3 = cv[j3];
                sc += (double)c0;
                sc += (double)c1;
                sc += (double)c2;
                sc += (double)c3;
            }
            for (; q < s1; ++q) sc += (double)cv[lst[q]];
            const double d = a.lam * a.nn[vbase + k] + sc;
            const float mi = d > 0.0 ? (float)(1.0 / d) : 0.0f;
            a.o.sc[vbase + k] = (float)sc;
            a.o.diag[vbase + k] = (float)d;
            a.o.minv[vbase + k] = mi;
            a.o.nfm[vbase + k] = make_float2(a.nf[vbase + k], mi);
        }
        const int CH = max(1, min(C, kSplatVals / max(n, 1)));
        for (int c0 = 0; c0 < C; c0 += CH) {
            const int cn = min(CH, C - c0);
            __syncthreads();
            // eight values' loads issued together while all eight exist
            const int tot = cn * n;
            auto val = [&](int e) {
                const int cc = e / n, j = e - cc * n;
                const int r = j / wx;
                return vals[(int64_t)(c0 + cc) * P + (y0 + r) * W + x0 + (j - r * wx)];
            };
            int e0 = threadIdx.x;
            for (; e0 + 7 * B < tot; e0 += 8 * B) {
                float t8[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) t8[u] = val(e0 + u * B);
#pragma unroll
                for (int u = 0; u < 8; ++u) tv[e0 + u * B] = t8[u];
            }
            for (; e0 < tot; e0 += B) tv[e0] = val(e0);
            __syncthreads();
            for (int e = threadIdx.x; e < cnt * cn; e += B) {
                const int k = e / cn, cc = e - k * cn;
                const int s0 = sp[k], s1 = sp[k + 1];
                const float* __restrict__ tc = tv + cc * n;
                double acc = 0.0;
                int q = s0;
                for (; q + 4 <= s1; q += 4) {
                    int jl[4];
                    float tq[4], wq[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) jl[u] = lst[q + u];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        tq[u] = tc[jl[u]];
                        wq[u] = WEIGHTED ? cv[jl[u]] : 1.0f;
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        acc += WEIGHTED ? (double)wq[u] * (double)tq[u] : (double)tq[u];
                }
                for (; q < s1; ++q) {
                    const int jl = lst[q];
                    acc += WEIGHTED ? (double)cv[jl] * (double)tc[jl] : (double)tc[jl];
                }
                b[(int64_t)(vbase + k) * Cp + c0 + cc] = (float)acc;
            }
        }
        const int pad = Cp - C;
        for (int e = threadIdx.x; e < cnt * pad; e += B) {
            const int k = e / pad, cc = e - k * pad;
            b[(int64_t)(vbase + k) * Cp + C + cc] = 0.0f;
        }
    }
};

// Which splat form an image takes: per cell while a cell's pixels (at most
// sigma_xy^2) fit the LDS staging (kind 0, 1, 2: 64, 256, 1024 pixels), else
// per vertex (kind 3).
inline int splat_kind(int sigma_xy) {
    const int items = sigma_xy * sigma_xy;
    return items <= 64 ? 0 : (items <= 256 ? 1 : (items <= 1024 ? 2 : 3));
}

// ---------------------------------------------------------------------------
// Initial state.
// ---------------------------------------------------------------------------

// Flat init: y = b / S c, 0 where S c = 0.
struct FlatInit {
    static constexpr int kThreads = kBlock;
    struct Args {
        const float* b;
        const float* sc;
        const int32_t* counts;
        float* y;
        int C;
    };
    __device__ static void run(const Args& a, int jb, int nb, int) {
        const int C = a.C;
        const int64_t n = (int64_t)a.counts[CNT_V] * C;
        const XcdTiles tl((n + kBlock - 1) / kBlock, jb, nb);
        for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
            const int64_t e = tile * kBlock + threadIdx.x;
            if (e >= n) continue;
            const float s = a.sc[e / C];
            a.y[e] = s > 0.0f ? a.b[e] / s : 0.0f;
        }
    }
};

// Pyramid lift, level k >= 1: child sums of level k-1 for C channels of b and
// S c (channel C).  up_k[u][ch] = sum over children of the child's value.
// Sum over the children clist[j0 .. j1) of get(child), in ascending order,
// four children's loads issued together.
template <class F>
__device__ inline double sum_children(const int32_t* __restrict__ clist, int j0, int j1, F get) {
    double s = 0.0;
    int j = j0;
    for (; j + 4 <= j1; j += 4) {
        int c[4];
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] = clist[j + q];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = get(c[q]);
#pragma unroll
        for (int q = 0; q < 4; ++q) s += (double)v[q];
    }
    for (; j < j1; ++j) s += (double)get(clist[j]);
    return s;
}

struct PyrUp {
    static constexpr int kThreads = kBlock;
    struct Args {
        const int32_t* cptr;
        const int32_t* clist;
        const float* b;
        const float* sc;
        const float* prev;   // level k-1's sums, nullptr at k = 1 (read b and S c)
        float* up;
        const int32_t* counts;
        int C, level;
    };
    __device__ static void run(const Args& a, int jb, int nb, int) {
        const int32_t* __restrict__ counts = a.counts;
        const int level = a.level, C = a.C;
        if (counts[CNT_K] < level) return;
        const int Vk = counts[CNT_LEVEL0 + level];
        const int C1 = C + 1;
        const int64_t n = (int64_t)Vk * C1;
        const float* __restrict__ prev = a.prev;
        const XcdTiles tl((n + kBlock - 1) / kBlock, jb, nb);
        for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
            const int64_t e = tile * kBlock + threadIdx.x;
            if (e >= n) continue;
            const int u = (int)(e / C1), ch = (int)(e - (int64_t)u * C1);
            const int j0 = a.cptr[u], j1 = a.cptr[u + 1];
            // the level below, or at level 1 [b | S c] (both read, one kept:
            // no load under a branch inside the sum)
            const double s =
                prev ? sum_children(a.clist, j0, j1,
                                    [&](int c) { return prev[(int64_t)c * C1 + ch]; })
                     : sum_children(a.clist, j0, j1, [&](int c) {
                           const float bv = a.b[(int64_t)c * C + min(ch, C - 1)];
                           const float sv = a.sc[c];
                           return ch < C ? bv : sv;
                       });
            a.up[e] = (float)s;
        }
    }
};

// Pyramid collapse, level k >= 1 (top-down): acc_k = w_k P_k / P(1)_k + acc_{k+1}[parent].
struct PyrDown {
    static constexpr int kThreads = kBlock;
    struct Args {
        float* up;
        const float* up_parent;
        const int32_t* parent;
        const int32_t* ones;
        const int32_t* counts;
        float wk;
        int C, level;
    };
    __device__ static void run(const Args& a, int jb, int nb, int) {
        const int K = a.counts[CNT_K];
        const int level = a.level;
        if (K < level) return;
        const int Vk = a.counts[CNT_LEVEL0 + level];
        const int C1 = a.C + 1;
        const int64_t n = (int64_t)Vk * C1;
        float* __restrict__ up = a.up;
        const XcdTiles tl((n + kBlock - 1) / kBlock, jb, nb);
        for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
            const int64_t e = tile * kBlock + threadIdx.x;
            if (e >= n) continue;
            const int u = (int)(e / C1), ch = (int)(e - (int64_t)u * C1);
            float v = a.wk * up[e] / (float)a.ones[u];
            if (level < K) v += a.up_parent[(int64_t)a.parent[u] * C1 + ch];
            up[e] = v;
        }
    }
};

// The small top of the pyramid, levels k0 .. levels-1, in one block: the lift
// bottom-up, then the collapse top-down, with the arithmetic of PyrUp and
// PyrDown (the coarse levels would otherwise cost two launches each).
constexpr int kSmallPyrElems = 16384;   // cap_k x (C + 1) of a level done in one block

struct PyrLevels {
    int k0, levels;
    const int32_t* cptr[BS_MAX_LEVELS];    // level k: CSR of children (level k-1 vertices)
    const int32_t* clist[BS_MAX_LEVELS];
    const int32_t* ones[BS_MAX_LEVELS];
    const int32_t* parent[BS_MAX_LEVELS];  // level k vertex -> level k+1 vertex
    float* up[BS_MAX_LEVELS];
    float wk[BS_MAX_LEVELS];
};

struct PyrSmall {
    static constexpr int kThreads = 1024;
    struct Args {
        PyrLevels lv;
        const float* b;
        const float* sc;
        const int32_t* counts;
        int C;
    };
    __device__ static void run(const Args& A, int, int, int) {
        const PyrLevels& a = A.lv;
        const int K = A.counts[CNT_K];
        const int C = A.C;
        const int C1 = C + 1;
        for (int k = a.k0; k < a.levels && k <= K; ++k) {
            const int Vk = A.counts[CNT_LEVEL0 + k];
            const float* prev = k >= 2 ? a.up[k - 1] : nullptr;
            const int32_t* cptr = a.cptr[k];
            const int32_t* clist = a.clist[k];
            float* up = a.up[k];
            const int64_t n = (int64_t)Vk * C1;
            for (int64_t e = threadIdx.x; e < n; e += kThreads) {
                const int u = (int)(e / C1), ch = (int)(e - (int64_t)u * C1);
                const int j0 = cptr[u], j1 = cptr[u + 1];
                // the level below, or at level 1 [b | S c] (both read, one
                // kept: no load under a branch inside the sum)
                const double s =
                    prev ? sum_children(clist, j0, j1,
                                        [&](int c) { return prev[(int64_t)c * C1 + ch]; })
                         : sum_children(clist, j0, j1, [&](int c) {
                               const float bv = A.b[(int64_t)c * C + min(ch, C - 1)];
                               const float sv = A.sc[c];
                               return ch < C ? bv : sv;
                           });
                up[e] = (float)s;
            }
            __syncthreads();
        }
        for (int k = a.levels - 1; k >= a.k0; --k) {
            if (K < k) continue;
            const int Vk = A.counts[CNT_LEVEL0 + k];
            float* up = a.up[k];
            const float* upp = (k < K) ? a.up[k + 1] : nullptr;
            const int32_t* parent = a.parent[k];
            const int32_t* ones = a.ones[k];
            const float wk = a.wk[k];
            const int64_t n = (int64_t)Vk * C1;
            for (int64_t e = threadIdx.x; e < n; e += kThreads) {
                const int u = (int)(e / C1), ch = (int)(e - (int64_t)u * C1);
                float v = wk * up[e] / (float)ones[u];
                if (upp) v += upp[(int64_t)parent[u] * C1 + ch];
                up[e] = v;
            }
            __syncthreads();
        }
    }
};

// Level 0 of the collapse and the ratio of the two push-pull filters:
// y0 = (b + acc_1[parent]) / (S c + acc_1[parent][C]), 0 where the
// denominator is 0 (zero total confidence).
struct HierFinal {
    static constexpr int kThreads = kBlock;
    struct Args {
        const float* b;
        const float* sc;
        const float* up1;
        const int32_t* parent0;
        const int32_t* counts;
        float* y;
        int C;
    };
    __device__ static void run(const Args& a, int jb, int nb, int) {
        const int K = a.counts[CNT_K];
        const int C = a.C;
        const int64_t n = (int64_t)a.counts[CNT_V] * C;
        const int C1 = C + 1;
        const XcdTiles tl((n + kBlock - 1) / kBlock, jb, nb);
        for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
            const int64_t e = tile * kBlock + threadIdx.x;
            if (e >= n) continue;
            const int v = (int)(e / C), ch = (int)(e - (int64_t)v * C);
            float num = a.b[e], den = a.sc[v];
            if (K >= 1) {
                const int64_t p = (int64_t)a.parent0[v] * C1;
                num += a.up1[p + ch];
                den += a.up1[p + C];
            }
            a.y[e] = den > 0.0f ? num / den : 0.0f;
        }
    }
};

// ---------------------------------------------------------------------------
// Hierarchical preconditioner (Section 4, Eq. hier_precond):
//     M_hier^-1 r = P^T(s o P(r)),   s_k = w_k P(1)_k / P(diag A)_k,
// w_0 = 1 (at level 0, s_0 = 1 / diag(A): the Jacobi inverse), w_k =
// alpha^-(beta + k) above; a coefficient with P(diag A)_k = 0 is 0.  Level
// k >= 1 uses the pyramid buffer up_k [cap_k][Cp + 1]: channel Cp holds s_k
// (set once per solve), channels 0..Cp-1 hold P_k(r) and then the collapse.
// ---------------------------------------------------------------------------

// Set-up: P_k(diag A) into channel Cp of up_k (level 1 sums diag(A) over its
// children, level k >= 2 the channel Cp of level k-1).
struct PrecLift {
    static constexpr int kThreads = kBlock;
    struct Args {
        const int32_t* cptr;
        const int32_t* clist;
        const float* diag;
        const float* prev;
        float* up;
        const int32_t* counts;
        int Cp, level;
    };
    __device__ static void run(const Args& a, int jb, int nb, int) {
        if (a.counts[CNT_K] < a.level) return;
        const int Vk = a.counts[CNT_LEVEL0 + a.level];
        const int C1 = a.Cp + 1;
        const XcdTiles tl((Vk + kBlock - 1) / kBlock, jb, nb);
        for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
            const int u = (int)(tile * kBlock) + threadIdx.x;
            if (u >= Vk) continue;
            const int j0 = a.cptr[u], j1 = a.cptr[u + 1];
            const float* __restrict__ prev = a.prev;
            const double s =
                prev ? sum_children(a.clist, j0, j1,
                                    [&](int c) { return prev[(int64_t)c * C1 + a.Cp]; })
                     : sum_children(a.clist, j0, j1, [&](int c) { return a.diag[c]; });
            a.up[(int64_t)u * C1 + a.Cp] = (float)s;
        }
    }
};

// Set-up: s_k = w_k P(1)_k / P(diag A)_k in place of P(diag A)_k (after every
// level is lifted).
struct PrecScale {
    static constexpr int kThreads = kBlock;
    struct Args {
        float* up;
        const int32_t* ones;
        const int32_t* counts;
        float wk;
        int Cp, level;
    };
    __device__ static void run(const Args& a, int jb, int nb, int) {
        if (a.counts[CNT_K] < a.level) return;
        const int Vk = a.counts[CNT_LEVEL0 + a.level];
        const int C1 = a.Cp + 1;
        const XcdTiles tl((Vk + kBlock - 1) / kBlock, jb, nb);
        for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
            const int u = (int)(tile * kBlock) + threadIdx.x;
            if (u >= Vk) continue;
            const float pd = a.up[(int64_t)u * C1 + a.Cp];
            a.up[(int64_t)u * C1 + a.Cp] =
                pd > 0.0f ? (float)((double)a.wk * (double)a.ones[u] / (double)pd) : 0.0f;
        }
    }
};

// Per application: channels 0..Cp-1 of up_k = child sums of r (level 1,
// stride Cp) or of level k-1's channels (stride Cp + 1).
struct PrecUp {
    static constexpr int kThreads = kBlock;
    struct Args {
        const int32_t* cptr;
        const int32_t* clist;
        const float* r;
        const float* prev;
        float* up;
        const int32_t* counts;
        int Cp, level;
    };
    __device__ static void run(const Args& a, int jb, int nb, int) {
        if (a.counts[CNT_K] < a.level) return;
        const int Vk = a.counts[CNT_LEVEL0 + a.level];
        const int Cp = a.Cp, C1 = Cp + 1;
        const int64_t n = (int64_t)Vk * Cp;
        const XcdTiles tl((n + kBlock - 1) / kBlock, jb, nb);
        for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
            const int64_t e = tile * kBlock + threadIdx.x;
            if (e >= n) continue;
            const int u = (int)(e / Cp), ch = (int)(e - (int64_t)u * Cp);
            const int j0 = a.cptr[u], j1 = a.cptr[u + 1];
            const float* __restrict__ prev = a.prev;
            const double s =
                prev ? sum_children(a.clist, j0, j1,
                                    [&](int c) { return prev[(int64_t)c * C1 + ch]; })
                     : sum_children(a.clist, j0, j1,
                                    [&](int c) { return a.r[(int64_t)c * Cp + ch]; });
            a.up[(int64_t)u * C1 + ch] = (float)s;
        }
    }
};

// Per application, top-down: up_k = s_k o up_k + up_{k+1}[parent] (channels
// 0..Cp-1; the top level has no parent term).
struct PrecDown {
    static constexpr int kThreads = kBlock;
    struct Args {
        float* up;
        const float* up_parent;
        const int32_t* parent;
        const int32_t* counts;
        int Cp, level;
    };
    __device__ static void run(const Args& a, int jb, int nb, int) {
        const int K = a.counts[CNT_K];
        if (K < a.level) return;
        const int Vk = a.counts[CNT_LEVEL0 + a.level];
        const int Cp = a.Cp, C1 = Cp + 1;
        const int64_t n = (int64_t)Vk * Cp;
        const XcdTiles tl((n + kBlock - 1) / kBlock, jb, nb);
        for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
            const int64_t e = tile * kBlock + threadIdx.x;
            if (e >= n) continue;
            const int u = (int)(e / Cp), ch = (int)(e - (int64_t)u * Cp);
            float v = a.up[(int64_t)u * C1 + Cp] * a.up[(int64_t)u * C1 + ch];
            if (a.level < K) v += a.up_parent[(int64_t)a.parent[u] * C1 + ch];
            a.up[(int64_t)u * C1 + ch] = v;
        }
    }
};

// The small top levels k0 .. levels-1 of one application in one block: the
// lift bottom-up, then the collapse top-down (PrecUp and PrecDown).
struct PrecSmall {
    static constexpr int kThreads = 1024;
    struct Args {
        PyrLevels lv;        // cptr, clist, parent and up of every level (wk, ones unused)
        const float* r;
        const int32_t* counts;
        int Cp;
    };
    __device__ static void run(const Args& A, int, int, int) {
        const PyrLevels& a = A.lv;
        const int K = A.counts[CNT_K];
        const int Cp = A.Cp, C1 = Cp + 1;
        for (int k = a.k0; k < a.levels && k <= K; ++k) {
            const int Vk = A.counts[CNT_LEVEL0 + k];
            const float* prev = k >= 2 ? a.up[k - 1] : nullptr;
            const int64_t n = (int64_t)Vk * Cp;
            for (int64_t e = threadIdx.x; e < n; e += kThreads) {
                const int u = (int)(e / Cp), ch = (int)(e - (int64_t)u * Cp);
                const int j0 = a.cptr[k][u], j1 = a.cptr[k][u + 1];
                const double s =
                    prev ? sum_children(a.clist[k], j0, j1,
                                        [&](int c) { return prev[(int64_t)c * C1 + ch]; })
                         : sum_children(a.clist[k], j0, j1,
                                        [&](int c) { return A.r[(int64_t)c * Cp + ch]; });
                a.up[k][(int64_t)u * C1 + ch] = (float)s;
            }
            __syncthreads();
        }
        for (int k = a.levels - 1; k >= a.k0; --k) {
            if (K < k) continue;
            const int Vk = A.counts[CNT_LEVEL0 + k];
            float* up = a.up[k];
            const float* upp = (k < K) ? a.up[k + 1] : nullptr;
            const int64_t n = (int64_t)Vk * Cp;
            for (int64_t e = threadIdx.x; e < n; e += kThreads) {
                const int u = (int)(e / Cp), ch = (int)(e - (int64_t)u * Cp);
                float v = up[(int64_t)u * C1 + Cp] * up[(int64_t)u * C1 + ch];
                if (upp) v += upp[(int64_t)a.parent[k][u] * C1 + ch];
                up[(int64_t)u * C1 + ch] = v;
            }
            __syncthreads();
        }
    }
};

// ---------------------------------------------------------------------------
// Output.
// ---------------------------------------------------------------------------

// dst[v][c] = src[v][c] for c < C, src with stride Cp.
struct Unpad {
    static constexpr int kThreads = kBlock;
    struct Args {
        const float* src;
        const int32_t* counts;
        float* dst;
        int Cp, C;
    };
    __device__ static void run(const Args& a, int jb, int nb, int) {
        const int C = a.C;
        const int64_t n = (int64_t)a.counts[CNT_V] * C;
        const XcdTiles tl((n + kBlock - 1) / kBlock, jb, nb);
        for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
            const int64_t e = tile * kBlock + threadIdx.x;
            if (e >= n) continue;
            const int64_t v = e / C;
            a.dst[e] = a.src[v * a.Cp + (e - v * C)];
        }
    }
};

// x[c][p] = y[idx[p]][c].
constexpr int kSliceChunk = 4;   // channels per batch of loads (slice, gradient scatter)

struct Slice {
    static constexpr int kThreads = kBlock;
    struct Args {
        const int32_t* idx;
        const float* y;
        float* x;
        int C, P;
    };
    __device__ static void run(const Args& a, int jb, int nb, int) {
        const int C = a.C, P = a.P;
        const float* __restrict__ y = a.y;
        float* __restrict__ x = a.x;
        const XcdTiles tl((P + kBlock - 1) / kBlock, jb, nb);
        for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
            const int p = (int)(tile * kBlock) + threadIdx.x;
            if (p >= P) continue;
            const int64_t v = a.idx[p];
            // kSliceChunk channels' loads issued together (channels past C read
            // channel C - 1 and are not stored): a load and store per channel
            // would wait for each load in turn
            if (C == 1) {
                x[p] = y[v];
                continue;
            }
            for (int c0 = 0; c0 < C; c0 += kSliceChunk) {
                float t[kSliceChunk];
#pragma unroll
                for (int k = 0; k < kSliceChunk; ++k) t[k] = y[v * C + min(c0 + k, C - 1)];
#pragma unroll
                for (int k = 0; k < kSliceChunk; ++k)
                    if (c0 + k < C) x[(int64_t)(c0 + k) * P + p] = t[k];
            }
        }
    }
};

// dL/dt[c][p] = conf[p] g[idx[p]][c];  dL/dconf[p] = sum_c g[idx][c] (t[c][p] - y[idx][c]).
// g has stride Cg, y stride C.  The sum over channels is formed in float64
// from the float32 operands (each product and difference exact), so the
// only rounding is the final one: the channels' terms cancel where the
// solution follows the target, and float32 partial sums would add errors
// of the size of the terms.
struct GradScatter {
    static constexpr int kThreads = kBlock;
    struct Args {
        const int32_t* idx;
        const float* g;
        const float* yhat;
        const float* target;
        const float* conf;
        float* gt;
        float* gc;
        int Cg, C, P;
    };
    __device__ static void run(const Args& a, int jb, int nb, int) {
        const int C = a.C, P = a.P, Cg = a.Cg;
        const float* __restrict__ g = a.g;
        const float* __restrict__ yhat = a.yhat;
        const float* __restrict__ target = a.target;
        float* __restrict__ gt = a.gt;
        const XcdTiles tl((P + kBlock - 1) / kBlock, jb, nb);
        for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
            const int p = (int)(tile * kBlock) + threadIdx.x;
            if (p >= P) continue;
            const int64_t v = a.idx[p];
            const float cp = a.conf[p];
            double s = 0.0;
            // as in the slice, kSliceChunk channels' loads at a time; the
            // channels are summed in order
            if (C == 1) {
                const float gv = g[v * Cg];
                gt[p] = cp * gv;
                a.gc[p] = (float)((double)gv * ((double)target[p] - (double)yhat[v]));
                continue;
            }
            for (int c0 = 0; c0 < C; c0 += kSliceChunk) {
                float gv[kSliceChunk], tv[kSliceChunk], yv[kSliceChunk];
#pragma unroll
                for (int k = 0; k < kSliceChunk; ++k) {
                    const int c = min(c0 + k, C - 1);
                    gv[k] = g[v * Cg + c];
                    tv[k] = target[(int64_t)c * P + p];
                    yv[k] = yhat[v * C + c];
                }
#pragma unroll
                for (int k = 0; k < kSliceChunk; ++k) {
                    if (c0 + k < C) {
                        gt[(int64_t)(c0 + k) * P + p] = cp * gv[k];
                        s = fma((double)gv[k], (double)tv[k] - (double)yv[k], s);
                    }
                }
            }
            a.gc[p] = (float)s;
        }
    }
};

// ---------------------------------------------------------------------------
// Arguments of one image's launches.
// ---------------------------------------------------------------------------
// Arguments of the splat of image g into workspace w.
template <bool WEIGHTED>
typename SplatVertex<WEIGHTED>::Args splat_vertex_args(const GridImpl& g, const SolveWs& w,
                                                       const float* conf, const float* vals,
                                                       double lam) {
    typename SplatVertex<WEIGHTED>::Args a;
    a.ptr = g.lv[0].ptr;
    a.list = g.lv[0].list;
    a.conf = conf;
    a.vals = vals;
    a.nn = g.nn;
    a.nf = g.nf;
    a.counts = g.counts;
    a.o = SplatOut{w.sc, w.diag, w.minv, w.nfm, w.b};
    a.lam = lam;
    a.C = w.C;
    a.Cp = w.Cp;
    a.P = g.P;
    return a;
}

template <int B, int CAP, bool WEIGHTED>
typename SplatCells<B, CAP, WEIGHTED>::Args splat_cells_args(const GridImpl& g, const SolveWs& w,
                                                             const float* conf, const float* vals,
                                                             double lam) {
    const Level& L = g.lv[0];
    typename SplatCells<B, CAP, WEIGHTED>::Args a;
    a.cell_vbase = L.cell_vbase;
    a.cell_ibase = L.cell_ibase;
    a.ptr = L.ptr;
    a.list = L.list;
    a.conf = conf;
    a.vals = vals;
    a.nn = g.nn;
    a.nf = g.nf;
    a.o = SplatOut{w.sc, w.diag, w.minv, w.nfm, w.b};
    a.lam = lam;
    a.H = g.H;
    a.W = g.W;
    a.sxy = g.sg.sigma_xy;
    a.ncx = L.ncx;
    a.C = w.C;
    a.Cp = w.Cp;
    a.P = g.P;
    return a;
}

// Arguments of the initial-state kernels of image g, workspace w (into y,
// stride Cp), with the init level weights of p (alpha, beta).
inline FlatInit::Args flat_init_args(const GridImpl& g, const SolveWs& w, float* y) {
    return {w.b, w.sc, g.counts, y, w.Cp};
}

inline float level_weight(const bs_solve_params& p, int k) {
    return (float)std::pow((double)p.init_alpha, -((double)p.init_beta + k));
}

inline PyrUp::Args pyr_up_args(const GridImpl& g, const SolveWs& w, int k) {
    return {g.lv[k].ptr, g.lv[k].list, w.b, w.sc, k >= 2 ? w.up[k - 1] : nullptr, w.up[k],
            g.counts, w.Cp, k};
}

inline PyrDown::Args pyr_down_args(const GridImpl& g, const SolveWs& w, const bs_solve_params& p, int k) {
    const float* upp = (k + 1 < g.levels) ? w.up[k + 1] : nullptr;
    const int32_t* par = (k + 1 < g.levels) ? g.lv[k + 1].item_parent : nullptr;
    return {w.up[k], upp, par, g.lv[k].ones, g.counts, level_weight(p, k), w.Cp, k};
}

inline int small_pyr_level(const GridImpl& g, int C) {
    int k0 = 1;
    while (k0 < g.levels && g.lv[k0].cap * (C + 1) > kSmallPyrElems) ++k0;
    return k0;
}

inline PyrSmall::Args pyr_small_args(const GridImpl& g, const SolveWs& w, const bs_solve_params& p,
                              int k0) {
    PyrSmall::Args A;
    std::memset(&A, 0, sizeof(A));
    PyrLevels& a = A.lv;
    a.k0 = k0;
    a.levels = g.levels;
    for (int k = 1; k < g.levels; ++k) {
        a.cptr[k] = g.lv[k].ptr;
        a.clist[k] = g.lv[k].list;
        a.ones[k] = g.lv[k].ones;
        a.parent[k] = (k + 1 < g.levels) ? g.lv[k + 1].item_parent : nullptr;
        a.up[k] = w.up[k];
        a.wk[k] = level_weight(p, k);
    }
    A.b = w.b;
    A.sc = w.sc;
    A.counts = g.counts;
    A.C = w.Cp;
    return A;
}

inline HierFinal::Args hier_final_args(const GridImpl& g, const SolveWs& w, float* y) {
    return {w.b, w.sc, g.levels > 1 ? w.up[1] : nullptr,
            g.levels > 1 ? g.lv[1].item_parent : nullptr, g.counts, y, w.Cp};
}

}  // namespace bs
