// Kernel bodies of the grid and pyramid construction (paper Section 2,
// Eq. factorization and Eq. equiv; supplement Section 1 Eq. SS and Section 2),
// as Ops: the single-image entry points run them through one_launch, the
// batch engine through multi_launch.
#pragma once

#include "bs_internal.h"

namespace bs {

// ---------------------------------------------------------------------------
// Item sources of a level.
// ---------------------------------------------------------------------------

// 8-bit code of a [0, 1] value: clamp(floor(255 v + 1/2), 0, 255), NaN -> 0.
__device__ inline int quantise8(float v) {
    const double s = floor((double)v * 255.0 + 0.5);
    return s >= 255.0 ? 255 : (s >= 0.0 ? (int)s : 0);
}

__device__ inline int clamp255(int v) { return v < 0 ? 0 : (v > 255 ? 255 : v); }

// Level 0: the items of a cell are the pixels of an image rectangle.
struct PixelSource {
    const float* ref;
    int H, W, P, sxy, sl, suv, ncx;

    struct Ctx {
        int y0, x0, wx, n;
    };
    __device__ bool active(const int32_t*) const { return true; }
    __device__ Ctx ctx(int c, int& cy, int& cx) const {
        cy = c / ncx;
        cx = c - cy * ncx;
        Ctx t;
        t.y0 = cell_lo(cy, sxy);
        const int y1 = min(cell_lo(cy + 1, sxy), H);
        t.x0 = cell_lo(cx, sxy);
        const int x1 = min(cell_lo(cx + 1, sxy), W);
        t.wx = x1 - t.x0;
        t.n = (y1 - t.y0) * t.wx;
        return t;
    }
    __device__ int gid(const Ctx& t, int j) const {
        const int r = j / t.wx;
        return (t.y0 + r) * W + t.x0 + (j - r * t.wx);
    }
    // Colour key l:8 u:8 v:8 of a pixel: 8-bit RGB -> JFIF YCbCr (16.16 fixed
    // point, round half up) -> round_half_up(code / sigma).
    __device__ uint32_t key(const Ctx& t, int j) const {
        const int p = gid(t, j);
        const int r = quantise8(ref[p]);
        const int g = quantise8(ref[P + p]);
        const int b = quantise8(ref[2 * P + p]);
        const int yy = clamp255((19595 * r + 38470 * g + 7471 * b + 32768) >> 16);
        const int cb = clamp255((-11058 * r - 21710 * g + 32768 * b + 8421376) >> 16);
        const int cr = clamp255((32768 * r - 27439 * g - 5329 * b + 8421376) >> 16);
        return ((uint32_t)grid_coord(yy, sl) << 16) | ((uint32_t)grid_coord(cb, suv) << 8) |
               (uint32_t)grid_coord(cr, suv);
    }
};

// Level k >= 1: the items of cell (cy, cx) are the level-(k-1) vertices of the
// child cells (2cy + a, 2cx + b), a, b in {0, 1}, in ascending id order.
struct VertexSource {
    const uint64_t* child_key;
    const int32_t* child_vbase;
    const int32_t* counts;
    int child_ncx, child_ncy, ncx, level;

    struct Ctx {
        int s[4], len[4], n;
    };
    __device__ bool active(const int32_t* cnt) const { return cnt[CNT_LEVEL0 + level - 1] > 1; }
    __device__ Ctx ctx(int c, int& cy, int& cx) const {
        cy = c / ncx;
        cx = c - cy * ncx;
        Ctx t;
        t.n = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int yy = 2 * cy + (q >> 1), xx = 2 * cx + (q & 1);
            int s = 0, e = 0;
            if (yy < child_ncy && xx < child_ncx) {
                const int cc = yy * child_ncx + xx;
                s = child_vbase[cc];
                e = child_vbase[cc + 1];
            }
            t.s[q] = s;
            t.len[q] = e - s;
            t.n += e - s;
        }
        return t;
    }
    __device__ int gid(const Ctx& t, int j) const {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            if (j < t.len[q]) return t.s[q] + j;
            j -= t.len[q];
        }
        return t.s[3] + j;
    }
    __device__ uint32_t key(const Ctx& t, int j) const {
        const uint64_t k = child_key[gid(t, j)];
        const uint32_t l = (uint32_t)(k >> 16) & 0xffu, u = (uint32_t)(k >> 8) & 0xffu,
                       v = (uint32_t)k & 0xffu;
        return ((l >> 1) << 16) | ((u >> 1) << 8) | (v >> 1);
    }
};

// ---------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------
constexpr uint32_t kFirst = 0x80000000u;
constexpr uint32_t kKeyMask = 0x7fffffffu;

template <int B>
__device__ inline int block_sum_int(int v) {
    __shared__ int red[B / 64];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int s = 0;
#pragma unroll
    for (int w = 0; w < B / 64; ++w) s += red[w];
    return s;
}

// Cells with at most CAP items are sorted in LDS: the items' packed
// (colour key, item index) pairs are bitonic-sorted, so equal keys form runs in
// ascending item order.  Larger cells (only possible at coarse pyramid levels
// of unusual images) use a quadratic counting pass tiled through LDS; both
// give identical results.
// CAP is a power of two >= 64; the quadratic fallback tiles CAP items at a time
// through the same LDS.
template <int CAP>
struct CellSmem {
    uint64_t s[CAP];      // sorted (key << 32 | item) pairs
    int32_t rank[CAP];    // local vertex of each sorted position
    int32_t start[CAP];   // sorted position of each local vertex's first item
};

// Sorts the cell's (key, item) pairs ascending; returns the padded size.
template <int B, class Src>
__device__ inline int sort_cell(const Src& src, const typename Src::Ctx& t, int n,
                                uint64_t* __restrict__ s) {
    int N = 64;
    while (N < n) N <<= 1;
    for (int i = threadIdx.x; i < N; i += B)
        s[i] = i < n ? (((uint64_t)src.key(t, i) << 32) | (uint32_t)i) : ~0ull;
    __syncthreads();
    for (int k = 2; k <= N; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < N; i += B) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint64_t a = s[i], b = s[ixj];
                    if ((a > b) == ((i & k) == 0)) {
                        s[i] = b;
                        s[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    return N;
}

__device__ inline bool run_head(const uint64_t* s, int i) {
    return i == 0 || (s[i] >> 32) != (s[i - 1] >> 32);
}

// Pass 1: the number of distinct colour keys (future vertices) of each cell
// (block c: cell c).
template <int B, int CAP, class Src>
struct LevelCount {
    static constexpr int kThreads = B;
    struct Args {
        Src src;
        int32_t* cell_cnt;
        int32_t* cell_items;
        uint32_t* ikey;
        const int32_t* counts;
    };
    __device__ static void run(const Args& a, int c, int, int);
};

template <int B, int CAP, class Src>
__device__ inline void LevelCount<B, CAP, Src>::run(const Args& a, int c, int, int) {
    const Src& src = a.src;
    int32_t* __restrict__ cell_cnt = a.cell_cnt;
    int32_t* __restrict__ cell_items = a.cell_items;
    uint32_t* __restrict__ ikey = a.ikey;
    if (!src.active(a.counts)) return;
    __shared__ CellSmem<CAP> sm;
    int cy, cx;
    const typename Src::Ctx t = src.ctx(c, cy, cx);
    const int n = t.n;
    int cnt = 0;
    if (n <= CAP) {
        sort_cell<B>(src, t, n, sm.s);
        for (int i = threadIdx.x; i < n; i += B) cnt += run_head(sm.s, i) ? 1 : 0;
    } else {
        // quadratic fallback: flag the first occurrence of each key in item order
        uint32_t* tile = reinterpret_cast<uint32_t*>(sm.s);
        for (int base = 0; base < n; base += B) {
            const int i = base + threadIdx.x;
            const bool have = i < n;
            const uint32_t ki = have ? src.key(t, i) : 0u;
            bool first = have;
            const int jend = min(base + B, n);
            for (int t0 = 0; t0 < jend; t0 += CAP) {
                const int tn = min(CAP, jend - t0);
                __syncthreads();
                for (int j = threadIdx.x; j < tn; j += B) tile[j] = src.key(t, t0 + j);
                __syncthreads();
                if (first) {
                    const int lim = min(tn, i - t0);
                    for (int j = 0; j < lim; ++j) {
                        if (tile[j] == ki) {
                            first = false;
                            break;
                        }
                    }
                }
            }
            if (have) {
                ikey[src.gid(t, i)] = ki | (first ? kFirst : 0u);
                cnt += first ? 1 : 0;
            }
        }
    }
    cnt = block_sum_int<B>(cnt);
    if (threadIdx.x == 0) {
        cell_cnt[c] = cnt;
        cell_items[c] = n;
    }
}

// Pass 2: exclusive scan of the per-cell vertex and item counts (one block).
// Writes the level's vertex count and, when it reaches one vertex, the
// pyramid height K.
constexpr int kScanBlock = 1024;

struct LevelScan {
    static constexpr int kThreads = kScanBlock;
    struct Args {
        const int32_t* cnt;
        const int32_t* items;
        int32_t* vbase;
        int32_t* ibase;
        int32_t* ptr;
        int32_t* counts;
        int ncells, level;
    };
    __device__ static void run(const Args& a, int, int, int);
};

__device__ inline void LevelScan::run(const Args& A, int, int, int) {
    const int32_t* __restrict__ cnt = A.cnt;
    const int32_t* __restrict__ items = A.items;
    int32_t* __restrict__ vbase = A.vbase;
    int32_t* __restrict__ ibase = A.ibase;
    int32_t* __restrict__ ptr = A.ptr;
    int32_t* __restrict__ counts = A.counts;
    const int ncells = A.ncells, level = A.level;
    if (level > 0 && counts[CNT_LEVEL0 + level - 1] <= 1) {
        if (threadIdx.x == 0) counts[CNT_LEVEL0 + level] = 0;
        return;
    }
    __shared__ int sa[kScanBlock / 64], sb[kScanBlock / 64];
    const int tid = threadIdx.x;
    const int chunk = (ncells + kScanBlock - 1) / kScanBlock;
    const int s = min(tid * chunk, ncells), e = min(s + chunk, ncells);
    int a = 0, b = 0;
    for (int i = s; i < e; ++i) {
        a += cnt[i];
        b += items[i];
    }
    // inclusive wave scan
    const int lane = tid & 63, wave = tid >> 6;
    int ia = a, ib = b;
    for (int o = 1; o < 64; o <<= 1) {
        const int ta = __shfl_up(ia, o, 64), tb = __shfl_up(ib, o, 64);
        if (lane >= o) {
            ia += ta;
            ib += tb;
        }
    }
    if (lane == 63) {
        sa[wave] = ia;
        sb[wave] = ib;
    }
    __syncthreads();
    int wa = 0, wb = 0, ta = 0, tb = 0;
    for (int w = 0; w < kScanBlock / 64; ++w) {
        if (w < wave) {
            wa += sa[w];
            wb += sb[w];
        }
        ta += sa[w];
        tb += sb[w];
    }
    int pa = wa + ia - a, pb = wb + ib - b;
    for (int i = s; i < e; ++i) {
        vbase[i] = pa;
        ibase[i] = pb;
        pa += cnt[i];
        pb += items[i];
    }
    if (tid == 0) {
        vbase[ncells] = ta;
        ibase[ncells] = tb;
        ptr[ta] = tb;
        counts[CNT_LEVEL0 + level] = ta;
        if (level == 0) {
            counts[CNT_V] = ta;
            counts[CNT_K] = (ta == 1) ? 0 : -1;
            counts[CNT_BIST_DONE] = 0;
            counts[CNT_BIST_ITERS] = 0;
            counts[CNT_BIST_SRC] = 0;
        } else if (ta == 1 && counts[CNT_K] < 0) {
            counts[CNT_K] = level;
        }
    }
}

// Pass 3: per cell, the vertex of each item, the vertices' keys,
// multiplicities and P(1) sums, and the item CSR (items of a vertex in
// ascending item order).
template <int B, int CAP, class Src>
struct LevelWrite {
    static constexpr int kThreads = B;
    struct Args {
        Src src;
        const uint32_t* ikey;
        const int32_t* ones_prev;
        const int32_t* counts;
        Level L;
    };
    __device__ static void run(const Args& a, int c, int, int);
};

template <int B, int CAP, class Src>
__device__ inline void LevelWrite<B, CAP, Src>::run(const Args& a, int c, int, int) {
    const Src& src = a.src;
    const uint32_t* __restrict__ ikey = a.ikey;
    const int32_t* __restrict__ ones_prev = a.ones_prev;
    const Level& L = a.L;
    if (!src.active(a.counts)) return;
    __shared__ CellSmem<CAP> sm;
    __shared__ int wsum[B / 64];
    int cy, cx;
    const typename Src::Ctx t = src.ctx(c, cy, cx);
    const int n = t.n;
    const int vbase = L.cell_vbase[c], ibase = L.cell_ibase[c];
    const uint64_t cellkey = ((uint64_t)cy << 40) | ((uint64_t)cx << 24);
    if (n <= CAP) {
        const int N = sort_cell<B>(src, t, n, sm.s);
        // local vertex of each sorted position: inclusive scan of run heads
        const int per = (N + B - 1) / B;
        const int i0 = threadIdx.x * per;
        int local = 0;
        for (int q = 0; q < per; ++q) {
            const int i = i0 + q;
            if (i < n && run_head(sm.s, i)) ++local;
        }
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        int incl = local;
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        int before = incl - local;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        const int cnt = [&] {
            int tot = 0;
            for (int w = 0; w < B / 64; ++w) tot += wsum[w];
            return tot;
        }();
        int r = before - 1;
        for (int q = 0; q < per; ++q) {
            const int i = i0 + q;
            if (i >= n) break;
            if (run_head(sm.s, i)) {
                ++r;
                sm.start[r] = i;
            }
            sm.rank[i] = r;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += B) {
            const int r2 = sm.rank[i];
            const int gi = src.gid(t, (int)(sm.s[i] & 0xffffffffu));
            const int v = vbase + r2;
            L.item_parent[gi] = v;
            L.list[ibase + i] = gi;
            if (sm.start[r2] == i) {
                const int end = (r2 + 1 < cnt) ? sm.start[r2 + 1] : n;
                L.key[v] = cellkey | (sm.s[i] >> 32);
                L.ptr[v] = ibase + i;
                L.mult[v] = end - i;
                if (L.ones) {
                    int sum = 0;
                    for (int q = i; q < end; ++q)
                        sum += ones_prev ? ones_prev[src.gid(t, (int)(sm.s[q] & 0xffffffffu))] : 1;
                    L.ones[v] = sum;
                }
            }
        }
        return;
    }
    // quadratic fallback, using the first-occurrence flags of pass 1
    uint32_t* tile = reinterpret_cast<uint32_t*>(sm.s);
    int32_t* tones = reinterpret_cast<int32_t*>(sm.s) + CAP;
    for (int base = 0; base < n; base += B) {
        const int i = base + threadIdx.x;
        const bool have = i < n;
        const int gi = have ? src.gid(t, i) : 0;
        const uint32_t wi = have ? ikey[gi] : 0u;
        const uint32_t ki = wi & kKeyMask;
        int rank = 0, less = 0, mult = 0, eqb = 0, onesum = 0;
        for (int t0 = 0; t0 < n; t0 += CAP) {
            const int tn = min(CAP, n - t0);
            __syncthreads();
            for (int j = threadIdx.x; j < tn; j += B) {
                const int gj = src.gid(t, t0 + j);
                tile[j] = ikey[gj];
                tones[j] = ones_prev ? ones_prev[gj] : 1;
            }
            __syncthreads();
            if (have) {
                for (int j = 0; j < tn; ++j) {
                    const uint32_t w = tile[j];
                    const uint32_t kj = w & kKeyMask;
                    const int lt = kj < ki, eq = kj == ki;
                    less += lt;
                    rank += lt & (int)(w >> 31);
                    mult += eq;
                    eqb += eq & (t0 + j < i);
                    onesum += eq ? tones[j] : 0;
                }
            }
        }
        if (have) {
            const int v = vbase + rank;
            L.item_parent[gi] = v;
            if (wi & kFirst) {
                L.key[v] = cellkey | ki;
                L.mult[v] = mult;
                L.ptr[v] = ibase + less;
                if (L.ones) L.ones[v] = onesum;
            }
            L.list[ibase + less + eqb] = gi;
        }
    }
}

// Neighbour table of level 0: for each vertex and unit step along each of
// (y, x, l, u, v), the neighbour's id or -1.  Colour neighbours share the
// vertex's spatial cell; spatial neighbours lie in the adjacent cell; both are
// looked up in that cell's key range.  The table is written twice: as 32-bit
// ids, and packed as 16-bit offsets from the vertex (half the bytes for the
// stencil passes of grids whose offsets provably fit); a vertex whose offset
// does not fit sets CNT_NB_WIDE.
struct NeighbourTable {
    static constexpr int kThreads = kBlock;
    struct Args {
        const uint64_t* key;
        const int32_t* vbase;
        int32_t* counts;
        int32_t* nbr;
        uint32_t* nb16;
        int64_t vcap;
        int ncx, ncy;
    };
    __device__ static void run(const Args& a, int jb, int nb, int);
};

__device__ inline void NeighbourTable::run(const Args& a, int jb, int nb, int) {
    const uint64_t* __restrict__ key = a.key;
    const int32_t* __restrict__ vbase = a.vbase;
    int32_t* __restrict__ counts = a.counts;
    int32_t* __restrict__ nbr = a.nbr;
    uint32_t* __restrict__ nb16 = a.nb16;
    const int64_t vcap = a.vcap;
    const int ncx = a.ncx, ncy = a.ncy;
    const int V = counts[CNT_V];
    const int ncells = ncx * ncy;
    const XcdTiles tl((V + kBlock - 1) / kBlock, jb, nb);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int v = (int)(tile * kBlock) + threadIdx.x;
        if (v >= V) continue;
        const uint64_t k = key[v];
        const int cy = (int)(k >> 40), cx = (int)((k >> 24) & 0xffff);
        const int cell = cy * ncx + cx;
        // the key ranges of the ten searches: the cells above, below, left and
        // right (read from clamped cell indices, empty where there is no such
        // cell), and the vertex's own cell for the colour steps
        const int up = max(cell - ncx, 0), dn = min(cell + ncx, ncells - 1);
        const int lf = max(cell - 1, 0), rt = min(cell + 1, ncells - 1);
        const int b_up0 = vbase[up], b_up1 = vbase[up + 1];
        const int b_dn0 = vbase[dn], b_dn1 = vbase[dn + 1];
        const int b_lf0 = vbase[lf], s = vbase[cell], e = vbase[cell + 1];
        const int b_rt1 = vbase[rt + 1];
        int lo[10], hi[10];
        uint64_t want[10];
        lo[0] = b_up0; hi[0] = cy > 0 ? b_up1 : b_up0; want[0] = k - (1ull << 40);
        lo[1] = b_dn0; hi[1] = cy + 1 < ncy ? b_dn1 : b_dn0; want[1] = k + (1ull << 40);
        lo[2] = b_lf0; hi[2] = cx > 0 ? s : b_lf0; want[2] = k - (1ull << 24);
        lo[3] = e; hi[3] = cx + 1 < ncx ? b_rt1 : e; want[3] = k + (1ull << 24);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int sh = 16 - 8 * d;
            const int f = (int)((k >> sh) & 0xff);
            lo[4 + 2 * d] = s;
            hi[4 + 2 * d] = f > 0 ? e : s;
            want[4 + 2 * d] = k - (1ull << sh);
            lo[5 + 2 * d] = s;
            hi[5 + 2 * d] = f < 255 ? e : s;
            want[5 + 2 * d] = k + (1ull << sh);
        }
        // the ten binary searches in lockstep: every round reads the midpoint
        // of each unfinished search (finished ones read key 0), so their loads
        // are in flight together rather than one search's chain after another
        int rr[10];
#pragma unroll
        for (int j = 0; j < 10; ++j) rr[j] = -1;
        for (bool any = true; any;) {
            int mid[10];
            uint64_t kv[10];
#pragma unroll
            for (int j = 0; j < 10; ++j) mid[j] = lo[j] < hi[j] ? (lo[j] + hi[j]) >> 1 : 0;
#pragma unroll
            for (int j = 0; j < 10; ++j) kv[j] = key[mid[j]];
            any = false;
#pragma unroll
            for (int j = 0; j < 10; ++j) {
                if (lo[j] < hi[j]) {
                    if (kv[j] == want[j]) {
                        rr[j] = mid[j];
                        hi[j] = lo[j];
                    } else if (kv[j] < want[j]) {
                        lo[j] = mid[j] + 1;
                    } else {
                        hi[j] = mid[j];
                    }
                    any = any || lo[j] < hi[j];
                }
            }
        }
        bool fits = true;
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            nbr[j * vcap + v] = rr[j];
            if (rr[j] >= 0) fits = fits && rr[j] - v >= -kNbOffsetMax && rr[j] - v <= kNbOffsetMax;
        }
#pragma unroll
        for (int i = 0; i < 5; ++i) nb16[i * vcap + v] = pack_offsets(v, rr[2 * i], rr[2 * i + 1]);
        if (!fits) counts[CNT_NB_WIDE] = 1;
    }
}

struct ClearCounts {
    static constexpr int kThreads = 64;
    struct Args {
        int32_t* counts;
    };
    __device__ static void run(const Args& a, int, int, int) {
        const int t = threadIdx.x;
        if (t < CNT_SIZE) a.counts[t] = 0;
    }
};

inline NeighbourTable::Args neighbour_args(const GridImpl& g) {
    return {g.lv[0].key, g.lv[0].cell_vbase, g.counts, g.nbr, g.nb16, g.vcap, g.lv[0].ncx,
            g.lv[0].ncy};
}

// Arguments of the three passes of level k of a grid, items from `src`.
template <int B, int CAP, class Src>
typename LevelCount<B, CAP, Src>::Args level_count_args(const Src& src, const GridImpl& g) {
    return {src, g.cell_cnt, g.cell_items, g.ikey, g.counts};
}
inline LevelScan::Args level_scan_args(const GridImpl& g, int k) {
    const Level& L = g.lv[k];
    return {g.cell_cnt, g.cell_items, L.cell_vbase, L.cell_ibase, L.ptr, g.counts,
            L.ncy * L.ncx, k};
}
template <int B, int CAP, class Src>
typename LevelWrite<B, CAP, Src>::Args level_write_args(const Src& src, const GridImpl& g, int k) {
    return {src, g.ikey, (k >= 2) ? g.lv[k - 1].ones : nullptr, g.counts, g.lv[k]};
}

}  // namespace bs
