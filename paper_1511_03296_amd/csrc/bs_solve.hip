// The bilateral-space solve (paper Eq. quad_min and Eq. solution, supplement
// Algorithm 2, Section 4 initialisation) and its backward pass (Section 3).
//
// Layouts: pixel planes [C][P] float32; bilateral-space vectors [V][Cp]
// float32, channels contiguous per vertex.  A lane of the vertex kernels owns
// K consecutive channels of one vertex: K = C for C <= 2, else 4 when 4
// divides C, 3 when 3 does, 4 otherwise (one float, float2, 3-float or float4
// access).  The channel stride Cp is C rounded up to a multiple of K (padding
// channels hold zeros and never iterate); Lv = Cp / K lanes cover a vertex, so
// the neighbour table and the per-vertex scalars are read by Lv lanes rather
// than by every channel.
//
// PCG (supplement Algorithm 2) runs one independent PCG per channel.  One
// iteration is two kernels, each with one grid-wide reduction:
//   pcg_matvec:  z = M^-1 r,  d = z + beta d,  q = A d,  d^T q;
//   pcg_update:  y += alpha d,  r -= alpha q,  r^T r,  r^T M^-1 r.
// The step y += alpha d is taken by the next matvec, which reads d anyway
// (for lanes of 2 and more channels every other matvec takes two steps).
// With the Jacobi preconditioner the residual is stored scaled, as
// w = n o M^-1 r (s = n M^-1 per vertex): the neighbours' share of A z is
// n o z = w, so the matvec gathers the stored residual itself, and
// z = w / n, r = w / s are recovered per vertex (r = 0 on a row with
// diag(A) = 0, where s = 0).  The new d is not stored before the reduction
// that yields beta, so the matvec either recomputes the neighbours' new d
// from their gathered w, old d and n (two gathered vectors), or, on 3 of
// every 4 iterations, takes q = A z + beta q by linearity and gathers w
// alone.  (With the hierarchical preconditioner r is stored as it is, and z
// beside it in w.)
// A z is evaluated in Laplacian form,
//   (A z)_v = (S c)_v z_v + lam n_v sum_u n_u (z_v - z_u),
// which equals diag(A) z - lam n o N(n o z) with diag(A) = lam n o N n + S c,
// but cancels constants exactly and keeps float32 rounding relative to the
// result rather than to lam m z (the difference matters where confidence is
// sparse).  Dot products accumulate in float64; the next kernel reduces the
// per-block partials in its prologue in a fixed order, so results are
// deterministic and no host synchronisation is needed.
//
// The PCG kernels take either one image or a table of images: a batch of
// images of any sizes runs each PCG phase as one launch, every block working
// on one image (a per-block image table), each image with its own channel
// state, partials and stopping rule.
#include "bs_setup_ops.h"
#include "bs_solve_impl.h"
#include <atomic>
#include <type_traits>

namespace bs {

enum Ctl : int { CTL_SIZE = 8 };

// A pointer into global memory.  The PCG kernels reach their vectors through
// such typed pointers: pointers read from a table in memory carry no address
// space, and accesses through them would be flat instructions, which also
// count against the LDS counter (every LDS wait would then wait for the
// outstanding memory loads too).
// (The host compilation pass only type-checks the kernels; there it is a
// plain pointer.  No value of this type crosses between host and device.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T>
using gp = __attribute__((address_space(1))) T*;
#else
template <class T>
using gp = T*;
#endif

size_t layout_solve(const GridImpl& g, int C, int nb, void* base, SolveWs& w) {
    w.C = C;
    w.Cp = padded_channels(C);
    w.K = lane_width(C);
    w.nb = nb > 0 ? nb : solve_blocks(g, C);
    Carver c(base);
    const int64_t n = g.vcap * w.Cp;
    w.sc = c.take<float>(g.vcap);
    w.diag = c.take<float>(g.vcap);
    w.minv = c.take<float>(g.vcap);
    w.nfm = c.take<float2>(g.vcap);
    w.b = c.take<float>(n);
    w.r = c.take<float>(n);
    w.d[0] = c.take<float>(n);
    w.d[1] = c.take<float>(n);
    w.q = c.take<float>(n);
    w.w = c.take<float>(n);
    w.yi = c.take<float>(n);
    w.up[0] = nullptr;
    for (int k = 1; k < BS_MAX_LEVELS; ++k)
        w.up[k] = (k < g.levels) ? c.take<float>(g.lv[k].cap * (w.Cp + 1)) : nullptr;
    w.cs[0] = c.take<ChanRec>((int64_t)w.nb * w.Cp);
    w.cs[1] = c.take<ChanRec>((int64_t)w.nb * w.Cp);
    w.part[0] = c.take<double>((int64_t)3 * w.Cp * w.nb);
    w.part[1] = c.take<double>((int64_t)3 * w.Cp * w.nb);
    w.sums[0] = c.take<double>(3 * w.Cp);
    w.sums[1] = c.take<double>(3 * w.Cp);
    w.act = c.take<int32_t>(CTL_SIZE);
    w.bytes = align_up(c.off, 256);
    return w.bytes;
}

int solve_blocks(const GridImpl& g, int C) {
    return red_grid(g.vcap * (padded_channels(C) / lane_width(C)));
}

// ---------------------------------------------------------------------------
// K-wide lane values.
// ---------------------------------------------------------------------------
template <int K>
struct Vec {
    float v[K];
};

template <int K>
__device__ inline Vec<K> ldv(gp<const float> p) {
    Vec<K> o;
    if constexpr (K == 4) {
        const float4 t = *reinterpret_cast<gp<const float4>>(p);
        o.v[0] = t.x;
        o.v[1] = t.y;
        o.v[2] = t.z;
        o.v[3] = t.w;
    } else if constexpr (K == 2) {
        const float2 t = *reinterpret_cast<gp<const float2>>(p);
        o.v[0] = t.x;
        o.v[1] = t.y;
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) o.v[k] = p[k];
    }
    return o;
}

template <int K>
__device__ inline void stv(gp<float> p, const Vec<K>& a) {
    if constexpr (K == 4) {
        *reinterpret_cast<gp<float4>>(p) = make_float4(a.v[0], a.v[1], a.v[2], a.v[3]);
    } else if constexpr (K == 2) {
        *reinterpret_cast<gp<float2>>(p) = make_float2(a.v[0], a.v[1]);
    } else {
#pragma unroll
        for (int k = 0; k < K; ++k) p[k] = a.v[k];
    }
}

// Element e of a vector as a 32-bit byte offset from its base: the base is
// uniform over the block, so the loads and stores take the offset as their
// only address register (no 64-bit address arithmetic per gather).  The
// host keeps every [Vcap][Cp] vector below 2^30 elements.
template <class T>
__device__ inline gp<T> elem(gp<T> base, uint32_t e) {
    using C = std::conditional_t<std::is_const_v<T>, const char, char>;
    return reinterpret_cast<gp<T>>(reinterpret_cast<gp<C>>(base) + (e * (uint32_t)sizeof(T)));
}

template <int K>
__device__ inline Vec<K> ldv(gp<const float> base, uint32_t e) {
    return ldv<K>(elem(base, e));
}
template <int K>
__device__ inline Vec<K> ldv(gp<float> base, uint32_t e) {
    return ldv<K>(elem((gp<const float>)base, e));
}
template <int K>
__device__ inline void stv(gp<float> base, uint32_t e, const Vec<K>& a) {
    stv<K>(elem(base, e), a);
}

// Element offset of lane g's K channels of vertex v (stride Cp).
__device__ inline uint32_t lane_elem(int v, int Cp, int g, int K) {
    return (uint32_t)v * (uint32_t)Cp + (uint32_t)(g * K);
}

// Lane geometry of one image: lane t owns channels [g K, g K + K) of the
// tile's vertex vl.
struct Lanes {
    int Lv, vpb, vl, g;
    bool ok;
    __device__ Lanes(int Cp, int K) {
        Lv = Cp / K;
        vpb = kRedBlock / Lv;
        vl = (int)threadIdx.x / Lv;
        g = (int)threadIdx.x - vl * Lv;
        ok = vl < vpb;
    }
};

// ---------------------------------------------------------------------------
// Reductions over the lanes of a block.
// ---------------------------------------------------------------------------

// Sums NV x K per-lane values over the vertices of the block, per channel,
// with a fixed tree, and writes the block's partials to
// part[(k Cp + ch) nb + slot].
template <int NV, int K>
__device__ inline void lane_partials(const double (&acc)[NV][K], const Lanes& ln, int Cp,
                                     int nb, int slot, gp<double> part) {
    const int t = threadIdx.x;
    if (ln.Lv == 1) {
        // one lane per vertex: shuffle trees per wave, then one pass over the waves
        __shared__ double red[NV * K][kRedBlock / 64];
        double v[NV * K];
#pragma unroll
        for (int i = 0; i < NV * K; ++i) v[i] = wave_sum(acc[i / K][i % K]);
        __syncthreads();
        if ((t & 63) == 0) {
#pragma unroll
            for (int i = 0; i < NV * K; ++i) red[i][t >> 6] = v[i];
        }
        __syncthreads();
        if (t < NV * K) {
            double s = 0.0;
            for (int w = 0; w < kRedBlock / 64; ++w) s += red[t][w];
            part[((int64_t)(t / K) * Cp + t % K) * nb + slot] = s;
        }
        return;
    }
    // one tree for all NV x K values: every index below is a constant
    __shared__ double s[NV * K][kRedBlock];
#pragma unroll
    for (int i = 0; i < NV * K; ++i) s[i][t] = acc[i / K][i % K];
    __syncthreads();
    int n = ln.vpb;
    while (n > 1) {
        const int h = (n + 1) >> 1;
        if (t < (n - h) * ln.Lv) {
#pragma unroll
            for (int i = 0; i < NV * K; ++i) s[i][t] += s[i][t + h * ln.Lv];
        }
        __syncthreads();
        n = h;
    }
    if (t < ln.Lv) {
#pragma unroll
        for (int i = 0; i < NV * K; ++i)
            part[((int64_t)(i / K) * Cp + t * K + i % K) * nb + slot] = s[i][t];
    }
}

// out[k Cp + ch] = sum over the nb blocks of the producer's partials,
// computed identically by every block.  The pair sums are spread over the
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
    gp<const double> pre;   // sums already reduced by pcg_reduce, or nullptr

    // Lanes per pair for `pairs` sums over G partials, and whether each lane's
    // share fits in registers (the host uses the same rule to decide when to
    // run pcg_reduce instead).
    // (q divides G, so that the q lanes of a sum share its G partials evenly.)
    __host__ __device__ static int lanes(int pairs, int G) {
        int q = 64;
        while (q > 1 && (q * pairs > kRedBlock || G % q != 0)) q >>= 1;
        return q;
    }
    __host__ __device__ static bool fits(int pairs, int G) {
        const int q = lanes(pairs, G);
        return pairs * q <= kRedBlock && G / q <= kMax;
    }

    __device__ void load(gp<const double> part, int nv_c, int grid,
                         gp<const double> sums = nullptr) {
        pre = sums;
        pairs = nv_c;
        G = grid;
        if (pre) {
            if ((int)threadIdx.x < pairs) v[0] = pre[threadIdx.x];
            return;
        }
        q = lanes(pairs, G);
        pair = threadIdx.x / q;
        seg = threadIdx.x - pair * q;
        held = fits(pairs, G);
        if (held && pair < pairs) {
#pragma unroll
            for (int i = 0; i < kMax; ++i)
                if (i < G / q) v[i] = part[(int64_t)pair * G + seg + q * i];
        }
    }

    __device__ void sum(gp<const double> part, double* out) {
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
__device__ inline void reduce_partials(gp<const double> part, int Cp, int G, double* out,
                                       gp<const double> sums = nullptr) {
    PartialSums ps;
    ps.load(part, NV * Cp, G, sums);
    ps.sum(part, out);
}

// Field-wise copies of a channel state: whole-struct copies leave parts of
// the state in private memory (spilled to LDS or scratch).
__device__ inline ChanState load_state(const ChanState& r) {
    ChanState s;
    s.rho = r.rho;
    s.alpha = r.alpha;
    s.alpha_prev = r.alpha_prev;
    s.beta = r.beta;
    s.bnorm = r.bnorm;
    s.res = r.res;
    s.active = r.active;
    s.iters = r.iters;
    s.reason = r.reason;
    s.phase = r.phase;
    return s;
}

__device__ inline void store_state(ChanState& d, const ChanState& s) {
    d.rho = s.rho;
    d.alpha = s.alpha;
    d.alpha_prev = s.alpha_prev;
    d.beta = s.beta;
    d.bnorm = s.bnorm;
    d.res = s.res;
    d.active = s.active;
    d.iters = s.iters;
    d.reason = s.reason;
    d.phase = s.phase;
}

__device__ inline ChanState load_state(gp<const ChanRec> p) {
    ChanState s;
    s.rho = p->s.rho;
    s.alpha = p->s.alpha;
    s.alpha_prev = p->s.alpha_prev;
    s.beta = p->s.beta;
    s.bnorm = p->s.bnorm;
    s.res = p->s.res;
    s.active = p->s.active;
    s.iters = p->s.iters;
    s.reason = p->s.reason;
    s.phase = p->s.phase;
    return s;
}

__device__ inline void store_state(gp<ChanRec> p, const ChanState& s) {
    p->s.rho = s.rho;
    p->s.alpha = s.alpha;
    p->s.alpha_prev = s.alpha_prev;
    p->s.beta = s.beta;
    p->s.bnorm = s.bnorm;
    p->s.res = s.res;
    p->s.active = s.active;
    p->s.iters = s.iters;
    p->s.reason = s.reason;
    p->s.phase = s.phase;
}

__device__ inline ChanState zero_state() {
    ChanState z;
    z.rho = z.alpha = z.beta = z.bnorm = z.res = z.alpha_prev = 0.0;
    z.active = z.iters = z.reason = z.phase = 0;
    return z;
}

// Completes the previous PCG step of one channel from the reduced slot-0
// partials: the initial residual (phase 0) or the end of an iteration, with
// the stopping rule and the next beta.
__device__ inline ChanState advance_state(const ChanState& st, double rr, double bb,
                                          double rho_new, int max_iters, double tol) {
    ChanState o = load_state(st);
    if (st.phase != 0 && !st.active) return o;
    int reason = 0;
    if (st.phase == 0) {
        o.phase = 1;
        o.bnorm = sqrt(bb);
        o.rho = rho_new;
        o.beta = 0.0;
        o.iters = 0;
        o.res = bb == 0.0 ? 0.0 : sqrt(rr) / o.bnorm;
        if (bb == 0.0) reason = 5;
        else if (o.res <= tol) reason = 1;
        else if (max_iters <= 0) reason = 2;
        else if (rho_new == 0.0) reason = 3;
    } else {
        o.beta = rho_new / st.rho;
        o.rho = rho_new;
        o.iters = st.iters + 1;
        o.res = sqrt(rr) / st.bnorm;
        if (o.res <= tol) reason = 1;
        else if (o.iters >= max_iters) reason = 2;
        else if (rho_new == 0.0) reason = 3;
    }
    o.active = reason == 0;
    o.reason = reason ? reason : st.reason;
    return o;
}

// ---------------------------------------------------------------------------
// Splat and initialisation (per image).
// ---------------------------------------------------------------------------

// Launches the splat: per cell when a cell's pixels fit the LDS staging,
// otherwise per vertex.
template <bool WEIGHTED>
static bs_status launch_splat(const GridImpl& g, const SolveWs& w, const float* conf,
                              const float* vals, double lam, hipStream_t s) {
    const Level& L = g.lv[0];
    const int ncells = L.ncx * L.ncy;
#define BS_SPLAT_CELLS(B, CAP)                                                                 \
    BS_LAUNCH(s, K_SPLAT, "splat_cells", (one_launch<SplatCells<B, CAP, WEIGHTED>>),            \
              dim3(ncells), dim3(B), 0, s,                                                      \
              (splat_cells_args<B, CAP, WEIGHTED>(g, w, conf, vals, lam)), 0)
    switch (splat_kind(g.sg.sigma_xy)) {
        case 0: BS_SPLAT_CELLS(64, 64); break;
        case 1: BS_SPLAT_CELLS(256, 256); break;
        case 2: BS_SPLAT_CELLS(256, 1024); break;
        default: {
            const int vblocks = grid_blocks(ceil_div(g.vcap, kBlock));
            BS_LAUNCH(s, K_SPLAT, "splat", one_launch<SplatVertex<WEIGHTED>>, dim3(vblocks),
                      dim3(kBlock), 0, s, (splat_vertex_args<WEIGHTED>(g, w, conf, vals, lam)),
                      0);
        }
    }
#undef BS_SPLAT_CELLS
    return BS_OK;
}

// Every lane width takes q by its recurrence and computes q = A d directly
// every kExactEvery-th iteration (iterations it with
// (it + 1) % kExactEvery == 0).  The recurrence accumulates the rounding of
// every A z it adds, while A d shrinks as d grows smooth, so near the float32
// floor of an ill-conditioned system (sparse confidence) q drifts from A d
// and the iteration diverges unless the drift is reset often enough (on a
// 2048x1536 depth super-resolution backward pass every 8 iterations sufficed
// and every 16 did not; every 4 costs 765 iterations against 730 without the
// recurrence).  The recurrence form gathers one vector per neighbour instead
// of three, and its matvec is the faster for every lane width (a depth
// launch averages 31.5 us with it against 35.4 without; with 3 channels per
// lane a 16-image launch takes 384 us against 565 for the exact form).
constexpr int kExactEvery = 4;
template <int K>
constexpr bool uses_recurrence() { return K >= 1; }

// Whether iteration `it` of a K-lane PCG computes q = A d directly.
template <int K>
inline bool exact_iteration(int it) {
    return !uses_recurrence<K>() || (it + 1) % kExactEvery == 0;
}

// ---------------------------------------------------------------------------
// PCG kernels.  Each takes one image (MULTI false, by value) or a table of
// images with the image of every block (MULTI true).
// ---------------------------------------------------------------------------

// In a launch over an image table, blocks past the images' blocks (a
// schedule of fewer blocks than the launch's) have no image and return.
template <bool MULTI>
__device__ inline bool idle_block(const PcgArgs& a) {
    if constexpr (MULTI) return a.blk2img[blockIdx.x] < 0;
    else return false;
}

template <bool MULTI>
__device__ inline const PcgImage& block_image(const PcgArgs& a, int& jb) {
    if constexpr (MULTI) {
        const PcgImage& I = a.imgs[a.blk2img[blockIdx.x]];
        jb = (int)blockIdx.x - I.block0;
        return I;
    } else {
        jb = (int)blockIdx.x;
        return a.one;
    }
}

// The kernels' view of one image: the descriptor's fields as separate
// scalars (run-time indices into its two-slot arrays would keep a copy in
// private memory), with every pointer typed global.
struct ImgView {
    gp<const int32_t> nbr;
    gp<const uint32_t> nb16;
    gp<const float2> nfm;
    gp<const float> sc;
    gp<const float> b;
    gp<float> y;
    gp<float> r;
    gp<float> d0;
    gp<float> d1;
    gp<float> q;
    gp<float> w;
    gp<const int32_t> counts;
    gp<ChanRec> cs0;
    gp<ChanRec> cs1;
    gp<double> part0;
    gp<double> part1;
    gp<const double> sums0;
    gp<const double> sums1;
    gp<double> wsums0;
    gp<double> wsums1;
    gp<int32_t> active;
    gp<bs_chan_stats> stats;
    int64_t vcap;
    float lam;
    int C, Cp, nb;
    int zmode;
};

__device__ inline ImgView view_of(const PcgImage& s) {
    ImgView I;
    I.nbr = (gp<const int32_t>)s.nbr;
    I.nb16 = (gp<const uint32_t>)s.nb16;
    I.nfm = (gp<const float2>)s.nfm;
    I.sc = (gp<const float>)s.sc;
    I.b = (gp<const float>)s.b;
    I.y = (gp<float>)s.y;
    I.r = (gp<float>)s.r;
    I.d0 = (gp<float>)s.d[0];
    I.d1 = (gp<float>)s.d[1];
    I.q = (gp<float>)s.q;
    I.w = (gp<float>)s.w;
    I.counts = (gp<const int32_t>)s.counts;
    I.cs0 = (gp<ChanRec>)s.cs[0];
    I.cs1 = (gp<ChanRec>)s.cs[1];
    I.part0 = (gp<double>)s.part[0];
    I.part1 = (gp<double>)s.part[1];
    I.wsums0 = (gp<double>)s.sums[0];
    I.wsums1 = (gp<double>)s.sums[1];
    I.sums0 = I.wsums0;
    I.sums1 = I.wsums1;
    I.active = (gp<int32_t>)s.active;
    I.stats = (gp<bs_chan_stats>)s.stats;
    I.vcap = s.vcap;
    I.lam = s.lam;
    I.C = s.C;
    I.Cp = s.Cp;
    I.nb = s.nb;
    I.zmode = s.zmode;
    return I;
}

// Neighbour indices of vertex v (phase 1 of a tile's loads): five packed
// words when every image of the launch has a packed table, else ten ids.
template <bool PACKED>
__device__ inline void load_nbr(int (&nb)[10], int v, const ImgView& I) {
    load_neighbours(nb, v, I.vcap, PACKED, I.nbr, I.nb16);
}

// The packed words of vertex v as loaded (raw[0..4]), decoded only where the
// gathers are formed (load_ops_late), which keeps the wait for them out of
// the previous tile's arithmetic.  Measured on one-channel single images,
// both matvec forms gain (the 1.58 M-vertex depth matvec: 30.8 us per launch
// on average, 25.7 with the recurrence form decoding late, 24.7 with both).
// In launches over an image table it sped the one-channel recurrence form by
// a fifth but slowed the one-channel exact form (8 %), the two-channel
// recurrence (4 %) and 21-channel lanes (6 %), whose live ranges across the
// tile loop grow instead; those launches decode early.
__device__ inline void load_nbr_words(int (&raw)[10], int v, const ImgView& I) {
#pragma unroll
    for (int i = 0; i < 5; ++i) raw[i] = (int)I.nb16[i * I.vcap + v];
}

template <int K, bool EXACT, bool PACKED, bool MULTI>
constexpr bool late_decode() { return K == 1 && PACKED && !MULTI; }

// Clears the channel state; the image is active until its first stop test.
template <bool MULTI>
__global__ void __launch_bounds__(kRedBlock) pcg_prologue(PcgArgs a) {
    int jb;
    if (idle_block<MULTI>(a)) return;
    const ImgView I = view_of(block_image<MULTI>(a, jb));
    const int t = threadIdx.x;
    if (t < I.Cp) {
        const ChanState z = zero_state();
        store_state(I.cs0 + (int64_t)jb * I.Cp + t, z);
        store_state(I.cs1 + (int64_t)jb * I.Cp + t, z);
    }
    if (jb == 0 && t == 0) *I.active = 1;
}

// w = s o r, s = n M^-1 (rounded to float32 once, as the update's s), the
// stored form of the Jacobi iteration's residual.
template <int K>
__device__ inline Vec<K> scaled_residual(const Vec<K>& r, float2 nm) {
    Vec<K> w;
    const float sv = nm.x * nm.y;
#pragma unroll
    for (int k = 0; k < K; ++k) w.v[k] = sv * r.v[k];
    return w;
}

// Per-vertex factors that recover z = w / n and r = w / s (s = n M^-1) from
// the stored residual w; r is 0 on a row with diag(A) = 0 (M^-1 = 0).  n > 0
// on every vertex (bistochastization scales are positive).
struct ResScale {
    float inv_n, inv_s;
};
__device__ inline ResScale res_scale(float2 nm) {
    ResScale o;
    o.inv_n = __builtin_amdgcn_rcpf(nm.x);
    o.inv_s = nm.y > 0.0f ? __builtin_amdgcn_rcpf(nm.x * nm.y) : 0.0f;
    return o;
}

// r = b - A y0, stored as w = n o M^-1 r (as r with the hierarchical
// preconditioner); partials r^T r, b^T b, r^T M^-1 r.
template <int K, bool MULTI, bool PACKED>
__global__ void __launch_bounds__(kRedBlock) pcg_start(PcgArgs a) {
    int jb;
    if (idle_block<MULTI>(a)) return;
    const ImgView I = view_of(block_image<MULTI>(a, jb));
    const int V = I.counts[CNT_V];
    const int Cp = I.Cp, nb = I.nb;
    const Lanes ln(Cp, K);
    const float lam = I.lam;
    double acc[3][K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[0][k] = acc[1][k] = acc[2][k] = 0.0;
    const XcdTiles tl((V + ln.vpb - 1) / ln.vpb, jb, nb);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int v = (int)(tile * ln.vpb) + ln.vl;
        if (!ln.ok || v >= V) continue;
        const uint32_t e = lane_elem(v, Cp, ln.g, K);
        const Vec<K> yv = ldv<K>(I.y, e);
        float ns[K];
#pragma unroll
        for (int k = 0; k < K; ++k) ns[k] = 0.0f;
        int nbv[10];
        load_nbr<PACKED>(nbv, v, I);
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            const int u = nbv[j];
            if (u >= 0) {
                const float nu = elem(I.nfm, (uint32_t)u)->x;
                const Vec<K> yu = ldv<K>(I.y, lane_elem(u, Cp, ln.g, K));
#pragma unroll
                for (int k = 0; k < K; ++k) ns[k] += nu * (yv.v[k] - yu.v[k]);
            }
        }
        const float2 nmv = *elem(I.nfm, (uint32_t)v);
        const float scv = I.sc[v];
        const Vec<K> bv = ldv<K>(I.b, e);
        Vec<K> rv;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const float ay = scv * yv.v[k] + lam * nmv.x * ns[k];
            rv.v[k] = bv.v[k] - ay;
            acc[0][k] += (double)rv.v[k] * (double)rv.v[k];
            acc[1][k] += (double)bv.v[k] * (double)bv.v[k];
            acc[2][k] += (double)rv.v[k] * (double)(nmv.y * rv.v[k]);
        }
        if (I.zmode) stv<K>(I.r, e, rv);
        else stv<K>(I.w, e, scaled_residual<K>(rv, nmv));
    }
    lane_partials<3, K>(acc, ln, Cp, nb, partial_slot(jb, nb), I.part0);
}

// Whether lanes of width K take the steps y += alpha d every other iteration
// (lazy) or every iteration.  With one channel per lane y is 4 of some 60
// bytes a vertex moves per iteration and the deferred step's registers cost
// the exact form a wave per SIMD (depth: 66.0 against 65.0 Mpix/s every
// iteration); with 2 and more channels it saves a y pass every other
// iteration (seg16 45.6 -> 47.5, mixed64 150.3 -> 155.3 Mpix/s).
template <int K>
constexpr bool lazy_y() { return K >= 2; }

// Operands of one lane of pcg_matvec.  Loading them does not depend on the
// iteration's scalars, so the first tile's loads are issued before the
// prologue and overlap its reduction.  The exact form gathers the
// neighbours' w, old d and {n, M^-1}; the recurrence form their w alone.
// rv is the vertex's own stored residual w (z with the hierarchical
// preconditioner).
template <int K, bool EXACT>
struct MatOps {
    int v;
    uint32_t have;                 // bit j: neighbour j exists
    Vec<K> g[10];                  // w (z with the hierarchical preconditioner)
    Vec<K> d[EXACT ? 10 : 1];
    float2 nm[EXACT ? 10 : 1];
    Vec<K> rv, dv, qv, yv;
    Vec<K> d2;                     // the other d buffer's old value (a deferred step's d)
    bool with_y;                   // yv and d2 loaded
    float2 nmv;
    float scv;
};

// The gathers and per-vertex operands of vertex v (phase 2).
template <int K, bool EXACT>
__device__ inline void load_ops(MatOps<K, EXACT>& o, int v, const int (&nb)[10], const Lanes& ln,
                                const ImgView& I, gp<const float> din, gp<const float> dold,
                                bool with_y) {
    o.v = v;
    o.have = 0;
    const int Cp = I.Cp;
    // Missing neighbours (about half of the slots) load nothing: the lanes
    // are masked off, which halves the bytes the texture path delivers.
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        const int u = nb[j];
        if (u >= 0) {
            o.have |= 1u << j;
            const uint32_t eu = lane_elem(u, Cp, ln.g, K);
            o.g[j] = ldv<K>(I.w, eu);
            if constexpr (EXACT) {
                o.d[j] = ldv<K>(din, eu);
                o.nm[j] = *elem(I.nfm, (uint32_t)u);
            }
        }
    }
    const uint32_t e = lane_elem(v, Cp, ln.g, K);
    o.rv = ldv<K>(I.w, e);
    o.dv = ldv<K>(din, e);
    // (lane widths that take every step load y unconditionally: a branch
    // here would make the compiler wait for the loads in flight)
    o.with_y = lazy_y<K>() ? with_y : true;
    if (o.with_y) {
        o.yv = ldv<K>(I.y, e);
        if constexpr (lazy_y<K>()) o.d2 = ldv<K>(dold, e);
    }
    o.nmv = *elem(I.nfm, (uint32_t)v);
    if constexpr (EXACT) o.scv = I.sc[v];
    else o.qv = ldv<K>(I.q, e);
}

// load_ops from the packed words of load_nbr_words.
template <int K, bool EXACT>
__device__ inline void load_ops_late(MatOps<K, EXACT>& o, int v, const int (&raw)[10],
                                     const Lanes& ln, const ImgView& I, gp<const float> din,
                                     gp<const float> dold, bool with_y) {
    if constexpr (EXACT) {
        int nb[10];
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            const uint32_t wd = (uint32_t)raw[j >> 1];
            nb[j] = unpack_offset(v, (j & 1) ? wd >> 16 : wd & 0xffffu);
        }
        load_ops<K, true>(o, v, nb, ln, I, din, dold, with_y);
        return;
    } else {
    o.v = v;
    o.have = 0;
    const int Cp = I.Cp;
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        const uint32_t wd = (uint32_t)raw[j >> 1];
        const int u = unpack_offset(v, (j & 1) ? wd >> 16 : wd & 0xffffu);
        if (u >= 0) {
            o.have |= 1u << j;
            o.g[j] = ldv<K>(I.w, lane_elem(u, Cp, ln.g, K));
        }
    }
    const uint32_t e = lane_elem(v, Cp, ln.g, K);
    o.rv = ldv<K>(I.w, e);
    o.dv = ldv<K>(din, e);
    o.with_y = lazy_y<K>() ? with_y : true;
    if (o.with_y) {
        o.yv = ldv<K>(I.y, e);
        if constexpr (lazy_y<K>()) o.d2 = ldv<K>(dold, e);
    }
    o.nmv = *elem(I.nfm, (uint32_t)v);
    o.qv = ldv<K>(I.q, e);
    }
}

// New search direction of one element: z + beta d_old.
__device__ inline float pcg_dir(float z, float d_old, float beta, bool first) {
    return first ? z : fmaf(beta, d_old, z);
}

// Prologue: finish the previous step (stopping rule, beta) from the slot-0
// partials.  Then the pending steps y += alpha d: the previous update's step
// on d_old (read here anyway) is taken on even iterations (`defer` 0) and on
// odd ones deferred to the next matvec, which then also takes it on the
// direction still in the other d buffer (read before d_new overwrites it), so
// y is read and written every other iteration; a channel that stops takes
// its steps at once, and pcg_flush takes the last ones.  With
// z = M^-1 r = w / n, d = z + beta d and partials of d^T q, where q = A d is
// either
//   EXACT false:  A z + beta q, its recurrence.  diag(A) z = r, so
//                   (A z)_v = r_v - lam n_v sum_u w_u,  r_v = w_v / s_v,
//                 and only the stored residual w is gathered from the
//                 neighbours.  A row with diag(A) = 0 is zero: (A z)_v = 0.
//   EXACT true:   A d itself, in Laplacian form, with the neighbours' new d
//                 recomputed from their gathered w, n and old d.  It resets
//                 the rounding that the recurrence accumulates.
// Both read d_old from d[src] and write d_new to d[src ^ 1] (the recurrence
// form of lane widths without deferred steps updates d[src] in place).
// On a channel's first iteration d = z and q = A z.
template <int K, bool MULTI, bool EXACT, bool PACKED, bool ZMODE = false>
__global__ void __launch_bounds__(kRedBlock) pcg_matvec(PcgArgs a, int src, int defer) {
    static_assert(!ZMODE || (EXACT && !MULTI), "z is stored for single-image exact matvecs");
    __shared__ ChanState S[BS_MAX_CHANNELS];
    __shared__ double fin[3 * BS_MAX_CHANNELS];
    __shared__ float pend[BS_MAX_CHANNELS], pend2[BS_MAX_CHANNELS];
    __shared__ int n_active, n_pend;
    int jb;
    if (idle_block<MULTI>(a)) return;
    const ImgView I = view_of(block_image<MULTI>(a, jb));
    if constexpr (MULTI) {
        if (*I.active == 0) return;   // stopped image (its last steps applied)
    }
    // the new d goes to the other buffer, except in the recurrence form of
    // lane widths that take every step at once, which updates d in place
    gp<const float> din = src ? I.d1 : I.d0;
    const int dst = (EXACT || lazy_y<K>()) ? (src ^ 1) : src;
    gp<float> dout = dst ? I.d1 : I.d0;
    const int t = threadIdx.x;
    const int V = I.counts[CNT_V];
    const int Cp = I.Cp, nb = I.nb;
    const Lanes ln(Cp, K);
    const XcdTiles tl((V + ln.vpb - 1) / ln.vpb, jb, nb);
    // Loads complete in issue order: partials and state first, then the first
    // tile's operands, which stay in flight during the reduction.
    PartialSums ps;
    ps.load(I.part0, 3 * Cp, nb, I.sums0);
    // every lane loads a record (lanes >= Cp a duplicate): a conditional load
    // merged with a default would be waited for before the operand loads
    ChanState st0 = load_state(I.cs0 + (int64_t)jb * Cp + min(t, Cp - 1));
    MatOps<K, EXACT> o;
    int nbn[10];
    int v = (int)(tl.first * ln.vpb) + ln.vl;
    bool have = ln.ok && tl.first < tl.end && v < V;
    constexpr bool kLate = late_decode<K, EXACT, PACKED, MULTI>();
    // y and the other buffer's d are read on the iterations that take steps
    // (the host passes defer = 0 to lane widths that take them every time)
    const bool y_guess = defer == 0;
    if (have) {
        if constexpr (kLate) {
            load_nbr_words(nbn, v, I);
            load_ops_late<K, EXACT>(o, v, nbn, ln, I, din, dout, y_guess);
        } else {
            load_nbr<PACKED>(nbn, v, I);
            load_ops<K, EXACT>(o, v, nbn, ln, I, din, dout, y_guess);
        }
    }
    ps.sum(I.part0, fin);
    if (t == 0) n_active = n_pend = 0;
    __syncthreads();
    if (t < Cp) {
        // a channel the update left active has its step alpha d_old pending;
        // a step deferred by the previous matvec waits on the other buffer
        const bool p = st0.phase != 0 && st0.active;
        float cur = p ? (float)st0.alpha : 0.0f;
        float prev = 0.0f;
        st0 = advance_state(st0, fin[t], fin[Cp + t], fin[2 * Cp + t], a.max_iters, a.tol);
        if constexpr (lazy_y<K>()) {
            prev = (float)st0.alpha_prev;
            if (defer && st0.active) {
                st0.alpha_prev = cur;   // taken by the next matvec
                cur = 0.0f;
            } else {
                st0.alpha_prev = 0.0;
            }
            pend2[t] = prev;
        }
        pend[t] = cur;
        if (cur != 0.0f || prev != 0.0f) atomicAdd(&n_pend, 1);
        store_state(S[t], st0);
        if (st0.active) atomicAdd(&n_active, 1);
        store_state(I.cs1 + (int64_t)jb * Cp + t, st0);
    }
    __syncthreads();
    // Blocks of this launch that start later read the count and return at
    // once when it is 0; with steps still pending it reads -1 instead (the
    // next update stores the true count).
    if (jb == 0 && t == 0) *I.active = n_active > 0 ? n_active : (n_pend > 0 ? -1 : 0);
    if (n_active == 0 && n_pend == 0) return;
    float beta[K], alpha[K], alpha2[K];
    bool first[K], act[K];
    bool any = false, lane_y = false;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int c = ln.ok ? ln.g * K + k : 0;
        const ChanState& s = S[c];
        act[k] = ln.ok && s.active;
        alpha[k] = ln.ok ? pend[c] : 0.0f;
        alpha2[k] = (lazy_y<K>() && ln.ok) ? pend2[c] : 0.0f;
        lane_y = lane_y || alpha[k] != 0.0f || alpha2[k] != 0.0f;
        beta[k] = (float)s.beta;
        // stopped channels restart their (unused) recurrences, which keeps
        // them bounded while the other channels iterate
        first[k] = s.iters == 0 || !act[k];
        any = any || act[k];
    }
    any = any || lane_y;
    const bool need_y = n_pend > 0;
    const float lam = I.lam;
    double acc[1][K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[0][k] = 0.0;
    // Software pipeline over the block's tiles: the next tile's neighbour
    // indices are loaded before this tile's arithmetic waits for its gathers,
    // and its gathers are issued as soon as this tile is stored.
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int64_t nt = tile + tl.step;
        const int vn = (int)(nt * ln.vpb) + ln.vl;
        const bool hn = any && ln.ok && nt < tl.end && vn < V;
        if (hn) {
            if constexpr (kLate) load_nbr_words(nbn, vn, I);
            else load_nbr<PACKED>(nbn, vn, I);
        }
        if (any && have) {
            float zv[K], ns[K];
            Vec<K> dv, qv;
            // z = M^-1 r: the stored residual over n, or as stored (ZMODE)
            constexpr bool zm = ZMODE;
            const ResScale rs = res_scale(o.nmv);
#pragma unroll
            for (int k = 0; k < K; ++k) {
                zv[k] = zm ? o.rv.v[k] : o.rv.v[k] * rs.inv_n;
                dv.v[k] = pcg_dir(zv[k], o.dv.v[k], beta[k], first[k]);
                ns[k] = 0.0f;
            }
            if constexpr (EXACT) {
#pragma unroll
                for (int j = 0; j < 10; ++j) {
                    if (o.have & (1u << j)) {
                        const float inu = zm ? 1.0f : __builtin_amdgcn_rcpf(o.nm[j].x);
#pragma unroll
                        for (int k = 0; k < K; ++k)
                            ns[k] += o.nm[j].x *
                                     (dv.v[k] - pcg_dir(o.g[j].v[k] * inu, o.d[j].v[k], beta[k],
                                                        first[k]));
                    }
                }
#pragma unroll
                for (int k = 0; k < K; ++k) qv.v[k] = o.scv * dv.v[k] + lam * o.nmv.x * ns[k];
            } else {
#pragma unroll
                for (int j = 0; j < 10; ++j) {
                    if (o.have & (1u << j)) {
#pragma unroll
                        for (int k = 0; k < K; ++k) ns[k] += o.g[j].v[k];
                    }
                }
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const float az = o.rv.v[k] * rs.inv_s - lam * o.nmv.x * ns[k];
                    qv.v[k] = first[k] ? az : fmaf(beta[k], o.qv.v[k], az);
                }
            }
            const uint32_t e = lane_elem(o.v, Cp, ln.g, K);
            if (!lazy_y<K>() || lane_y) {
                if (!o.with_y) {   // a channel stops on an iteration that defers
                    o.yv = ldv<K>(I.y, e);
                    if constexpr (lazy_y<K>()) o.d2 = ldv<K>((gp<const float>)dout, e);
                }
                Vec<K> yv;
                // (a buffer without a step may hold anything, even non-finite
                // values: only the steps taken read it)
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    float yk = o.yv.v[k];
                    if constexpr (lazy_y<K>())
                        if (alpha2[k] != 0.0f) yk = fmaf(alpha2[k], o.d2.v[k], yk);
                    if (alpha[k] != 0.0f) yk = fmaf(alpha[k], o.dv.v[k], yk);
                    yv.v[k] = yk;
                }
                stv<K>(I.y, e, yv);
            }
            stv<K>(dout, e, dv);
            stv<K>(I.q, e, qv);
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (act[k]) acc[0][k] += (double)dv.v[k] * (double)qv.v[k];
        }
        if (hn) {
            if constexpr (kLate) load_ops_late<K, EXACT>(o, vn, nbn, ln, I, din, dout, need_y);
            else load_ops<K, EXACT>(o, vn, nbn, ln, I, din, dout, need_y);
        }
        have = hn;
    }
    lane_partials<1, K>(acc, ln, Cp, nb, partial_slot(jb, nb), I.part1);
}

// Prologue: alpha = r^T M^-1 r / d^T q from the slot-1 partials (a channel
// with d^T q <= 0 stops).  Then r -= alpha q, on the stored residual
// w = s o r as w -= (alpha s) q, and partials of r^T r and r^T M^-1 r from
// r = w / s and z = w / n (with the hierarchical preconditioner r itself is
// stored and updated).  The step y += alpha d is left to the next matvec (or
// pcg_flush).  Stopped channels keep their values.
template <int K, bool MULTI, bool ZMODE = false>
__global__ void __launch_bounds__(kRedBlock) pcg_update(PcgArgs a) {
    __shared__ ChanState S[BS_MAX_CHANNELS];
    __shared__ double fin[BS_MAX_CHANNELS];
    __shared__ int n_active, n_defer;
    int jb;
    if (idle_block<MULTI>(a)) return;
    const ImgView I = view_of(block_image<MULTI>(a, jb));
    if constexpr (MULTI) {
        if (*I.active == 0) return;
    }
    const int t = threadIdx.x;
    const int V = I.counts[CNT_V];
    const int Cp = I.Cp, nb = I.nb;
    const Lanes ln(Cp, K);
    const XcdTiles tl((V + ln.vpb - 1) / ln.vpb, jb, nb);
    PartialSums ps;
    ps.load(I.part1, Cp, nb, I.sums1);
    ChanState st0 = load_state(I.cs1 + (int64_t)jb * Cp + min(t, Cp - 1));
    // the stored residual: w = s o r (Jacobi), or r itself (ZMODE)
    gp<float> res = ZMODE ? I.r : I.w;
    // first tile's operands in flight during the reduction
    int v = (int)(tl.first * ln.vpb) + ln.vl;
    bool have = ln.ok && tl.first < tl.end && v < V;
    Vec<K> rv, qv;
    float2 nmv = make_float2(0.0f, 0.0f);
    if (have) {
        const uint32_t e = lane_elem(v, Cp, ln.g, K);
        rv = ldv<K>(res, e);
        qv = ldv<K>(I.q, e);
        nmv = *elem(I.nfm, (uint32_t)v);
    }
    ps.sum(I.part1, fin);
    if (t == 0) n_active = n_defer = 0;
    __syncthreads();
    if (t < Cp) {
        if (st0.active) {
            const double dq = fin[t];
            if (!(dq > 0.0)) {
                st0.active = 0;
                st0.reason = 4;
            } else {
                st0.alpha = st0.rho / dq;
            }
        }
        store_state(S[t], st0);
        if (st0.active) atomicAdd(&n_active, 1);
        else if (st0.alpha_prev != 0.0) atomicAdd(&n_defer, 1);
        store_state(I.cs0 + (int64_t)jb * Cp + t, st0);
    }
    __syncthreads();
    // a channel stopped here with a deferred step keeps the image running
    // (-1) until the next matvec (or pcg_flush) takes the step
    if (jb == 0 && t == 0) *I.active = n_active > 0 ? n_active : (n_defer > 0 ? -1 : 0);
    if (n_active == 0) return;
    float alpha[K];
    bool act[K];
    bool any = false;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const ChanState& s = S[ln.ok ? ln.g * K + k : 0];
        alpha[k] = (float)s.alpha;
        act[k] = ln.ok && s.active;
        any = any || act[k];
    }
    double acc[3][K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[0][k] = acc[1][k] = acc[2][k] = 0.0;
    // Software pipeline: the next tile's operands are loaded before this
    // tile's arithmetic waits for its own.
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int64_t nt = tile + tl.step;
        const int vn = (int)(nt * ln.vpb) + ln.vl;
        const bool hn = any && ln.ok && nt < tl.end && vn < V;
        Vec<K> rn, qn;
        float2 nmn = make_float2(0.0f, 0.0f);
        if (hn) {
            const uint32_t e = lane_elem(vn, Cp, ln.g, K);
            rn = ldv<K>(res, e);
            qn = ldv<K>(I.q, e);
            nmn = *elem(I.nfm, (uint32_t)vn);
        }
        if (any && have) {
            Vec<K> w1;
            if constexpr (ZMODE) {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    if (act[k]) {
                        w1.v[k] = fmaf(-alpha[k], qv.v[k], rv.v[k]);
                        acc[0][k] += (double)w1.v[k] * (double)w1.v[k];
                    } else {
                        w1.v[k] = rv.v[k];
                    }
                }
            } else {
                const ResScale rs = res_scale(nmv);
                const double sv = (double)(nmv.x * nmv.y);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    if (act[k]) {
                        // w - alpha s q rounded once, as r - alpha q would be:
                        // the implied r = w / s keeps one rounding per step
                        w1.v[k] = (float)fma(-(double)alpha[k] * sv, (double)qv.v[k],
                                             (double)rv.v[k]);
                        const float r1 = w1.v[k] * rs.inv_s;
                        acc[0][k] += (double)r1 * (double)r1;
                        acc[2][k] += (double)r1 * (double)(w1.v[k] * rs.inv_n);
                    } else {
                        w1.v[k] = rv.v[k];
                    }
                }
            }
            stv<K>(res, lane_elem(v, Cp, ln.g, K), w1);
        }
        v = vn;
        have = hn;
        rv = rn;
        qv = qn;
        nmv = nmn;
    }
    lane_partials<3, K>(acc, ln, Cp, nb, partial_slot(jb, nb), I.part0);
}

// Level 0 of the hierarchical preconditioner's collapse (one image):
// z = M^-1_jacobi r + up1[parent0] (the coarser levels' share), stored in w,
// and the partials of r^T z into the third slot-0 partial (the residual
// update or pcg_start wrote the first two).
template <int K>
__global__ void __launch_bounds__(kRedBlock) pcg_prec_final(PcgArgs a, const float* up1,
                                                             const int32_t* parent0) {
    const ImgView I = view_of(a.one);
    const int jb = (int)blockIdx.x;
    const int V = I.counts[CNT_V];
    const int Ktop = I.counts[CNT_K];
    const int Cp = I.Cp, nb = I.nb, C1 = Cp + 1;
    const Lanes ln(Cp, K);
    double acc[1][K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[0][k] = 0.0;
    const XcdTiles tl((V + ln.vpb - 1) / ln.vpb, jb, nb);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int v = (int)(tile * ln.vpb) + ln.vl;
        if (!ln.ok || v >= V) continue;
        const uint32_t e = lane_elem(v, Cp, ln.g, K);
        const Vec<K> rv = ldv<K>(I.r, e);
        const float mi = elem(I.nfm, (uint32_t)v)->y;
        Vec<K> zv;
#pragma unroll
        for (int k = 0; k < K; ++k) zv.v[k] = mi * rv.v[k];
        if (Ktop >= 1) {
            const int64_t pu = (int64_t)parent0[v] * C1 + ln.g * K;
#pragma unroll
            for (int k = 0; k < K; ++k) zv.v[k] += up1[pu + k];
        }
        stv<K>(I.w, e, zv);
#pragma unroll
        for (int k = 0; k < K; ++k) acc[0][k] += (double)rv.v[k] * (double)zv.v[k];
    }
    lane_partials<1, K>(acc, ln, Cp, nb, partial_slot(jb, nb), I.part0 + (int64_t)2 * Cp * nb);
}

// After the last enqueued iteration: applies the step y += alpha d that the
// last update left pending (d = d[src]) for the channels it left active, and
// a step the last matvec deferred (on the other buffer).  An image whose
// active count is 0 has none pending: its channels stopped in an update with
// no deferred step, or in a matvec, which applied their steps.
template <int K, bool MULTI>
__global__ void __launch_bounds__(kRedBlock) pcg_flush(PcgArgs a, int src) {
    __shared__ float pend[BS_MAX_CHANNELS], pend2[BS_MAX_CHANNELS];
    __shared__ int n_pend;
    int jb;
    if (idle_block<MULTI>(a)) return;
    const ImgView I = view_of(block_image<MULTI>(a, jb));
    if (*I.active == 0) return;
    const int t = threadIdx.x;
    const int V = I.counts[CNT_V];
    const int Cp = I.Cp, nb = I.nb;
    const Lanes ln(Cp, K);
    gp<const float> d = src ? I.d1 : I.d0;
    gp<const float> d_other = src ? I.d0 : I.d1;
    if (t == 0) n_pend = 0;
    __syncthreads();
    if (t < Cp) {
        const ChanState st = load_state(I.cs0 + (int64_t)jb * Cp + t);
        const bool p = st.phase != 0 && st.active;
        pend[t] = p ? (float)st.alpha : 0.0f;
        pend2[t] = (float)st.alpha_prev;
        if (p || st.alpha_prev != 0.0) atomicAdd(&n_pend, 1);
    }
    __syncthreads();
    if (n_pend == 0 || !ln.ok) return;
    float alpha[K], alpha2[K];
    bool any = false, any2 = false;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        alpha[k] = pend[ln.g * K + k];
        alpha2[k] = pend2[ln.g * K + k];
        any = any || alpha[k] != 0.0f;
        any2 = any2 || alpha2[k] != 0.0f;
    }
    if (!any && !any2) return;
    const XcdTiles tl((V + ln.vpb - 1) / ln.vpb, jb, nb);
    for (int64_t tile = tl.first; tile < tl.end; tile += tl.step) {
        const int v = (int)(tile * ln.vpb) + ln.vl;
        if (v >= V) continue;
        const uint32_t e = lane_elem(v, Cp, ln.g, K);
        Vec<K> yv = ldv<K>(I.y, e);
        if (any2) {   // the deferred step, on the older direction
            const Vec<K> dv2 = ldv<K>(d_other, e);
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (alpha2[k] != 0.0f) yv.v[k] = fmaf(alpha2[k], dv2.v[k], yv.v[k]);
        }
        if (any) {
            const Vec<K> dv = ldv<K>(d, e);
#pragma unroll
            for (int k = 0; k < K; ++k)
                if (alpha[k] != 0.0f) yv.v[k] = fmaf(alpha[k], dv.v[k], yv.v[k]);
        }
        stv<K>(I.y, e, yv);
    }
}

// With many channels the per-block partials are reduced once, by one block
// per (value, channel) pair, rather than redundantly in every consumer block.
// Block (pair, image); `mult` values per channel in slot `which`.
template <bool MULTI>
__global__ void __launch_bounds__(kRedBlock) pcg_reduce(PcgArgs a, int which, int mult) {
    const ImgView I = view_of(MULTI ? a.imgs[blockIdx.y] : a.one);
    gp<double> sums = which ? I.wsums1 : I.wsums0;
    if (!sums || (int)blockIdx.x >= mult * I.Cp) return;
    if constexpr (MULTI) {
        if (*I.active == 0) return;
    }
    gp<const double> part = which ? I.part1 : I.part0;
    const int G = I.nb;
    double v = 0.0;
    for (int i = threadIdx.x; i < G; i += kRedBlock) v += part[(int64_t)blockIdx.x * G + i];
    const double s = block_sum<kRedBlock>(v);
    if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

// After the last enqueued iteration (one block per image): completes the
// pending step and writes the per-channel stats.
template <bool MULTI>
__global__ void __launch_bounds__(kRedBlock) pcg_finish(PcgArgs a) {
    __shared__ double fin[3 * BS_MAX_CHANNELS];
    const ImgView I = view_of(MULTI ? a.imgs[blockIdx.x] : a.one);
    const int t = threadIdx.x;
    reduce_partials<3>(I.part0, I.Cp, I.nb, fin, I.sums0);
    if (t < I.C && I.stats) {
        ChanState st = load_state(I.cs0 + t);
        st = advance_state(st, fin[t], fin[I.Cp + t], fin[2 * I.Cp + t], a.max_iters, a.tol);
        bs_chan_stats o;
        o.iters = st.iters;
        o.reason = st.reason;
        o.rel_residual = st.res;
        o.bnorm = st.bnorm;
        I.stats[t] = o;
    }
}

// ---------------------------------------------------------------------------
// Host sequencing.
// ---------------------------------------------------------------------------
bs_status validate_solve(const bs_grid* grid, int C, const bs_solve_params* p) {
    if (!grid || impl(grid)->magic != kGridMagic) return fail(BS_EINVAL, "grid was not built");
    if (!impl(grid)->bistochastized) return fail(BS_EINVAL, "grid was not bistochastized");
    if (C < 1 || C > BS_MAX_CHANNELS) return fail(BS_EINVAL, "channel count must be in 1..64");
    if (!solve_fits(impl(grid)->vcap, C))
        return fail(BS_EUNSUPPORTED, "grid too large for 32-bit vector offsets at this channel count");
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
    if (p->precond != BS_PRECOND_JACOBI && p->precond != BS_PRECOND_HIER)
        return fail(BS_EINVAL, "unknown preconditioner");
    if (p->precond == BS_PRECOND_HIER &&
        !(p->pre_alpha > 0.0f && std::isfinite(p->pre_alpha) && std::isfinite(p->pre_beta)))
        return fail(BS_EINVAL, "pre_alpha must be positive and pre_beta finite");
    return BS_OK;
}

static bool misaligned(const void* p) { return ((uintptr_t)p & 3) != 0; }

// Initial state into `y` (stride Cp) from the right-hand side in w.b.
static bs_status run_init(const GridImpl& g, const SolveWs& w, const bs_solve_params& p,
                          float* y, hipStream_t s) {
    const int C = w.Cp;
    const int blocks = grid_blocks(ceil_div(g.vcap * C, kBlock));
    if (p.init == BS_INIT_FLAT) {
        BS_LAUNCH(s, K_INIT, "flat_init", one_launch<FlatInit>, dim3(blocks), dim3(kBlock), 0, s,
                  flat_init_args(g, w, y), 0);
        return BS_OK;
    }
    // levels k0.. are small enough for one block (capacities decrease with k)
    const int k0 = small_pyr_level(g, C);
    for (int k = 1; k < k0; ++k) {
        const int bk = grid_blocks(ceil_div(g.lv[k].cap * (C + 1), kBlock));
        BS_LAUNCH(s, K_INIT, "pyr_up", one_launch<PyrUp>, dim3(bk), dim3(kBlock), 0, s,
                  pyr_up_args(g, w, k), 0);
    }
    if (k0 < g.levels)
        BS_LAUNCH(s, K_INIT, "pyr_small", one_launch<PyrSmall>, dim3(1), dim3(1024), 0, s,
                  pyr_small_args(g, w, p, k0), 0);
    for (int k = k0 - 1; k >= 1; --k) {
        const int bk = grid_blocks(ceil_div(g.lv[k].cap * (C + 1), kBlock));
        BS_LAUNCH(s, K_INIT, "pyr_down", one_launch<PyrDown>, dim3(bk), dim3(kBlock), 0, s,
                  pyr_down_args(g, w, p, k), 0);
    }
    BS_LAUNCH(s, K_INIT, "hier_final", one_launch<HierFinal>, dim3(blocks), dim3(kBlock), 0, s,
              hier_final_args(g, w, y), 0);
    return BS_OK;
}

bs_status splat_setup(const GridImpl& g, const SolveWs& w, const float* conf, const float* vals,
                      bool weighted, double lambda, hipStream_t s) {
    return weighted ? launch_splat<true>(g, w, conf, vals, lambda, s)
                    : launch_splat<false>(g, w, conf, vals, lambda, s);
}

bs_status init_state(const GridImpl& g, const SolveWs& w, const bs_solve_params& p, float* yw,
                     hipStream_t s) {
    return run_init(g, w, p, yw, s);
}

bs_status solve_setup(const GridImpl& g, const SolveWs& w, const float* conf, const float* vals,
                      bool weighted, const bs_solve_params& p, float* yw, hipStream_t s) {
    const bs_status st = splat_setup(g, w, conf, vals, weighted, (double)p.lambda, s);
    if (st != BS_OK) return st;
    return run_init(g, w, p, yw, s);
}

bool pcg_partials_fit(int Cp, int nb) { return PartialSums::fits(3 * Cp, nb); }

static std::atomic<int> g_lane_override[BS_MAX_CHANNELS + 1];

int lane_width_override(int C) {
    return (C < 1 || C > BS_MAX_CHANNELS) ? 0 : g_lane_override[C].load(std::memory_order_relaxed);
}

PcgImage make_image(const GridImpl& g, const SolveWs& w, float lam, float* yw,
                    bs_chan_stats* stats) {
    PcgImage I;
    std::memset(&I, 0, sizeof(I));
    I.nbr = g.nbr;
    I.nb16 = g.nb_packed ? g.nb16 : nullptr;
    I.nfm = w.nfm;
    I.sc = w.sc;
    I.b = w.b;
    I.y = yw;
    I.r = w.r;
    I.d[0] = w.d[0];
    I.d[1] = w.d[1];
    I.q = w.q;
    I.w = w.w;
    I.counts = g.counts;
    I.cs[0] = w.cs[0];
    I.cs[1] = w.cs[1];
    I.part[0] = w.part[0];
    I.part[1] = w.part[1];
    // Consumers reduce the partials themselves while they fit in registers;
    // beyond that a pcg_reduce launch does it once.
    const bool sep = !PartialSums::fits(3 * w.Cp, w.nb);
    I.sums[0] = sep ? w.sums[0] : nullptr;
    I.sums[1] = sep ? w.sums[1] : nullptr;
    I.active = w.act;
    I.stats = stats;
    I.vcap = g.vcap;
    I.lam = lam;
    I.C = w.C;
    I.Cp = w.Cp;
    I.nb = w.nb;
    I.block0 = 0;
    return I;
}


bs_status prec_setup(const GridImpl& g, const SolveWs& w, float alpha, float beta,
                     HierPrecPlan& hp, hipStream_t s) {
    const int Cp = w.Cp;
    hp.levels = g.levels;
    hp.Cp = Cp;
    hp.counts = g.counts;
    hp.r = w.r;
    hp.up1 = g.levels > 1 ? w.up[1] : nullptr;
    hp.parent0 = g.levels > 1 ? g.lv[1].item_parent : nullptr;
    // levels whose application fits one block run in one launch
    int k0 = 1;
    while (k0 < g.levels && g.lv[k0].cap * (Cp + 1) > kSmallPyrElems) ++k0;
    hp.k0 = k0;
    for (int k = 1; k < g.levels; ++k) {
        HierPrecPlan::Level& L = hp.lv[k];
        L.cptr = g.lv[k].ptr;
        L.clist = g.lv[k].list;
        L.prev = k >= 2 ? w.up[k - 1] : nullptr;
        L.up = w.up[k];
        L.up_parent = (k + 1 < g.levels) ? w.up[k + 1] : nullptr;
        L.parent = (k + 1 < g.levels) ? g.lv[k + 1].item_parent : nullptr;
        L.blocks = grid_blocks(ceil_div(g.lv[k].cap * Cp, kBlock));
    }
    // P(diag A) bottom-up, then the scales
    for (int k = 1; k < g.levels; ++k) {
        const int bk = grid_blocks(ceil_div(g.lv[k].cap, kBlock));
        BS_LAUNCH(s, K_INIT, "prec_lift", one_launch<PrecLift>, dim3(bk), dim3(kBlock), 0, s,
                  (PrecLift::Args{g.lv[k].ptr, g.lv[k].list, w.diag,
                                  k >= 2 ? w.up[k - 1] : nullptr, w.up[k], g.counts, Cp, k}),
                  0);
    }
    for (int k = 1; k < g.levels; ++k) {
        const int bk = grid_blocks(ceil_div(g.lv[k].cap, kBlock));
        const float wk = (float)std::pow((double)alpha, -((double)beta + k));
        BS_LAUNCH(s, K_INIT, "prec_scale", one_launch<PrecScale>, dim3(bk), dim3(kBlock), 0, s,
                  (PrecScale::Args{w.up[k], g.lv[k].ones, g.counts, wk, Cp, k}), 0);
    }
    return BS_OK;
}

// One application z = M_hier^-1 r into w, with the r^T z partials.
template <int K>
static bs_status prec_apply(const PcgArgs& a, const HierPrecPlan& hp, int G, hipStream_t s) {
    for (int k = 1; k < hp.k0; ++k) {
        const HierPrecPlan::Level& L = hp.lv[k];
        BS_LAUNCH(s, K_PCG_UPDATE, "prec_up", one_launch<PrecUp>, dim3(L.blocks), dim3(kBlock), 0,
                  s, (PrecUp::Args{L.cptr, L.clist, hp.r, L.prev, L.up, hp.counts, hp.Cp, k}), 0);
    }
    if (hp.k0 < hp.levels) {
        PrecSmall::Args A;
        std::memset(&A, 0, sizeof(A));
        A.lv.k0 = hp.k0;
        A.lv.levels = hp.levels;
        for (int k = 1; k < hp.levels; ++k) {
            A.lv.cptr[k] = hp.lv[k].cptr;
            A.lv.clist[k] = hp.lv[k].clist;
            A.lv.parent[k] = hp.lv[k].parent;
            A.lv.up[k] = hp.lv[k].up;
        }
        A.r = hp.r;
        A.counts = hp.counts;
        A.Cp = hp.Cp;
        BS_LAUNCH(s, K_PCG_UPDATE, "prec_small", one_launch<PrecSmall>, dim3(1), dim3(1024), 0, s,
                  A, 0);
    }
    for (int k = hp.k0 - 1; k >= 1; --k) {
        const HierPrecPlan::Level& L = hp.lv[k];
        BS_LAUNCH(s, K_PCG_UPDATE, "prec_down", one_launch<PrecDown>, dim3(L.blocks), dim3(kBlock),
                  0, s, (PrecDown::Args{L.up, L.up_parent, L.parent, hp.counts, hp.Cp, k}), 0);
    }
    BS_LAUNCH(s, K_PCG_UPDATE, "pcg_prec_final", pcg_prec_final<K>, dim3(G), dim3(kRedBlock), 0, s,
              a, hp.up1, hp.parent0);
    return BS_OK;
}

template <int K, bool MULTI, bool PACKED>
static bs_status run_pcg_k(const PcgArgs& a, int n, int G, int max_cp, bool sep,
                           const bs_solve_params& p, const int32_t* act, hipStream_t s,
                           const HierPrecPlan* hp) {
    const dim3 grid(G), block(kRedBlock);
    if constexpr (MULTI) {
        if (hp) return fail(BS_EUNSUPPORTED, "hierarchical preconditioner on an image table");
    }
    BS_LAUNCH(s, K_INIT, "pcg_prologue", pcg_prologue<MULTI>, grid, block, 0, s, a);
    BS_LAUNCH(s, K_PCG_START, "pcg_start", (pcg_start<K, MULTI, PACKED>), grid, block, 0, s, a);
    if constexpr (!MULTI) {
        if (hp) {
            const bs_status st = prec_apply<K>(a, *hp, G, s);
            if (st != BS_OK) return st;
        }
    }
    if (sep)
        BS_LAUNCH(s, K_PCG_REDUCE, "pcg_reduce", pcg_reduce<MULTI>, dim3(3 * max_cp, n), block, 0,
                  s, a, 0, 3);
    StopPoller poller(act, n, s);
    int src = 0;   // the buffer holding d
    for (int it = 0; it < p.max_iters; ++it) {
        // with the hierarchical preconditioner every matvec is the exact form
        // (the recurrence needs diag(A) z = r)
        // odd iterations defer their y step to the next matvec
        const int defer = lazy_y<K>() ? (it & 1) : 0;
        if constexpr (!MULTI) {
            if (hp)
                BS_LAUNCH(s, K_PCG_MATVEC, "pcg_matvec", (pcg_matvec<K, false, true, PACKED, true>),
                          grid, block, 0, s, a, src, defer);
        }
        if (hp) {
        } else if (exact_iteration<K>(it)) {
            BS_LAUNCH(s, K_PCG_MATVEC, "pcg_matvec", (pcg_matvec<K, MULTI, true, PACKED>), grid, block, 0,
                      s, a, src, defer);
        } else if constexpr (uses_recurrence<K>()) {
            BS_LAUNCH(s, K_PCG_MATVEC, "pcg_matvec", (pcg_matvec<K, MULTI, false, PACKED>), grid, block, 0,
                      s, a, src, defer);
        }
        // the matvec wrote the new d to the other buffer (in place: the
        // recurrence form of lane widths without deferred steps)
        if (lazy_y<K>() || hp || exact_iteration<K>(it)) src ^= 1;
        if (sep)
            BS_LAUNCH(s, K_PCG_REDUCE, "pcg_reduce", pcg_reduce<MULTI>, dim3(max_cp, n), block, 0,
                      s, a, 1, 1);
        if constexpr (!MULTI) {
            if (hp)
                BS_LAUNCH(s, K_PCG_UPDATE, "pcg_update", (pcg_update<K, false, true>), grid, block, 0,
                          s, a);
        }
        if (!hp)
            BS_LAUNCH(s, K_PCG_UPDATE, "pcg_update", (pcg_update<K, MULTI>), grid, block, 0, s, a);
        if constexpr (!MULTI) {
            if (hp) {
                const bs_status st = prec_apply<K>(a, *hp, G, s);
                if (st != BS_OK) return st;
            }
        }
        if (sep)
            BS_LAUNCH(s, K_PCG_REDUCE, "pcg_reduce", pcg_reduce<MULTI>, dim3(3 * max_cp, n), block,
                      0, s, a, 0, 3);
        if (p.check_every > 0 && (it + 1) % p.check_every == 0 && it + 1 < p.max_iters) {
            bool stop = false;
            const bs_status st = poller.check(stop);
            if (st != BS_OK) return st;
            if (stop) break;
        }
    }
    BS_LAUNCH(s, K_PCG_UPDATE, "pcg_flush", (pcg_flush<K, MULTI>), grid, block, 0, s, a, src);
    BS_LAUNCH(s, K_INIT, "pcg_finish", pcg_finish<MULTI>, dim3(n), block, 0, s, a);
    return BS_OK;
}

bs_status run_pcg(int K, const PcgImage* imgs, int n, const PcgImage* dev_imgs,
                  const int32_t* blk2img, int G, int max_cp, const bs_solve_params& p,
                  const int32_t* act, hipStream_t s, const HierPrecPlan* hp) {
    PcgArgs a;
    std::memset(&a, 0, sizeof(a));
    a.one = imgs[0];
    a.imgs = dev_imgs;
    a.blk2img = blk2img;
    a.max_iters = p.max_iters;
    a.tol = p.rel_tol;
    bool sep = false;
    for (int i = 0; i < n; ++i) sep = sep || imgs[i].sums[0] != nullptr;
    const bool multi = dev_imgs != nullptr;
    if (multi && !blk2img) return fail(BS_EINVAL, "image tables missing");
    // the packed neighbour table when every image has one
    bool packed = true;
    for (int i = 0; i < n; ++i) packed = packed && imgs[i].nb16 != nullptr;
    const int mode = (multi ? 1 : 0) | (packed ? 2 : 0);
    auto go = [&](auto k) -> bs_status {
        constexpr int Kc = decltype(k)::value;
        switch (mode) {
            case 0: return run_pcg_k<Kc, false, false>(a, n, G, max_cp, sep, p, act, s, hp);
            case 1: return run_pcg_k<Kc, true, false>(a, n, G, max_cp, sep, p, act, s, hp);
            case 2: return run_pcg_k<Kc, false, true>(a, n, G, max_cp, sep, p, act, s, hp);
            default: return run_pcg_k<Kc, true, true>(a, n, G, max_cp, sep, p, act, s, hp);
        }
    };
    switch (K) {
        case 1: return go(std::integral_constant<int, 1>{});
        case 2: return go(std::integral_constant<int, 2>{});
        case 3: return go(std::integral_constant<int, 3>{});
        case 4: return go(std::integral_constant<int, 4>{});
        default: return fail(BS_EINVAL, "unsupported lane width");
    }
}

bs_status copy_unpadded(const GridImpl& g, const float* yw, int C, int Cp, float* y,
                        hipStream_t s) {
    const int blocks = grid_blocks(ceil_div(g.vcap * C, kBlock));
    BS_LAUNCH(s, K_INIT, "unpad", one_launch<Unpad>, dim3(blocks), dim3(kBlock), 0, s,
              (Unpad::Args{yw, g.counts, y, Cp, C}), 0);
    return BS_OK;
}

bs_status grad_scatter_launch(const GridImpl& g, const float* gb, int Cp, const float* y_hat,
                              const float* target, const float* conf, int C, float* grad_t,
                              float* grad_c, hipStream_t s) {
    const int pblocks = grid_blocks(ceil_div(g.P, kBlock));
    BS_LAUNCH(s, K_GRAD_SCATTER, "grad_scatter", one_launch<GradScatter>, dim3(pblocks),
              dim3(kBlock), 0, s,
              (GradScatter::Args{g.lv[0].item_parent, gb, y_hat, target, conf, grad_t, grad_c, Cp,
                                 C, g.P}),
              0);
    return BS_OK;
}

}  // namespace bs

using namespace bs;

extern "C" size_t bs_solve_workspace_bytes(const bs_grid* grid, int32_t C) {
    if (!grid || impl(grid)->magic != kGridMagic || C < 1 || C > BS_MAX_CHANNELS) return 0;
    SolveWs w;
    return layout_solve(*impl(grid), C, 0, nullptr, w);
}

extern "C" bs_status bs_solve_ws_view(const bs_grid* grid, int32_t C, void* ws, size_t ws_bytes,
                                      const float** b, const float** sc, const float** diag,
                                      const float** minv) {
    if (!grid || impl(grid)->magic != kGridMagic || C < 1 || C > BS_MAX_CHANNELS)
        return fail(BS_EINVAL, "bad grid or channel count");
    SolveWs w;
    if (ws_bytes < layout_solve(*impl(grid), C, 0, nullptr, w))
        return fail(BS_EWORKSPACE, "workspace too small");
    layout_solve(*impl(grid), C, 0, ws, w);
    if (b) *b = w.b;
    if (sc) *sc = w.sc;
    if (diag) *diag = w.diag;
    if (minv) *minv = w.minv;
    return BS_OK;
}

extern "C" bs_status bs_set_lane_width(int32_t C, int32_t K) {
    if (C < 1 || C > BS_MAX_CHANNELS) return fail(BS_EINVAL, "channel count must be in 1..64");
    if (K < 0 || K > 4) return fail(BS_EINVAL, "lane width must be in 0..4");
    g_lane_override[C].store(K, std::memory_order_relaxed);
    return BS_OK;
}

extern "C" int32_t bs_solve_channel_stride(int32_t C) {
    return (C < 1 || C > BS_MAX_CHANNELS) ? 0 : padded_channels(C);
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
    const size_t need = layout_solve(g, C, 0, nullptr, w);
    if (ws_bytes < need)
        return fail(BS_EWORKSPACE, "solve workspace needs " + std::to_string(need) + " bytes");
    layout_solve(g, C, 0, ws, w);
    hipStream_t s = (hipStream_t)stream;
    const bs_solve_params& p = *params;
    // y is used in place unless the channel stride is padded
    float* yw = (w.Cp == C && ((uintptr_t)y & 15) == 0) ? y : w.yi;
    st = solve_setup(g, w, conf, target, true, p, yw, s);
    if (st != BS_OK) return st;
    PcgImage I = make_image(g, w, p.lambda, yw, stats);
    HierPrecPlan hp;
    if (p.precond == BS_PRECOND_HIER) {
        st = prec_setup(g, w, p.pre_alpha, p.pre_beta, hp, s);
        if (st != BS_OK) return st;
        I.zmode = 1;
    }
    st = run_pcg(w.K, &I, 1, nullptr, nullptr, w.nb, w.Cp, p, w.act, s,
                 p.precond == BS_PRECOND_HIER ? &hp : nullptr);
    if (st != BS_OK) return st;
    if (yw != y) return copy_unpadded(g, yw, C, w.Cp, y, s);
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
    BS_LAUNCH(s, K_SLICE, "slice", one_launch<Slice>, dim3(blocks), dim3(kBlock), 0, s,
              (Slice::Args{g.lv[0].item_parent, y, x, C, g.P}), 0);
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
    const size_t need = layout_solve(g, C, 0, nullptr, w);
    if (ws_bytes < need)
        return fail(BS_EWORKSPACE, "solve workspace needs " + std::to_string(need) + " bytes");
    layout_solve(g, C, 0, ws, w);
    hipStream_t s = (hipStream_t)stream;
    const bs_solve_params& p = *params;
    // the adjoint solution goes to g_out in place unless the stride is padded
    float* gb = (g_out && w.Cp == C && ((uintptr_t)g_out & 15) == 0) ? g_out : w.yi;
    st = solve_setup(g, w, conf, grad_x, false, p, gb, s);
    if (st != BS_OK) return st;
    PcgImage I = make_image(g, w, p.lambda, gb, stats);
    HierPrecPlan hp;
    if (p.precond == BS_PRECOND_HIER) {
        st = prec_setup(g, w, p.pre_alpha, p.pre_beta, hp, s);
        if (st != BS_OK) return st;
        I.zmode = 1;
    }
    st = run_pcg(w.K, &I, 1, nullptr, nullptr, w.nb, w.Cp, p, w.act, s,
                 p.precond == BS_PRECOND_HIER ? &hp : nullptr);
    if (st != BS_OK) return st;
    st = grad_scatter_launch(g, gb, w.Cp, y_hat, target, conf, C, grad_t, grad_c, s);
    if (st != BS_OK) return st;
    if (g_out && gb != g_out) return copy_unpadded(g, gb, C, w.Cp, g_out, s);
    return BS_OK;
}
