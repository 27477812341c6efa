// Internal interface of the solve: workspace layout, the per-image PCG
// descriptor and the host sequencing shared by the single-image entry points
// and the batch engine.
#pragma once

#include "bs_internal.h"

namespace bs {

// PCG state of one channel.
struct ChanState {
    double rho, alpha, beta, bnorm, res;
    double alpha_prev;   // a deferred step alpha d on the direction in the other d buffer
    int32_t active, iters, reason, phase;   // phase 0: initial residual not yet reduced
};

// One record per 128-byte cache line: each block reads back its own record,
// written by the block of the same index (same die) in the previous launch.
// With 48- or 64-byte records a line held records of blocks on two dies and
// that read cost ~12 us per launch on MI355X.  Only the payload is copied.
struct alignas(128) ChanRec {
    ChanState s;
};
static_assert(sizeof(ChanRec) == 128, "one record per cache line");

// Channels per lane of the vertex kernels (1, 2, 3 or 4: one float, float2,
// 3-float or float4 access) and the channel stride of the bilateral-space
// vectors, C rounded up to a multiple of the lane width (C = 21 = 7 x 3
// needs no padding).  The default rule takes the widest access that needs
// little padding; bs_set_lane_width replaces it for a channel count (read
// when a workspace is laid out).
inline int default_lane_width(int C) {
    if (C <= 2) return C;
    if (C % 4 == 0) return 4;
    if (C % 3 == 0) return 3;
    return 4;
}
int lane_width_override(int C);   // 0: none
inline int lane_width(int C) {
    const int k = lane_width_override(C);
    return k > 0 ? k : default_lane_width(C);
}
inline int padded_channels(int C) {
    const int K = lane_width(C);
    return (C + K - 1) / K * K;
}

// The PCG kernels address a vector element by a 32-bit byte offset from the
// vector's base: every [Vcap][Cp] float vector, and the packed neighbour
// table [5][Vcap], must stay below 2^30 elements (4 GiB).
inline bool solve_fits(int64_t vcap, int C) {
    return vcap * padded_channels(C) < ((int64_t)1 << 30) && 5 * vcap < ((int64_t)1 << 30);
}

// One image of a PCG launch.  In a launch over several images, blocks
// [block0, block0 + nb) work on this image; block0 and nb are multiples of 8,
// so the image's local block j runs on die j % 8.  Vectors are [V][Cp].
struct PcgImage {
    const int32_t* nbr;      // [10][vcap] neighbour table
    const uint32_t* nb16;    // [5][vcap] the table as packed 16-bit offsets (read unless
                             // counts[CNT_NB_WIDE])
    const float2* nfm;       // [V] {n, 1 / diag(A)}
    const float* sc;         // [V] S c
    const float* b;          // right-hand side
    float* y;                // solution (initial state on entry)
    float* r;
    float* d[2];             // search direction (two buffers for the exact matvec)
    float* q;
    float* w;                // n o M^-1 r, gathered by the recurrence matvec
    const int32_t* counts;   // V = counts[CNT_V]
    ChanRec* cs[2];          // [nb][Cp] per-block channel state, ping-pong
    double* part[2];         // [3][Cp][nb] per-block partials: 0 start/update, 1 matvec
    double* sums[2];         // [3][Cp] partials reduced by pcg_reduce, or nullptr
    int32_t* active;         // channels still iterating (written by local block 0)
    bs_chan_stats* stats;    // [C] or nullptr
    int64_t vcap;
    float lam;
    int32_t C, Cp, nb, block0;
    int32_t zmode;           // 1: the preconditioned residual z is stored in w (hierarchical
                             // preconditioner) and the matvec reads it; 0: z = M^-1 r, Jacobi
};

// Kernel argument of the PCG kernels: one image by value, or a table of
// images and the image of every block.
struct PcgArgs {
    PcgImage one;
    const PcgImage* imgs;
    const int32_t* blk2img;
    int32_t max_iters;
    double tol;
};

struct SolveWs {
    int C, Cp, K, nb;
    float* sc;
    float* diag;
    float* minv;
    float2* nfm;
    float* b;
    float* r;
    float* d[2];
    float* q;
    float* w;
    float* yi;               // [V][Cp] solution when the caller's buffer is not used in place
    float* up[BS_MAX_LEVELS];
    ChanRec* cs[2];
    double* part[2];
    double* sums[2];
    int32_t* act;
    size_t bytes;
};

// Lays out (base != nullptr) or sizes a solve workspace for C channels with
// nb reducing blocks (0: the single-image default).
size_t layout_solve(const GridImpl& g, int C, int nb, void* base, SolveWs& w);

// Reducing blocks of a single-image solve.
int solve_blocks(const GridImpl& g, int C);

// Argument checks shared by the solve entry points (grid built and
// bistochastized, channel count, parameters).
bs_status validate_solve(const bs_grid* grid, int C, const bs_solve_params* p);

// Splat alone: S c, diag(A), its Jacobi inverse, {n, M^-1} and b (weighted:
// b = S(c o t), else b = S t).
bs_status splat_setup(const GridImpl& g, const SolveWs& w, const float* conf, const float* vals,
                      bool weighted, double lambda, hipStream_t s);

// Initial state of w's right-hand side w.b into yw (flat or hierarchical).
bs_status init_state(const GridImpl& g, const SolveWs& w, const bs_solve_params& p, float* yw,
                     hipStream_t s);

// Splat (weighted: b = S(c o t), else b = S t) and initial state into yw.
bs_status solve_setup(const GridImpl& g, const SolveWs& w, const float* conf, const float* vals,
                      bool weighted, const bs_solve_params& p, float* yw, hipStream_t s);

// Whether the consumers of a Cp-channel image's per-block partials over nb
// blocks sum them in registers (else make_image points the image at sums
// that a pcg_reduce launch computes once).
bool pcg_partials_fit(int Cp, int nb);

// The descriptor of one image's PCG (block0 = 0).
PcgImage make_image(const GridImpl& g, const SolveWs& w, float lam, float* yw,
                    bs_chan_stats* stats);

// Launches of the hierarchical preconditioner z = M_hier^-1 r of one image
// (set up by prec_setup, applied after every residual update).
struct HierPrecPlan {
    int levels = 0, k0 = 1;              // levels k0.. run in one block
    struct Level {
        const int32_t* cptr;
        const int32_t* clist;
        const float* prev;               // level k-1's buffer (k >= 2)
        float* up;
        const float* up_parent;          // level k+1's buffer
        const int32_t* parent;           // level k vertex -> level k+1 vertex
        int blocks;
    };
    Level lv[BS_MAX_LEVELS];
    const float* up1 = nullptr;          // level 1's collapse, read by the final kernel
    const int32_t* parent0 = nullptr;    // level-0 vertex -> level-1 vertex
    const int32_t* counts = nullptr;
    const float* r = nullptr;
    int Cp = 0;
};

// Lifts diag(A) and sets the level scales s_k of M_hier^-1 (alpha, beta:
// the preconditioner's level weighting) into the pyramid buffers of w, and
// fills `hp` with the launches of one application.
bs_status prec_setup(const GridImpl& g, const SolveWs& w, float alpha, float beta,
                     HierPrecPlan& hp, hipStream_t s);

// PCG over n images sharing lane width K.  `dev_imgs` / `blk2img` are device
// copies of `imgs` and of the block-to-image map (-1: an idle block); with
// dev_imgs NULL the one image is passed by value, with block0 = 0, and runs
// on G = its nb blocks.  G is the launch's block count,
// max_cp the largest Cp; `act` is the device array the images' active
// counters point into (contiguous, n entries), polled every check_every
// iterations.
bs_status run_pcg(int K, const PcgImage* imgs, int n, const PcgImage* dev_imgs,
                  const int32_t* blk2img, int G, int max_cp, const bs_solve_params& p,
                  const int32_t* act, hipStream_t s, const HierPrecPlan* hp = nullptr);

// y[v][c] = yw[v][c] for c < C (yw has stride Cp).
bs_status copy_unpadded(const GridImpl& g, const float* yw, int C, int Cp, float* y,
                        hipStream_t s);

// dL/dt, dL/dc from the adjoint solution g (stride Cp).
bs_status grad_scatter_launch(const GridImpl& g, const float* gb, int Cp, const float* y_hat,
                              const float* target, const float* conf, int C, float* grad_t,
                              float* grad_c, hipStream_t s);

// Low-rank reduction of many right-hand sides (the part after the splat and
// before the expansion).  The reduced system of t channels shares A's arrays
// with w1 and keeps its own vectors in `extra` (lowrank_extra_bytes, laid
// out for nb reducing blocks, 0: the single-image default).
struct LowRankPlan {
    SolveWs w;                 // the reduced system (t channels)
    int t = 0;
    const float* Rt = nullptr; // device [t][C]
};
size_t lowrank_extra_bytes(const GridImpl& g, int C, int nb);
// Gram matrix, host factorisation (synchronises s), projection of w1.b onto
// Q~ and the reduced system's initial state in out.w.yi.
bs_status lowrank_prepare(const GridImpl& g, const SolveWs& w1, char* extra, int nb, double eps,
                          const bs_solve_params& p, hipStream_t s, LowRankPlan& out);
// y [Vcap][C] = Z R~ (0 when t = 0).
bs_status lowrank_finish(const GridImpl& g, const LowRankPlan& lr, int C, float* y,
                         hipStream_t s);

}  // namespace bs
