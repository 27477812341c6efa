/*
 * bsolve.h -- C ABI of the MI355X bilateral-space solver.
 *
 * Implements the bilateral solver of Barron & Poole, "The Fast Bilateral
 * Solver": build a simplified bilateral grid from a reference image
 * (Section 2, Eq. factorization and Eq. equiv), bistochastize its blur
 * (supplement Algorithm 1), solve A y = b with
 *     A = lam (D_m - D_n B D_n) + diag(S c),   b = S (c o t)   (Eq. quad_min)
 * by preconditioned conjugate gradients (supplement Algorithm 2) with the
 * Jacobi preconditioner and flat or hierarchical initialisation (Section 4,
 * supplement Section 2), slice y back to pixels (Eq. solution), and
 * back-propagate onto the target and confidence (Section 3).  On top of the
 * solve: batches of images of uneven size and channel count, the robust
 * solver (supplement Algorithm RBS), the low-rank reduction of many
 * right-hand sides (supplement Section Multiple Output Channels) and the
 * domain-transform post-process of the output (Section 4).
 *
 * Conventions shared by every entry point:
 *  - Pointers named as device pointers must point to device memory of the
 *    GPU current on the calling thread; the caller allocates and owns all of
 *    it.  No entry point allocates device memory.  Buffers must be 4-byte
 *    aligned, workspaces 256-byte aligned.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Entry points
 *    enqueue work on `stream` and return; results are ready when the stream
 *    reaches them.  The exceptions synchronise `stream` while they run and
 *    say so: bs_grid_vertex_count and bs_read_counters, solves and batch
 *    runs with convergence polls (check_every > 0), bs_batch_plan_create,
 *    the synchronous batch calls and the low-rank solves.
 *  - Arguments are validated on the host before anything is enqueued.  On an
 *    error nothing is launched, outputs are untouched and bs_last_error()
 *    returns a description (thread-local).
 *  - Images are planar float32: reference [3][H][W] (R, G, B in [0, 1]),
 *    target [C][H][W], confidence [H][W].  Bilateral-space vectors are
 *    vertex-major float32 [V][C] (channels contiguous per vertex) with
 *    room for Vcap vertices (bs_grid_view.vcap; Vcap <= H*W, so H*W rows
 *    always suffice).
 *  - Device data are not scanned: targets and confidences are expected to be
 *    finite, confidences >= 0.  A non-finite value reaches the channels whose
 *    arithmetic it enters (all of them, for a confidence): they stop after
 *    their first iteration with reason 4 and a non-finite rel_residual in
 *    bs_chan_stats, and their output is not finite; other channels are
 *    unaffected.  A negative confidence can make A indefinite, which stops a
 *    channel with reason 4 once d^T A d <= 0.
 *  - Readings of passages the paper leaves open (colour space, rounding,
 *    vertex order, blur form, stopping rules) are documented with the
 *    operation they affect below.
 */
#ifndef BSOLVE_H
#define BSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bs_status {
    BS_OK = 0,
    BS_EINVAL = -1,        /* an argument is invalid                            */
    BS_EWORKSPACE = -2,    /* a workspace is smaller than its query returned     */
    BS_EDEVICE = -3,       /* a HIP call failed; bs_last_error() holds its text  */
    BS_EUNSUPPORTED = -4   /* valid but outside what this library implements     */
} bs_status;

#define BS_MAX_CHANNELS 64
#define BS_MAX_LEVELS 24
#define BS_GRID_BYTES 4096

/* Grid scales of the bilateral affinity (Section 2, Eq. bilateral_affinity):
 * sigma_xy in pixels, sigma_l and sigma_uv in 8-bit colour codes.  All three
 * are positive integers (sigma_xy <= 128, colour scales <= 255). */
typedef struct bs_grid_params {
    int32_t sigma_xy;
    int32_t sigma_l;
    int32_t sigma_uv;
} bs_grid_params;

/* Bistochastization (supplement Algorithm 1).  The iteration
 *     n <- sqrt(n o m / (B n)),  n = 1 initially
 * stops when max_v |n_v (B n)_v - m_v| / m_v <= tol or after max_iters
 * updates.  `check_every` > 0 makes the host poll the device-side stop flag
 * every `check_every` launches: the flag is copied to pinned host memory
 * behind each check point and the host waits for the copy of the check point
 * before (the device keeps one check period of launches queued, which do
 * nothing once the fixed point is reached), and the call waits for its last
 * copy before returning; 0 enqueues all max_iters + 1 launches without any
 * synchronisation (graph-capturable; launches after convergence do
 * nothing). */
typedef struct bs_bistoch_params {
    int32_t max_iters;     /* default 200   */
    int32_t check_every;   /* default 8     */
    double tol;            /* default 1e-10 */
} bs_bistoch_params;

enum { BS_INIT_FLAT = 0, BS_INIT_HIER = 1 };
enum { BS_PRECOND_JACOBI = 0, BS_PRECOND_HIER = 1 };

/* The solve (Eq. quad_min, supplement Algorithm 2, Section 4).
 * Preconditioner (Section 4, Eq. hier_precond): the Jacobi inverse
 * 1 / diag(A), or the hierarchical M_hier^-1 r = P^T(s o P(r)) with level
 * scales s_k = pre_alpha^-(pre_beta + k) P(1)_k / P(diag A)_k for k >= 1 and
 * 1 / diag(A) at k = 0 (a coefficient with P(diag A) = 0 is 0).  With the
 * hierarchical preconditioner every PCG iteration applies A directly and runs
 * the preconditioner's pyramid passes (about 2 K launches per iteration);
 * single-image solves only (batch plans return BS_EUNSUPPORTED).
 * One PCG per channel with its own scalars.  A channel stops when its
 * recursive ||r|| / ||b|| <= rel_tol (rel_tol = 0: never), after max_iters
 * iterations, when r^T s = 0, or when d^T A d <= 0.  `check_every` works as
 * for bistochastization: > 0 polls the all-channels-done flag every that many
 * iterations, 0 enqueues exactly max_iters iterations. */
typedef struct bs_solve_params {
    float lambda;          /* smoothness multiplier, >= 0                       */
    int32_t init;          /* BS_INIT_FLAT or BS_INIT_HIER (default)            */
    int32_t max_iters;     /* PCG iterations cap (the paper's default is 25)    */
    int32_t check_every;   /* default 8                                         */
    double rel_tol;        /* relative residual target, 0 = fixed iterations    */
    float init_alpha;      /* hierarchical init level weighting, default 4      */
    float init_beta;       /* default 0                                         */
    int32_t precond;       /* BS_PRECOND_JACOBI (default) or BS_PRECOND_HIER     */
    float pre_alpha;       /* hierarchical preconditioner level weighting,     */
    float pre_beta;        /* default 2 and 5                                   */
} bs_solve_params;

/* Per-channel outcome, written to device memory by a solve. */
typedef struct bs_chan_stats {
    int32_t iters;         /* PCG iterations performed                          */
    int32_t reason;        /* 0 running, 1 tolerance met, 2 max_iters, 3 r^T s = 0,
                              4 d^T A d <= 0, 5 b = 0                           */
    double rel_residual;   /* recursive ||r|| / ||b|| at exit                   */
    double bnorm;          /* ||b||                                             */
} bs_chan_stats;

/* A grid handle: a host-side plain struct holding the grid's dimensions and
 * device pointers into the workspace given to bs_build_grid.  Copyable; the
 * workspace must outlive every use.  There is no destroy call. */
typedef struct bs_grid {
    uint64_t opaque[BS_GRID_BYTES / 8];
} bs_grid;

/* Device pointers to a built grid's arrays, for inspection and tests.
 * counts (int32, device): [0] V, [1] K, [2] bistochastization updates,
 * [3] bistochastization done flag, [4] ping-pong buffer of the final n,
 * [5] 1 when some neighbour lies more than 32767 ids from its vertex (never
 * on grids with nb_packed), [8 + k] V_k for k < levels (0 for levels above K). */
typedef struct bs_grid_view {
    int32_t H, W, P, levels;           /* levels = capacity of the pyramid (K <= levels - 1) */
    int32_t ncells_x, ncells_y;        /* spatial cells of level 0                          */
    int64_t vcap;                      /* capacity of level-0 vertex arrays                  */
    const int32_t* counts;
    const double* bist_residual;       /* [1] device                                        */
    const uint64_t* key;               /* [vcap] packed (y:16 x:16 l:8 u:8 v:8), ascending   */
    const int32_t* idx;                /* [P] vertex of each pixel (S as an index)           */
    const int32_t* m;                  /* [vcap] pixels per vertex, m = S 1                  */
    const int32_t* nbr;                /* [10][vcap] neighbour id or -1, slot 2d: -1 step and
                                          2d+1: +1 step along dim d of (y, x, l, u, v)       */
    const int32_t* pix_ptr;            /* [vcap + 1] CSR of pixels per vertex                */
    const int32_t* pix_list;           /* [P] pixel ids, ascending within each vertex        */
    const double* n;                   /* [vcap] bistochastization vector n                   */
    const float* nf;                   /* [vcap] n rounded to float                          */
    const double* nn;                  /* [vcap] n o (N n), the smoothness diagonal / lam    */
    int64_t level_cap[BS_MAX_LEVELS];  /* capacity of level-k arrays                         */
    const uint64_t* level_key[BS_MAX_LEVELS];   /* [k >= 1] keys of level k                  */
    const int32_t* parent[BS_MAX_LEVELS];       /* [k < levels-1] level-k vertex -> level k+1 */
    const int32_t* ones[BS_MAX_LEVELS];         /* [k >= 1] level-0 vertices under each vertex (P(1)) */
    const uint32_t* nb16;              /* [5][vcap] nbr packed: word i holds slots 2i (low half)
                                          and 2i+1 (high half) as signed 16-bit u - v, 0 for -1;
                                          exact where counts[5] == 0                          */
    int32_t nb_packed;                 /* 1: every offset fits by construction (at most one row
                                          of cells plus one cell apart; checked on the host from
                                          the image width and the scales), and the stencil
                                          passes read nb16; 0: they read nbr                  */
} bs_grid_view;

/* ---------------------------------------------------------------------- */
/* Grid construction: supplement Section 1 (simplified bilateral grid,     */
/* Eq. SS) and Section 2 (bilateral pyramid).                              */
/* ---------------------------------------------------------------------- */

/* Bytes of device workspace bs_build_grid needs for an H x W image (host,
 * pure).  Returns 0 for invalid arguments. */
size_t bs_grid_workspace_bytes(int32_t H, int32_t W, const bs_grid_params* params);

/* Builds the simplified bilateral grid of `ref` (its pyramid is built by the
 * first bs_bistochastize call on the handle).
 *  ref  device float32 [3][H][W], RGB in [0, 1].
 * Each pixel is quantised to 8 bits (clamp(floor(255 v + 1/2), 0, 255), NaN
 * -> 0), converted to JFIF (BT.601 full-range) YCbCr in 16.16 fixed point, and
 * mapped to the integer grid coordinates round_half_up(v / sigma) of
 * (y, x, l=Y, u=Cb, v=Cr).  Vertices are the distinct coordinates in ascending
 * (y, x, l, u, v) order; each pixel lies on exactly one vertex (S S^T = D_m).
 * The blur B is the sum over the five dimensions of [1 2 1] blurs (diagonal
 * 10, neighbours missing from the grid contribute 0).  Pyramid level k+1
 * halves level-k coordinates (floor) until one vertex remains.
 *  ws   device workspace of bs_grid_workspace_bytes(H, W, params) bytes; the
 *       grid lives in it.
 *  out  host struct receiving the handle. */
bs_status bs_build_grid(const float* ref, int32_t H, int32_t W, const bs_grid_params* params,
                        void* ws, size_t ws_bytes, void* stream, bs_grid* out);

/* Bistochastizes the grid's blur in float64 (supplement Algorithm 1), storing
 * n, its float copy and n o (N n) in the grid.  The first call on a handle
 * also builds the pyramid levels k >= 1, on a library stream that overlaps the
 * bistochastization and is joined back into `stream` before the call returns
 * (work enqueued on `stream` afterwards sees both).  Must follow
 * bs_build_grid on the same stream; updates the handle. */
bs_status bs_bistochastize(bs_grid* grid, const bs_bistoch_params* params, void* stream);

/* ---------------------------------------------------------------------- */
/* Solve, slice and backward: Eq. quad_min, Eq. solution, Section 3/4.     */
/* ---------------------------------------------------------------------- */

/* Bytes of device workspace bs_solve / bs_solve_backward need for C channels
 * (host, pure).  Returns 0 for invalid arguments. */
size_t bs_solve_workspace_bytes(const bs_grid* grid, int32_t C);

/* Solves A y = b for C channels sharing the confidence (supplement Section 4).
 *  target  device float32 [C][H][W];  conf device float32 [H][W], >= 0.
 *  y       device float32 [Vcap][C] output: the bilateral-space solution.
 *  stats   device bs_chan_stats [C] output, or NULL.
 * S c and b = S (c o t) are deterministic per-vertex sums in ascending pixel
 * order; diag(A) = lam n o (N n) + S c (the value of lam (m - 10 n^2) + S c at
 * the bistochastization fixed point, free of cancellation); the Jacobi inverse
 * is 0 where diag(A) <= 0.  Flat init is S(c t)/S(c) (0 where S c = 0); the
 * hierarchical init is P^T(w P(b)/P(1)) / P^T(w P(S c)/P(1)) with
 * w_0 = 1, w_k = alpha^-(beta + k); all-zero confidence gives y0 = 0.
 * Dot products are accumulated in float64; vectors are float32. */
bs_status bs_solve(const bs_grid* grid, const float* target, const float* conf, int32_t C,
                   const bs_solve_params* params, float* y, void* ws, size_t ws_bytes,
                   bs_chan_stats* stats, void* stream);

/* Slices y [Vcap][C] back to pixels: x[c][p] = y[idx[p]][c] (Eq. solution).
 *  x  device float32 [C][H][W] output. */
bs_status bs_slice(const bs_grid* grid, const float* y, int32_t C, float* x, void* stream);

/* Back-propagates dL/dx through the solver (Section 3):
 *  u = S dL/dx,  g = A^{-1} u  (same A, preconditioner and init operator),
 *  dL/dt[c][p] = conf[p] g[idx[p]][c],
 *  dL/dconf[p] = sum_c g[idx[p]][c] (t[c][p] - y_hat[idx[p]][c]).
 * A connected component of the grid (vertices joined by blur neighbours)
 * without any confidence makes A singular.  If dL/dx does not vanish on it,
 * A g = u has no solution: the adjoint PCG cannot meet its tolerance
 * (bs_chan_stats reports it) and the gradients are not defined, as with the
 * paper's formula.  If it vanishes there (a confidence-weighted dL/dx does),
 * g on that component is what PCG keeps of its initial state.  The forward
 * solve is always defined (b = 0 on such a component).
 *  y_hat   device float32 [Vcap][C], the forward solution from bs_solve.
 *  grad_x  device float32 [C][H][W].
 *  grad_t  device float32 [C][H][W] output;  grad_c device float32 [H][W] output.
 *  g_out   device float32 [Vcap][C] output receiving dL/db, or NULL. */
bs_status bs_solve_backward(const bs_grid* grid, const float* target, const float* conf,
                            const float* y_hat, const float* grad_x, int32_t C,
                            const bs_solve_params* params, float* grad_t, float* grad_c,
                            float* g_out, void* ws, size_t ws_bytes, bs_chan_stats* stats,
                            void* stream);

/* ---------------------------------------------------------------------- */
/* The solve without a workspace argument.                                 */
/* ---------------------------------------------------------------------- */

/* Size of the library's static device scratch array (64 MiB per GPU). */
#define BS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory around a solve: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Does what bs_solve does, with the same kernels and results, but the solve
 * workspace is a static device array of the library (BS_NOALLOC_SCRATCH_BYTES
 * on every GPU that loads the library, held until the process ends) instead
 * of a buffer of the caller.  The caller still passes the grid (built in its
 * own workspace), the inputs and the outputs y and stats.  The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine): the array's
 * device address is looked up once per device, on the first call there.
 *  - params->check_every must be 0: the call only enqueues and never waits
 *    (BS_EINVAL otherwise);
 *  - BS_EUNSUPPORTED when bs_solve_workspace_bytes(grid, C) exceeds
 *    BS_NOALLOC_SCRATCH_BYTES (e.g. 64 MiB holds one channel of a 1024 x 768
 *    image, or three of a 512 x 512 one), and while kernel timing is enabled
 *    (timing records events);
 *  - every call on one GPU uses that GPU's one array, which keeps the last
 *    call's contents.  Nothing in it needs clearing (a solve writes every
 *    workspace byte before reading it), but calls whose work overlaps on one
 *    GPU (several streams, or several host threads) race on it and give
 *    undefined results: order them on one stream, or with events. */
bs_status bs_solve_noalloc(const bs_grid* grid, const float* target, const float* conf,
                           int32_t C, const bs_solve_params* params, float* y,
                           bs_chan_stats* stats, void* stream);

/* ---------------------------------------------------------------------- */
/* Robust solver: supplement Section Robustness, Algorithm RBS.            */
/* ---------------------------------------------------------------------- */

/* Bytes of device workspace bs_robust_solve needs for C channels: the solve
 * workspace followed by the IRLS weights (float32 [H][W]).  Host, pure;
 * 0 for invalid arguments. */
size_t bs_robust_workspace_bytes(const bs_grid* grid, int32_t C);

/* The robust bilateral solver: iteratively reweighted least squares with the
 * Geman-McClure loss rho(e) = e^2 / (sigma_gm^2 + e^2).  Round i (of
 * irls_iters >= 1) runs bs_solve with confidence c_i and slices its solution
 * to x; c_0 = conf_init and c_{i+1} = 2 sigma_gm^2 / (sigma_gm^2 + e)^2 per
 * pixel, e = sum over channels of (x - t)^2 (the printed weight for one
 * channel), computed in float64 and stored as float32.  Each round solves
 * from its own initial state, as bs_solve does.
 *  target     device float32 [C][H][W];  conf_init device float32 [H][W].
 *  y          device float32 [Vcap][C] output: the last round's solution.
 *  x          device float32 [C][H][W] output: the last round's S^T y.
 *  stats      device bs_chan_stats [C] output for the last round, or NULL.
 *  ws         device workspace of bs_robust_workspace_bytes, 256-byte
 *             aligned, owned by the caller.
 * Errors: BS_EINVAL for sigma_gm <= 0 or not finite, irls_iters < 1, a NULL
 * or misaligned x, and every argument error of bs_solve; BS_EWORKSPACE for a
 * short workspace.  Checked before any work is enqueued; conf_init is not
 * modified.  Enqueues on `stream` (synchronising it only where bs_solve does,
 * for check_every > 0). */
bs_status bs_robust_solve(const bs_grid* grid, const float* target, const float* conf_init,
                          int32_t C, const bs_solve_params* params, float sigma_gm,
                          int32_t irls_iters, float* y, float* x, void* ws, size_t ws_bytes,
                          bs_chan_stats* stats, void* stream);

/* ---------------------------------------------------------------------- */
/* Low-rank reduction of many right-hand sides: supplement Section         */
/* Multiple Output Channels.                                               */
/* ---------------------------------------------------------------------- */

/* Bytes of device workspace bs_solve_lowrank needs for C channels (host,
 * pure; 0 for invalid arguments). */
size_t bs_lowrank_workspace_bytes(const bs_grid* grid, int32_t C);

/* Solves A Y = B, B = S(c o t) [V][C], through a low-rank reduction of B:
 * B P = Q R with column pivoting, the rows of R P^T ordered by non-increasing
 * mass (squared norm) with the columns of Q alike, and the fewest rows t whose
 * mass reaches (1 - eps) of the total, so that at most eps of B's squared
 * norm is dropped; then A Z = Q~ (t right-hand sides, each by the same
 * initialisation and PCG as bs_solve) and Y = Z R~.  R is computed from the
 * Gram matrix B^T B, summed in float64 in a fixed order, by bs_lowrank_factor.
 *  target  device float32 [C][H][W];  conf device float32 [H][W], >= 0.
 *  eps     in [0, 1): 0 keeps every independent row.
 *  y       device float32 [Vcap][C] output (all zero when B = 0).
 *  stats   device bs_chan_stats [C] or NULL: entries 0..t-1 describe the
 *          reduced systems; the rest are not written.
 *  rank    host int32 output: t.
 * Synchronises `stream` (the factorisation runs on the host, between the
 * splat and the reduced solve).  Errors as bs_solve, plus BS_EINVAL for eps
 * outside [0, 1) or a NULL rank. */
bs_status bs_solve_lowrank(const bs_grid* grid, const float* target, const float* conf,
                           int32_t C, const bs_solve_params* params, double eps, float* y,
                           void* ws, size_t ws_bytes, bs_chan_stats* stats, int32_t* rank,
                           void* stream);

/* The factorisation step of bs_solve_lowrank on the host (pure, no device
 * work): from the Gram matrix G = B^T B (float64 [C][C], row-major,
 * symmetric), a Cholesky factorisation with diagonal pivoting gives R of
 * B P = Q R (the largest remaining diagonal is the largest remaining column
 * norm); pivots at or below 1e-13 of the largest diagonal end it.  Writes
 * t, M (float32 [C][t], Q~ = B M) and R~ (float32 [t][C], the kept rows of
 * R P^T in order of mass).  M and Rt must hold C*C floats. */
bs_status bs_lowrank_factor(const double* gram, int32_t C, double eps, float* M, float* Rt,
                            int32_t* rank);

/* ---------------------------------------------------------------------- */
/* Domain transform: the post-process of the solver's output (Section 4,   */
/* post-processing) and the robust solver's initial confidence (supplement */
/* Section Robustness, the equations for V and c_init).                    */
/* ---------------------------------------------------------------------- */

/* The recursive filter of Gastal and Oliveira's domain transform, guided by
 * the reference image.  Neighbouring pixels lie d = 1 + (sigma_s / sigma_r)
 * sum_c |I_c(p) - I_c(q)| apart, I the reference's 8-bit R, G, B codes
 * (clamp(floor(255 v + 1/2), 0, 255), as the grid quantises them).  Each of
 * `iters` iterations filters every row, then every column: the recursion
 * J[x] = (1 - a^d) I[x] + a^d J[x-1] forwards along the line, then backwards
 * on its output, a = exp(-sqrt(2) / sigma_i), sigma_i = sigma_s sqrt(3)
 * 2^(iters - i) / sqrt(4^iters - 1) for iteration i = 1..iters (the
 * iterations' variances add up to sigma_s^2).  The first pixel of a line in
 * each direction passes unchanged.  The paper does not state the iteration
 * count; 3 is the filter's usual one. */
typedef struct bs_dt_params {
    float sigma_s;         /* spatial bandwidth sigma'_xy in pixels, > 0        */
    float sigma_r;         /* range bandwidth sigma'_rgb in 8-bit codes, > 0    */
    int32_t iters;         /* 1..16                                             */
} bs_dt_params;

/* Bytes of device workspace of bs_domain_transform and bs_dt_confidence for
 * an H x W image: the domain distances (uint32 [H][W]), the two signals of
 * the variance (float32 [2][H][W]) and 256 float64 partial sums.  Host, pure; 0 for
 * invalid sides (below 1, above 65535, or above 2^30 pixels). */
size_t bs_dt_workspace_bytes(int32_t H, int32_t W);

/* Filters x (device float32 [C][H][W], 1 <= C <= BS_MAX_CHANNELS) into out
 * (device float32 [C][H][W]; out == x filters in place, any other overlap is
 * BS_EINVAL), guided by ref (device float32 [3][H][W] in [0, 1], as for
 * bs_build_grid).  ws: device workspace of bs_dt_workspace_bytes(H, W) bytes,
 * 256-byte aligned.  Errors: BS_EINVAL for a NULL or misaligned pointer,
 * sides below 1, C out of range, sigma_s or sigma_r not positive and finite,
 * iters outside 1..16; BS_EUNSUPPORTED for sides above 65535 or more than
 * 2^30 pixels; BS_EWORKSPACE for a short workspace.  Enqueues 1 + 2 iters
 * launches on `stream` and never synchronises it (graph-capturable). */
bs_status bs_domain_transform(const float* ref, int32_t H, int32_t W, const float* x, int32_t C,
                              const bs_dt_params* params, float* out, void* ws, size_t ws_bytes,
                              void* stream);

/* The initial confidence of the robust solver from the edge-aware variance
 * of a depth or disparity map z (device float32 [H][W]):
 *     V = DT(z^2) - DT(z)^2,   conf = exp(-max(V, 0) / (2 sigma_dt^2)),
 * DT the filter of bs_domain_transform with `params`, and conf = 0 in the
 * leftmost zero_cols columns (the paper zeroes 80 columns of its stereo
 * pairs, whose left side has no match in the other view).  V is evaluated on
 * z minus its mean (float64), which leaves it unchanged and keeps float32
 * rounding relative to the spread of z.  conf: device float32 [H][W] output.
 * Errors as bs_domain_transform, plus BS_EINVAL for sigma_dt not positive and
 * finite or zero_cols < 0.  Enqueues on `stream` without synchronising. */
bs_status bs_dt_confidence(const float* ref, int32_t H, int32_t W, const float* z,
                           const bs_dt_params* params, float sigma_dt, int32_t zero_cols,
                           float* conf, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Batches: many images of uneven size and channel count (Section 3's      */
/* forward and backward over a batch, e.g. a segmentation minibatch).      */
/* ---------------------------------------------------------------------- */

/* One image of a batch.  All pointers are device pointers except as noted.
 *  ref [3][H][W], target [C][H][W], conf [H][W]: inputs as for bs_build_grid
 *      and bs_solve.
 *  grid_ws, grid_ws_bytes: the image's grid workspace
 *      (bs_grid_workspace_bytes(H, W, &sigma) bytes), kept by the caller from
 *      the forward to the backward call.
 *  y  [Vcap][C]: written by bs_batch_forward, read by bs_batch_backward.
 *  x  [C][H][W]: the sliced output of bs_batch_forward, or NULL.
 *  grad_x [C][H][W] in, grad_t [C][H][W] and grad_c [H][W] out: backward.
 *  stats [C]: per-channel outcome of the image's last solve, or NULL. */
typedef struct bs_batch_item {
    const float* ref;
    const float* target;
    const float* conf;
    int32_t H, W, C;
    bs_grid_params sigma;
    void* grid_ws;
    size_t grid_ws_bytes;
    float* y;
    float* x;
    const float* grad_x;
    float* grad_t;
    float* grad_c;
    bs_chan_stats* stats;
} bs_batch_item;

/* A batch plan (opaque, host memory): the layout of every image's grid and
 * solve workspace inside one device workspace, and the device tables of
 * every launch of a forward and a backward run.  Made on the host from the
 * images' sizes, grid scales and channel counts alone. */
typedef struct bs_batch_plan bs_batch_plan;

/* Device workspace bytes of a plan over `items` (host, pure; 0 for an invalid
 * batch).  Items with grid_ws NULL get their grid inside the workspace; the
 * others keep theirs in grid_ws.  Only H, W, C, sigma and grid_ws are read. */
size_t bs_batch_plan_workspace_bytes(const bs_batch_item* items, int32_t n);

/* Makes a plan over n <= 4096 images (Section 3's minibatch: many images of
 * uneven size and channel count, solved forward and backward together).  The
 * items' device pointers are bound into the plan: runs read and write those
 * buffers, whose contents the caller may change between runs.
 *  fwd  parameters of the forward solves (one set for every image);
 *  bwd  parameters of the adjoint solves, with fwd's lambda and init; NULL
 *       makes a forward-only plan (grad_x, grad_t, grad_c may then be NULL);
 *  bist bistochastization parameters (NULL: 200 updates, tol 1e-10, no polls);
 *  ws   device workspace of bs_batch_plan_workspace_bytes bytes, 256-byte
 *       aligned, owned by the caller and used by every run of the plan.
 * Uploads the plan's tables on `stream` and synchronises it (not capturable).
 *  out  receives the plan; free it with bs_batch_plan_destroy.
 * Errors: BS_EINVAL for a bad item or parameter (the message names the item),
 * BS_EWORKSPACE for a short workspace, BS_EUNSUPPORTED above 4096 images. */
bs_status bs_batch_plan_create(const bs_batch_item* items, int32_t n, const bs_solve_params* fwd,
                               const bs_solve_params* bwd, const bs_bistoch_params* bist,
                               void* ws, size_t ws_bytes, void* stream, bs_batch_plan** out);

/* Forward run of a plan: every image's grid and pyramid, bistochastization,
 * splat, initial state, PCG and slice (into x where the item has one; y
 * receives the solution).  Each stage is one launch over all images; the PCG
 * runs one launch per phase for each lane width (1, 2, 3 or 4 channels per
 * lane, see bs_solve_channel_stride), each image with its own per-channel
 * stopping rule; launches over vertices share their blocks among the images
 * by a schedule computed on the device from the vertex counts.  With
 * check_every = 0 in fwd and in bist the run only enqueues kernels on
 * `stream` (no host synchronisation): exactly max_iters PCG iterations and
 * max_iters + 1 bistochastization updates, which do nothing for an image
 * once it has stopped, so a run can be captured into a HIP graph and
 * replayed.  With check_every > 0 the run polls the stop flags and
 * synchronises `stream`.  Results match bs_solve per image to the solver's
 * tolerance (block partial sums run in another order) and are deterministic
 * for a given batch. */
bs_status bs_batch_run_forward(bs_batch_plan* plan, void* stream);

/* Backward run (as bs_solve_backward per image: splat of grad_x, adjoint
 * PCG, gradient scatter into grad_t and grad_c), after a forward run of the
 * same plan; y must hold the forward solutions.  Enqueue-only and
 * capturable under the same conditions as the forward run (bwd's
 * check_every). */
bs_status bs_batch_run_backward(bs_batch_plan* plan, void* stream);

/* The grid handle of image i of a plan (valid after a forward run). */
bs_status bs_batch_plan_grid(const bs_batch_plan* plan, int32_t i, bs_grid* out);

/* Frees a plan (host memory only; NULL is allowed). */
void bs_batch_plan_destroy(bs_batch_plan* plan);

/* Scratch bytes of the synchronous batch calls below (n_streams must be in
 * 1..16 and is otherwise unused); 0 for invalid arguments (host, pure).  One
 * workspace serves a forward call and the backward call that follows it. */
size_t bs_batch_workspace_bytes(const bs_batch_item* items, int32_t n, int32_t n_streams);

/* A forward run on a plan made for this call over items that each bring
 * their grid workspace (grid_ws): grid, bistochastization, solve, slice,
 * with the same params for all images, polling as params->check_every and
 * bist->check_every say.  The plan's table upload synchronises `stream`.
 *  grids  host array [n] receiving the grid handles, for bs_batch_backward.
 * Errors as bs_batch_plan_create. */
bs_status bs_batch_forward(const bs_batch_item* items, int32_t n, const bs_solve_params* params,
                           const bs_bistoch_params* bist, bs_grid* grids, int32_t n_streams,
                           void* ws, size_t ws_bytes, void* stream);

/* Backward run on a plan made for this call, on the grids of a previous
 * bs_batch_forward with the same items (each grid in its item's grid_ws), y
 * holding the forward solutions. */
bs_status bs_batch_backward(const bs_batch_item* items, int32_t n, const bs_grid* grids,
                            const bs_solve_params* params, int32_t n_streams, void* ws,
                            size_t ws_bytes, void* stream);

/* Tuning of the batched PCG: vertex tiles per block for lanes of K channels
 * (K in 1..4; a lane is K consecutive channels of one vertex, K =
 * bs_lane_width(C)), 1..64, or 0 for the default (16 for K >= 3, 8
 * otherwise).  Fewer tiles per block means more, shorter blocks.
 * Process-wide; read by the next batch call; BS_EINVAL out of range.  For
 * the autotuner, which times candidates on the caller's own batch. */
bs_status bs_batch_set_tiles_per_block(int32_t K, int32_t tiles);
/* The tiles per block in effect for lane width K (0 for K outside 1..4). */
int32_t bs_batch_tiles_per_block(int32_t K);
/* The lane width of C channels (host, pure; 0 outside 1..64). */
int32_t bs_lane_width(int32_t C);
/* Sets the lane width of C channels (1..4; 0 restores the default rule:
 * C for C <= 2, 4 when 4 divides C, 3 when 3 does, else 4).  The channel
 * stride becomes C rounded up to a multiple of it.  Process-wide; read when a
 * workspace is laid out (workspace queries, solves, batch plans), so a
 * workspace sized before a change may be too small after it (BS_EWORKSPACE).
 * For the autotuner.  BS_EINVAL out of range. */
bs_status bs_set_lane_width(int32_t C, int32_t K);

/* Scratch bytes of bs_batch_forward_lowrank: every image's solve workspace
 * and reduced system, plus the batched PCG's tables (0 for an invalid
 * batch). */
size_t bs_batch_lowrank_workspace_bytes(const bs_batch_item* items, int32_t n,
                                        int32_t n_streams);

/* Forward pass of every image through the low-rank reduction of its
 * right-hand sides (as bs_solve_lowrank, with the same eps for all images):
 * grid, bistochastization and splat of every image as in a batch run, the
 * reduction image by image (each factorisation synchronises `stream`), then
 * the reduced systems of rank > 0 through the batched PCG (grouped by lane
 * width of their rank), then Y = Z R~ into y and the slice into x.  ranks: host
 * int32 [n] output.  stats [C] of an item: entries 0..t-1 describe its
 * reduced systems.  Errors as bs_batch_forward, plus BS_EINVAL for eps
 * outside [0, 1) or a NULL rank array.  Returns after enqueuing; the stream
 * has been synchronised by the set-up. */
bs_status bs_batch_forward_lowrank(const bs_batch_item* items, int32_t n,
                                   const bs_solve_params* params, const bs_bistoch_params* bist,
                                   bs_grid* grids, int32_t n_streams, double eps, int32_t* ranks,
                                   void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------- */
/* Queries and diagnostics.                                                */
/* ---------------------------------------------------------------------- */

/* Copies the grid's device counters (see bs_grid_view.counts) to host
 * `out[n]`; synchronises `stream`. */
bs_status bs_read_counters(const bs_grid* grid, int32_t* out, int32_t n, void* stream);

/* Number of vertices V of a built grid; synchronises `stream`. */
bs_status bs_grid_vertex_count(const bs_grid* grid, int32_t* V, void* stream);

/* Fills `view` with the grid's device pointers and capacities (host only). */
bs_status bs_grid_get_view(const bs_grid* grid, bs_grid_view* view);

/* Device pointers into a solve workspace, valid after bs_solve: the splatted
 * right-hand side b [Vcap][Cs] with Cs = bs_solve_channel_stride(C) (after
 * bs_solve_backward: u = S dL/dx; channels C..Cs-1 are zero), S c [Vcap],
 * diag(A) [Vcap] and the Jacobi inverse [Vcap] (host only; for inspection and
 * tests).  Run bs_solve with max_iters = 0 to obtain the initial state y0 in
 * y. */
/* Channel stride of the solver's internal [V][Cs] vectors for C channels: C
 * for C <= 2, for C divisible by 4 or by 3, else C rounded up to a multiple
 * of 4 (0 for C outside 1..64). */
int32_t bs_solve_channel_stride(int32_t C);

bs_status bs_solve_ws_view(const bs_grid* grid, int32_t C, void* ws, size_t ws_bytes,
                           const float** b, const float** sc, const float** diag,
                           const float** minv);

/* Kernel timing for benchmarks.  While enabled, every kernel launch of the
 * library carries two hipEvents of its own, taken at the kernel's start and
 * end (hipExtLaunchKernelGGL; not graph-capturable).  bs_timing_read waits for
 * the events and
 * returns the summed elapsed milliseconds and launch count of one kernel:
 * "level_count", "level_scan", "level_write", "neighbour_table", "bist_step",
 * "bist_other", "splat", "init", "pcg_start", "pcg_matvec", "pcg_update",
 * "pcg_reduce", "slice", "grad_scatter", "dt_rows", "dt_cols" or "dt_other"
 * (the domain transform's other kernels).  bs_timing_reset clears the sums.
 * Every call enqueues its launches on one stream, one after another, so each
 * timed launch has the device to itself. */
bs_status bs_timing_enable(int32_t on);
bs_status bs_timing_reset(void);
bs_status bs_timing_read(const char* kernel, double* total_ms, int64_t* launches);

const char* bs_status_string(bs_status status);
const char* bs_last_error(void);
/* Library ABI version, (major << 16) | minor. */
int32_t bs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BSOLVE_H */
