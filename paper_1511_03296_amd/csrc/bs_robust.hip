// The robust bilateral solver (supplement Section Robustness, Algorithm RBS):
// iteratively reweighted least squares around the solve.  Each round solves
// with the current confidence, slices, and replaces the confidence by the
// Geman-McClure weights of the output's errors,
//   c_p = 2 s^2 / (s^2 + e_p)^2,   e_p = sum_ch (x[ch][p] - t[ch][p])^2
// (with one channel, the printed weight of e = x - t).
#include "bs_solve_impl.h"

namespace bs {

// One thread per pixel; the weight in float64 from float32 x and t.
__global__ void __launch_bounds__(kBlock) gm_reweight(const float* __restrict__ x,
                                                      const float* __restrict__ t, int C,
                                                      int64_t P, double s2,
                                                      float* __restrict__ c) {
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < P;
         p += (int64_t)gridDim.x * kBlock) {
        double e2 = 0.0;
        for (int ch = 0; ch < C; ++ch) {
            const double e = (double)x[(int64_t)ch * P + p] - (double)t[(int64_t)ch * P + p];
            e2 += e * e;
        }
        const double d = s2 + e2;
        c[p] = (float)(2.0 * s2 / (d * d));
    }
}

}  // namespace bs

using namespace bs;

extern "C" size_t bs_robust_workspace_bytes(const bs_grid* grid, int32_t C) {
    const size_t solve = bs_solve_workspace_bytes(grid, C);
    if (solve == 0) return 0;
    return solve + align_up((size_t)impl(grid)->P * sizeof(float), 256);
}

extern "C" bs_status bs_robust_solve(const bs_grid* grid, const float* target,
                                     const float* conf_init, int32_t C,
                                     const bs_solve_params* params, float sigma_gm,
                                     int32_t irls_iters, float* y, float* x, void* ws,
                                     size_t ws_bytes, bs_chan_stats* stats, void* stream) {
    const size_t solve = bs_solve_workspace_bytes(grid, C);
    if (solve == 0) return fail(BS_EINVAL, "bad grid or channel count");
    if (!(sigma_gm > 0.0f) || !std::isfinite(sigma_gm))
        return fail(BS_EINVAL, "sigma_gm must be positive and finite");
    if (irls_iters < 1) return fail(BS_EINVAL, "irls_iters must be >= 1");
    if (!x) return fail(BS_EINVAL, "NULL pointer argument");
    if (((uintptr_t)x & 3) != 0) return fail(BS_EINVAL, "misaligned buffer");
    const size_t need = bs_robust_workspace_bytes(grid, C);
    if (ws_bytes < need)
        return fail(BS_EWORKSPACE, "robust workspace needs " + std::to_string(need) + " bytes");
    const GridImpl& g = *impl(grid);
    hipStream_t s = (hipStream_t)stream;
    // the IRLS weights follow the solve workspace (256-byte aligned)
    float* c = ws ? (float*)((char*)ws + solve) : nullptr;
    const double s2 = (double)sigma_gm * (double)sigma_gm;
    for (int i = 0; i < irls_iters; ++i) {
        // bs_solve checks the remaining arguments before enqueuing anything
        bs_status st = bs_solve(grid, target, i == 0 ? conf_init : c, C, params, y, ws, solve,
                                stats, stream);
        if (st != BS_OK) return st;
        st = bs_slice(grid, y, C, x, stream);
        if (st != BS_OK) return st;
        if (i + 1 < irls_iters) {
            const int blocks = grid_blocks(ceil_div(g.P, kBlock));
            BS_LAUNCH(s, K_SLICE, "gm_reweight", gm_reweight, dim3(blocks), dim3(kBlock), 0, s, x,
                      target, C, (int64_t)g.P, s2, c);
        }
    }
    return BS_OK;
}
