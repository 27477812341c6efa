// Low-rank reduction of many right-hand sides (supplement Section Multiple
// Output Channels).  B = S(c o t) [V][C] is factorised B P = Q R with column
// pivoting, the rows of R P^T are ordered by their mass (squared norm), the
// fewest rows t that hold (1 - eps) of the mass are kept, A Z = Q~ is solved
// for the t columns of Q~ by the same initialisation and PCG as any
// right-hand side, and Y = Z R~.
//
// R comes from the Gram matrix B^T B, summed in float64 on the device in a
// fixed order, by a Cholesky factorisation with diagonal pivoting on the
// host: pivoting on the largest remaining diagonal is pivoting on the largest
// remaining column norm, so in exact arithmetic this is the R of the
// column-pivoted QR.  Q~ = B M with M = P R^-1 restricted to the kept rows.
#include <algorithm>
#include <cstring>
#include <vector>

#include "bs_solve_impl.h"

namespace bs {

constexpr int kGramBlocks = 256;   // blocks of the Gram kernel; their partials go to the host
constexpr int kGramRows = 64;      // vertices staged in LDS per round
constexpr int kPairSlots = (BS_MAX_CHANNELS * (BS_MAX_CHANNELS + 1) / 2 + kBlock - 1) / kBlock;

__host__ __device__ inline int pair_count(int C) { return C * (C + 1) / 2; }

// Block j sums b[v][i] b[v][k] (i <= k) over its rounds of kGramRows
// vertices, in float64, into part[j][pair]; pairs enumerate the upper
// triangle row by row.
__global__ void __launch_bounds__(kBlock) gram_partials(const float* __restrict__ b, int Cp, int C,
                                                        const int32_t* __restrict__ counts,
                                                        double* __restrict__ part) {
    __shared__ float rows[kGramRows * BS_MAX_CHANNELS];
    const int V = counts[CNT_V];
    const int np = pair_count(C);
    int pi[kPairSlots], pk[kPairSlots];
    double acc[kPairSlots];
#pragma unroll
    for (int s = 0; s < kPairSlots; ++s) {
        int q = (int)threadIdx.x + s * kBlock, i = 0;
        if (q < np) {
            while (q >= C - i) {
                q -= C - i;
                ++i;
            }
        }
        pi[s] = i;
        pk[s] = i + q;
        acc[s] = 0.0;
    }
    for (int64_t v0 = (int64_t)blockIdx.x * kGramRows; v0 < V;
         v0 += (int64_t)gridDim.x * kGramRows) {
        const int n = (int)std::min<int64_t>(kGramRows, V - v0);
        __syncthreads();
        for (int e = threadIdx.x; e < n * C; e += kBlock) {
            const int r = e / C;
            rows[e] = b[(v0 + r) * Cp + (e - r * C)];
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kPairSlots; ++s) {
            if ((int)threadIdx.x + s * kBlock < np) {
                for (int r = 0; r < n; ++r)
                    acc[s] += (double)rows[r * C + pi[s]] * (double)rows[r * C + pk[s]];
            }
        }
    }
#pragma unroll
    for (int s = 0; s < kPairSlots; ++s) {
        const int q = (int)threadIdx.x + s * kBlock;
        if (q < np) part[(int64_t)blockIdx.x * np + q] = acc[s];
    }
}

// z[v][j] = sum_i b[v][i] M[i][j] for j < t (Q~), 0 for t <= j < Cpz.
__global__ void __launch_bounds__(kBlock) lowrank_project(const float* __restrict__ b, int Cp,
                                                          int C, const float* __restrict__ M,
                                                          int t, float* __restrict__ z, int Cpz,
                                                          const int32_t* __restrict__ counts) {
    __shared__ float Ms[BS_MAX_CHANNELS * BS_MAX_CHANNELS];
    for (int e = threadIdx.x; e < C * t; e += kBlock) Ms[e] = M[e];
    __syncthreads();
    const int64_t n = (int64_t)counts[CNT_V] * Cpz;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kBlock) {
        const int64_t v = e / Cpz;
        const int j = (int)(e - v * Cpz);
        double s = 0.0;
        if (j < t) {
            for (int i = 0; i < C; ++i) s += (double)b[v * Cp + i] * (double)Ms[i * t + j];
        }
        z[e] = (float)s;
    }
}

// y[v][c] = sum_j z[v][j] Rt[j][c] (y with stride C).
__global__ void __launch_bounds__(kBlock) lowrank_expand(const float* __restrict__ z, int Cpz,
                                                         int t, const float* __restrict__ Rt,
                                                         int C, float* __restrict__ y,
                                                         const int32_t* __restrict__ counts) {
    __shared__ float Rs[BS_MAX_CHANNELS * BS_MAX_CHANNELS];
    for (int e = threadIdx.x; e < t * C; e += kBlock) Rs[e] = Rt[e];
    __syncthreads();
    const int64_t n = (int64_t)counts[CNT_V] * C;
    for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * kBlock) {
        const int64_t v = e / C;
        const int c = (int)(e - v * C);
        double s = 0.0;
        for (int j = 0; j < t; ++j) s += (double)z[v * Cpz + j] * (double)Rs[j * C + c];
        y[e] = (float)s;
    }
}

namespace {

struct Reduction {
    int t = 0;
    std::vector<float> M;    // [C][t]
    std::vector<float> Rt;   // [t][C]
};

// Pivoted Cholesky of the Gram matrix G (C x C, float64), the row masses of
// R P^T, the rank t and the factors M and R~.  t is the fewest rows, taken
// by decreasing mass, whose mass reaches (1 - eps) of the total, so at most
// eps of B's squared norm is dropped; R~ is those rows of R P^T (rows of R
// with their pivoted columns put back in channel order).
Reduction reduce_gram(const std::vector<double>& G, int C, double eps) {
    std::vector<int> perm(C);
    for (int i = 0; i < C; ++i) perm[i] = i;
    std::vector<double> R((size_t)C * C, 0.0);   // R[k][j]: row k, pivoted column j
    std::vector<double> d(C);
    double dmax0 = 0.0;
    for (int i = 0; i < C; ++i) {
        d[i] = G[(size_t)i * C + i];
        dmax0 = std::max(dmax0, d[i]);
    }
    auto g = [&](int a, int b) { return G[(size_t)perm[a] * C + perm[b]]; };
    int r = 0;
    for (int k = 0; k < C; ++k) {
        int jm = k;
        for (int j = k + 1; j < C; ++j)
            if (d[j] > d[jm]) jm = j;
        if (!(d[jm] > 1e-13 * dmax0)) break;
        if (jm != k) {
            std::swap(perm[k], perm[jm]);
            std::swap(d[k], d[jm]);
            for (int i = 0; i < k; ++i) std::swap(R[(size_t)i * C + k], R[(size_t)i * C + jm]);
        }
        const double rkk = std::sqrt(d[k]);
        R[(size_t)k * C + k] = rkk;
        for (int j = k + 1; j < C; ++j) {
            double s = g(k, j);
            for (int i = 0; i < k; ++i) s -= R[(size_t)i * C + k] * R[(size_t)i * C + j];
            R[(size_t)k * C + j] = s / rkk;
            d[j] -= R[(size_t)k * C + j] * R[(size_t)k * C + j];
        }
        r = k + 1;
    }
    Reduction out;
    if (r == 0) return out;
    // masses of the rows (column order does not change a row's norm)
    std::vector<double> mass(r, 0.0);
    for (int k = 0; k < r; ++k)
        for (int j = k; j < C; ++j) mass[k] += R[(size_t)k * C + j] * R[(size_t)k * C + j];
    std::vector<int> order(r);
    for (int k = 0; k < r; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return mass[a] > mass[b]; });
    double total = 0.0;
    for (int k = 0; k < r; ++k) total += mass[order[k]];
    const double want = (1.0 - eps) * total;
    double run = 0.0;
    int t = r;
    for (int k = 0; k < r; ++k) {
        run += mass[order[k]];
        if (run >= want) {
            t = k + 1;
            break;
        }
    }
    // R11^-1 (r x r upper triangular) by back substitution, column by column
    std::vector<double> Ri((size_t)r * r, 0.0);
    for (int c = 0; c < r; ++c) {
        Ri[(size_t)c * r + c] = 1.0 / R[(size_t)c * C + c];
        for (int i = c - 1; i >= 0; --i) {
            double s = 0.0;
            for (int k = i + 1; k <= c; ++k) s += R[(size_t)i * C + k] * Ri[(size_t)k * r + c];
            Ri[(size_t)i * r + c] = -s / R[(size_t)i * C + i];
        }
    }
    out.t = t;
    out.M.assign((size_t)C * t, 0.0f);
    out.Rt.assign((size_t)t * C, 0.0f);
    for (int j = 0; j < t; ++j) {
        const int o = order[j];
        for (int k = 0; k <= o; ++k) out.M[(size_t)perm[k] * t + j] = (float)Ri[(size_t)k * r + o];
        for (int k = 0; k < C; ++k) out.Rt[(size_t)j * C + perm[k]] = (float)R[(size_t)o * C + k];
    }
    return out;
}

size_t reduced_bytes(const GridImpl& g, int C, int nb) {
    SolveWs w;
    size_t r = 0;
    for (int t = 1; t <= C; ++t) r = std::max(r, layout_solve(g, t, nb, nullptr, w));
    return r;
}

}  // namespace

size_t lowrank_extra_bytes(const GridImpl& g, int C, int nb) {
    return align_up(reduced_bytes(g, C, nb), 256) +
           align_up((size_t)kGramBlocks * pair_count(C) * sizeof(double), 256) +
           align_up((size_t)2 * C * C * sizeof(float), 256);
}

bs_status lowrank_prepare(const GridImpl& g, const SolveWs& w1, char* extra, int nb, double eps,
                          const bs_solve_params& p, hipStream_t s, LowRankPlan& out) {
    const int C = w1.C;
    const int np = pair_count(C);
    double* part = (double*)(extra + align_up(reduced_bytes(g, C, nb), 256));
    float* dmat = (float*)((char*)part + align_up((size_t)kGramBlocks * np * sizeof(double), 256));
    BS_LAUNCH(s, K_SPLAT, "gram_partials", gram_partials, dim3(kGramBlocks), dim3(kBlock), 0, s,
              w1.b, w1.Cp, C, g.counts, part);
    std::vector<double> hp((size_t)kGramBlocks * np);
    BS_TRY_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost,
                              s));
    BS_TRY_HIP(hipStreamSynchronize(s));
    std::vector<double> G((size_t)C * C, 0.0);
    for (int q = 0, i = 0, k = 0; q < np; ++q) {
        double acc = 0.0;
        for (int j = 0; j < kGramBlocks; ++j) acc += hp[(size_t)j * np + q];
        G[(size_t)i * C + k] = G[(size_t)k * C + i] = acc;
        if (++k == C) k = ++i;
    }
    const Reduction rd = reduce_gram(G, C, eps);
    out.t = rd.t;
    out.Rt = nullptr;
    if (rd.t == 0) return BS_OK;
    std::vector<float> mats(rd.M);
    mats.insert(mats.end(), rd.Rt.begin(), rd.Rt.end());
    BS_TRY_HIP(hipMemcpyAsync(dmat, mats.data(), mats.size() * sizeof(float),
                              hipMemcpyHostToDevice, s));
    out.Rt = dmat + (size_t)C * rd.t;
    SolveWs& w2 = out.w;
    layout_solve(g, rd.t, nb, extra, w2);
    // the reduced system shares A: S c, diag(A), M^-1 and {n, M^-1}
    w2.sc = w1.sc;
    w2.diag = w1.diag;
    w2.minv = w1.minv;
    w2.nfm = w1.nfm;
    const int pblocks = grid_blocks(ceil_div(g.vcap * w2.Cp, kBlock));
    BS_LAUNCH(s, K_SPLAT, "lowrank_project", lowrank_project, dim3(pblocks), dim3(kBlock), 0, s,
              w1.b, w1.Cp, C, (const float*)dmat, rd.t, w2.b, w2.Cp, g.counts);
    bs_status st = init_state(g, w2, p, w2.yi, s);
    if (st != BS_OK) return st;
    // the host copy of the factors must outlive its transfer
    BS_TRY_HIP(hipStreamSynchronize(s));
    return BS_OK;
}

bs_status lowrank_finish(const GridImpl& g, const LowRankPlan& lr, int C, float* y,
                         hipStream_t s) {
    if (lr.t == 0) {
        // B = 0: Y = 0 (the solve's b = 0 case)
        BS_TRY_HIP(hipMemsetAsync(y, 0, (size_t)g.vcap * C * sizeof(float), s));
        return BS_OK;
    }
    const int eblocks = grid_blocks(ceil_div(g.vcap * C, kBlock));
    BS_LAUNCH(s, K_SLICE, "lowrank_expand", lowrank_expand, dim3(eblocks), dim3(kBlock), 0, s,
              lr.w.yi, lr.w.Cp, lr.t, lr.Rt, C, y, g.counts);
    return BS_OK;
}

}  // namespace bs

using namespace bs;

extern "C" bs_status bs_lowrank_factor(const double* gram, int32_t C, double eps, float* M,
                                       float* Rt, int32_t* rank) {
    if (!gram || !M || !Rt || !rank) return fail(BS_EINVAL, "NULL pointer argument");
    if (C < 1 || C > BS_MAX_CHANNELS) return fail(BS_EINVAL, "channel count must be in 1..64");
    if (!(eps >= 0.0 && eps < 1.0)) return fail(BS_EINVAL, "eps must be in [0, 1)");
    std::vector<double> G(gram, gram + (size_t)C * C);
    for (double v : G)
        if (!std::isfinite(v)) return fail(BS_EINVAL, "Gram matrix is not finite");
    const Reduction rd = reduce_gram(G, C, eps);
    *rank = rd.t;
    std::copy(rd.M.begin(), rd.M.end(), M);
    std::copy(rd.Rt.begin(), rd.Rt.end(), Rt);
    return BS_OK;
}

extern "C" size_t bs_lowrank_workspace_bytes(const bs_grid* grid, int32_t C) {
    const size_t full = bs_solve_workspace_bytes(grid, C);
    if (full == 0) return 0;
    return full + lowrank_extra_bytes(*impl(grid), C, 0);
}

extern "C" bs_status bs_solve_lowrank(const bs_grid* grid, const float* target, const float* conf,
                                      int32_t C, const bs_solve_params* params, double eps,
                                      float* y, void* ws, size_t ws_bytes, bs_chan_stats* stats,
                                      int32_t* rank, void* stream) {
    bs_status st = validate_solve(grid, C, params);
    if (st != BS_OK) return st;
    if (params->precond != BS_PRECOND_JACOBI)
        return fail(BS_EUNSUPPORTED, "the low-rank solve uses the Jacobi preconditioner");
    if (!(eps >= 0.0 && eps < 1.0)) return fail(BS_EINVAL, "eps must be in [0, 1)");
    if (!target || !conf || !y || !ws || !rank) return fail(BS_EINVAL, "NULL pointer argument");
    if (((uintptr_t)target & 3) || ((uintptr_t)conf & 3) || ((uintptr_t)y & 3) ||
        ((uintptr_t)ws & 255))
        return fail(BS_EINVAL, "misaligned buffer");
    const size_t need = bs_lowrank_workspace_bytes(grid, C);
    if (ws_bytes < need)
        return fail(BS_EWORKSPACE, "low-rank workspace needs " + std::to_string(need) + " bytes");
    const GridImpl& g = *impl(grid);
    const bs_solve_params& p = *params;
    hipStream_t s = (hipStream_t)stream;
    SolveWs w1;
    const size_t full = layout_solve(g, C, 0, ws, w1);
    st = splat_setup(g, w1, conf, target, true, (double)p.lambda, s);
    if (st != BS_OK) return st;
    LowRankPlan lr;
    st = lowrank_prepare(g, w1, (char*)ws + full, 0, eps, p, s, lr);
    if (st != BS_OK) return st;
    *rank = lr.t;
    if (lr.t > 0) {
        const PcgImage I = make_image(g, lr.w, p.lambda, lr.w.yi, stats);
        st = run_pcg(lr.w.K, &I, 1, nullptr, nullptr, lr.w.nb, lr.w.Cp, p, lr.w.act, s);
        if (st != BS_OK) return st;
    }
    return lowrank_finish(g, lr, C, y, s);
}
