// The C ABI used directly from a host program, without the Python binding:
// build the grid, bistochastize, solve and slice one image, then smooth the
// output with the domain transform (the calls of include/bsolve.h), with
// device memory from the HIP runtime.
//
//   solve_c H W C sigma_xy sigma_l sigma_uv lambda max_iters rel_tol in.bin out.bin
//
// in.bin holds float32 reference [3][H][W], target [C][H][W] and confidence
// [H][W]; out.bin receives x [C][H][W] as float32, the iteration count of
// every channel (int32 [C]) and the post-processed output [C][H][W] (domain
// transform with sigma'_xy = 4, sigma'_rgb = 8, 3 iterations).  Exits 1 with
// the library's error text on any failure.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#include "bsolve.h"

static void check(bs_status st, const char* what) {
    if (st != BS_OK) {
        std::fprintf(stderr, "%s: %s (%s)\n", what, bs_status_string(st), bs_last_error());
        std::exit(1);
    }
}

static void check_hip(hipError_t e, const char* what) {
    if (e != hipSuccess) {
        std::fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
        std::exit(1);
    }
}

static void* device(size_t bytes) {
    void* p = nullptr;
    check_hip(hipMalloc(&p, bytes ? bytes : 256), "hipMalloc");
    return p;
}

int main(int argc, char** argv) {
    if (argc != 12) {
        std::fprintf(stderr, "usage: %s H W C sigma_xy sigma_l sigma_uv lambda max_iters rel_tol "
                             "in.bin out.bin\n", argv[0]);
        return 2;
    }
    const int H = std::atoi(argv[1]), W = std::atoi(argv[2]), C = std::atoi(argv[3]);
    const bs_grid_params gp = {std::atoi(argv[4]), std::atoi(argv[5]), std::atoi(argv[6])};
    const float lambda = (float)std::atof(argv[7]);
    const int max_iters = std::atoi(argv[8]);
    const double rel_tol = std::atof(argv[9]);
    const size_t P = (size_t)H * W;

    std::vector<float> host(P * (3 + C + 1));
    FILE* f = std::fopen(argv[10], "rb");
    if (!f || std::fread(host.data(), sizeof(float), host.size(), f) != host.size()) {
        std::fprintf(stderr, "cannot read %s\n", argv[10]);
        return 1;
    }
    std::fclose(f);

    float* ref = (float*)device(P * 3 * sizeof(float));
    float* target = (float*)device(P * C * sizeof(float));
    float* conf = (float*)device(P * sizeof(float));
    check_hip(hipMemcpy(ref, host.data(), P * 3 * sizeof(float), hipMemcpyHostToDevice), "copy");
    check_hip(hipMemcpy(target, host.data() + P * 3, P * C * sizeof(float),
                        hipMemcpyHostToDevice), "copy");
    check_hip(hipMemcpy(conf, host.data() + P * (3 + C), P * sizeof(float),
                        hipMemcpyHostToDevice), "copy");

    // grid (Section 2) and bistochastization (supplement Algorithm 1)
    const size_t gws_bytes = bs_grid_workspace_bytes(H, W, &gp);
    if (gws_bytes == 0) check(BS_EINVAL, "bs_grid_workspace_bytes");
    void* gws = device(gws_bytes);
    bs_grid grid;
    check(bs_build_grid(ref, H, W, &gp, gws, gws_bytes, nullptr, &grid), "bs_build_grid");
    const bs_bistoch_params bp = {200, 8, 1e-10};
    check(bs_bistochastize(&grid, &bp, nullptr), "bs_bistochastize");

    // solve (Eq. quad_min, supplement Algorithm 2) and slice (Eq. solution)
    const size_t ws_bytes = bs_solve_workspace_bytes(&grid, C);
    void* ws = device(ws_bytes);
    float* y = (float*)device(P * C * sizeof(float));
    float* x = (float*)device(P * C * sizeof(float));
    bs_chan_stats* stats = (bs_chan_stats*)device(C * sizeof(bs_chan_stats));
    const bs_solve_params sp = {lambda,  BS_INIT_HIER, max_iters, 8, rel_tol, 4.0f, 0.0f,
                                BS_PRECOND_JACOBI, 2.0f, 5.0f};
    check(bs_solve(&grid, target, conf, C, &sp, y, ws, ws_bytes, stats, nullptr), "bs_solve");
    check(bs_slice(&grid, y, C, x, nullptr), "bs_slice");

    // domain-transform post-process (Section 4)
    const size_t dws_bytes = bs_dt_workspace_bytes(H, W);
    if (dws_bytes == 0) check(BS_EINVAL, "bs_dt_workspace_bytes");
    void* dws = device(dws_bytes);
    float* xd = (float*)device(P * C * sizeof(float));
    const bs_dt_params dp = {4.0f, 8.0f, 3};
    check(bs_domain_transform(ref, H, W, x, C, &dp, xd, dws, dws_bytes, nullptr),
          "bs_domain_transform");
    check_hip(hipDeviceSynchronize(), "hipDeviceSynchronize");

    std::vector<float> xo(P * C), xdo(P * C);
    std::vector<bs_chan_stats> so(C);
    check_hip(hipMemcpy(xo.data(), x, xo.size() * sizeof(float), hipMemcpyDeviceToHost), "copy");
    check_hip(hipMemcpy(xdo.data(), xd, xdo.size() * sizeof(float), hipMemcpyDeviceToHost),
              "copy");
    check_hip(hipMemcpy(so.data(), stats, so.size() * sizeof(bs_chan_stats),
                        hipMemcpyDeviceToHost), "copy");
    std::vector<int32_t> iters(C);
    for (int c = 0; c < C; ++c) iters[c] = so[c].iters;
    FILE* o = std::fopen(argv[11], "wb");
    if (!o) {
        std::fprintf(stderr, "cannot write %s\n", argv[11]);
        return 1;
    }
    std::fwrite(xo.data(), sizeof(float), xo.size(), o);
    std::fwrite(iters.data(), sizeof(int32_t), iters.size(), o);
    std::fwrite(xdo.data(), sizeof(float), xdo.size(), o);
    std::fclose(o);
    for (void* p : {(void*)ref, (void*)target, (void*)conf, gws, ws, (void*)y, (void*)x,
                    (void*)stats, dws, (void*)xd})
        check_hip(hipFree(p), "hipFree");
    return 0;
}
