// A solve that allocates nothing: bs_solve with its workspace taken from a
// static device array of the library instead of a buffer of the caller.
//
// The array is a file-scope __device__ variable: every GPU that loads the
// library's code object holds its own copy, at its own address, until the
// process ends.  In host code its name is only a stand-in for the symbol;
// the device address comes from hipGetSymbolAddress, asked once per device
// (with that device current) on the first call there, and kept.  Kernels and
// copies only ever see that address.
//
// Nothing in the array needs clearing between calls: every byte a solve
// reads from its workspace is written earlier by the same solve (the splat
// writes b, S c, diag(A) and the Jacobi inverse, the initialisation writes
// the pyramid buffers and y0, the PCG prologue writes the channel state).
#include "bs_solve_impl.h"

#include <mutex>
#include <vector>

static_assert(BS_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");

static __device__ __align__(256) unsigned char scratch[BS_NOALLOC_SCRATCH_BYTES];

namespace bs {
namespace {

struct ScratchTable {
    std::mutex mu;
    std::vector<void*> ptr;   // device address of `scratch` on each device (nullptr: not asked yet)
};

ScratchTable& table() {
    static ScratchTable t;
    return t;
}

// The address of the current device's copy of `scratch`.
bs_status scratch_address(void** out) {
    int dev = 0;
    BS_TRY_HIP(hipGetDevice(&dev));
    ScratchTable& t = table();
    std::lock_guard<std::mutex> lock(t.mu);
    if ((int)t.ptr.size() <= dev) t.ptr.resize(dev + 1, nullptr);
    if (!t.ptr[dev]) {
        void* p = nullptr;
        BS_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255) != 0)
            return fail(BS_EDEVICE, "scratch array has no usable device address");
        t.ptr[dev] = p;
    }
    *out = t.ptr[dev];
    return BS_OK;
}

}  // namespace
}  // namespace bs

using namespace bs;

extern "C" bs_status bs_solve_noalloc(const bs_grid* grid, const float* target, const float* conf,
                                      int32_t C, const bs_solve_params* params, float* y,
                                      bs_chan_stats* stats, void* stream) {
    bs_status st = validate_solve(grid, C, params);
    if (st != BS_OK) return st;
    if (params->check_every != 0)
        return fail(BS_EINVAL, "bs_solve_noalloc needs check_every = 0 (it never synchronises)");
    if (timing_enabled())
        return fail(BS_EUNSUPPORTED, "bs_solve_noalloc does not run while kernel timing is on "
                                     "(timing creates events)");
    const size_t need = bs_solve_workspace_bytes(grid, C);
    if (need == 0) return fail(BS_EINVAL, "bad grid or channel count");
    if (need > (size_t)BS_NOALLOC_SCRATCH_BYTES)
        return fail(BS_EUNSUPPORTED, "solve needs " + std::to_string(need) +
                                         " bytes of workspace; the scratch array holds " +
                                         std::to_string((size_t)BS_NOALLOC_SCRATCH_BYTES));
    void* ws = nullptr;
    st = scratch_address(&ws);
    if (st != BS_OK) return st;
    return bs_solve(grid, target, conf, C, params, y, ws, (size_t)BS_NOALLOC_SCRATCH_BYTES, stats,
                    stream);
}
