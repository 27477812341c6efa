// Simplified bilateral grid and bilateral pyramid construction (paper Section 2,
// Eq. factorization and Eq. equiv; supplement Section 1 Eq. SS and Section 2).
//
// Level 0 (the grid): every pixel is mapped to integer coordinates
// (y, x, l, u, v) and the vertices are the distinct coordinates in ascending
// packed-key order.  Level k+1 halves the coordinates of level k.  Because the
// spatial part (y, x) of a key is its most significant part, the ascending
// order groups vertices by spatial cell in raster order.  So each level is
// built without a device-wide sort:
//   1. count:  one block per spatial cell dedups the cell's item colour keys
//              (counting in LDS; deterministic) -> unique count per cell;
//   2. scan:   exclusive scan of the per-cell counts -> first vertex id per cell;
//   3. write:  one block per cell ranks each item's key among the cell's unique
//              keys -> vertex ids, keys, multiplicities and the item CSR.
// The items of level 0 are pixels (a cell is a rectangle of the image); the
// items of level k >= 1 are the vertices of the 2 x 2 child cells of level k-1,
// which are contiguous id ranges, visited in ascending id order.
#include "bs_grid_ops.h"

#include <mutex>
#include <vector>

namespace bs {

// ---------------------------------------------------------------------------
// Errors.
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

bs_status fail(bs_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

bs_status check_hip(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return BS_EDEVICE;
}

// ---------------------------------------------------------------------------
// Layout.
// ---------------------------------------------------------------------------
size_t layout_grid(GridImpl& g, int H, int W, const bs_grid_params& sp, void* base) {
    std::memset(&g, 0, sizeof(g));
    g.magic = kGridMagic;
    g.H = H;
    g.W = W;
    g.P = H * W;
    g.sg = sp;
    const int ncy0 = grid_coord(H - 1, sp.sigma_xy) + 1;
    const int ncx0 = grid_coord(W - 1, sp.sigma_xy) + 1;
    const int cl = grid_coord(255, sp.sigma_l);
    const int cu = grid_coord(255, sp.sigma_uv);
    int kmax = bit_length(ncy0 - 1);
    kmax = std::max(kmax, bit_length(ncx0 - 1));
    kmax = std::max(kmax, bit_length(cl));
    kmax = std::max(kmax, bit_length(cu));
    g.levels = kmax + 1;

    int64_t prev_cap = g.P;
    int max_cells = 0;
    for (int k = 0; k < g.levels; ++k) {
        Level& L = g.lv[k];
        L.ncy = ((ncy0 - 1) >> k) + 1;
        L.ncx = ((ncx0 - 1) >> k) + 1;
        const int64_t ncells = (int64_t)L.ncy * L.ncx;
        const int64_t colours = (int64_t)((cl >> k) + 1) * ((cu >> k) + 1) * ((cu >> k) + 1);
        const int64_t bound = ncells * colours;
        L.item_cap = (k == 0) ? g.P : prev_cap;
        L.cap = std::min<int64_t>(prev_cap, bound);
        if (L.cap < 1) L.cap = 1;
        prev_cap = L.cap;
        max_cells = std::max<int>(max_cells, (int)ncells);
    }
    g.vcap = g.lv[0].cap;
    g.max_cells = max_cells;
    {
        const int64_t colours = (int64_t)(cl + 1) * (cu + 1) * (cu + 1);
        const int64_t cell_max = std::min<int64_t>((int64_t)sp.sigma_xy * sp.sigma_xy, colours);
        g.nb_packed = packed_table_fits(ncx0, cell_max) ? 1 : 0;
    }

    Carver c(base);
    g.counts = c.take<int32_t>(CNT_SIZE);
    g.bist_res = c.take<double>(1);
    g.bist_part = c.take<double>(2 * kRedGridMax);
    g.cell_cnt = c.take<int32_t>(max_cells);
    g.cell_items = c.take<int32_t>(max_cells);
    g.ikey = c.take<uint32_t>(g.P);
    for (int k = 0; k < g.levels; ++k) {
        Level& L = g.lv[k];
        const int64_t ncells = (int64_t)L.ncy * L.ncx;
        L.key = c.take<uint64_t>(L.cap);
        L.mult = c.take<int32_t>(L.cap);
        L.ones = (k == 0) ? nullptr : c.take<int32_t>(L.cap);
        L.cell_vbase = c.take<int32_t>(ncells + 1);
        L.cell_ibase = c.take<int32_t>(ncells + 1);
        L.ptr = c.take<int32_t>(L.cap + 1);
        L.list = c.take<int32_t>(L.item_cap);
        L.item_parent = c.take<int32_t>(L.item_cap);
    }
    g.nbr = c.take<int32_t>(10 * g.vcap);
    g.nb16 = c.take<uint32_t>(5 * g.vcap);
    g.nbuf[0] = c.take<double>(g.vcap);
    g.nbuf[1] = c.take<double>(g.vcap);
    g.n64 = c.take<double>(g.vcap);
    g.nf = c.take<float>(g.vcap);
    g.nn = c.take<double>(g.vcap);
    g.ws = base;
    g.ws_bytes = align_up(c.off, 256);
    return g.ws_bytes;
}

// ---------------------------------------------------------------------------
// Host.
// ---------------------------------------------------------------------------
static bs_status validate_grid_args(int32_t H, int32_t W, const bs_grid_params* p) {
    if (!p) return fail(BS_EINVAL, "grid params is NULL");
    if (H < 1 || W < 1) return fail(BS_EINVAL, "image size must be positive");
    if (H > 65535 || W > 65535) return fail(BS_EUNSUPPORTED, "image side above 65535");
    if ((int64_t)H * W > (int64_t)1 << 30) return fail(BS_EUNSUPPORTED, "image above 2^30 pixels");
    if (p->sigma_xy < 1 || p->sigma_l < 1 || p->sigma_uv < 1)
        return fail(BS_EINVAL, "grid scales must be positive integers");
    if (p->sigma_xy > 128) return fail(BS_EUNSUPPORTED, "sigma_xy above 128");
    if (p->sigma_l > 255 || p->sigma_uv > 255) return fail(BS_EUNSUPPORTED, "colour scale above 255");
    return BS_OK;
}

template <int B, int CAP, class Src>
static bs_status launch_level(const Src& src, GridImpl& g, int k, hipStream_t st) {
    Level& L = g.lv[k];
    const int ncells = L.ncy * L.ncx;
    BS_LAUNCH(st, K_LEVEL_COUNT, "level_count", (one_launch<LevelCount<B, CAP, Src>>), dim3(ncells),
              dim3(B), 0, st, level_count_args<B, CAP>(src, g), 0);
    BS_LAUNCH(st, K_LEVEL_SCAN, "level_scan", one_launch<LevelScan>, dim3(1), dim3(kScanBlock), 0,
              st, level_scan_args(g, k), 0);
    BS_LAUNCH(st, K_LEVEL_WRITE, "level_write", (one_launch<LevelWrite<B, CAP, Src>>), dim3(ncells),
              dim3(B), 0, st, level_write_args<B, CAP>(src, g, k), 0);
    return BS_OK;
}

// Pyramid levels k >= 1 (they read level 0 only, so they may run on another
// stream than the bistochastization, which also reads level 0 only).
bs_status build_pyramid(const GridImpl& g0, hipStream_t s) {
    GridImpl& g = const_cast<GridImpl&>(g0);
    for (int k = 1; k < g.levels; ++k) {
        const Level& C = g.lv[k - 1];
        VertexSource vs{C.key, C.cell_vbase, g.counts, C.ncx, C.ncy, g.lv[k].ncx, k};
        const bs_status st = launch_level<128, 1024>(vs, g, k, s);
        if (st != BS_OK) return st;
    }
    return BS_OK;
}

}  // namespace bs

using namespace bs;

extern "C" size_t bs_grid_workspace_bytes(int32_t H, int32_t W, const bs_grid_params* params) {
    if (validate_grid_args(H, W, params) != BS_OK) return 0;
    GridImpl g;
    return layout_grid(g, H, W, *params, nullptr);
}

extern "C" bs_status bs_build_grid(const float* ref, int32_t H, int32_t W,
                                   const bs_grid_params* params, void* ws, size_t ws_bytes,
                                   void* stream, bs_grid* out) {
    bs_status st = validate_grid_args(H, W, params);
    if (st != BS_OK) return st;
    if (!ref || !ws || !out) return fail(BS_EINVAL, "NULL pointer argument");
    if (((uintptr_t)ws & 255) != 0) return fail(BS_EINVAL, "workspace must be 256-byte aligned");
    if (((uintptr_t)ref & 3) != 0) return fail(BS_EINVAL, "reference must be 4-byte aligned");
    GridImpl g;
    const size_t need = layout_grid(g, H, W, *params, nullptr);
    if (ws_bytes < need)
        return fail(BS_EWORKSPACE, "grid workspace needs " + std::to_string(need) + " bytes");
    layout_grid(g, H, W, *params, ws);
    hipStream_t s = (hipStream_t)stream;

    BS_LAUNCH(s, K_BIST_OTHER, "clear_counts", one_launch<ClearCounts>, dim3(1), dim3(64), 0, s,
              ClearCounts::Args{g.counts}, 0);
    PixelSource ps{ref, H, W, g.P, params->sigma_xy, params->sigma_l, params->sigma_uv,
                   g.lv[0].ncx};
    const int items = params->sigma_xy * params->sigma_xy;
    if (items <= 64) st = launch_level<64, 64>(ps, g, 0, s);
    else if (items <= 256) st = launch_level<256, 256>(ps, g, 0, s);
    else if (items <= 1024) st = launch_level<256, 1024>(ps, g, 0, s);
    else st = launch_level<256, 2048>(ps, g, 0, s);
    if (st != BS_OK) return st;

    const int blocks = grid_blocks(ceil_div(g.vcap, kBlock));
    BS_LAUNCH(s, K_NEIGHBOURS, "neighbour_table", one_launch<NeighbourTable>, dim3(blocks),
              dim3(kBlock), 0, s, neighbour_args(g), 0);
    std::memcpy(out->opaque, &g, sizeof(g));
    return BS_OK;
}

static bs_status check_grid(const bs_grid* grid) {
    if (!grid) return fail(BS_EINVAL, "grid is NULL");
    if (impl(grid)->magic != kGridMagic) return fail(BS_EINVAL, "grid was not built");
    return BS_OK;
}

extern "C" bs_status bs_read_counters(const bs_grid* grid, int32_t* out, int32_t n, void* stream) {
    bs_status st = check_grid(grid);
    if (st != BS_OK) return st;
    if (!out || n < 1 || n > CNT_SIZE) return fail(BS_EINVAL, "bad counter request");
    hipStream_t s = (hipStream_t)stream;
    BS_TRY_HIP(hipMemcpyAsync(out, impl(grid)->counts, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    BS_TRY_HIP(hipStreamSynchronize(s));
    return BS_OK;
}

extern "C" bs_status bs_grid_vertex_count(const bs_grid* grid, int32_t* V, void* stream) {
    if (!V) return fail(BS_EINVAL, "V is NULL");
    return bs_read_counters(grid, V, 1, stream);
}

extern "C" bs_status bs_grid_get_view(const bs_grid* grid, bs_grid_view* v) {
    bs_status st = check_grid(grid);
    if (st != BS_OK) return st;
    if (!v) return fail(BS_EINVAL, "view is NULL");
    const GridImpl& g = *impl(grid);
    std::memset(v, 0, sizeof(*v));
    v->H = g.H;
    v->W = g.W;
    v->P = g.P;
    v->levels = g.levels;
    v->ncells_x = g.lv[0].ncx;
    v->ncells_y = g.lv[0].ncy;
    v->vcap = g.vcap;
    v->counts = g.counts;
    v->bist_residual = g.bist_res;
    v->key = g.lv[0].key;
    v->idx = g.lv[0].item_parent;
    v->m = g.lv[0].mult;
    v->nbr = g.nbr;
    v->nb16 = g.nb16;
    v->nb_packed = g.nb_packed;
    v->pix_ptr = g.lv[0].ptr;
    v->pix_list = g.lv[0].list;
    v->n = g.n64;
    v->nf = g.nf;
    v->nn = g.nn;
    for (int k = 0; k < g.levels; ++k) {
        v->level_cap[k] = g.lv[k].cap;
        v->level_key[k] = g.lv[k].key;
        v->ones[k] = g.lv[k].ones;
        if (k + 1 < g.levels) v->parent[k] = g.lv[k + 1].item_parent;
    }
    return BS_OK;
}

extern "C" const char* bs_status_string(bs_status s) {
    switch (s) {
        case BS_OK: return "ok";
        case BS_EINVAL: return "invalid argument";
        case BS_EWORKSPACE: return "workspace too small";
        case BS_EDEVICE: return "device error";
        case BS_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

extern "C" const char* bs_last_error(void) { return bs::g_last_error.c_str(); }

extern "C" int32_t bs_version(void) { return (1 << 16) | 0; }
