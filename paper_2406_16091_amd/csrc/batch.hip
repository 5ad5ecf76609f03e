// Batched binning + sweep of many independent systems (the paper's pipeline
// of Sec. 2 applied to a set of systems at once).  The systems' particles are
// concatenated; one radix sort orders them by global cell id (system cell
// base + local cell), which keeps every system's particles contiguous and in
// system order, and one work-list sweep covers all systems' tiles.  The whole
// sequence is captured once into a hipGraph per batch layout (systems,
// pointers, options) and replayed afterwards with a single launch.
#include <string.h>

#include <vector>

#include "pair.h"

struct pi_batch {
    pi_ctx *ctx;
    pi_cells *cells;            // concatenated binned system
    SysDev *d_sys;
    KernelConst *d_kcs;
    int32_t cap_sys;
    int32_t nsys;
    std::vector<SysDev> h_sys;
    std::vector<int64_t> cell_base; // host copy, nsys entries
    int tile;
    int64_t total_blocks;
    // graph cache
    std::vector<unsigned char> sig;
    hipGraph_t graph;
    hipGraphExec_t exec;
    hipStream_t graph_stream;
};

extern "C" pi_status pi_batch_create(pi_ctx *ctx, pi_batch **out)
{
    if (!ctx || !out) return PI_EINVAL;
    *out = nullptr;
    pi_batch *b = new (std::nothrow) pi_batch();
    if (!b) return PI_ENOMEM;
    b->ctx = ctx;
    pi_status st = pi_cells_create(ctx, &b->cells);
    if (st != PI_OK) {
        delete b;
        return st;
    }
    *out = b;
    return PI_OK;
}

static void drop_graph(pi_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->sig.clear();
}

extern "C" pi_status pi_batch_destroy(pi_batch *b)
{
    if (!b) return PI_EINVAL;
    (void)hipSetDevice(b->ctx->device);
    drop_graph(b);
    if (b->d_sys) (void)hipFree(b->d_sys);
    if (b->d_kcs) (void)hipFree(b->d_kcs);
    pi_cells_destroy(b->cells);
    delete b;
    return PI_OK;
}

namespace {

void append(std::vector<unsigned char> &v, const void *p, size_t n)
{
    const unsigned char *c = (const unsigned char *)p;
    v.insert(v.end(), c, c + n);
}

pi_status launch_all(pi_batch *b, const float *x, const float *y, const float *z, const float *w, int64_t n_total,
                     int64_t cells_total, const pi_interact_opts &o, float *rho, float *gx, float *gy, float *gz,
                     int32_t *count, pi_invariants *inv, hipStream_t stream)
{
    GridDev g0;
    memset(&g0, 0, sizeof(g0));
    pi_status st = pi_bin_systems(b->ctx, b->cells, x, y, z, w, n_total, cells_total, b->nsys, b->d_sys, g0, stream);
    if (st != PI_OK) return st;
    return pi_sweep_batch(b->ctx, b->cells, b->nsys, b->d_sys, b->d_kcs, b->total_blocks, b->tile, o, rho, gx, gy,
                          gz, count, inv, stream);
}

} // namespace

extern "C" pi_status pi_batch_run(pi_ctx *ctx, pi_batch *b, int32_t nsys, const pi_system_desc *sys, const float *x,
                                  const float *y, const float *z, const float *w, const pi_interact_opts *opts,
                                  float *rho, float *gx, float *gy, float *gz, int32_t *count, pi_invariants *inv,
                                  pi_stream stream_)
{
    if (!ctx || !b || b->ctx != ctx || nsys < 1 || !sys) return PI_EINVAL;
    pi_interact_opts o;
    memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.precision < PI_PREC_COMPENSATED || o.precision > PI_PREC_FP64ACC) return PI_EINVAL;
    if (o.sweep < PI_SWEEP_AUTO || o.sweep > PI_SWEEP_SUBBOX) return PI_EINVAL;
    if (o.order != PI_ORDER_SORTED && o.order != PI_ORDER_ORIGINAL) return PI_EINVAL;
    const bool anyf = rho || gx || gy || gz;
    if (anyf && !(rho && gx && gy && gz)) return PI_EINVAL;
    // systems must be concatenated in order, each on a valid grid
    int64_t n_total = 0, cells_total = 0;
    for (int32_t s = 0; s < nsys; ++s) {
        if (sys[s].offset != n_total || sys[s].n < 0) return PI_EINVAL;
        if (!pi_grid_valid(&sys[s].grid)) return PI_EINVAL;
        n_total += sys[s].n;
        cells_total += (int64_t)sys[s].grid.dims[0] * sys[s].grid.dims[1] * sys[s].grid.dims[2];
        if (n_total >= ((int64_t)1 << 31) || cells_total >= ((int64_t)1 << 31)) return PI_EINVAL;
    }
    if (n_total > 0 && (!x || !y || !z || !w)) return PI_EINVAL;
    hipStream_t stream = (hipStream_t)stream_;
    PI_CHECK_HIP(hipSetDevice(ctx->device));

    // layout signature: systems, pointers, options, stream
    std::vector<unsigned char> sig;
    append(sig, &nsys, sizeof(nsys));
    append(sig, sys, sizeof(pi_system_desc) * (size_t)nsys);
    const void *ptrs[] = {x, y, z, w, rho, gx, gy, gz, count, inv, stream};
    append(sig, ptrs, sizeof(ptrs));
    append(sig, &o, sizeof(o));
    if (b->exec && sig == b->sig) {
        PI_CHECK_HIP(hipGraphLaunch(b->exec, stream));
        return PI_OK;
    }
    drop_graph(b);

    // system table and kernel constants
    const double ppc = cells_total > 0 ? (double)n_total / (double)cells_total : 0.0;
    const int tile = pi_pick_tile(o, ppc);
    if (tile < 0) return PI_EINVAL;
    b->h_sys.assign((size_t)nsys, SysDev());
    b->cell_base.assign((size_t)nsys, 0);
    std::vector<KernelConst> kcs((size_t)nsys);
    int64_t cb = 0;
    for (int32_t s = 0; s < nsys; ++s) {
        SysDev &d = b->h_sys[s];
        memset(&d, 0, sizeof(d));
        const pi_grid &g = sys[s].grid;
        d.first = sys[s].offset;
        d.n = (int32_t)sys[s].n;
        d.cell_base = (int32_t)cb;
        b->cell_base[s] = cb;
        d.g.ox = g.origin[0];
        d.g.oy = g.origin[1];
        d.g.oz = g.origin[2];
        d.g.w = g.cell_w;
        d.g.nx = g.dims[0];
        d.g.ny = g.dims[1];
        d.g.nz = g.dims[2];
        cb += (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
        kcs[s] = pi_make_kernel_const(g.rc, g.cell_w);
    }
    b->tile = tile;
    b->total_blocks = pi_batch_layout(tile, b->h_sys.data(), nsys);
    b->nsys = nsys;
    if (nsys > b->cap_sys) {
        PI_CHECK_HIP(hipStreamSynchronize(stream));
        if (b->d_sys) (void)hipFree(b->d_sys);
        if (b->d_kcs) (void)hipFree(b->d_kcs);
        b->d_sys = nullptr;
        b->d_kcs = nullptr;
        b->cap_sys = 0;
        if (hipMalloc((void **)&b->d_sys, sizeof(SysDev) * (size_t)nsys) != hipSuccess ||
            hipMalloc((void **)&b->d_kcs, sizeof(KernelConst) * (size_t)nsys) != hipSuccess)
            return PI_ENOMEM;
        b->cap_sys = nsys;
    }
    pi_cells *c = b->cells;
    pi_status st = pi_ensure_capacity(c, n_total, cells_total, stream);
    if (st != PI_OK) return st;
    if (b->total_blocks + 64 > c->cap_partials) {
        PI_CHECK_HIP(hipStreamSynchronize(stream));
        if (c->partials) (void)hipFree(c->partials);
        c->partials = nullptr;
        const int64_t need = b->total_blocks + 64;
        if (hipMalloc(&c->partials, (size_t)need * 64) != hipSuccess) {
            c->cap_partials = 0;
            return PI_ENOMEM;
        }
        c->cap_partials = need;
    }
    // the table is read by kernels already queued on `stream` for an older
    // layout; wait for them before overwriting it
    PI_CHECK_HIP(hipStreamSynchronize(stream));
    PI_CHECK_HIP(hipMemcpy(b->d_sys, b->h_sys.data(), sizeof(SysDev) * (size_t)nsys, hipMemcpyHostToDevice));
    PI_CHECK_HIP(hipMemcpy(b->d_kcs, kcs.data(), sizeof(KernelConst) * (size_t)nsys, hipMemcpyHostToDevice));
    c->n = n_total;
    c->n_cells = cells_total;
    memset(&c->grid, 0, sizeof(c->grid));
    c->last_stream = stream;
    c->binned = true;

    if (!stream) // the null stream cannot be captured: launch directly
        return launch_all(b, x, y, z, w, n_total, cells_total, o, rho, gx, gy, gz, count, inv, stream);

    const int was_timing = ctx->timing_on;
    ctx->timing_on = 0; // no event records inside a captured graph
    pi_status lst = PI_OK;
    hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        lst = launch_all(b, x, y, z, w, n_total, cells_total, o, rho, gx, gy, gz, count, inv, stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(stream, &g);
        if (e == hipSuccess && lst == PI_OK) {
            b->graph = g;
            e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    ctx->timing_on = was_timing;
    if (lst != PI_OK) return lst;
    if (e != hipSuccess) {
        drop_graph(b);
        return pi_hip_fail(e, "graph capture");
    }
    b->sig = sig;
    PI_CHECK_HIP(hipGraphLaunch(b->exec, stream));
    return PI_OK;
}

extern "C" pi_status pi_batch_get_view(const pi_batch *b, pi_cells_view *out, int64_t *cell_base, int32_t max_sys)
{
    if (!b || !out) return PI_EINVAL;
    pi_status st = pi_cells_get_view(b->cells, out);
    if (st != PI_OK) return st;
    if (cell_base) {
        if (max_sys < b->nsys) return PI_EINVAL;
        for (int32_t s = 0; s < b->nsys; ++s) cell_base[s] = b->cell_base[s];
    }
    return PI_OK;
}

extern "C" pi_status pi_batch_sync(pi_ctx *ctx, pi_batch *b, pi_stream stream)
{
    if (!b) return PI_EINVAL;
    return pi_sync(ctx, b->cells, stream);
}
