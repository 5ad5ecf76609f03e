// Batched binning + sweep of many independent systems (the paper's pipeline
// of Sec. 2 applied to a set of systems at once).  The systems' particles are
// concatenated; one radix sort orders them by global cell id (system cell
// base + local cell), which keeps every system's particles contiguous and in
// system order.  Each system gets its own sweep organisation (the tuner's
// choice for its size and occupancy, or the caller's explicit one); systems
// with the same organisation share one work-list launch, so a batch costs at
// most one sweep launch per organisation.  The whole sequence is captured
// once into a hipGraph per batch layout (systems, pointers, options) and
// replayed afterwards with a single launch.
#include <string.h>

#include <algorithm>
#include <vector>

#include "pair.h"

// Systems sharing one sweep organisation: entries [first, first + count) of
// the sweep table, their workgroups' partials from record part_base on.
struct BatchGroup {
    int tile;
    int32_t first, count;
    int64_t blocks, part_base;
};

struct pi_batch {
    pi_ctx *ctx;
    pi_cells *cells;            // concatenated binned system
    SysDev *d_sys;              // binning table, caller's order
    SysDev *d_sweep;            // sweep table, grouped by organisation
    KernelConst *d_kcs;         // kernel constants, sweep-table order
    int32_t *d_hint;            // coarse cell-to-system index (binning)
    int64_t cap_hint;
    int32_t cap_sys;
    int32_t nsys;
    std::vector<SysDev> h_sys;
    std::vector<SysDev> h_sweep;
    std::vector<int64_t> cell_base; // host copy, nsys entries
    std::vector<int> tile_of;       // organisation of each system (caller's order)
    std::vector<BatchGroup> groups;
    int64_t total_blocks;
    // graph cache (or, with `direct`, the layout the tables hold)
    std::vector<unsigned char> sig;
    hipGraph_t graph;
    hipGraphExec_t exec;
    bool direct;       // launch the sequence directly instead of capturing it
    bool layout_valid; // direct: the tables hold the layout of `sig`
    hipStream_t graph_stream;
    // side streams and events that fork the sweep groups off the binning
    // and join them back (default priority, created on first use)
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> done;
    hipEvent_t binned;
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
    b->layout_valid = false;
    b->sig.clear();
}

void pi_batch_set_direct(pi_batch *b, bool direct)
{
    drop_graph(b);
    b->direct = direct;
}

pi_cells *pi_batch_cells(pi_batch *b)
{
    return b->cells;
}

extern "C" pi_status pi_batch_destroy(pi_batch *b)
{
    if (!b) return PI_EINVAL;
    (void)hipSetDevice(b->ctx->device);
    drop_graph(b);
    if (b->d_sys) (void)hipFree(b->d_sys);
    if (b->d_sweep) (void)hipFree(b->d_sweep);
    if (b->d_kcs) (void)hipFree(b->d_kcs);
    if (b->d_hint) (void)hipFree(b->d_hint);
    for (hipStream_t st : b->side) (void)hipStreamDestroy(st);
    for (hipEvent_t e : b->done) (void)hipEventDestroy(e);
    if (b->binned) (void)hipEventDestroy(b->binned);
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

// Side streams and events for the fork of launch_all (created outside any
// graph capture).
pi_status ensure_side(pi_batch *b)
{
    const size_t ng = b->groups.size();
    if (!b->binned) PI_CHECK_HIP(hipEventCreateWithFlags(&b->binned, hipEventDisableTiming));
    while (b->side.size() + 1 < ng) {
        hipStream_t sst = nullptr;
        PI_CHECK_HIP(hipStreamCreateWithFlags(&sst, hipStreamNonBlocking));
        b->side.push_back(sst);
        hipEvent_t ev = nullptr;
        PI_CHECK_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        b->done.push_back(ev);
    }
    return PI_OK;
}

pi_status launch_all(pi_batch *b, const float *x, const float *y, const float *z, const float *w, int64_t n_total,
                     int64_t cells_total, const pi_interact_opts &o, float *rho, float *gx, float *gy, float *gz,
                     int32_t *count, pi_invariants *inv, hipStream_t stream)
{
    GridDev g0;
    memset(&g0, 0, sizeof(g0));
    pi_status st = pi_bin_systems(b->ctx, b->cells, x, y, z, w, n_total, cells_total, b->nsys, b->d_sys, b->d_hint,
                                  g0, stream);
    if (st != PI_OK) return st;
    // The groups write disjoint outputs and partial records, so on a real
    // stream they run side by side: group 0 on `stream`, the others on side
    // streams forked after the binning and joined back (small groups then
    // fill the GPU together instead of one after another).  The null
    // stream launches them in order.
    const size_t ng = b->groups.size();
    const bool fork = stream != nullptr && ng > 1;
    if (fork) {
        if (!b->binned || b->side.size() < ng - 1) return PI_EINVAL; // ensure_side() not called
        PI_CHECK_HIP(hipEventRecord(b->binned, stream));
    }
    for (size_t i = 0; i < ng; ++i) {
        const BatchGroup &g = b->groups[i];
        hipStream_t gs = stream;
        if (fork && i > 0) {
            gs = b->side[i - 1];
            PI_CHECK_HIP(hipStreamWaitEvent(gs, b->binned, 0));
        }
        st = pi_sweep_batch(b->ctx, b->cells, g.count, b->d_sweep + g.first, b->d_kcs + g.first, g.blocks,
                            g.part_base, g.tile, o, rho, gx, gy, gz, count, inv, gs);
        if (st != PI_OK) return st;
        if (fork && i > 0) PI_CHECK_HIP(hipEventRecord(b->done[i - 1], gs));
    }
    if (fork)
        for (size_t i = 1; i < ng; ++i) PI_CHECK_HIP(hipStreamWaitEvent(stream, b->done[i - 1], 0));
    return PI_OK;
}

} // namespace

extern "C" pi_status pi_batch_run(pi_ctx *ctx, pi_batch *b, int32_t nsys, const pi_system_desc *sys, const float *x,
                                  const float *y, const float *z, const float *w, const pi_interact_opts *opts,
                                  float *rho, float *gx, float *gy, float *gz, int32_t *count, pi_invariants *inv,
                                  pi_stream stream_)
{
    return pi_batch_run_orgs(ctx, b, nsys, sys, nullptr, x, y, z, w, opts, rho, gx, gy, gz, count, inv, stream_);
}

pi_status pi_batch_run_orgs(pi_ctx *ctx, pi_batch *b, int32_t nsys, const pi_system_desc *sys, const int32_t *org,
                            const float *x, const float *y, const float *z, const float *w,
                            const pi_interact_opts *opts, float *rho, float *gx, float *gy, float *gz,
                            int32_t *count, pi_invariants *inv, pi_stream stream_)
{
    if (!ctx || !b || b->ctx != ctx || nsys < 1 || !sys) return PI_EINVAL;
    pi_interact_opts o;
    memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.precision < PI_PREC_COMPENSATED || o.precision > PI_PREC_FP64ACC) return PI_EINVAL;
    if (o.sweep < PI_SWEEP_AUTO || o.sweep > PI_SWEEP_CELL) return PI_EINVAL;
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
    if (org) append(sig, org, sizeof(int32_t) * (size_t)nsys);
    if (b->exec && sig == b->sig) {
        PI_CHECK_HIP(hipGraphLaunch(b->exec, stream));
        return PI_OK;
    }
    if (b->direct && b->layout_valid && sig == b->sig && stream) {
        pi_status sst = ensure_side(b);
        if (sst != PI_OK) return sst;
        return launch_all(b, x, y, z, w, b->cells->n, b->cells->n_cells, o, rho, gx, gy, gz, count, inv, stream);
    }
    drop_graph(b);

    // binning table (caller's order)
    b->h_sys.assign((size_t)nsys, SysDev());
    b->cell_base.assign((size_t)nsys, 0);
    b->tile_of.assign((size_t)nsys, 0);
    int64_t cb = 0;
    for (int32_t s = 0; s < nsys; ++s) {
        SysDev &d = b->h_sys[s];
        memset(&d, 0, sizeof(d));
        const pi_grid &g = sys[s].grid;
        d.first = sys[s].offset;
        d.n = (int32_t)sys[s].n;
        d.cell_base = (int32_t)cb;
        d.orig = s;
        b->cell_base[s] = cb;
        d.g.ox = g.origin[0];
        d.g.oy = g.origin[1];
        d.g.oz = g.origin[2];
        d.g.w = g.cell_w;
        d.g.nx = g.dims[0];
        d.g.ny = g.dims[1];
        d.g.nz = g.dims[2];
        grid_set_magic(d.g);
        const int64_t nc = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
        cb += nc;
        // organisation of this system
        const double ppc = (double)sys[s].n / (double)nc;
        int t = pi_pick_tile(o, ppc);
        if (t < 0) return PI_EINVAL;
        if (o.sweep == PI_SWEEP_AUTO) t = pi_auto_tile(ctx, o.precision, sys[s].n, ppc);
        if (org && org[s] >= 0) {
            if (!pi_org_valid(org[s])) return PI_EINVAL;
            t = org[s];
        }
        b->tile_of[s] = pi_batch_org(t);
    }
    // sweep table: systems grouped by organisation (caller's order within a
    // group), one work-list layout per group
    std::vector<int32_t> order((size_t)nsys);
    for (int32_t s = 0; s < nsys; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t p, int32_t q) { return b->tile_of[p] < b->tile_of[q]; });
    b->h_sweep.assign((size_t)nsys, SysDev());
    std::vector<KernelConst> kcs((size_t)nsys);
    b->groups.clear();
    int64_t part_base = 0;
    for (int32_t i = 0; i < nsys;) {
        int32_t j = i;
        while (j < nsys && b->tile_of[order[j]] == b->tile_of[order[i]]) {
            b->h_sweep[j] = b->h_sys[order[j]];
            kcs[j] = pi_make_kernel_const(sys[order[j]].grid.rc, sys[order[j]].grid.cell_w);
            ++j;
        }
        BatchGroup g;
        g.tile = b->tile_of[order[i]];
        g.first = i;
        g.count = j - i;
        g.blocks = pi_batch_layout(g.tile, b->h_sweep.data() + i, g.count);
        g.part_base = part_base;
        part_base += g.blocks;
        b->groups.push_back(g);
        i = j;
    }
    b->total_blocks = part_base;
    b->nsys = nsys;
    if (nsys > b->cap_sys) {
        PI_CHECK_HIP(hipStreamSynchronize(stream));
        if (b->d_sys) (void)hipFree(b->d_sys);
        if (b->d_sweep) (void)hipFree(b->d_sweep);
        if (b->d_kcs) (void)hipFree(b->d_kcs);
        b->d_sys = nullptr;
        b->d_sweep = nullptr;
        b->d_kcs = nullptr;
        b->cap_sys = 0;
        if (hipMalloc((void **)&b->d_sys, sizeof(SysDev) * (size_t)nsys) != hipSuccess ||
            hipMalloc((void **)&b->d_sweep, sizeof(SysDev) * (size_t)nsys) != hipSuccess ||
            hipMalloc((void **)&b->d_kcs, sizeof(KernelConst) * (size_t)nsys) != hipSuccess)
            return PI_ENOMEM;
        b->cap_sys = nsys;
    }
    // coarse cell-to-system index: entry k is the system owning global cell
    // k << kCellHintShift (the last system past the end)
    const int64_t nhint = ((cells_total + (1 << kCellHintShift) - 1) >> kCellHintShift) + 1;
    std::vector<int32_t> hint((size_t)nhint);
    for (int64_t k = 0, s = 0; k < nhint; ++k) {
        const int64_t cell = k << kCellHintShift;
        while (s + 1 < nsys && b->cell_base[s + 1] <= cell) ++s;
        hint[k] = (int32_t)s;
    }
    if (nhint > b->cap_hint) {
        PI_CHECK_HIP(hipStreamSynchronize(stream));
        if (b->d_hint) (void)hipFree(b->d_hint);
        b->d_hint = nullptr;
        b->cap_hint = 0;
        if (hipMalloc((void **)&b->d_hint, sizeof(int32_t) * (size_t)nhint) != hipSuccess) return PI_ENOMEM;
        b->cap_hint = nhint;
    }
    pi_cells *c = b->cells;
    pi_status st = pi_ensure_capacity(c, n_total, cells_total, stream);
    if (st != PI_OK) {
        pi_cells_forget(c);
        return st;
    }
    if (b->total_blocks > c->cap_tflag) {
        // one overflow flag per workgroup of the sweep launches
        PI_CHECK_HIP(hipStreamSynchronize(stream));
        if (c->tflag) (void)hipFree(c->tflag);
        c->tflag = nullptr;
        c->cap_tflag = 0;
        if (hipMalloc((void **)&c->tflag, (size_t)b->total_blocks) != hipSuccess) {
            pi_cells_forget(c);
            return PI_ENOMEM;
        }
        c->cap_tflag = b->total_blocks;
    }
    if (b->total_blocks + 64 > c->cap_partials) {
        PI_CHECK_HIP(hipStreamSynchronize(stream));
        if (c->partials) (void)hipFree(c->partials);
        c->partials = nullptr;
        const int64_t need = b->total_blocks + 64;
        if (hipMalloc(&c->partials, (size_t)need * 64) != hipSuccess) {
            c->cap_partials = 0;
            pi_cells_forget(c);
            return PI_ENOMEM;
        }
        c->cap_partials = need;
    }
    // the table is read by kernels already queued on `stream` for an older
    // layout; wait for them before overwriting it
    PI_CHECK_HIP(hipStreamSynchronize(stream));
    PI_CHECK_HIP(hipMemcpy(b->d_sys, b->h_sys.data(), sizeof(SysDev) * (size_t)nsys, hipMemcpyHostToDevice));
    PI_CHECK_HIP(hipMemcpy(b->d_sweep, b->h_sweep.data(), sizeof(SysDev) * (size_t)nsys, hipMemcpyHostToDevice));
    PI_CHECK_HIP(hipMemcpy(b->d_kcs, kcs.data(), sizeof(KernelConst) * (size_t)nsys, hipMemcpyHostToDevice));
    PI_CHECK_HIP(hipMemcpy(b->d_hint, hint.data(), sizeof(int32_t) * (size_t)nhint, hipMemcpyHostToDevice));
    c->n = n_total;
    c->n_cells = cells_total;
    memset(&c->grid, 0, sizeof(c->grid));
    c->last_stream = stream;
    c->binned = true;

    if (!stream) // the null stream cannot be captured: launch directly
        return launch_all(b, x, y, z, w, n_total, cells_total, o, rho, gx, gy, gz, count, inv, stream);
    if (b->direct) {
        pi_status sst = ensure_side(b);
        if (sst != PI_OK) return sst;
        b->sig = sig;
        b->layout_valid = true;
        return launch_all(b, x, y, z, w, n_total, cells_total, o, rho, gx, gy, gz, count, inv, stream);
    }

    pi_status sst = ensure_side(b);
    if (sst != PI_OK) return sst;
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

extern "C" pi_status pi_batch_get_view(pi_batch *b, pi_cells_view *out, int64_t *cell_base, int32_t max_sys)
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
