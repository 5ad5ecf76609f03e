// Context, cell-object lifetime, status reporting: the non-kernel part of the
// C ABI declared in include/pi.h.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "pi_internal.h"

// ------------------------------------------------------------- kernel timing

thread_local bool pi_tls_no_timing = false;

struct pi_timing {
    struct Pending {
        int slot;
        hipEvent_t a, b;
    };
    std::mutex mu;
    std::vector<std::string> names;  // first-launch order
    std::vector<int64_t> launches;
    std::vector<double> total_ms;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
    std::string only; // if not empty: time only launches of this name

    int slot_of(const char *name)
    {
        for (size_t i = 0; i < names.size(); ++i)
            if (names[i] == name) return (int)i;
        names.emplace_back(name);
        launches.push_back(0);
        total_ms.push_back(0.0);
        return (int)names.size() - 1;
    }
    hipEvent_t get_event()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    // Fold every pending pair into the totals (waits for the events).
    void drain()
    {
        for (Pending &p : pending) {
            float ms = 0.f;
            if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
                launches[p.slot] += 1;
                total_ms[p.slot] += (double)ms;
            }
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
    }
};

// A launch's event pair lives on the heap between begin and end, and joins
// the pending list only once both events are recorded, so a concurrent drain
// never waits on a half-recorded pair.
void *pi_timer_begin(pi_ctx *ctx, hipStream_t s, const char *name)
{
    pi_timing *t = ctx->timing;
    if (!t) return nullptr;
    pi_timing::Pending *p = new (std::nothrow) pi_timing::Pending();
    if (!p) return nullptr;
    {
        std::lock_guard<std::mutex> g(t->mu);
        if (!t->only.empty() && t->only != name) {
            delete p;
            return nullptr;
        }
        if (t->pending.size() > 4096) t->drain();
        p->slot = t->slot_of(name);
        p->a = t->get_event();
        p->b = t->get_event();
    }
    if (!p->a || !p->b || hipEventRecord(p->a, s) != hipSuccess) {
        std::lock_guard<std::mutex> g(t->mu);
        if (p->a) t->pool.push_back(p->a);
        if (p->b) t->pool.push_back(p->b);
        delete p;
        return nullptr;
    }
    return p;
}

void pi_timer_end(pi_ctx *ctx, hipStream_t s, void *tok)
{
    pi_timing *t = ctx->timing;
    if (!t || !tok) return;
    pi_timing::Pending *p = (pi_timing::Pending *)tok;
    const bool ok = hipEventRecord(p->b, s) == hipSuccess;
    std::lock_guard<std::mutex> g(t->mu);
    if (ok) {
        t->pending.push_back(*p);
    } else {
        t->pool.push_back(p->a);
        t->pool.push_back(p->b);
    }
    delete p;
}

extern "C" pi_status pi_timing_enable(pi_ctx *ctx, int32_t on)
{
    if (!ctx || !ctx->timing) return PI_EINVAL;
    ctx->timing_on = on ? 1 : 0;
    return PI_OK;
}

extern "C" pi_status pi_timing_only(pi_ctx *ctx, const char *name)
{
    if (!ctx || !ctx->timing) return PI_EINVAL;
    if (name && strlen(name) >= sizeof(pi_kernel_time::name)) return PI_EINVAL;
    std::lock_guard<std::mutex> g(ctx->timing->mu);
    ctx->timing->only = name ? name : "";
    return PI_OK;
}

extern "C" pi_status pi_timing_reset(pi_ctx *ctx)
{
    if (!ctx || !ctx->timing) return PI_EINVAL;
    std::lock_guard<std::mutex> g(ctx->timing->mu);
    ctx->timing->drain();
    for (auto &v : ctx->timing->launches) v = 0;
    for (auto &v : ctx->timing->total_ms) v = 0.0;
    return PI_OK;
}

extern "C" pi_status pi_timing_read(pi_ctx *ctx, pi_kernel_time *out, int32_t max, int32_t *n_out)
{
    if (!ctx || !ctx->timing || !n_out || max < 0 || (max > 0 && !out)) return PI_EINVAL;
    PI_CHECK_HIP(hipSetDevice(ctx->device));
    std::lock_guard<std::mutex> g(ctx->timing->mu);
    pi_timing *t = ctx->timing;
    t->drain();
    int32_t k = 0;
    for (size_t i = 0; i < t->names.size() && k < max; ++i) {
        if (t->launches[i] == 0) continue;
        memset(out[k].name, 0, sizeof(out[k].name));
        strncpy(out[k].name, t->names[i].c_str(), sizeof(out[k].name) - 1);
        out[k].launches = t->launches[i];
        out[k].total_ms = t->total_ms[i];
        ++k;
    }
    *n_out = k;
    return PI_OK;
}

pi_status pi_hip_fail(hipError_t e, const char *what)
{
    if (getenv("PI_DEBUG")) fprintf(stderr, "pi: %s failed: %s\n", what, hipGetErrorString(e));
    (void)hipGetLastError(); // clear the sticky-less error state
    return e == hipErrorOutOfMemory ? PI_ENOMEM : PI_EDEVICE;
}

extern "C" const char *pi_status_str(pi_status s)
{
    switch (s) {
    case PI_OK: return "PI_OK";
    case PI_EINVAL: return "PI_EINVAL: invalid argument";
    case PI_ENOMEM: return "PI_ENOMEM: out of device memory or budget";
    case PI_ERANGE: return "PI_ERANGE: particle outside the grid box";
    case PI_EDEVICE: return "PI_EDEVICE: HIP runtime error";
    case PI_EAGAIN: return "PI_EAGAIN: try again";
    case PI_ENOTFOUND: return "PI_ENOTFOUND: unknown handle";
    case PI_ESTATE: return "PI_ESTATE: call out of order";
    case PI_ESTEP: return "PI_ESTEP: a step moved a particle more than half a cell width (displacement cut)";
    default: return "unknown pi_status";
    }
}

extern "C" const char *pi_version(void) { return "pi 0.1 (gfx950)"; }

extern "C" pi_status pi_ctx_create(int32_t device, pi_ctx **out)
{
    if (!out) return PI_EINVAL;
    *out = nullptr;
    int ndev = 0;
    PI_CHECK_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return PI_EINVAL;
    PI_CHECK_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    PI_CHECK_HIP(hipGetDeviceProperties(&prop, device));
    pi_ctx *c = (pi_ctx *)calloc(1, sizeof(pi_ctx));
    if (!c) return PI_ENOMEM;
    c->device = device;
    c->num_cu = prop.multiProcessorCount;
    c->num_xcd = 8;
    c->lds_per_block = prop.sharedMemPerBlock;
    c->timing_on = 0;
    c->timing = new (std::nothrow) pi_timing();
    c->tuner = new (std::nothrow) pi_tuner();
    if (!c->timing || !c->tuner) {
        delete c->timing;
        delete c->tuner;
        free(c);
        return PI_ENOMEM;
    }
    const pi_status ss = pi_noalloc_scratch_setup(device, &c->scratch);
    if (ss != PI_OK) {
        delete c->timing;
        delete c->tuner;
        free(c);
        return ss;
    }
    if (const char *m = getenv("PI_AUTOTUNE")) {
        if (!strcmp(m, "off") || !strcmp(m, "0")) c->tuner->mode = PI_TUNE_STATIC;
    }
    *out = c;
    return PI_OK;
}

extern "C" pi_status pi_ctx_destroy(pi_ctx *ctx)
{
    if (!ctx) return PI_EINVAL;
    if (ctx->timing) {
        {
            std::lock_guard<std::mutex> g(ctx->timing->mu);
            ctx->timing->drain();
            for (hipEvent_t e : ctx->timing->pool) (void)hipEventDestroy(e);
        }
        delete ctx->timing;
    }
    delete ctx->tuner;
    free(ctx);
    return PI_OK;
}

extern "C" pi_status pi_cells_create(pi_ctx *ctx, pi_cells **out)
{
    if (!ctx || !out) return PI_EINVAL;
    pi_cells *c = (pi_cells *)calloc(1, sizeof(pi_cells));
    if (!c) return PI_ENOMEM;
    c->ctx = ctx;
    PI_CHECK_HIP(hipSetDevice(ctx->device));
    if (hipMalloc((void **)&c->d_err, 256) != hipSuccess) { free(c); return PI_ENOMEM; }
    if (hipMemset(c->d_err, 0, 256) != hipSuccess) { (void)hipFree(c->d_err); free(c); return PI_EDEVICE; }
    c->max_per_cell = (int32_t *)((char *)c->d_err + 64);
    *out = c;
    return PI_OK;
}

// Every device buffer of a pi_cells object except the error word, with the
// capacity class it is sized by.
enum BufClass { BUF_N, BUF_CELLS, BUF_CELLS1, BUF_CELLS64, BUF_HIST, BUF_PARTIALS, BUF_RADIX, BUF_SCAN };

struct BufRef {
    void **ptr;
    BufClass cls;
    size_t elem;
};

static int list_buffers(pi_cells *c, BufRef *out)
{
    int k = 0;
    auto add = [&](void **p, BufClass cls, size_t elem) { out[k++] = BufRef{p, cls, elem}; };
    add((void **)&c->counts, BUF_CELLS, 4);
    add((void **)&c->offsets, BUF_CELLS1, 4);
    add((void **)&c->perm, BUF_N, 4);
    add((void **)&c->cell, BUF_N, 4);
    add((void **)&c->xs, BUF_N, 4);
    add((void **)&c->ys, BUF_N, 4);
    add((void **)&c->zs, BUF_N, 4);
    add((void **)&c->ws, BUF_N, 4);
    add((void **)&c->xyzw, BUF_N, 16);
    for (int b = 0; b < 2; ++b) {
        add((void **)&c->skv[b], BUF_N, 8);
        add((void **)&c->sp[b], BUF_N, 16);
    }
    add((void **)&c->hist, BUF_HIST, 4);
    add((void **)&c->partials, BUF_PARTIALS, 64);
    add((void **)&c->tflag, BUF_CELLS64, 1);
    add((void **)&c->dtot, BUF_RADIX, 4);
    if (c->stepping) {
        add((void **)&c->vel, BUF_N, 16);
        add((void **)&c->vel2, BUF_N, 16);
        add((void **)&c->perm2, BUF_N, 4);
        add((void **)&c->cell2, BUF_N, 4);
        add((void **)&c->newcell, BUF_N, 4);
        add((void **)&c->xyzw2, BUF_N, 16);
        add((void **)&c->grho, BUF_N, 4);
        add((void **)&c->ggx, BUF_N, 4);
        add((void **)&c->ggy, BUF_N, 4);
        add((void **)&c->ggz, BUF_N, 4);
        add((void **)&c->offsets2, BUF_CELLS1, 4);
        add((void **)&c->ncnt, BUF_CELLS, 4);
        add((void **)&c->nstart, BUF_CELLS1, 4);
        add((void **)&c->midx, BUF_N, 4);
        add((void **)&c->nlist, BUF_N, 8);
        add((void **)&c->scan, BUF_SCAN, 4);
    }
    return k;
}

static void free_buffers(pi_cells *c)
{
    BufRef b[40];
    const int nb = list_buffers(c, b);
    for (int i = 0; i < nb; ++i) {
        if (*b[i].ptr) (void)hipFree(*b[i].ptr);
        *b[i].ptr = nullptr;
    }
}

extern "C" pi_status pi_cells_destroy(pi_cells *c)
{
    if (!c) return PI_EINVAL;
    (void)hipSetDevice(c->ctx->device);
    if (c->perm || c->counts) (void)hipStreamSynchronize(c->last_stream);
    free_buffers(c);
    if (c->d_err) (void)hipFree(c->d_err);
    free(c);
    return PI_OK;
}

// Capacities grow to the next power of two of what is needed, so that a
// cell object reused for systems of varied sizes (the server's slots) stops
// growing after a few steps; growing frees the old buffers, which waits for
// the device.
static int64_t grow(int64_t need, int64_t have)
{
    if (need <= have) return have;
    int64_t g = 64;
    while (g < need) g <<= 1;
    return g;
}

// Grow the per-particle / per-cell buffers to hold n particles on n_cells
// cells.  Growing waits for the object's previous stream, since the old
// buffers may still be in use there.
pi_status pi_ensure_capacity(pi_cells *c, int64_t n, int64_t n_cells, hipStream_t stream)
{
    (void)stream;
    const bool grow_n = n > c->cap_n || !c->perm;
    const bool grow_c = n_cells > c->cap_cells || !c->counts;
    if (!grow_n && !grow_c) return PI_OK;
    // (buffers from an earlier binning may still be read by work queued on
    // that binning's stream, whether or not it succeeded)
    if (c->perm || c->counts) PI_CHECK_HIP(hipStreamSynchronize(c->last_stream));
    const int64_t cap_n = grow_n ? grow(n < 64 ? 64 : n, c->cap_n) : c->cap_n;
    const int64_t cap_c = grow_c ? grow(n_cells < 64 ? 64 : n_cells, c->cap_cells) : c->cap_cells;
    const int64_t sort_tiles = (cap_n + 4095) / 4096 + 1;
    const int64_t cap_hist = 256 * sort_tiles;
    const int64_t cap_parts = 2 * (cap_c + cap_n / 64) + 64;
    BufRef b[40];
    const int nb = list_buffers(c, b);
    for (int i = 0; i < nb; ++i) {
        int64_t count = 0;
        bool redo = false;
        switch (b[i].cls) {
        case BUF_N: count = cap_n; redo = grow_n; break;
        case BUF_HIST: count = cap_hist; redo = grow_n; break;
        case BUF_CELLS: count = cap_c; redo = grow_c; break;
        case BUF_CELLS1: count = cap_c + 1; redo = grow_c; break;
        case BUF_CELLS64: count = cap_c + 64; redo = grow_c; break;
        case BUF_PARTIALS: count = cap_parts; redo = grow_n || grow_c; break;
        case BUF_RADIX: count = 256; redo = false; break;
        case BUF_SCAN: count = 4 * (cap_c / 1024 + 2); redo = grow_c; break;
        }
        if (!redo && *b[i].ptr) continue;
        if (*b[i].ptr) (void)hipFree(*b[i].ptr);
        *b[i].ptr = nullptr;
        if (hipMalloc(b[i].ptr, (size_t)count * b[i].elem) != hipSuccess) {
            free_buffers(c);
            c->cap_n = c->cap_cells = 0;
            c->cap_tflag = 0;
            return PI_ENOMEM;
        }
        if (b[i].ptr == (void **)&c->tflag) c->cap_tflag = count;
    }
    c->cap_n = cap_n;
    c->cap_cells = cap_c;
    c->ncnt_zeroed = false;
    c->cap_hist = cap_hist;
    c->cap_partials = cap_parts;
    return PI_OK;
}

// The time-stepping buffers are the last ones list_buffers names.
pi_status pi_stepping_enable(pi_cells *c)
{
    if (c->stepping) return PI_OK;
    c->ncnt_zeroed = false;
    BufRef b0[40];
    const int first = list_buffers(c, b0);
    c->stepping = true;
    BufRef b[40];
    const int nb = list_buffers(c, b);
    for (int i = first; i < nb; ++i) {
        int64_t count = 0;
        switch (b[i].cls) {
        case BUF_N: count = c->cap_n; break;
        case BUF_CELLS: count = c->cap_cells; break;
        case BUF_CELLS1: count = c->cap_cells + 1; break;
        default: count = 4 * (c->cap_cells / 1024 + 2); break;
        }
        if (hipMalloc(b[i].ptr, (size_t)std::max<int64_t>(count, 1) * b[i].elem) != hipSuccess) {
            for (int q = first; q < nb; ++q) {
                if (*b[q].ptr) (void)hipFree(*b[q].ptr);
                *b[q].ptr = nullptr;
            }
            c->stepping = false;
            return PI_ENOMEM;
        }
    }
    return PI_OK;
}

void pi_cells_forget(pi_cells *c)
{
    c->vel_valid = false;
    c->stepped = false;
    c->binned = false;
    c->n = 0;
    c->n_cells = 0;
    c->soa_stale = false;
}

bool pi_cells_ready(const pi_cells *c)
{
    return c->binned && c->counts && c->offsets && c->perm && c->cell && c->xyzw && c->partials &&
           c->cap_n >= c->n && c->cap_cells >= c->n_cells;
}

extern "C" pi_status pi_cells_get_view(pi_cells *c, pi_cells_view *v)
{
    if (!c || !v) return PI_EINVAL;
    if (!pi_cells_ready(c) || !c->xs) return PI_ESTATE;
    const pi_status st = pi_split_records(c->ctx, c);
    if (st != PI_OK) return st;
    v->n = c->n;
    v->n_cells = c->n_cells;
    v->grid = c->grid;
    v->counts = c->counts;
    v->offsets = c->offsets;
    v->perm = c->perm;
    v->cell = c->cell;
    v->xs = c->xs;
    v->ys = c->ys;
    v->zs = c->zs;
    v->ws = c->ws;
    v->max_per_cell = c->max_per_cell;
    return PI_OK;
}

extern "C" pi_status pi_sync(pi_ctx *ctx, pi_cells *cells, pi_stream stream)
{
    if (!ctx) return PI_EINVAL;
    PI_CHECK_HIP(hipSetDevice(ctx->device));
    PI_CHECK_HIP(hipStreamSynchronize((hipStream_t)stream));
    if (!cells) return PI_OK;
    uint32_t err = 0;
    PI_CHECK_HIP(hipMemcpy(&err, cells->d_err, 4, hipMemcpyDeviceToHost));
    if (err) {
        uint32_t zero = 0;
        PI_CHECK_HIP(hipMemcpy(cells->d_err, &zero, 4, hipMemcpyHostToDevice));
        if (err & PI_DERR_RANGE) return PI_ERANGE;
        if (err & PI_DERR_STEP) return PI_ESTEP;
        return PI_EDEVICE;
    }
    return PI_OK;
}
