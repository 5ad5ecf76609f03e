// Request server: many particle systems submitted over time, each swept R
// times with small random displacements between sweeps and its cell list
// kept resident on the GPU.  A scheduler thread admits queued requests as
// soon as a slot is free and the request's HBM footprint fits the budget,
// and queues the request's whole sequence (upload, R x [jitter, re-bin,
// sweep], download) on one of the server's streams; requests on different
// streams overlap on the device, and new ones are admitted while older ones
// are still running.  Results land in pinned host memory owned by the
// server until the ticket is released.
#include <math.h>
#include <string.h>
#include <time.h>

#include <algorithm>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>
#include <vector>

#include "pi_internal.h"

namespace {

double now_s()
{
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

// splitmix64 (Steele, Lea, Flood 2014): a counter-based 64-bit mixer.
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Displace every particle by sigma * N(0,1) per axis (Box-Muller on two
// uniforms drawn from the counter (seed, step, particle, axis)), reflect at
// the faces of the box [o, o + L), L = n w, and round the offset from o down
// to the lattice (if > 0).  The stored coordinate o + v is rounded once more
// when o is large against L; pi_keep_inside then moves it by single ulps
// until the binning's float32 decision keeps it inside the box.

__global__ __launch_bounds__(256) void k_jitter(int32_t n, float *x, float *y, float *z, uint64_t seed,
                                                int32_t step, float sigma, float lattice, float ox, float oy,
                                                float oz, float w, int32_t nx, int32_t ny, int32_t nz)
{
    const int32_t i = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (i >= n) return;
    float *p[3] = {x, y, z};
    const float o[3] = {ox, oy, oz};
    const int32_t dims[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
        const float L = (float)dims[a] * w;
        const uint64_t r = mix64(seed ^ mix64(((uint64_t)step << 40) ^ ((uint64_t)i << 2) ^ (uint64_t)a));
        const float u1 = ((float)(uint32_t)(r >> 40) + 0.5f) * (1.0f / 16777216.0f); // (0, 1)
        const float u2 = (float)(uint32_t)(r & 0xffffffu) * (1.0f / 16777216.0f);     // [0, 1)
        const float g = sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
        float v = p[a][i] - o[a] + sigma * g;
        if (v < 0.0f) v = -v;
        if (v >= L) v = 2.0f * L - v;
        if (lattice > 0.0f) {
            v = floorf(v / lattice) * lattice;
            v = fminf(fmaxf(v, 0.0f), L - lattice);
        } else {
            v = fminf(fmaxf(v, 0.0f), L * (1.0f - 1e-7f));
        }
        p[a][i] = pi_keep_inside(o[a] + v, o[a], w, dims[a]);
    }
}

// The device error word of a binned system back to zero (a fill kernel, not
// a memset, so that the sequence stays capturable).
__global__ void k_clear_err(uint32_t *err)
{
    if (threadIdx.x == 0) err[0] = 0u;
}

} // namespace

namespace {

struct Ticket {
    uint64_t id;
    pi_request req;
    int64_t footprint;
    int32_t status;
    bool done;
    int slot;
    double t_submit, t_start, t_done;
    // pinned host buffer: the inputs (x, y, z, w) on the way in; then the
    // outputs rho, gx, gy, gz, count, x, y, z, the per-sweep invariants and
    // the device error word (pinned_size)
    void *pinned;
    size_t pinned_bytes;
};

struct Slot {
    bool busy = false;
    uint64_t ticket = 0;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    pi_cells *cells = nullptr;
    float *d_in = nullptr;           // x, y, z, w (4 x cap)
    float *d_out = nullptr;          // rho, gx, gy, gz, count (5 x cap)
    pi_invariants *d_inv = nullptr;  // [cap_sweeps]
    int64_t cap = 0, cap_sweeps = 0;
    pi_status launch_status = PI_OK; // error queuing the request (retired with it)
};

} // namespace

struct pi_server {
    pi_ctx *ctx;
    pi_server_opts opts;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Ticket *> tickets;
    std::vector<Slot> slots;
    std::vector<hipStream_t> streams;
    uint64_t next_id = 1;
    int64_t in_use = 0;
    bool stop = false;
    std::thread worker;
    std::vector<std::pair<size_t, void *>> pool;
};

namespace {

int64_t footprint_bytes(int64_t n, int64_t nc, int32_t sweeps)
{
    // device bytes a request holds: inputs 16, outputs 20, binned arrays 24,
    // radix ping-pong 48 and histograms ~1 per particle; counts, offsets and
    // invariant partials per cell; a fixed allowance
    return 109 * n + 8 * nc + 2 * 64 * (nc + n / 64) + 64 * (int64_t)sweeps + (1 << 20);
}

// Pinned host buffer of a request: inputs x, y, z, w on the way in; then
// rho, gx, gy, gz, count, x, y, z (8 arrays of max(n, 1) words), the
// per-sweep invariants and the device error word.
size_t pinned_size(int64_t n, int32_t sweeps)
{
    return (size_t)std::max<int64_t>(1, n) * 32 + sizeof(pi_invariants) * (size_t)sweeps + 256;
}

pi_invariants *pinned_invariants(void *pin, int64_t n)
{
    return (pi_invariants *)((float *)pin + 8 * std::max<int64_t>(n, 1));
}

uint32_t *pinned_err(void *pin, int64_t n, int32_t sweeps)
{
    return (uint32_t *)(pinned_invariants(pin, n) + sweeps);
}

// Pinned buffers come in size classes (powers of two from 1 MiB), so that a
// released buffer serves later requests of any size up to its class: with
// requests of varied sizes, pinning new host memory (slow, milliseconds per
// tens of MB) then stops once the pool holds a buffer per request in flight.
size_t pinned_class(size_t bytes)
{
    size_t c = (size_t)1 << 20;
    while (c < bytes) c <<= 1;
    return c;
}

// The smallest pooled buffer of at least `bytes` (lock held), or nullptr.
void *pool_take(pi_server *s, size_t bytes, size_t *got)
{
    size_t best = s->pool.size();
    for (size_t i = 0; i < s->pool.size(); ++i)
        if (s->pool[i].first >= bytes && (best == s->pool.size() || s->pool[i].first < s->pool[best].first)) best = i;
    if (best == s->pool.size()) return nullptr;
    void *p = s->pool[best].second;
    *got = s->pool[best].first;
    s->pool.erase(s->pool.begin() + (long)best);
    return p;
}

// Device buffers of a slot grow to the next power of two of the particles
// they must hold, so that a stream of varied request sizes stops growing
// them (each growth frees the old buffers, which waits for the device).
pi_status slot_reserve(pi_server *s, Slot &sl, int64_t n, int32_t sweeps)
{
    if (n > sl.cap || !sl.d_in) {
        int64_t cap = 1024;
        while (cap < n) cap <<= 1;
        if (sl.d_in) (void)hipFree(sl.d_in);
        if (sl.d_out) (void)hipFree(sl.d_out);
        sl.d_in = sl.d_out = nullptr;
        if (hipMalloc((void **)&sl.d_in, (size_t)cap * 16) != hipSuccess) return PI_ENOMEM;
        if (hipMalloc((void **)&sl.d_out, (size_t)cap * 20) != hipSuccess) return PI_ENOMEM;
        sl.cap = cap;
    }
    if (sweeps > sl.cap_sweeps || !sl.d_inv) {
        if (sl.d_inv) (void)hipFree(sl.d_inv);
        sl.d_inv = nullptr;
        if (hipMalloc((void **)&sl.d_inv, sizeof(pi_invariants) * (size_t)sweeps) != hipSuccess) return PI_ENOMEM;
        sl.cap_sweeps = sweeps;
    }
    if (!sl.cells) return pi_cells_create(s->ctx, &sl.cells);
    return PI_OK;
}

// Queue a request's whole sequence on its slot's stream (the caller records
// the slot's completion event after it).
pi_status launch_request(pi_server *s, Slot &sl, Ticket *t)
{
    const pi_request &r = t->req;
    const int64_t n = r.n;
    pi_status st = slot_reserve(s, sl, n, r.n_sweeps);
    if (st != PI_OK) return st;
    hipStream_t q = sl.stream;
    const int64_t c = sl.cap;
    float *dx = sl.d_in, *dy = dx + c, *dz = dy + c, *dw = dz + c;
    float *rho = sl.d_out, *gx = rho + c, *gy = gx + c, *gz = gy + c;
    int32_t *cnt = (int32_t *)(gz + c);
    float *h = (float *)t->pinned;
    const size_t b = (size_t)n * 4;
    if (n > 0) {
        PI_CHECK_HIP(hipMemcpyAsync(dx, h, b, hipMemcpyHostToDevice, q));
        PI_CHECK_HIP(hipMemcpyAsync(dy, h + n, b, hipMemcpyHostToDevice, q));
        PI_CHECK_HIP(hipMemcpyAsync(dz, h + 2 * n, b, hipMemcpyHostToDevice, q));
        PI_CHECK_HIP(hipMemcpyAsync(dw, h + 3 * n, b, hipMemcpyHostToDevice, q));
    }
    pi_interact_opts o;
    memset(&o, 0, sizeof(o));
    o.precision = r.precision;
    o.sweep = r.sweep;
    o.order = PI_ORDER_ORIGINAL;
    const pi_grid &g = r.grid;
    if (o.sweep == PI_SWEEP_AUTO) {
        // no timed trials on a request's path: the tuner's cached choice for
        // the request's class if there is one, else the static rule
        const double nc = (double)g.dims[0] * g.dims[1] * g.dims[2];
        pi_tile_opts(pi_auto_tile(s->ctx, r.precision, n, (double)n / nc), &o);
    }
    for (int32_t k = 0; k < r.n_sweeps; ++k) {
        if (k > 0 && r.jitter_sigma > 0.0f && n > 0)
            PI_LAUNCH(s->ctx, "k_jitter", k_jitter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, q, (int32_t)n,
                      dx, dy, dz, r.seed, k, r.jitter_sigma, r.lattice, g.origin[0], g.origin[1], g.origin[2],
                      g.cell_w, g.dims[0], g.dims[1], g.dims[2]);
        st = pi_bin(s->ctx, sl.cells, dx, dy, dz, dw, n, &g, q);
        if (st != PI_OK) return st;
        st = pi_interact(s->ctx, sl.cells, &o, rho, gx, gy, gz, cnt, sl.d_inv + k, q);
        if (st != PI_OK) return st;
    }
    // the inputs were consumed by the first copy; the same pinned buffer
    // receives rho, gx, gy, gz, count, x, y, z, the invariants and the
    // device error word (cleared on the stream for the next request)
    if (n > 0) {
        const void *src[8] = {rho, gx, gy, gz, cnt, dx, dy, dz};
        for (int a = 0; a < 8; ++a)
            PI_CHECK_HIP(hipMemcpyAsync(h + (size_t)a * n, src[a], b, hipMemcpyDeviceToHost, q));
    }
    PI_CHECK_HIP(hipMemcpyAsync(pinned_invariants(t->pinned, n), sl.d_inv,
                                sizeof(pi_invariants) * (size_t)r.n_sweeps, hipMemcpyDeviceToHost, q));
    PI_CHECK_HIP(hipMemcpyAsync(pinned_err(t->pinned, n, r.n_sweeps), sl.cells->d_err, sizeof(uint32_t),
                                hipMemcpyDeviceToHost, q));
    PI_LAUNCH(s->ctx, "k_clear_err", k_clear_err, dim3(1), dim3(64), 0, q, sl.cells->d_err);
    PI_CHECK_HIP(hipGetLastError());
    return PI_OK;
}

// Retire finished requests (lock held; never waits).  A request's status
// comes from its launch, else from the device error word its stream copied
// into the ticket's pinned buffer before the completion event.
bool retire(pi_server *s)
{
    bool changed = false;
    for (Slot &sl : s->slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        Ticket *t = s->tickets[sl.ticket];
        pi_status st = sl.launch_status;
        if (st == PI_OK && q != hipSuccess) st = PI_EDEVICE;
        if (st == PI_OK) {
            const uint32_t err = *(volatile uint32_t *)pinned_err(t->pinned, t->req.n, t->req.n_sweeps);
            if (err) st = (err & PI_DERR_RANGE) ? PI_ERANGE : PI_EDEVICE;
        }
        if (q != hipSuccess && q != hipErrorNotReady) (void)hipGetLastError();
        t->status = st;
        t->t_done = now_s();
        t->done = true;
        s->in_use -= t->footprint;
        sl.busy = false;
        changed = true;
    }
    return changed;
}

// Admit queued requests in arrival order while a slot is free and the
// budget allows (lock held): the slots are marked busy and listed in `go`.
void admit(pi_server *s, std::vector<Slot *> &go)
{
    while (!s->queue.empty()) {
        Ticket *t = s->tickets[s->queue.front()];
        if (s->in_use + t->footprint > s->opts.hbm_budget) break; // first in, first served
        Slot *free_slot = nullptr;
        for (Slot &sl : s->slots)
            if (!sl.busy) {
                free_slot = &sl;
                break;
            }
        if (!free_slot) break;
        s->queue.pop_front();
        free_slot->busy = true;
        free_slot->ticket = t->id;
        free_slot->launch_status = PI_OK;
        t->slot = (int)(free_slot - s->slots.data());
        t->t_start = now_s();
        s->in_use += t->footprint;
        go.push_back(free_slot);
    }
}

// The scheduler thread.  Requests are queued on their slots' streams with
// the lock released (allocations, binning set-up and launches take time;
// pi_submit, pi_poll and pi_wait stay responsive meanwhile).  Only this
// thread marks slots busy or free, so the admitted slots stay its own while
// it launches them.
void worker_loop(pi_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    std::vector<Slot *> go;
    while (!s->stop) {
        bool changed = retire(s);
        go.clear();
        admit(s, go);
        if (!go.empty()) {
            std::vector<Ticket *> ts;
            for (Slot *sl : go) ts.push_back(s->tickets[sl->ticket]);
            lk.unlock();
            for (size_t i = 0; i < go.size(); ++i) {
                Slot &sl = *go[i];
                pi_status st = launch_request(s, sl, ts[i]);
                // the completion event follows whatever was queued, so a
                // failed request is retired only once its stream is idle
                if (hipEventRecord(sl.done, sl.stream) != hipSuccess) {
                    (void)hipGetLastError();
                    (void)hipStreamSynchronize(sl.stream);
                    (void)hipGetLastError();
                    if (st == PI_OK) st = PI_EDEVICE;
                }
                sl.launch_status = st;
            }
            lk.lock();
            changed = true;
        }
        if (changed) s->cv.notify_all();
        bool busy = !s->queue.empty();
        for (const Slot &sl : s->slots) busy = busy || sl.busy;
        // poll in-flight work every 20 us; sleep until a submit otherwise
        if (busy) s->cv.wait_for(lk, std::chrono::microseconds(20));
        else s->cv.wait(lk);
    }
}

} // namespace

extern "C" pi_status pi_server_create(pi_ctx *ctx, const pi_server_opts *opts, pi_server **out)
{
    if (!ctx || !out) return PI_EINVAL;
    *out = nullptr;
    pi_server_opts o;
    memset(&o, 0, sizeof(o));
    o.hbm_budget = (int64_t)64 << 30;
    o.max_slots = 8;
    o.n_streams = 4;
    o.queue_capacity = 1024;
    if (opts) o = *opts;
    if (o.hbm_budget <= 0 || o.max_slots < 1 || o.max_slots > 256 || o.n_streams < 1 || o.n_streams > 16 ||
        o.queue_capacity < 1)
        return PI_EINVAL;
    PI_CHECK_HIP(hipSetDevice(ctx->device));
    pi_server *s = new (std::nothrow) pi_server();
    if (!s) return PI_ENOMEM;
    s->ctx = ctx;
    s->opts = o;
    for (int i = 0; i < o.n_streams; ++i) {
        hipStream_t q = nullptr;
        if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
            delete s;
            return PI_EDEVICE;
        }
        s->streams.push_back(q);
    }
    s->slots.resize((size_t)o.max_slots);
    for (int i = 0; i < o.max_slots; ++i) {
        s->slots[i].stream = s->streams[(size_t)i % s->streams.size()];
        (void)hipEventCreateWithFlags(&s->slots[i].done, hipEventDisableTiming);
    }
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return PI_OK;
}

extern "C" pi_status pi_submit(pi_server *s, const pi_request *r, uint64_t *ticket)
{
    if (!s || !r || !ticket) return PI_EINVAL;
    if (r->n < 0 || r->n >= ((int64_t)1 << 31) || r->n_sweeps < 1 || r->n_sweeps > 1 << 20) return PI_EINVAL;
    if (r->n > 0 && (!r->x || !r->y || !r->z || !r->w)) return PI_EINVAL;
    if (!pi_grid_valid(&r->grid) || !(r->jitter_sigma >= 0.0f) || !(r->lattice >= 0.0f)) return PI_EINVAL;
    if (r->precision < PI_PREC_COMPENSATED || r->precision > PI_PREC_FP64ACC) return PI_EINVAL;
    if (r->sweep < PI_SWEEP_AUTO || r->sweep > PI_SWEEP_CELL) return PI_EINVAL;
    const int64_t nc = (int64_t)r->grid.dims[0] * r->grid.dims[1] * r->grid.dims[2];
    const int64_t fp = footprint_bytes(r->n, nc, r->n_sweeps);
    if (fp > s->opts.hbm_budget) return PI_ENOMEM;
    size_t bytes = pinned_size(r->n, r->n_sweeps);
    void *pin;
    {
        std::lock_guard<std::mutex> g(s->mu);
        if ((int64_t)s->queue.size() >= s->opts.queue_capacity) return PI_EAGAIN;
        pin = pool_take(s, bytes, &bytes);
    }
    if (!pin) {
        // a new buffer, pinned with the lock released
        bytes = pinned_class(bytes);
        if (hipHostMalloc(&pin, bytes, hipHostMallocDefault) != hipSuccess) return PI_ENOMEM;
    }
    // the caller may reuse its arrays as soon as this returns
    float *h = (float *)pin;
    const size_t b = (size_t)r->n * 4;
    if (r->n > 0) {
        memcpy(h, r->x, b);
        memcpy(h + r->n, r->y, b);
        memcpy(h + 2 * r->n, r->z, b);
        memcpy(h + 3 * r->n, r->w, b);
    }
    Ticket *t = new (std::nothrow) Ticket();
    if (!t) return PI_ENOMEM;
    t->req = *r;
    t->req.x = t->req.y = t->req.z = t->req.w = nullptr;
    t->footprint = fp;
    t->status = PI_OK;
    t->done = false;
    t->slot = -1;
    t->pinned = pin;
    t->pinned_bytes = bytes;
    t->t_submit = now_s();
    t->t_start = t->t_done = 0.0;
    {
        std::lock_guard<std::mutex> g(s->mu);
        if ((int64_t)s->queue.size() >= s->opts.queue_capacity) {
            s->pool.emplace_back(bytes, pin);
            delete t;
            return PI_EAGAIN;
        }
        t->id = s->next_id++;
        s->tickets[t->id] = t;
        s->queue.push_back(t->id);
        *ticket = t->id;
    }
    s->cv.notify_all();
    return PI_OK;
}

static void fill_result(const Ticket *t, pi_result *out)
{
    memset(out, 0, sizeof(*out));
    out->done = t->done ? 1 : 0;
    out->status = t->status;
    out->t_submit = t->t_submit;
    out->t_start = t->t_start;
    out->t_done = t->t_done;
    if (!t->done || t->status != PI_OK) return;
    const int64_t n = t->req.n;
    const float *h = (const float *)t->pinned;
    out->n = n;
    out->rho = h;
    out->gx = h + n;
    out->gy = h + 2 * n;
    out->gz = h + 3 * n;
    out->count = (const int32_t *)(h + 4 * n);
    out->x = h + 5 * n;
    out->y = h + 6 * n;
    out->z = h + 7 * n;
    const pi_invariants *inv = pinned_invariants(t->pinned, n);
    out->sweeps = t->req.n_sweeps;
    out->invariants = inv;
    int64_t pairs = 0;
    for (int32_t k = 0; k < t->req.n_sweeps; ++k) pairs += inv[k].pairs;
    out->pairs_total = pairs;
}

extern "C" pi_status pi_poll(pi_server *s, uint64_t ticket, pi_result *out)
{
    if (!s || !out) return PI_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return PI_ENOTFOUND;
    fill_result(it->second, out);
    return PI_OK;
}

extern "C" pi_status pi_wait(pi_server *s, uint64_t ticket, pi_result *out)
{
    if (!s || !out) return PI_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        auto it = s->tickets.find(ticket);
        if (it == s->tickets.end()) return PI_ENOTFOUND;
        if (it->second->done) {
            fill_result(it->second, out);
            return PI_OK;
        }
        s->cv.wait_for(lk, std::chrono::milliseconds(1));
    }
}

extern "C" pi_status pi_release(pi_server *s, uint64_t ticket)
{
    if (!s) return PI_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return PI_ENOTFOUND;
    Ticket *t = it->second;
    if (!t->done) return PI_EAGAIN;
    s->pool.emplace_back(t->pinned_bytes, t->pinned);
    s->tickets.erase(it);
    delete t;
    return PI_OK;
}

extern "C" pi_status pi_server_stats(pi_server *s, pi_server_stats_t *out)
{
    if (!s || !out) return PI_EINVAL;
    std::lock_guard<std::mutex> g(s->mu);
    memset(out, 0, sizeof(*out));
    out->queued = (int32_t)s->queue.size();
    for (const Slot &sl : s->slots) out->running += sl.busy ? 1 : 0;
    out->hbm_in_use = s->in_use;
    return PI_OK;
}

extern "C" pi_status pi_server_destroy(pi_server *s)
{
    if (!s) return PI_EINVAL;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        // finish what was admitted; drop what is still queued
        for (uint64_t id : s->queue) {
            Ticket *t = s->tickets[id];
            t->status = PI_EAGAIN;
            t->done = true;
        }
        s->queue.clear();
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->worker.joinable()) s->worker.join();
    (void)hipSetDevice(s->ctx->device);
    for (Slot &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.cells) pi_cells_destroy(sl.cells);
        if (sl.d_in) (void)hipFree(sl.d_in);
        if (sl.d_out) (void)hipFree(sl.d_out);
        if (sl.d_inv) (void)hipFree(sl.d_inv);
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    for (hipStream_t q : s->streams) (void)hipStreamDestroy(q);
    for (auto &kv : s->tickets) {
        (void)hipHostFree(kv.second->pinned);
        delete kv.second;
    }
    for (auto &p : s->pool) (void)hipHostFree(p.second);
    delete s;
    return PI_OK;
}
