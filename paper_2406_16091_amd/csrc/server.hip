// Request server: many particle systems submitted over time, each swept R
// times with small random displacements between sweeps and its cell list
// kept resident on the GPU for the whole request.  A scheduler thread admits
// queued requests first-in first-out while the request cap and the HBM
// budget allow, and runs the requests it admits together as one batch on a
// free lane (a stream with its own buffers): one upload per request, then R
// times [batched displacement, batched re-binning and sweep of every system
// at once (pi_batch_run)], then one download per request.  A request of
// 2^18 particles or more, which fills the GPU by itself, or one admitted
// alone takes the plain single-system path (pi_bin, pi_interact) instead,
// which gives the same results.  Lanes run side by
// side, so requests that arrive while a batch is on the GPU start on
// another lane as soon as one is free.  Results land in pinned host memory
// owned by the server until the ticket is released.
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

// One request of a batch, as the device kernels see it.
struct BatchReq {
    int64_t off;      // first particle in the concatenated arrays
    int64_t in_byte;  // its inputs (x, y, z, w of n each) in the upload area
    int64_t out_byte; // its results in the download area
    int32_t n;
    int32_t pad0;
    float sigma, lattice;
    float ox, oy, oz, w;
    int32_t nx, ny, nz;
    int32_t pad1;
    uint64_t seed;
};

// The request owning concatenated particle i (requests in offset order).
__device__ __forceinline__ int req_of(const BatchReq *__restrict__ t, int32_t m, int64_t i)
{
    int lo = 0, hi = m; // t[lo].off <= i < t[hi].off
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (t[mid].off <= i) lo = mid; else hi = mid;
    }
    return lo;
}

// Upload area (each request's x, y, z, w back to back) to the concatenated
// arrays x, y, z, w (cap entries apart).
__global__ __launch_bounds__(256) void k_unpack_inputs(int64_t ntot, const BatchReq *__restrict__ t, int32_t m,
                                                       const char *__restrict__ up, float *__restrict__ xyzw,
                                                       int64_t cap)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= ntot) return;
    const BatchReq &r = t[req_of(t, m, i)];
    const float *src = reinterpret_cast<const float *>(up + r.in_byte);
    const int64_t j = i - r.off;
    xyzw[i] = src[j];
    xyzw[cap + i] = src[r.n + j];
    xyzw[2 * cap + i] = src[2 * (int64_t)r.n + j];
    xyzw[3 * cap + i] = src[3 * (int64_t)r.n + j];
}

// Displace every particle by sigma * N(0,1) per axis (Box-Muller on two
// uniforms drawn from the counter (seed, step, particle, axis), the particle
// counted within its own request), reflect at the faces of the box [o, o +
// L), L = n w, and round the offset from o down to the lattice (if > 0).  The
// stored coordinate o + v is rounded once more when o is large against L;
// pi_keep_inside then moves it by single ulps until the binning's float32
// decision keeps it inside the box.
__global__ __launch_bounds__(256) void k_jitter(int64_t ntot, const BatchReq *__restrict__ t, int32_t m,
                                                float *__restrict__ xyzw, int64_t cap, int32_t step)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= ntot) return;
    const BatchReq &r = t[req_of(t, m, i)];
    if (!(r.sigma > 0.0f)) return;
    const uint64_t li = (uint64_t)(i - r.off);
    const float o[3] = {r.ox, r.oy, r.oz};
    const int32_t dims[3] = {r.nx, r.ny, r.nz};
    for (int a = 0; a < 3; ++a) {
        float *p = xyzw + (int64_t)a * cap + i;
        const float L = (float)dims[a] * r.w;
        const uint64_t h = mix64(r.seed ^ mix64(((uint64_t)step << 40) ^ (li << 2) ^ (uint64_t)a));
        const float u1 = ((float)(uint32_t)(h >> 40) + 0.5f) * (1.0f / 16777216.0f); // (0, 1)
        const float u2 = (float)(uint32_t)(h & 0xffffffu) * (1.0f / 16777216.0f);     // [0, 1)
        const float g = sqrtf(-2.0f * logf(u1)) * cospif(2.0f * u2);
        float v = *p - o[a] + r.sigma * g;
        if (v < 0.0f) v = -v;
        if (v >= L) v = 2.0f * L - v;
        if (r.lattice > 0.0f) {
            v = floorf(v / r.lattice) * r.lattice;
            v = fminf(fmaxf(v, 0.0f), L - r.lattice);
        } else {
            v = fminf(fmaxf(v, 0.0f), L * (1.0f - 1e-7f));
        }
        *p = pi_keep_inside(o[a] + v, o[a], r.w, dims[a]);
    }
}

// Results to the download area: per request rho, gx, gy, gz, count, x, y, z
// (max(n, 1) entries each), then its R invariants.
__global__ __launch_bounds__(256) void k_pack_results(int64_t ntot, const BatchReq *__restrict__ t, int32_t m,
                                                      const float *__restrict__ out5,
                                                      const float *__restrict__ xyzw, int64_t cap,
                                                      char *__restrict__ down)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= ntot) return;
    const BatchReq &r = t[req_of(t, m, i)];
    float *dst = reinterpret_cast<float *>(down + r.out_byte);
    const int64_t j = i - r.off, nn = r.n > 0 ? r.n : 1;
#pragma unroll
    for (int a = 0; a < 5; ++a) dst[a * nn + j] = out5[a * cap + i];
#pragma unroll
    for (int a = 0; a < 3; ++a) dst[(5 + a) * nn + j] = xyzw[a * cap + i];
}

// The device error word of a binned system back to zero (a fill kernel, not
// a memset, so that the sequence stays capturable).
__global__ void k_clear_err(uint32_t *err)
{
    if (threadIdx.x == 0) err[0] = 0u;
}

// hist[k * m + q] (sweep k of request q) to request q's download block.
__global__ __launch_bounds__(256) void k_pack_invariants(const BatchReq *__restrict__ t, int32_t m, int32_t sweeps,
                                                         const pi_invariants *__restrict__ hist,
                                                         char *__restrict__ down)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)m * sweeps) return;
    const int q = (int)(e / sweeps), k = (int)(e % sweeps);
    const BatchReq &r = t[q];
    const int64_t nn = r.n > 0 ? r.n : 1;
    pi_invariants *dst = reinterpret_cast<pi_invariants *>(down + r.out_byte + 32 * nn);
    dst[k] = hist[(int64_t)k * m + q];
}

} // namespace

namespace {

struct Ticket {
    uint64_t id;
    pi_request req;
    int64_t footprint;
    int32_t status;
    bool done;
    int lane;
    int32_t max_ppc; // the most particles in one cell (-1: not counted)
    double t_submit, t_start, t_done;
    // pinned host buffer: the inputs (x, y, z, w) on the way in; then the
    // outputs rho, gx, gy, gz, count, x, y, z (max(n, 1) entries each) and
    // the per-sweep invariants (pinned_size)
    void *pinned;
    size_t pinned_bytes;
};

// A stream with its own buffers, running one batch of requests at a time.
struct Lane {
    bool busy = false;
    std::vector<uint64_t> tickets;   // the batch in flight
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    pi_batch *batch = nullptr;       // batches of two or more requests
    pi_cells *cells = nullptr;       // a request alone
    bool alone = false;              // the batch in flight is one request
    char *d_up = nullptr;            // upload area (16 bytes per particle)
    char *d_down = nullptr;          // download area
    float *d_xyzw = nullptr;         // x, y, z, w (4 x cap)
    float *d_out = nullptr;          // rho, gx, gy, gz, count (5 x cap)
    pi_invariants *d_inv = nullptr;  // one sweep's invariants [cap_req]
    pi_invariants *d_hist = nullptr; // every sweep's [cap_hist]
    BatchReq *d_req = nullptr;
    BatchReq *h_req = nullptr;       // pinned staging of the request table
    uint32_t *h_err = nullptr;       // pinned copy of the batch's device error word
    int64_t cap = 0, cap_up = 0, cap_down = 0, cap_req = 0, cap_hist = 0;
    pi_status launch_status = PI_OK; // error queuing the batch (retired with it)
};

} // namespace

struct pi_server {
    pi_ctx *ctx;
    pi_server_opts opts;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Ticket *> tickets;
    std::vector<Lane> lanes;
    uint64_t next_id = 1;
    int64_t in_use = 0;
    int32_t in_flight = 0;
    bool stop = false;
    std::thread worker;
    std::vector<std::pair<size_t, void *>> pool;
};

namespace {

int64_t footprint_bytes(int64_t n, int64_t nc, int32_t sweeps)
{
    // device bytes a request holds: upload 16, inputs 16, outputs 20,
    // download 32, binned arrays 24, radix ping-pong 48 and histograms ~1
    // per particle; counts, offsets and invariant partials per cell; per
    // sweep invariants; a fixed allowance
    return 157 * n + 8 * nc + 2 * 64 * (nc + n / 64) + 2 * 64 * (int64_t)sweeps + (1 << 20);
}

// Pinned host buffer of a request: inputs x, y, z, w on the way in; then
// rho, gx, gy, gz, count, x, y, z (8 arrays of max(n, 1) words) and the
// per-sweep invariants.
size_t pinned_size(int64_t n, int32_t sweeps)
{
    return (size_t)std::max<int64_t>(1, n) * 32 + sizeof(pi_invariants) * (size_t)sweeps + 256;
}

size_t result_bytes(int64_t n, int32_t sweeps)
{
    return (size_t)std::max<int64_t>(1, n) * 32 + sizeof(pi_invariants) * (size_t)sweeps;
}

pi_invariants *pinned_invariants(void *pin, int64_t n)
{
    return (pi_invariants *)((float *)pin + 8 * std::max<int64_t>(n, 1));
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

int64_t grow_pow2(int64_t need, int64_t floor_)
{
    int64_t c = floor_;
    while (c < need) c <<= 1;
    return c;
}

// Device buffers of a lane grow to the next power of two of what a batch
// needs (each growth frees the old buffers, which waits for the device, so
// a stream of varied batches soon stops growing them).  The lane is idle.
pi_status lane_reserve(Lane &ln, int64_t n, int64_t down, int32_t m, int64_t hist)
{
    auto realloc_ = [](void **p, size_t bytes) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
        return hipMalloc(p, bytes) == hipSuccess;
    };
    if (n > ln.cap || !ln.d_xyzw) {
        const int64_t cap = grow_pow2(n, 1024);
        if (!realloc_((void **)&ln.d_xyzw, (size_t)cap * 16) || !realloc_((void **)&ln.d_out, (size_t)cap * 20) ||
            !realloc_((void **)&ln.d_up, (size_t)cap * 16)) {
            ln.cap = 0;
            return PI_ENOMEM;
        }
        ln.cap = ln.cap_up = cap;
    }
    if (down > ln.cap_down || !ln.d_down) {
        const int64_t cap = grow_pow2(down, 1 << 16);
        if (!realloc_((void **)&ln.d_down, (size_t)cap)) {
            ln.cap_down = 0;
            return PI_ENOMEM;
        }
        ln.cap_down = cap;
    }
    if (!ln.h_err) {
        if (hipHostMalloc((void **)&ln.h_err, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) return PI_ENOMEM;
        *ln.h_err = 0;
    }
    if (m > ln.cap_req || !ln.d_req) {
        const int64_t cap = grow_pow2(m, 64);
        if (!realloc_((void **)&ln.d_req, sizeof(BatchReq) * (size_t)cap) ||
            !realloc_((void **)&ln.d_inv, sizeof(pi_invariants) * (size_t)cap)) {
            ln.cap_req = 0;
            return PI_ENOMEM;
        }
        if (ln.h_req) (void)hipHostFree(ln.h_req);
        ln.h_req = nullptr;
        if (hipHostMalloc((void **)&ln.h_req, sizeof(BatchReq) * (size_t)cap, hipHostMallocDefault) != hipSuccess) {
            ln.cap_req = 0;
            return PI_ENOMEM;
        }
        ln.cap_req = cap;
    }
    if (hist > ln.cap_hist || !ln.d_hist) {
        const int64_t cap = grow_pow2(hist, 64);
        if (!realloc_((void **)&ln.d_hist, sizeof(pi_invariants) * (size_t)cap)) {
            ln.cap_hist = 0;
            return PI_ENOMEM;
        }
        ln.cap_hist = cap;
    }
    return PI_OK;
}

bool clustered(const Ticket *t);

// Queue a batch of requests (same sweep count and options) on an idle lane;
// the caller records the lane's completion event after it.
pi_status launch_batch(pi_server *s, Lane &ln, const std::vector<Ticket *> &ts)
{
    const int32_t m = (int32_t)ts.size();
    const pi_request &r0 = ts[0]->req;
    const int32_t R = r0.n_sweeps;
    int64_t ntot = 0, down = 0;
    for (const Ticket *t : ts) {
        ntot += t->req.n;
        down += (int64_t)result_bytes(t->req.n, R);
    }
    // a request alone runs the plain single-system path (pi_bin, pi_interact)
    ln.alone = m == 1;
    if (ln.alone && !ln.cells) {
        pi_status st = pi_cells_create(s->ctx, &ln.cells);
        if (st != PI_OK) return st;
    }
    if (!ln.alone && !ln.batch) {
        pi_status st = pi_batch_create(s->ctx, &ln.batch);
        if (st != PI_OK) return st;
        // a batch's layout serves its own sweeps only: launched directly,
        // no graph to capture per batch
        pi_batch_set_direct(ln.batch, true);
    }
    pi_status st = lane_reserve(ln, ntot, down, m, (int64_t)m * R);
    if (st != PI_OK) return st;
    hipStream_t q = ln.stream;
    std::vector<pi_system_desc> sys((size_t)m);
    int64_t off = 0, ob = 0;
    for (int32_t i = 0; i < m; ++i) {
        const pi_request &r = ts[i]->req;
        BatchReq &b = ln.h_req[i];
        memset(&b, 0, sizeof(b));
        b.off = off;
        b.in_byte = 16 * off;
        b.out_byte = ob;
        b.n = (int32_t)r.n;
        b.sigma = r.jitter_sigma;
        b.lattice = r.lattice;
        b.ox = r.grid.origin[0];
        b.oy = r.grid.origin[1];
        b.oz = r.grid.origin[2];
        b.w = r.grid.cell_w;
        b.nx = r.grid.dims[0];
        b.ny = r.grid.dims[1];
        b.nz = r.grid.dims[2];
        b.seed = r.seed;
        sys[i].offset = off;
        sys[i].n = r.n;
        sys[i].grid = r.grid;
        off += r.n;
        ob += (int64_t)result_bytes(r.n, R);
    }
    PI_CHECK_HIP(hipMemcpyAsync(ln.d_req, ln.h_req, sizeof(BatchReq) * (size_t)m, hipMemcpyHostToDevice, q));
    for (int32_t i = 0; i < m; ++i)
        if (ts[i]->req.n > 0)
            PI_CHECK_HIP(hipMemcpyAsync(ln.d_up + ln.h_req[i].in_byte, ts[i]->pinned, (size_t)ts[i]->req.n * 16,
                                        hipMemcpyHostToDevice, q));
    const int64_t cap = ln.cap;
    float *x = ln.d_xyzw, *y = x + cap, *z = y + cap, *w = z + cap;
    float *rho = ln.d_out, *gx = rho + cap, *gy = gx + cap, *gz = gy + cap;
    int32_t *cnt = (int32_t *)(gz + cap);
    const unsigned nb = (unsigned)((ntot + 255) / 256);
    if (ntot > 0)
        PI_LAUNCH(s->ctx, "k_unpack_inputs", k_unpack_inputs, dim3(nb), dim3(256), 0, q, ntot,
                  (const BatchReq *)ln.d_req, m, (const char *)ln.d_up, ln.d_xyzw, cap);
    pi_interact_opts o;
    memset(&o, 0, sizeof(o));
    o.precision = r0.precision;
    o.sweep = r0.sweep;
    o.order = PI_ORDER_ORIGINAL;
    // AUTO never runs timed trials on a request's path: the tuner's cached
    // choice for the request's class if there is one, else the static rule;
    // a request whose densest cell would overflow the LDS tilings takes the
    // no-LDS walk (the same choice alone and in a batch)
    pi_interact_opts o1 = o;
    if (ln.alone && o1.sweep == PI_SWEEP_AUTO) {
        const double nc = (double)r0.grid.dims[0] * r0.grid.dims[1] * r0.grid.dims[2];
        pi_tile_opts(clustered(ts[0]) ? 0 : pi_auto_tile(s->ctx, r0.precision, r0.n, (double)r0.n / nc), &o1);
    }
    std::vector<int32_t> org((size_t)m, -1);
    if (o.sweep == PI_SWEEP_AUTO)
        for (int32_t i = 0; i < m; ++i) org[i] = clustered(ts[i]) ? 0 : -1;
    bool jitter = false;
    for (const Ticket *t : ts) jitter = jitter || t->req.jitter_sigma > 0.0f;
    for (int32_t k = 0; k < R; ++k) {
        if (k > 0 && jitter && ntot > 0)
            PI_LAUNCH(s->ctx, "k_jitter", k_jitter, dim3(nb), dim3(256), 0, q, ntot, (const BatchReq *)ln.d_req, m,
                      ln.d_xyzw, cap, k);
        if (ln.alone) {
            st = pi_bin(s->ctx, ln.cells, x, y, z, w, ntot, &r0.grid, (pi_stream)q);
            if (st != PI_OK) return st;
            st = pi_interact(s->ctx, ln.cells, &o1, rho, gx, gy, gz, cnt, ln.d_inv, (pi_stream)q);
        } else {
            // (AUTO: the tuner's cached choice per system, else the static
            // rule; a batch never runs timed trials)
            st = pi_batch_run_orgs(s->ctx, ln.batch, m, sys.data(), org.data(), x, y, z, w, &o, rho, gx, gy, gz,
                                   cnt, ln.d_inv, (pi_stream)q);
        }
        if (st != PI_OK) return st;
        PI_CHECK_HIP(hipMemcpyAsync(ln.d_hist + (int64_t)k * m, ln.d_inv, sizeof(pi_invariants) * (size_t)m,
                                    hipMemcpyDeviceToDevice, q));
    }
    if (ntot > 0)
        PI_LAUNCH(s->ctx, "k_pack_results", k_pack_results, dim3(nb), dim3(256), 0, q, ntot,
                  (const BatchReq *)ln.d_req, m, (const float *)ln.d_out, (const float *)ln.d_xyzw, cap, ln.d_down);
    const int64_t ninv = (int64_t)m * R;
    PI_LAUNCH(s->ctx, "k_pack_invariants", k_pack_invariants, dim3((unsigned)((ninv + 255) / 256)), dim3(256), 0, q,
              (const BatchReq *)ln.d_req, m, R, (const pi_invariants *)ln.d_hist, ln.d_down);
    for (int32_t i = 0; i < m; ++i)
        PI_CHECK_HIP(hipMemcpyAsync(ts[i]->pinned, ln.d_down + ln.h_req[i].out_byte, result_bytes(ts[i]->req.n, R),
                                    hipMemcpyDeviceToHost, q));
    // the device error word, copied before the completion event and cleared
    // on the stream, so that retiring the batch never waits on the device
    uint32_t *d_err = (ln.alone ? ln.cells : pi_batch_cells(ln.batch))->d_err;
    PI_CHECK_HIP(hipMemcpyAsync(ln.h_err, d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, q));
    PI_LAUNCH(s->ctx, "k_clear_err", k_clear_err, dim3(1), dim3(64), 0, q, d_err);
    PI_CHECK_HIP(hipGetLastError());
    return PI_OK;
}

// Retire finished batches (lock held; never waits on the device).  A
// request's status comes from its batch's launch, else from the copy of the
// batch's device error word that its stream made before the completion
// event (a range error cannot come from a request that pi_submit accepted,
// since it checks every position with the binning's own decision and the
// displacements keep particles inside).
bool retire(pi_server *s)
{
    bool changed = false;
    for (Lane &ln : s->lanes) {
        if (!ln.busy) continue;
        const hipError_t q = hipEventQuery(ln.done);
        if (q == hipErrorNotReady) continue;
        pi_status st = ln.launch_status;
        if (st == PI_OK && q != hipSuccess) st = PI_EDEVICE;
        if (q != hipSuccess && q != hipErrorNotReady) (void)hipGetLastError();
        if (st == PI_OK) {
            const uint32_t err = *(volatile uint32_t *)ln.h_err;
            if (err) st = (err & PI_DERR_RANGE) ? PI_ERANGE : PI_EDEVICE;
        }
        const double t = now_s();
        for (uint64_t id : ln.tickets) {
            Ticket *tk = s->tickets[id];
            tk->status = st;
            tk->t_done = t;
            tk->done = true;
            s->in_use -= tk->footprint;
            --s->in_flight;
        }
        ln.tickets.clear();
        ln.busy = false;
        changed = true;
    }
    return changed;
}

// Requests of at least this many particles fill the GPU on their own and
// run alone (the plain single-system path); smaller ones share batches.
constexpr int64_t kAloneN = (int64_t)1 << 18;

// Requests that may share a batch (same sweep count and options, both
// small).
bool same_batch(const pi_request &a, const pi_request &b)
{
    return a.n < kAloneN && b.n < kAloneN && a.n_sweeps == b.n_sweeps && a.precision == b.precision &&
           a.sweep == b.sweep;
}

// Admit queued requests in arrival order onto free lanes while the request
// cap and the budget allow (lock held): each free lane takes the longest
// run at the head of the queue that may share a batch; the lanes are marked
// busy and listed in `go`.
void admit(pi_server *s, std::vector<Lane *> &go)
{
    for (Lane &ln : s->lanes) {
        if (ln.busy) continue;
        int64_t ntot = 0, ctot = 0;
        while (!s->queue.empty() && s->in_flight < s->opts.max_slots) {
            Ticket *t = s->tickets[s->queue.front()];
            if (s->in_use + t->footprint > s->opts.hbm_budget) break; // first in, first served
            if (!ln.tickets.empty() && !same_batch(s->tickets[ln.tickets[0]]->req, t->req)) break;
            const int64_t nc = (int64_t)t->req.grid.dims[0] * t->req.grid.dims[1] * t->req.grid.dims[2];
            if (!ln.tickets.empty() && (ntot + t->req.n >= ((int64_t)1 << 30) || ctot + nc >= ((int64_t)1 << 30)))
                break;
            s->queue.pop_front();
            ln.tickets.push_back(t->id);
            t->lane = (int)(&ln - s->lanes.data());
            t->t_start = now_s();
            s->in_use += t->footprint;
            ++s->in_flight;
            ntot += t->req.n;
            ctot += nc;
        }
        if (ln.tickets.empty()) break;
        ln.busy = true;
        ln.launch_status = PI_OK;
        go.push_back(&ln);
    }
}

// The scheduler thread.  Batches are queued on their lanes' streams with the
// lock released (allocations, binning set-up and launches take time;
// pi_submit, pi_poll and pi_wait stay responsive meanwhile).  Only this
// thread marks lanes busy or free, so the admitted lanes stay its own while
// it launches them.
void worker_loop(pi_server *s)
{
    (void)hipSetDevice(s->ctx->device);
    std::unique_lock<std::mutex> lk(s->mu);
    std::vector<Lane *> go;
    while (!s->stop) {
        bool changed = retire(s);
        go.clear();
        admit(s, go);
        if (!go.empty()) {
            std::vector<std::vector<Ticket *>> ts(go.size());
            for (size_t i = 0; i < go.size(); ++i)
                for (uint64_t id : go[i]->tickets) ts[i].push_back(s->tickets[id]);
            lk.unlock();
            for (size_t i = 0; i < go.size(); ++i) {
                Lane &ln = *go[i];
                pi_status st = launch_batch(s, ln, ts[i]);
                // the completion event follows whatever was queued, so a
                // failed batch is retired only once its stream is idle
                if (hipEventRecord(ln.done, ln.stream) != hipSuccess) {
                    (void)hipGetLastError();
                    (void)hipStreamSynchronize(ln.stream);
                    (void)hipGetLastError();
                    if (st == PI_OK) st = PI_EDEVICE;
                }
                ln.launch_status = st;
            }
            lk.lock();
            changed = true;
        }
        if (changed) s->cv.notify_all();
        bool busy = !s->queue.empty();
        for (const Lane &ln : s->lanes) busy = busy || ln.busy;
        // poll in-flight work every 20 us; sleep until a submit otherwise
        if (busy) s->cv.wait_for(lk, std::chrono::microseconds(20));
        else s->cv.wait(lk);
    }
}

// Whether every particle of a request lies in its box by the binning's own
// float32 decision; with `occupancy`, also the most particles in one cell
// (counted when the grid has at most 8n + 4096 cells, else -1).
bool inside_box(const pi_request &r, bool occupancy, int32_t *max_ppc)
{
    const pi_grid &g = r.grid;
    const int64_t nc = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
    std::vector<int32_t> cnt;
    if (occupancy && nc <= 8 * r.n + 4096) cnt.assign((size_t)nc, 0);
    int32_t most = 0;
    for (int64_t i = 0; i < r.n; ++i) {
        int32_t ix, iy, iz;
        if (!axis_index(r.x[i], g.origin[0], g.cell_w, g.dims[0], ix) ||
            !axis_index(r.y[i], g.origin[1], g.cell_w, g.dims[1], iy) ||
            !axis_index(r.z[i], g.origin[2], g.cell_w, g.dims[2], iz))
            return false;
        if (!cnt.empty()) most = std::max(most, ++cnt[(size_t)(ix + (int64_t)g.dims[0] * (iy + (int64_t)g.dims[1] * iz))]);
    }
    *max_ppc = cnt.empty() ? -1 : most;
    return true;
}

// Whether a request's densest cell makes the LDS tilings overflow there, so
// that AUTO should take the no-LDS walk: its most-occupied cell holds more
// than four times the mean plus eight (the clustered inputs; the static rule
// reads only the mean).
bool clustered(const Ticket *t)
{
    const pi_grid &g = t->req.grid;
    const double nc = (double)g.dims[0] * g.dims[1] * g.dims[2];
    return t->max_ppc >= 0 && (double)t->max_ppc > 4.0 * (double)t->req.n / nc + 8.0;
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
    if (o.hbm_budget <= 0 || o.max_slots < 1 || o.max_slots > 4096 || o.n_streams < 1 || o.n_streams > 16 ||
        o.queue_capacity < 1)
        return PI_EINVAL;
    PI_CHECK_HIP(hipSetDevice(ctx->device));
    pi_server *s = new (std::nothrow) pi_server();
    if (!s) return PI_ENOMEM;
    s->ctx = ctx;
    s->opts = o;
    s->lanes.resize((size_t)o.n_streams);
    for (Lane &ln : s->lanes) {
        if (hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ln.done, hipEventDisableTiming) != hipSuccess) {
            for (Lane &l2 : s->lanes) {
                if (l2.stream) (void)hipStreamDestroy(l2.stream);
                if (l2.done) (void)hipEventDestroy(l2.done);
            }
            delete s;
            return PI_EDEVICE;
        }
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
    int32_t max_ppc = -1;
    if (!inside_box(*r, r->n < kAloneN, &max_ppc)) return PI_ERANGE;
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
    if (!t) {
        std::lock_guard<std::mutex> g(s->mu);
        s->pool.emplace_back(bytes, pin);
        return PI_ENOMEM;
    }
    t->req = *r;
    t->req.x = t->req.y = t->req.z = t->req.w = nullptr;
    t->footprint = fp;
    t->status = PI_OK;
    t->done = false;
    t->lane = -1;
    t->max_ppc = max_ppc;
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
    out->running = s->in_flight;
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
    for (Lane &ln : s->lanes) {
        if (ln.stream) (void)hipStreamSynchronize(ln.stream);
        if (ln.batch) pi_batch_destroy(ln.batch);
        if (ln.cells) pi_cells_destroy(ln.cells);
        void *bufs[] = {ln.d_up, ln.d_down, ln.d_xyzw, ln.d_out, ln.d_inv, ln.d_hist, ln.d_req};
        for (void *p : bufs)
            if (p) (void)hipFree(p);
        if (ln.h_req) (void)hipHostFree(ln.h_req);
        if (ln.h_err) (void)hipHostFree(ln.h_err);
        if (ln.done) (void)hipEventDestroy(ln.done);
        if (ln.stream) (void)hipStreamDestroy(ln.stream);
    }
    for (auto &kv : s->tickets) {
        (void)hipHostFree(kv.second->pinned);
        delete kv.second;
    }
    for (auto &p : s->pool) (void)hipHostFree(p.second);
    delete s;
    return PI_OK;
}
