// Internal declarations of the gfx950 library: context and cell objects,
// launch helpers, wave64 primitives and the B-spline pair term.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>

#include "../../include/pi.h"

#define PI_CHECK_HIP(expr)                                  \
    do {                                                    \
        hipError_t _e = (expr);                             \
        if (_e != hipSuccess) return pi_hip_fail(_e, #expr); \
    } while (0)

pi_status pi_hip_fail(hipError_t e, const char *what);

// Device-side error bits latched in pi_cells::d_err.
#define PI_DERR_RANGE 1u
#define PI_DERR_STEP 2u   // a step's displacement was cut to half a cell width
#define PI_DERR_INTERNAL 4u // a kernel found its own invariant broken (no write made)

struct pi_timing; // per-context kernel timing state (abi.hip)

// Sweep-organisation choices of the tuner, keyed by a size/occupancy class.
struct pi_tuner {
    std::mutex mu;
    std::map<uint64_t, int> choice; // class -> tile id (0 = no LDS)
    int mode = 1;                   // PI_TUNE_STATIC / PI_TUNE_TIMED
};

struct pi_ctx {
    int device;
    int num_cu;
    int num_xcd;
    size_t lds_per_block;
    volatile int timing_on;
    pi_timing *timing;
    pi_tuner *tuner;
    void *scratch; // this device's copy of the fixed sweep scratch (sweep.hip)
};

// Device address of the fixed scratch array of pi_interact_noalloc on
// `device`, which must be current (looked up once per device and kept).
pi_status pi_noalloc_scratch_setup(int device, void **out);

// Set on a thread while it queues work that must not record timing events
// (event records take events from a pool that may need to create one).
extern thread_local bool pi_tls_no_timing;

// Kernel timing: bracket one launch with events on its stream when enabled.
void *pi_timer_begin(pi_ctx *ctx, hipStream_t s, const char *name);
void pi_timer_end(pi_ctx *ctx, hipStream_t s, void *tok);

#define PI_LAUNCH(ctx, name, kern, grid, block, shmem, stream, ...)                 \
    do {                                                                          \
        void *_tok = ((ctx)->timing_on && !pi_tls_no_timing) ? pi_timer_begin((ctx), (stream), (name)) : nullptr; \
        hipLaunchKernelGGL(kern, grid, block, shmem, stream, __VA_ARGS__);         \
        if (_tok) pi_timer_end((ctx), (stream), _tok);                             \
    } while (0)

// Device buffers of one binned system.  Capacities grow, never shrink.
struct pi_cells {
    pi_ctx *ctx;
    int64_t n;          // particles of the last pi_bin
    int64_t n_cells;
    pi_grid grid;
    int64_t cap_n;      // capacity in particles
    int64_t cap_cells;  // capacity in cells
    int64_t cap_hist;   // radix histogram entries (256 per sort tile)
    hipStream_t last_stream;
    bool binned;
    // per cell
    int32_t *counts;    // [cap_cells]
    int32_t *offsets;   // [cap_cells + 1]
    // per particle, sorted order (the results of binning)
    int32_t *perm;      // [cap_n] stable sorted order
    int32_t *cell;      // [cap_n] cell of sorted slot
    float *xs, *ys, *zs, *ws;   // [cap_n]
    float4 *xyzw;       // [cap_n] sorted cell-relative (x, y, z, w) records
    bool soa_stale;     // xs .. ws not yet written from the records of the last bin
    // radix-sort ping-pong buffers: key, original index, x, y, z, w
    uint2 *skv[2];       // radix ping-pong records (cell id, original index)
    float4 *sp[2];       // payload records (x, y, z, w)
    int32_t *dtot;       // radix digit totals (256)
    // radix histograms (digit-major, 256 x sort tiles) and their scan scratch
    int32_t *hist;        // [cap_hist]
    // cell-scan scratch
    int32_t *max_per_cell; // [1]
    uint32_t *d_err;       // 256 bytes: error word [0], max_per_cell [16], the
                           // epoch of the last tile sweep that overflowed [32],
                           // a step's receiving-cell count [40]
    // invariant partials
    int64_t cap_partials;
    void *partials;
    // per workgroup of a sweep launch: whether its tile's halo overflowed
    // the LDS area (cap_tflag bytes: cap_cells + 64, as a single system has
    // at most one tile per cell; a batch may enlarge it to its workgroups)
    uint8_t *tflag;
    int64_t cap_tflag;
    uint32_t sweep_epoch; // number of the last tile sweep launched on the object
    // time stepping (allocated once pi_state_set_velocity is first called on
    // the object; the "2" arrays are the other half of a double buffer whose
    // halves swap after every step)
    bool stepping;       // the buffers below exist
    bool vel_valid;      // vel holds the velocities of the binned system
    bool stepped;        // a step ran since: grho .. ggz hold its sweep outputs
    bool ncnt_zeroed;    // ncnt was zeroed since it was (re)allocated
    float4 *vel, *vel2;  // [cap_n] sorted (vx, vy, vz, 0)
    int32_t *perm2, *cell2, *newcell; // [cap_n]
    float4 *xyzw2;       // [cap_n]
    float *grho, *ggx, *ggy, *ggz; // [cap_n] sorted sweep outputs of the last step
    int32_t *offsets2;   // [cap_cells + 1]
    int32_t *ncnt;       // [cap_cells] newcomers per cell during a step, zero between steps
    int32_t *nstart;     // [cap_cells + 1] start of each cell's newcomer list
    int32_t *midx;       // [cap_n] a mover's place in its new cell's newcomer list
    uint2 *nlist;        // [cap_n] newcomer lists (original index, slot)
    int32_t *scan;       // block partials of the offsets scan (4 x (cap_cells / 1024 + 2))
};

// Allocate the time-stepping buffers of a cell object at its capacities.
pi_status pi_stepping_enable(pi_cells *cells);

// ------------------------------------------------------------- launch helpers

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup g runs on
// XCD g % 8).  Remap so that each XCD processes one contiguous range of
// logical tiles: neighbouring tiles then share that XCD's L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t g, uint32_t ng)
{
    constexpr uint32_t X = 8;
    const uint32_t q = ng / X, r = ng % X;
    const uint32_t xcd = g % X, idx = g / X;
    return (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// ------------------------------------------------------------- wave64 scan

// Inclusive prefix sum over the 64 lanes of a wavefront: four row_shr DPP
// steps scan each 16-lane row, then row_bcast:15 / row_bcast:31 carry the row
// totals into the rows above (GFX9 DPP controls, available on gfx950).
__device__ __forceinline__ int32_t wave_incl_scan(int32_t v)
{
    int32_t t;
    t = __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false); v += t; // row_shr:1
    t = __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false); v += t; // row_shr:2
    t = __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false); v += t; // row_shr:4
    t = __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false); v += t; // row_shr:8
    t = __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false); v += t; // row_bcast:15
    t = __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false); v += t; // row_bcast:31
    return v;
}

__device__ __forceinline__ int32_t wave_max(int32_t v)
{
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int32_t wave_sum(int32_t v)
{
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ------------------------------------------------------------- geometry

struct GridDev {
    float ox, oy, oz;
    float w;        // cell width
    int32_t nx, ny, nz;
    int32_t pad;
    // multipliers for dividing a cell id by nx and by nx * ny (div_by)
    uint64_t mx, mxy;
};

// Multiplier M for exact division n / d of any n < 2^31 by a fixed d < 2^31
// (division by a constant as a multiply-high): with M = ceil(2^62 / d) * 4,
// floor(n / d) = mulhi64(n, M).  Since d * M / 4 = 2^62 + e with 0 <= e < d,
// n M / 2^64 = n / d + n e / (d 2^62), and n e < 2^62 keeps the floor.
// d = 1 is marked by M = 0.
inline uint64_t div_magic(int64_t d)
{
    if (d <= 1) return 0;
    const unsigned __int128 one = 1;
    return (uint64_t)(((one << 62) + (unsigned __int128)(d - 1)) / (unsigned __int128)d) << 2;
}

inline void grid_set_magic(GridDev &g)
{
    g.mx = div_magic(g.nx);
    g.mxy = div_magic((int64_t)g.nx * g.ny);
}

inline GridDev grid_dev(const pi_grid &grid)
{
    GridDev g;
    g.ox = grid.origin[0];
    g.oy = grid.origin[1];
    g.oz = grid.origin[2];
    g.w = grid.cell_w;
    g.nx = grid.dims[0];
    g.ny = grid.dims[1];
    g.nz = grid.dims[2];
    g.pad = 0;
    grid_set_magic(g);
    return g;
}

__device__ __forceinline__ uint32_t div_by(uint32_t n, uint64_t m)
{
    return m ? (uint32_t)__umul64hi((uint64_t)n, m) : n;
}

// One axis of the cell decision: t = (x - o) / w in float32 (IEEE), inside
// iff 0 <= t < n, index floor(t).  NaN fails the test.  The host takes the
// same decision with the same two roundings (the library is built without
// floating-point contraction).
__host__ __device__ __forceinline__ bool axis_index(float x, float o, float w, int32_t n, int32_t &out)
{
    const float u = x - o;
    const float t = u / w;
    if (!(t >= 0.0f && t < (float)n)) return false;
    out = (int32_t)t; // t >= 0: truncation is floor
    return true;
}

// A coordinate p meant to lie in the box [o, o + n w) on one axis, moved by
// single ulps until the binning's float32 decision (axis_index) keeps it
// inside: o + v rounds once more when o is large against the box, and a
// reflection at the far face can land on it.
__device__ __forceinline__ float pi_keep_inside(float p, float o, float w, int32_t n)
{
    for (int it = 0; it < 64; ++it) {
        const float t = (p - o) / w;
        if (t >= 0.0f && t < (float)n) return p;
        p = t < 0.0f ? nextafterf(p, INFINITY) : nextafterf(p, -INFINITY);
    }
    return o; // t = 0: the low corner is always inside
}

pi_status pi_ensure_capacity(pi_cells *cells, int64_t n, int64_t n_cells, hipStream_t stream);
// Mark a cell object as holding no binned system (after a failed binning).
void pi_cells_forget(pi_cells *cells);
// Whether every buffer a sweep of the object's binned system reads exists.
bool pi_cells_ready(const pi_cells *cells);

// One system of a batch, as the batched kernels see it.  Systems are
// concatenated in order: system s owns input (and sorted) particles
// [first, first + n) and global cells [cell_base, cell_base + nx ny nz).
struct SysDev {
    int64_t first;
    int32_t n;
    int32_t cell_base;
    int32_t block_base; // first workgroup of this system in a sweep launch
    int32_t ntx, nty;   // tiles per axis in that launch
    int32_t orig;       // index of the system in the caller's list
    GridDev g;
};

bool pi_grid_valid(const pi_grid *g);

struct KernelConst;
struct pi_interact_opts;
KernelConst pi_make_kernel_const(float rc, float cell_w);
bool pi_tile_shape(int tile_id, int *tx, int *ty, int *tz);
int pi_pick_tile(const pi_interact_opts &o, double ppc);
void pi_tile_opts(int tile_id, pi_interact_opts *out);
int pi_auto_tile(pi_ctx *ctx, int precision, int64_t n, double ppc);
int64_t pi_batch_layout(int tile_id, SysDev *h_sys, int32_t nsys);
int pi_batch_org(int tile_id);
bool pi_org_valid(int id);
// A batch object that launches its sequence directly on every call instead
// of capturing it into a graph (for layouts used a few times only); the
// tables are rebuilt only when the layout changes.
void pi_batch_set_direct(pi_batch *batch, bool direct);
// The cell object a batch bins its systems into (its device error word).
pi_cells *pi_batch_cells(pi_batch *batch);
// pi_batch_run with per-system organisations: org[s] >= 0 (an organisation
// id, 0 = no LDS) replaces system s's AUTO or explicit choice; org may be
// null.
pi_status pi_batch_run_orgs(pi_ctx *ctx, pi_batch *b, int32_t nsys, const pi_system_desc *sys, const int32_t *org,
                            const float *x, const float *y, const float *z, const float *w,
                            const pi_interact_opts *opts, float *rho, float *gx, float *gy, float *gz,
                            int32_t *count, pi_invariants *inv, pi_stream stream);
pi_status pi_sweep_batch(pi_ctx *ctx, pi_cells *cells, int32_t nsys, const SysDev *d_sys, const KernelConst *d_kcs,
                         int64_t total_blocks, int64_t part_base, int tile_id, const pi_interact_opts &o, float *rho,
                         float *gx, float *gy, float *gz, int32_t *count, pi_invariants *inv, hipStream_t stream);

// The sweep of pi_interact (sweep.hip) on a binned system whose invariant
// partial records live in `partials` (cap_partials records of 64 bytes).
// With no_alloc the call allocates nothing, waits for nothing and runs no
// timed tuner trials: AUTO takes the tuner's cached choice or the static
// rule, and a tiling that needs more records than cap_partials gives
// PI_ENOMEM (AUTO falls back to the no-LDS sweep first).
pi_status pi_interact_run(pi_ctx *ctx, const pi_cells *cells, const pi_interact_opts &o, float *rho, float *gx,
                          float *gy, float *gz, int32_t *count, pi_invariants *inv, hipStream_t stream,
                          void *partials, int64_t cap_partials, bool no_alloc);
// Host checks of pi_interact's options and output pointers for n particles.
pi_status pi_check_interact_opts(const pi_interact_opts &o, int64_t n, const float *rho, const float *gx,
                                 const float *gy, const float *gz, const int32_t *count, const pi_invariants *inv);

// Host-side binning of a concatenated set of systems (bin.hip): one radix
// sort over global cell ids; sorted arrays hold local cell ids.
// Write the SoA arrays xs, ys, zs, ws of a binned system from its records
// (bin.hip), on the stream of its last binning.
pi_status pi_split_records(pi_ctx *ctx, pi_cells *cells);

// Coarse cell-to-system index of a batch: entry b is the system owning
// global cell b << kCellHintShift (entries 0 .. ceil(cells_total / 2^shift)
// inclusive, the last ones the last system), so the system of cell c lies
// between entries c >> shift and (c >> shift) + 1.
constexpr int kCellHintShift = 10;

pi_status pi_bin_systems(pi_ctx *ctx, pi_cells *cells, const float *x, const float *y, const float *z,
                         const float *w, int64_t n_total, int64_t cells_total, int32_t nsys,
                         const SysDev *d_sys, const int32_t *d_cell_hint, const GridDev &g0, hipStream_t stream);
