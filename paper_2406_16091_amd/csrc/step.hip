// Time stepping on a binned system (Sec. 2: the interactions are computed,
// then the particles' positions are updated).  The state stays in the
// cell-sorted order the binning produced -- positions as cell-relative
// records, velocities beside them -- and one step is:
//   1. the sweep (pi_interact's kernels, sorted outputs);
//   2. the update: with the B-spline as a soft pair potential
//      E = (kappa / 2) sum_i sum_{j != i} w_i w_j W(r_ij) and w_i the mass,
//      the force on i is -kappa w_i G_i, so the acceleration is -kappa G_i;
//      symplectic Euler v <- v - dt kappa G, x <- x + dt v, with reflection
//      at the box faces and the box-relative coordinate rounded down to a
//      lattice (optional), so that lattice inputs stay lattice inputs;
//   3. the re-binning, incremental: a particle that stays in its cell keeps
//      its rank among the cell's stayers; a particle that changes cell takes
//      a place in its new cell's newcomer list (a per-cell counter); the
//      offsets come from one scan over the cells, which also places every
//      newcomer list; then every particle finds its slot in the new order by
//      counting: the stayers of its cell before it, and in a cell that
//      receives anybody the members (stayers and newcomers) with a smaller
//      original index.  The result is the stable counting sort of the new
//      positions -- ascending original index inside each cell -- exactly as
//      pi_bin would produce it, written into the other half of a double
//      buffer whose halves then swap.  The updated state is never stored in
//      the old order: the placement recomputes each particle's update from
//      the old state (the same operations on the same operands, so the same
//      bits) and writes it straight to its new slot.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "pi_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kScanThreads = 1024;                  // threads per block of the offsets scan
constexpr int kScanPer = 4;                          // consecutive cells per thread
constexpr int kScanBlock = kScanThreads * kScanPer;  // cells per block

struct StepArgs {
    int32_t n;
    int64_t nc;
    GridDev g;
    const int32_t *off;  // offsets of the binning before the step
    const int32_t *cell; // cell of each sorted slot before the step
    const int32_t *perm;
    const float4 *xyzw;  // records before the step
    const float4 *vel;   // velocities before the step
    const float *gx, *gy, *gz;
    int32_t *counts;     // stayers after the update; the new counts after the scan
    int32_t *ncnt;       // newcomers per cell (zero outside a step)
    int32_t *nstart;     // start of each cell's newcomer list (n_cells + 1 entries)
    int32_t *midx;       // a mover's place in its new cell's newcomer list
    uint2 *nlist;        // newcomer lists: (original index, slot before the step)
    int32_t *newcell;
    uint32_t *err;
    float dk;            // dt * kappa
    float dt;
    float half_w;        // largest displacement per axis in one step
    float lattice;
    // placement
    const int32_t *off2; // offsets after the step
    int32_t *perm2, *cell2;
    float4 *xyzw2, *vel2;
};

__device__ __forceinline__ void decode(const GridDev &g, int32_t c, int32_t &ix, int32_t &iy, int32_t &iz)
{
    const uint32_t q = div_by((uint32_t)c, g.mx);
    ix = c - (int32_t)q * g.nx;
    iz = (int32_t)div_by((uint32_t)c, g.mxy);
    iy = (int32_t)q - iz * g.ny;
}

// One axis of the update: the new velocity and box-relative coordinate of a
// particle at u in [0, L) (rounded to the lattice when one is given), with
// reflection at both faces.  Returns true when the displacement was cut.
__device__ __forceinline__ bool advance(float &u, float &v, float gacc, const StepArgs &a, float L)
{
    v = __builtin_fmaf(-a.dk, gacc, v);
    float d = a.dt * v;
    bool cut = false;
    if (fabsf(d) > a.half_w) {
        d = copysignf(a.half_w, d);
        cut = true;
    }
    float x = u + d;
    if (x < 0.0f) {
        x = -x;
        v = -v;
    }
    if (x >= L) {
        x = 2.0f * L - x;
        v = -v;
    }
    if (a.lattice > 0.0f) {
        x = floorf(x / a.lattice) * a.lattice;
        x = fminf(fmaxf(x, 0.0f), L - a.lattice);
    }
    u = x;
    return cut;
}

// The update of the particle in sorted slot k (old state), its new record
// relative to its new cell, and that cell.
struct Moved {
    float4 rec, vel;
    int32_t cell;
    bool cut;
};

__device__ __forceinline__ Moved move_particle(const StepArgs &a, int32_t k)
{
    const GridDev &g = a.g;
    int32_t ix, iy, iz;
    decode(g, a.cell[k], ix, iy, iz);
    const float4 r = a.xyzw[k];
    float4 v = a.vel[k];
    // box-relative coordinates, as the binning measured them
    float ux = __builtin_fmaf((float)ix, g.w, r.x);
    float uy = __builtin_fmaf((float)iy, g.w, r.y);
    float uz = __builtin_fmaf((float)iz, g.w, r.z);
    bool cut = advance(ux, v.x, a.gx[k], a, (float)g.nx * g.w);
    cut |= advance(uy, v.y, a.gy[k], a, (float)g.ny * g.w);
    cut |= advance(uz, v.z, a.gz[k], a, (float)g.nz * g.w);
    const float x = pi_keep_inside(g.ox + ux, g.ox, g.w, g.nx);
    const float y = pi_keep_inside(g.oy + uy, g.oy, g.w, g.ny);
    const float z = pi_keep_inside(g.oz + uz, g.oz, g.w, g.nz);
    int32_t jx = 0, jy = 0, jz = 0;
    axis_index(x, g.ox, g.w, g.nx, jx);
    axis_index(y, g.oy, g.w, g.ny, jy);
    axis_index(z, g.oz, g.w, g.nz, jz);
    Moved m;
    m.cell = jx + g.nx * (jy + g.ny * jz);
    m.rec = make_float4(__builtin_fmaf(-(float)jx, g.w, x - g.ox), __builtin_fmaf(-(float)jy, g.w, y - g.oy),
                        __builtin_fmaf(-(float)jz, g.w, z - g.oz), r.w);
    m.vel = make_float4(v.x, v.y, v.z, 0.0f);
    m.cut = cut;
    return m;
}

// 1. The new cell of every particle; the counts follow the particles that
// change cell.
__global__ __launch_bounds__(kBlock) void k_step_move(StepArgs a)
{
    const int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (k >= a.n) return;
    const int32_t c = a.cell[k];
    const Moved m = move_particle(a, k);
    a.newcell[k] = m.cell;
    if (m.cell != c) {
        atomicSub(a.counts + c, 1);
        a.midx[k] = atomicAdd(a.ncnt + m.cell, 1);
    }
    if (m.cut) atomicOr(a.err, PI_DERR_STEP);
}

// 2. One scan over the cells, in three passes (block totals, one
// workgroup scanning them, each block's own scan plus its prefix), of the
// new counts (stayers + newcomers) into the new offsets and of the
// newcomers into the start of each cell's newcomer list (n_cells + 1
// entries); it also finds M_C and leaves the newcomer counters at zero for
// the next step.
template <int NT>
__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t *wsum, int32_t &total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int32_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int32_t before = 0;
    total = 0;
    for (int w = 0; w < NT / 64; ++w) {
        if (w < wid) before += wsum[w];
        total += wsum[w];
    }
    __syncthreads();
    return before + inc - v;
}

// The new counts (stayers + newcomers) and the newcomers of the kScanPer
// cells from `base` (16-byte loads where all four are inside; zero past nc).
static_assert(kScanPer == 4, "the scan loads four cells at once");
__device__ __forceinline__ void load_cells(const int32_t *__restrict__ cnt, const int32_t *__restrict__ ncnt,
                                           int64_t nc, int64_t base, int32_t *v, int32_t *nw)
{
    if (base + kScanPer <= nc) {
        const int4 c4 = *reinterpret_cast<const int4 *>(cnt + base);
        const int4 n4 = *reinterpret_cast<const int4 *>(ncnt + base);
        nw[0] = n4.x; nw[1] = n4.y; nw[2] = n4.z; nw[3] = n4.w;
        v[0] = c4.x + n4.x; v[1] = c4.y + n4.y; v[2] = c4.z + n4.z; v[3] = c4.w + n4.w;
    } else {
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) {
            const bool in = base + q < nc;
            nw[q] = in ? ncnt[base + q] : 0;
            v[q] = in ? cnt[base + q] + nw[q] : 0;
        }
    }
}

// Block b's totals: sums of new counts and of newcomers at tot[0 * ns + b]
// and tot[1 * ns + b]; the largest new count at tot[2 * ns + b].
__global__ __launch_bounds__(kScanThreads) void k_scan_totals(const int32_t *__restrict__ cnt,
                                                              const int32_t *__restrict__ ncnt, int64_t nc,
                                                              int32_t *__restrict__ tot, int32_t ns)
{
    __shared__ int32_t part[3][kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
    int32_t v[kScanPer], nw[kScanPer];
    load_cells(cnt, ncnt, nc, base, v, nw);
    int32_t sc = 0, sn = 0, m = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        sc += v[q];
        sn += nw[q];
        m = max(m, v[q]);
    }
    sc = wave_sum(sc);
    sn = wave_sum(sn);
    m = wave_max(m);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        part[0][w] = sc;
        part[1][w] = sn;
        part[2][w] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t0 = 0, t1 = 0, t2 = 0;
        for (int q = 0; q < kScanThreads / 64; ++q) {
            t0 += part[0][q];
            t1 += part[1][q];
            t2 = max(t2, part[2][q]);
        }
        tot[blockIdx.x] = t0;
        tot[ns + blockIdx.x] = t1;
        tot[2 * ns + blockIdx.x] = t2;
    }
}

// One workgroup: the exclusive prefixes of the two block sums (in place),
// the largest count into *max_per_cell, the newcomer total into nstart[nc].
__global__ __launch_bounds__(kBlock) void k_scan_top(int32_t *__restrict__ tot, int32_t nb, int32_t ns,
                                                     int32_t *__restrict__ max_per_cell,
                                                     int32_t *__restrict__ nstart, int64_t nc)
{
    __shared__ int32_t wsum[kBlock / 64];
    __shared__ int32_t wmax[kBlock / 64];
    int32_t m = 0;
    for (int q = 0; q < 2; ++q) {
        int32_t *t = tot + q * ns;
        int32_t carry = 0;
        for (int32_t b0 = 0; b0 < nb; b0 += kBlock) {
            const int32_t b = b0 + (int32_t)threadIdx.x;
            const int32_t v = b < nb ? t[b] : 0;
            if (q == 0) m = max(m, b < nb ? tot[2 * ns + b] : 0);
            int32_t total;
            const int32_t ex = block_excl_scan<kBlock>(v, wsum, total);
            if (b < nb) t[b] = carry + ex;
            carry += total;
        }
        if (q == 1 && threadIdx.x == 0) nstart[nc] = carry;
    }
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t u = 0;
        for (int w = 0; w < kBlock / 64; ++w) u = max(u, wmax[w]);
        *max_per_cell = u;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_apply(int32_t *__restrict__ cnt, int32_t *__restrict__ ncnt,
                                                             int64_t nc, const int32_t *__restrict__ tot, int32_t ns,
                                                             int32_t *__restrict__ off, int32_t *__restrict__ nstart,
                                                             int32_t n)
{
    __shared__ int32_t wsum[kScanThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanPer;
    int32_t v[kScanPer], nw[kScanPer], sc = 0, sn = 0;
    load_cells(cnt, ncnt, nc, base, v, nw);
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        sc += v[q];
        sn += nw[q];
    }
    int32_t total;
    int32_t ec = tot[blockIdx.x] + block_excl_scan<kScanThreads>(sc, wsum, total);
    int32_t en = tot[ns + blockIdx.x] + block_excl_scan<kScanThreads>(sn, wsum, total);
    int32_t eo[kScanPer], es[kScanPer];
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
        eo[q] = ec;
        es[q] = en;
        ec += v[q];
        en += nw[q];
    }
    if (base + kScanPer <= nc) {
        *reinterpret_cast<int4 *>(off + base) = make_int4(eo[0], eo[1], eo[2], eo[3]);
        *reinterpret_cast<int4 *>(nstart + base) = make_int4(es[0], es[1], es[2], es[3]);
        *reinterpret_cast<int4 *>(cnt + base) = make_int4(v[0], v[1], v[2], v[3]);
    } else {
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) {
            if (base + q < nc) {
                off[base + q] = eo[q];
                nstart[base + q] = es[q];
                cnt[base + q] = v[q];
            }
        }
    }
#pragma unroll
    for (int q = 0; q < kScanPer; ++q)
        if (nw[q] != 0) ncnt[base + q] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) off[nc] = n;
}

// The particle in old slot k, whose update is m, to slot s of cell c in the
// new order.
__device__ __forceinline__ void place_moved(const StepArgs &a, int32_t c, int32_t s, int32_t k, const Moved &m)
{
    if (s >= a.off2[c + 1]) { // cannot happen: the counts add up
        atomicOr(a.err, PI_DERR_INTERNAL);
        return;
    }
    a.perm2[s] = a.perm[k];
    a.cell2[s] = c;
    a.xyzw2[s] = m.rec;
    a.vel2[s] = m.vel;
}

// Stayers of cell c in old slots before k (old slots of a cell are in
// ascending original index).
__device__ __forceinline__ int32_t stayers_before(const StepArgs &a, int32_t c, int32_t k)
{
    int32_t r = 0;
    for (int32_t j = a.off[c]; j < k; ++j) r += a.newcell[j] == c ? 1 : 0;
    return r;
}

// 3a. The newcomer lists: one thread per old slot, a particle that changed
// cell writes (original index, old slot) at its place in its new cell's list.
__global__ __launch_bounds__(kBlock) void k_step_list(StepArgs a)
{
    const int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (k >= a.n) return;
    const int32_t c2 = a.newcell[k];
    if (c2 != a.cell[k]) a.nlist[a.nstart[c2] + a.midx[k]] = make_uint2((uint32_t)a.perm[k], (uint32_t)k);
}

// 3b. One thread per old slot (coalesced reads of the particle's own state):
// its slot in its new cell is the number of the cell's members with a
// smaller original index -- stayers (old slots of the cell still in it; for
// a stayer, those before it) and newcomers (the cell's newcomer list, empty
// for most cells).
__global__ __launch_bounds__(kBlock) void k_step_place(StepArgs a)
{
    const int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (k >= a.n) return;
    const int32_t c = a.cell[k], c2 = a.newcell[k];
    const Moved m = move_particle(a, k);
    const int32_t o = a.perm[k];
    int32_t r = 0;
    if (c2 == c) {
        r = stayers_before(a, c, k);
    } else {
        for (int32_t j = a.off[c2]; j < a.off[c2 + 1]; ++j) r += (a.newcell[j] == c2 && a.perm[j] < o) ? 1 : 0;
    }
    for (int32_t q = a.nstart[c2]; q < a.nstart[c2 + 1]; ++q) r += (int32_t)a.nlist[q].x < o ? 1 : 0;
    place_moved(a, c2, a.off2[c2] + r, k, m);
}

__global__ __launch_bounds__(kBlock) void k_gather_velocity(int32_t n, const int32_t *__restrict__ perm,
                                                            const float *__restrict__ vx,
                                                            const float *__restrict__ vy,
                                                            const float *__restrict__ vz, float4 *__restrict__ vel)
{
    const int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (k >= n) return;
    const int32_t i = perm[k];
    vel[k] = make_float4(vx[i], vy[i], vz[i], 0.0f);
}

// The state back in the caller's (original) order: positions from the
// records (origin + cell corner + cell-relative part), velocities, and the
// sweep outputs of the last step.
__global__ __launch_bounds__(kBlock) void k_scatter_state(int32_t n, GridDev g, const int32_t *__restrict__ perm,
                                                          const int32_t *__restrict__ cell,
                                                          const float4 *__restrict__ xyzw,
                                                          const float4 *__restrict__ vel, float *x, float *y,
                                                          float *z, float *vx, float *vy, float *vz)
{
    const int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (k >= n) return;
    const int32_t i = perm[k];
    int32_t ix, iy, iz;
    decode(g, cell[k], ix, iy, iz);
    const float4 r = xyzw[k];
    if (x) {
        x[i] = g.ox + __builtin_fmaf((float)ix, g.w, r.x);
        y[i] = g.oy + __builtin_fmaf((float)iy, g.w, r.y);
        z[i] = g.oz + __builtin_fmaf((float)iz, g.w, r.z);
    }
    if (vx) {
        const float4 v = vel[k];
        vx[i] = v.x;
        vy[i] = v.y;
        vz[i] = v.z;
    }
}

__global__ __launch_bounds__(kBlock) void k_scatter_forces(int32_t n, const int32_t *__restrict__ perm,
                                                           const float *__restrict__ grho,
                                                           const float *__restrict__ ggx,
                                                           const float *__restrict__ ggy,
                                                           const float *__restrict__ ggz, float *rho, float *gx,
                                                           float *gy, float *gz)
{
    const int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (k >= n) return;
    const int32_t i = perm[k];
    rho[i] = grho[k];
    gx[i] = ggx[k];
    gy[i] = ggy[k];
    gz[i] = ggz[k];
}

inline unsigned nblocks(int64_t n, int b) { return (unsigned)std::max<int64_t>(1, (n + b - 1) / b); }

} // namespace

extern "C" pi_status pi_state_set_velocity(pi_ctx *ctx, pi_cells *cells, const float *vx, const float *vy,
                                           const float *vz, pi_stream stream_)
{
    if (!ctx || !cells || cells->ctx != ctx) return PI_EINVAL;
    if (!pi_cells_ready(cells)) return PI_ESTATE;
    const int64_t n = cells->n;
    if (n > 0 && (!vx || !vy || !vz)) return PI_EINVAL;
    PI_CHECK_HIP(hipSetDevice(ctx->device));
    const pi_status st = pi_stepping_enable(cells);
    if (st != PI_OK) return st;
    hipStream_t s = (hipStream_t)stream_;
    if (n > 0)
        PI_LAUNCH(ctx, "k_gather_velocity", k_gather_velocity, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, s,
                  (int32_t)n, cells->perm, vx, vy, vz, cells->vel);
    PI_CHECK_HIP(hipGetLastError());
    cells->vel_valid = true;
    cells->stepped = false;
    cells->last_stream = s;
    return PI_OK;
}

extern "C" pi_status pi_step(pi_ctx *ctx, pi_cells *cells, const pi_step_opts *opts, pi_invariants *inv,
                             pi_stream stream_)
{
    if (!ctx || !cells || !opts || cells->ctx != ctx) return PI_EINVAL;
    if (!pi_cells_ready(cells) || !cells->stepping || !cells->vel_valid) return PI_ESTATE;
    const pi_step_opts &o = *opts;
    if (!isfinite(o.dt) || !(o.dt >= 0.0f) || !isfinite(o.kappa) || !(o.lattice >= 0.0f) || !isfinite(o.lattice))
        return PI_EINVAL;
    const int64_t n = cells->n, nc = cells->n_cells;
    hipStream_t s = (hipStream_t)stream_;
    PI_CHECK_HIP(hipSetDevice(ctx->device));

    // 1. the sweep, outputs in sorted order
    pi_interact_opts io;
    memset(&io, 0, sizeof(io));
    io.precision = o.precision;
    io.sweep = o.sweep;
    io.order = PI_ORDER_SORTED;
    for (int q = 0; q < 3; ++q) io.tile[q] = o.tile[q];
    pi_status st = pi_check_interact_opts(io, n, cells->grho, cells->ggx, cells->ggy, cells->ggz, nullptr, inv);
    if (st != PI_OK) return st;
    st = pi_interact_run(ctx, cells, io, cells->grho, cells->ggx, cells->ggy, cells->ggz, nullptr, inv, s,
                         cells->partials, cells->cap_partials, false);
    if (st != PI_OK) return st;
    if (n == 0) return PI_OK;

    // 2. update and new cells
    StepArgs a;
    memset(&a, 0, sizeof(a));
    a.n = (int32_t)n;
    a.nc = nc;
    a.g = grid_dev(cells->grid);
    a.off = cells->offsets;
    a.cell = cells->cell;
    a.perm = cells->perm;
    a.xyzw = cells->xyzw;
    a.vel = cells->vel;
    a.gx = cells->ggx;
    a.gy = cells->ggy;
    a.gz = cells->ggz;
    a.counts = cells->counts;
    // the newcomer counters are zero between steps: zeroed once after an
    // allocation, and back to zero in every step's scan
    if (!cells->ncnt_zeroed) {
        PI_CHECK_HIP(hipMemsetAsync(cells->ncnt, 0, (size_t)std::max<int64_t>(nc, 1) * sizeof(int32_t), s));
        cells->ncnt_zeroed = true;
    }
    a.ncnt = cells->ncnt;
    a.nstart = cells->nstart;
    a.midx = cells->midx;
    a.nlist = cells->nlist;
    a.newcell = cells->newcell;
    a.err = cells->d_err;
    a.dt = o.dt;
    a.dk = o.dt * o.kappa;
    a.half_w = 0.5f * cells->grid.cell_w;
    a.lattice = o.lattice;
    a.off2 = cells->offsets2;
    a.perm2 = cells->perm2;
    a.cell2 = cells->cell2;
    a.xyzw2 = cells->xyzw2;
    a.vel2 = cells->vel2;
    PI_LAUNCH(ctx, "k_step_move", k_step_move, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, s, a);
    // 3. new offsets, newcomer list starts and M_C
    const int32_t nb = (int32_t)((nc + kScanBlock - 1) / kScanBlock);
    const int32_t ns = (int32_t)(nc / kScanBlock + 2);
    int32_t *tot = cells->scan;
    PI_LAUNCH(ctx, "k_scan_totals", k_scan_totals, dim3((unsigned)nb), dim3(kScanThreads), 0, s, cells->counts,
              cells->ncnt, nc, tot, ns);
    PI_LAUNCH(ctx, "k_scan_top", k_scan_top, dim3(1), dim3(kBlock), 0, s, tot, nb, ns, cells->max_per_cell,
              cells->nstart, nc);
    PI_LAUNCH(ctx, "k_scan_apply", k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s, cells->counts,
              cells->ncnt, nc, tot, ns, cells->offsets2, cells->nstart, (int32_t)n);
    // 4. the newcomer lists, then the new stable order
    PI_LAUNCH(ctx, "k_step_list", k_step_list, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, s, a);
    PI_LAUNCH(ctx, "k_step_place", k_step_place, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, s, a);
    PI_CHECK_HIP(hipGetLastError());
    std::swap(cells->perm, cells->perm2);
    std::swap(cells->cell, cells->cell2);
    std::swap(cells->xyzw, cells->xyzw2);
    std::swap(cells->vel, cells->vel2);
    std::swap(cells->offsets, cells->offsets2);
    cells->soa_stale = true;
    cells->stepped = true;
    cells->last_stream = s;
    return PI_OK;
}

extern "C" pi_status pi_state_get(pi_ctx *ctx, pi_cells *cells, float *x, float *y, float *z, float *vx, float *vy,
                                  float *vz, float *rho, float *gx, float *gy, float *gz, pi_stream stream_)
{
    if (!ctx || !cells || cells->ctx != ctx) return PI_EINVAL;
    if (!pi_cells_ready(cells) || !cells->stepping || !cells->vel_valid) return PI_ESTATE;
    const bool px = x || y || z, pv = vx || vy || vz, pg = rho || gx || gy || gz;
    if ((px && !(x && y && z)) || (pv && !(vx && vy && vz)) || (pg && !(rho && gx && gy && gz))) return PI_EINVAL;
    if (pg && !cells->stepped) return PI_ESTATE;
    const int64_t n = cells->n;
    if (n == 0) return PI_OK;
    PI_CHECK_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream_;
    if (px || pv)
        PI_LAUNCH(ctx, "k_scatter_state", k_scatter_state, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, s, (int32_t)n,
                  grid_dev(cells->grid), cells->perm, cells->cell, cells->xyzw, cells->vel, px ? x : nullptr, y, z,
                  pv ? vx : nullptr, vy, vz);
    // the sweep outputs of the last step are in the order before it, whose
    // permutation is the other half of the double buffer
    if (pg)
        PI_LAUNCH(ctx, "k_scatter_forces", k_scatter_forces, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, s,
                  (int32_t)n, cells->perm2, cells->grho, cells->ggx, cells->ggy, cells->ggz, rho, gx, gy, gz);
    PI_CHECK_HIP(hipGetLastError());
    return PI_OK;
}
