// Binning (paper Sec. 2 and Fig. 1): cell of every particle, per-cell counts
// with atomics, exclusive prefix sum (n_cells + 1 entries, last = n) and the
// scatter into a cell-sorted order, made stable (ascending original index
// inside each cell) so that every later result is reproducible.
//
// Kernels, in launch order on the caller's stream:
//   k_fill_i32      counts = 0 (a kernel, not a memset, so the sequence can
//                   be captured into a graph)
//   k_bin_count     cell id (float32 decision), atomicAdd on counts -> the
//                   particle's arrival slot inside its cell
//   k_scan_reduce   per 4096-cell tile: sum and max of counts
//   k_scan_tiles    one workgroup: exclusive scan of tile sums, M_C, total
//   k_scan_down     per tile: wave64 DPP scan, writes offsets
//   k_bin_scatter   perm_u[offsets[c] + slot] = i (arrival order)
//   k_bin_finalize  per sorted slot: stable rank inside the cell, gathers
//                   the particle, writes perm, cell, xs, ys, zs, ws
#include "pi_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems; // 4096 cells per scan tile

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_bin_count(int32_t n, const float *__restrict__ x,
                                                      const float *__restrict__ y,
                                                      const float *__restrict__ z, GridDev g,
                                                      int32_t *__restrict__ counts,
                                                      int32_t *__restrict__ cell_in,
                                                      int32_t *__restrict__ slot_in,
                                                      uint32_t *__restrict__ err)
{
    const int32_t i = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (i >= n) return;
    int32_t ix, iy, iz;
    const int ok = (int)axis_index(x[i], g.ox, g.w, g.nx, ix) & (int)axis_index(y[i], g.oy, g.w, g.ny, iy) &
                   (int)axis_index(z[i], g.oz, g.w, g.nz, iz);
    if (!ok) {
        cell_in[i] = -1;
        slot_in[i] = 0;
        atomicOr(err, PI_DERR_RANGE);
        return;
    }
    const int32_t c = ix + g.nx * (iy + g.ny * iz);
    cell_in[i] = c;
    slot_in[i] = atomicAdd(&counts[c], 1);
}

// Block-wide sum and max of one value per thread (256 threads, 4 waves).
__device__ __forceinline__ void block_sum_max(int32_t &s, int32_t &m, int32_t *lds)
{
    s = wave_sum(s);
    m = wave_max(m);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        lds[wid] = s;
        lds[4 + wid] = m;
    }
    __syncthreads();
    s = lds[0] + lds[1] + lds[2] + lds[3];
    m = max(max(lds[4], lds[5]), max(lds[6], lds[7]));
}

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int32_t *__restrict__ counts, int64_t nc,
                                                        int32_t *__restrict__ tile_sum,
                                                        int32_t *__restrict__ tile_max)
{
    __shared__ int32_t lds[8];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    int32_t s = 0, m = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        const int64_t c = base + j * kBlock + threadIdx.x; // coalesced
        if (c < nc) {
            const int32_t v = counts[c];
            s += v;
            m = max(m, v);
        }
    }
    block_sum_max(s, m, lds);
    if (threadIdx.x == 0) {
        tile_sum[blockIdx.x] = s;
        tile_max[blockIdx.x] = m;
    }
}

// Exclusive scan of a block of 1024 values held one per thread (16 waves);
// returns the exclusive prefix and writes the block total to *total.
__device__ __forceinline__ int32_t block_excl_scan_1024(int32_t v, int32_t *lds, int32_t *total)
{
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t inc = wave_incl_scan(v);
    if (lane == 63) lds[wid] = inc;
    __syncthreads();
    if (wid == 0) {
        const int32_t wv = lane < 16 ? lds[lane] : 0;
        const int32_t wi = wave_incl_scan(wv);
        if (lane < 16) lds[16 + lane] = wi - wv; // exclusive per wave
        if (lane == 15) lds[32] = wi;
    }
    __syncthreads();
    const int32_t r = inc - v + lds[16 + wid];
    *total = lds[32];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(1024) void k_scan_tiles(int32_t *__restrict__ tile_sum,
                                                     const int32_t *__restrict__ tile_max, int32_t ntiles,
                                                     int32_t *__restrict__ off_last,
                                                     int32_t *__restrict__ mc_out)
{
    __shared__ int32_t lds[40];
    __shared__ int32_t red[32];
    int32_t carry = 0, m = 0;
    for (int32_t b = 0; b < ntiles; b += 1024) {
        const int32_t t = b + (int32_t)threadIdx.x;
        const int32_t v = t < ntiles ? tile_sum[t] : 0;
        if (t < ntiles) m = max(m, tile_max[t]);
        int32_t tot;
        const int32_t ex = block_excl_scan_1024(v, lds, &tot);
        if (t < ntiles) tile_sum[t] = carry + ex;
        carry += tot;
    }
    // max over the block
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t mm = 0;
        for (int k = 0; k < 16; ++k) mm = max(mm, red[k]);
        *mc_out = mm;
        *off_last = carry;
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_down(const int32_t *__restrict__ counts, int64_t nc,
                                                      const int32_t *__restrict__ tile_off,
                                                      int32_t *__restrict__ off)
{
    __shared__ int32_t lds[8];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    if (base + kScanItems <= nc) {
        const int4 *p = reinterpret_cast<const int4 *>(counts + base);
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q) {
            const int4 t = p[q];
            v[4 * q] = t.x;
            v[4 * q + 1] = t.y;
            v[4 * q + 2] = t.z;
            v[4 * q + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) v[j] = (base + j < nc) ? counts[base + j] : 0;
    }
    int32_t tsum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) tsum += v[j];
    // block exclusive scan of per-thread sums (4 waves)
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t inc = wave_incl_scan(tsum);
    if (lane == 63) lds[wid] = inc;
    __syncthreads();
    int32_t wofs = 0;
    for (int k = 0; k < wid; ++k) wofs += lds[k];
    int32_t run = tile_off[blockIdx.x] + wofs + inc - tsum;
    int32_t o[kScanItems];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        o[j] = run;
        run += v[j];
    }
    if (base + kScanItems <= nc) {
        int4 *p = reinterpret_cast<int4 *>(off + base);
#pragma unroll
        for (int q = 0; q < kScanItems / 4; ++q) p[q] = make_int4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
    } else {
#pragma unroll
        for (int j = 0; j < kScanItems; ++j)
            if (base + j < nc) off[base + j] = o[j];
    }
}

__global__ __launch_bounds__(kBlock) void k_bin_scatter(int32_t n, const int32_t *__restrict__ cell_in,
                                                        const int32_t *__restrict__ slot_in,
                                                        const int32_t *__restrict__ off,
                                                        int32_t *__restrict__ perm_u)
{
    const int32_t i = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    if (i >= n) return;
    const int32_t c = cell_in[i];
    if (c < 0) return;
    perm_u[off[c] + slot_in[i]] = i;
}

__global__ __launch_bounds__(kBlock) void k_bin_finalize(
    int32_t n, int64_t nc, const int32_t *__restrict__ perm_u, const int32_t *__restrict__ cell_in,
    const int32_t *__restrict__ off, const float *__restrict__ x, const float *__restrict__ y,
    const float *__restrict__ z, const float *__restrict__ w, GridDev g, int32_t *__restrict__ perm,
    int32_t *__restrict__ cell, float *__restrict__ xs, float *__restrict__ ys, float *__restrict__ zs,
    float *__restrict__ ws)
{
    const int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x);
    const int32_t nb = off[nc]; // particles inside the box
    if (k >= nb || k >= n) return;
    const int32_t p = perm_u[k];
    const int32_t c = cell_in[p];
    const int32_t s = off[c], e = off[c + 1];
    int32_t rank = 0;
    for (int32_t q = s; q < e; ++q) rank += (perm_u[q] < p) ? 1 : 0;
    const int32_t d = s + rank;
    const int32_t ix = c % g.nx;
    const int32_t iy = (c / g.nx) % g.ny;
    const int32_t iz = c / (g.nx * g.ny);
    perm[d] = p;
    cell[d] = c;
    xs[d] = __builtin_fmaf(-(float)ix, g.w, x[p] - g.ox);
    ys[d] = __builtin_fmaf(-(float)iy, g.w, y[p] - g.oy);
    zs[d] = __builtin_fmaf(-(float)iz, g.w, z[p] - g.oz);
    ws[d] = w[p];
}

inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

} // namespace

static bool grid_valid(const pi_grid *g)
{
    if (!g) return false;
    for (int a = 0; a < 3; ++a) {
        if (g->dims[a] < 1 || g->dims[a] > (1 << 24)) return false;
        if (!__builtin_isfinite(g->origin[a])) return false;
    }
    if ((int64_t)g->dims[0] * g->dims[1] * g->dims[2] >= ((int64_t)1 << 31)) return false;
    if (!(g->cell_w > 0.0f) || !__builtin_isfinite(g->cell_w)) return false;
    if (!(g->rc > 0.0f) || !__builtin_isfinite(g->rc)) return false;
    if (g->cell_w < g->rc) return false;
    return true;
}

extern "C" pi_status pi_bin(pi_ctx *ctx, pi_cells *cells, const float *x, const float *y, const float *z,
                            const float *w, int64_t n, const pi_grid *grid, pi_stream stream_)
{
    if (!ctx || !cells || cells->ctx != ctx) return PI_EINVAL;
    if (n < 0 || n >= ((int64_t)1 << 31)) return PI_EINVAL;
    if (n > 0 && (!x || !y || !z || !w)) return PI_EINVAL;
    if (!grid_valid(grid)) return PI_EINVAL;
    hipStream_t stream = (hipStream_t)stream_;
    PI_CHECK_HIP(hipSetDevice(ctx->device));
    const int64_t nc = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
    pi_status st = pi_ensure_capacity(cells, n, nc, stream);
    if (st != PI_OK) return st;
    cells->n = n;
    cells->n_cells = nc;
    cells->grid = *grid;
    cells->last_stream = stream;
    cells->binned = true;

    GridDev g;
    g.ox = grid->origin[0];
    g.oy = grid->origin[1];
    g.oz = grid->origin[2];
    g.w = grid->cell_w;
    g.nx = grid->dims[0];
    g.ny = grid->dims[1];
    g.nz = grid->dims[2];
    g.pad = 0;

    const int32_t ntiles = (int32_t)((nc + kScanTile - 1) / kScanTile);
    PI_LAUNCH(ctx, "k_fill_i32", k_fill_i32, dim3(nblocks(nc, kBlock)), dim3(kBlock), 0, stream, cells->counts, nc,
              0);
    if (n > 0)
        PI_LAUNCH(ctx, "k_bin_count", k_bin_count, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, stream, (int32_t)n, x,
                  y, z, g, cells->counts, cells->cell_in, cells->slot_in, cells->d_err);
    PI_LAUNCH(ctx, "k_scan_reduce", k_scan_reduce, dim3(ntiles), dim3(kBlock), 0, stream, cells->counts, nc,
              cells->tile_sum, cells->tile_max);
    PI_LAUNCH(ctx, "k_scan_tiles", k_scan_tiles, dim3(1), dim3(1024), 0, stream, cells->tile_sum, cells->tile_max,
              ntiles, cells->offsets + nc, cells->max_per_cell);
    PI_LAUNCH(ctx, "k_scan_down", k_scan_down, dim3(ntiles), dim3(kBlock), 0, stream, cells->counts, nc,
              cells->tile_sum, cells->offsets);
    if (n > 0) {
        PI_LAUNCH(ctx, "k_bin_scatter", k_bin_scatter, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, stream,
                  (int32_t)n, cells->cell_in, cells->slot_in, cells->offsets, cells->perm_u);
        PI_LAUNCH(ctx, "k_bin_finalize", k_bin_finalize, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, stream,
                  (int32_t)n, nc, cells->perm_u, cells->cell_in, cells->offsets, x, y, z, w, g, cells->perm,
                  cells->cell, cells->xs, cells->ys, cells->zs, cells->ws);
    }
    PI_CHECK_HIP(hipGetLastError());
    return PI_OK;
}
