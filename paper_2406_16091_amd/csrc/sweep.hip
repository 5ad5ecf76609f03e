// The 27-neighbour-cell interaction sweep (paper Sec. 2; Sec. 4.1 /
// Algorithm 1 for the cache-only organisation, Sec. 5.1 / Algorithm 4 and
// Sec. 5.2 / Algorithm 5 for the LDS-staged tiles).
//
// Every organisation walks a target's neighbour cells in the same canonical
// order -- (dz, dy, dx) lexicographic from -1, sources in sorted order -- and
// evaluates each candidate with the same code (pair.h), so all of them give
// bit-identical outputs.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "inv.h"
#include "pair.h"

namespace {

constexpr int kBlock = 256;

struct SweepArgs {
    const int32_t *off;
    const int32_t *cell;
    const int32_t *perm;
    const float4 *p4; // sorted cell-relative (x, y, z, w), one record per slot
    int64_t nc;
    int32_t n;
    int32_t nx, ny, nz;
    int32_t orig_order;
    float *rho, *gx, *gy, *gz;
    int32_t *count;
    InvPartial *partials;
    // single-system tiles: per tile, 1 if its halo overflowed the LDS area
    // and its targets are left to the dense pass; a word that a launch whose
    // tiles overflowed sets to its epoch (a number the host gives each tile
    // launch on a cell object, from the counter at host_epoch)
    uint8_t *tflag;
    uint32_t *ovf;
    uint32_t epoch;
    uint32_t *host_epoch; // host memory, not read by the kernels
    // no-LDS walk: > 0 skips the targets of cells holding at least this many
    // particles (the cell-SM pass takes them)
    int32_t dense_min;
    KernelConst k;
    // batch mode: system table, per-system kernel constants
    const SysDev *sys;
    const KernelConst *kcs;
    int32_t nsys;
};

// Batch mode: the system owning logical workgroup lb; narrows the sweep
// arguments to that system (its grid, cell offsets and kernel constants).
__device__ __forceinline__ int enter_system(SweepArgs &a, uint32_t lb)
{
    int lo = 0, hi = a.nsys; // sys[lo].block_base <= lb < sys[hi].block_base
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((uint32_t)a.sys[mid].block_base <= lb) lo = mid; else hi = mid;
    }
    const SysDev &sd = a.sys[lo];
    a.nx = sd.g.nx;
    a.ny = sd.g.ny;
    a.nz = sd.g.nz;
    a.nc = (int64_t)sd.g.nx * sd.g.ny * sd.g.nz;
    a.off += sd.cell_base;
    a.k = a.kcs[lo];
    return lo;
}

template <int PREC, bool INV>
__device__ __forceinline__ void write_target(const SweepArgs &a, int32_t k, const Target<PREC, INV> &T)
{
    const int32_t o = a.orig_order ? a.perm[k] : k;
    if (a.rho) {
        a.rho[o] = T.acc.r_rho();
        a.gx[o] = T.acc.r_gx();
        a.gy[o] = T.acc.r_gy();
        a.gz[o] = T.acc.r_gz();
    }
    if (a.count) a.count[o] = T.count;
}

// FP64 block reduction of the invariant partials (256 threads).
__device__ __forceinline__ void reduce_invariants(const SweepArgs &a, uint32_t slot, long long cnt, double nx,
                                                  double ny, double nz, double sc, double rs)
{
    block_reduce_partial(a.partials + slot, cnt, nx, ny, nz, sc, rs);
}

// The same reduction through LDS for workgroups that have a free LDS area of
// at least 12 KB (256 lanes x 6 doubles): every lane parks its partials, and
// the first wavefront alone folds the 256 entries (4 per lane, then a wave
// butterfly), so the other wavefronts skip the butterfly.  The order of the
// additions is fixed, so the result is deterministic.
__device__ __forceinline__ void reduce_invariants_lds(const SweepArgs &a, uint32_t slot, long long cnt, double nx,
                                                      double ny, double nz, double sc, double rs, double *park)
{
    const int t = threadIdx.x;
    __syncthreads(); // the area may still be read by other lanes
    park[0 * kBlock + t] = (double)cnt;
    park[1 * kBlock + t] = nx;
    park[2 * kBlock + t] = ny;
    park[3 * kBlock + t] = nz;
    park[4 * kBlock + t] = sc;
    park[5 * kBlock + t] = rs;
    __syncthreads();
    if (t >= 64) return;
    double v[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
        const double *col = park + q * kBlock;
        v[q] = (col[t] + col[t + 64]) + (col[t + 128] + col[t + 192]);
    }
    for (int o = 32; o >= 1; o >>= 1) {
#pragma unroll
        for (int q = 0; q < 6; ++q) v[q] += __shfl_xor(v[q], o, 64);
    }
    if (t == 0) {
        InvPartial p;
        p.pairs = (long long)v[0];
        p.net[0] = v[1];
        p.net[1] = v[2];
        p.net[2] = v[3];
        p.scale = v[4];
        p.rho_sum = v[5];
        p.pad[0] = p.pad[1] = 0.0;
        a.partials[slot] = p;
    }
}

template <int PREC, bool INV>
__device__ __forceinline__ void target_invariants(const Target<PREC, INV> &T, float wi, long long &cnt,
                                                  double &nx, double &ny, double &nz, double &sc, double &rs)
{
    const double w = (double)wi;
    cnt = T.count;
    nx = w * (double)T.acc.r_gx();
    ny = w * (double)T.acc.r_gy();
    nz = w * (double)T.acc.r_gz();
    sc = w * (double)T.ascale;
    rs = (double)T.acc.r_rho();
}

// ------------------------------------------------------------------ no LDS
// One thread per sorted target; sources read through L1/L2 (Algorithm 1,
// Par-Part-NoLoop, with targets in cell-sorted order so that a wavefront's
// neighbour rows overlap in cache).  Each neighbour X-row is walked as one
// index range over its (up to) three cells, so a wavefront's loop runs as
// long as its longest row rather than its longest cell, three times a row;
// cells beyond the cutoff's reach are trimmed as in the tiles.  The sources
// and their order are those of the 27-cell walk, so the results are too.
template <int PREC, bool INV, bool BATCH>
__global__ __launch_bounds__(kBlock) void k_sweep_nolds(SweepArgs a)
{
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    int32_t k, kend;
    if (BATCH) {
        const SysDev &sd = a.sys[enter_system(a, lb)];
        k = (int32_t)sd.first + (int32_t)(lb - sd.block_base) * kBlock + (int32_t)threadIdx.x;
        kend = (int32_t)sd.first + sd.n;
    } else {
        k = (int32_t)(lb * kBlock + threadIdx.x);
        kend = min(a.off[a.nc], a.n);
    }
    bool active = k < kend;
    if (!BATCH && active && a.dense_min > 0) {
        const int32_t c = a.cell[k];
        active = a.off[c + 1] - a.off[c] < a.dense_min;
    }
    Target<PREC, INV> T;
    float wi = 0.f;
    if (active) {
        const int32_t c = a.cell[k];
        const int32_t ix = c % a.nx, iy = (c / a.nx) % a.ny, iz = c / (a.nx * a.ny);
        const float4 pk = a.p4[k];
        const float xi = pk.x, yi = pk.y, zi = pk.z;
        wi = pk.w;
        const float W = a.k.w;
        const float reach2 = a.k.reach2;
        // the target in the frame of its left and right neighbour cells
        const float xm = xi - (float)(-1) * W, xp = xi - (float)(1) * W;
        // the reach test of the tiles: a neighbour cell whose nearest face is
        // surely beyond the cutoff is skipped (no pair there is accepted), and
        // the left (right) cell of a row is kept iff gyz < tl (tr)
        const float gyl = yi * yi, gyr = (W - yi) * (W - yi);
        const float gzl = zi * zi, gzr = (W - zi) * (W - zi);
        const float tl = ix > 0 ? reach2 - xi * xi : -1.0f;
        const float tr = ix + 1 < a.nx ? reach2 - (W - xi) * (W - xi) : -1.0f;
        // each X-row's (up to) three cells are one index range, walked in
        // one loop; the two inner cell boundaries give each source's shift
        for (int dz = -1; dz <= 1; ++dz) {
            const int32_t cz = iz + dz;
            if (cz < 0 || cz >= a.nz) continue;
            const float tz = zi - (float)dz * W;
            const float gz = dz < 0 ? gzl : (dz > 0 ? gzr : 0.f);
            for (int dy = -1; dy <= 1; ++dy) {
                const int32_t cy = iy + dy;
                if (cy < 0 || cy >= a.ny) continue;
                const float gyz = (dy < 0 ? gyl : (dy > 0 ? gyr : 0.f)) + gz;
                if (gyz >= reach2) continue; // the whole row is out of reach
                const float ty = yi - (float)dy * W;
                const int64_t rb = (int64_t)a.nx * (cy + (int64_t)a.ny * cz) + ix;
                const int32_t b1 = a.off[rb], b2 = a.off[rb + 1];
                const int32_t j0 = gyz < tl ? a.off[rb - 1] : b1;
                const int32_t j3 = gyz < tr ? a.off[rb + 2] : b2;
                for (int32_t j = j0; j < j3; ++j) {
                    const float tx = j < b1 ? xm : (j < b2 ? xi : xp);
                    const float4 s = a.p4[j];
                    const float ddx = tx - s.x, ddy = ty - s.y, ddz = tz - s.z;
                    const float t = sq_dist(ddx, ddy, ddz);
                    if (t < a.k.hi && j != k && inside_cutoff(ddx, ddy, ddz, t, a.k))
                        T.accept(ddx, ddy, ddz, t, s.w, a.k);
                }
            }
        }
        write_target(a, k, T);
    }
    if (INV) {
        long long cnt = 0;
        double nx = 0, ny = 0, nz = 0, sc = 0, rs = 0;
        if (active) target_invariants(T, wi, cnt, nx, ny, nz, sc, rs);
        reduce_invariants(a, lb, cnt, nx, ny, nz, sc, rs);
    }
}

// ------------------------------------------------------------------ stream
// One thread per sorted target with sources read through the caches, as in
// NOLDS (the same trimmed X-row walk, one row of the 9 at a time for the
// whole wavefront), but with candidate testing decoupled from pair
// evaluation by a per-lane LDS FIFO as in the tiles: the test of one
// candidate is a few instructions, the evaluation of an accepted pair about a
// hundred, and at several particles per cell some lane of a wavefront
// accepts on nearly every step.  A queue entry holds the differences the
// test computed and the source's weight, so a pop reads nothing from global
// memory and evaluates the same values.  Nothing is staged, so the
// organisation works at any occupancy.
template <int Q, int PREC, bool INV, bool BATCH>
__global__ __launch_bounds__(kBlock) void k_sweep_stream(SweepArgs a)
{
    static_assert((Q & (Q - 1)) == 0, "FIFO depth must be a power of two");
    __shared__ float4 fifo[kBlock / 64][Q][64];   // accepted pair: (dx, dy, dz, w_j)

    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    int32_t k, kend;
    if (BATCH) {
        const SysDev &sd = a.sys[enter_system(a, lb)];
        k = (int32_t)sd.first + (int32_t)(lb - sd.block_base) * kBlock + (int32_t)threadIdx.x;
        kend = (int32_t)sd.first + sd.n;
    } else {
        k = (int32_t)(lb * kBlock + threadIdx.x);
        kend = min(a.off[a.nc], a.n);
    }
    const bool active = k < kend;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const float W = a.k.w;
    const float reach2 = a.k.reach2;
    float xi = 0.f, yi = 0.f, zi = 0.f, wi = 0.f;
    int32_t ix = 0, iy = 0, iz = 0;
    if (active) {
        const int32_t c = a.cell[k];
        ix = c % a.nx;
        iy = (c / a.nx) % a.ny;
        iz = c / (a.nx * a.ny);
        const float4 pk = a.p4[k];
        xi = pk.x;
        yi = pk.y;
        zi = pk.z;
        wi = pk.w;
    }
    // the target in the frame of a neighbour cell: x - d W for d = -1, 0, 1
    // (the same roundings as the no-LDS walk)
    const float xm = xi - (float)(-1) * W, xp = xi - (float)(1) * W;
    const float ym = yi - (float)(-1) * W, yp = yi - (float)(1) * W;
    const float zm = zi - (float)(-1) * W, zp = zi - (float)(1) * W;
    auto sel = [](int q, float m, float o, float p) { return q == 0 ? m : (q == 1 ? o : p); };
    const float gyl = yi * yi, gyr = (W - yi) * (W - yi);
    const float gzl = zi * zi, gzr = (W - zi) * (W - zi);
    const float tl = ix > 0 ? reach2 - xi * xi : -1.0f;
    const float tr = ix + 1 < a.nx ? reach2 - (W - xi) * (W - xi) : -1.0f;

    Target<PREC, INV> T;
    float4 *myq = &fifo[wid][0][lane];
    int qh = 0, qc = 0;
    auto pop = [&]() {
        const float4 e = myq[qh * 64];
        qh = (qh + 1) & (Q - 1);
        --qc;
        T.template accept<true>(e.x, e.y, e.z, sq_dist(e.x, e.y, e.z), e.w, a.k);
    };
    for (int dz = -1; dz <= 1; ++dz) {
        const float tz = dz < 0 ? zm : (dz > 0 ? zp : zi);
        const float gz = dz < 0 ? gzl : (dz > 0 ? gzr : 0.f);
        const bool zok = active && iz + dz >= 0 && iz + dz < a.nz;
        for (int dy = -1; dy <= 1; ++dy) {
            const float ty = dy < 0 ? ym : (dy > 0 ? yp : yi);
            const float gyz = (dy < 0 ? gyl : (dy > 0 ? gyr : 0.f)) + gz;
            // this lane's range of the row (empty if the row is outside the
            // grid or out of reach) and its two inner cell boundaries
            int32_t j = 0, j3 = 0, b1 = 0, b2 = 0;
            if (zok && iy + dy >= 0 && iy + dy < a.ny && gyz < reach2) {
                const int64_t rb = (int64_t)a.nx * ((iy + dy) + (int64_t)a.ny * (iz + dz)) + ix;
                b1 = a.off[rb];
                b2 = a.off[rb + 1];
                j = gyz < tl ? a.off[rb - 1] : b1;
                j3 = gyz < tr ? a.off[rb + 2] : b2;
            }
            // tests until some lane's queue is full (the accumulators are
            // not touched in this inner loop, which keeps it free of
            // register copies), then one round of pops.  The lanes walk the
            // same row together, so their loads fall on neighbouring cells
            // (walking each lane's rows as one sequence, so that the loop
            // runs to the longest lane total instead of the sum of the
            // longest rows, scattered the loads over rows and was 1.5x
            // slower at 8 per cell).
            while (__any(j < j3)) {
                do {
                    if (j < j3) {
                        const int dxc = j < b1 ? 0 : (j < b2 ? 1 : 2);
                        const float4 s = a.p4[j];
                        const float ddx = sel(dxc, xm, xi, xp) - s.x, ddy = ty - s.y, ddz = tz - s.z;
                        const float t = sq_dist(ddx, ddy, ddz);
                        bool acc = t < a.k.lo;
                        if (t >= a.k.lo && t < a.k.hi) acc = h2_minus_d2(ddx, ddy, ddz, a.k) > 0.0f;
                        if (acc && j != k) {
                            myq[((qh + qc) & (Q - 1)) * 64] = make_float4(ddx, ddy, ddz, s.w);
                            ++qc;
                        }
                        ++j;
                    }
                } while (!__any(qc == Q) && __any(j < j3));
                if (__any(qc == Q)) {
                    if (qc > 0) pop();
                }
            }
        }
    }
    for (int left = wave_max(qc); left > 0; --left) {
        if (qc > 0) pop();
    }
    if (active) write_target(a, k, T);
    if (INV) {
        long long cnt = 0;
        double nx = 0, ny = 0, nz = 0, sc = 0, rs = 0;
        if (active) target_invariants(T, wi, cnt, nx, ny, nz, sc, rs);
        reduce_invariants(a, lb, cnt, nx, ny, nz, sc, rs);
    }
}

// ------------------------------------------------------------------ LDS tiles
// A workgroup owns a tile of TX x TY x TZ target cells.  The tile's halo box
// ((TX+2) x (TY+2) x (TZ+2) cells, clipped to the grid) is staged in LDS:
// each X-row of the halo is one contiguous range of the sorted arrays, so
// the load is (TY+2)(TZ+2) coalesced row copies.  The LDS position of every
// row comes from an exclusive scan of the row counts, which are differences
// of global offsets (the paper's local-offset construction, Sec. 5.1).
// TY = TZ = 1 is the X-pencil (Sec. 5.2), with all nine neighbour pencils
// resident at once instead of streamed; larger TY, TZ is the full sub-box
// (Sec. 5.1).
//
// Staged coordinates are relative to the corner of the halo box, so the
// difference of two staged positions is the pair's difference vector (exact
// for positions on a power-of-two lattice with a power-of-two cell width,
// and then bit-identical to the cell-relative differences of the other
// organisations), and the (up to) three cells a target needs from one X-row
// form a single range: 9 row segments per target instead of 27 cells.  Each
// lane first writes its target's non-empty segments, in canonical order,
// into an LDS table; a neighbour cell whose nearest face is provably beyond
// the cutoff (a conservative test in squared distances) is left out of its
// segment, which removes about a quarter of the candidates without changing
// which pairs are accepted or their order.
//
// Candidate testing and pair evaluation are decoupled: each lane walks its
// segments in lockstep with the wavefront and pushes the staging-area byte
// offset of every accepted source into a private FIFO of Q entries in LDS
// (segments and queue entries are byte offsets, so no step scales an index);
// whenever some
// lane's FIFO is full, the wavefront pops one entry per non-empty lane and
// evaluates the kernel.  Otherwise the wavefront would run the long
// evaluation on almost every candidate step (about one candidate in six is
// accepted, so some lane of 64 nearly always accepts).  FIFO order keeps each
// target's accumulation order canonical, so results stay bit-identical to the
// other organisations.
//
// A tile whose halo holds more than CAP particles is flagged and left to the
// dense pass, which walks each of its targets from global memory with the
// row walk of the no-LDS sweep (each neighbour X-row's up to three cells as
// one range, cells surely beyond the cutoff trimmed; same sources, same
// order, same roundings, so the same results).
template <int PREC, bool INV>
__device__ __forceinline__ void walk_rows_global(const SweepArgs &a, int32_t k, int32_t ix, int32_t iy, int32_t iz,
                                                 float xi, float yi, float zi, Target<PREC, INV> &T)
{
    const float W = a.k.w;
    const float reach2 = a.k.reach2;
    const float xm = xi - (float)(-1) * W, xp = xi - (float)(1) * W;
    const float gyl = yi * yi, gyr = (W - yi) * (W - yi);
    const float gzl = zi * zi, gzr = (W - zi) * (W - zi);
    const float tl = ix > 0 ? reach2 - xi * xi : -1.0f;
    const float tr = ix + 1 < a.nx ? reach2 - (W - xi) * (W - xi) : -1.0f;
    for (int dz = -1; dz <= 1; ++dz) {
        const int32_t cz = iz + dz;
        if (cz < 0 || cz >= a.nz) continue;
        const float tz = zi - (float)dz * W;
        const float gz = dz < 0 ? gzl : (dz > 0 ? gzr : 0.f);
        for (int dy = -1; dy <= 1; ++dy) {
            const int32_t cy = iy + dy;
            if (cy < 0 || cy >= a.ny) continue;
            const float gyz = (dy < 0 ? gyl : (dy > 0 ? gyr : 0.f)) + gz;
            if (gyz >= reach2) continue;
            const float ty = yi - (float)dy * W;
            const int64_t rb = (int64_t)a.nx * (cy + (int64_t)a.ny * cz) + ix;
            const int32_t b1 = a.off[rb], b2 = a.off[rb + 1];
            const int32_t j0 = gyz < tl ? a.off[rb - 1] : b1;
            const int32_t j3 = gyz < tr ? a.off[rb + 2] : b2;
            for (int32_t j = j0; j < j3; ++j) {
                const float tx = j < b1 ? xm : (j < b2 ? xi : xp);
                const float4 s = a.p4[j];
                const float ddx = tx - s.x, ddy = ty - s.y, ddz = tz - s.z;
                const float t = sq_dist(ddx, ddy, ddz);
                if (t < a.k.hi && j != k && inside_cutoff(ddx, ddy, ddz, t, a.k))
                    T.accept(ddx, ddy, ddz, t, s.w, a.k);
            }
        }
    }
}

template <int TX, int TY, int TZ, int CAP, int Q, int PREC, bool INV, bool BATCH>
__global__ __launch_bounds__(kBlock) void k_sweep_tile(SweepArgs a, int32_t ntx, int32_t nty)
{
    constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
    constexpr int R = HY * HZ;   // halo rows
    constexpr int TR = TY * TZ;  // target rows
    static_assert(R <= 64 && TR <= 64, "row tables are scanned by one wavefront");
    static_assert((Q & (Q - 1)) == 0, "FIFO depth must be a power of two");
    static_assert(CAP * 16 < 65536, "segment table packs byte offsets in 16 bits");
    __shared__ float4 sp[CAP];
    // accepted source: its byte offset in the staging area
    __shared__ uint32_t fifo[kBlock / 64][Q][64];
    // staging-area byte ranges of the row segments (start | end << 16); the
    // target's own row is cut in two around the target itself, so at most 10
    __shared__ uint32_t segtab[10][kBlock];
    // staging-area byte offset of every halo cell's first particle
    __shared__ int32_t cs[R][HX + 1];
    // halo row of every staged slot, and target row of every target
    __shared__ uint8_t hrow[CAP];
    __shared__ uint8_t trow[CAP];
    __shared__ int32_t rstart[R + 1];
    __shared__ int32_t gstart[R];
    __shared__ int32_t rbase[R];
    __shared__ int32_t tstart[TR + 1];
    __shared__ int32_t tfirst[TR];

    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    uint32_t tl = lb; // tile index within its system
    if (BATCH) {
        const SysDev &sd = a.sys[enter_system(a, lb)];
        tl = lb - (uint32_t)sd.block_base;
        ntx = sd.ntx;
        nty = sd.nty;
        // the system's workgroups past its tiles belong to its dense pass
        if (tl >= (uint32_t)(ntx * nty * ((a.nz + TZ - 1) / TZ))) return;
    }
    const int32_t bx = (int32_t)(tl % (uint32_t)ntx);
    const int32_t by = (int32_t)((tl / (uint32_t)ntx) % (uint32_t)nty);
    const int32_t bz = (int32_t)(tl / ((uint32_t)ntx * (uint32_t)nty));
    const int32_t x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    const int32_t cxlo = max(x0 - 1, 0);
    const int32_t cxhi = min(x0 + TX, a.nx - 1);
    const int32_t ncx = cxhi - cxlo + 1;
    const int32_t txhi = min(x0 + TX, a.nx); // exclusive end of target cells
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const float W = a.k.w;

    // 1. halo row ranges and their LDS starts; target row ranges
    if (tid < 64) {
        int32_t cnt = 0, gs = 0, rb32 = 0;
        if (tid < R) {
            const int32_t y = y0 - 1 + tid % HY, z = z0 - 1 + tid / HY;
            if (y >= 0 && y < a.ny && z >= 0 && z < a.nz) {
                const int64_t rb = (int64_t)a.nx * (y + (int64_t)a.ny * z);
                rb32 = (int32_t)rb;
                gs = a.off[rb + cxlo];
                cnt = a.off[rb + cxhi + 1] - gs;
            }
        }
        const int32_t inc = wave_incl_scan(cnt);
        if (tid < R) {
            rstart[tid] = inc - cnt;
            gstart[tid] = gs;
            rbase[tid] = rb32;
            for (int32_t f = inc - cnt; f < min(inc, CAP); ++f) hrow[f] = (uint8_t)tid;
        }
        if (tid == R - 1) rstart[R] = inc;

        int32_t tc = 0, tf = 0;
        if (tid < TR) {
            const int32_t y = y0 + tid % TY, z = z0 + tid / TY;
            if (y < a.ny && z < a.nz && x0 < a.nx) {
                const int64_t rb = (int64_t)a.nx * (y + (int64_t)a.ny * z);
                tf = a.off[rb + x0];
                tc = a.off[rb + txhi] - tf;
            }
        }
        const int32_t tinc = wave_incl_scan(tc);
        if (tid < TR) {
            tstart[tid] = tinc - tc;
            tfirst[tid] = tf;
            for (int32_t f = tinc - tc; f < min(tinc, CAP); ++f) trow[f] = (uint8_t)tid;
        }
        if (tid == TR - 1) tstart[TR] = tinc;
    }
    __syncthreads();
    const int32_t total = rstart[R];
    const int32_t ntarget = tstart[TR];
    long long icnt = 0;
    double inx = 0, iny = 0, inz = 0, isc = 0, irs = 0;

    if (tid == 0) a.tflag[lb] = total > CAP ? 1 : 0;
    if (total > CAP) {
        // halo too large for LDS: the dense pass (k_sweep_dense, or
        // k_sweep_dense_batch for a batch) takes this tile's targets, one
        // thread each across the system, so a dense region is not left to
        // one workgroup
        if (!BATCH && tid == 0) *a.ovf = a.epoch;
        if (INV) reduce_invariants(a, lb, 0, 0.0, 0.0, 0.0, 0.0, 0.0);
        return;
    }

    // 2. LDS start of every halo cell
    for (int e = tid; e < R * (HX + 1); e += kBlock) {
        const int r = e / (HX + 1), jj = e % (HX + 1);
        const int32_t y = y0 - 1 + r % HY, z = z0 - 1 + r / HY;
        int32_t v = 0;
        if (jj <= ncx && y >= 0 && y < a.ny && z >= 0 && z < a.nz)
            v = a.off[(int64_t)rbase[r] + cxlo + jj] - gstart[r] + rstart[r];
        cs[r][jj] = v * (int32_t)sizeof(float4);
    }
    // 3. stage the halo particles in tile-relative coordinates: offsets from
    //    the corner of the halo box clipped to the grid (cell (cxlo,
    //    max(y0 - 1, 0), max(z0 - 1, 0))), so that a difference of two staged
    //    positions is the pair's difference vector with no per-row shift, and
    //    every staged coordinate lies inside the grid's extent (exact whenever
    //    the positions are, measured from the grid's origin)
    const int yoff = y0 > 0 ? 0 : 1, zoff = z0 > 0 ? 0 : 1;
    for (int32_t f = tid; f < total; f += kBlock) {
        const int lo = hrow[f]; // rstart[lo] <= f < rstart[lo + 1]
        const int32_t g = gstart[lo] + (f - rstart[lo]);
        const int32_t cx = a.cell[g] - rbase[lo];
        const float4 q = a.p4[g];
        sp[f] = make_float4(__builtin_fmaf((float)(cx - cxlo), W, q.x),
                            __builtin_fmaf((float)(lo % HY - yoff), W, q.y),
                            __builtin_fmaf((float)(lo / HY - zoff), W, q.z), q.w);
    }
    __syncthreads();

    // 4. targets, in rounds of one per thread
    uint32_t *myq = &fifo[wid][0][lane];
    const char *spb = reinterpret_cast<const char *>(sp);
    auto staged = [&](uint32_t byte) { return *reinterpret_cast<const float4 *>(spb + byte); };
    const float reach2 = a.k.reach2; // conservative squared reach
    for (int32_t f0 = 0; f0 < ntarget; f0 += kBlock) {
        const int32_t f = f0 + tid;
        const bool tgt = f < ntarget;
        int32_t k = 0, self = -1, nseg = 0;
        float xt = 0.f, yt = 0.f, zt = 0.f, wi = 0.f;
        if (tgt) {
            const int lo = trow[f]; // tstart[lo] <= f < tstart[lo + 1]
            k = tfirst[lo] + (f - tstart[lo]);
            const int32_t ty_ = lo % TY, tz_ = lo / TY;
            const int32_t y = y0 + ty_, z = z0 + tz_;
            const int32_t ix = a.cell[k] - a.nx * (y + a.ny * z);
            const int hr = (ty_ + 1) + HY * (tz_ + 1);
            self = rstart[hr] + (k - gstart[hr]);
            const int32_t selfb = self * (int32_t)sizeof(float4);
            const float4 p = sp[self];
            xt = p.x; yt = p.y; zt = p.z; wi = p.w;
            // cell-relative position of the target, for the reach test
            const float4 pk = a.p4[k];
            const float xc = pk.x, yc = pk.y, zc = pk.z;
            const float gxl = xc * xc, gxr = (W - xc) * (W - xc);
            const float gyl = yc * yc, gyr = (W - yc) * (W - yc);
            const float gzl = zc * zc, gzr = (W - zc) * (W - zc);
            const int32_t jc = ix - cxlo;
            // the left (right) cell of a row is kept iff gyz < tl (tr): the
            // same test as gx + gyz < reach2 up to one rounding, which the
            // 16u margin of reach2 covers (a missing neighbour cell: -1)
            const float tl = ix > 0 ? reach2 - gxl : -1.0f;
            const float tr = ix + 1 < a.nx ? reach2 - gxr : -1.0f;
            const bool zlo = z > 0, zhi = z + 1 < a.nz, ylo = y > 0, yhi = y + 1 < a.ny;
            // the target's own cell in its own halo row; a neighbour row is a
            // compile-time offset from it
            const int32_t *own = &cs[(ty_ + 1) + HY * (tz_ + 1)][jc];
            uint32_t *segp = &segtab[0][tid];
            // segments in canonical (dz, dy) order
            for (int dz = -1; dz <= 1; ++dz) {
                if (dz < 0 ? !zlo : (dz > 0 && !zhi)) continue;
                const float gz = dz < 0 ? gzl : (dz > 0 ? gzr : 0.f);
                for (int dy = -1; dy <= 1; ++dy) {
                    if (dy < 0 ? !ylo : (dy > 0 && !yhi)) continue;
                    const float gyz = (dy < 0 ? gyl : (dy > 0 ? gyr : 0.f)) + gz;
                    if (gyz >= reach2) continue; // the whole row is out of reach
                    const bool left = gyz < tl;
                    const bool right = gyz < tr;
                    const int32_t *row = own + (dy + HY * dz) * (HX + 1);
                    const int32_t s0 = row[left ? -1 : 0];
                    const int32_t s1 = row[right ? 2 : 1];
                    // (byte offsets: start | end << 16)
                    if (dy == 0 && dz == 0) {
                        // s0 <= self < s1: the parts before and after it
                        const int32_t after = selfb + (int32_t)sizeof(float4);
                        if (selfb > s0) {
                            *segp = (uint32_t)s0 | ((uint32_t)selfb << 16);
                            segp += kBlock;
                        }
                        if (s1 > after) {
                            *segp = (uint32_t)after | ((uint32_t)s1 << 16);
                            segp += kBlock;
                        }
                    } else if (s1 > s0) {
                        *segp = (uint32_t)s0 | ((uint32_t)s1 << 16);
                        segp += kBlock;
                    }
                }
            }
            nseg = (int32_t)((segp - &segtab[0][tid]) / kBlock);
        }
        Target<PREC, INV> T;
        int seg = 0;
        uint32_t j = 0, jend = 0; // byte offsets in the staging area
        // Queue positions count entries pushed (qt) and popped (qh) in units
        // of one queue row (64 lanes x 4 bytes), so that (position & kQMask)
        // is the byte offset of the entry in this lane's column; qlim = qh + Q
        // rows marks a full queue.
        constexpr uint32_t kRow = 64u * (uint32_t)sizeof(uint32_t);
        constexpr uint32_t kQMask = (uint32_t)(Q - 1) * kRow;
        uint32_t qt = 0, qh = 0, qlim = (uint32_t)Q * kRow;
        char *myqb = reinterpret_cast<char *>(myq);
        // Evaluate the oldest queued pair of this lane: the differences are
        // recomputed from the same operands, so they are bit-identical to the
        // ones the test used.
        auto pop = [&]() {
            const uint32_t e = *reinterpret_cast<const uint32_t *>(myqb + (qh & kQMask));
            qh += kRow;
            qlim += kRow;
            const float4 s = staged(e);
            const float ddx = xt - s.x, ddy = yt - s.y, ddz = zt - s.z;
            T.template accept<true>(ddx, ddy, ddz, sq_dist(ddx, ddy, ddz), s.w, a.k);
        };
        while (true) {
            if (j >= jend && seg < nseg) {
                const uint32_t sg = segtab[seg][tid];
                ++seg;
                j = sg & 0xffffu;
                jend = sg >> 16;
            }
            const bool have = j < jend;
            if (!__any(have)) break;
            if (have) {
                const float4 s = staged(j);
                const float ddx = xt - s.x, ddy = yt - s.y, ddz = zt - s.z;
                const float t = sq_dist(ddx, ddy, ddz);
                // surely inside below lo; the thin band [lo, hi) takes the
                // exact test (inside_cutoff, unrolled to keep the step short)
                bool acc = t < a.k.lo;
                const bool below_hi = t < a.k.hi;
                if (below_hi && !acc) acc = h2_minus_d2(ddx, ddy, ddz, a.k) > 0.0f;
                // the slot after the queue's tail is free (the queue is
                // never full at this point), so it is written always and
                // kept if accepted
                *reinterpret_cast<uint32_t *>(myqb + (qt & kQMask)) = j;
                qt += acc ? kRow : 0u;
                j += (uint32_t)sizeof(float4);
            }
            if (__any(qt == qlim)) {
                if (qt != qh) pop();
            }
        }
        // drain: as many rounds as the fullest queue holds (a uniform count)
        for (int left = wave_max((int)((qt - qh) / kRow)); left > 0; --left) {
            if (qt != qh) pop();
        }
        if (tgt) {
            write_target(a, k, T);
            if (INV) {
                long long c1;
                double a1, a2, a3, a4, a5;
                target_invariants(T, wi, c1, a1, a2, a3, a4, a5);
                icnt += c1; inx += a1; iny += a2; inz += a3; isc += a4; irs += a5;
            }
        }
    }
    static_assert(sizeof(float4) * CAP >= sizeof(double) * 6 * kBlock, "the staging area parks the partials");
    if (INV) reduce_invariants_lds(a, lb, icnt, inx, iny, inz, isc, irs, reinterpret_cast<double *>(sp));
}

// ------------------------------------------------------------------ pencil-reg
// The X-pencil-reg organisation (Sec. 5.3): a workgroup owns a sub-box of
// TX x TY x TZ target cells, and each thread keeps one target in registers
// (targets beyond 256 are taken in further rounds).  The halo's source
// X-pencils are then streamed through LDS one Z-sheet at a time (the HY
// pencils of one z, clipped to the grid): a particle of a target cell of
// the current round is copied into the sheet by the thread that holds it,
// every other particle is read from global memory.  After each sheet is
// staged, every target within one cell of it in z walks the three cells
// around it in each of its three rows of the sheet.  Sheets go in z order,
// rows in y order, cells in x order and particles in sorted order, so each
// target sees its 27 cells in the canonical order and the outputs are
// those of every other organisation.  A sub-box whose largest sheet holds
// more than SCAP particles is left to the dense pass, like an overflowing
// tile.
template <int TX, int TY, int TZ, int SCAP, int PREC, bool INV, bool BATCH>
__global__ __launch_bounds__(kBlock) void k_sweep_pencilreg(SweepArgs a, int32_t ntx, int32_t nty)
{
    constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
    constexpr int TR = TY * TZ; // target rows
    static_assert(HY * HZ <= 64 && TR <= 64, "row tables are scanned by one wavefront");
    __shared__ float4 sp[SCAP];
    __shared__ int32_t cs[HY][HX + 1]; // staged index of each cell's first particle in the sheet
    __shared__ int32_t rstart[HY + 1], gstart[HY], rbase[HY];
    __shared__ int32_t tstart[TR + 1], tfirst[TR];
    __shared__ int32_t sheetmax;

    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    uint32_t tl = lb;
    if (BATCH) {
        const SysDev &sd = a.sys[enter_system(a, lb)];
        tl = lb - (uint32_t)sd.block_base;
        ntx = sd.ntx;
        nty = sd.nty;
        // the system's workgroups past its tiles belong to its dense pass
        if (tl >= (uint32_t)(ntx * nty * ((a.nz + TZ - 1) / TZ))) return;
    }
    const int32_t bx = (int32_t)(tl % (uint32_t)ntx);
    const int32_t by = (int32_t)((tl / (uint32_t)ntx) % (uint32_t)nty);
    const int32_t bz = (int32_t)(tl / ((uint32_t)ntx * (uint32_t)nty));
    const int32_t x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    const int32_t cxlo = max(x0 - 1, 0), cxhi = min(x0 + TX, a.nx - 1);
    const int32_t txhi = min(x0 + TX, a.nx);
    const int32_t ylo = max(y0 - 1, 0), zlo = max(z0 - 1, 0); // the staging frame's corner
    const int tid = threadIdx.x;
    const float W = a.k.w;

    // 1. target rows, and the largest sheet of the halo
    if (tid < 64) {
        int32_t tc = 0, tf = 0;
        if (tid < TR) {
            const int32_t y = y0 + tid % TY, z = z0 + tid / TY;
            if (y < a.ny && z < a.nz && x0 < a.nx) {
                const int64_t rb = (int64_t)a.nx * (y + (int64_t)a.ny * z);
                tf = a.off[rb + x0];
                tc = a.off[rb + txhi] - tf;
            }
        }
        const int32_t tinc = wave_incl_scan(tc);
        if (tid < TR) {
            tstart[tid] = tinc - tc;
            tfirst[tid] = tf;
        }
        if (tid == TR - 1) tstart[TR] = tinc;
        // halo row (y, z) counts, summed per sheet
        int32_t sheet = 0;
        if (tid < HZ) {
            const int32_t z = z0 - 1 + tid;
            if (z >= 0 && z < a.nz)
                for (int r = 0; r < HY; ++r) {
                    const int32_t y = y0 - 1 + r;
                    if (y < 0 || y >= a.ny) continue;
                    const int64_t rb = (int64_t)a.nx * (y + (int64_t)a.ny * z);
                    sheet += a.off[rb + cxhi + 1] - a.off[rb + cxlo];
                }
        }
        sheet = wave_max(sheet);
        if (tid == 0) sheetmax = sheet;
    }
    __syncthreads();
    const int32_t ntarget = tstart[TR];
    const bool overflow = sheetmax > SCAP;
    long long icnt = 0;
    double inx = 0, iny = 0, inz = 0, isc = 0, irs = 0;
    if (tid == 0) a.tflag[lb] = overflow ? 1 : 0;
    if (overflow) {
        if (!BATCH && tid == 0) *a.ovf = a.epoch;
        if (INV) reduce_invariants(a, lb, 0, 0.0, 0.0, 0.0, 0.0, 0.0);
        return;
    }
    auto target_row = [&](int32_t f) {
        int tr = 0;
        for (int r = 1; r < TR; ++r) tr = tstart[r] <= f ? r : tr;
        return tr;
    };

    for (int32_t f0 = 0; f0 < ntarget; f0 += kBlock) {
        // this round's target, in registers
        const int32_t f = f0 + tid;
        const bool tgt = f < ntarget;
        int32_t k = -1, ix = 0, ty_ = 0, tz_ = 0;
        float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
        if (tgt) {
            const int tr = target_row(f);
            ty_ = tr % TY;
            tz_ = tr / TY;
            k = tfirst[tr] + (f - tstart[tr]);
            ix = a.cell[k] - a.nx * ((y0 + ty_) + a.ny * (z0 + tz_));
            const float4 q = a.p4[k];
            t = make_float4(__builtin_fmaf((float)(ix - cxlo), W, q.x), __builtin_fmaf((float)(y0 + ty_ - ylo), W, q.y),
                            __builtin_fmaf((float)(z0 + tz_ - zlo), W, q.z), q.w);
        }
        const int32_t fend = min(f0 + kBlock, ntarget); // targets of this round: [f0, fend)
        Target<PREC, INV> T;
        const int jl = ix > 0 ? (ix - cxlo) - 1 : (ix - cxlo);
        const int jr = ix + 1 < a.nx ? (ix - cxlo) + 2 : (ix - cxlo) + 1;
        for (int32_t zs = z0 - 1; zs <= z0 + TZ; ++zs) {
            if (zs < 0 || zs >= a.nz) continue;
            // 2. stage the sheet: row ranges, their LDS starts, cell starts
            if (tid < 64) {
                int32_t cnt = 0, gs = 0, rb32 = 0;
                if (tid < HY) {
                    const int32_t y = y0 - 1 + tid;
                    if (y >= 0 && y < a.ny) {
                        const int64_t rb = (int64_t)a.nx * (y + (int64_t)a.ny * zs);
                        rb32 = (int32_t)rb;
                        gs = a.off[rb + cxlo];
                        cnt = a.off[rb + cxhi + 1] - gs;
                    }
                }
                const int32_t inc = wave_incl_scan(cnt);
                if (tid < HY) {
                    rstart[tid] = inc - cnt;
                    gstart[tid] = gs;
                    rbase[tid] = rb32;
                }
                if (tid == HY - 1) rstart[HY] = inc;
            }
            __syncthreads();
            for (int e = tid; e < HY * (HX + 1); e += kBlock) {
                const int r = e / (HX + 1), jj = e % (HX + 1);
                const int32_t y = y0 - 1 + r;
                int32_t v = rstart[r];
                if (jj <= cxhi - cxlo + 1 && y >= 0 && y < a.ny)
                    v = a.off[(int64_t)rbase[r] + cxlo + jj] - gstart[r] + rstart[r];
                cs[r][jj] = v;
            }
            // the round's targets in this sheet come from registers ...
            const bool in_sheet_z = zs >= z0 && zs < z0 + TZ;
            if (tgt && in_sheet_z && z0 + tz_ == zs) {
                const int r = ty_ + 1;
                sp[rstart[r] + (k - gstart[r])] = t;
            }
            // ... every other particle from global memory
            const int32_t total = rstart[HY];
            for (int32_t g2 = tid; g2 < total; g2 += kBlock) {
                int r = 0;
                for (int q = 1; q < HY; ++q) r = rstart[q] <= g2 ? q : r;
                const int32_t g = gstart[r] + (g2 - rstart[r]);
                const int32_t cx = a.cell[g] - rbase[r];
                // a target of this round? (its row is a target row and it
                // lies in the round's range of targets)
                if (in_sheet_z && r >= 1 && r <= TY && cx >= x0 && cx < txhi) {
                    const int trow = (r - 1) + TY * (zs - z0);
                    const int32_t ft = tstart[trow] + (g - tfirst[trow]);
                    if (ft >= f0 && ft < fend) continue;
                }
                const float4 q = a.p4[g];
                sp[g2] = make_float4(__builtin_fmaf((float)(cx - cxlo), W, q.x),
                                     __builtin_fmaf((float)(y0 - 1 + r - ylo), W, q.y),
                                     __builtin_fmaf((float)(zs - zlo), W, q.z), q.w);
            }
            __syncthreads();
            // 3. targets within one cell of the sheet walk their three rows
            if (tgt) {
                const int dz = zs - (z0 + tz_);
                if (dz >= -1 && dz <= 1) {
                    const int own = (dz == 0) ? rstart[ty_ + 1] + (k - gstart[ty_ + 1]) : -1;
                    for (int dy = -1; dy <= 1; ++dy) {
                        const int r = ty_ + 1 + dy;
                        const int32_t y = y0 + ty_ + dy;
                        if (y < 0 || y >= a.ny) continue;
                        const int32_t j1 = cs[r][jr];
                        for (int32_t j = cs[r][jl]; j < j1; ++j) {
                            const float4 src = sp[j];
                            const float ddx = t.x - src.x, ddy = t.y - src.y, ddz = t.z - src.z;
                            const float d2 = sq_dist(ddx, ddy, ddz);
                            if (d2 < a.k.hi && j != own && inside_cutoff(ddx, ddy, ddz, d2, a.k))
                                T.accept(ddx, ddy, ddz, d2, src.w, a.k);
                        }
                    }
                }
            }
            __syncthreads(); // the sheet area is restaged next
        }
        if (tgt) {
            write_target(a, k, T);
            if (INV) {
                long long c1;
                double a1, a2, a3, a4, a5;
                target_invariants(T, t.w, c1, a1, a2, a3, a4, a5);
                icnt += c1; inx += a1; iny += a2; inz += a3; isc += a4; irs += a5;
            }
        }
    }
    if (INV) reduce_invariants(a, lb, icnt, inx, iny, inz, isc, irs);
}

// ------------------------------------------------------------------ cell-SM
// The cell-based organisation with LDS staging (Par-Cell-SM, Sec. 4.4,
// Algorithm 3) on one-wavefront workgroups, also as a path for dense cells.
// A workgroup owns a run of SEG consecutive cells of one X-row and takes each
// of them that holds at least DENSE particles in turn (DENSE = 1: every
// cell, the paper's organisation; larger: the no-LDS walk takes the other
// cells' targets in the same launch sequence).  One lane keeps one target,
// 64 at a time (the paper's loop over a cell's targets in steps of the block
// size).  The 27 neighbour cells are 9 X-rows of three cells, each row one
// contiguous range of the sorted arrays; the rows are copied into LDS in
// fills of up to CAP particles, and the wavefront walks each staged cell
// with one trip count, every lane reading the same LDS word, G sources per
// LDS round trip.  A lane skips a neighbour cell whose nearest face is surely
// beyond the cutoff from its target (the reach test of the no-LDS walk, which
// changes no result) and evaluates an accepted pair at once.  Differences
// are taken in the target's own cell frame with the roundings of the no-LDS
// walk, and each target sees its 27 cells in the canonical order, so the
// outputs are bitwise those of the no-LDS walk, also off the lattice.
__device__ __forceinline__ void wave_reduce_partial(InvPartial *dst, long long cnt, double nx, double ny, double nz,
                                                    double sc, double rs)
{
    for (int o = 32; o >= 1; o >>= 1) {
        cnt += __shfl_xor(cnt, o, 64);
        nx += __shfl_xor(nx, o, 64);
        ny += __shfl_xor(ny, o, 64);
        nz += __shfl_xor(nz, o, 64);
        sc += __shfl_xor(sc, o, 64);
        rs += __shfl_xor(rs, o, 64);
    }
    if (threadIdx.x == 0) {
        InvPartial p;
        p.pairs = cnt;
        p.net[0] = nx;
        p.net[1] = ny;
        p.net[2] = nz;
        p.scale = sc;
        p.rho_sum = rs;
        p.pad[0] = p.pad[1] = 0.0;
        *dst = p;
    }
}

constexpr int kCellBlock = 64;
constexpr int kCellGroup = 4; // staged sources read per LDS round trip

template <int CAP, int PREC, bool INV, bool BATCH>
__global__ __launch_bounds__(kCellBlock) void k_sweep_cell(SweepArgs a, int32_t seg, int32_t dense, int32_t ntx,
                                                           int32_t nty)
{
    constexpr int G = kCellGroup;
    __shared__ float4 stage[CAP];
    __shared__ int4 rows[9];          // per neighbour row: first sorted index of its left, centre and
                                      // right cell (x, y, z) and of the cell after them (w)
    __shared__ int32_t rstart[10];    // each row's start in the concatenated source list

    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    uint32_t tl = lb;
    if (BATCH) {
        const SysDev &sd = a.sys[enter_system(a, lb)];
        tl = lb - (uint32_t)sd.block_base;
        ntx = sd.ntx;
        nty = sd.nty;
    }
    const int32_t bx = (int32_t)(tl % (uint32_t)ntx);
    const int32_t iy = (int32_t)((tl / (uint32_t)ntx) % (uint32_t)nty);
    const int32_t iz = (int32_t)(tl / ((uint32_t)ntx * (uint32_t)nty));
    const int32_t x0 = bx * seg, nrun = min(seg, a.nx - x0);
    const int64_t rc0 = (int64_t)a.nx * (iy + (int64_t)a.ny * iz);
    const int lane = threadIdx.x;
    const float W = a.k.w;
    const float reach2 = a.k.reach2;
    auto sel = [](int q, float m, float o, float p) { return q == 0 ? m : (q == 1 ? o : p); };

    // the run's cells that this workgroup takes (lane q: cell x0 + q)
    int32_t cb = 0, ce = 0;
    if (lane < nrun) {
        cb = a.off[rc0 + x0 + lane];
        ce = a.off[rc0 + x0 + lane + 1];
    }
    uint64_t todo = __ballot(lane < nrun && ce - cb >= dense);

    long long icnt = 0;
    double inx = 0, iny = 0, inz = 0, isc = 0, irs = 0;
    while (todo) {
        const int q = __builtin_ctzll(todo);
        todo &= todo - 1;
        const int32_t ix = x0 + q;
        const int32_t c0 = __shfl(cb, q, 64), c1 = __shfl(ce, q, 64);
        // the 9 neighbour rows (lane r: dy = r % 3 - 1, dz = r / 3 - 1)
        int32_t total;
        {
            int4 rg = make_int4(0, 0, 0, 0);
            if (lane < 9) {
                const int32_t cy = iy + lane % 3 - 1, cz = iz + lane / 3 - 1;
                if (cy >= 0 && cy < a.ny && cz >= 0 && cz < a.nz) {
                    const int64_t rb = (int64_t)a.nx * (cy + (int64_t)a.ny * cz) + ix;
                    rg.y = a.off[rb];
                    rg.z = a.off[rb + 1];
                    rg.x = ix > 0 ? a.off[rb - 1] : rg.y;
                    rg.w = ix + 1 < a.nx ? a.off[rb + 2] : rg.z;
                }
            }
            const int32_t len = rg.w - rg.x;
            const int32_t inc = wave_incl_scan(len);
            if (lane < 9) {
                rows[lane] = rg;
                rstart[lane] = inc - len;
            }
            if (lane == 8) rstart[9] = inc;
            total = __shfl(inc, 8, 64);
        }
        __syncthreads();
        for (int32_t t0 = c0; t0 < c1; t0 += 64) {
            const int32_t k = t0 + lane;
            const bool tgt = k < c1;
            const float4 pk = tgt ? a.p4[k] : make_float4(0.f, 0.f, 0.f, 0.f);
            const float xi = pk.x, yi = pk.y, zi = pk.z;
            const float xm = xi - (float)(-1) * W, xp = xi - (float)(1) * W;
            const float ym = yi - (float)(-1) * W, yp = yi - (float)(1) * W;
            const float zm = zi - (float)(-1) * W, zp = zi - (float)(1) * W;
            // the reach test per row: bit r of `rowok` if row r is within
            // reach, of `useL` / `useR` if its left / right cell is too
            uint32_t rowok = 0, useL = 0, useR = 0;
            if (tgt) {
                const float gyl = yi * yi, gyr = (W - yi) * (W - yi);
                const float gzl = zi * zi, gzr = (W - zi) * (W - zi);
                const float tlx = ix > 0 ? reach2 - xi * xi : -1.0f;
                const float trx = ix + 1 < a.nx ? reach2 - (W - xi) * (W - xi) : -1.0f;
#pragma unroll
                for (int r = 0; r < 9; ++r) {
                    const int dy = r % 3 - 1, dz = r / 3 - 1;
                    const float gyz = (dy < 0 ? gyl : (dy > 0 ? gyr : 0.f)) + (dz < 0 ? gzl : (dz > 0 ? gzr : 0.f));
                    rowok |= (gyz < reach2 ? 1u : 0u) << r;
                    useL |= (gyz < tlx ? 1u : 0u) << r;
                    useR |= (gyz < trx ? 1u : 0u) << r;
                }
            }
            Target<PREC, INV> T;
            for (int32_t p0 = 0; p0 < total; p0 += CAP) {
                const int32_t nfill = min(CAP, total - p0);
                // stage the fill: list position p is in the last row whose start is <= p
#pragma unroll 4
                for (int32_t e = lane; e < nfill; e += 64) {
                    const int32_t p = p0 + e;
                    int r = 0;
#pragma unroll
                    for (int u = 1; u < 9; ++u) r += rstart[u] <= p ? 1 : 0;
                    stage[e] = a.p4[rows[r].x + (p - rstart[r])];
                }
                __syncthreads();
                for (int r = 0; r < 9; ++r) {
                    const int4 rgl = rows[r];
                    const int4 rg = make_int4(__builtin_amdgcn_readfirstlane(rgl.x), __builtin_amdgcn_readfirstlane(rgl.y),
                                              __builtin_amdgcn_readfirstlane(rgl.z), __builtin_amdgcn_readfirstlane(rgl.w));
                    // sorted index of slot s: base + s
                    const int32_t base = rg.x - __builtin_amdgcn_readfirstlane(rstart[r]) + p0;
                    if (rg.w == rg.x || rg.x - base >= nfill || rg.w - base <= 0) continue;
                    const int dyc = r % 3, dzc = r / 3;
                    const float ty = sel(dyc, ym, yi, yp), tz = sel(dzc, zm, zi, zp);
                    const bool rin = (rowok >> r) & 1u;
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        const int32_t ja = d == 0 ? rg.x : (d == 1 ? rg.y : rg.z);
                        const int32_t jz = d == 0 ? rg.y : (d == 1 ? rg.z : rg.w);
                        const int32_t sa = max(ja - base, 0), sz = min(jz - base, nfill);
                        if (sa >= sz) continue;
                        const bool en = tgt && rin && (d == 0 ? ((useL >> r) & 1u) : (d == 2 ? ((useR >> r) & 1u) : true));
                        if (!__any(en)) continue;
                        const float tx = sel(d, xm, xi, xp);
                        // the target itself is a source only in its own cell
                        const int32_t self = (r == 4 && d == 1) ? k - base : -1;
                        // one staged source, tested by every lane and taken by
                        // those whose neighbour cell this is
                        auto test = [&](int32_t sl, const float4 &src) {
                            const float ddx = tx - src.x, ddy = ty - src.y, ddz = tz - src.z;
                            const float t = sq_dist(ddx, ddy, ddz);
                            if (en && t < a.k.hi && sl != self && inside_cutoff(ddx, ddy, ddz, t, a.k))
                                T.accept(ddx, ddy, ddz, t, src.w, a.k);
                        };
                        int32_t s = sa;
                        for (; s + G <= sz; s += G) {
                            float4 src[G];
#pragma unroll
                            for (int u = 0; u < G; ++u) src[u] = stage[s + u];
#pragma unroll
                            for (int u = 0; u < G; ++u) test(s + u, src[u]);
                        }
                        for (; s < sz; ++s) test(s, stage[s]);
                    }
                }
                __syncthreads(); // the area is refilled next
            }
            if (tgt) {
                write_target(a, k, T);
                if (INV) {
                    long long c1n;
                    double a1, a2, a3, a4, a5;
                    target_invariants(T, pk.w, c1n, a1, a2, a3, a4, a5);
                    icnt += c1n; inx += a1; iny += a2; inz += a3; isc += a4; irs += a5;
                }
            }
        }
        __syncthreads(); // the row tables are rewritten for the next cell
    }
    if (INV) wave_reduce_partial(a.partials + lb, icnt, inx, iny, inz, isc, irs);
}

// The dense pass of a single-system tile sweep: the targets of every tile
// whose halo overflowed the LDS area, each walked from global memory by one
// thread (the same walk and order as the tiles, so the same results).  A
// persistent grid strides over the particles; when the overflow word does
// not hold this launch's epoch, no tile overflowed and each workgroup only
// writes an empty partial record.  Tile shape (tx, ty, tz) and tile counts
// are those of the tile launch.
template <int PREC, bool INV>
__global__ __launch_bounds__(kBlock) void k_sweep_dense(SweepArgs a, int32_t tx, int32_t ty, int32_t tz,
                                                        int32_t ntx, int32_t nty, uint32_t rec0)
{
    __shared__ uint32_t any;
    if (threadIdx.x == 0) any = *(volatile uint32_t *)a.ovf == a.epoch ? 1u : 0u;
    __syncthreads();
    if (!any) {
        if (INV && threadIdx.x == 0) {
            InvPartial p;
            p.pairs = 0;
            p.net[0] = p.net[1] = p.net[2] = 0.0;
            p.scale = p.rho_sum = 0.0;
            p.pad[0] = p.pad[1] = 0.0;
            a.partials[rec0 + blockIdx.x] = p;
        }
        return;
    }
    long long icnt = 0;
    double inx = 0, iny = 0, inz = 0, isc = 0, irs = 0;
    {
        const int32_t kend = min(a.off[a.nc], a.n);
        for (int32_t k = (int32_t)(blockIdx.x * kBlock + threadIdx.x); k < kend; k += (int32_t)(gridDim.x * kBlock)) {
            const int32_t c = a.cell[k];
            const int32_t ix = c % a.nx, iy = (c / a.nx) % a.ny, iz = c / (a.nx * a.ny);
            const int32_t tile = ix / tx + ntx * (iy / ty + nty * (iz / tz));
            if (!a.tflag[tile]) continue;
            Target<PREC, INV> T;
            const float4 pk = a.p4[k];
            walk_rows_global(a, k, ix, iy, iz, pk.x, pk.y, pk.z, T);
            write_target(a, k, T);
            if (INV) {
                long long c1;
                double a1, a2, a3, a4, a5;
                target_invariants(T, pk.w, c1, a1, a2, a3, a4, a5);
                icnt += c1; inx += a1; iny += a2; inz += a3; isc += a4; irs += a5;
            }
        }
    }
    if (INV) reduce_invariants(a, rec0 + blockIdx.x, icnt, inx, iny, inz, isc, irs);
}

// The dense pass of a batch tile sweep.  Each system's workgroups in the
// launch are its tiles followed by its dense workgroups (the batch layout);
// a dense workgroup first checks whether any tile of its system overflowed
// (the flags the tile launch just wrote) and, if so, strides over the
// system's particles and walks from global memory the targets of flagged
// tiles.  Its invariant partial record stays in the system's range.
template <int PREC, bool INV>
__global__ __launch_bounds__(kBlock) void k_sweep_dense_batch(SweepArgs a, int32_t tx, int32_t ty, int32_t tz,
                                                              int32_t total_blocks)
{
    const uint32_t lb = blockIdx.x;
    const int s = enter_system(a, lb);
    const SysDev &sd = a.sys[s];
    const int32_t ntx = sd.ntx, nty = sd.nty, ntz = (a.nz + tz - 1) / tz;
    const int32_t ntiles = ntx * nty * ntz;
    const int32_t d = (int32_t)(lb - (uint32_t)sd.block_base) - ntiles;
    if (d < 0) return; // a tile's workgroup
    const int32_t nd = (s + 1 < a.nsys ? a.sys[s + 1].block_base : total_blocks) - sd.block_base - ntiles;
    const uint8_t *flags = a.tflag + sd.block_base;
    int any = 0;
    for (int32_t t = (int32_t)threadIdx.x; t < ntiles && !any; t += kBlock) any = flags[t];
    any = __syncthreads_or(any);
    long long icnt = 0;
    double inx = 0, iny = 0, inz = 0, isc = 0, irs = 0;
    if (any) {
        const int32_t kend = (int32_t)sd.first + sd.n;
        for (int32_t k = (int32_t)sd.first + d * kBlock + (int32_t)threadIdx.x; k < kend; k += nd * kBlock) {
            const int32_t c = a.cell[k];
            const int32_t ix = c % a.nx, iy = (c / a.nx) % a.ny, iz = c / (a.nx * a.ny);
            if (!flags[ix / tx + ntx * (iy / ty + nty * (iz / tz))]) continue;
            Target<PREC, INV> T;
            const float4 pk = a.p4[k];
            walk_rows_global(a, k, ix, iy, iz, pk.x, pk.y, pk.z, T);
            write_target(a, k, T);
            if (INV) {
                long long c1;
                double a1, a2, a3, a4, a5;
                target_invariants(T, pk.w, c1, a1, a2, a3, a4, a5);
                icnt += c1; inx += a1; iny += a2; inz += a3; isc += a4; irs += a5;
            }
        }
    }
    if (INV) reduce_invariants(a, lb, icnt, inx, iny, inz, isc, irs);
}

// FP64 reduction of the per-workgroup partials in two fixed-order stages
// (deterministic): stage 1 folds each run of up to 1024 records into one,
// stage 2 (one workgroup) folds those into the output.
constexpr int kInvRun = 1024;

__device__ __forceinline__ void inv_block_reduce(long long c, double *v, long long *redc, double (*red)[5])
{
    redc[threadIdx.x] = c;
    for (int q = 0; q < 5; ++q) red[threadIdx.x][q] = v[q];
    __syncthreads();
    for (int s = kBlock / 2; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) {
            redc[threadIdx.x] += redc[threadIdx.x + s];
            for (int q = 0; q < 5; ++q) red[threadIdx.x][q] += red[threadIdx.x + s][q];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kBlock) void k_inv_stage1(const InvPartial *__restrict__ parts, int32_t np,
                                                       InvPartial *__restrict__ out)
{
    __shared__ double red[kBlock][5];
    __shared__ long long redc[kBlock];
    long long c = 0;
    double v[5] = {0, 0, 0, 0, 0};
    const int32_t base = (int32_t)blockIdx.x * kInvRun;
    const int32_t end = min(np, base + kInvRun);
    for (int32_t i = base + (int32_t)threadIdx.x; i < end; i += kBlock) {
        const InvPartial p = parts[i];
        c += p.pairs;
        v[0] += p.net[0];
        v[1] += p.net[1];
        v[2] += p.net[2];
        v[3] += p.scale;
        v[4] += p.rho_sum;
    }
    inv_block_reduce(c, v, redc, red);
    if (threadIdx.x == 0) {
        InvPartial p;
        p.pairs = redc[0];
        p.net[0] = red[0][0];
        p.net[1] = red[0][1];
        p.net[2] = red[0][2];
        p.scale = red[0][3];
        p.rho_sum = red[0][4];
        p.pad[0] = p.pad[1] = 0.0;
        out[blockIdx.x] = p;
    }
}

__global__ __launch_bounds__(kBlock) void k_inv_stage2(const InvPartial *__restrict__ parts, int32_t np,
                                                       pi_invariants *__restrict__ out)
{
    __shared__ double red[kBlock][5];
    __shared__ long long redc[kBlock];
    long long c = 0;
    double v[5] = {0, 0, 0, 0, 0};
    for (int32_t i = threadIdx.x; i < np; i += kBlock) {
        const InvPartial p = parts[i];
        c += p.pairs;
        v[0] += p.net[0];
        v[1] += p.net[1];
        v[2] += p.net[2];
        v[3] += p.scale;
        v[4] += p.rho_sum;
    }
    inv_block_reduce(c, v, redc, red);
    if (threadIdx.x == 0) {
        out->pairs = redc[0];
        out->net[0] = red[0][0];
        out->net[1] = red[0][1];
        out->net[2] = red[0][2];
        out->scale = red[0][3];
        out->rho_sum = red[0][4];
    }
}

// Batch mode: invariants of table entry s from its workgroups' partials
// [block_base[s], block_base[s+1]) (one workgroup per system, fixed order),
// written to the system's place in the caller's list.
__global__ __launch_bounds__(kBlock) void k_inv_systems(const InvPartial *__restrict__ parts,
                                                        const SysDev *__restrict__ sys, int32_t nsys,
                                                        int32_t total_blocks, pi_invariants *__restrict__ out)
{
    __shared__ double red[kBlock][5];
    __shared__ long long redc[kBlock];
    const int s = blockIdx.x;
    const int32_t b0 = sys[s].block_base;
    const int32_t b1 = s + 1 < nsys ? sys[s + 1].block_base : total_blocks;
    long long c = 0;
    double v[5] = {0, 0, 0, 0, 0};
    for (int32_t i = b0 + (int32_t)threadIdx.x; i < b1; i += kBlock) {
        const InvPartial p = parts[i];
        c += p.pairs;
        v[0] += p.net[0];
        v[1] += p.net[1];
        v[2] += p.net[2];
        v[3] += p.scale;
        v[4] += p.rho_sum;
    }
    inv_block_reduce(c, v, redc, red);
    if (threadIdx.x == 0) {
        pi_invariants &o = out[sys[s].orig];
        o.pairs = redc[0];
        o.net[0] = red[0][0];
        o.net[1] = red[0][1];
        o.net[2] = red[0][2];
        o.scale = red[0][3];
        o.rho_sum = red[0][4];
    }
}

__global__ void k_inv_zero(pi_invariants *__restrict__ out)
{
    if (threadIdx.x == 0) {
        out->pairs = 0;
        out->net[0] = out->net[1] = out->net[2] = 0.0;
        out->scale = 0.0;
        out->rho_sum = 0.0;
    }
}

// ------------------------------------------------------------------ host side

} // namespace

KernelConst pi_make_kernel_const(float rc, float cell_w)
{
    KernelConst k;
    const float h = rc;
    const double hd = (double)h;
    const double r2 = hd * hd; // exact
    const double u = ldexp(1.0, -24);
    k.lo = nextafterf((float)(r2 * (1.0 - 4.0 * u)), 0.0f);
    k.hi = nextafterf((float)(r2 * (1.0 + 4.0 * u)), INFINITY);
    k.reach2 = nextafterf((float)(r2 * (1.0 + 16.0 * u)), INFINITY);
    k.hh = h * h;
    k.eh = fmaf(h, h, -k.hh);
    k.hh_quarter = k.hh * 0.25f;
    k.h = h;
    k.inv_h = (float)(1.0 / hd);
    const double sigma = 8.0 / (M_PI * hd * hd * hd);
    k.sigma = (float)sigma;
    k.two_sigma = (float)(2.0 * sigma);
    k.sig_h2 = (float)(sigma / (hd * hd));
    k.six_sig_h = (float)(6.0 * sigma / hd);
    k.w = cell_w;
    return k;
}

namespace {

// Tile shapes compiled in.  id: 0 = no LDS; 1.. = tiles.
struct TileCfg {
    int id;
    int tx, ty, tz, cap;
    int sweep; // PI_SWEEP_PENCIL / PI_SWEEP_SUBBOX
};

const TileCfg kTiles[] = {
    {1, 254, 1, 1, 2560, PI_SWEEP_PENCIL},
    {2, 62, 1, 1, 1024, PI_SWEEP_PENCIL},
    {3, 30, 1, 1, 2560, PI_SWEEP_PENCIL},
    {4, 8, 8, 3, 768, PI_SWEEP_SUBBOX},
    {5, 6, 6, 6, 768, PI_SWEEP_SUBBOX},
    {6, 4, 4, 4, 1536, PI_SWEEP_SUBBOX},
    {7, 4, 4, 2, 1536, PI_SWEEP_SUBBOX},
    {8, 16, 4, 3, 768, PI_SWEEP_SUBBOX},
    {10, 7, 7, 5, 768, PI_SWEEP_SUBBOX},
    // X-pencil-reg sub-boxes; cap = the largest Z-sheet staged at once
    {11, 8, 8, 4, 1024, PI_SWEEP_PENCILREG},
    {12, 4, 4, 2, 1024, PI_SWEEP_PENCILREG},
    // cell-SM: tx = cells of an X-row per workgroup, ty = the fewest particles
    // a cell must hold to be taken (1: all; larger: the no-LDS walk takes the
    // rest); cap = particles per LDS fill
    {13, 1, 1, 1, 256, PI_SWEEP_CELL},
    {14, 4, 1, 1, 256, PI_SWEEP_CELL},
    {15, 2, 16, 1, 256, PI_SWEEP_CELL},
    {16, 2, 32, 1, 256, PI_SWEEP_CELL},
    {17, 2, 64, 1, 256, PI_SWEEP_CELL},
};

#ifndef PI_FIFO_DEPTH
#define PI_FIFO_DEPTH 4
#endif
constexpr int kFifo = PI_FIFO_DEPTH; // pair queue entries per lane
constexpr int kCellCap = 256;       // cell-SM: particles per LDS fill
constexpr int kStreamId = 9; // organisation id of the FIFO stream sweep
constexpr int kMaxOrgId = 17; // organisation ids are 0 .. kMaxOrgId

// Workgroups of the dense pass that follows a single-system tile launch: a
// persistent grid of up to four per compute unit, one per 256 particles at
// most.
unsigned dense_blocks(int64_t n)
{
    const int64_t b = (n + kBlock - 1) / kBlock;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 1024));
}

// Dense workgroups of one system of a batch tile sweep: one per 512
// particles, at most 1024 (a workgroup of a system without an overflowing
// tile only reads the system's tile flags).
int64_t batch_dense_blocks(int64_t n)
{
    return std::max<int64_t>(1, std::min<int64_t>((n + 511) / 512, 1024));
}

// nblk: in single-system mode computed here from the grid, and then the
// count of invariant partial records the launch writes (the tiles', then
// the dense pass's); in batch mode given (the sum of the systems' tile
// counts).
template <int TX, int TY, int TZ, int CAP, int PREC, bool INV, bool BATCH, bool REG = false>
void launch_tile(pi_ctx *ctx, const char *name, const SweepArgs &a, hipStream_t s, unsigned &nblk)
{
    int32_t ntx = 0, nty = 0;
    if (!BATCH) {
        ntx = (a.nx + TX - 1) / TX;
        nty = (a.ny + TY - 1) / TY;
        const int32_t ntz = (a.nz + TZ - 1) / TZ;
        nblk = (unsigned)((int64_t)ntx * nty * ntz);
    }
    if (BATCH) {
        // (nblk counts every system's tiles and dense workgroups)
        if (REG)
            PI_LAUNCH(ctx, name, (k_sweep_pencilreg<TX, TY, TZ, CAP, PREC, INV, BATCH>), dim3(nblk), dim3(kBlock), 0,
                      s, a, ntx, nty);
        else
            PI_LAUNCH(ctx, name, (k_sweep_tile<TX, TY, TZ, CAP, kFifo, PREC, INV, BATCH>), dim3(nblk), dim3(kBlock),
                      0, s, a, ntx, nty);
        PI_LAUNCH(ctx, "k_sweep_dense_batch", (k_sweep_dense_batch<PREC, INV>), dim3(nblk), dim3(kBlock), 0, s, a, TX,
                  TY, TZ, (int32_t)nblk);
        return;
    }
    SweepArgs b = a;
    b.epoch = ++*a.host_epoch;
    if (b.epoch == 0) b.epoch = ++*a.host_epoch; // 0 is the word's initial value
    if (REG)
        PI_LAUNCH(ctx, name, (k_sweep_pencilreg<TX, TY, TZ, CAP, PREC, INV, BATCH>), dim3(nblk), dim3(kBlock), 0, s,
                  b, ntx, nty);
    else
        PI_LAUNCH(ctx, name, (k_sweep_tile<TX, TY, TZ, CAP, kFifo, PREC, INV, BATCH>), dim3(nblk), dim3(kBlock), 0,
                  s, b, ntx, nty);
    const unsigned nd = dense_blocks(a.n);
    PI_LAUNCH(ctx, "k_sweep_dense", (k_sweep_dense<PREC, INV>), dim3(nd), dim3(kBlock), 0, s, b, TX, TY, TZ, ntx,
              nty, nblk);
    nblk += nd;
}

// The cell-SM sweep: one workgroup per run of `seg` cells of an X-row (the
// LDS fills take any occupancy, so there is no dense pass).  With dense > 1
// (single system only) the no-LDS walk first takes the targets of the cells
// holding fewer than `dense` particles; nblk counts both launches'
// workgroups, the no-LDS walk's partial records first.

template <int CAP, int PREC, bool INV, bool BATCH>
void launch_cell(pi_ctx *ctx, const char *name, int32_t seg, int32_t dense, const SweepArgs &a, hipStream_t s,
                 unsigned &nblk)
{
    if (BATCH) {
        PI_LAUNCH(ctx, name, (k_sweep_cell<CAP, PREC, INV, BATCH>), dim3(nblk), dim3(kCellBlock), 0, s, a,
                  seg, 1, 0, 0);
        return;
    }
    SweepArgs b = a;
    unsigned n0 = 0;
    if (dense > 1) {
        n0 = (unsigned)((a.n + kBlock - 1) / kBlock);
        SweepArgs c = a;
        c.dense_min = dense;
        PI_LAUNCH(ctx, "k_sweep_nolds", (k_sweep_nolds<PREC, INV, false>), dim3(n0), dim3(kBlock), 0, s, c);
        if (b.partials) b.partials += n0;
    }
    const int32_t ntx = (a.nx + seg - 1) / seg;
    const unsigned n1 = (unsigned)((int64_t)ntx * a.ny * a.nz);
    PI_LAUNCH(ctx, name, (k_sweep_cell<CAP, PREC, INV, false>), dim3(n1), dim3(kCellBlock), 0, s, b, seg,
              dense, ntx, a.ny);
    nblk = n0 + n1;
}

template <int PREC, bool INV, bool BATCH>
void launch_sweep(pi_ctx *ctx, int tile_id, const SweepArgs &a, hipStream_t s, unsigned &nblk)
{
    switch (tile_id) {
    case 1: launch_tile<254, 1, 1, 2560, PREC, INV, BATCH>(ctx, "k_sweep_tile<254,1,1>", a, s, nblk); break;
    case 2: launch_tile<62, 1, 1, 1024, PREC, INV, BATCH>(ctx, "k_sweep_tile<62,1,1>", a, s, nblk); break;
    case 3: launch_tile<30, 1, 1, 2560, PREC, INV, BATCH>(ctx, "k_sweep_tile<30,1,1>", a, s, nblk); break;
    case 4: launch_tile<8, 8, 3, 768, PREC, INV, BATCH>(ctx, "k_sweep_tile<8,8,3>", a, s, nblk); break;
    case 5: launch_tile<6, 6, 6, 768, PREC, INV, BATCH>(ctx, "k_sweep_tile<6,6,6>", a, s, nblk); break;
    case 6: launch_tile<4, 4, 4, 1536, PREC, INV, BATCH>(ctx, "k_sweep_tile<4,4,4>", a, s, nblk); break;
    case 7: launch_tile<4, 4, 2, 1536, PREC, INV, BATCH>(ctx, "k_sweep_tile<4,4,2>", a, s, nblk); break;
    case 8: launch_tile<16, 4, 3, 768, PREC, INV, BATCH>(ctx, "k_sweep_tile<16,4,3>", a, s, nblk); break;
    case 10: launch_tile<7, 7, 5, 768, PREC, INV, BATCH>(ctx, "k_sweep_tile<7,7,5>", a, s, nblk); break;
    case 11: launch_tile<8, 8, 4, 1024, PREC, INV, BATCH, true>(ctx, "k_sweep_pencilreg<8,8,4>", a, s, nblk); break;
    case 12: launch_tile<4, 4, 2, 1024, PREC, INV, BATCH, true>(ctx, "k_sweep_pencilreg<4,4,2>", a, s, nblk); break;
    case 13: launch_cell<kCellCap, PREC, INV, BATCH>(ctx, "k_sweep_cell<1,1>", 1, 1, a, s, nblk); break;
    case 14: launch_cell<kCellCap, PREC, INV, BATCH>(ctx, "k_sweep_cell<4,1>", 4, 1, a, s, nblk); break;
    case 15: launch_cell<kCellCap, PREC, INV, BATCH>(ctx, "k_sweep_cell<2,16>", 2, 16, a, s, nblk); break;
    case 16: launch_cell<kCellCap, PREC, INV, BATCH>(ctx, "k_sweep_cell<2,32>", 2, 32, a, s, nblk); break;
    case 17: launch_cell<kCellCap, PREC, INV, BATCH>(ctx, "k_sweep_cell<2,64>", 2, 64, a, s, nblk); break;
    case kStreamId:
        if (!BATCH) {
            nblk = (unsigned)((a.n + kBlock - 1) / kBlock);
            if (nblk == 0) nblk = 1;
        }
        PI_LAUNCH(ctx, "k_sweep_stream", (k_sweep_stream<kFifo, PREC, INV, BATCH>), dim3(nblk), dim3(kBlock), 0, s,
                  a);
        break;
    default:
        if (!BATCH) {
            nblk = (unsigned)((a.n + kBlock - 1) / kBlock);
            if (nblk == 0) nblk = 1;
        }
        PI_LAUNCH(ctx, "k_sweep_nolds", (k_sweep_nolds<PREC, INV, BATCH>), dim3(nblk), dim3(kBlock), 0, s, a);
        break;
    }
}

template <bool BATCH>
void launch_sweep_prec(pi_ctx *ctx, int prec, bool inv, int tile_id, const SweepArgs &a, hipStream_t s,
                       unsigned &nblk)
{
    switch (prec) {
    case PI_PREC_PLAIN:
        if (inv) launch_sweep<PI_PREC_PLAIN, true, BATCH>(ctx, tile_id, a, s, nblk);
        else if (!BATCH) launch_sweep<PI_PREC_PLAIN, false, false>(ctx, tile_id, a, s, nblk);
        break;
    case PI_PREC_FP64ACC:
        if (inv) launch_sweep<PI_PREC_FP64ACC, true, BATCH>(ctx, tile_id, a, s, nblk);
        else if (!BATCH) launch_sweep<PI_PREC_FP64ACC, false, false>(ctx, tile_id, a, s, nblk);
        break;
    default:
        if (inv) launch_sweep<PI_PREC_COMPENSATED, true, BATCH>(ctx, tile_id, a, s, nblk);
        else if (!BATCH) launch_sweep<PI_PREC_COMPENSATED, false, false>(ctx, tile_id, a, s, nblk);
        break;
    }
}

const TileCfg &tile_cfg(int id)
{
    for (const TileCfg &t : kTiles)
        if (t.id == id) return t;
    return kTiles[0];
}

// Whether tile `id`'s staged halo is expected to fit its LDS capacity at
// mean occupancy ppc: the halo count is about Poisson, so its mean plus six
// standard deviations must stay within the capacity (a tile that overflows
// still gives the same results, from the slower global walk).
bool halo_fits(int id, double ppc)
{
    const TileCfg &t = tile_cfg(id);
    const double m = (double)(t.tx + 2) * (t.ty + 2) * (t.tz + 2) * ppc;
    return m + 6.0 * sqrt(m) <= (double)t.cap;
}

// Static rule: the 6x6x6 sub-box while its halo fits (up to about 1.2 per
// cell), then 4x4x4 (up to about 6), then no LDS.
int pick_tile_default(double ppc)
{
    return halo_fits(5, ppc) ? 5 : (halo_fits(6, ppc) ? 6 : 0);
}

} // namespace

bool pi_tile_shape(int tile_id, int *tx, int *ty, int *tz)
{
    for (const TileCfg &t : kTiles)
        if (t.id == tile_id) {
            *tx = t.tx;
            *ty = t.ty;
            *tz = t.tz;
            return true;
        }
    return false;
}

// Whether id names an organisation: 0 (no LDS), the stream sweep, or an
// entry of the tile table.
bool pi_org_valid(int id)
{
    int tx, ty, tz;
    return id == 0 || id == kStreamId || pi_tile_shape(id, &tx, &ty, &tz);
}

// The explicit options (organisation and tile shape) that run organisation
// `tile`; precision and order are left as they are.
void pi_tile_opts(int tile, pi_interact_opts *out)
{
    int tx = 0, ty = 0, tz = 0;
    out->tile[0] = out->tile[1] = out->tile[2] = 0;
    if (tile > 0 && pi_tile_shape(tile, &tx, &ty, &tz)) {
        out->sweep = tile_cfg(tile).sweep;
        out->tile[0] = tx;
        out->tile[1] = ty;
        out->tile[2] = tz;
    } else {
        out->sweep = tile == kStreamId ? PI_SWEEP_STREAM : PI_SWEEP_NOLDS;
    }
}

// Tile id for explicit options; -1 if the shape is not compiled in; AUTO
// returns the static default (the tuner refines it per system).
int pi_pick_tile(const pi_interact_opts &o, double ppc)
{
    if (o.sweep == PI_SWEEP_NOLDS) return 0;
    if (o.sweep == PI_SWEEP_STREAM) return kStreamId;
    if (o.sweep == PI_SWEEP_CELL) {
        if (o.tile[0] > 0) {
            for (const TileCfg &t : kTiles)
                if (t.sweep == o.sweep && t.tx == o.tile[0] && t.ty == o.tile[1] && t.tz == o.tile[2]) return t.id;
            return -1;
        }
        return ppc >= 32.0 ? 13 : 16;
    }
    if (o.sweep == PI_SWEEP_PENCILREG) {
        if (o.tile[0] > 0) {
            for (const TileCfg &t : kTiles)
                if (t.sweep == o.sweep && t.tx == o.tile[0] && t.ty == o.tile[1] && t.tz == o.tile[2]) return t.id;
            return -1;
        }
        return ppc <= 2.0 ? 11 : 12;
    }
    if (o.sweep == PI_SWEEP_PENCIL || o.sweep == PI_SWEEP_SUBBOX) {
        if (o.tile[0] > 0) {
            for (const TileCfg &t : kTiles)
                if (t.sweep == o.sweep && t.tx == o.tile[0] && t.ty == o.tile[1] && t.tz == o.tile[2]) return t.id;
            return -1;
        }
        if (o.sweep == PI_SWEEP_PENCIL) return halo_fits(1, ppc) ? 1 : (halo_fits(2, ppc) ? 2 : 3);
        return halo_fits(5, ppc) ? 5 : (halo_fits(6, ppc) ? 6 : 7);
    }
    return pick_tile_default(ppc);
}

// The organisation a batch runs for a system whose own choice is `tile`: the
// cell-SM's dense-cell pass, which pairs it with a no-LDS launch, is run as
// the no-LDS walk alone (the same outputs).
int pi_batch_org(int tile)
{
    if (tile > 0 && tile_cfg(tile).id == tile && tile_cfg(tile).sweep == PI_SWEEP_CELL && tile_cfg(tile).ty > 1)
        return 0;
    return tile;
}

// Batch sweep: h_sys gets each system's block_base / ntx / nty for tile_id
// (the caller uploads the table to d_sys before launching).  Returns the
// total workgroup count.
int64_t pi_batch_layout(int tile_id, SysDev *h_sys, int32_t nsys)
{
    int tx = 0, ty = 0, tz = 0;
    const bool tiled = tile_id > 0 && pi_tile_shape(tile_id, &tx, &ty, &tz);
    const bool cell = tiled && tile_cfg(tile_id).sweep == PI_SWEEP_CELL;
    if (cell) ty = tz = 1; // runs of tx cells
    int64_t base = 0;
    for (int32_t s = 0; s < nsys; ++s) {
        SysDev &d = h_sys[s];
        d.block_base = (int32_t)base;
        if (tiled) {
            d.ntx = (d.g.nx + tx - 1) / tx;
            d.nty = (d.g.ny + ty - 1) / ty;
            const int32_t ntz = (d.g.nz + tz - 1) / tz;
            base += (int64_t)d.ntx * d.nty * ntz;
            // the dense workgroups of an LDS tiling (none for the cell-SM)
            if (!cell) base += batch_dense_blocks(d.n);
        } else {
            d.ntx = d.nty = 0;
            base += (d.n + kBlock - 1) / kBlock;
        }
    }
    return base;
}

// One sweep launch over the systems of table d_sys[0 .. nsys) (all with tile
// tile_id); their workgroup partials go to records part_base + block.
pi_status pi_sweep_batch(pi_ctx *ctx, pi_cells *cells, int32_t nsys, const SysDev *d_sys, const KernelConst *d_kcs,
                         int64_t total_blocks, int64_t part_base, int tile_id, const pi_interact_opts &o, float *rho,
                         float *gx, float *gy, float *gz, int32_t *count, pi_invariants *inv, hipStream_t stream)
{
    if (part_base + total_blocks > cells->cap_partials) return PI_ENOMEM;
    SweepArgs a;
    memset(&a, 0, sizeof(a));
    a.off = cells->offsets;
    a.cell = cells->cell;
    a.perm = cells->perm;
    a.p4 = cells->xyzw;
    a.n = (int32_t)cells->n;
    a.orig_order = o.order == PI_ORDER_ORIGINAL;
    a.rho = rho;
    a.gx = gx;
    a.gy = gy;
    a.gz = gz;
    a.count = count;
    a.partials = (InvPartial *)cells->partials + part_base;
    a.tflag = cells->tflag + part_base; // (one flag per workgroup of the group)
    a.sys = d_sys;
    a.kcs = d_kcs;
    a.nsys = nsys;
    unsigned nblk = (unsigned)total_blocks;
    if (nblk > 0) launch_sweep_prec<true>(ctx, o.precision, true, tile_id, a, stream, nblk);
    if (inv)
        PI_LAUNCH(ctx, "k_inv_systems", k_inv_systems, dim3(nsys), dim3(kBlock), 0, stream,
                  (const InvPartial *)a.partials, d_sys, nsys, (int32_t)total_blocks, inv);
    PI_CHECK_HIP(hipGetLastError());
    return PI_OK;
}

namespace {

uint64_t tune_key(int prec, int64_t n, double ppc, bool batch)
{
    const int kn = n > 1 ? (int)floor(2.0 * log2((double)n)) : 0;
    const int kp = (int)fmin(1023.0, floor(4.0 * ppc + 0.5));
    return (uint64_t)prec + 4ull * (uint64_t)kn + 256ull * (uint64_t)kp + (batch ? (1ull << 30) : 0ull);
}

// Time every compiled organisation on this system (the fastest of up to
// three runs after a first one, with
// the invariant partials when the call computes them, since they change the
// ranking: at 1 per cell the 7x7x5 tile is 5% faster than 6x6x6 without
// them and 5% slower with them) and return the fastest; the outputs and
// partial records in `a` are overwritten.  The static default is timed first and a later organisation
// displaces the current best only when it is faster by more than 5%, so that
// near-ties (within run-to-run noise) resolve the same way every time.
// Organisations that cannot win at mean occupancy ppc and are not timed: the
// cell-SM over every cell below 16 particles per cell (a wavefront of mostly
// idle lanes per cell), and its dense-cell pass below 2.
bool worth_timing(int id, double ppc)
{
    if (id < 13 || id > 17) return true;
    return id <= 14 ? ppc >= 16.0 : ppc >= 2.0;
}

int time_candidates(pi_ctx *ctx, const SweepArgs &a0, int prec, int first, bool inv, double ppc, hipStream_t s)
{
    SweepArgs a = a0;
    if (!inv) a.partials = nullptr;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1;
    }
    const int was = ctx->timing_on;
    ctx->timing_on = 0;
    int best = -1;
    float best_ms = 0.f;
    for (int i = -1; i <= kMaxOrgId; ++i) {
        const int cand = i < 0 ? first : i;
        if (i >= 0 && (cand == first || !worth_timing(cand, ppc))) continue;
        // one untimed run, then the fastest of up to three timed ones (one
        // if that is already 1.5x the best: single runs vary by a few
        // percent, which near-ties between tilings would otherwise follow)
        unsigned nblk = 0;
        float ms = 0.f;
        bool ok = true;
        for (int rep = 0; rep < 4 && ok; ++rep) {
            float t = 0.f;
            ok = hipEventRecord(e0, s) == hipSuccess;
            launch_sweep_prec<false>(ctx, prec, inv, cand, a, s, nblk);
            ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(e1, s) == hipSuccess &&
                 hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&t, e0, e1) == hipSuccess;
            if (rep == 1 || (rep > 1 && t < ms)) ms = t;
            if (rep == 1 && best >= 0 && ms > 1.5f * best_ms) break;
        }
        if (ok && (best < 0 || ms < 0.95f * best_ms)) {
            best = cand;
            best_ms = ms;
        }
    }
    ctx->timing_on = was;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

pi_status tuned_tile(pi_ctx *ctx, const SweepArgs &a, int prec, int64_t n, double ppc, bool inv, hipStream_t s,
                     int *tile)
{
    pi_tuner *t = ctx->tuner;
    *tile = pick_tile_default(ppc);
    if (!t || t->mode != PI_TUNE_TIMED) return PI_OK;
    const uint64_t key = tune_key(prec, n, ppc, false);
    {
        std::lock_guard<std::mutex> g(t->mu);
        auto it = t->choice.find(key);
        if (it != t->choice.end()) {
            *tile = it->second;
            return PI_OK;
        }
    }
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return PI_OK;
    const int best = time_candidates(ctx, a, prec, *tile, inv, ppc, s);
    if (best < 0) return PI_EDEVICE;
    std::lock_guard<std::mutex> g(t->mu);
    t->choice[key] = best;
    *tile = best;
    return PI_OK;
}

} // namespace

// AUTO organisation of one system of a batch: the tuner's cached choice for
// the system's class if there is one, else the static rule (no trials are
// run inside a batch).
int pi_auto_tile(pi_ctx *ctx, int precision, int64_t n, double ppc)
{
    pi_tuner *t = ctx->tuner;
    if (t && t->mode == PI_TUNE_TIMED) {
        std::lock_guard<std::mutex> g(t->mu);
        auto it = t->choice.find(tune_key(precision, n, ppc, false));
        if (it != t->choice.end()) return it->second;
    }
    return pick_tile_default(ppc);
}

extern "C" pi_status pi_tuner_mode(pi_ctx *ctx, int32_t mode)
{
    if (!ctx || !ctx->tuner || (mode != PI_TUNE_STATIC && mode != PI_TUNE_TIMED)) return PI_EINVAL;
    std::lock_guard<std::mutex> g(ctx->tuner->mu);
    ctx->tuner->mode = mode;
    return PI_OK;
}

extern "C" pi_status pi_tuner_choice(pi_ctx *ctx, const pi_cells *cells, int32_t precision, pi_interact_opts *out,
                                     pi_stream stream)
{
    if (!ctx || !cells || !out || cells->ctx != ctx) return PI_EINVAL;
    if (!pi_cells_ready(cells)) return PI_ESTATE;
    if (precision < PI_PREC_COMPENSATED || precision > PI_PREC_FP64ACC) return PI_EINVAL;
    const int64_t n = cells->n;
    const double ppc = cells->n_cells > 0 ? (double)n / (double)cells->n_cells : 0.0;
    int tile = pick_tile_default(ppc);
    if (n > 0) {
        SweepArgs a;
        memset(&a, 0, sizeof(a));
        a.off = cells->offsets;
        a.cell = cells->cell;
        a.perm = cells->perm;
        a.p4 = cells->xyzw;
        a.nc = cells->n_cells;
        a.n = (int32_t)n;
        a.nx = cells->grid.dims[0];
        a.ny = cells->grid.dims[1];
        a.nz = cells->grid.dims[2];
        a.k = pi_make_kernel_const(cells->grid.rc, cells->grid.cell_w);
        a.tflag = cells->tflag;
        a.ovf = cells->d_err + 32;
        a.host_epoch = &const_cast<pi_cells *>(cells)->sweep_epoch;
        // count-only outputs so that tuning writes nothing the caller owns
        a.rho = a.gx = a.gy = a.gz = nullptr;
        a.count = nullptr;
        PI_CHECK_HIP(hipSetDevice(ctx->device));
        pi_status st = tuned_tile(ctx, a, precision, n, ppc, false, (hipStream_t)stream, &tile);
        if (st != PI_OK) return st;
    }
    memset(out, 0, sizeof(*out));
    out->precision = precision;
    pi_tile_opts(tile, out);
    return PI_OK;
}

namespace {

// Invariant partial records of one single-system sweep launch of
// organisation `tile` (as launch_sweep counts them: a tiling's workgroups
// and those of its dense pass).
int64_t sweep_blocks(int tile, int64_t n, int32_t nx, int32_t ny, int32_t nz)
{
    int tx = 0, ty = 0, tz = 0;
    if (tile > 0 && tile != kStreamId && pi_tile_shape(tile, &tx, &ty, &tz)) {
        if (tile_cfg(tile).sweep == PI_SWEEP_CELL) // runs of tx cells, after the no-LDS walk's records
            return (int64_t)((nx + tx - 1) / tx) * ny * nz + (ty > 1 ? (n + kBlock - 1) / kBlock : 0);
        return (int64_t)((nx + tx - 1) / tx) * ((ny + ty - 1) / ty) * ((nz + tz - 1) / tz) + dense_blocks(n);
    }
    const int64_t b = (n + kBlock - 1) / kBlock;
    return b > 0 ? b : 1;
}

} // namespace

void pi_reduce_partials(pi_ctx *ctx, void *partials, unsigned nblk, pi_invariants *inv, hipStream_t stream)
{
    if (nblk == 0) {
        PI_LAUNCH(ctx, "k_inv_zero", k_inv_zero, dim3(1), dim3(64), 0, stream, inv);
        return;
    }
    // stage-1 records go after the sweep's records in the same buffer
    const int32_t n1 = (int32_t)((nblk + kInvRun - 1) / kInvRun);
    InvPartial *parts = (InvPartial *)partials;
    InvPartial *stage = parts + nblk;
    PI_LAUNCH(ctx, "k_inv_stage1", k_inv_stage1, dim3(n1), dim3(kBlock), 0, stream, (const InvPartial *)parts,
              (int32_t)nblk, stage);
    PI_LAUNCH(ctx, "k_inv_stage2", k_inv_stage2, dim3(1), dim3(kBlock), 0, stream, (const InvPartial *)stage, n1,
              inv);
}

pi_status pi_interact_run(pi_ctx *ctx, const pi_cells *cells, const pi_interact_opts &o, float *rho, float *gx,
                          float *gy, float *gz, int32_t *count, pi_invariants *inv, hipStream_t stream,
                          void *partials, int64_t cap_partials, bool no_alloc)
{
    const int64_t n = cells->n;
    const double ppc = cells->n_cells > 0 ? (double)n / (double)cells->n_cells : 0.0;
    int tile = pi_pick_tile(o, ppc);
    if (tile < 0) return PI_EINVAL;

    SweepArgs a;
    memset(&a, 0, sizeof(a));
    a.off = cells->offsets;
    a.cell = cells->cell;
    a.perm = cells->perm;
    a.p4 = cells->xyzw;
    a.nc = cells->n_cells;
    a.n = (int32_t)n;
    a.nx = cells->grid.dims[0];
    a.ny = cells->grid.dims[1];
    a.nz = cells->grid.dims[2];
    a.orig_order = o.order == PI_ORDER_ORIGINAL;
    a.rho = rho;
    a.gx = gx;
    a.gy = gy;
    a.gz = gz;
    a.count = count;
    a.partials = (InvPartial *)partials;
    a.k = pi_make_kernel_const(cells->grid.rc, cells->grid.cell_w);

    if (n == 0) {
        if (inv) PI_LAUNCH(ctx, "k_inv_zero", k_inv_zero, dim3(1), dim3(64), 0, stream, inv);
        PI_CHECK_HIP(hipGetLastError());
        return PI_OK;
    }

    unsigned nblk = 0;
    const bool want_inv = inv != nullptr;
    // partial records: one per workgroup, then the stage-1 records
    auto records = [&](int t) {
        const int64_t b = sweep_blocks(t, n, a.nx, a.ny, a.nz);
        return b + (b + kInvRun - 1) / kInvRun;
    };
    a.tflag = cells->tflag;
    a.ovf = cells->d_err + 32;
    a.host_epoch = &const_cast<pi_cells *>(cells)->sweep_epoch;
    if (no_alloc) {
        if (o.sweep == PI_SWEEP_AUTO) {
            // the tuner's cached choice or the static rule (no trials); no
            // LDS when a tiling needs more partial records than there are
            tile = pi_auto_tile(ctx, o.precision, n, ppc);
            if (want_inv && records(tile) > cap_partials) tile = 0;
        }
        if (want_inv && records(tile) > cap_partials) return PI_ENOMEM;
    } else if (want_inv) {
        // enough partial records for any tiling of this grid
        const int64_t need = 2 * (cells->n_cells + (n + kBlock - 1) / kBlock) + 64;
        if (need > cap_partials) {
            pi_cells *mc = const_cast<pi_cells *>(cells);
            PI_CHECK_HIP(hipStreamSynchronize(stream));
            if (mc->partials) (void)hipFree(mc->partials);
            mc->partials = nullptr;
            if (hipMalloc(&mc->partials, (size_t)need * sizeof(InvPartial)) != hipSuccess) {
                mc->cap_partials = 0;
                return PI_ENOMEM;
            }
            mc->cap_partials = need;
            a.partials = (InvPartial *)mc->partials;
        }
    }
    if (!no_alloc && o.sweep == PI_SWEEP_AUTO) {
        pi_status ts = tuned_tile(ctx, a, o.precision, n, ppc, want_inv, stream, &tile);
        if (ts != PI_OK) return ts;
    }
    launch_sweep_prec<false>(ctx, o.precision, want_inv, tile, a, stream, nblk);
    if (want_inv) pi_reduce_partials(ctx, a.partials, nblk, inv, stream);
    PI_CHECK_HIP(hipGetLastError());
    return PI_OK;
}

pi_status pi_check_interact_opts(const pi_interact_opts &o, int64_t n, const float *rho, const float *gx,
                                 const float *gy, const float *gz, const int32_t *count, const pi_invariants *inv)
{
    if (o.precision < PI_PREC_COMPENSATED || o.precision > PI_PREC_FP64ACC) return PI_EINVAL;
    if (o.sweep < PI_SWEEP_AUTO || o.sweep > PI_SWEEP_CELL) return PI_EINVAL;
    if (o.order != PI_ORDER_SORTED && o.order != PI_ORDER_ORIGINAL) return PI_EINVAL;
    const bool anyf = rho || gx || gy || gz;
    const bool allf = rho && gx && gy && gz;
    if (anyf && !allf) return PI_EINVAL;
    if (n > 0 && !anyf && !count && !inv) return PI_EINVAL;
    return PI_OK;
}

// ------------------------------------------------------------------ no-alloc sweep
//
// The invariant partial records of pi_interact_noalloc live in one fixed
// array per device, so the call never allocates.  In host code `scratch`
// names a host-side stand-in, not device memory: kernels get the device
// address looked up once per device by pi_noalloc_scratch_setup.

static __device__ __align__(256) InvPartial scratch[PI_NOALLOC_SCRATCH_RECORDS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
} // namespace

pi_status pi_noalloc_scratch_setup(int device, void **out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return PI_EINVAL;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return pi_hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                        "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[device] = ptr;
    }
    *out = g_scratch_ptr[device];
    return PI_OK;
}

extern "C" pi_status pi_interact_noalloc(pi_ctx *ctx, const pi_cells *cells, const pi_interact_opts *opts,
                                         float *rho, float *gx, float *gy, float *gz, int32_t *count,
                                         pi_invariants *inv, pi_stream stream_)
{
    if (!ctx || !cells || cells->ctx != ctx) return PI_EINVAL;
    if (!ctx->scratch) return PI_ESTATE;
    if (!pi_cells_ready(cells)) return PI_ESTATE;
    pi_interact_opts o;
    memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    const pi_status vs = pi_check_interact_opts(o, cells->n, rho, gx, gy, gz, count, inv);
    if (vs != PI_OK) return vs;
    PI_CHECK_HIP(hipSetDevice(ctx->device));
    pi_tls_no_timing = true;
    const pi_status st = pi_interact_run(ctx, cells, o, rho, gx, gy, gz, count, inv, (hipStream_t)stream_,
                                         ctx->scratch, PI_NOALLOC_SCRATCH_RECORDS, true);
    pi_tls_no_timing = false;
    return st;
}

extern "C" pi_status pi_interact(pi_ctx *ctx, const pi_cells *cells, const pi_interact_opts *opts, float *rho,
                                 float *gx, float *gy, float *gz, int32_t *count, pi_invariants *inv,
                                 pi_stream stream_)
{
    if (!ctx || !cells || cells->ctx != ctx) return PI_EINVAL;
    if (!pi_cells_ready(cells)) return PI_ESTATE;
    pi_interact_opts o;
    memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    const pi_status vs = pi_check_interact_opts(o, cells->n, rho, gx, gy, gz, count, inv);
    if (vs != PI_OK) return vs;
    PI_CHECK_HIP(hipSetDevice(ctx->device));
    return pi_interact_run(ctx, cells, o, rho, gx, gy, gz, count, inv, (hipStream_t)stream_, cells->partials,
                           cells->cap_partials, false);
}
