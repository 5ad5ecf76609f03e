// Binning (paper Sec. 2 and Fig. 1): the cell of every particle, per-cell
// counts, the exclusive prefix sum of the counts (n_cells + 1 entries, last =
// n) and the particles moved into a cell-sorted order.  The order inside a
// cell is ascending original index: the paper places particles inside their
// cell with atomics in any order; fixing the order makes every later result
// reproducible.
//
// On MI355X the move is a least-significant-digit radix sort of the cell ids,
// 8 bits per pass, which is stable by construction and keeps every HBM access
// coalesced (the input order is a random permutation of the cells, so a
// scatter by per-particle atomics costs a whole cache line per 4-byte access).
// Per pass, in launch order on the caller's stream:
//   k_radix_hist     per 4096-key tile: LDS histogram of the pass's digit,
//                    stored digit-major (digit * tiles + tile)
//   k_digit_scan     exclusive scan of each digit's per-tile counts (one
//                    workgroup per digit, wave64 DPP scans) -> where each
//                    (digit, tile) run starts among that digit's keys
//   k_radix_scatter  per tile: stable rank of every key among the tile's
//                    keys with the same digit (wave64 ballots + per-wave
//                    counters), the tile reordered by digit in LDS, then
//                    written out in runs (key, index, x, y, z, w)
// The first pass computes the cell id from the position (float32 decision,
// see axis_index); the last pass writes the final arrays perm, cell and the
// cell-relative coordinates.  Counts, offsets and M_C then come from the
// runs of equal ids in the sorted cell ids (k_cell_ranges: wave ballots,
// each count and offset written once).
#include <string.h>

#include "pi_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kScanItems = 16;                 // histogram entries per thread and round (digit scan)
constexpr int kScanTile = kBlock * kScanItems; // 4096 entries per round
constexpr int kSortItems = 16;
constexpr int kSortTile = kBlock * kSortItems; // 4096 keys per sort tile
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
#ifndef PI_SCATTER_BLOCK
#define PI_SCATTER_BLOCK 512
#endif
constexpr int kSBlock = PI_SCATTER_BLOCK;     // scatter threads per tile (256, 512 or 1024)
constexpr int kSItems = kSortTile / kSBlock;  // keys per thread
static_assert(kSBlock >= kRadix && kSBlock <= 1024 && kSortTile % kSBlock == 0, "scatter block size");

// p[0 .. n) = v, four entries per thread (p 16-byte aligned)
__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t *p, int64_t n, int32_t v)
{
    const int64_t i = 4 * ((int64_t)blockIdx.x * kBlock + threadIdx.x);
    if (i + 3 < n) {
        *reinterpret_cast<int4 *>(p + i) = make_int4(v, v, v, v);
    } else {
        for (int64_t q = i; q < n; ++q) p[q] = v;
    }
}

// ------------------------------------------------------------- radix sort

// Exclusive scan, in place, of each digit's per-tile counts (the histogram is
// digit-major, so a digit's counts are contiguous); one workgroup per digit,
// 4096 entries per round; the digit's total goes to dtot[digit].
__global__ __launch_bounds__(kBlock) void k_digit_scan(int32_t *hist, int32_t ntiles, int32_t *dtot)
{
    __shared__ int32_t wsum[4];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int32_t *h = hist + (int64_t)blockIdx.x * ntiles;
    int32_t carry = 0;
    for (int32_t base = 0; base < ntiles; base += kScanTile) {
        const int32_t t0 = base + (int32_t)threadIdx.x * kScanItems;
        int32_t v[kScanItems];
        int32_t sum = 0;
#pragma unroll
        for (int q = 0; q < kScanItems; ++q) {
            v[q] = t0 + q < ntiles ? h[t0 + q] : 0;
            sum += v[q];
        }
        const int32_t inc = wave_incl_scan(sum);
        if (lane == 63) wsum[wid] = inc;
        __syncthreads();
        int32_t run = carry + inc - sum;
        for (int k = 0; k < wid; ++k) run += wsum[k];
        const int32_t round_total = (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
#pragma unroll
        for (int q = 0; q < kScanItems; ++q) {
            if (t0 + q < ntiles) h[t0 + q] = run;
            run += v[q];
        }
        carry += round_total;
        __syncthreads(); // wsum is rewritten by the next round
    }
    if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

// Cell id of a position (X fastest, Fig. 1).  A particle outside the box
// raises the error bit and is put in the last cell, so that every kernel
// stays inside its buffers; the results of that call are then unspecified.
__device__ __forceinline__ uint32_t cell_key(float x, float y, float z, const GridDev &g, uint32_t *err)
{
    int32_t ix, iy, iz;
    const int ok = (int)axis_index(x, g.ox, g.w, g.nx, ix) & (int)axis_index(y, g.oy, g.w, g.ny, iy) &
                   (int)axis_index(z, g.oz, g.w, g.nz, iz);
    if (!ok) {
        atomicOr(err, PI_DERR_RANGE);
        return (uint32_t)g.nx * (uint32_t)g.ny * (uint32_t)g.nz - 1u;
    }
    return (uint32_t)(ix + g.nx * (iy + g.ny * iz));
}

// System owning global particle e (systems concatenated in order).
__device__ __forceinline__ int sys_of_particle(const SysDev *sys, int nsys, int64_t e)
{
    int lo = 0, hi = nsys; // sys[lo].first <= e < sys[hi].first
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sys[mid].first <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// The same, for e known to lie in one of the systems lo .. hi (particles
// are stored in system order, so those of one sort tile lie between the
// systems of its first and last particle, mostly one system: then no load).
__device__ __forceinline__ int sys_of_particle_in(const SysDev *sys, int lo, int hi, int64_t e)
{
    ++hi; // sys[lo].first <= e < sys[hi].first (hi may be one past the table)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (sys[mid].first <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// System owning global cell key, between the two coarse-index entries
// around it (systems have at least one cell, so a block of 2^10 cells spans
// few of them).
__device__ __forceinline__ int sys_of_cell(const SysDev *sys, const int32_t *hint, uint32_t key)
{
    const uint32_t blk = key >> kCellHintShift;
    int lo = hint[blk], hi = hint[blk + 1] + 1; // sys[lo].cell_base <= key < sys[hi].cell_base
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((uint32_t)sys[mid].cell_base <= key) lo = mid; else hi = mid;
    }
    return lo;
}

struct SortArgs {
    int32_t n;
    int32_t ntiles;
    int32_t shift;
    GridDev g;
    const SysDev *sys; // batch mode: system table (nsys entries), else null
    int32_t nsys;
    const int32_t *cell_hint; // batch mode: coarse cell-to-system index
    // the first pass reads the caller's arrays
    const float *x, *y, *z, *w;
    // later passes read the previous pass's records: (cell id, original
    // index) and the payload (x, y, z, w)
    const uint2 *kv_in;
    const float4 *p_in;
    // every pass but the last writes records of the same two kinds
    // (ping-pong buffers)
    uint2 *kv_out;
    float4 *p_out;
    // the last pass writes the final arrays in sorted order: local cell id,
    // original index, cell-relative (x, y, z) and w; in batch mode also the
    // global cell ids (for the run count)
    int32_t *cell, *perm;
    float4 *xyzw;
    uint32_t *ids;
    const int32_t *gbase; // per digit: exclusive scan of its per-tile counts
    const int32_t *dtot;  // per digit: total count
    int32_t *hist;
    uint32_t *err;
};

// Systems of the first and last particle of the sort tile starting at
// particle `base` (batch mode).
struct TileSys {
    int lo, hi;
};

__device__ __forceinline__ TileSys tile_systems(const SortArgs &a, int64_t base)
{
    const int64_t end = min(base + (int64_t)kSortTile, (int64_t)a.n) - 1;
    return TileSys{sys_of_particle(a.sys, a.nsys, base), sys_of_particle(a.sys, a.nsys, end)};
}

// Global cell key of caller particle e (of the tile whose systems are ts)
// at position (x, y, z).
template <bool BATCH>
__device__ __forceinline__ uint32_t key_at(const SortArgs &a, const TileSys &ts, int64_t e, float x, float y,
                                           float z)
{
    if (!BATCH) return cell_key(x, y, z, a.g, a.err);
    const SysDev &s = a.sys[sys_of_particle_in(a.sys, ts.lo, ts.hi, e)];
    return (uint32_t)s.cell_base + cell_key(x, y, z, s.g, a.err);
}

template <bool FIRST, bool BATCH>
__global__ __launch_bounds__(kBlock) void k_radix_hist(SortArgs a)
{
    __shared__ int32_t h[4][kRadix]; // one histogram per wavefront
    const int wid = threadIdx.x >> 6;
    for (int w = 0; w < 4; ++w) h[w][threadIdx.x] = 0;
    // all of the tile's loads first (indices past the end clamped; their
    // keys are not counted)
    // (each XCD takes a contiguous run of tiles: neighbouring tiles share
    // its L2, which merges their partial-line writes of a histogram column)
    const int32_t tile = (int32_t)xcd_remap(blockIdx.x, gridDim.x);
    const int64_t base = (int64_t)tile * kSortTile;
    const int64_t last = (int64_t)a.n - 1;
    uint32_t key[kSortItems];
    if (FIRST) {
        const TileSys ts = BATCH ? tile_systems(a, base) : TileSys{0, 0};
        float px[kSortItems], py[kSortItems], pz[kSortItems];
#pragma unroll
        for (int q = 0; q < kSortItems; ++q) {
            const int64_t e = min(base + q * kBlock + threadIdx.x, last);
            px[q] = a.x[e];
            py[q] = a.y[e];
            pz[q] = a.z[e];
        }
#pragma unroll
        for (int q = 0; q < kSortItems; ++q)
            key[q] = key_at<BATCH>(a, ts, min(base + q * kBlock + threadIdx.x, last), px[q], py[q], pz[q]);
    } else {
#pragma unroll
        for (int q = 0; q < kSortItems; ++q) key[q] = a.kv_in[min(base + q * kBlock + threadIdx.x, last)].x;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kSortItems; ++q)
        if (base + q * kBlock + threadIdx.x < a.n) atomicAdd(&h[wid][(key[q] >> a.shift) & (kRadix - 1)], 1);
    __syncthreads();
    const int d = threadIdx.x;
    a.hist[(int64_t)d * a.ntiles + tile] = (h[0][d] + h[1][d]) + (h[2][d] + h[3][d]);
}

// Lanes of the wavefront whose digit equals this lane's (among `valid`).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t valid)
{
    uint64_t m = valid;
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        const uint64_t bal = __ballot((d >> b) & 1);
        m &= ((d >> b) & 1u) ? bal : ~bal;
    }
    return m;
}

// Local cell id of global key `key` and the position relative to that
// cell's low corner, fma(-i, w, x - o) per axis (the cell coordinates come
// from the id by two exact multiply-high divisions).
template <bool BATCH>
__device__ __forceinline__ uint32_t to_cell_relative(const SortArgs &a, uint32_t key, float &x, float &y, float &z)
{
    GridDev g = a.g;
    uint32_t lc = key;
    if (BATCH) {
        const SysDev &sd = a.sys[sys_of_cell(a.sys, a.cell_hint, key)];
        lc = key - (uint32_t)sd.cell_base;
        g = sd.g;
    }
    const int32_t iz = (int32_t)div_by(lc, g.mxy);
    const int32_t rem = (int32_t)lc - iz * g.nx * g.ny;
    const int32_t iy = (int32_t)div_by((uint32_t)rem, g.mx);
    const int32_t ix = rem - iy * g.nx;
    x = __builtin_fmaf(-(float)ix, g.w, x - g.ox);
    y = __builtin_fmaf(-(float)iy, g.w, y - g.oy);
    z = __builtin_fmaf(-(float)iz, g.w, z - g.oz);
    return lc;
}

// (LDS allows two workgroups, i.e. 4 wavefronts per SIMD: registers are
// budgeted for that, so the prefetched tile stays in registers)
template <bool FIRST, bool LAST, bool BATCH>
__global__ __launch_bounds__(kSBlock) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_radix_scatter(SortArgs a)
{
    constexpr int W = kSBlock / 64;      // wavefronts per block
    __shared__ int32_t wcnt[W][kRadix];  // per-wave digit counters, then wave bases
    __shared__ int32_t lstart[kRadix];   // tile-local start of each digit
    __shared__ int32_t gdst[kRadix];     // global start of each digit's run
    __shared__ int32_t scan_tmp[4];
    __shared__ int32_t dscan_tmp[4];
    // reorder buffer: the (key, index) records (8 bytes per position; 16
    // in the last pass of a batch, which also carries the global id), then
    // the payload (16 bytes); plus a spare slot
    __shared__ float4 lbuf[kSortTile + 1];

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    // (each XCD takes a contiguous run of tiles: the two ends of a digit's
    // run, written by neighbouring tiles, meet in one L2, as do the
    // per-tile digit offsets they read)
    const int32_t tile = (int32_t)xcd_remap(blockIdx.x, gridDim.x);
    const int64_t tile_base = (int64_t)tile * kSortTile;
    for (int i = tid; i < W * kRadix; i += kSBlock) (&wcnt[0][0])[i] = 0;
    // this tile's digit offsets (threads 0..255), loaded with the tile
    const int d = tid & (kRadix - 1);
    const int32_t dt = tid < kRadix ? a.dtot[d] : 0;
    const int32_t gb = tid < kRadix ? a.gbase[(int64_t)d * a.ntiles + tile] : 0;

    // 0. the whole tile's keys and payload in registers: every global load
    //    of the tile is issued before the first barrier (indices past the
    //    end are clamped, so the loads need no branches; the clamped copies
    //    are never ranked or written)
    auto elem = [&](int r) { return tile_base + wid * (kSItems * 64) + r * 64 + lane; };
    const int64_t last_e = (int64_t)a.n - 1;
    uint32_t key[kSItems];
    int32_t pidx[kSItems];
    float px[kSItems], py[kSItems], pz[kSItems], pw[kSItems];
#pragma unroll
    for (int r = 0; r < kSItems; ++r) {
        const int64_t e = min(elem(r), last_e);
        if (FIRST) {
            px[r] = a.x[e];
            py[r] = a.y[e];
            pz[r] = a.z[e];
            pw[r] = a.w[e];
            pidx[r] = (int32_t)e;
        } else {
            const uint2 kv = a.kv_in[e];
            key[r] = kv.x;
            pidx[r] = (int32_t)kv.y;
            const float4 q = a.p_in[e];
            px[r] = q.x;
            py[r] = q.y;
            pz[r] = q.z;
            pw[r] = q.w;
        }
    }
    if (FIRST) {
        const TileSys ts = BATCH ? tile_systems(a, tile_base) : TileSys{0, 0};
#pragma unroll
        for (int r = 0; r < kSItems; ++r) key[r] = key_at<BATCH>(a, ts, min(elem(r), last_e), px[r], py[r], pz[r]);
    }
    __syncthreads();

    // 1. stable rank of each key among the keys of its wavefront's chunk with
    //    the same digit (rounds in key order, lanes in key order)
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int32_t pos[kSItems];
#pragma unroll
    for (int r = 0; r < kSItems; ++r) {
        const bool valid = elem(r) < a.n;
        const uint32_t d = (key[r] >> a.shift) & (kRadix - 1);
        const uint64_t vmask = __ballot(valid);
        const uint64_t peers = match_digit(d, vmask);
        int32_t rk = -1;
        if (valid) {
            const int32_t before = __popcll(peers & lt);
            const int32_t base = wcnt[wid][d];
            rk = base + before;
            if (before == 0) wcnt[wid][d] = base + __popcll(peers);
        }
        pos[r] = rk; // rank within the wave for now, -1 past the end
    }
    __syncthreads();

    // 2. per digit (threads 0..255): bases of the waves, tile total,
    //    tile-local start (scan over the first four wavefronts), and where
    //    the digit's run of this tile starts in the output: the totals of
    //    the smaller digits plus this digit's count in the tiles before
    int32_t tot = 0;
    if (tid < kRadix) {
        int32_t run = 0;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int32_t c = wcnt[k][d];
            wcnt[k][d] = run;
            run += c;
        }
        tot = run;
    }
    const int32_t inc = wave_incl_scan(tot);
    const int32_t dinc = wave_incl_scan(dt);
    if (tid < kRadix && lane == 63) {
        scan_tmp[wid] = inc;
        dscan_tmp[wid] = dinc;
    }
    __syncthreads();
    if (tid < kRadix) {
        int32_t wofs = 0, dofs = 0;
        for (int k = 0; k < wid; ++k) {
            wofs += scan_tmp[k];
            dofs += dscan_tmp[k];
        }
        lstart[d] = wofs + inc - tot;
        gdst[d] = dofs + dinc - dt + gb;
    }
    __syncthreads();

    // 3. tile-local position of every key (consecutive positions of one
    //    digit go to consecutive addresses, so the copies below are
    //    coalesced runs); keys past the end get the spare slot kSortTile,
    //    written but never read
#pragma unroll
    for (int r = 0; r < kSItems; ++r) {
        const uint32_t dg = (key[r] >> a.shift) & (kRadix - 1);
        pos[r] = pos[r] >= 0 ? lstart[dg] + wcnt[wid][dg] + pos[r] : kSortTile;
    }
    const int32_t nvalid = (int32_t)min((int64_t)kSortTile, (int64_t)a.n - tile_base);

    // 4. the (key, index) records, then the payload, reordered through LDS
    //    and written out in runs; the last pass writes the final arrays
    //    instead (local cell id and index, cell-relative payload).  The
    //    reader of position p takes the digit from the record there, and p's
    //    destination is that digit's global start plus p's offset in the
    //    digit's tile-local run.
    auto dest = [&](int p, uint32_t k) {
        const uint32_t dg = (k >> a.shift) & (kRadix - 1);
        return gdst[dg] + (p - lstart[dg]);
    };
    int32_t dst[kSItems];
    if (LAST && BATCH) {
        uint4 *lb16 = reinterpret_cast<uint4 *>(lbuf);
#pragma unroll
        for (int r = 0; r < kSItems; ++r) {
            const uint32_t lc = to_cell_relative<BATCH>(a, key[r], px[r], py[r], pz[r]);
            lb16[pos[r]] = make_uint4(lc, (uint32_t)pidx[r], key[r], 0u);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kSItems; ++k) {
            const int p = tid + k * kSBlock;
            dst[k] = 0;
            if (p < nvalid) {
                const uint4 c = lb16[p];
                dst[k] = dest(p, c.z);
                a.cell[dst[k]] = (int32_t)c.x;
                a.perm[dst[k]] = (int32_t)c.y;
                a.ids[dst[k]] = c.z;
            }
        }
    } else {
        // (in the last pass of one system the local cell id is the key)
        uint2 *lb8 = reinterpret_cast<uint2 *>(lbuf);
#pragma unroll
        for (int r = 0; r < kSItems; ++r) {
            const uint32_t k0 = LAST ? to_cell_relative<BATCH>(a, key[r], px[r], py[r], pz[r]) : key[r];
            lb8[pos[r]] = make_uint2(k0, (uint32_t)pidx[r]);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kSItems; ++k) {
            const int p = tid + k * kSBlock;
            dst[k] = 0;
            if (p < nvalid) {
                const uint2 c = lb8[p];
                dst[k] = dest(p, c.x);
                if (LAST) {
                    a.cell[dst[k]] = (int32_t)c.x;
                    a.perm[dst[k]] = (int32_t)c.y;
                } else {
                    a.kv_out[dst[k]] = c;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSItems; ++r) lbuf[pos[r]] = make_float4(px[r], py[r], pz[r], pw[r]);
    __syncthreads();
    float4 *pout = LAST ? a.xyzw : a.p_out;
#pragma unroll
    for (int k = 0; k < kSItems; ++k) {
        const int p = tid + k * kSBlock;
        if (p < nvalid) pout[dst[k]] = lbuf[p];
    }
}

// After the last pass: the per-cell counts and the exclusive offsets
// straight from the sorted global cell ids, with no separate scan (Fig. 1:
// offsets[c] is the number of particles in cells before c, which in sorted
// order is the position of the first id >= c).  A wavefront takes 256
// consecutive sorted ids (positions [wbase, wbase + 256)) and owns the cells
// (before, last]: `before` is the id just before its range (-1 for the
// first) and `last` the last id in it.  It writes those cells 64 at a time,
// each lane finding its cell's rank among the wavefront's ids by an 8-step
// binary search in LDS, so every store is coalesced and every entry is
// written exactly once:
//   offsets[c] = wbase + #(ids in range < c)
//   counts[c]  = #(ids in range == c), except that the run of `last` may
//                continue past the range: its end is found in the 64 ids
//                after it, else by galloping over the sorted ids.
// The wavefront holding position n - 1 also writes the cells after its
// last id (offset n, count 0) and offsets[nc] = n.  Each wavefront writes its
// largest count to wmax[wave]; k_max_reduce folds those into M_C.  (An
// atomicMax per wavefront on M_C itself serialised on that one address: 750
// µs at 2^24 ids.)
constexpr int kRunIds = 256; // sorted ids per wavefront

__global__ __launch_bounds__(kBlock) void k_cell_ranges(int32_t n, int32_t nc, const uint32_t *__restrict__ ids,
                                                        int32_t *__restrict__ counts, int32_t *__restrict__ offsets,
                                                        int32_t *__restrict__ wmaxes)
{
    __shared__ uint32_t sid[kBlock / 64][kRunIds];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
    const int64_t wbase = wave * kRunIds;
    if (wbase >= n) return; // uniform over the wavefront (no barriers below)
    const int64_t lastpos = (int64_t)n - 1;
    const int64_t wend = wbase + kRunIds; // first position past the range
    uint32_t *s = sid[wid];
    // ids past n repeat ids[n-1], which keeps the range sorted
#pragma unroll
    for (int r = 0; r < kRunIds / 64; ++r) s[r * 64 + lane] = ids[min(wbase + r * 64 + lane, lastpos)];
    __builtin_amdgcn_wave_barrier(); // the lanes read each other's entries below
    const int32_t before = wbase > 0 ? (int32_t)ids[wbase - 1] : -1;
    const uint32_t after = ids[min(wend + lane, lastpos)];
    const int32_t last = (int32_t)s[kRunIds - 1];

    // end of the run of `last`: in the 64 ids after the range, else gallop
    const uint64_t cont = __ballot(wend + lane < n && after == (uint32_t)last);
    int64_t end;
    if (cont != ~0ull) {
        end = wend + (__ffsll((unsigned long long)~cont) - 1);
    } else {
        int64_t lo = wend + 63, hi = wend + 64, step = 64; // id lo == last
        while (hi < n && ids[hi] == (uint32_t)last) {
            lo = hi;
            hi = hi + step;
            step *= 2;
        }
        if (hi > n) hi = n;
        while (hi - lo > 1) {
            const int64_t mid = lo + (hi - lo) / 2;
            if (ids[mid] == (uint32_t)last) lo = mid; else hi = mid;
        }
        end = hi;
    }
    if (end > n) end = n;

    // number of ids in the range below c (lower bound over 256 sorted ids)
    auto rank = [&](int32_t c) {
        int32_t pos = 0;
#pragma unroll
        for (int step = kRunIds / 2; step > 0; step >>= 1)
            if ((int32_t)s[pos + step - 1] < c) pos += step;
        return pos;
    };
    // rounds of 63 cells: lane 63 ranks the cell after the round, so each
    // count is a difference of neighbouring lanes' ranks
    int32_t wmax = 0;
    for (int64_t c0 = (int64_t)before + 1; c0 <= last; c0 += 63) {
        const int32_t c = (int32_t)min(c0 + lane, (int64_t)last + 1);
        const int32_t rc = rank(c);
        const int32_t rnext = __shfl_down(rc, 1);
        if (lane < 63 && c <= last) {
            const int32_t cnt = c < last ? rnext - rc : (int32_t)(end - (wbase + rc));
            offsets[c] = (int32_t)wbase + rc;
            counts[c] = cnt;
            wmax = max(wmax, cnt);
        }
    }
    if (lastpos < wend) {
        // the cells after the last id
        for (int64_t c = (int64_t)last + 1 + lane; c < nc; c += 64) {
            offsets[c] = n;
            counts[c] = 0;
        }
        if (lane == 0) offsets[nc] = n;
    }
    wmax = wave_max(wmax);
    if (lane == 0) wmaxes[wave] = wmax;
}

// out[0] = max of v[0 .. count) (all >= 0), v 16-byte aligned: one
// workgroup of 1024 threads, 16-byte loads, sixteen in flight per thread.
__global__ __launch_bounds__(1024) void k_max_reduce(const int32_t *__restrict__ v, int32_t count,
                                                     int32_t *__restrict__ out)
{
    __shared__ int32_t part[16];
    const int4 *v4 = reinterpret_cast<const int4 *>(v);
    const int32_t n4 = count / 4;
    int32_t m = 0;
    for (int32_t i = threadIdx.x; i < n4; i += 16 * 1024) {
        int4 q[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) q[u] = i + u * 1024 < n4 ? v4[i + u * 1024] : make_int4(0, 0, 0, 0);
#pragma unroll
        for (int u = 0; u < 16; ++u) m = max(m, max(max(q[u].x, q[u].y), max(q[u].z, q[u].w)));
    }
    for (int32_t i = 4 * n4 + (int32_t)threadIdx.x; i < count; i += 1024) m = max(m, v[i]);
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x < 64) {
        m = threadIdx.x < 16 ? part[threadIdx.x] : 0;
        m = wave_max(m);
        if (threadIdx.x == 0) out[0] = m;
    }
}

// The sorted coordinates as four arrays, from the records (in order).
__global__ __launch_bounds__(kBlock) void k_split_records(int32_t n, const float4 *__restrict__ p, float *xs,
                                                          float *ys, float *zs, float *ws)
{
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n) return;
    const float4 q = p[e];
    xs[e] = q.x;
    ys[e] = q.y;
    zs[e] = q.z;
    ws[e] = q.w;
}

inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

} // namespace

bool pi_grid_valid(const pi_grid *g)
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

// Radix sort of n particles by global cell id, then counts and offsets.
// nsys == 0: one system on grid g0; else d_sys describes nsys concatenated
// systems with cells_total cells in all.
pi_status pi_bin_systems(pi_ctx *ctx, pi_cells *cells, const float *x, const float *y, const float *z,
                         const float *w, int64_t n, int64_t nc, int32_t nsys, const SysDev *d_sys,
                         const int32_t *d_cell_hint, const GridDev &g0, hipStream_t stream)
{
    const bool batch = nsys > 0;
    if (n > 0) {
        // 8-bit digits needed to sort keys 0 .. nc-1
        int bits = 1;
        while (bits < 31 && ((int64_t)1 << bits) < nc) ++bits;
        const int passes = (bits + kRadixBits - 1) / kRadixBits;
        const int32_t ntiles = (int32_t)((n + kSortTile - 1) / kSortTile);
        SortArgs a;
        memset(&a, 0, sizeof(a));
        a.n = (int32_t)n;
        a.ntiles = ntiles;
        a.g = g0;
        a.sys = d_sys;
        a.cell_hint = d_cell_hint;
        a.nsys = nsys;
        a.x = x;
        a.y = y;
        a.z = z;
        a.w = w;
        a.hist = cells->hist;
        a.gbase = cells->hist;
        a.dtot = cells->dtot;
        a.err = cells->d_err;
        a.cell = cells->cell;
        a.perm = cells->perm;
        a.xyzw = cells->xyzw;
        // the last pass writes no records, so its output record buffer is
        // free: in batch mode it takes the sorted global ids
        uint32_t *ids = batch ? reinterpret_cast<uint32_t *>(cells->skv[(passes - 1) & 1])
                              : reinterpret_cast<uint32_t *>(cells->cell);
        a.ids = ids;
        for (int p = 0; p < passes; ++p) {
            const bool first = p == 0, last = p == passes - 1;
            const int src = (p + 1) & 1, dst = p & 1;
            a.shift = p * kRadixBits;
            a.kv_in = cells->skv[src];
            a.p_in = cells->sp[src];
            a.kv_out = last ? nullptr : cells->skv[dst];
            a.p_out = last ? nullptr : cells->sp[dst];
            const dim3 grid(ntiles), block(kBlock);
            if (first && batch) PI_LAUNCH(ctx, "k_radix_hist", (k_radix_hist<true, true>), grid, block, 0, stream, a);
            else if (first) PI_LAUNCH(ctx, "k_radix_hist", (k_radix_hist<true, false>), grid, block, 0, stream, a);
            else PI_LAUNCH(ctx, "k_radix_hist", (k_radix_hist<false, false>), grid, block, 0, stream, a);
            PI_LAUNCH(ctx, "k_digit_scan", k_digit_scan, dim3(kRadix), dim3(kBlock), 0, stream, cells->hist, ntiles,
                      cells->dtot);
            const dim3 sb(kSBlock);
            const char *nm = "k_radix_scatter";
            if (first && last) {
                if (batch) PI_LAUNCH(ctx, nm, (k_radix_scatter<true, true, true>), grid, sb, 0, stream, a);
                else PI_LAUNCH(ctx, nm, (k_radix_scatter<true, true, false>), grid, sb, 0, stream, a);
            } else if (first) {
                if (batch) PI_LAUNCH(ctx, nm, (k_radix_scatter<true, false, true>), grid, sb, 0, stream, a);
                else PI_LAUNCH(ctx, nm, (k_radix_scatter<true, false, false>), grid, sb, 0, stream, a);
            } else if (last) {
                if (batch) PI_LAUNCH(ctx, nm, (k_radix_scatter<false, true, true>), grid, sb, 0, stream, a);
                else PI_LAUNCH(ctx, nm, (k_radix_scatter<false, true, false>), grid, sb, 0, stream, a);
            } else {
                PI_LAUNCH(ctx, nm, (k_radix_scatter<false, false, false>), grid, sb, 0, stream, a);
            }
        }
        // the per-wavefront maxima go to the histogram buffer, free after
        // the last pass (256 entries per 4096 particles, one per 256 needed)
        const int64_t waves = (n + kRunIds - 1) / kRunIds;
        PI_LAUNCH(ctx, "k_cell_ranges", k_cell_ranges, dim3(nblocks(waves * 64, kBlock)), dim3(kBlock), 0, stream,
                  (int32_t)n, (int32_t)nc, (const uint32_t *)ids, cells->counts, cells->offsets, cells->hist);
        PI_LAUNCH(ctx, "k_max_reduce", k_max_reduce, dim3(1), dim3(1024), 0, stream, (const int32_t *)cells->hist,
                  (int32_t)waves, cells->max_per_cell);
    } else {
        // no particles: every count and offset is zero, and M_C
        PI_LAUNCH(ctx, "k_fill_i32", k_fill_i32, dim3(nblocks((nc + 3) / 4, kBlock)), dim3(kBlock), 0, stream,
                  cells->counts, nc, 0);
        PI_LAUNCH(ctx, "k_fill_i32", k_fill_i32, dim3(nblocks((nc + 4) / 4, kBlock)), dim3(kBlock), 0, stream,
                  cells->offsets, nc + 1, 0);
        PI_LAUNCH(ctx, "k_fill_i32", k_fill_i32, dim3(1), dim3(kBlock), 0, stream, cells->max_per_cell, (int64_t)1,
                  0);
    }
    cells->soa_stale = n > 0;
    PI_CHECK_HIP(hipGetLastError());
    return PI_OK;
}

extern "C" pi_status pi_bin(pi_ctx *ctx, pi_cells *cells, const float *x, const float *y, const float *z,
                            const float *w, int64_t n, const pi_grid *grid, pi_stream stream_)
{
    if (!ctx || !cells || cells->ctx != ctx) return PI_EINVAL;
    // whatever happens below, the object no longer holds the previous
    // system: a failed call leaves it unbinned (sweeps and views then return
    // PI_ESTATE), a successful one marks the new system binned
    pi_cells_forget(cells);
    if (n < 0 || n >= ((int64_t)1 << 31)) return PI_EINVAL;
    if (n > 0 && (!x || !y || !z || !w)) return PI_EINVAL;
    if (!pi_grid_valid(grid)) return PI_EINVAL;
    hipStream_t stream = (hipStream_t)stream_;
    PI_CHECK_HIP(hipSetDevice(ctx->device));
    const int64_t nc = (int64_t)grid->dims[0] * grid->dims[1] * grid->dims[2];
    pi_status st = pi_ensure_capacity(cells, n, nc, stream);
    if (st != PI_OK) return st;
    cells->n = n;
    cells->n_cells = nc;
    cells->grid = *grid;
    cells->last_stream = stream;

    const GridDev g = grid_dev(*grid);
    st = pi_bin_systems(ctx, cells, x, y, z, w, n, nc, 0, nullptr, nullptr, g, stream);
    if (st != PI_OK) {
        pi_cells_forget(cells);
        return st;
    }
    cells->binned = true;
    return PI_OK;
}

pi_status pi_split_records(pi_ctx *ctx, pi_cells *cells)
{
    if (!cells->soa_stale) return PI_OK;
    PI_CHECK_HIP(hipSetDevice(ctx->device));
    const int64_t n = cells->n;
    PI_LAUNCH(ctx, "k_split_records", k_split_records, dim3(nblocks(n, kBlock)), dim3(kBlock), 0, cells->last_stream,
              (int32_t)n, (const float4 *)cells->xyzw, cells->xs, cells->ys, cells->zs, cells->ws);
    PI_CHECK_HIP(hipGetLastError());
    cells->soa_stale = false;
    return PI_OK;
}
