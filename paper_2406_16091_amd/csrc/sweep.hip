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

#include "pair.h"

namespace {

constexpr int kBlock = 256;

// One record of FP64 invariant partial sums per workgroup (64 bytes).
struct InvPartial {
    long long pairs;
    double net[3];
    double scale;
    double rho_sum;
    double pad[2];
};

struct SweepArgs {
    const int32_t *off;
    const int32_t *cell;
    const int32_t *perm;
    const float *xs, *ys, *zs, *ws;
    int64_t nc;
    int32_t n;
    int32_t nx, ny, nz;
    int32_t orig_order;
    float *rho, *gx, *gy, *gz;
    int32_t *count;
    InvPartial *partials;
    KernelConst k;
};

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
    __shared__ double red[4][6];
    for (int o = 32; o >= 1; o >>= 1) {
        cnt += __shfl_xor(cnt, o, 64);
        nx += __shfl_xor(nx, o, 64);
        ny += __shfl_xor(ny, o, 64);
        nz += __shfl_xor(nz, o, 64);
        sc += __shfl_xor(sc, o, 64);
        rs += __shfl_xor(rs, o, 64);
    }
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[wid][0] = (double)cnt;
        red[wid][1] = nx;
        red[wid][2] = ny;
        red[wid][3] = nz;
        red[wid][4] = sc;
        red[wid][5] = rs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        InvPartial p;
        p.pairs = (long long)(red[0][0] + red[1][0] + red[2][0] + red[3][0]);
        p.net[0] = ((red[0][1] + red[1][1]) + red[2][1]) + red[3][1];
        p.net[1] = ((red[0][2] + red[1][2]) + red[2][2]) + red[3][2];
        p.net[2] = ((red[0][3] + red[1][3]) + red[2][3]) + red[3][3];
        p.scale = ((red[0][4] + red[1][4]) + red[2][4]) + red[3][4];
        p.rho_sum = ((red[0][5] + red[1][5]) + red[2][5]) + red[3][5];
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
// neighbour rows overlap in cache).
template <int PREC, bool INV>
__global__ __launch_bounds__(kBlock) void k_sweep_nolds(SweepArgs a)
{
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int32_t k = (int32_t)(lb * kBlock + threadIdx.x);
    const int32_t nb = a.off[a.nc];
    const bool active = k < nb && k < a.n;
    Target<PREC, INV> T;
    float wi = 0.f;
    if (active) {
        const int32_t c = a.cell[k];
        const int32_t ix = c % a.nx, iy = (c / a.nx) % a.ny, iz = c / (a.nx * a.ny);
        const float xi = a.xs[k], yi = a.ys[k], zi = a.zs[k];
        wi = a.ws[k];
        const float W = a.k.w;
        for (int dz = -1; dz <= 1; ++dz) {
            const int32_t cz = iz + dz;
            if (cz < 0 || cz >= a.nz) continue;
            const float tz = zi - (float)dz * W;
            for (int dy = -1; dy <= 1; ++dy) {
                const int32_t cy = iy + dy;
                if (cy < 0 || cy >= a.ny) continue;
                const float ty = yi - (float)dy * W;
                const int64_t rb = (int64_t)a.nx * (cy + (int64_t)a.ny * cz);
                for (int dx = -1; dx <= 1; ++dx) {
                    const int32_t cx = ix + dx;
                    if (cx < 0 || cx >= a.nx) continue;
                    const float tx = xi - (float)dx * W;
                    const int32_t j0 = a.off[rb + cx], j1 = a.off[rb + cx + 1];
                    for (int32_t j = j0; j < j1; ++j) {
                        const float ddx = tx - a.xs[j], ddy = ty - a.ys[j], ddz = tz - a.zs[j];
                        const float t = sq_dist(ddx, ddy, ddz);
                        if (t < a.k.hi && j != k && inside_cutoff(ddx, ddy, ddz, t, a.k))
                            T.accept(ddx, ddy, ddz, t, a.ws[j], a.k);
                    }
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

// ------------------------------------------------------------------ LDS tiles
// A workgroup owns a tile of TX x TY x TZ target cells.  The tile's halo box
// ((TX+2) x (TY+2) x (TZ+2) cells, clipped to the grid) is staged in LDS:
// each X-row of the halo is one contiguous range of the sorted arrays, so
// the load is (TY+2)(TZ+2) coalesced row copies.  The LDS position of every
// row comes from an exclusive scan of the row counts, which are differences
// of global offsets (the paper's local-offset construction, Sec. 5.1).
// TY = TZ = 1 is the X-pencil (Sec. 5.2), with all nine neighbour pencils
// resident at once instead of streamed; larger TY, TZ is the full sub-box
// (Sec. 5.1).  A tile whose halo holds more than CAP particles reads its
// sources from global memory instead (same order, same results).
template <int TX, int TY, int TZ, int CAP, int PREC, bool INV>
__global__ __launch_bounds__(kBlock) void k_sweep_tile(SweepArgs a, int32_t ntx, int32_t nty)
{
    constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
    constexpr int R = HY * HZ;   // halo rows
    constexpr int TR = TY * TZ;  // target rows
    static_assert(R <= 64 && TR <= 64, "row tables are scanned by one wavefront");
    __shared__ float4 sp[CAP];
    __shared__ int32_t cs[R][HX + 1];
    __shared__ int32_t rstart[R + 1];
    __shared__ int32_t gstart[R];
    __shared__ int32_t tstart[TR + 1];
    __shared__ int32_t tfirst[TR];

    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int32_t bx = (int32_t)(lb % (uint32_t)ntx);
    const int32_t by = (int32_t)((lb / (uint32_t)ntx) % (uint32_t)nty);
    const int32_t bz = (int32_t)(lb / ((uint32_t)ntx * (uint32_t)nty));
    const int32_t x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    const int32_t cxlo = max(x0 - 1, 0);
    const int32_t cxhi = min(x0 + TX, a.nx - 1);
    const int32_t ncx = cxhi - cxlo + 1;
    const int32_t txhi = min(x0 + TX, a.nx); // exclusive end of target cells
    const int tid = threadIdx.x;

    // 1. halo row ranges and their LDS starts; target row ranges
    if (tid < 64) {
        int32_t cnt = 0, gs = 0;
        if (tid < R) {
            const int32_t y = y0 - 1 + tid % HY, z = z0 - 1 + tid / HY;
            if (y >= 0 && y < a.ny && z >= 0 && z < a.nz) {
                const int64_t rb = (int64_t)a.nx * (y + (int64_t)a.ny * z);
                gs = a.off[rb + cxlo];
                cnt = a.off[rb + cxhi + 1] - gs;
            }
        }
        const int32_t inc = wave_incl_scan(cnt);
        if (tid < R) {
            rstart[tid] = inc - cnt;
            gstart[tid] = gs;
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
        }
        if (tid == TR - 1) tstart[TR] = tinc;
    }
    __syncthreads();
    const int32_t total = rstart[R];
    const bool staged = total <= CAP;

    // 2. start of every halo cell in source space (LDS index when staged,
    //    sorted global index otherwise)
    for (int e = tid; e < R * (HX + 1); e += kBlock) {
        const int r = e / (HX + 1), jj = e % (HX + 1);
        const int32_t y = y0 - 1 + r % HY, z = z0 - 1 + r / HY;
        int32_t v = 0;
        if (jj <= ncx && y >= 0 && y < a.ny && z >= 0 && z < a.nz) {
            const int64_t rb = (int64_t)a.nx * (y + (int64_t)a.ny * z);
            const int32_t g = a.off[rb + cxlo + jj];
            v = staged ? g - gstart[r] + rstart[r] : g;
        }
        cs[r][jj] = v;
    }
    // 3. stage the halo particles (flat index -> row by binary search)
    if (staged) {
        for (int32_t f = tid; f < total; f += kBlock) {
            int lo = 0, hi = R; // rstart[lo] <= f < rstart[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (rstart[mid] <= f) lo = mid; else hi = mid;
            }
            const int32_t g = gstart[lo] + (f - rstart[lo]);
            sp[f] = make_float4(a.xs[g], a.ys[g], a.zs[g], a.ws[g]);
        }
    }
    __syncthreads();

    // 4. targets
    const int32_t ntarget = tstart[TR];
    long long icnt = 0;
    double inx = 0, iny = 0, inz = 0, isc = 0, irs = 0;
    const float W = a.k.w;
    for (int32_t f = tid; f < ntarget; f += kBlock) {
        int lo = 0, hi = TR;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (tstart[mid] <= f) lo = mid; else hi = mid;
        }
        const int32_t k = tfirst[lo] + (f - tstart[lo]);
        const int32_t ty_ = lo % TY, tz_ = lo / TY;
        const int32_t y = y0 + ty_, z = z0 + tz_;
        const int32_t ix = a.cell[k] - a.nx * (y + a.ny * z);
        const int hr = (ty_ + 1) + HY * (tz_ + 1); // halo row of the target
        float xi, yi, zi, wi;
        int32_t self;
        if (staged) {
            self = rstart[hr] + (k - gstart[hr]);
            const float4 p = sp[self];
            xi = p.x; yi = p.y; zi = p.z; wi = p.w;
        } else {
            self = k;
            xi = a.xs[k]; yi = a.ys[k]; zi = a.zs[k]; wi = a.ws[k];
        }
        Target<PREC, INV> T;
        for (int dz = -1; dz <= 1; ++dz) {
            const int32_t cz = z + dz;
            if (cz < 0 || cz >= a.nz) continue;
            const float tz = zi - (float)dz * W;
            for (int dy = -1; dy <= 1; ++dy) {
                const int32_t cy = y + dy;
                if (cy < 0 || cy >= a.ny) continue;
                const float tyy = yi - (float)dy * W;
                const int r = (ty_ + 1 + dy) + HY * (tz_ + 1 + dz);
                for (int dx = -1; dx <= 1; ++dx) {
                    const int32_t cx = ix + dx;
                    if (cx < 0 || cx >= a.nx) continue;
                    const float tx = xi - (float)dx * W;
                    const int jj = cx - cxlo;
                    const int32_t j0 = cs[r][jj], j1 = cs[r][jj + 1];
                    if (staged) {
                        for (int32_t j = j0; j < j1; ++j) {
                            const float4 s = sp[j];
                            const float ddx = tx - s.x, ddy = tyy - s.y, ddz = tz - s.z;
                            const float t = sq_dist(ddx, ddy, ddz);
                            if (t < a.k.hi && j != self && inside_cutoff(ddx, ddy, ddz, t, a.k))
                                T.accept(ddx, ddy, ddz, t, s.w, a.k);
                        }
                    } else {
                        for (int32_t j = j0; j < j1; ++j) {
                            const float ddx = tx - a.xs[j], ddy = tyy - a.ys[j], ddz = tz - a.zs[j];
                            const float t = sq_dist(ddx, ddy, ddz);
                            if (t < a.k.hi && j != self && inside_cutoff(ddx, ddy, ddz, t, a.k))
                                T.accept(ddx, ddy, ddz, t, a.ws[j], a.k);
                        }
                    }
                }
            }
        }
        write_target(a, k, T);
        if (INV) {
            long long c1;
            double a1, a2, a3, a4, a5;
            target_invariants(T, wi, c1, a1, a2, a3, a4, a5);
            icnt += c1;
            inx += a1;
            iny += a2;
            inz += a3;
            isc += a4;
            irs += a5;
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

KernelConst make_kernel_const(float rc, float cell_w)
{
    KernelConst k;
    const float h = rc;
    const double hd = (double)h;
    const double r2 = hd * hd; // exact
    const double u = ldexp(1.0, -24);
    k.lo = nextafterf((float)(r2 * (1.0 - 4.0 * u)), 0.0f);
    k.hi = nextafterf((float)(r2 * (1.0 + 4.0 * u)), INFINITY);
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

// Tile shapes compiled in.  id: 0 = no LDS; 1.. = tiles.
struct TileCfg {
    int id;
    int tx, ty, tz, cap;
    int sweep; // PI_SWEEP_PENCIL / PI_SWEEP_SUBBOX
};

const TileCfg kTiles[] = {
    {1, 254, 1, 1, 3072, PI_SWEEP_PENCIL},
    {2, 62, 1, 1, 3072, PI_SWEEP_PENCIL},
    {3, 30, 1, 1, 3072, PI_SWEEP_PENCIL},
    {4, 8, 8, 4, 1536, PI_SWEEP_SUBBOX},
    {5, 4, 4, 4, 2048, PI_SWEEP_SUBBOX},
    {6, 4, 4, 2, 2048, PI_SWEEP_SUBBOX},
};

template <int TX, int TY, int TZ, int CAP, int PREC, bool INV>
void launch_tile(pi_ctx *ctx, const char *name, const SweepArgs &a, hipStream_t s, unsigned &nblk)
{
    const int32_t ntx = (a.nx + TX - 1) / TX, nty = (a.ny + TY - 1) / TY, ntz = (a.nz + TZ - 1) / TZ;
    nblk = (unsigned)((int64_t)ntx * nty * ntz);
    PI_LAUNCH(ctx, name, (k_sweep_tile<TX, TY, TZ, CAP, PREC, INV>), dim3(nblk), dim3(kBlock), 0, s, a, ntx, nty);
}

template <int PREC, bool INV>
void launch_sweep(pi_ctx *ctx, int tile_id, const SweepArgs &a, hipStream_t s, unsigned &nblk)
{
    switch (tile_id) {
    case 1: launch_tile<254, 1, 1, 3072, PREC, INV>(ctx, "k_sweep_tile<254,1,1>", a, s, nblk); break;
    case 2: launch_tile<62, 1, 1, 3072, PREC, INV>(ctx, "k_sweep_tile<62,1,1>", a, s, nblk); break;
    case 3: launch_tile<30, 1, 1, 3072, PREC, INV>(ctx, "k_sweep_tile<30,1,1>", a, s, nblk); break;
    case 4: launch_tile<8, 8, 4, 1536, PREC, INV>(ctx, "k_sweep_tile<8,8,4>", a, s, nblk); break;
    case 5: launch_tile<4, 4, 4, 2048, PREC, INV>(ctx, "k_sweep_tile<4,4,4>", a, s, nblk); break;
    case 6: launch_tile<4, 4, 2, 2048, PREC, INV>(ctx, "k_sweep_tile<4,4,2>", a, s, nblk); break;
    default:
        nblk = (unsigned)((a.n + kBlock - 1) / kBlock);
        if (nblk == 0) nblk = 1;
        PI_LAUNCH(ctx, "k_sweep_nolds", (k_sweep_nolds<PREC, INV>), dim3(nblk), dim3(kBlock), 0, s, a);
        break;
    }
}

int pick_tile(const pi_interact_opts &o, double ppc)
{
    if (o.sweep == PI_SWEEP_NOLDS) return 0;
    if (o.sweep == PI_SWEEP_PENCIL || o.sweep == PI_SWEEP_SUBBOX) {
        // an explicit tile shape must be one of the compiled ones
        if (o.tile[0] > 0) {
            for (const TileCfg &t : kTiles)
                if (t.sweep == o.sweep && t.tx == o.tile[0] && t.ty == o.tile[1] && t.tz == o.tile[2]) return t.id;
            return -1;
        }
        if (o.sweep == PI_SWEEP_PENCIL) return ppc <= 2.0 ? 1 : (ppc <= 5.0 ? 2 : 3);
        return ppc <= 2.0 ? 4 : (ppc <= 5.0 ? 5 : 6);
    }
    // AUTO
    return ppc <= 2.0 ? 4 : (ppc <= 5.0 ? 5 : 6);
}

} // namespace

extern "C" pi_status pi_interact(pi_ctx *ctx, const pi_cells *cells, const pi_interact_opts *opts, float *rho,
                                 float *gx, float *gy, float *gz, int32_t *count, pi_invariants *inv,
                                 pi_stream stream_)
{
    if (!ctx || !cells || cells->ctx != ctx) return PI_EINVAL;
    if (!cells->binned) return PI_ESTATE;
    pi_interact_opts o;
    memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    if (o.precision < PI_PREC_COMPENSATED || o.precision > PI_PREC_FP64ACC) return PI_EINVAL;
    if (o.sweep < PI_SWEEP_AUTO || o.sweep > PI_SWEEP_SUBBOX) return PI_EINVAL;
    if (o.order != PI_ORDER_SORTED && o.order != PI_ORDER_ORIGINAL) return PI_EINVAL;
    const bool anyf = rho || gx || gy || gz;
    const bool allf = rho && gx && gy && gz;
    if (anyf && !allf) return PI_EINVAL;
    const int64_t n = cells->n;
    if (n > 0 && !anyf && !count && !inv) return PI_EINVAL;
    hipStream_t stream = (hipStream_t)stream_;
    PI_CHECK_HIP(hipSetDevice(ctx->device));

    const double ppc = cells->n_cells > 0 ? (double)n / (double)cells->n_cells : 0.0;
    const int tile = pick_tile(o, ppc);
    if (tile < 0) return PI_EINVAL;

    SweepArgs a;
    a.off = cells->offsets;
    a.cell = cells->cell;
    a.perm = cells->perm;
    a.xs = cells->xs;
    a.ys = cells->ys;
    a.zs = cells->zs;
    a.ws = cells->ws;
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
    a.partials = (InvPartial *)cells->partials;
    a.k = make_kernel_const(cells->grid.rc, cells->grid.cell_w);

    if (n == 0) {
        if (inv) PI_LAUNCH(ctx, "k_inv_zero", k_inv_zero, dim3(1), dim3(64), 0, stream, inv);
        PI_CHECK_HIP(hipGetLastError());
        return PI_OK;
    }

    // enough partial records for any tiling of this grid
    unsigned nblk = 0;
    const bool want_inv = inv != nullptr;
    if (want_inv) {
        const int64_t need = 2 * (cells->n_cells + (n + kBlock - 1) / kBlock) + 64;
        if (need > cells->cap_partials) {
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
    switch (o.precision) {
    case PI_PREC_PLAIN:
        if (want_inv) launch_sweep<PI_PREC_PLAIN, true>(ctx, tile, a, stream, nblk);
        else launch_sweep<PI_PREC_PLAIN, false>(ctx, tile, a, stream, nblk);
        break;
    case PI_PREC_FP64ACC:
        if (want_inv) launch_sweep<PI_PREC_FP64ACC, true>(ctx, tile, a, stream, nblk);
        else launch_sweep<PI_PREC_FP64ACC, false>(ctx, tile, a, stream, nblk);
        break;
    default:
        if (want_inv) launch_sweep<PI_PREC_COMPENSATED, true>(ctx, tile, a, stream, nblk);
        else launch_sweep<PI_PREC_COMPENSATED, false>(ctx, tile, a, stream, nblk);
        break;
    }
    if (want_inv) {
        // stage-1 records go after the sweep's records in the same buffer
        const int32_t n1 = (int32_t)((nblk + kInvRun - 1) / kInvRun);
        InvPartial *stage = a.partials + nblk;
        PI_LAUNCH(ctx, "k_inv_stage1", k_inv_stage1, dim3(n1), dim3(kBlock), 0, stream,
                  (const InvPartial *)a.partials, (int32_t)nblk, stage);
        PI_LAUNCH(ctx, "k_inv_stage2", k_inv_stage2, dim3(1), dim3(kBlock), 0, stream, (const InvPartial *)stage,
                  n1, inv);
    }
    PI_CHECK_HIP(hipGetLastError());
    return PI_OK;
}
