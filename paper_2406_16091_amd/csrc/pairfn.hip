// The pair kernels of the paper's timing experiments on the binned cell
// lists: the Lennard-Jones potential with softening (Sec. 7.1) and the low-
// and high-FLOP kernels of Fig. 8.  They are evaluated on every candidate
// pair of the 27-cell stencil -- each source j != i whose cell is one of the
// 27 around the target's -- which is what those experiments count as
// interactions (Table 1, first column).
//
//   LJ:       u = sigma^2 / (r^2 + eps^2),  K = 4 e0 (u^6 - u^3)
//   LOWFLOP:  K = (x_i - x_j) + (y_i - y_j) + (z_i - z_j)
//   HIGHFLOP: the LJ value passed through 75 multiply-adds y <- y a + b with
//             run-time a = 1, b = 0 (150 more FLOP, same value)
// v_i = sum_j K(i, j), accumulated in the canonical order of the sweeps
// (cells in (dz, dy, dx) lexicographic order, sources in sorted order), so
// the organisations give bit-identical results on lattice inputs.
//
// Organisations: one thread per target with sources read through the caches
// (Algorithm 1, Par-Part-NoLoop), and LDS tiles -- X-pencils (Sec. 5.2,
// Algorithm 5) and 2 x 2 column sub-boxes (Sec. 5.1) -- whose length along X
// is a launch parameter, so that the staged halo fits the LDS area at any
// occupancy (the paper shortens its pencils the same way as the particles
// per cell grow, Sec. 7.1).  Every candidate is evaluated, so there is no
// accept test to decouple from the evaluation: each lane walks its
// target's nine neighbour rows (three cells each) straight through.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "inv.h"

namespace {

constexpr int kBlock = 256;
constexpr int kPfCap = 3072;  // staged particles per tile (48 KB)
// halo cells along X (tile length + 2) for t x t columns
constexpr int pf_max_hx(int t) { return t == 1 ? 256 : (t == 2 ? 160 : 96); }

struct PfConst {
    float sigma2, eps2; // sigma^2 and eps^2
    float four_e0;      // 4 e0
    float four_abs_e0;  // 4 |e0| (condition scale)
    float a, b;         // the high-FLOP multiply-add constants (1 and 0)
    float w;            // cell width
};

struct PfArgs {
    const int32_t *off;
    const int32_t *cell;
    const int32_t *perm;
    const float4 *p4; // sorted cell-relative (x, y, z, w) records
    int64_t nc;
    int32_t n;
    int32_t nx, ny, nz;
    int32_t orig_order;
    float *v;
    int32_t *count;
    InvPartial *partials;
    PfConst k;
};

// One pair term K and (with INV) its magnitude scale A.
template <int KF, bool INV>
__device__ __forceinline__ float pf_term(float dx, float dy, float dz, const PfConst &p, float &A)
{
    if (KF == PI_PAIRFN_LOWFLOP) {
        if (INV) A = (fabsf(dx) + fabsf(dy)) + fabsf(dz);
        return (dx + dy) + dz;
    }
    const float s2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, __builtin_fmaf(dx, dx, p.eps2)));
    const float u = p.sigma2 * __builtin_amdgcn_rcpf(s2);
    const float u3 = u * u * u;
    float K = p.four_e0 * __builtin_fmaf(u3, u3, -u3);
    if (INV) A = p.four_abs_e0 * __builtin_fmaf(u3, u3, u3);
    if (KF == PI_PAIRFN_HIGHFLOP) {
#pragma unroll
        for (int t = 0; t < 75; ++t) K = __builtin_fmaf(K, p.a, p.b);
    }
    return K;
}

// Scalar accumulators: plain FP32, or Kahan-compensated FP32 (the same
// update as the B-spline sweep's).
template <int PREC>
struct Acc1 {
    float s = 0.f;
    __device__ __forceinline__ void add(float v) { s += v; }
    __device__ __forceinline__ float r() const { return s; }
};

template <>
struct Acc1<PI_PREC_COMPENSATED> {
    float s = 0.f, c = 0.f;
    __device__ __forceinline__ void add(float v)
    {
        const float y = v - c;
        const float n = s + y;
        c = (n - s) - y;
        s = n;
    }
    __device__ __forceinline__ float r() const { return s - c; }
};

template <int KF, int PREC, bool INV>
struct PfTarget {
    Acc1<PREC> acc;
    int32_t count = 0;
    float ascale = 0.f;
    __device__ __forceinline__ void cand(float dx, float dy, float dz, const PfConst &p)
    {
        float A = 0.f;
        acc.add(pf_term<KF, INV>(dx, dy, dz, p, A));
        count += 1;
        if (INV) ascale += A;
    }
};

template <int KF, int PREC, bool INV>
__device__ __forceinline__ void pf_write(const PfArgs &a, int32_t k, const PfTarget<KF, PREC, INV> &T)
{
    const int32_t o = a.orig_order ? a.perm[k] : k;
    a.v[o] = T.acc.r();
    if (a.count) a.count[o] = T.count;
}

// The target's 27 cells from global memory, each neighbour X-row as one
// index range over its (up to) three cells; the two inner cell boundaries
// give each source's shift along X.
template <int KF, int PREC, bool INV>
__device__ __forceinline__ void pf_walk_global(const PfArgs &a, int32_t k, int32_t ix, int32_t iy, int32_t iz,
                                               float xi, float yi, float zi, PfTarget<KF, PREC, INV> &T)
{
    const float W = a.k.w;
    const float xm = xi - (float)(-1) * W, xp = xi - (float)(1) * W;
    for (int dz = -1; dz <= 1; ++dz) {
        const int32_t cz = iz + dz;
        if (cz < 0 || cz >= a.nz) continue;
        const float tz = zi - (float)dz * W;
        for (int dy = -1; dy <= 1; ++dy) {
            const int32_t cy = iy + dy;
            if (cy < 0 || cy >= a.ny) continue;
            const float ty = yi - (float)dy * W;
            const int64_t rb = (int64_t)a.nx * (cy + (int64_t)a.ny * cz) + ix;
            const int32_t b1 = a.off[rb], b2 = a.off[rb + 1];
            const int32_t j0 = ix > 0 ? a.off[rb - 1] : b1;
            const int32_t j3 = ix + 1 < a.nx ? a.off[rb + 2] : b2;
            for (int32_t j = j0; j < j3; ++j) {
                const float tx = j < b1 ? xm : (j < b2 ? xi : xp);
                const float4 s = a.p4[j];
                if (j != k) T.cand(tx - s.x, ty - s.y, tz - s.z, a.k);
            }
        }
    }
}

template <int KF, int PREC, bool INV>
__device__ __forceinline__ void pf_fold(const PfTarget<KF, PREC, INV> &T, long long &cnt, double &sc, double &rs)
{
    cnt += T.count;
    sc += (double)T.ascale;
    rs += (double)T.acc.r();
}

// ------------------------------------------------------------------ no LDS
template <int KF, int PREC, bool INV>
__global__ __launch_bounds__(kBlock) void k_pairfn_nolds(PfArgs a)
{
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int32_t k = (int32_t)(lb * kBlock + threadIdx.x);
    const int32_t kend = min(a.off[a.nc], a.n);
    long long cnt = 0;
    double sc = 0.0, rs = 0.0;
    if (k < kend) {
        const int32_t c = a.cell[k];
        const int32_t ix = c % a.nx, iy = (c / a.nx) % a.ny, iz = c / (a.nx * a.ny);
        const float4 pk = a.p4[k];
        PfTarget<KF, PREC, INV> T;
        pf_walk_global(a, k, ix, iy, iz, pk.x, pk.y, pk.z, T);
        pf_write(a, k, T);
        if (INV) pf_fold(T, cnt, sc, rs);
    }
    if (INV) block_reduce_partial(a.partials + lb, cnt, 0.0, 0.0, 0.0, sc, rs);
}

// ------------------------------------------------------------------ LDS tiles
// A workgroup owns tx_len x TY x TZ target cells; the halo box (clipped to
// the grid) is staged in LDS relative to its corner, one contiguous range
// of the sorted arrays per halo X-row.  A tile whose halo holds more than
// kPfCap particles walks its targets' cells from global memory instead
// (same order, same results on lattice inputs).
template <int TY, int TZ, int KF, int PREC, bool INV>
__global__ __launch_bounds__(kBlock) void k_pairfn_tile(PfArgs a, int32_t tx_len, int32_t ntx, int32_t nty)
{
    constexpr int HY = TY + 2, HZ = TZ + 2;
    constexpr int R = HY * HZ;  // halo rows
    constexpr int TR = TY * TZ; // target rows
    static_assert(R <= 64, "row tables are scanned by one wavefront");
    __shared__ float4 sp[kPfCap];
    __shared__ int32_t cs[R][pf_max_hx(TY) + 1]; // staged index of every halo cell's first particle
    __shared__ int32_t rstart[R + 1];
    __shared__ int32_t gstart[R];
    __shared__ int32_t rbase[R];
    __shared__ int32_t tstart[TR + 1];
    __shared__ int32_t tfirst[TR];

    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int32_t bx = (int32_t)(lb % (uint32_t)ntx);
    const int32_t by = (int32_t)((lb / (uint32_t)ntx) % (uint32_t)nty);
    const int32_t bz = (int32_t)(lb / ((uint32_t)ntx * (uint32_t)nty));
    const int32_t x0 = bx * tx_len, y0 = by * TY, z0 = bz * TZ;
    const int32_t cxlo = max(x0 - 1, 0);
    const int32_t cxhi = min(x0 + tx_len, a.nx - 1);
    const int32_t ncx = cxhi - cxlo + 1; // <= tx_len + 2 <= pf_max_hx(TY)
    const int32_t txhi = min(x0 + tx_len, a.nx);
    const int tid = threadIdx.x;
    const float W = a.k.w;

    // 1. halo row ranges and their staged starts; target row ranges
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
    const int32_t ntarget = tstart[TR];
    long long icnt = 0;
    double isc = 0.0, irs = 0.0;
    // target f of the tile: its row (the last row starting at or before f)
    auto target_row = [&](int32_t f) {
        int tr = 0;
        for (int r = 1; r < TR; ++r) tr = tstart[r] <= f ? r : tr;
        return tr;
    };

    if (total > kPfCap) {
        for (int32_t f = tid; f < ntarget; f += kBlock) {
            const int tr = target_row(f);
            const int32_t k = tfirst[tr] + (f - tstart[tr]);
            const int32_t y = y0 + tr % TY, z = z0 + tr / TY;
            const int32_t ix = a.cell[k] - a.nx * (y + a.ny * z);
            const float4 pk = a.p4[k];
            PfTarget<KF, PREC, INV> T;
            pf_walk_global(a, k, ix, y, z, pk.x, pk.y, pk.z, T);
            pf_write(a, k, T);
            if (INV) pf_fold(T, icnt, isc, irs);
        }
        if (INV) block_reduce_partial(a.partials + lb, icnt, 0.0, 0.0, 0.0, isc, irs);
        return;
    }

    // 2. staged index of every halo cell's first particle (rows outside the
    //    grid stay empty ranges)
    for (int e = tid; e < R * (ncx + 1); e += kBlock) {
        const int r = e / (ncx + 1), jj = e % (ncx + 1);
        const int32_t y = y0 - 1 + r % HY, z = z0 - 1 + r / HY;
        int32_t v = rstart[r];
        if (y >= 0 && y < a.ny && z >= 0 && z < a.nz) v = a.off[(int64_t)rbase[r] + cxlo + jj] - gstart[r] + rstart[r];
        cs[r][jj] = v;
    }
    // 3. stage the halo particles relative to the corner of the halo box
    //    clipped to the grid, so that every staged coordinate lies inside the
    //    grid's extent (exact whenever the positions are)
    const int yoff = y0 > 0 ? 0 : 1, zoff = z0 > 0 ? 0 : 1;
    for (int32_t f = tid; f < total; f += kBlock) {
        int lo = 0, hi = R; // the last row starting at or before f
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (rstart[mid] <= f) lo = mid; else hi = mid;
        }
        const int32_t g = gstart[lo] + (f - rstart[lo]);
        const int32_t cx = a.cell[g] - rbase[lo];
        const float4 q = a.p4[g];
        sp[f] = make_float4(__builtin_fmaf((float)(cx - cxlo), W, q.x),
                            __builtin_fmaf((float)(lo % HY - yoff), W, q.y),
                            __builtin_fmaf((float)(lo / HY - zoff), W, q.z), q.w);
    }
    __syncthreads();

    // 4. targets, one per thread per round
    for (int32_t f = tid; f < ntarget; f += kBlock) {
        const int tr = target_row(f);
        const int32_t k = tfirst[tr] + (f - tstart[tr]);
        const int32_t ty_ = tr % TY, tz_ = tr / TY;
        const int32_t y = y0 + ty_, z = z0 + tz_;
        const int32_t ix = a.cell[k] - a.nx * (y + a.ny * z);
        const int own = (ty_ + 1) + HY * (tz_ + 1);
        const int32_t self = rstart[own] + (k - gstart[own]);
        const float4 t = sp[self];
        const int32_t jc = ix - cxlo;
        const int jl = ix > 0 ? jc - 1 : jc;
        const int jr = ix + 1 < a.nx ? jc + 2 : jc + 1;
        PfTarget<KF, PREC, INV> T;
        for (int dz = -1; dz <= 1; ++dz) {
            for (int dy = -1; dy <= 1; ++dy) {
                const int hr = own + dy + HY * dz; // rows outside the grid are empty
                const int32_t s1 = cs[hr][jr];
                for (int32_t j = cs[hr][jl]; j < s1; ++j) {
                    const float4 s = sp[j];
                    if (j != self) T.cand(t.x - s.x, t.y - s.y, t.z - s.z, a.k);
                }
            }
        }
        pf_write(a, k, T);
        if (INV) pf_fold(T, icnt, isc, irs);
    }
    if (INV) block_reduce_partial(a.partials + lb, icnt, 0.0, 0.0, 0.0, isc, irs);
}

// ------------------------------------------------------------------ host side

// Largest tile length along X (1 .. pf_max_hx(t) - 2) whose staged halo --
// (len + 2) x (t + 2) x (t + 2) cells at mean occupancy ppc, about Poisson --
// keeps its mean plus six standard deviations within kPfCap; 0 if none does.
int pf_fit_length(int t, double ppc)
{
    for (int len = pf_max_hx(t) - 2; len >= 1; --len) {
        const double m = (double)(len + 2) * (t + 2) * (t + 2) * ppc;
        if (m + 6.0 * sqrt(m) <= (double)kPfCap) return len;
    }
    return 0;
}

// An organisation of the pair-kernel sweep: no LDS (t = 0), or tiles of
// len x t x t target cells (t = 1: X-pencil; t = 2, 4: sub-boxes).
struct PfOrg {
    int t;
    int32_t len;
};

// Workgroups of one launch.
int64_t pf_blocks(const PfOrg &g, const PfArgs &a)
{
    if (g.t == 0) {
        const int64_t b = ((int64_t)a.n + kBlock - 1) / kBlock;
        return b > 0 ? b : 1;
    }
    return (int64_t)((a.nx + g.len - 1) / g.len) * ((a.ny + g.t - 1) / g.t) * ((a.nz + g.t - 1) / g.t);
}

// Tile length for t x t columns at occupancy ppc: long enough for about 384
// targets per workgroup (one and a half rounds of 256 lanes), no longer than
// the grid or the staged halo's fit, and shortened while the launch would
// have fewer than two workgroups per compute unit (the paper shortens its
// pencils for the same reason, Sec. 7.1).  An explicit length is kept.
int32_t pf_length(int t, int32_t want, double ppc, const PfArgs &a, int num_cu)
{
    if (want > 0) return std::min<int32_t>(want, pf_max_hx(t) - 2);
    const int fit = pf_fit_length(t, ppc);
    if (fit == 0) return 1; // every tile overflows: each walks from global memory
    int32_t len = (int32_t)ceil(384.0 / ((double)t * t * fmax(ppc, 1e-3)));
    len = std::min<int32_t>(std::min<int32_t>(len, fit), a.nx);
    len = std::max<int32_t>(len, 1);
    const int64_t cols = (int64_t)((a.ny + t - 1) / t) * ((a.nz + t - 1) / t);
    while (len > 1 && cols * ((a.nx + len - 1) / len) < 2 * (int64_t)num_cu) len = (len + 1) / 2;
    return len;
}

template <int KF, int PREC, bool INV>
void pf_launch(pi_ctx *ctx, const PfOrg &g, const PfArgs &a, hipStream_t s, unsigned nblk)
{
    if (g.t == 0) {
        PI_LAUNCH(ctx, "k_pairfn_nolds", (k_pairfn_nolds<KF, PREC, INV>), dim3(nblk), dim3(kBlock), 0, s, a);
        return;
    }
    const int32_t ntx = (a.nx + g.len - 1) / g.len;
    const int32_t nty = (a.ny + g.t - 1) / g.t;
    if (g.t == 1)
        PI_LAUNCH(ctx, "k_pairfn_tile<1,1>", (k_pairfn_tile<1, 1, KF, PREC, INV>), dim3(nblk), dim3(kBlock), 0, s,
                  a, g.len, ntx, nty);
    else if (g.t == 2)
        PI_LAUNCH(ctx, "k_pairfn_tile<2,2>", (k_pairfn_tile<2, 2, KF, PREC, INV>), dim3(nblk), dim3(kBlock), 0, s,
                  a, g.len, ntx, nty);
    else
        PI_LAUNCH(ctx, "k_pairfn_tile<4,4>", (k_pairfn_tile<4, 4, KF, PREC, INV>), dim3(nblk), dim3(kBlock), 0, s,
                  a, g.len, ntx, nty);
}

void pf_dispatch(pi_ctx *ctx, int kernel, int prec, bool inv, const PfOrg &g, const PfArgs &a, hipStream_t s,
                 unsigned nblk)
{
#define PF_PREC(KF)                                                                          \
    do {                                                                                     \
        if (prec == PI_PREC_PLAIN) {                                                         \
            if (inv) pf_launch<KF, PI_PREC_PLAIN, true>(ctx, g, a, s, nblk);                 \
            else pf_launch<KF, PI_PREC_PLAIN, false>(ctx, g, a, s, nblk);                    \
        } else {                                                                             \
            if (inv) pf_launch<KF, PI_PREC_COMPENSATED, true>(ctx, g, a, s, nblk);           \
            else pf_launch<KF, PI_PREC_COMPENSATED, false>(ctx, g, a, s, nblk);              \
        }                                                                                    \
    } while (0)
    switch (kernel) {
    case PI_PAIRFN_LJ: PF_PREC(PI_PAIRFN_LJ); break;
    case PI_PAIRFN_LOWFLOP: PF_PREC(PI_PAIRFN_LOWFLOP); break;
    default: PF_PREC(PI_PAIRFN_HIGHFLOP); break;
    }
#undef PF_PREC
}

// Static rule for AUTO: no LDS from 6 particles per cell up (every candidate
// is evaluated, so the sweep is bound by its arithmetic there, and a staged
// halo holds too few targets per tile), else the widest sub-box whose halo
// fits the LDS area.
int pf_static_t(double ppc)
{
    if (ppc >= 6.0) return 0;
    if (pf_fit_length(4, ppc) > 0) return 4;
    if (pf_fit_length(2, ppc) > 0) return 2;
    return 0;
}

uint64_t pf_tune_key(int kernel, int prec, bool inv, int64_t n, double ppc)
{
    const uint64_t kn = n > 1 ? (uint64_t)floor(2.0 * log2((double)n)) : 0;
    const uint64_t kp = (uint64_t)fmin(1023.0, floor(4.0 * ppc + 0.5));
    return (1ull << 40) | ((uint64_t)kernel << 36) | ((uint64_t)prec << 34) | ((uint64_t)inv << 33) | (kn << 16) | kp;
}

// The profiling step the paper concludes is needed (Sec. 8): every
// organisation run twice on the system itself, the second run timed; the
// static pick is timed first and displaced only by one more than 5% faster.
// Outputs and partial records are overwritten.  Returns t, or -1 on error.
int pf_time_orgs(pi_ctx *ctx, int kernel, int prec, bool inv, int first, const PfArgs &a, int32_t want_len,
                 double ppc, hipStream_t s)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1;
    }
    const int was = ctx->timing_on;
    ctx->timing_on = 0;
    const int order[5] = {first, 0, 1, 2, 4};
    int best = -1;
    float best_ms = 0.f;
    for (int i = 0; i < 5; ++i) {
        const int t = order[i];
        if (i > 0 && t == first) continue;
        if (t > 0 && pf_fit_length(t, ppc) == 0) continue;
        const PfOrg g{t, t > 0 ? pf_length(t, want_len, ppc, a, ctx->num_cu) : 0};
        const unsigned nblk = (unsigned)pf_blocks(g, a);
        float ms = 0.f;
        bool ok = true;
        for (int rep = 0; rep < 2 && ok; ++rep) {
            ok = hipEventRecord(e0, s) == hipSuccess;
            pf_dispatch(ctx, kernel, prec, inv, g, a, s, nblk);
            ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(e1, s) == hipSuccess &&
                 hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        }
        if (ok && (best < 0 || ms < 0.95f * best_ms)) {
            best = t;
            best_ms = ms;
        }
    }
    ctx->timing_on = was;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

} // namespace

extern "C" pi_status pi_interact_pairfn(pi_ctx *ctx, const pi_cells *cells, const pi_pairfn_opts *opts, float *v,
                                        int32_t *count, pi_invariants *inv, pi_stream stream_)
{
    if (!ctx || !cells || !opts || cells->ctx != ctx) return PI_EINVAL;
    if (!pi_cells_ready(cells)) return PI_ESTATE;
    const pi_pairfn_opts &o = *opts;
    if (o.kernel < PI_PAIRFN_LJ || o.kernel > PI_PAIRFN_HIGHFLOP) return PI_EINVAL;
    if (o.precision != PI_PREC_COMPENSATED && o.precision != PI_PREC_PLAIN) return PI_EINVAL;
    if (o.sweep != PI_SWEEP_AUTO && o.sweep != PI_SWEEP_NOLDS && o.sweep != PI_SWEEP_PENCIL &&
        o.sweep != PI_SWEEP_SUBBOX)
        return PI_EINVAL;
    if (o.order != PI_ORDER_SORTED && o.order != PI_ORDER_ORIGINAL) return PI_EINVAL;
    const int64_t n = cells->n;
    if (n > 0 && !v) return PI_EINVAL;
    const float rc = cells->grid.rc;
    const float sigma = o.sigma != 0.0f ? o.sigma : 0.5f * rc;
    const float eps = o.eps != 0.0f ? o.eps : 0.25f * rc;
    const float e0 = o.e0 != 0.0f ? o.e0 : 1.0f;
    if (!(sigma > 0.0f) || !isfinite(sigma) || !(eps >= 0.0f) || !isfinite(eps) || !isfinite(e0)) return PI_EINVAL;

    const double ppc = cells->n_cells > 0 ? (double)n / (double)cells->n_cells : 0.0;
    int t = -1; // -1: chosen by AUTO below
    if (o.sweep == PI_SWEEP_NOLDS) {
        t = 0;
    } else if (o.sweep == PI_SWEEP_PENCIL) {
        if ((o.tile[1] != 0 && o.tile[1] != 1) || (o.tile[2] != 0 && o.tile[2] != 1)) return PI_EINVAL;
        t = 1;
    } else if (o.sweep == PI_SWEEP_SUBBOX) {
        const int ty = o.tile[1] != 0 ? o.tile[1] : o.tile[2];
        if (ty != 0 && ty != 2 && ty != 4) return PI_EINVAL;
        if ((o.tile[1] != 0 && o.tile[1] != ty) || (o.tile[2] != 0 && o.tile[2] != ty)) return PI_EINVAL;
        t = ty != 0 ? ty : (pf_fit_length(4, ppc) > 0 ? 4 : 2);
    }
    if (o.tile[0] < 0 || o.tile[0] > pf_max_hx(t > 0 ? t : 1) - 2) return PI_EINVAL;

    PfArgs a;
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
    a.v = v;
    a.count = count;
    a.partials = (InvPartial *)cells->partials;
    a.k.sigma2 = sigma * sigma;
    a.k.eps2 = eps * eps;
    a.k.four_e0 = 4.0f * e0;
    a.k.four_abs_e0 = 4.0f * fabsf(e0);
    a.k.a = 1.0f;
    a.k.b = 0.0f;
    a.k.w = cells->grid.cell_w;

    PI_CHECK_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream_;
    const bool want_inv = inv != nullptr;
    // every organisation's launch fits the partial records: one per
    // workgroup (at most one per cell or per 256 particles) plus the fold's
    if (n > 0 && t < 0) {
        t = pf_static_t(ppc);
        pi_tuner *tu = ctx->tuner;
        if (tu && tu->mode == PI_TUNE_TIMED) {
            const uint64_t key = pf_tune_key(o.kernel, o.precision, want_inv, n, ppc);
            bool cached = false;
            {
                std::lock_guard<std::mutex> g(tu->mu);
                auto it = tu->choice.find(key);
                if (it != tu->choice.end()) {
                    t = it->second;
                    cached = true;
                }
            }
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            const bool capturing = hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
            if (!cached && !capturing) {
                const int best = pf_time_orgs(ctx, o.kernel, o.precision, want_inv, t, a, o.tile[0], ppc, s);
                if (best < 0) return PI_EDEVICE;
                t = best;
                std::lock_guard<std::mutex> g(tu->mu);
                tu->choice[key] = t;
            }
        }
    }
    if (t < 0) t = 0;
    const PfOrg g{t, t > 0 ? pf_length(t, o.tile[0], ppc, a, ctx->num_cu) : 0};
    const int64_t blocks = n > 0 ? pf_blocks(g, a) : 0;
    if (want_inv && blocks + (blocks + 1023) / 1024 > cells->cap_partials) return PI_ENOMEM;
    const unsigned nblk = (unsigned)blocks;
    if (n > 0) pf_dispatch(ctx, o.kernel, o.precision, want_inv, g, a, s, nblk);
    if (inv) pi_reduce_partials(ctx, cells->partials, nblk, inv, s);
    PI_CHECK_HIP(hipGetLastError());
    return PI_OK;
}
