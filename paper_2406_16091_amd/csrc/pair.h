// The pair term of the sweep: exact cutoff predicate, cubic B-spline kernel
// and its gradient, and the three accumulation precisions.
#pragma once

#include "pi_internal.h"

// Constants of one sweep, derived on the host from rc (= h, the support).
struct KernelConst {
    float lo, hi;       // filter on fl(r^2): < lo surely inside, >= hi surely outside
    float reach2;       // rc^2 (1 + 16 u) rounded up: a cell whose nearest face is at
                        // fl(distance^2) >= reach2 surely holds no pair inside the cutoff
    float hh, eh;       // h*h rounded to float, and its residual: h^2 = hh + eh exactly
    float hh_quarter;   // hh / 4 (exact): r^2 <= hh/4  <=>  q <= 1/2
    float h, inv_h;
    float sigma;        // 8 / (pi h^3)
    float two_sigma;    // 2 sigma
    float sig_h2;       // sigma / h^2        (W'(r)/r = sig_h2 (18 q - 12) for q <= 1/2)
    float six_sig_h;    // 6 sigma / h        (W'(r)   = -six_sig_h (1-q)^2 for q > 1/2)
    float w;            // cell width
};

// Error of a + b = s (Knuth's TwoSum, branch-free): a + b == s + err exactly.
__device__ __forceinline__ float two_sum_err(float a, float b, float s)
{
    const float bb = s - a;
    return (a - (s - bb)) + (b - bb);
}

// h^2 - (dx^2 + dy^2 + dz^2) with error-free transforms: the squares are
// split into float + exact FMA residual, their sum into float + TwoSum
// errors, and the large part is subtracted from hh exactly (Sterbenz, since
// the sum is within a factor of two of hh wherever this matters).  The sign
// is exact whenever |h^2 - r^2| exceeds about 6 * 2^-48 h^2, which holds for
// every pair of points on a power-of-two lattice of spacing >= 2^-22 h.
__device__ __forceinline__ float h2_minus_d2(float dx, float dy, float dz, const KernelConst &k)
{
    const float p1 = dx * dx, e1 = __builtin_fmaf(dx, dx, -p1);
    const float p2 = dy * dy, e2 = __builtin_fmaf(dy, dy, -p2);
    const float p3 = dz * dz, e3 = __builtin_fmaf(dz, dz, -p3);
    const float a = p1 + p2;
    const float t1 = two_sum_err(p1, p2, a);
    const float s = a + p3;
    const float t2 = two_sum_err(a, p3, s);
    const float tail = ((t1 + t2) + (e1 + e2)) + e3; // r^2 = s + tail
    const float head = k.hh - s;
    return head + (k.eh - tail);
}

// Filtered exact predicate r < rc from the FP32 value t = fl(r^2) computed as
// fma(dz, dz, fma(dy, dy, dx * dx)) (relative error below 3.0001 * 2^-24).
__device__ __forceinline__ bool inside_cutoff(float dx, float dy, float dz, float t, const KernelConst &k)
{
    if (t < k.lo) return true;
    if (t >= k.hi) return false;
    return h2_minus_d2(dx, dy, dz, k) > 0.0f;
}

__device__ __forceinline__ float sq_dist(float dx, float dy, float dz)
{
    return __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
}

// Kernel value W(r) and W'(r)/r of an accepted pair.  With SELECT both
// pieces of the spline are evaluated and one is chosen, with the same
// values as the branch: where a wavefront evaluates queued pairs together it
// almost always holds pairs on both sides of q = 1/2, so the branch would
// run both anyway (and the merge after it costs register copies).  The
// unchosen piece may be infinite (the outer one at r = 0); it is not used.
template <int PREC, bool SELECT = false>
__device__ __forceinline__ void bspline_terms(float dx, float dy, float dz, float t, const KernelConst &k,
                                              float &W, float &Fr)
{
    const float r = __builtin_amdgcn_sqrtf(t);
    if (SELECT) {
        const float q = r * k.inv_h;
        const float w_in = k.sigma * __builtin_fmaf(q * q, __builtin_fmaf(6.0f, q, -6.0f), 1.0f);
        const float f_in = k.sig_h2 * __builtin_fmaf(18.0f, q, -12.0f);
        float omq;
        if (PREC == PI_PREC_PLAIN) {
            omq = fmaxf(1.0f - r * k.inv_h, 0.0f);
        } else {
            const float D = h2_minus_d2(dx, dy, dz, k);
            omq = D * __builtin_amdgcn_rcpf(k.h * (k.h + r));
        }
        const float omq2 = omq * omq;
        const float w_out = k.two_sigma * omq2 * omq;
        const float f_out = -k.six_sig_h * omq2 * __builtin_amdgcn_rsqf(t);
        const bool inner = t <= k.hh_quarter;
        W = inner ? w_in : w_out;
        Fr = inner ? f_in : f_out;
        return;
    }
    if (t <= k.hh_quarter) {
        const float q = r * k.inv_h;
        W = k.sigma * __builtin_fmaf(q * q, __builtin_fmaf(6.0f, q, -6.0f), 1.0f);
        Fr = k.sig_h2 * __builtin_fmaf(18.0f, q, -12.0f);
    } else {
        float omq;
        if (PREC == PI_PREC_PLAIN) {
            omq = fmaxf(1.0f - r * k.inv_h, 0.0f);
        } else {
            // 1 - q = (h^2 - r^2) / (h (h + r)), with h^2 - r^2 free of cancellation
            const float D = h2_minus_d2(dx, dy, dz, k);
            omq = D * __builtin_amdgcn_rcpf(k.h * (k.h + r));
        }
        const float omq2 = omq * omq;
        W = k.two_sigma * omq2 * omq;
        Fr = -k.six_sig_h * omq2 * __builtin_amdgcn_rsqf(t);
    }
}

// Per-target accumulators for rho, G and (optionally) A = sum w_j |W'(r)|.
template <int PREC>
struct Acc;

template <>
struct Acc<PI_PREC_PLAIN> {
    float rho = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
    __device__ __forceinline__ void add(float a, float bx, float by, float bz)
    {
        rho += a;
        gx += bx;
        gy += by;
        gz += bz;
    }
    __device__ __forceinline__ float r_rho() const { return rho; }
    __device__ __forceinline__ float r_gx() const { return gx; }
    __device__ __forceinline__ float r_gy() const { return gy; }
    __device__ __forceinline__ float r_gz() const { return gz; }
};

// Kahan's compensated summation: c is the rounding excess of the running
// sum so far (what was added minus what was meant), taken off the next
// term; the error of the result is at most about 2u sum |v_i| (u = 2^-24),
// for rho (positive terms) 2u rho and for G at most 2u A, against the 1e-5
// tolerance.  4 operations per term, against 7 for TwoSum with a separate
// error sum.
template <>
struct Acc<PI_PREC_COMPENSATED> {
    float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
    float c0 = 0.f, c1 = 0.f, c2 = 0.f, c3 = 0.f;
    __device__ __forceinline__ static void ks(float &s, float &c, float v)
    {
        const float y = v - c;
        const float n = s + y;
        c = (n - s) - y;
        s = n;
    }
    __device__ __forceinline__ void add(float a, float bx, float by, float bz)
    {
        ks(s0, c0, a);
        ks(s1, c1, bx);
        ks(s2, c2, by);
        ks(s3, c3, bz);
    }
    __device__ __forceinline__ float r_rho() const { return s0 - c0; }
    __device__ __forceinline__ float r_gx() const { return s1 - c1; }
    __device__ __forceinline__ float r_gy() const { return s2 - c2; }
    __device__ __forceinline__ float r_gz() const { return s3 - c3; }
};

template <>
struct Acc<PI_PREC_FP64ACC> {
    double rho = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    __device__ __forceinline__ void add(float a, float bx, float by, float bz)
    {
        rho += (double)a;
        gx += (double)bx;
        gy += (double)by;
        gz += (double)bz;
    }
    __device__ __forceinline__ float r_rho() const { return (float)rho; }
    __device__ __forceinline__ float r_gx() const { return (float)gx; }
    __device__ __forceinline__ float r_gy() const { return (float)gy; }
    __device__ __forceinline__ float r_gz() const { return (float)gz; }
};

// Everything a target keeps while it walks its 27 cells.
template <int PREC, bool INV>
struct Target {
    Acc<PREC> acc;
    int32_t count = 0;
    float ascale = 0.f; // sum w_j |W'(r)| (only with INV)

    // One candidate source at offset (dx, dy, dz) = x_i - x_j, weight wj.
    __device__ __forceinline__ void candidate(float dx, float dy, float dz, float wj, const KernelConst &k)
    {
        const float t = sq_dist(dx, dy, dz);
        if (t < k.hi && inside_cutoff(dx, dy, dz, t, k)) accept(dx, dy, dz, t, wj, k);
    }

    template <bool SELECT = false>
    __device__ __forceinline__ void accept(float dx, float dy, float dz, float t, float wj, const KernelConst &k)
    {
        float W, Fr;
        bspline_terms<PREC, SELECT>(dx, dy, dz, t, k, W, Fr);
        const float f = wj * Fr;
        acc.add(wj * W, f * dx, f * dy, f * dz);
        count += 1;
        if (INV) ascale += wj * fabsf(Fr) * __builtin_amdgcn_sqrtf(t);
    }
};
