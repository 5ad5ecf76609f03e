// FP64 invariant partial sums of a sweep: one 64-byte record per workgroup,
// folded afterwards in a fixed order (pi_reduce_partials).
#pragma once

#include "pi_internal.h"

struct InvPartial {
    long long pairs;
    double net[3];
    double scale;
    double rho_sum;
    double pad[2];
};

// Block reduction of per-lane partials (256-thread workgroups) into one
// record at `dst`: a wavefront butterfly, then the four wavefronts' sums in
// a fixed order, so the record is deterministic.
__device__ __forceinline__ void block_reduce_partial(InvPartial *dst, long long cnt, double nx, double ny,
                                                     double nz, double sc, double rs)
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
        *dst = p;
    }
}

// The invariants of one sweep launch from its nblk workgroup records at
// `partials` (its two-stage fold writes ceil(nblk / 1024) more records after
// them), or zeros when nblk is 0 (sweep.hip).
void pi_reduce_partials(pi_ctx *ctx, void *partials, unsigned nblk, pi_invariants *inv, hipStream_t stream);
