// The squared norms behind the BB step length (Sec. 4 reading of the inner steps): a
// workgroup's partial sums of ||p||^2 and ||D p||^2 over its pixels and of ||A p||^2
// over its rows.  Used by k_bb_partials (bb.hip) and, for one image whose A p comes
// from the one-pass product, by extra workgroups of that product's band sum
// (gemv.hip), so that the partials need no launch of their own; both give the same
// partials bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include "tvcs_internal.h"

namespace tvcs {

// fixed-order sum over a 256-thread workgroup (every thread gets the total)
__device__ inline double bb_block_sum(double x, double *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = x;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];   // fixed order
    return t;
}

// three such sums at once (the same order for each, one exchange through LDS)
__device__ inline void bb_block_sum3(double &x0, double &x1, double &x2) {
    __shared__ double red3[3][4];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        x0 += __shfl_xor(x0, off, 64);
        x1 += __shfl_xor(x1, off, 64);
        x2 += __shfl_xor(x2, off, 64);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        red3[0][wave] = x0;
        red3[1][wave] = x1;
        red3[2][wave] = x2;
    }
    __syncthreads();
    x0 = x1 = x2 = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {   // fixed order
        x0 += red3[0][w];
        x1 += red3[1][w];
        x2 += red3[2][w];
    }
}

// block x of nm.nblk for image b: sums over pixels [x pc, (x + 1) pc) of p^2 and
// |D p|^2 (forward differences, periodic) and over rows [x rc, (x + 1) rc) of
// (A p)^2, written to nm.parts[(b nblk + x) 3 ..] (every thread of a 256-thread
// workgroup must call it)
__device__ inline void bb_norms_block(const BBNorms &nm, int b, int x) {
    const int n = nm.n, N = n * n, nb = nm.nblk, m = nm.m;
    const int pc = (N + nb - 1) / nb, rc = (m + nb - 1) / nb;
    const float *p = nm.P + (size_t)b * N;
    double pp = 0.0, dd = 0.0, aa = 0.0;
    const int p0 = x * pc, p1 = min(N, p0 + pc);
    const int T = blockDim.x;
    // kNormBatch pixels per thread at a time: their loads are issued together (an
    // index past the range reads a valid pixel whose values are not used), then
    // added in the order e = p0 + t, p0 + t + T, ...
    constexpr int kNormBatch = 4;
    for (int e0 = p0 + threadIdx.x; e0 < p1; e0 += kNormBatch * T) {
        float v[kNormBatch], vx[kNormBatch], vy[kNormBatch];
#pragma unroll
        for (int i = 0; i < kNormBatch; ++i) {
            const int e = min(e0 + i * T, N - 1);
            const int r = e / n, c = e - r * n;
            v[i] = p[e];
            vx[i] = p[r * n + (c + 1 == n ? 0 : c + 1)];
            vy[i] = p[(r + 1 == n ? 0 : r + 1) * n + c];
        }
#pragma unroll
        for (int i = 0; i < kNormBatch; ++i) {   // selects, not branches: no load sinks
            const bool ok = e0 + i * T < p1;
            const double vv = v[i];
            const double dx = (double)vx[i] - vv;
            const double dy = (double)vy[i] - vv;
            pp = ok ? pp + vv * vv : pp;
            dd = ok ? dd + (dx * dx + dy * dy) : dd;
        }
    }
    const float *ap = nm.AP + (size_t)b * nm.ldap;
    const int r0 = x * rc, r1 = min(m, r0 + rc);
    for (int i = r0 + threadIdx.x; i < r1; i += T) {
        const double v = ap[i];
        aa += v * v;
    }
    bb_block_sum3(pp, dd, aa);
    if (threadIdx.x == 0) {
        double *o = nm.parts + ((size_t)b * nb + x) * 3;
        o[0] = pp;
        o[1] = dd;
        o[2] = aa;
    }
}

}  // namespace tvcs
