// The per-pixel step of the fused shrinkage: differences, 2-D shrinkage, D^T and
// the right-hand side of the u-step (increment form), shared by k_shrink_rhs and
// the fused shrink + row-FFT pass.  See shrink.hip for the formulas.
#pragma once

#include <hip/hip_runtime.h>

#include "tvcs_internal.h"

#ifndef TVCS_PARTIAL_LOADS
#define TVCS_PARTIAL_LOADS 16  // A^T r partial sums loaded in flight per pixel (8 or 16)
#endif

namespace tvcs {
namespace shrinkdev {

struct D2 {
    double x, y;
};

__device__ inline D2 shrink2(D2 z, double inv_beta) {
    const double t = sqrt(z.x * z.x + z.y * z.y);
    const double s = t > inv_beta ? (t - inv_beta) / t : 0.0;   // 0 * (0/0) = 0
    return {z.x * s, z.y * s};
}

__device__ inline int log2i(int n) { return __ffs(n) - 1; }

// Right-hand side at pixel p of image b (IADM also writes q^k at p into Qnew).
template <bool IADM>
__device__ inline double rhs_at(const ShrinkArgs &a, int b, int p) {
    const int n = a.n, N = n * n, mask = n - 1, ln = log2i(n);
    const int r = p >> ln, c = p & mask;
    const float *u = a.U + (size_t)b * N;
    auto U = [&](int rr, int cc) -> double { return (double)u[((rr & mask) << ln) | (cc & mask)]; };
    const double u0 = U(r, c), uE = U(r, c + 1), uS = U(r + 1, c), uW = U(r, c - 1),
                 uSW = U(r + 1, c - 1), uN = U(r - 1, c), uNE = U(r - 1, c + 1);
    const D2 d0 = {uE - u0, uS - u0};      // D u at (r, c)
    const D2 dW = {u0 - uW, uSW - uW};     // D u at (r, c-1)
    const D2 dN = {uNE - uN, u0 - uN};     // D u at (r-1, c)
    const double ib = 1.0 / a.beta;
    D2 q0, qW, qN;
    if (IADM) {
        const double *Q1 = a.Qold + (size_t)b * 2 * N, *Q2 = Q1 + N;
        const int pW = (r << ln) | ((c - 1) & mask), pN = (((r - 1) & mask) << ln) | c;
        const D2 o0 = {Q1[p], Q2[p]}, oW = {Q1[pW], Q2[pW]}, oN = {Q1[pN], Q2[pN]};
        auto step = [&](D2 d, D2 o) {
            const D2 s = shrink2({2.0 * d.x - o.x, 2.0 * d.y - o.y}, ib);
            return D2{s.x - d.x + o.x, s.y - d.y + o.y};
        };
        q0 = step(d0, o0);
        qW = step(dW, oW);
        qN = step(dN, oN);
        double *W1 = a.Qnew + (size_t)b * 2 * N;
        W1[p] = q0.x;
        W1[N + p] = q0.y;
    } else {
        q0 = shrink2(d0, ib);
        qW = shrink2(dW, ib);
        qN = shrink2(dN, ib);
    }
    // g_k at this pixel: fixed-order sum of the A^T r partials, TVCS_PARTIAL_LOADS
    // independent loads in flight (the sum is latency-bound, not bandwidth-bound)
    constexpr int PL = TVCS_PARTIAL_LOADS;
    const float *g = a.G + (size_t)(b / a.gnv) * a.g_group_stride + (size_t)(b % a.gnv) * N + p;
    double gs[PL];
#pragma unroll
    for (int j = 0; j < PL; ++j) gs[j] = 0.0;
    int k = 0;
    for (; k + PL <= a.nchunk; k += PL) {
#pragma unroll
        for (int j = 0; j < PL; ++j) gs[j] += (double)g[(size_t)(k + j) * a.g_chunk_stride];
    }
    for (int j = 0; k < a.nchunk; ++k, ++j) gs[j] += (double)g[(size_t)k * a.g_chunk_stride];
#pragma unroll
    for (int w = PL / 2; w > 0; w >>= 1)
#pragma unroll
        for (int j = 0; j < w; ++j) gs[j] += gs[j + w];
    const double gk = gs[0];
    // D^T (q - D u) at (r, c): needs (q - D u) here, at (r, c-1) and at (r-1, c)
    const double dtq = ((qW.x - dW.x) - (q0.x - d0.x)) + ((qN.y - dN.y) - (q0.y - d0.y));
    return dtq - a.ctau * gk;
}

}  // namespace shrinkdev
}  // namespace tvcs
