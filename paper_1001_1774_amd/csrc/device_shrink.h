// Per-pixel pieces of the fused shrinkage (see shrink.hip for the formulas): the
// 2-D shrinkage, the q update of FTVCS / IADM, the fixed-order sum of the A^T r
// partials, and the loads and arithmetic of the pixel-parallel form of the pass.
// Used by the shrink + row-FFT passes in fft.hip and by shrink.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "device_index.h"
#include "tvcs_internal.h"

#ifndef TVCS_PARTIAL_LOADS
#define TVCS_PARTIAL_LOADS 16  // A^T r partial sums loaded in flight per pixel (8 or 16)
#endif

namespace tvcs {
namespace shrinkdev {

struct D2 {
    double x, y;
};

// s(z) = max(||z|| - 1/beta, 0) z / ||z|| (eq. (shrink)) as z (1 - (1/beta) / ||z||)
// for ||z|| > 1/beta and 0 otherwise: one reciprocal square root instead of a
// square root and a division (0 at z = 0 and at ||z|| = 1/beta; NaN propagates).
__device__ inline D2 shrink2(D2 z, double inv_beta) {
    const double t2 = z.x * z.x + z.y * z.y;
    const double s = t2 > inv_beta * inv_beta ? 1.0 - inv_beta * rsqrt(t2) : 0.0;
    return {z.x * s, z.y * s};
}

// q at one pixel from d = D u there and (IADM) the previous q there:
//   FTVCS: q = s(d);   IADM: q = s(2 d - o) - d + o
template <bool IADM>
__device__ inline D2 q_of(D2 d, D2 o, double inv_beta) {
    if (!IADM) return shrink2(d, inv_beta);
    const D2 s = shrink2({2.0 * d.x - o.x, 2.0 * d.y - o.y}, inv_beta);
    return {s.x - d.x + o.x, s.y - d.y + o.y};
}

// g_k at pixel p of image b: fixed-order sum of the A^T r partials, PL loads in
// flight.  For nchunk <= PL every PL gives the same bits (the pairwise tree over
// the first nchunk slots, the rest exact zeros).  With a running g (MFMA storage,
// a.Gacc): fresh iterations store the sum as the running g, increment iterations
// add it to the running g (FP64 addition, FP32 store); the pass visits every pixel
// once, so each thread updates its own pixel.
template <int PL>
__device__ inline double g_at(const ShrinkArgs &a, int b, int p) {
    const int N = a.n * a.n;
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
    if (a.Gacc) {
        float *acc = a.Gacc + (size_t)b * N + p;
        if (!a.st[b].mode[a.parity]) gs[0] += (double)*acc;
        *acc = (float)gs[0];
    }
    return gs[0];
}

// ---- pixel-parallel form (short row blocks): each thread takes whole pixels and
// recomputes q at the left and upper neighbours it needs for D^T ----------------
// Everything the right-hand side at one pixel reads from memory.  Loading several
// pixels' inputs before computing any of them keeps many loads in flight.
// Loaded values stay in their stored FP32 form until finish_pix widens them: a
// conversion right after a load would wait for it there, before the other loads.
struct PixIn {
    float u0, uE, uS, uW, uSW, uN, uNE;   // u at (r,c), (r,c+1), (r+1,c), (r,c-1), (r+1,c-1), (r-1,c), (r-1,c+1)
    float2 q0, qW, qN;                    // q^{k-1} at (r,c), (r,c-1), (r-1,c) (IADM)
    double gk;                            // g_k = (A^T (A u - f)) at (r,c), unless single
    float g1;                             // single: g_k is this one stored partial
    bool single;
};

template <bool IADM, int PL, bool P2>
__device__ inline PixIn load_pix(const ShrinkArgs &a, int b, int p, bool with_g) {
    const int n = a.n, N = n * n;
    const Ring<P2> ring(n);
    const int r = ring.div(p), c = p - ring.mul(r);
    const float *u = a.U + (size_t)b * N;
    auto U = [&](int rr, int cc) { return u[ring.mul(ring.wrap(rr)) + ring.wrap(cc)]; };
    PixIn in;
    in.u0 = U(r, c);
    in.uE = U(r, c + 1);
    in.uS = U(r + 1, c);
    in.uW = U(r, c - 1);
    in.uSW = U(r + 1, c - 1);
    in.uN = U(r - 1, c);
    in.uNE = U(r - 1, c + 1);
    if (IADM) {
        const float2 *Q = a.Qold + (size_t)b * N;
        const int pW = ring.mul(r) + ring.wrap(c - 1), pN = ring.mul(ring.wrap(r - 1)) + c;
        in.q0 = Q[p];
        in.qW = Q[pW];
        in.qN = Q[pN];
    }
    // one partial and no running g (one image with FP32 storage): g_k is that value
    in.single = with_g && a.nchunk == 1 && !a.Gacc;
    in.gk = 0.0;
    if (in.single)
        in.g1 = a.G[(size_t)(b / a.gnv) * a.g_group_stride + (size_t)(b % a.gnv) * N + p];
    else if (with_g)
        in.gk = g_at<PL>(a, b, p);
    return in;
}

// Right-hand side at pixel p of image b from its inputs (IADM also writes q^k at p
// into Qnew).
template <bool IADM>
__device__ inline double finish_pix(const ShrinkArgs &a, int b, int p, const PixIn &in) {
    const double u0 = in.u0;
    const D2 d0 = {in.uE - u0, in.uS - u0};                              // D u at (r, c)
    const D2 dW = {u0 - in.uW, (double)in.uSW - in.uW};                  // D u at (r, c-1)
    const D2 dN = {(double)in.uNE - in.uN, u0 - in.uN};                  // D u at (r-1, c)
    const double ib = 1.0 / a.beta;
    const bool fz = IADM && a.frozen;   // q held fixed: the given field itself
    const D2 o0 = {in.q0.x, in.q0.y}, oW = {in.qW.x, in.qW.y}, oN = {in.qN.x, in.qN.y};
    const D2 q0 = fz ? o0 : q_of<IADM>(d0, o0, ib), qW = fz ? oW : q_of<IADM>(dW, oW, ib),
             qN = fz ? oN : q_of<IADM>(dN, oN, ib);
    if (IADM && !fz) {
        const int N = a.n * a.n;
        a.Qnew[(size_t)b * N + p] = make_float2((float)q0.x, (float)q0.y);
    }
    // D^T (q - D u) at (r, c): needs (q - D u) here, at (r, c-1) and at (r-1, c)
    const double dtq = ((qW.x - dW.x) - (q0.x - d0.x)) + ((qN.y - dN.y) - (q0.y - d0.y));
    // 0 + g as g_at forms it (a partial of -0 gives +0 there too)
    const double gk = in.single ? 0.0 + (double)in.g1 : in.gk;
    return dtq - a.ctau * gk;
}

}  // namespace shrinkdev
}  // namespace tvcs
