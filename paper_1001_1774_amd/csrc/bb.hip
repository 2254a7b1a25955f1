// IADM with inner steps on its u-subproblem (the acceleration suggested in the
// concluding remarks, Sec. 4: a gradient method with BB step lengths and a
// non-monotone line search on the u-subproblem of (ALP)).
//
// For fixed q = w^{k+1} - lambda^k / beta the subproblem is the quadratic
//   Phi(v) = beta/2 ||q - D v||^2 + mu/2 ||A v - f||^2,
// Hessian H = beta D^T D + mu A^T A.  Each inner step takes the direction
// p = -M^{-1} grad Phi(v), M = beta D^T D + (mu / tau) I, which the usual u-step
// kernels compute (shrink pass with q held fixed after the first step, FFT solve,
// the increment written to a separate array), then
//   * the squared norms of p, D p and A p (k_bb_partials, fixed-order sums),
//   * the step length a (k_bb_step, one lane per image): 1 for the first step (the
//     IADM u-step), else the BB length (p'M p / p'H p of the previous direction),
//     halved until Phi(v + a p) <= max of the last kBBMemory values + sigma a g'p
//     (non-monotone Armijo test), Phi along the line being the exact quadratic
//     Phi(v) + a g'p + a^2/2 p'H p with g'p = -p'M p,
//   * v += a p and r += a A p (k_bb_update; r = A v - f is carried, so an inner step
//     costs the products A^T r and A p).
// After the inner steps, k_bb_norms and k_bb_stop apply the stop rule (eq. (stop))
// to the outer iterates u^{k+1} = v and u^k.
#include "device_stop.h"
#include "tvcs_internal.h"

#include <algorithm>

namespace tvcs {
namespace {

constexpr int kThreads = 256;

__device__ inline double block_sum(double x, double *red) {
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

// block x of image b: sums over pixels [x * pc, (x + 1) * pc) of p^2 and |D p|^2
// (forward differences, periodic) and over rows [x * rc, (x + 1) * rc) of (A p)^2
__global__ __launch_bounds__(kThreads) void k_bb_partials(int n, int m, const float *__restrict__ P,
                                                          const float *__restrict__ AP, int ldap,
                                                          double *__restrict__ parts,
                                                          const ImgState *__restrict__ st) {
    const int b = blockIdx.y;
    if (!st[b].active) return;
    __shared__ double red[kThreads / 64];
    const int N = n * n, nb = gridDim.x;
    const int pc = (N + nb - 1) / nb, rc = (m + nb - 1) / nb;
    const float *p = P + (size_t)b * N;
    double pp = 0.0, dd = 0.0, aa = 0.0;
    const int p0 = blockIdx.x * pc, p1 = min(N, p0 + pc);
    for (int e = p0 + threadIdx.x; e < p1; e += kThreads) {
        const int r = e / n, c = e - r * n;
        const double v = p[e];
        const double dx = (double)p[r * n + (c + 1 == n ? 0 : c + 1)] - v;
        const double dy = (double)p[(r + 1 == n ? 0 : r + 1) * n + c] - v;
        pp += v * v;
        dd += dx * dx + dy * dy;
    }
    const float *ap = AP + (size_t)b * ldap;
    const int r0 = blockIdx.x * rc, r1 = min(m, r0 + rc);
    for (int i = r0 + threadIdx.x; i < r1; i += kThreads) {
        const double v = ap[i];
        aa += v * v;
    }
    pp = block_sum(pp, red);
    dd = block_sum(dd, red);
    aa = block_sum(aa, red);
    if (threadIdx.x == 0) {
        double *o = parts + ((size_t)b * nb + blockIdx.x) * 3;
        o[0] = pp;
        o[1] = dd;
        o[2] = aa;
    }
}

// one 64-lane block per image: the step length of inner step j
__global__ __launch_bounds__(64) void k_bb_step(const double *__restrict__ parts, int nb,
                                                BBState *__restrict__ bs,
                                                const ImgState *__restrict__ st, int j,
                                                double beta, double mu, double mu_tau,
                                                double sigma) {
    const int b = blockIdx.x;
    if (!st[b].active) return;
    const int lane = threadIdx.x;
    double pp = 0.0, dd = 0.0, aa = 0.0;
    for (int x = lane; x < nb; x += 64) {
        const double *o = parts + ((size_t)b * nb + x) * 3;
        pp += o[0];
        dd += o[1];
        aa += o[2];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        pp += __shfl_xor(pp, off, 64);
        dd += __shfl_xor(dd, off, 64);
        aa += __shfl_xor(aa, off, 64);
    }
    if (lane != 0) return;
    BBState s = bs[b];
    if (j == 0) {   // a new u-subproblem: its history starts at Phi(v_0) = 0
        s.nphi = 1;
        s.phis[0] = 0.0;
        s.phi = 0.0;
        s.prev_pMp = s.prev_pHp = 0.0;
    }
    const double pMp = beta * dd + mu_tau * pp, pHp = beta * dd + mu * aa, gp = -pMp;
    double a = (j == 0 || !(s.prev_pHp > 0.0) || !(s.prev_pMp > 0.0)) ? 1.0 : s.prev_pMp / s.prev_pHp;
    double ref = -INFINITY;   // the largest of the last kBBMemory accepted values
    const int cnt = min(s.nphi, kBBMemory);
    for (int i = 1; i <= cnt; ++i) ref = fmax(ref, s.phis[(s.nphi - i) % kBBMemory]);
    for (int it = 0; it < 64 && s.phi + a * gp + 0.5 * a * a * pHp > ref + sigma * a * gp; ++it)
        a *= 0.5;
    s.phi += a * gp + 0.5 * a * a * pHp;
    s.phis[s.nphi % kBBMemory] = s.phi;
    s.nphi += 1;
    s.prev_pMp = pMp;
    s.prev_pHp = pHp;
    s.alpha = a;
    bs[b] = s;
}

// v += a p over B x N and r += a A p over B x m (FP64 arithmetic, FP32 stores)
__global__ void k_bb_update(int B, int N, int m, float *__restrict__ U, const float *__restrict__ P,
                            float *__restrict__ R, const float *__restrict__ AP, int ldr,
                            const BBState *__restrict__ bs, const ImgState *__restrict__ st) {
    const size_t per = (size_t)N + m, total = (size_t)B * per;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int b = (int)(e / per);
        if (!st[b].active) continue;
        const size_t i = e - (size_t)b * per;
        const double a = bs[b].alpha;
        if (i < (size_t)N) {
            float *u = U + (size_t)b * N + i;
            *u = (float)((double)*u + a * (double)P[(size_t)b * N + i]);
        } else {
            const size_t k = i - N;
            float *r = R + (size_t)b * ldr + k;
            *r = (float)((double)*r + a * (double)AP[(size_t)b * ldr + k]);
        }
    }
}

// stop-rule partials of the outer step: ||u - u_k||^2 and ||u_k||^2 per block
__global__ __launch_bounds__(kThreads) void k_bb_norms(int N, const float *__restrict__ U,
                                                       const float *__restrict__ Uk,
                                                       double *__restrict__ parts,
                                                       const ImgState *__restrict__ st) {
    const int b = blockIdx.y;
    if (!st[b].active) return;
    __shared__ double red[kThreads / 64];
    const int nb = gridDim.x, pc = (N + nb - 1) / nb;
    const int p0 = blockIdx.x * pc, p1 = min(N, p0 + pc);
    double du = 0.0, uu = 0.0;
    for (int e = p0 + threadIdx.x; e < p1; e += kThreads) {
        const double o = Uk[(size_t)b * N + e], d = (double)U[(size_t)b * N + e] - o;
        du += d * d;
        uu += o * o;
    }
    du = block_sum(du, red);
    uu = block_sum(uu, red);
    if (threadIdx.x == 0) {
        parts[((size_t)b * nb + blockIdx.x) * 2] = du;
        parts[((size_t)b * nb + blockIdx.x) * 2 + 1] = uu;
    }
}

__global__ __launch_bounds__(64) void k_bb_stop(ImgState *__restrict__ st,
                                                const double *__restrict__ parts, int nb,
                                                int parity) {
    const int b = blockIdx.x;
    if (!st[b].active) return;
    stop_rule(st + b, parts + (size_t)b * nb * 2, nb, nullptr, parity);
}

__global__ void k_copy(const float *__restrict__ src, float *__restrict__ dst, size_t count) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

int grid_of(size_t count) { return (int)std::min<size_t>((count + 255) / 256, 8192); }

}  // namespace

int bb_blocks(int n) { return std::max(1, std::min(64, n * n / 1024)); }

void launch_bb_step(int n, int m, int B, const float *P, const float *AP, int ldap, double *parts,
                    BBState *bs, const ImgState *st, int j, double beta, double mu, double tau,
                    double sigma, hipStream_t s) {
    const int nb = bb_blocks(n);
    hipLaunchKernelGGL(k_bb_partials, dim3(nb, B), dim3(kThreads), 0, s, n, m, P, AP, ldap, parts,
                       st);
    hipLaunchKernelGGL(k_bb_step, dim3(B), dim3(64), 0, s, parts, nb, bs, st, j, beta, mu,
                       mu / tau, sigma);
}

void launch_bb_update(int B, int N, int m, float *U, const float *P, float *R, const float *AP,
                      int ldr, const BBState *bs, const ImgState *st, hipStream_t s) {
    hipLaunchKernelGGL(k_bb_update, dim3(grid_of((size_t)B * ((size_t)N + m))), dim3(256), 0, s, B,
                       N, m, U, P, R, AP, ldr, bs, st);
}

void launch_bb_stop(int n, int B, const float *U, const float *Uk, double *parts, ImgState *st,
                    int parity, hipStream_t s) {
    const int nb = bb_blocks(n);
    hipLaunchKernelGGL(k_bb_norms, dim3(nb, B), dim3(kThreads), 0, s, n * n, U, Uk, parts, st);
    hipLaunchKernelGGL(k_bb_stop, dim3(B), dim3(64), 0, s, st, parts, nb, parity);
}

void launch_copy(const float *src, float *dst, size_t count, hipStream_t s) {
    if (count == 0) return;
    hipLaunchKernelGGL(k_copy, dim3(grid_of(count)), dim3(256), 0, s, src, dst, count);
}

}  // namespace tvcs
