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
//   * the squared norms of p, D p and A p (k_bb_partials, fixed-order sums; after a
//     one-pass product, extra workgroups of its band sum),
//   * the step length a: 1 for the first step (the IADM u-step), else the BB length
//     (p'M p / p'H p of the previous direction), halved until Phi(v + a p) <= max of
//     the last kBBMemory values + sigma a g'p (non-monotone Armijo test), Phi along
//     the line being the exact quadratic Phi(v) + a g'p + a^2/2 p'H p, g'p = -p'M p,
//   * v += a p and r += a A p (r = A v - f is carried, so an inner step costs the
//     products A^T r and A p), or, for one image whose A^T (A p) comes from the
//     one-pass product (A read once for both), g += a A^T A p with g = A^T (A v - f)
//     carried instead of r (the last inner step needs only A p, for p'H p).
// One pass (k_bb_apply) does the last two: every workgroup of an image computes the
// step length from the partials itself (the same fixed-order sums, so the same a),
// then updates its share of v and r (or g).  The first inner step also saves u^k,
// and the last one adds the stop-rule partials ||u^{k+1} - u^k||^2 and ||u^k||^2 of
// its pixels; k_bb_stop then applies the stop rule (eq. (stop)) (with the one-pass
// products, the next outer step's first band sum does, but at the end of a graph).
#include "device_bb.h"
#include "device_stop.h"
#include "tvcs_internal.h"

#include <algorithm>

namespace tvcs {
namespace {

constexpr int kThreads = 256;
// pixels and rows per thread whose operands k_bb_apply loads before its step length
constexpr int kApplyPF = 4;

// block x of image b (blockIdx.y): the partial sums of the step length's norms
__global__ __launch_bounds__(kThreads) void k_bb_partials(BBNorms nm,
                                                          const ImgState *__restrict__ st) {
    const int b = blockIdx.y;
    if (!st[b].active) return;
    bb_norms_block(nm, b, blockIdx.x);
}

// The step length of inner step j for image b from the k_bb_partials sums (wave 0;
// lane 0 returns it, with the new state in s).
__device__ inline double bb_length(const double *__restrict__ parts, int nb, BBState &s, int b,
                                   int j, double beta, double mu, double mu_tau, double sigma) {
    const int lane = threadIdx.x & 63;
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
    if (j == 0) {   // a new u-subproblem: its history starts at Phi(v_0) = 0
        s.nphi = 1;
        s.phis[0] = 0.0;
        s.phi = 0.0;
        s.prev_pMp = s.prev_pHp = 0.0;
    }
    const double pMp = beta * dd + mu_tau * pp, pHp = beta * dd + mu * aa, gp = -pMp;
    double a = (j == 0 || !(s.prev_pHp > 0.0) || !(s.prev_pMp > 0.0)) ? 1.0 : s.prev_pMp / s.prev_pHp;
    // the largest of the last kBBMemory accepted values: the circular buffer holds
    // them in slots 0 .. min(nphi, kBBMemory) - 1 (constant indices keep s in registers)
    double ref = -INFINITY;
    const int cnt = min(s.nphi, kBBMemory);
#pragma unroll
    for (int k = 0; k < kBBMemory; ++k)
        if (k < cnt) ref = fmax(ref, s.phis[k]);
    for (int it = 0; it < 64 && s.phi + a * gp + 0.5 * a * a * pHp > ref + sigma * a * gp; ++it)
        a *= 0.5;
    s.phi += a * gp + 0.5 * a * a * pHp;
    const int slot = s.nphi % kBBMemory;
#pragma unroll
    for (int k = 0; k < kBBMemory; ++k)
        if (k == slot) s.phis[k] = s.phi;
    s.nphi += 1;
    s.prev_pMp = pMp;
    s.prev_pHp = pHp;
    s.alpha = a;
    return a;
}

// Inner step j of image b (blockIdx.y), workgroup x of nb: the step length (read
// from bs_in, the new state written by workgroup 0 to bs_out: the workgroups of the
// image all read the old state), then v += a p over pixels [x pc, (x + 1) pc) (and
// g += a h there, G non-null) and r += a A p over rows [x rc, (x + 1) rc) (R non-null),
// FP64 arithmetic, FP32 stores.  j == 0 first
// copies v to Uk (u^k); the last step (last) writes the block's ||v - u^k||^2 and
// ||u^k||^2 to nparts (2 doubles per block, fixed-order sums) for the stop rule.
__global__ __launch_bounds__(kThreads) void k_bb_apply(
    int N, int m, float *__restrict__ U, const float *__restrict__ P, float *__restrict__ R,
    const float *__restrict__ AP, int ldr, float *__restrict__ Uk, const double *__restrict__ parts,
    const BBState *__restrict__ bs_in, BBState *__restrict__ bs_out,
    const ImgState *__restrict__ st, int j, int last, double beta, double mu, double mu_tau,
    double sigma, double *__restrict__ nparts, float *__restrict__ G, const float *__restrict__ H) {
    const int b = blockIdx.y;
    __shared__ double red[kThreads / 64];
    __shared__ double s_a;
    const int nb = gridDim.x;
    const int pc = (N + nb - 1) / nb, rc = (m + nb - 1) / nb;
    const int p0 = blockIdx.x * pc, p1 = min(N, p0 + pc);
    const int r0 = blockIdx.x * rc, r1 = min(m, r0 + rc);
    float *u = U + (size_t)b * N;
    const float *p = P + (size_t)b * N;
    float *uk = Uk + (size_t)b * N;
    float *g = G ? G + (size_t)b * N : nullptr;
    const float *h = G ? H + (size_t)b * N : nullptr;
    float *r = R ? R + (size_t)b * ldr : nullptr;
    const float *ap = R ? AP + (size_t)b * ldr : nullptr;
    // Each thread's first kApplyPF pixels and rows of every operand are loaded before
    // the image's flag is read and before the step length is known (none depends on
    // it, every address is in bounds either way): their memory round trip overlaps
    // the partial sums' instead of following it.
    // (indices past the block's range read a valid element instead, so that no load
    // sits under a branch; those values are never used)
    const bool wuk = last && j != 0;   // u^k is read (the first step writes it)
    float xu[kApplyPF], xp[kApplyPF], xk[kApplyPF], xg[kApplyPF], xh[kApplyPF], xr[kApplyPF],
        xa[kApplyPF];
#pragma unroll
    for (int i = 0; i < kApplyPF; ++i) {
        const int e = min(p0 + (int)threadIdx.x + i * kThreads, N - 1);
        xu[i] = u[e];
        xp[i] = p[e];
    }
    if (wuk)
#pragma unroll
        for (int i = 0; i < kApplyPF; ++i) xk[i] = uk[min(p0 + (int)threadIdx.x + i * kThreads, N - 1)];
    if (G)
#pragma unroll
        for (int i = 0; i < kApplyPF; ++i) {
            const int e = min(p0 + (int)threadIdx.x + i * kThreads, N - 1);
            xg[i] = g[e];
            xh[i] = h[e];
        }
    if (R)
#pragma unroll
        for (int i = 0; i < kApplyPF; ++i) {
            const int q = min(r0 + (int)threadIdx.x + i * kThreads, m - 1);
            xr[i] = r[q];
            xa[i] = ap[q];
        }
    if (!st[b].active) return;
    if (threadIdx.x < 64) {
        BBState s = bs_in[b];
        const double a = bb_length(parts, nb, s, b, j, beta, mu, mu_tau, sigma);
        if (threadIdx.x == 0) {
            s_a = a;
            if (blockIdx.x == 0) bs_out[b] = s;
        }
    }
    __syncthreads();
    const double a = s_a;
    double du = 0.0, uu = 0.0;
    auto upd_u = [&](int e, float old, float pe, float ke) {
        if (j == 0) uk[e] = old;
        const float nv = (float)((double)old + a * (double)pe);
        u[e] = nv;
        if (last) {
            const double o = j == 0 ? (double)old : (double)ke, d = (double)nv - o;
            du += d * d;
            uu += o * o;
        }
    };
#pragma unroll
    for (int i = 0; i < kApplyPF; ++i) {
        const int e = p0 + threadIdx.x + i * kThreads;
        if (e < p1) upd_u(e, xu[i], xp[i], xk[i]);
    }
    for (int e = p0 + threadIdx.x + kApplyPF * kThreads; e < p1; e += kThreads)
        upd_u(e, u[e], p[e], wuk ? uk[e] : 0.f);
    if (G) {
#pragma unroll
        for (int i = 0; i < kApplyPF; ++i) {
            const int e = p0 + threadIdx.x + i * kThreads;
            if (e < p1) g[e] = (float)((double)xg[i] + a * (double)xh[i]);
        }
        for (int e = p0 + threadIdx.x + kApplyPF * kThreads; e < p1; e += kThreads)
            g[e] = (float)((double)g[e] + a * (double)h[e]);
    }
    if (R) {
#pragma unroll
        for (int i = 0; i < kApplyPF; ++i) {
            const int q = r0 + threadIdx.x + i * kThreads;
            if (q < r1) r[q] = (float)((double)xr[i] + a * (double)xa[i]);
        }
        for (int q = r0 + threadIdx.x + kApplyPF * kThreads; q < r1; q += kThreads)
            r[q] = (float)((double)r[q] + a * (double)ap[q]);
    }
    if (last) {
        du = bb_block_sum(du, red);
        uu = bb_block_sum(uu, red);
        if (threadIdx.x == 0) {
            nparts[((size_t)b * nb + blockIdx.x) * 2] = du;
            nparts[((size_t)b * nb + blockIdx.x) * 2 + 1] = uu;
        }
    }
}

__global__ __launch_bounds__(64) void k_bb_stop(ImgState *__restrict__ st,
                                                const double *__restrict__ parts, int nb,
                                                int parity) {
    const int b = blockIdx.x;
    if (!st[b].active) return;
    stop_rule(st + b, parts + (size_t)b * nb * 2, nb, nullptr, parity);
}

}  // namespace

int bb_blocks(int n) { return std::max(1, std::min(64, n * n / 1024)); }

BBNorms bb_norms(int n, int m, const float *P, const float *AP, int ldap, double *parts) {
    return BBNorms{P, AP, parts, n, m, ldap, bb_blocks(n)};
}

void launch_bb_step(int n, int m, int B, float *U, const float *P, float *R, const float *AP,
                    int ldr, float *Uk, double *parts, BBState *bs, const ImgState *st, int j,
                    bool last, double beta, double mu, double tau, double sigma, hipStream_t s,
                    float *G, const float *H, bool norms_done) {
    if (G && !H) fail(TVCS_EINVAL, "bb_step: the gradient update needs A^T A p");
    const int nb = bb_blocks(n);
    if (!norms_done)
        hipLaunchKernelGGL(k_bb_partials, dim3(nb, B), dim3(kThreads), 0, s,
                           bb_norms(n, m, P, AP, ldr, parts), st);
    // the state ping-pongs between bs[0 .. B) and bs[B .. 2B) by the parity of j
    const BBState *bs_in = bs + (size_t)(j & 1) * B;
    BBState *bs_out = bs + (size_t)((j + 1) & 1) * B;
    hipLaunchKernelGGL(k_bb_apply, dim3(nb, B), dim3(kThreads), 0, s, n * n, m, U, P, R, AP, ldr,
                       Uk, parts, bs_in, bs_out, st, j, last ? 1 : 0, beta, mu, mu / tau, sigma,
                       parts + (size_t)3 * B * nb, G, H);
}

void launch_bb_stop(int n, int B, double *parts, ImgState *st, int parity, hipStream_t s) {
    const int nb = bb_blocks(n);
    hipLaunchKernelGGL(k_bb_stop, dim3(B), dim3(64), 0, s, st, parts + (size_t)3 * B * nb, nb,
                       parity);
}


}  // namespace tvcs
