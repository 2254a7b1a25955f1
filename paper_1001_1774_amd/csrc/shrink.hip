// Fused finite differences + two-dimensional shrinkage + D^T, producing the
// right-hand side of the u-step.
//
// FTVCS (Alg. 1): w = s(D u^k) (eq. (shrink)); the u-step (eq. (eqnorm)) is
// (D^T D + c I) u^{k+1} = D^T w + c (u^k - tau g_k), c = mu / (beta tau),
// g_k = A^T (A u^k - f).  Subtracting (D^T D + c I) u^k from both sides gives the
// same step for the increment,
//     (D^T D + c I) (u^{k+1} - u^k) = D^T (w - D u^k) - c tau g_k,
// which is what this kernel's right-hand side holds: the FP32 FFT solve then only
// carries the small increment, so its rounding (~eps ||rhs||) scales with
// ||u^{k+1} - u^k|| instead of with c ||u^k||, and does not pile up over hundreds
// of iterations.  The inverse row pass adds the increment to u^k.
//
// IADM (Alg. 2) keeps one field q = w^{k+1} - lambda^k / beta instead of the pair
// (w, lambda).  With lambda^{k} = lambda^{k-1} - beta (w^k - D u^k)
// (eq. (udlamb)) this gives lambda^k / beta = D u^k - q^{k-1}, so the w-step
// (eq. (iadmw), shrinkage centre D u^k + lambda^k / beta) and the right-hand side
// of eq. (eqnorm11) become
//     q^k = s(2 D u^k - q^{k-1}) - D u^k + q^{k-1},   rhs = D^T (q^k - D u^k) - c tau g_k
// (increment form as above),
// and lambda^K = beta (D u^K - q^{K-1}) is recovered at the end.  q^{-1} is set to
// D u^0 - lambda^0 / beta.  q is stored as an FP32 pair per pixel (all arithmetic on
// it is FP64): this reads 8 bytes and writes 8 per pixel instead of the 48 that
// separate FP64 (w, lambda) fields would move.  Rounding q to FP32 every iteration
// moves the iterates by about 3e-9 (u) and 2e-7 (lambda) relative after 500
// iterations in an FP64 emulation, far below the FP32 path's other roundings.
//
// D is the periodic forward difference: (D u)[r,c] = (u[r,c+1] - u[r,c],
// u[r+1,c] - u[r,c]); (D^T q)[r,c] = q1[r,c-1] - q1[r,c] + q2[r-1,c] - q2[r,c].
// The fused pass (k_shrink_rows in fft.hip) computes each pixel's q once: threads
// walk down columns, keep z = q - D u of the row above in a register and exchange
// the left neighbour's z through LDS.  All per-pixel arithmetic is FP64; rhs is
// rounded to FP32 for the FFT.
#include "device_shrink.h"

namespace tvcs {
namespace {

using namespace shrinkdev;

__global__ void k_init_q(int n, const float *__restrict__ U, const double *__restrict__ lam0,
                         double inv_beta, float2 *__restrict__ Q) {
    const int b = blockIdx.y, N = n * n;
    const Ring<false> ring(n);
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int r = ring.div(p), c = p - ring.mul(r);
    const float *u = U + (size_t)b * N;
    const double u0 = u[p], uE = u[ring.mul(r) + ring.wrap(c + 1)],
                 uS = u[ring.mul(ring.wrap(r + 1)) + c];
    double q1 = uE - u0, q2 = uS - u0;
    if (lam0) {
        q1 -= lam0[(size_t)b * 2 * N + p] * inv_beta;
        q2 -= lam0[(size_t)b * 2 * N + N + p] * inv_beta;
    }
    Q[(size_t)b * N + p] = make_float2((float)q1, (float)q2);
}

__global__ void k_lambda_out(int n, const float *__restrict__ U, const float2 *__restrict__ Q0,
                             const float2 *__restrict__ Q1, const ImgState *__restrict__ st,
                             double beta, double *__restrict__ lam) {
    const int b = blockIdx.y, N = n * n;
    const Ring<false> ring(n);
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const float2 q = ((st[b].iters & 1) ? Q1 : Q0)[(size_t)b * N + p];
    const int r = ring.div(p), c = p - ring.mul(r);
    const float *u = U + (size_t)b * N;
    const double u0 = u[p], uE = u[ring.mul(r) + ring.wrap(c + 1)],
                 uS = u[ring.mul(ring.wrap(r + 1)) + c];
    lam[(size_t)b * 2 * N + p] = beta * ((uE - u0) - (double)q.x);
    lam[(size_t)b * 2 * N + N + p] = beta * ((uS - u0) - (double)q.y);
}

__global__ __launch_bounds__(256) void k_objective(int n, int m, const float *__restrict__ U,
                                                   const float *__restrict__ R, int ldr,
                                                   double mu, double *__restrict__ obj) {
    const int b = blockIdx.x, N = n * n;
    const Ring<false> ring(n);
    const float *u = U + (size_t)b * N;
    double tv = 0.0, rr = 0.0;
    for (int p = threadIdx.x; p < N; p += blockDim.x) {
        const int r = ring.div(p), c = p - ring.mul(r);
        const double u0 = u[p], d1 = u[ring.mul(r) + ring.wrap(c + 1)] - u0,
                     d2 = u[ring.mul(ring.wrap(r + 1)) + c] - u0;
        tv += sqrt(d1 * d1 + d2 * d2);
    }
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        const double x = R[(size_t)b * ldr + i];
        rr += x * x;
    }
    __shared__ double s_tv[256], s_rr[256];
    s_tv[threadIdx.x] = tv;
    s_rr[threadIdx.x] = rr;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_tv[threadIdx.x] += s_tv[threadIdx.x + w];
            s_rr[threadIdx.x] += s_rr[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) obj[b] = s_tv[0] + 0.5 * mu * s_rr[0];
}

}  // namespace

void launch_init_q(int n, int B, const float *U, const double *lam0, double beta, float2 *Q,
                   hipStream_t s) {
    const int N = n * n;
    hipLaunchKernelGGL(k_init_q, dim3((N + 255) / 256, B), dim3(256), 0, s, n, U, lam0,
                       1.0 / beta, Q);
}

void launch_lambda_out(int n, int B, const float *U, const float2 *Q0, const float2 *Q1,
                       const ImgState *st, double beta, double *lam, hipStream_t s) {
    const int N = n * n;
    hipLaunchKernelGGL(k_lambda_out, dim3((N + 255) / 256, B), dim3(256), 0, s, n, U, Q0, Q1, st,
                       beta, lam);
}

void launch_objective(int n, int m, int B, const float *U, const float *R, int ldr, double mu,
                      double *obj, hipStream_t s) {
    hipLaunchKernelGGL(k_objective, dim3(B), dim3(256), 0, s, n, m, U, R, ldr, mu, obj);
}

}  // namespace tvcs
