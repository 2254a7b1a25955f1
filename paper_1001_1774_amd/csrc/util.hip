// Small kernels: partial-sum reduction, fills, the per-image stop rule and the
// power iteration that estimates lambda_max(A^T A) for the step tau (Thm. 1).
// Every reduction adds its terms in a fixed order, so results are reproducible.
#include "tvcs_internal.h"

#include <algorithm>

namespace tvcs {
namespace {

__global__ void k_sum_partials(const float *__restrict__ P, int nchunk, long long chunk_stride,
                               int nv, int N, float *__restrict__ out, int ldo) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    if (j >= N) return;
    double acc = 0.0;
    for (int c = 0; c < nchunk; ++c) acc += (double)P[c * chunk_stride + (size_t)v * N + j];
    out[(size_t)v * ldo + j] = (float)acc;
}

__global__ void k_fill(float *x, size_t count, float value) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x)
        x[i] = value;
}

// x[i] = scale * h(i, seed) with h a hash of the index uniform in [-1, 1) (2^-23 steps)
// (+= with add): deterministic data that is neither zero nor structured
__global__ void k_fill_hash(float *x, size_t count, unsigned seed, float scale, int add) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x) {
        unsigned h = (unsigned)i * 0x9E3779B1u ^ (unsigned)(i >> 32) ^ seed;
        h ^= h >> 16;
        h *= 0x85EBCA6Bu;
        h ^= h >> 13;
        h *= 0xC2B2AE35u;
        h ^= h >> 16;
        const float v = scale * ((float)(h >> 8) * (1.0f / 8388608.0f) - 1.0f);
        x[i] = add ? x[i] + v : v;
    }
}

__global__ void k_init_state(ImgState *st, int B, double tol, int maxit, int fresh) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    ImgState s;
    s.iters = 0;
    s.active = 1;
    s.status = TVCS_OK;
    s.maxit = maxit;
    s.rel = 0.0;
    s.du2 = 0.0;
    s.u2 = 0.0;
    s.tol = tol;
    s.mode[0] = s.mode[1] = fresh;
    s.fresh = 0;
    s.pad_ = 0;
    st[b] = s;
}

__device__ inline double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

// Power-iteration step: rq = v . w (= ||A v||^2 for unit v), v <- w / ||w||.
// Stops (clears st->active) when |rq - rq_prev| <= rtol * rq.
__global__ __launch_bounds__(1024) void k_power_normalize(float *v, const float *__restrict__ w,
                                                          int N, ImgState *st, double rtol) {
    if (!st->active) return;
    __shared__ double s_dot[16], s_nrm[16];
    double d = 0.0, q = 0.0;
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
        const double wj = w[j];
        d += (double)v[j] * wj;
        q += wj * wj;
    }
    d = wave_sum(d);
    q = wave_sum(q);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        s_dot[wave] = d;
        s_nrm[wave] = q;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double dd = 0.0, qq = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            dd += s_dot[i];
            qq += s_nrm[i];
        }
        s_dot[0] = dd;
        s_nrm[0] = qq;
    }
    __syncthreads();
    const double rq = s_dot[0];
    const double inv = s_nrm[0] > 0.0 ? 1.0 / sqrt(s_nrm[0]) : 0.0;
    for (int j = threadIdx.x; j < N; j += blockDim.x) v[j] = (float)(w[j] * inv);
    if (threadIdx.x == 0) {
        const double prev = st->rel;
        st->iters += 1;
        st->rel = rq;
        if (st->iters > 1 && fabs(rq - prev) <= rtol * rq) st->active = 0;
    }
}

__global__ void k_round_f64_f32(const double *__restrict__ src, float *__restrict__ dst,
                                size_t count) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
         i += (size_t)gridDim.x * blockDim.x)
        dst[i] = (float)src[i];
}

}  // namespace

void launch_round_f64_f32(const double *src, float *dst, size_t count, hipStream_t s) {
    if (count == 0) return;
    const int grid = (int)std::min<size_t>((count + 255) / 256, 65536);
    hipLaunchKernelGGL(k_round_f64_f32, dim3(grid), dim3(256), 0, s, src, dst, count);
}

void launch_sum_partials(const float *P, int nchunk, long long chunk_stride, int nv, int N,
                         float *out, int ldo, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_partials, dim3((N + 255) / 256, nv), dim3(256), 0, s, P, nchunk,
                       chunk_stride, nv, N, out, ldo);
}

void launch_fill(float *x, size_t count, float value, hipStream_t s) {
    if (count == 0) return;
    const int grid = (int)std::min<size_t>((count + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill, dim3(grid), dim3(256), 0, s, x, count, value);
}

void launch_fill_hash(float *x, size_t count, unsigned seed, float scale, bool add, hipStream_t s) {
    if (count == 0) return;
    const int grid = (int)std::min<size_t>((count + 255) / 256, 16384);
    hipLaunchKernelGGL(k_fill_hash, dim3(grid), dim3(256), 0, s, x, count, seed, scale, add ? 1 : 0);
}

void launch_init_state(ImgState *st, int B, double tol, int maxit, hipStream_t s, int fresh) {
    hipLaunchKernelGGL(k_init_state, dim3((B + 63) / 64), dim3(64), 0, s, st, B, tol, maxit,
                       fresh);
}

void launch_power_normalize(float *v, const float *w, int N, ImgState *st, double rtol,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_power_normalize, dim3(1), dim3(1024), 0, s, v, w, N, st, rtol);
}

}  // namespace tvcs
