// Exact solve of the u-step system (D^T D + c I) u = rhs under periodic boundary
// conditions (eqs. (eqnorm) and (eqnorm11)).  D^T D is block-circulant, so the 2-D
// DFT diagonalises it with eigenvalues 4 sin^2(pi k1/n) + 4 sin^2(pi k2/n)
// (Sec. 2.1): one forward and one inverse 2-D FFT per iteration.
//
// Three passes over a half spectrum S = [k2 = 0 .. n/2][r = 0 .. n-1] (complex FP32,
// column-major so the column pass reads contiguous vectors):
//   rows_fwd : two real rows packed as x + i y, one complex FFT each pair, split
//              into the two half spectra with the Hermitian symmetry;
//   cols     : for each k2, FFT along r, multiply by 1 / (n^2 d(k1, k2)) (FP64
//              table, the 1/n^2 of the inverse transform folded in), inverse FFT;
//   rows_inv : rebuild the two rows' full spectra from the half spectra, one
//              inverse complex FFT per pair; the result is the increment
//              u^{k+1} - u^k (the right-hand side is the increment form of the
//              u-step), added to u^k in place, with the FP64 partial sums of
//              ||u^{k+1} - u^k||^2 and ||u^k||^2 for the stop rule.
// Every 1-D transform is a Stockham autosort FFT in LDS with radix-4 stages (one
// radix-2 stage first when log2 n is odd), the indexing of Govindaraju et al.,
// "High performance discrete Fourier transforms on graphics processors" (SC 2008).
// Twiddles come from a 512-entry table of exp(-2 pi i t / 512) computed in FP64.
#include "tvcs_internal.h"

#include <algorithm>

namespace tvcs {
namespace {

constexpr int kThreads = 256;

__device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline float2 cmulc(float2 a, float2 b) {   // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ inline float2 operator+(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 operator-(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// nf transforms of length L = 2^logL, transform f at src[f*fs .. f*fs + L).
// Returns the buffer (src or dst) that holds the result.  Ends with a barrier.
template <bool INV>
__device__ float2 *lds_fft(float2 *src, float2 *dst, int L, int logL, int nf, int fs,
                           const float2 *tw) {
    const int tid = threadIdx.x;
    int Ns = 1, lNs = 0;
    if (logL & 1) {   // radix-2 stage, Ns = 1 (unit twiddles)
        const int h = L >> 1;
        for (int t = tid; t < nf * h; t += kThreads) {
            const int f = t >> (logL - 1), j = t & (h - 1);
            const float2 v0 = src[f * fs + j], v1 = src[f * fs + j + h];
            dst[f * fs + 2 * j] = v0 + v1;
            dst[f * fs + 2 * j + 1] = v0 - v1;
        }
        __syncthreads();
        float2 *x = src;
        src = dst;
        dst = x;
        Ns = 2;
        lNs = 1;
    }
    const int q = L >> 2;
    for (; Ns < L; Ns <<= 2, lNs += 2) {
        for (int t = tid; t < nf * q; t += kThreads) {
            const int f = t >> (logL - 2), j = t & (q - 1);
            const int k = j & (Ns - 1);
            const float2 *s = src + f * fs;
            float2 v0 = s[j], v1 = s[j + q], v2 = s[j + 2 * q], v3 = s[j + 3 * q];
            // twiddle exp(-+2 pi i k r / (4 Ns)) = table[k r 128 / Ns]
            const int step = (k << 7) >> lNs;
            if (INV) {
                v1 = cmulc(v1, tw[step]);
                v2 = cmulc(v2, tw[2 * step]);
                v3 = cmulc(v3, tw[3 * step]);
            } else {
                v1 = cmul(v1, tw[step]);
                v2 = cmul(v2, tw[2 * step]);
                v3 = cmul(v3, tw[3 * step]);
            }
            const float2 a = v0 + v2, bb = v0 - v2, c = v1 + v3, d = v1 - v3;
            // -i d = (d.y, -d.x); +i d = (-d.y, d.x)
            const float2 mid = INV ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
            float2 *o = dst + f * fs + ((j >> lNs) << (lNs + 2)) + k;
            o[0] = a + c;
            o[Ns] = bb + mid;
            o[2 * Ns] = a - c;
            o[3 * Ns] = bb - mid;
        }
        __syncthreads();
        float2 *x = src;
        src = dst;
        dst = x;
    }
    return src;
}

__device__ inline int log2i(int n) { return __ffs(n) - 1; }

__device__ inline void load_twiddles(float2 *tl, const float2 *tw) {
    for (int t = threadIdx.x; t < kMaxN; t += kThreads) tl[t] = tw[t];
}

__global__ void k_twiddles(float2 *tw) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kMaxN) return;
    double s, c;
    sincospi(-2.0 * t / kMaxN, &s, &c);
    tw[t] = make_float2((float)c, (float)s);
}

// inv_d[k2 * n + k1] = 1 / (n^2 (4 sin^2(pi k1/n) + 4 sin^2(pi k2/n) + c))
__global__ void k_denominators(int n, double c, double *inv_d) {
    const int h = n / 2 + 1;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= h * n) return;
    const int k2 = e / n, k1 = e % n;
    const double s1 = sinpi((double)k1 / n), s2 = sinpi((double)k2 / n);
    const double d = 4.0 * s1 * s1 + 4.0 * s2 * s2 + c;
    inv_d[e] = 1.0 / ((double)n * (double)n * d);
}

__global__ __launch_bounds__(kThreads) void k_rows_fwd(int n, int rpb, const float *__restrict__ RHS,
                                                       float2 *__restrict__ S,
                                                       const float2 *__restrict__ tw,
                                                       const ImgState *__restrict__ st) {
    const int b = blockIdx.y;
    if (!st[b].active) return;
    extern __shared__ float2 lds[];
    const int ln = log2i(n), npair = rpb >> 1, h = n / 2 + 1;
    const int bufsz = npair * n + rpb;
    float2 *tl = lds, *X = lds + kMaxN, *Y = X + bufsz;
    load_twiddles(tl, tw);
    const int row0 = blockIdx.x * rpb;
    const float *src = RHS + (size_t)b * n * n + (size_t)row0 * n;
    for (int e = threadIdx.x; e < npair * n; e += kThreads) {
        const int pr = e >> ln, j = e & (n - 1);
        X[e] = make_float2(src[(2 * pr) * n + j], src[(2 * pr + 1) * n + j]);
    }
    __syncthreads();
    const float2 *Z = lds_fft<false>(X, Y, n, ln, npair, n, tl);
    float2 *dstS = S + (size_t)b * h * n + row0;
    for (int e = threadIdx.x; e < h * rpb; e += kThreads) {
        const int k = e / rpb, rr = e - k * rpb, pr = rr >> 1;
        const float2 zk = Z[pr * n + k], znk = Z[pr * n + ((n - k) & (n - 1))];
        float2 v;
        if ((rr & 1) == 0)   // X_k = (Z_k + conj Z_{n-k}) / 2
            v = make_float2(0.5f * (zk.x + znk.x), 0.5f * (zk.y - znk.y));
        else                 // Y_k = (Z_k - conj Z_{n-k}) / (2i)
            v = make_float2(0.5f * (zk.y + znk.y), -0.5f * (zk.x - znk.x));
        dstS[(size_t)k * n + rr] = v;
    }
}

__global__ __launch_bounds__(kThreads) void k_cols_solve(int n, int cpb, float2 *__restrict__ S,
                                                         const double *__restrict__ inv_d,
                                                         const float2 *__restrict__ tw,
                                                         const ImgState *__restrict__ st) {
    const int b = blockIdx.y;
    if (!st[b].active) return;
    extern __shared__ float2 lds[];
    const int ln = log2i(n), h = n / 2 + 1;
    const int k20 = blockIdx.x * cpb;
    const int nc = min(cpb, h - k20);
    float2 *tl = lds, *X = lds + kMaxN, *Y = X + cpb * n;
    load_twiddles(tl, tw);
    float2 *col = S + (size_t)b * h * n + (size_t)k20 * n;
    for (int e = threadIdx.x; e < nc * n; e += kThreads) X[e] = col[e];
    __syncthreads();
    float2 *Z = lds_fft<false>(X, Y, n, ln, nc, n, tl);
    const double *id = inv_d + (size_t)k20 * n;
    for (int e = threadIdx.x; e < nc * n; e += kThreads) {
        const float2 z = Z[e];
        const double d = id[e];
        Z[e] = make_float2((float)(z.x * d), (float)(z.y * d));
    }
    __syncthreads();
    float2 *W = (Z == X) ? Y : X;
    const float2 *out = lds_fft<true>(Z, W, n, ln, nc, n, tl);
    for (int e = threadIdx.x; e < nc * n; e += kThreads) col[e] = out[e];
}

__global__ __launch_bounds__(kThreads) void k_rows_inv(int n, int rpb, const float2 *__restrict__ S,
                                                       float *__restrict__ U,
                                                       double *__restrict__ parts,
                                                       const float2 *__restrict__ tw,
                                                       const ImgState *__restrict__ st) {
    const int b = blockIdx.y;
    if (!st[b].active) return;
    extern __shared__ float2 lds[];
    const int ln = log2i(n), npair = rpb >> 1, h = n / 2 + 1;
    const int bufsz = npair * n + rpb;
    float2 *tl = lds, *X = lds + kMaxN, *Y = X + bufsz;
    load_twiddles(tl, tw);
    const int row0 = blockIdx.x * rpb;
    // raw half spectra of the block's rows: Y[rr * h + k]
    const float2 *srcS = S + (size_t)b * h * n + row0;
    for (int e = threadIdx.x; e < h * rpb; e += kThreads) {
        const int k = e / rpb, rr = e - k * rpb;
        Y[rr * h + k] = srcS[(size_t)k * n + rr];
    }
    __syncthreads();
    // full spectrum of x + i y: Z_k = X_k + i Y_k (k <= n/2), conj(X) + i conj(Y) above
    for (int e = threadIdx.x; e < npair * n; e += kThreads) {
        const int pr = e >> ln, k = e & (n - 1);
        const bool lo = k <= n / 2;
        const int kk = lo ? k : n - k;
        const float2 x = Y[(2 * pr) * h + kk], y = Y[(2 * pr + 1) * h + kk];
        X[e] = lo ? make_float2(x.x - y.y, x.y + y.x) : make_float2(x.x + y.y, y.x - x.y);
    }
    __syncthreads();
    const float2 *z = lds_fft<true>(X, Y, n, ln, npair, n, tl);
    float *dstU = U + (size_t)b * n * n + (size_t)row0 * n;
    double du2 = 0.0, u2 = 0.0;
    for (int e = threadIdx.x; e < npair * n; e += kThreads) {
        const int pr = e >> ln, j = e & (n - 1);
        const float2 v = z[e];
        float *p0 = dstU + (2 * pr) * n + j, *p1 = p0 + n;
        const double o0 = *p0, o1 = *p1;
        const float n0 = (float)(o0 + (double)v.x), n1 = (float)(o1 + (double)v.y);
        const double d0 = (double)n0 - o0, d1 = (double)n1 - o1;   // the stored change
        du2 += d0 * d0 + d1 * d1;
        u2 += o0 * o0 + o1 * o1;
        *p0 = n0;
        *p1 = n1;
    }
    // block reduction in a fixed order
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        du2 += __shfl_xor(du2, off, 64);
        u2 += __shfl_xor(u2, off, 64);
    }
    __shared__ double red[2][kThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wave] = du2;
        red[1][wave] = u2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, c = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) {
            a += red[0][w];
            c += red[1][w];
        }
        double *pp = parts + ((size_t)b * gridDim.x + blockIdx.x) * 2;
        pp[0] = a;
        pp[1] = c;
    }
}

// Rows (columns) per workgroup: enough workgroups for one image to spread over
// the chip, and at most 64 KiB of LDS per workgroup (rpb * n <= 4096 complex,
// cpb * n <= 2048 complex per buffer).  The row blocking fixes the order in which
// the stop-rule norms are summed, so it depends on n only: an image's iterates and
// stop decisions are then the same whatever batch it is solved in.
int rows_per_block(int n, int /*B*/) {
    return std::max(2, std::min(n / 32, 4096 / n));
}
int cols_per_block(int n, int B) {
    const int h = n / 2 + 1;
    int cpb = B == 1 ? std::max(1, h / 32) : 8;
    return std::max(1, std::min(std::min(cpb, 2048 / n), h));
}

}  // namespace

void launch_twiddles(float2 *tw, hipStream_t s) {
    hipLaunchKernelGGL(k_twiddles, dim3((kMaxN + 255) / 256), dim3(256), 0, s, tw);
}

void launch_denominators(int n, double c, double *inv_d, hipStream_t s) {
    const int cnt = (n / 2 + 1) * n;
    hipLaunchKernelGGL(k_denominators, dim3((cnt + 255) / 256), dim3(256), 0, s, n, c, inv_d);
}

int fft_row_parts(int n, int B) { return n / rows_per_block(n, B); }

void launch_fft_rows_fwd(int n, int B, const float *RHS, float2 *S, const float2 *tw,
                         const ImgState *st, hipStream_t s) {
    const int rpb = rows_per_block(n, B);
    const size_t lds = sizeof(float2) * (kMaxN + 2 * ((rpb / 2) * n + rpb));
    hipLaunchKernelGGL(k_rows_fwd, dim3(n / rpb, B), dim3(kThreads), lds, s, n, rpb, RHS, S, tw,
                       st);
}

void launch_fft_cols_solve(int n, int B, float2 *S, const double *inv_d, const float2 *tw,
                           const ImgState *st, hipStream_t s) {
    const int cpb = cols_per_block(n, B), h = n / 2 + 1;
    const size_t lds = sizeof(float2) * (kMaxN + 2 * cpb * n);
    hipLaunchKernelGGL(k_cols_solve, dim3((h + cpb - 1) / cpb, B), dim3(kThreads), lds, s, n, cpb,
                       S, inv_d, tw, st);
}

void launch_fft_rows_inv(int n, int B, const float2 *S, float *U, double *parts,
                         const float2 *tw, const ImgState *st, hipStream_t s) {
    const int rpb = rows_per_block(n, B);
    const size_t lds = sizeof(float2) * (kMaxN + 2 * ((rpb / 2) * n + rpb));
    hipLaunchKernelGGL(k_rows_inv, dim3(n / rpb, B), dim3(kThreads), lds, s, n, rpb, S, U, parts,
                       tw, st);
}

}  // namespace tvcs
