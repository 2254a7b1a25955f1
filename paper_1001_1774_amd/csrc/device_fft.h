// Device helpers of the FFT kernels: complex arithmetic and the in-LDS Stockham
// FFT (shared by fft.hip and the fused shrink + row-FFT pass).
#pragma once

#include <hip/hip_runtime.h>

#include "tvcs_internal.h"

namespace tvcs {
namespace fftdev {

constexpr int kThreads = 256;   // every FFT kernel runs 256-thread workgroups

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

#ifndef TVCS_XCD_ROWS
#define TVCS_XCD_ROWS 1   // XCD-aware row-block order in the row passes
#endif
// Workgroups are dealt to the 8 XCDs round-robin by linear id, so with a row-block
// count gx that is a multiple of 8 the XCD of block x is x % 8 for every image.
// Giving each XCD a contiguous range of row blocks keeps in one L2 the cache lines
// of the column-major arrays that neighbouring row blocks share, and the halo rows
// one block reads from its neighbour.
__device__ inline int xcd_block(int x, int gx) {
    return (!TVCS_XCD_ROWS || (gx & 7)) ? x : (x & 7) * (gx >> 3) + (x >> 3);
}

__device__ inline void load_twiddles(float2 *tl, const float2 *tw) {
    for (int t = threadIdx.x; t < kMaxN; t += kThreads) tl[t] = tw[t];
}

}  // namespace fftdev
}  // namespace tvcs
