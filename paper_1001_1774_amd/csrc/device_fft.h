// Device helpers of the FFT kernels: complex arithmetic and the in-LDS Stockham
// FFTs (shared by fft.hip, dct.hip and the fused shrink + row-FFT pass).
#pragma once

#include <hip/hip_runtime.h>

#include "device_index.h"
#include "tvcs_internal.h"

namespace tvcs {
namespace fftdev {

constexpr int kThreads = 256;   // every FFT kernel runs 256-thread workgroups

#ifndef TVCS_LDS_PAD
#define TVCS_LDS_PAD 0   // pad the FFT buffers in LDS against bank conflicts (measured slower)
#endif
// LDS slot of complex element i of an FFT buffer: one pad slot after every 4
// elements.  The early Stockham stages write with strides of 4 and 16 elements
// (32 and 128 bytes), which put 4 lanes of every 16 on one bank pair; with the pad
// the stride becomes 5 elements and the 16 lanes of a pass hit distinct banks.
__host__ __device__ inline int lp(int i) { return TVCS_LDS_PAD ? i + (i >> 2) : i; }
// slots a buffer of cnt elements occupies (even, so later regions stay 16-byte aligned)
__host__ __device__ inline int lp_size(int cnt) {
    return TVCS_LDS_PAD ? ((cnt + (cnt >> 2) + 2) & ~1) : ((cnt + 1) & ~1);
}

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
            const float2 v0 = src[lp(f * fs + j)], v1 = src[lp(f * fs + j + h)];
            dst[lp(f * fs + 2 * j)] = v0 + v1;
            dst[lp(f * fs + 2 * j + 1)] = v0 - v1;
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
            const int sb = f * fs + j;
            float2 v0 = src[lp(sb)], v1 = src[lp(sb + q)], v2 = src[lp(sb + 2 * q)],
                   v3 = src[lp(sb + 3 * q)];
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
            const int ob = f * fs + ((j >> lNs) << (lNs + 2)) + k;
            dst[lp(ob)] = a + c;
            dst[lp(ob + Ns)] = bb + mid;
            dst[lp(ob + 2 * Ns)] = a - c;
            dst[lp(ob + 3 * Ns)] = bb - mid;
        }
        __syncthreads();
        float2 *x = src;
        src = dst;
        dst = x;
    }
    return src;
}

__device__ inline int log2i(int n) { return __ffs(n) - 1; }

// ---- mixed radix: any n = 2^a 3^b 5^c ---------------------------------------
#ifndef TVCS_FFT_R8
#define TVCS_FFT_R8 0   // radix-8 stages (and powers of two through this code): measured
#endif                  // slower than radix 4 (0.478 vs 0.465 ms per 512^2 x 64 DCT iteration)
// Stages take radix 4 while it divides the remaining length (8 first with
// TVCS_FFT_R8), then 2, 3 and 5.
// Stage (radix R, Ns = product of the earlier radices, q = L / R): for j < q,
// k = j mod Ns, the inputs x[j + r q] (r < R) are multiplied by w^{r k} with
// w = exp(-+2 pi i / (Ns R)), transformed by a length-R DFT, and output q goes to
// ((j / Ns) Ns R + k + q Ns): the Stockham autosort order of the radix-4 code above,
// generalised.  Twiddles come from a table exp(-2 pi i t / TL) with TL = L * tscale
// (the 512-entry table for powers of two, an L-entry table otherwise): w^{r k} is
// entry r k tscale L / (Ns R).  Fewer, wider stages mean fewer LDS round trips and
// barriers.
__device__ inline int next_radix(int rest) {
    return (TVCS_FFT_R8 && (rest & 7) == 0) ? 8
           : (rest & 3) == 0                ? 4
           : (rest & 1) == 0                ? 2
           : rest % 3 == 0                  ? 3
                                            : 5;
}

// -i z (forward) or +i z (inverse)
template <bool INV>
__device__ inline float2 rot(float2 z) {
    return INV ? make_float2(-z.y, z.x) : make_float2(z.y, -z.x);
}
__device__ inline float2 scl(float a, float2 z) { return make_float2(a * z.x, a * z.y); }

template <int R, bool INV>
__device__ inline void dft_small(float2 *v) {
    if (R == 2) {
        const float2 a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    } else if (R == 3) {
        constexpr float s3 = 0.866025403784438647f;   // sin(2 pi / 3)
        const float2 t1 = v[1] + v[2], t2 = v[0] - scl(0.5f, t1);
        const float2 t3 = rot<INV>(scl(s3, v[1] - v[2]));
        v[0] = v[0] + t1;
        v[1] = t2 + t3;
        v[2] = t2 - t3;
    } else if (R == 4) {
        const float2 a = v[0] + v[2], b = v[0] - v[2], c = v[1] + v[3];
        const float2 mid = rot<INV>(v[1] - v[3]);
        v[0] = a + c;
        v[1] = b + mid;
        v[2] = a - c;
        v[3] = b - mid;
    } else if (R == 8) {   // two length-4 DFTs (even, odd inputs) and a radix-2 step
        float2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
        dft_small<4, INV>(e);
        dft_small<4, INV>(o);
        constexpr float r2 = 0.707106781186547524f;   // 1 / sqrt(2)
        // o_q times w8^q, w8 = exp(-+ i pi / 4)
        const float2 t1 = INV ? make_float2(r2 * (o[1].x - o[1].y), r2 * (o[1].x + o[1].y))
                              : make_float2(r2 * (o[1].x + o[1].y), r2 * (o[1].y - o[1].x));
        const float2 t2 = rot<INV>(o[2]);
        const float2 t3 = INV ? make_float2(-r2 * (o[3].x + o[3].y), r2 * (o[3].x - o[3].y))
                              : make_float2(r2 * (o[3].y - o[3].x), -r2 * (o[3].x + o[3].y));
        v[0] = e[0] + o[0];
        v[4] = e[0] - o[0];
        v[1] = e[1] + t1;
        v[5] = e[1] - t1;
        v[2] = e[2] + t2;
        v[6] = e[2] - t2;
        v[3] = e[3] + t3;
        v[7] = e[3] - t3;
    } else {   // R == 5
        constexpr float c1 = 0.309016994374947424f, c2 = -0.809016994374947424f;   // cos(2pi/5), cos(4pi/5)
        constexpr float s1 = 0.951056516295153572f, s2 = 0.587785252292473129f;    // sin(2pi/5), sin(4pi/5)
        const float2 a1 = v[1] + v[4], b1 = v[1] - v[4], a2 = v[2] + v[3], b2 = v[2] - v[3];
        const float2 p1 = v[0] + scl(c1, a1) + scl(c2, a2), p2 = v[0] + scl(c2, a1) + scl(c1, a2);
        const float2 q1 = rot<INV>(scl(s1, b1) + scl(s2, b2));
        const float2 q2 = rot<INV>(scl(s2, b1) - scl(s1, b2));
        v[0] = v[0] + a1 + a2;
        v[1] = p1 + q1;
        v[2] = p2 + q2;
        v[3] = p2 - q2;
        v[4] = p1 - q1;
    }
}

// P2: L and Ns are powers of two, so the index arithmetic is shifts and masks.
template <bool INV, int R, bool P2>
__device__ inline void mixed_stage(const float2 *src, float2 *dst, int L, int Ns, int nf, int fs,
                                   const float2 *tw, int tscale) {
    const int q = L / R, tstep = (L / (Ns * R)) * tscale;
    const int lq = P2 ? __ffs(q) - 1 : 0, lNs = P2 ? __ffs(Ns) - 1 : 0;
    const float rq = P2 ? 0.f : 1.0f / (float)q, rNs = P2 ? 0.f : 1.0f / (float)Ns;
    for (int t = threadIdx.x; t < nf * q; t += kThreads) {
        const int f = P2 ? t >> lq : div_by(t, q, rq), j = t - f * q;
        const int jn = P2 ? j >> lNs : div_by(j, Ns, rNs), k = j - jn * Ns;
        const int sb = f * fs + j;
        float2 v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = src[lp(sb + r * q)];
        const int step = k * tstep;
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = INV ? cmulc(v[r], tw[r * step]) : cmul(v[r], tw[r * step]);
        dft_small<R, INV>(v);
        const int ob = f * fs + jn * Ns * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[lp(ob + r * Ns)] = v[r];
    }
}

// nf transforms of length L (any 2^a 3^b 5^c) at src[f*fs ..]; tw: L-entry table.
// Returns the buffer holding the result.  Ends with a barrier.
template <bool INV, bool P2>
__device__ float2 *lds_fft_mixed(float2 *src, float2 *dst, int L, int nf, int fs,
                                 const float2 *tw, int tscale) {
    for (int Ns = 1; Ns < L;) {
        const int R = next_radix(L / Ns);   // the same for every thread
        if (R == 8) mixed_stage<INV, 8, P2>(src, dst, L, Ns, nf, fs, tw, tscale);
        else if (R == 4) mixed_stage<INV, 4, P2>(src, dst, L, Ns, nf, fs, tw, tscale);
        else if (R == 2) mixed_stage<INV, 2, P2>(src, dst, L, Ns, nf, fs, tw, tscale);
        else if (P2) __builtin_unreachable();
        else if (R == 3) mixed_stage<INV, 3, false>(src, dst, L, Ns, nf, fs, tw, tscale);
        else mixed_stage<INV, 5, false>(src, dst, L, Ns, nf, fs, tw, tscale);
        __syncthreads();
        float2 *x = src;
        src = dst;
        dst = x;
        Ns *= R;
    }
    return src;
}

// Powers of two use the 512-entry table, other lengths an L-entry table.
template <bool INV, bool P2>
__device__ inline float2 *lds_fft_any(float2 *src, float2 *dst, int L, int nf, int fs,
                                      const float2 *tw) {
    if (P2 && !TVCS_FFT_R8) return lds_fft<INV>(src, dst, L, log2i(L), nf, fs, tw);
    return lds_fft_mixed<INV, P2>(src, dst, L, nf, fs, tw, P2 ? kMaxN / L : 1);
}

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

// ---- DCT-II of real lines through one complex FFT (Makhoul): shared by the
// partial-DCT passes and the inverse row FFT that produces the next iteration's
// row transforms -------------------------------------------------------------------
__device__ inline int makhoul_pos(int j, int n) {   // position of x_j in the reordered v
    return (j & 1) ? n - 1 - (j >> 1) : (j >> 1);
}

// Coefficient k of line l after the FFT of the reordered lines (two per complex
// transform: line l is component l & 1 of pair l >> 1); dt[k] = (w_k cos, -w_k sin,
// ...) of pi k / 2n.
template <bool P2>
__device__ inline float dct_coef(const float2 *Z, const float4 *dt, int n, int l, int k) {
    const float2 zk = Z[lp((l >> 1) * n + k)], znk = Z[lp((l >> 1) * n + Ring<P2>(n).neg(k))];
    float2 v;
    if ((l & 1) == 0)   // V of the real part: (Z_k + conj Z_{n-k}) / 2
        v = make_float2(0.5f * (zk.x + znk.x), 0.5f * (zk.y - znk.y));
    else                // V of the imaginary part: (Z_k - conj Z_{n-k}) / (2i)
        v = make_float2(0.5f * (zk.y + znk.y), -0.5f * (zk.x - znk.x));
    const float4 t = dt[k];
    return t.x * v.x - t.y * v.y;   // Re(w_k e^{-i pi k/(2n)} V_k)
}

// Inverse DCT-II (C_n^T) of `lines` lines whose coefficients are in A[l * n + k]:
// the spectra of the reordered sequences, two lines per complex transform, are
// built in P, V_k = e^{i pi k/(2n)} (X_k / w_k - i X_{n-k} / w_{n-k}) (X_n = 0, the
// factors in dt[k].zw with the 1/n of the inverse FFT), then inverse-transformed
// with Q as the second buffer (Q may hold A).  Returns the buffer holding v: x_j of
// line l is component l & 1 of v[(l >> 1) * n + makhoul_pos(j, n)].
template <bool P2>
__device__ inline float2 *idct_lines_lds(const float2 *tl, const float4 *dt, int n, int lines,
                                         const float *A, float2 *P, float2 *Q) {
    const Ring<P2> ring(n);
    const int npair = lines >> 1;
    for (int e = threadIdx.x; e < npair * n; e += kThreads) {
        const int pr = ring.div(e), k = e - ring.mul(pr);
        const float *a = A + (2 * pr) * n, *b = a + n;
        const float ak = a[k], bk = b[k];
        const float ank = k ? a[n - k] : 0.f, bnk = k ? b[n - k] : 0.f;
        const float4 t = dt[k];
        // V_a = t (a_k - i a_{n-k}), V_b likewise; Z = V_a + i V_b
        const float2 va = make_float2(t.z * ak + t.w * ank, t.w * ak - t.z * ank);
        const float2 vb = make_float2(t.z * bk + t.w * bnk, t.w * bk - t.z * bnk);
        P[lp(e)] = make_float2(va.x - vb.y, va.y + vb.x);
    }
    __syncthreads();
    return lds_fft_any<true, P2>(P, Q, n, npair, n, tl);
}

// the twiddle table of a length-n transform: 512 entries for powers of two, n otherwise.
// Fetched into registers first and stored to LDS later, so that a pass can issue its
// other loads in between and wait for all of them once (a loop that stores what it
// loads waits for each load before it issues the next).
struct Twiddles {
    static constexpr int kPer = (kMaxN + kThreads - 1) / kThreads;
    float2 v[kPer];
};

template <bool P2>
__device__ inline void fetch_twiddles(Twiddles &f, const float2 *tw, int n) {
    const int cnt = P2 ? kMaxN : n;
#pragma unroll
    for (int i = 0; i < Twiddles::kPer; ++i) {
        const int t = threadIdx.x + i * kThreads;
        if (t < cnt) f.v[i] = tw[t];
    }
}

template <bool P2>
__device__ inline void store_twiddles(const Twiddles &f, float2 *tl, int n) {
    const int cnt = P2 ? kMaxN : n;
#pragma unroll
    for (int i = 0; i < Twiddles::kPer; ++i) {
        const int t = threadIdx.x + i * kThreads;
        if (t < cnt) tl[t] = f.v[i];
    }
}

template <bool P2>
__device__ inline void load_twiddles(float2 *tl, const float2 *tw, int n) {
    Twiddles f;
    fetch_twiddles<P2>(f, tw, n);
    store_twiddles<P2>(f, tl, n);
}

}  // namespace fftdev
}  // namespace tvcs
