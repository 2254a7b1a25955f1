// The partial-DCT measurement operator (Sec. 3.2): A = P C, where C is the
// orthonormal 2-D DCT-II of n x n images and P keeps m of its n^2 coefficients.
// The rows of C are orthonormal, so A A^T = I, lambda_max(A^T A) = 1, and
// A^T r = C^T (P^T r) is the inverse transform of the zero-filled coefficients.
//
// The 2-D transform is separable: X = C_n U C_n^T for the 1-D orthonormal DCT-II
// matrix C_n.  Three passes, each a batch of 1-D transforms in LDS:
//   rows_fwd : Y = U C_n^T (each row of u transformed), written column-major
//              T[b][k_c][r] so that the next pass reads contiguous columns;
//   cols     : X = C_n Y along r; the kept coefficients give r = X[sel] - f;
//              f and r are held in the order this pass visits the kept
//              coefficients (k_c-major), so each workgroup reads and writes one
//              contiguous range of them; with the adjoint fused, the
//              masked residual is transformed back along k_r in the same block
//              (C_n^T along the columns), in place in T;
//   rows_inv : G = T' C_n along each row, written row-major: g = A^T r.
// In the iteration loop only the column pass runs as its own kernel: the row pass
// of u^{k+1} is done by the inverse row FFT that produces those rows, and the
// inverse row pass by the shrink pass that consumes g (both already hold the rows
// in LDS).  The standalone row kernels serve set-up, the objective and timing.
// Each 1-D DCT-II of length n is one complex FFT of length n (Makhoul, "A fast
// cosine transform in one and multiple dimensions", IEEE TASSP 1980): reorder
// v_j = x_{2j}, v_{n-1-j} = x_{2j+1}; V = FFT(v); X_k = w_k Re(e^{-i pi k/(2n)} V_k),
// w_0 = sqrt(1/n), w_k = sqrt(2/n).  Its inverse rebuilds the Hermitian V from
// V_k = e^{i pi k/(2n)} (X_k / w_k - i X_{n-k} / w_{n-k}) (X_n = 0), inverse FFT,
// and undoes the reordering.  Two real lines share one complex transform (the
// second line as the imaginary part), split again with the Hermitian symmetry.
// The FFTs are the LDS Stockham FFTs of the u-step solve.
#include "device_fft.h"
#include "device_stop.h"

#include <algorithm>
#include <cmath>

namespace tvcs {
namespace {

using namespace fftdev;

// tab[k] = (w_k cos(pi k / 2n), -w_k sin(pi k / 2n), t_k cos(pi k / 2n), t_k sin(pi k / 2n))
// with t_k = 1 / (n w_k): the forward weight w_k e^{-i pi k/(2n)} and the inverse
// factor e^{i pi k/(2n)} / (n w_k) (the 1/n of the inverse FFT folded in).
__global__ void k_dct_table(int n, float4 *tab) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double s, c;
    sincospi((double)k / (2.0 * n), &s, &c);
    const double w = k == 0 ? sqrt(1.0 / n) : sqrt(2.0 / n);
    const double t = 1.0 / (n * w);
    tab[k] = make_float4((float)(w * c), (float)(-w * s), (float)(t * c), (float)(t * s));
}

// LDS of every pass: the two tables and two FFT buffers of (lines / 2) * n complex.
// Real staging (lines * n floats) uses whichever FFT buffer is idle at the time.
struct DctLds {
    float2 *tl;    // FFT twiddles (kMaxN)
    float4 *dt;    // DCT table (n)
    float2 *X, *Y; // FFT buffers
};

// entries per thread of a column block that k_dct_cols loads before its flag
constexpr int kDctPF = 4;

__device__ inline DctLds dct_lds(int n, int lines) {
    extern __shared__ float2 lds[];
    DctLds L;
    L.tl = lds;
    L.dt = reinterpret_cast<float4 *>(lds + kMaxN);
    L.X = lds + kMaxN + 2 * n;
    L.Y = L.X + lp_size((lines / 2) * n);
    return L;
}

size_t dct_lds_bytes(int n, int lines) {
    return sizeof(float2) * (kMaxN + 2 * n + 2 * lp_size((lines / 2) * n));
}


// The twiddles and the DCT table (n <= kMaxN entries), fetched into registers and
// stored to LDS later: a loop that stores what it loads waits for every load in turn.
struct DctTables {
    Twiddles tw;
    float4 dt[(kMaxN + kThreads - 1) / kThreads];
};

template <bool P2>
__device__ inline void fetch_tables(DctTables &f, int n, const float2 *tw, const float4 *tab) {
    fetch_twiddles<P2>(f.tw, tw, n);
#pragma unroll
    for (int i = 0; i < (kMaxN + kThreads - 1) / kThreads; ++i)
        f.dt[i] = tab[min((int)threadIdx.x + i * kThreads, n - 1)];   // in bounds, unused past n
}

template <bool P2>
__device__ inline void store_tables(const DctTables &f, const DctLds &L, int n) {
    store_twiddles<P2>(f.tw, L.tl, n);
#pragma unroll
    for (int i = 0; i < (kMaxN + kThreads - 1) / kThreads; ++i) {
        const int k = threadIdx.x + i * kThreads;
        if (k < n) L.dt[k] = f.dt[i];
    }
}

template <bool P2>
__device__ inline void load_tables(const DctLds &L, int n, const float2 *tw, const float4 *tab) {
    DctTables f;
    fetch_tables<P2>(f, n, tw, tab);
    store_tables<P2>(f, L, n);
}

template <bool P2>
__device__ inline float2 *idct_lines(const DctLds &L, int n, int lines, const float *A, float2 *P,
                                     float2 *Q) {
    return idct_lines_lds<P2>(L.tl, L.dt, n, lines, A, P, Q);
}

// rows_fwd: T[b][k][row] = (DCT-II of row `row` of u_b)_k, `lines` rows per block.
template <bool P2>
__global__ __launch_bounds__(kThreads) void k_dct_rows_fwd(int n, int lines,
                                                           const float *__restrict__ U,
                                                           float *__restrict__ T,
                                                           const float2 *__restrict__ tw,
                                                           const float4 *__restrict__ tab,
                                                           const ImgState *__restrict__ st) {
    const int b = blockIdx.y;
    if (st && !st[b].active) return;
    const DctLds L = dct_lds(n, lines);
    load_tables<P2>(L, n, tw, tab);
    const Ring<P2> ring(n);
    const int N = n * n, row0 = xcd_block(blockIdx.x, gridDim.x) * lines;
    const float *src = U + (size_t)b * N + (size_t)row0 * n;
    float *Xf = reinterpret_cast<float *>(L.X);
    for (int e = threadIdx.x; e < lines * n; e += kThreads) {
        const int l = ring.div(e), j = e - ring.mul(l);
        Xf[2 * lp((l >> 1) * n + makhoul_pos(j, n)) + (l & 1)] = src[e];
    }
    __syncthreads();
    const float2 *Z = lds_fft_any<false, P2>(L.X, L.Y, n, lines >> 1, n, L.tl);
    float *dst = T + (size_t)b * N + row0;
    const float rlines = 1.0f / (float)lines;
    for (int e = threadIdx.x; e < lines * n; e += kThreads) {
        const int k = div_by(e, lines, rlines), l = e - k * lines;
        dst[(size_t)k * n + l] = dct_coef<P2>(Z, L.dt, n, l, k);
    }
}

// cols: for the block's columns k_c of T (contiguous, indexed by r):
//   FWD: X = DCT-II along r; for each kept coefficient (k_r, k_c), R[sel] = X - F[sel]
//        (F may be null); without FWD the kept coefficients are read from R instead;
//   ADJ: the zero-filled coefficients are transformed back along k_r into T.
// selT[k_c * n + k_r] is the measurement index of coefficient k_r * n + k_c, or -1.
template <bool FWD, bool ADJ, bool P2>
__global__ __launch_bounds__(kThreads) void k_dct_cols(int n, int lines, float *__restrict__ T,
                                                       const int *__restrict__ selT,
                                                       const float *__restrict__ F, int ldf,
                                                       float *__restrict__ R, int ldr,
                                                       const float2 *__restrict__ tw,
                                                       const float4 *__restrict__ tab,
                                                       const ImgState *st, ImgState *stw,
                                                       const double *parts, int nparts) {
    const int b = blockIdx.y;
    const DctLds L = dct_lds(n, lines);
    const Ring<P2> ring(n);
    const int N = n * n, col0 = blockIdx.x * lines, total = lines * n;
    float *col = T + (size_t)b * N + (size_t)col0 * n;
    const int *sel = selT + (size_t)col0 * n;
    float *Rb = R + (size_t)b * ldr;
    const float *Fb = F ? F + (size_t)b * ldf : nullptr;
    // The tables and each thread's first kDctPF entries of the block's columns and of
    // its coefficient map are loaded first, before the stop rule and the image's flag
    // (every address is in bounds whether or not the image is active; an index past
    // the block reads its last entry, unused): one memory round trip for all of them.
    DctTables tabs;
    fetch_tables<P2>(tabs, n, tw, tab);
    float cv[kDctPF];
    int sv[kDctPF];
#pragma unroll
    for (int i = 0; i < kDctPF; ++i) {
        const int e = min((int)threadIdx.x + i * kThreads, total - 1);
        if (FWD) cv[i] = col[e];
        sv[i] = sel[e];
    }
    // stw: the first workgroup of each image first applies the previous iteration's
    // stop rule to it, as in the A u product of FP32 storage (the image's other
    // workgroups may read the flag before or after; a stopped image's r and
    // transformed residual are not read)
    if (stw && blockIdx.x == 0) {
        if (threadIdx.x < 64 && stw[b].active)
            stop_rule(stw + b, parts + (size_t)b * nparts * 2, nparts, nullptr);
        __syncthreads();
    }
    if (st && !st[b].active) return;
    // the measurements (or residuals) of the kept coefficients among those entries:
    // issued now, used after the FFT
    float mv[kDctPF];
#pragma unroll
    for (int i = 0; i < kDctPF; ++i) {
        const int s = max(sv[i], 0);
        mv[i] = FWD ? (Fb ? Fb[s] : 0.f) : Rb[s];
    }
    store_tables<P2>(tabs, L, n);
    float2 *P = L.X, *Q = L.Y;   // inverse transform: built in P from the staging in Q
    if (FWD) {
        float *Xf = reinterpret_cast<float *>(L.X);
        auto put = [&](int e, float x) {
            const int l = ring.div(e), j = e - ring.mul(l);
            Xf[2 * lp((l >> 1) * n + makhoul_pos(j, n)) + (l & 1)] = x;
        };
#pragma unroll
        for (int i = 0; i < kDctPF; ++i) {
            const int e = threadIdx.x + i * kThreads;
            if (e < total) put(e, cv[i]);
        }
        for (int e = threadIdx.x + kDctPF * kThreads; e < total; e += kThreads) put(e, col[e]);
        __syncthreads();
        const float2 *Z = lds_fft_any<false, P2>(L.X, L.Y, n, lines >> 1, n, L.tl);
        // the residual is staged in the FFT buffer that does not hold Z
        P = const_cast<float2 *>(Z);
        Q = (Z == L.X) ? L.Y : L.X;
        float *A = reinterpret_cast<float *>(Q);
        auto res = [&](int e, int s, float f) {
            const int l = ring.div(e), k = e - ring.mul(l);
            float rv = 0.f;
            if (s >= 0) {
                rv = dct_coef<P2>(Z, L.dt, n, l, k) - f;
                Rb[s] = rv;
            }
            if (ADJ) A[e] = rv;
        };
#pragma unroll
        for (int i = 0; i < kDctPF; ++i) {
            const int e = threadIdx.x + i * kThreads;
            if (e < total) res(e, sv[i], mv[i]);
        }
        for (int e = threadIdx.x + kDctPF * kThreads; e < total; e += kThreads) {
            const int s = sel[e];
            res(e, s, s >= 0 && Fb ? Fb[s] : 0.f);
        }
    } else {
        float *A = reinterpret_cast<float *>(Q);
#pragma unroll
        for (int i = 0; i < kDctPF; ++i) {
            const int e = threadIdx.x + i * kThreads;
            if (e < total) A[e] = sv[i] >= 0 ? mv[i] : 0.f;
        }
        for (int e = threadIdx.x + kDctPF * kThreads; e < total; e += kThreads) {
            const int s = sel[e];
            A[e] = s >= 0 ? Rb[s] : 0.f;
        }
    }
    if (!ADJ) return;
    __syncthreads();
    const float2 *v = idct_lines<P2>(L, n, lines, reinterpret_cast<const float *>(Q), P, Q);
    for (int e = threadIdx.x; e < lines * n; e += kThreads) {
        const int l = ring.div(e), r = e - ring.mul(l);
        const float2 z = v[lp((l >> 1) * n + makhoul_pos(r, n))];
        col[e] = (l & 1) ? z.y : z.x;
    }
}

// rows_inv: G[b][row][c] = (DCT-II^T along k_c of T[b][.][row])_c.
template <bool P2>
__global__ __launch_bounds__(kThreads) void k_dct_rows_inv(int n, int lines,
                                                           const float *__restrict__ T,
                                                           float *__restrict__ G, int ldg,
                                                           const float2 *__restrict__ tw,
                                                           const float4 *__restrict__ tab,
                                                           const ImgState *__restrict__ st) {
    const int b = blockIdx.y;
    if (st && !st[b].active) return;
    const DctLds L = dct_lds(n, lines);
    load_tables<P2>(L, n, tw, tab);
    const Ring<P2> ring(n);
    const int N = n * n, row0 = xcd_block(blockIdx.x, gridDim.x) * lines;
    const float *src = T + (size_t)b * N + row0;
    float *A = reinterpret_cast<float *>(L.Y);
    const float rlines = 1.0f / (float)lines;
    for (int e = threadIdx.x; e < lines * n; e += kThreads) {
        const int k = div_by(e, lines, rlines), l = e - k * lines;
        A[l * n + k] = src[(size_t)k * n + l];
    }
    __syncthreads();
    const float2 *v = idct_lines<P2>(L, n, lines, A, L.X, L.Y);
    float *dst = G + (size_t)b * ldg + (size_t)row0 * n;
    for (int e = threadIdx.x; e < lines * n; e += kThreads) {
        const int l = ring.div(e), c = e - ring.mul(l);
        const float2 z = v[lp((l >> 1) * n + makhoul_pos(c, n))];
        dst[e] = (l & 1) ? z.y : z.x;
    }
}

// dst[b * m + j] = src[b * m + perm[j]]
__global__ void k_permute(int m, const int *__restrict__ perm, const float *__restrict__ src,
                          float *__restrict__ dst) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const size_t o = (size_t)blockIdx.y * m;
    dst[o + j] = src[o + perm[j]];
}

}  // namespace

// Lines (rows or columns) per workgroup: 2048 values per block where the image
// allows it, at least one pair.
#ifndef TVCS_DCT_LINE_VALUES
#define TVCS_DCT_LINE_VALUES 1024   // values per workgroup of the DCT passes
#endif
int dct_lines(int n) {
    return even_divisor_at_most(n, std::max(2, std::min(n, std::min(16, TVCS_DCT_LINE_VALUES / n))));
}

void launch_dct_permute(int m, int B, const int *perm, const float *src, float *dst,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_permute, dim3((m + 255) / 256, B), dim3(256), 0, s, m, perm, src, dst);
}

void launch_dct_table(int n, float4 *tab, hipStream_t s) {
    hipLaunchKernelGGL(k_dct_table, dim3((n + 255) / 256), dim3(256), 0, s, n, tab);
}

void launch_dct_rows_fwd(int n, int B, const float *U, float *T, const float2 *tw,
                         const float4 *tab, const ImgState *st, hipStream_t s) {
    const int lines = dct_lines(n);
    const size_t lds = dct_lds_bytes(n, lines);
    const dim3 grid(n / lines, B);
    if (is_pow2(n))
        hipLaunchKernelGGL(k_dct_rows_fwd<true>, grid, dim3(kThreads), lds, s, n, lines, U, T, tw,
                           tab, st);
    else
        hipLaunchKernelGGL(k_dct_rows_fwd<false>, grid, dim3(kThreads), lds, s, n, lines, U, T, tw,
                           tab, st);
}

void launch_dct_cols_fwd(int n, int B, float *T, const int *selT, const float *F, int ldf,
                         float *R, int ldr, bool adjoint, const float2 *tw, const float4 *tab,
                         const ImgState *st, hipStream_t s, ImgState *stw, const double *parts,
                         int nparts) {
    if (stw && (st != stw || !parts || nparts < 1))
        fail(TVCS_EINVAL, "dct_cols: the folded stop rule needs the image states and partials");
    const int lines = dct_lines(n);
    const size_t lds = dct_lds_bytes(n, lines);
    const dim3 grid(n / lines, B);
#define TVCS_DCT_COLS(P2V)                                                                        \
    if (adjoint)                                                                                  \
        hipLaunchKernelGGL((k_dct_cols<true, true, P2V>), grid, dim3(kThreads), lds, s, n, lines, \
                           T, selT, F, ldf, R, ldr, tw, tab, st, stw, parts, nparts);             \
    else                                                                                          \
        hipLaunchKernelGGL((k_dct_cols<true, false, P2V>), grid, dim3(kThreads), lds, s, n, lines, \
                           T, selT, F, ldf, R, ldr, tw, tab, st, stw, parts, nparts)
    if (is_pow2(n)) {
        TVCS_DCT_COLS(true);
    } else {
        TVCS_DCT_COLS(false);
    }
#undef TVCS_DCT_COLS
}

void launch_dct_forward(int n, int B, const float *U, float *T, const int *selT, const float *F,
                        int ldf, float *R, int ldr, bool adjoint, const float2 *tw,
                        const float4 *tab, const ImgState *st, hipStream_t s) {
    launch_dct_rows_fwd(n, B, U, T, tw, tab, st, s);
    launch_dct_cols_fwd(n, B, T, selT, F, ldf, R, ldr, adjoint, tw, tab, st, s);
}

void launch_dct_adjoint(int n, int B, const float *R, int ldr, float *T, const int *selT,
                        bool from_R, float *G, int ldg, const float2 *tw, const float4 *tab,
                        const ImgState *st, hipStream_t s) {
    const int lines = dct_lines(n);
    const size_t lds = dct_lds_bytes(n, lines);
    const dim3 grid(n / lines, B);
#define TVCS_DCT_ADJ(P2V)                                                                        \
    if (from_R)                                                                                  \
        hipLaunchKernelGGL((k_dct_cols<false, true, P2V>), grid, dim3(kThreads), lds, s, n, lines, \
                           T, selT, nullptr, 0, const_cast<float *>(R), ldr, tw, tab, st, nullptr, \
                           nullptr, 0);                                                          \
    hipLaunchKernelGGL(k_dct_rows_inv<P2V>, grid, dim3(kThreads), lds, s, n, lines, T, G, ldg, tw, \
                       tab, st)
    if (is_pow2(n)) {
        TVCS_DCT_ADJ(true);
    } else {
        TVCS_DCT_ADJ(false);
    }
#undef TVCS_DCT_ADJ
}

}  // namespace tvcs
