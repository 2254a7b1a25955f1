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
#include "device_fft.h"
#include "device_shrink.h"
#include "device_stop.h"

#include <algorithm>

namespace tvcs {

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

bool supported_side(int n) {
    if (n < 8 || n > kMaxN || (n & 1)) return false;
    int r = n;
    for (int p : {2, 3, 5})
        while (r % p == 0) r /= p;
    return r == 1;
}

int even_divisor_at_most(int n, int want) {
    for (int d = std::max(2, want & ~1); d > 2; d -= 2)
        if (n % d == 0) return d;
    return 2;
}

namespace {

using namespace fftdev;

// elements per thread whose global operands (denominators, u) the column and inverse
// row passes load before their FFTs (the rest after them)
constexpr int kPrefetch = 2;

// tw[t] = exp(-2 pi i t / L), t < L (L = 512 for every power-of-two n, else L = n)
__global__ void k_twiddles(float2 *tw, int L) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= L) return;
    double s, c;
    sincospi(-2.0 * t / L, &s, &c);
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

// Partial DCT: g of the block's rows (rows row0 .. row0 + rpb - 1 of image b) from
// T, computed in the shrink pass: the rows' coefficients (column-major in T) are
// staged in Y, inverse-transformed (C_n^T along each row) with X and Y as the FFT
// buffers, and left in gl[rr * n + c].  gl first holds the DCT table.  Needs
// max(rpb * n floats, n float4) at gl; ends with a barrier.
template <bool P2>
__device__ inline void shrink_g_from_T(const ShrinkArgs &a, int b, int row0, int rpb,
                                       const float2 *tl, float2 *X, float2 *Y, float *gl) {
    const int n = a.n;
    float4 *dt = reinterpret_cast<float4 *>(gl);
    for (int k = threadIdx.x; k < n; k += kThreads) dt[k] = a.dtab[k];
    float *A = reinterpret_cast<float *>(Y);
    const float *src = a.T + (size_t)b * n * n + row0;
    const float rrpb = 1.0f / (float)rpb;
    for (int e = threadIdx.x; e < rpb * n; e += kThreads) {
        const int k = div_by(e, rpb, rrpb), l = e - k * rpb;
        A[l * n + k] = src[(size_t)k * n + l];
    }
    __syncthreads();
    const float2 *v = idct_lines_lds<P2>(tl, dt, n, rpb, A, X, Y);
    // (the transform ended with a barrier: the table is no longer read)
    const Ring<P2> ring(n);
    for (int e = threadIdx.x; e < rpb * n; e += kThreads) {
        const int l = ring.div(e), c = e - ring.mul(l);
        const float2 z = v[lp((l >> 1) * n + makhoul_pos(c, n))];
        gl[e] = (l & 1) ? z.y : z.x;
    }
    __syncthreads();
}

// FFT of the block's packed row pairs in X, split into the half spectra and
// written to S (rows row0 .. row0 + rpb - 1 of image b).
template <bool P2>
__device__ inline void rows_fwd_tail(int n, int rpb, float2 *X, float2 *Y, const float2 *tl,
                                     float2 *dstS) {
    const Ring<P2> ring(n);
    const int npair = rpb >> 1, h = n / 2 + 1;
    const float2 *Z = lds_fft_any<false, P2>(X, Y, n, npair, n, tl);
    const float rrpb = 1.0f / (float)rpb;
    for (int e = threadIdx.x; e < h * rpb; e += kThreads) {
        const int k = div_by(e, rpb, rrpb), rr = e - k * rpb, pr = rr >> 1;
        const float2 zk = Z[lp(pr * n + k)], znk = Z[lp(pr * n + ring.neg(k))];
        float2 v;
        if ((rr & 1) == 0)   // X_k = (Z_k + conj Z_{n-k}) / 2
            v = make_float2(0.5f * (zk.x + znk.x), 0.5f * (zk.y - znk.y));
        else                 // Y_k = (Z_k - conj Z_{n-k}) / (2i)
            v = make_float2(0.5f * (zk.y + znk.y), -0.5f * (zk.x - znk.x));
        dstS[(size_t)k * n + rr] = v;
    }
}

// Fused shrinkage + forward row FFT for short row blocks (fewer than 4 rows: small
// n, one image spread over the chip): threads take whole pixels, PX per thread and
// round with all their loads issued before any is computed, and each recomputes
// q at its left and upper neighbours (formulas in shrink.hip).
template <bool IADM, int PX, bool P2, int PL>
__global__ __launch_bounds__(kThreads) void k_shrink_pix(ShrinkArgs a, int rpb,
                                                         float2 *__restrict__ S,
                                                         const float2 *__restrict__ tw) {
    const int b = blockIdx.y;
    extern __shared__ float2 lds[];
    const int n = a.n, npair = rpb >> 1, h = n / 2 + 1;
    const Ring<P2> ring(n);
    const int bufsz = npair * n + rpb;
    float2 *tl = lds, *X = lds + kMaxN, *Y = X + lp_size(bufsz);
    float *gl = reinterpret_cast<float *>(Y + lp_size(bufsz));   // partial DCT: g rows
    // the twiddles are fetched before the image's flag is read (both loads in
    // flight together; the table is read whether or not the image is active)
    Twiddles twf;
    fetch_twiddles<P2>(twf, tw, n);
    const int row0 = xcd_block(blockIdx.x, gridDim.x) * rpb;
    const int total = rpb * n;
    // Without the partial DCT's g pass and the running g of MFMA storage (which
    // load_pix updates), loading a pixel has no side effect: the first round of
    // pixels is then loaded before the image's flag is read (an index past the block
    // reads its last pixel, unused, so that no load sits under a branch).
    const bool early = !a.T && !a.Gacc;
    shrinkdev::PixIn pre[PX];
    if (early)
#pragma unroll
        for (int j = 0; j < PX; ++j)
            pre[j] = shrinkdev::load_pix<IADM, PL, P2>(
                a, b, ring.mul(row0) + min((int)threadIdx.x + j * kThreads, total - 1), true);
    if (!a.st[b].active) return;
    if (a.T) {
        store_twiddles<P2>(twf, tl, n);
        shrink_g_from_T<P2>(a, b, row0, rpb, tl, X, Y, gl);
    }
    float *Xf = reinterpret_cast<float *>(X);
    for (int e0 = threadIdx.x; e0 < total; e0 += kThreads * PX) {
        shrinkdev::PixIn in[PX];
        if (early && e0 == (int)threadIdx.x) {
#pragma unroll
            for (int j = 0; j < PX; ++j) in[j] = pre[j];
        } else {
#pragma unroll
            for (int j = 0; j < PX; ++j) {
                const int e = e0 + j * kThreads;
                if (e < total) {
                    in[j] = shrinkdev::load_pix<IADM, PL, P2>(a, b, ring.mul(row0) + e, !a.T);
                    if (a.T) in[j].gk = gl[e];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < PX; ++j) {
            const int e = e0 + j * kThreads;
            if (e >= total) break;
            const int rr = ring.div(e), c = e - ring.mul(rr);
            const float v = (float)shrinkdev::finish_pix<IADM>(a, b, ring.mul(row0) + e, in[j]);
            Xf[2 * lp((rr >> 1) * n + c) + (rr & 1)] = v;   // even row: real part, odd row: imaginary
        }
    }
    if (!a.T) store_twiddles<P2>(twf, tl, n);   // used from the row FFT on
    __syncthreads();
    rows_fwd_tail<P2>(n, rpb, X, Y, tl, S + (size_t)b * h * n + row0);
}

// Fused shrinkage + forward row FFT for row blocks of 4 rows or more (formulas in
// shrink.hip).  Each pixel's q,
// and z = q - D u, is computed once: thread t owns column t (and t + kThreads) of
// its row group and walks the group's rows downwards, starting one row above them.
// D^T z at (r, c) takes z_y of (r-1, c) from the walk's previous step (a register)
// and z_x of (r, c-1) from that step's row of z_x in LDS (double-buffered: one
// barrier per row).  The right-hand side goes straight into the packed FFT input.
// Row groups: `groups` groups of n threads when n < kThreads, else one group.
template <bool IADM, bool P2, int PL>
__global__ __launch_bounds__(kThreads) void k_shrink_walk(ShrinkArgs a, int rpb, int groups,
                                                          float2 *__restrict__ S,
                                                          const float2 *__restrict__ tw) {
    constexpr int kCols = kMaxN / kThreads;   // columns per thread when n >= kThreads
    const int b = blockIdx.y;
    if (!a.st[b].active) return;
    extern __shared__ float2 lds[];
    const int n = a.n, N = n * n, h = n / 2 + 1;
    const Ring<P2> ring(n);
    const int bufsz = (rpb >> 1) * n + rpb;
    float2 *tl = lds, *X = lds + kMaxN, *Y = X + lp_size(bufsz);
    double *zx = reinterpret_cast<double *>(Y);   // 2 x groups x n, before the FFT uses Y
    // partial DCT: g rows after the Y region (the larger of the FFT buffer and zx)
    const int ybytes = max((int)sizeof(float2) * lp_size(bufsz), (int)sizeof(double) * 2 * groups * n);
    float *gl = reinterpret_cast<float *>(reinterpret_cast<char *>(Y) + ybytes);
    load_twiddles<P2>(tl, tw, n);
    const int row0 = xcd_block(blockIdx.x, gridDim.x) * rpb;
    if (a.T) shrink_g_from_T<P2>(a, b, row0, rpb, tl, X, Y, gl);
    const int rg = rpb / groups;   // own rows per group
    const int t = threadIdx.x;
    // threads past groups * n (n < kThreads) own no column and only join barriers
    const int g = groups > 1 ? min(t / n, groups - 1) : 0;
    int c[kCols];
    bool has[kCols];
#pragma unroll
    for (int j = 0; j < kCols; ++j) {
        const int cc = groups > 1 ? t - g * n : t + j * kThreads;
        has[j] = groups > 1 ? (j == 0 && cc < n) : cc < n;
        c[j] = has[j] ? cc : 0;
    }
    const float *u = a.U + (size_t)b * N;
    const float2 *qold = a.Qold + (size_t)b * N;
    float2 *qnew = a.Qnew + (size_t)b * N;
    const double ib = 1.0 / a.beta;
    float *Xf = reinterpret_cast<float *>(X);
    double zy[kCols];
    float ucur[kCols];
    // loads of the next step, issued one step ahead: u east and south, q^{k-1}
    float nE[kCols], nS[kCols];
    float2 nq[kCols];
    int r = ring.wrap(row0 + g * rg - 1);
    auto prefetch = [&](int rr_) {
        const int rs = ring.wrap(rr_ + 1);
#pragma unroll
        for (int j = 0; j < kCols; ++j) {
            if (!has[j]) continue;
            nE[j] = u[ring.mul(rr_) + ring.wrap(c[j] + 1)];
            nS[j] = u[ring.mul(rs) + c[j]];
            if (IADM) nq[j] = qold[ring.mul(rr_) + c[j]];
        }
    };
#pragma unroll
    for (int j = 0; j < kCols; ++j) {
        zy[j] = 0.0;
        ucur[j] = has[j] ? u[ring.mul(r) + c[j]] : 0.f;
        nE[j] = nS[j] = 0.f;
        nq[j] = make_float2(0.f, 0.f);
    }
    prefetch(r);
    for (int s = 0; s <= rg; ++s) {
        const int rn = ring.wrap(r + 1);
        float uE[kCols], uS[kCols];
        float2 qo[kCols];
#pragma unroll
        for (int j = 0; j < kCols; ++j) {
            uE[j] = nE[j];
            uS[j] = nS[j];
            qo[j] = nq[j];
        }
        if (s < rg) prefetch(rn);
        double gk[kCols];
#pragma unroll
        for (int j = 0; j < kCols; ++j)
            gk[j] = (s > 0 && has[j])
                        ? (a.T ? (double)gl[(g * rg + s - 1) * n + c[j]]
                               : shrinkdev::g_at<PL>(a, b, ring.mul(r) + c[j]))
                        : 0.0;
        double zxv[kCols], zyv[kCols];
#pragma unroll
        for (int j = 0; j < kCols; ++j) {
            zxv[j] = zyv[j] = 0.0;
            if (!has[j]) continue;
            const int p = ring.mul(r) + c[j];
            const shrinkdev::D2 d = {(double)uE[j] - ucur[j], (double)uS[j] - ucur[j]};
            const shrinkdev::D2 o = {(double)qo[j].x, (double)qo[j].y};
            const shrinkdev::D2 q = (IADM && a.frozen) ? o : shrinkdev::q_of<IADM>(d, o, ib);
            if (IADM && s > 0 && !a.frozen) qnew[p] = make_float2((float)q.x, (float)q.y);
            zxv[j] = q.x - d.x;
            zyv[j] = q.y - d.y;
            ucur[j] = uS[j];
        }
        if (s > 0) {   // the same for every thread
            double *zrow = zx + ((s & 1) * groups + g) * n;
#pragma unroll
            for (int j = 0; j < kCols; ++j)
                if (has[j]) zrow[c[j]] = zxv[j];
            __syncthreads();
            const int rr = g * rg + s - 1;   // row within the block
#pragma unroll
            for (int j = 0; j < kCols; ++j) {
                if (!has[j]) continue;
                const double zw = zrow[ring.wrap(c[j] - 1)];
                // D^T z at (r, c) - c tau g_k: the right side of the increment
                const double rhs = (zw - zxv[j]) + (zy[j] - zyv[j]) - a.ctau * gk[j];
                Xf[2 * lp((rr >> 1) * n + c[j]) + (rr & 1)] = (float)rhs;
            }
        }
#pragma unroll
        for (int j = 0; j < kCols; ++j) zy[j] = zyv[j];
        r = rn;
    }
    __syncthreads();
    rows_fwd_tail<P2>(n, rpb, X, Y, tl, S + (size_t)b * h * n + row0);
}

template <bool P2>
__global__ __launch_bounds__(kThreads) void k_cols_solve(int n, int cpb, float2 *__restrict__ S,
                                                         const double *__restrict__ inv_d,
                                                         const float2 *__restrict__ tw,
                                                         const ImgState *__restrict__ st) {
    const int b = blockIdx.y;
    extern __shared__ float2 lds[];
    const int h = n / 2 + 1;
    const int k20 = blockIdx.x * cpb;
    const int nc = min(cpb, h - k20);
    float2 *tl = lds, *X = lds + kMaxN, *Y = X + lp_size(cpb * n);
    // The twiddles, each thread's first kPrefetch spectrum entries and denominators
    // are all loaded before anything waits, and before the image's flag is read
    // (every address is in bounds whether or not the image is active): one memory
    // round trip instead of one per loop and one more after the forward FFT.
    Twiddles twf;
    fetch_twiddles<P2>(twf, tw, n);
    float2 *col = S + (size_t)b * h * n + (size_t)k20 * n;
    const double *id = inv_d + (size_t)k20 * n;
    float2 cpre[kPrefetch];
    double dpre[kPrefetch];
#pragma unroll
    for (int i = 0; i < kPrefetch; ++i) {
        const int e = threadIdx.x + i * kThreads;
        cpre[i] = e < nc * n ? col[e] : make_float2(0.f, 0.f);
        dpre[i] = e < nc * n ? id[e] : 0.0;
    }
    if (!st[b].active) return;
    store_twiddles<P2>(twf, tl, n);
#pragma unroll
    for (int i = 0; i < kPrefetch; ++i) {
        const int e = threadIdx.x + i * kThreads;
        if (e < nc * n) X[lp(e)] = cpre[i];
    }
    for (int e = threadIdx.x + kPrefetch * kThreads; e < nc * n; e += kThreads) X[lp(e)] = col[e];
    __syncthreads();
    float2 *Z = lds_fft_any<false, P2>(X, Y, n, nc, n, tl);
    auto divide = [&](int e, double d) {
        const float2 z = Z[lp(e)];
        Z[lp(e)] = make_float2((float)(z.x * d), (float)(z.y * d));
    };
#pragma unroll
    for (int i = 0; i < kPrefetch; ++i) {
        const int e = threadIdx.x + i * kThreads;
        if (e < nc * n) divide(e, dpre[i]);
    }
    for (int e = threadIdx.x + kPrefetch * kThreads; e < nc * n; e += kThreads) divide(e, id[e]);
    __syncthreads();
    float2 *W = (Z == X) ? Y : X;
    const float2 *out = lds_fft_any<true, P2>(Z, W, n, nc, n, tl);
    for (int e = threadIdx.x; e < nc * n; e += kThreads) col[e] = out[lp(e)];
}


// Inverse row pass (see the file header).  FUSED: the last block of each image to
// finish (counted in `counters`, one zeroed int per image) also applies the stop
// rule; this needs a device-scope fence per block.  Off by default: a separate
// k_stop_rule pass is faster even for one image (TVCS_FUSED_STOP).
// With T non-null (the partial-DCT operator) the block also transforms its new
// rows of u (DCT-II along each row, the first pass of the next iteration's
// forward product) and writes them column-major to T, as the DCT row pass does.
template <bool FUSED, bool P2>
__global__ __launch_bounds__(kThreads) void k_rows_inv(int n, int rpb, const float2 *__restrict__ S,
                                                       float *__restrict__ U,
                                                       double *__restrict__ parts,
                                                       const float2 *__restrict__ tw,
                                                       ImgState *__restrict__ st,
                                                       int *__restrict__ counters,
                                                       float *__restrict__ T,
                                                       const float4 *__restrict__ dtab,
                                                       int parity, float *__restrict__ dir) {
    const int b = blockIdx.y;
    extern __shared__ float2 lds[];
    const int npair = rpb >> 1, h = n / 2 + 1;
    const Ring<P2> ring(n);
    const int bufsz = npair * n + rpb;
    float2 *tl = lds, *X = lds + kMaxN, *Y = X + lp_size(bufsz);
    float4 *dt = reinterpret_cast<float4 *>(Y + lp_size(bufsz));   // DCT table (T non-null)
    const int blk = xcd_block(blockIdx.x, gridDim.x), row0 = blk * rpb;
    // The twiddles, each thread's first kPrefetch half-spectrum entries and the
    // pixel pairs of u it will update are all loaded before anything waits, and
    // before the image's flag is read (every address is in bounds whether or not the
    // image is active): one memory round trip instead of one per loop and one more
    // after the inverse FFT.
    Twiddles twf;
    fetch_twiddles<P2>(twf, tw, n);
    const float2 *srcS = S + (size_t)b * h * n + row0;
    const float rrpb = 1.0f / (float)rpb;
    float *dstU = U + (size_t)b * n * n + (size_t)row0 * n;
    float2 spre[kPrefetch];
    float upre[kPrefetch][2];
#pragma unroll
    for (int i = 0; i < kPrefetch; ++i) {
        const int e = threadIdx.x + i * kThreads;
        spre[i] = make_float2(0.f, 0.f);
        if (e < h * rpb) {
            const int k = div_by(e, rpb, rrpb), rr = e - k * rpb;
            spre[i] = srcS[(size_t)k * n + rr];
        }
        upre[i][0] = upre[i][1] = 0.f;
        if (!dir && e < npair * n) {
            const int pr = ring.div(e), j = e - ring.mul(pr);
            upre[i][0] = dstU[(2 * pr) * n + j];
            upre[i][1] = dstU[(2 * pr + 1) * n + j];
        }
    }
    if (!st[b].active) return;
    store_twiddles<P2>(twf, tl, n);
    if (T)
        for (int k = threadIdx.x; k < n; k += kThreads) dt[k] = dtab[k];
    // raw half spectra of the block's rows: Y[rr * h + k]
#pragma unroll
    for (int i = 0; i < kPrefetch; ++i) {
        const int e = threadIdx.x + i * kThreads;
        if (e < h * rpb) {
            const int k = div_by(e, rpb, rrpb), rr = e - k * rpb;
            Y[rr * h + k] = spre[i];
        }
    }
    for (int e = threadIdx.x + kPrefetch * kThreads; e < h * rpb; e += kThreads) {
        const int k = div_by(e, rpb, rrpb), rr = e - k * rpb;
        Y[rr * h + k] = srcS[(size_t)k * n + rr];
    }
    __syncthreads();
    // full spectrum of x + i y: Z_k = X_k + i Y_k (k <= n/2), conj(X) + i conj(Y) above
    for (int e = threadIdx.x; e < npair * n; e += kThreads) {
        const int pr = ring.div(e), k = e - ring.mul(pr);
        const bool lo = k <= n / 2;
        const int kk = lo ? k : n - k;
        const float2 x = Y[(2 * pr) * h + kk], y = Y[(2 * pr + 1) * h + kk];
        X[lp(e)] = lo ? make_float2(x.x - y.y, x.y + y.x) : make_float2(x.x + y.y, y.x - x.y);
    }
    __syncthreads();
    float2 *z = lds_fft_any<true, P2>(X, Y, n, npair, n, tl);
    float2 *W = (z == X) ? Y : X;   // free: receives the new rows for the DCT
    float *Wf = reinterpret_cast<float *>(W);
    double du2 = 0.0, u2 = 0.0;
    if (dir) {   // the increment is a search direction: stored apart, with its squared norm
        float *dstD = dir + (size_t)b * n * n + (size_t)row0 * n;
        for (int e = threadIdx.x; e < npair * n; e += kThreads) {
            const int pr = ring.div(e), j = e - ring.mul(pr);
            const float2 v = z[lp(e)];
            dstD[(2 * pr) * n + j] = v.x;
            dstD[(2 * pr + 1) * n + j] = v.y;
            du2 += (double)v.x * v.x + (double)v.y * v.y;
        }
    }
    auto update = [&](int e, float u0, float u1) {
        const int pr = ring.div(e), j = e - ring.mul(pr);
        const float2 v = z[lp(e)];
        float *p0 = dstU + (2 * pr) * n + j, *p1 = p0 + n;
        const double o0 = u0, o1 = u1;
        const float n0 = (float)(o0 + (double)v.x), n1 = (float)(o1 + (double)v.y);
        const double d0 = (double)n0 - o0, d1 = (double)n1 - o1;   // the stored change
        du2 += d0 * d0 + d1 * d1;
        u2 += o0 * o0 + o1 * o1;
        *p0 = n0;
        *p1 = n1;
        if (T) {   // rows 2 pr and 2 pr + 1, reordered, as one complex line pair
            const int q = 2 * lp(pr * n + makhoul_pos(j, n));
            Wf[q] = n0;
            Wf[q + 1] = n1;
        }
    };
    if (!dir) {   // in the order e = t, t + kThreads, ... (the sums' order)
#pragma unroll
        for (int i = 0; i < kPrefetch; ++i) {
            const int e = threadIdx.x + i * kThreads;
            if (e < npair * n) update(e, upre[i][0], upre[i][1]);
        }
        for (int e = threadIdx.x + kPrefetch * kThreads; e < npair * n; e += kThreads) {
            const int pr = ring.div(e), j = e - ring.mul(pr);
            update(e, dstU[(2 * pr) * n + j], dstU[(2 * pr + 1) * n + j]);
        }
    }
    if (T) {   // the same for every thread
        __syncthreads();
        const float2 *Z = lds_fft_any<false, P2>(W, z, n, npair, n, tl);
        float *dstT = T + (size_t)b * n * n + row0;
        const float rrpb = 1.0f / (float)rpb;
        for (int e = threadIdx.x; e < rpb * n; e += kThreads) {
            const int k = div_by(e, rpb, rrpb), l = e - k * rpb;
            dstT[(size_t)k * n + l] = dct_coef<P2>(Z, dt, n, l, k);
        }
    }
    // block reduction in a fixed order
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        du2 += __shfl_xor(du2, off, 64);
        u2 += __shfl_xor(u2, off, 64);
    }
    __shared__ double red[2][kThreads / 64];
    __shared__ int s_last;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wave] = du2;
        red[1][wave] = u2;
    }
    __syncthreads();
    double *myparts = parts + (size_t)b * gridDim.x * 2;
    if (threadIdx.x == 0) {
        double a = 0.0, c = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) {
            a += red[0][w];
            c += red[1][w];
        }
        // publish this block's sums device-wide, then count the block as done
        __hip_atomic_store(myparts + 2 * blk, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(myparts + 2 * blk + 1, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (FUSED) {
            __threadfence();
            s_last = atomicAdd(&counters[b], 1) == (int)gridDim.x - 1;
        }
    }
    if (!FUSED) return;
    __syncthreads();
    if (!s_last) return;
    // The last block of image b applies the stop rule
    __threadfence();
    if (threadIdx.x < 64) stop_rule(st + b, myparts, gridDim.x, counters + b, parity);
}

// Stop rule after an inverse row pass, for images whose row passes ran without
// the fused reduction (batches): one 64-lane block per image.
__global__ __launch_bounds__(64) void k_stop_rule(ImgState *__restrict__ st,
                                                  const double *__restrict__ parts, int nparts,
                                                  int parity) {
    const int b = blockIdx.x;
    if (!st[b].active) return;
    stop_rule(st + b, parts + (size_t)b * nparts * 2, nparts, nullptr, parity);
}

// Rows (columns) per workgroup: enough workgroups for one image to spread over
// the chip, and at most 64 KiB of LDS per workgroup (rpb * n <= 4096 complex,
// cpb * n <= 2048 complex per buffer).  The row blocking fixes the order in which
// the stop-rule norms are summed, so it depends on n only: an image's iterates and
// stop decisions are then the same whatever batch it is solved in.
#ifndef TVCS_FFT_ROW_DIV
#define TVCS_FFT_ROW_DIV 64    // rows per workgroup = n / TVCS_FFT_ROW_DIV (at least 2)
#endif
#ifndef TVCS_FFT_ROW_MAX
#define TVCS_FFT_ROW_MAX 4     // at most this many rows per workgroup (measured best at 512)
#endif
int rows_per_block(int n, int /*B*/) {
    const int want =
        std::max(2, std::min(std::min(n / TVCS_FFT_ROW_DIV, 4096 / n), TVCS_FFT_ROW_MAX));
    int d = even_divisor_at_most(n, want);
    if (d < want)   // sides with factors 3 and 5: the nearest even divisor above, within 2x
        for (int e = want + (want & 1); e <= 2 * want && e <= n; e += 2)
            if (n % e == 0) {
                d = e;
                break;
            }
    return d;
}
#ifndef TVCS_FFT_COLS_BATCH
#define TVCS_FFT_COLS_BATCH 2   // columns per workgroup of the batched column pass
#endif
#ifndef TVCS_FFT_COLS_SINGLE_DIV
#define TVCS_FFT_COLS_SINGLE_DIV 32   // one image: columns per workgroup = (n/2 + 1) / this (at least 1)
#endif
int cols_per_block(int n, int B) {
    const int h = n / 2 + 1;
    int cpb = B == 1 ? std::max(1, h / TVCS_FFT_COLS_SINGLE_DIV) : TVCS_FFT_COLS_BATCH;
    return std::max(1, std::min(std::min(cpb, 2048 / n), h));
}

}  // namespace

void launch_twiddles(int n, float2 *tw, hipStream_t s) {
    const int L = is_pow2(n) ? kMaxN : n;
    hipLaunchKernelGGL(k_twiddles, dim3((L + 255) / 256), dim3(256), 0, s, tw, L);
}

void launch_denominators(int n, double c, double *inv_d, hipStream_t s) {
    const int cnt = (n / 2 + 1) * n;
    hipLaunchKernelGGL(k_denominators, dim3((cnt + 255) / 256), dim3(256), 0, s, n, c, inv_d);
}

void launch_fft_cols_solve(int n, int B, float2 *S, const double *inv_d, const float2 *tw,
                           const ImgState *st, hipStream_t s) {
    const int cpb = cols_per_block(n, B), h = n / 2 + 1;
    const size_t lds = sizeof(float2) * (kMaxN + 2 * lp_size(cpb * n));
    if (is_pow2(n))
        hipLaunchKernelGGL(k_cols_solve<true>, dim3((h + cpb - 1) / cpb, B), dim3(kThreads), lds, s,
                           n, cpb, S, inv_d, tw, st);
    else
        hipLaunchKernelGGL(k_cols_solve<false>, dim3((h + cpb - 1) / cpb, B), dim3(kThreads), lds, s,
                           n, cpb, S, inv_d, tw, st);
}

#ifndef TVCS_FUSED_STOP
#define TVCS_FUSED_STOP 0   // 1: for one image the inverse row pass applies the stop rule itself
#endif
int stop_parts(int n, int B) { return n / rows_per_block(n, B); }

void launch_fft_rows_inv(int n, int B, const float2 *S, float *U, double *parts,
                         const float2 *tw, ImgState *st, int *counters, hipStream_t s, float *T,
                         const float4 *dtab, bool stop_pass, int parity, float *dir) {
    const int rpb = rows_per_block(n, B);
    const size_t lds = sizeof(float2) * (kMaxN + 2 * lp_size((rpb / 2) * n + rpb)) +
                       (T ? sizeof(float4) * n : 0);
#define TVCS_ROWS_INV(FUSEDV, P2V)                                                            \
    hipLaunchKernelGGL((k_rows_inv<FUSEDV, P2V>), dim3(n / rpb, B), dim3(kThreads), lds, s, n, rpb, \
                       S, U, parts, tw, st, counters, T, dtab, parity, dir)
    const bool p2 = is_pow2(n);
    if (TVCS_FUSED_STOP && B == 1 && stop_pass) {
        if (p2) TVCS_ROWS_INV(true, true);
        else TVCS_ROWS_INV(true, false);
    } else {
        if (p2) TVCS_ROWS_INV(false, true);
        else TVCS_ROWS_INV(false, false);
        if (stop_pass)
            hipLaunchKernelGGL(k_stop_rule, dim3(B), dim3(64), 0, s, st, parts, n / rpb, parity);
    }
#undef TVCS_ROWS_INV
}

#ifndef TVCS_SHRINK_PX
#define TVCS_SHRINK_PX 4       // pixels per thread and round of the pixel-parallel pass
#endif
#ifndef TVCS_SHRINK_WALK_ROWS
#define TVCS_SHRINK_WALK_ROWS 4   // row blocks at least this tall use the column walk
#endif
void launch_shrink_rows(const ShrinkArgs &a, bool iadm, float2 *S, const float2 *tw,
                        hipStream_t s) {
    const int n = a.n, rpb = rows_per_block(n, a.B);
    const dim3 grid(n / rpb, a.B);
    const size_t bufsz = (size_t)(rpb / 2) * n + rpb;
    const bool p2 = is_pow2(n);
    // few partial sums of g: fewer loads in flight, fewer registers (same bits)
    const bool few = a.nchunk <= 4;
    // partial DCT: the g rows (or, first, the DCT table) after the FFT buffers
    const size_t gbytes =
        a.T ? std::max(sizeof(float) * (size_t)rpb * n, sizeof(float4) * (size_t)n) : 0;
    if (rpb < TVCS_SHRINK_WALK_ROWS) {
        const size_t lds = sizeof(float2) * (kMaxN + 2 * lp_size((int)bufsz)) + gbytes;
        // several pixels per round where the partial sums of g are few (their loads
        // would otherwise cost registers) and each thread has several pixels
        const bool multi = few && rpb * n >= 2 * kThreads;
#define TVCS_PIX(IADMV, PXV, PLV)                                                          \
    do {                                                                                   \
        if (p2)                                                                            \
            hipLaunchKernelGGL((k_shrink_pix<IADMV, PXV, true, PLV>), grid, dim3(kThreads), \
                               lds, s, a, rpb, S, tw);                                     \
        else                                                                               \
            hipLaunchKernelGGL((k_shrink_pix<IADMV, PXV, false, PLV>), grid, dim3(kThreads), \
                               lds, s, a, rpb, S, tw);                                     \
    } while (0)
        if (iadm) {
            if (multi) TVCS_PIX(true, TVCS_SHRINK_PX, 4);
            else if (few) TVCS_PIX(true, 1, 4);
            else TVCS_PIX(true, 1, TVCS_PARTIAL_LOADS);
        } else {
            if (multi) TVCS_PIX(false, TVCS_SHRINK_PX, 4);
            else if (few) TVCS_PIX(false, 1, 4);
            else TVCS_PIX(false, 1, TVCS_PARTIAL_LOADS);
        }
#undef TVCS_PIX
        return;
    }
    // column walk: as many row groups of n threads as fit, dividing the block's rows
    int groups = std::max(1, std::min(rpb, kThreads / n));
    while (rpb % groups) --groups;
    const size_t ybytes =
        std::max(sizeof(float2) * lp_size((int)bufsz), sizeof(double) * 2 * groups * n);
    const size_t lds = sizeof(float2) * (kMaxN + lp_size((int)bufsz)) + ybytes + gbytes;
#define TVCS_WALK(IADMV, P2V, PLV)                                                           \
    hipLaunchKernelGGL((k_shrink_walk<IADMV, P2V, PLV>), grid, dim3(kThreads), lds, s, a, rpb, \
                       groups, S, tw)
#define TVCS_WALK_PL(IADMV, P2V)                                 \
    do {                                                         \
        if (few) TVCS_WALK(IADMV, P2V, 4);                       \
        else TVCS_WALK(IADMV, P2V, TVCS_PARTIAL_LOADS);          \
    } while (0)
    if (iadm) {
        if (p2) TVCS_WALK_PL(true, true);
        else TVCS_WALK_PL(true, false);
    } else {
        if (p2) TVCS_WALK_PL(false, true);
        else TVCS_WALK_PL(false, false);
    }
#undef TVCS_WALK_PL
#undef TVCS_WALK
}

}  // namespace tvcs
