// FP32 dense products A u and A^T r for a row-major A (m x N), streamed from HBM.
//
// These are the "two matrix-vector multiplications" of each iteration (Sec. 2.1,
// g_k = A^T (A u^k - f) in eq. (line)).  Both read A once per call with 16-byte
// coalesced loads along its rows, so one row-major copy of A serves both:
//   * rows: one workgroup owns ROWS consecutive rows and sweeps them together, so
//     each u element loaded from cache feeds ROWS rows; the dot products are
//     reduced across the workgroup (wave shuffles, then LDS).
//   * cols: one workgroup owns 1024 consecutive columns (a float4 per thread) and
//     a chunk of rows; each row segment is a contiguous 4 KiB read.  Per-chunk
//     partial sums go to a buffer and are added in a fixed order by the consumer
//     (no atomics), so results are bit-reproducible run to run.
// Up to NV right-hand sides share one pass over A (batched solves).
//
// One image with n^2 <= 16384 takes both products in one pass (k_gemv_fused):
// g = A^T (A u - f) = sum_i a_i (a_i . u - f_i) needs only row i of A for row i's
// term, so a workgroup that holds a whole row in registers reduces a_i . u across
// its threads, forms r_i, and adds r_i a_i to its share of g before the row leaves
// the registers: A is read once per iteration instead of twice.  Each workgroup
// owns a contiguous band of rows and writes one partial g; k_sum_bands adds the
// bands' partials in a fixed order.
//
// Products and sums are formed in FP64 from the FP32 operands (each product is
// exact).  r = A u - f is a small residual of O(1) terms, so FP32 accumulation
// would put an error of ~sqrt(N) eps |A||u| into it; the FP64 units have an
// order of magnitude more throughput than this HBM-bound loop needs.
#include "device_bb.h"
#include "device_stop.h"
#include "tvcs_internal.h"

#include <algorithm>
#include <type_traits>

// Tile parameters (compile-time; the defaults are the measured best on MI355X)
#ifndef TVCS_GEMV_ROWS
#define TVCS_GEMV_ROWS 2      // rows per workgroup of the A u product (1-2 vectors)
#endif
#ifndef TVCS_GEMV_UNROLL
#define TVCS_GEMV_UNROLL 8    // float4 loads per row in flight
#endif
#ifndef TVCS_COLS_VEC
#define TVCS_COLS_VEC 4       // float4 column groups per thread of the A^T r product
#endif
#ifndef TVCS_COLS_TARGET_WG
#define TVCS_COLS_TARGET_WG 1024   // workgroups the A^T r product aims for
#endif
#ifndef TVCS_GEMV_NT_BYTES
// A larger than this is read with nontemporal (streaming) loads, a smaller one with
// ordinary loads (measured: ordinary loads win while A is about the size of the
// 256 MB Infinity Cache, streaming loads for multi-GB A)
#define TVCS_GEMV_NT_BYTES (512ull << 20)
#endif
#ifndef TVCS_COLS_NT_BYTES
#define TVCS_COLS_NT_BYTES TVCS_GEMV_NT_BYTES   // the same threshold for the A^T r product
#endif
#ifndef TVCS_GEMV_ROWS_REVERSE
#define TVCS_GEMV_ROWS_REVERSE 1   // the A u product visits rows last to first (0: first to last)
#endif
#ifndef TVCS_COLS_RS
#define TVCS_COLS_RS 1        // row phases (256 threads each) per workgroup of A^T r
#endif
#ifndef TVCS_COLS_SLOTS
#define TVCS_COLS_SLOTS 0     // >0: row-chunk slots per column block of A^T r (0: one per chunk)
#endif
#ifndef TVCS_COLS_R_LDS
#define TVCS_COLS_R_LDS 0     // 1: a chunk's r coefficients are staged in LDS first
#endif
#ifndef TVCS_COLS_REVERSE
#define TVCS_COLS_REVERSE 0   // 1: sweep row chunks last-to-first (after A u read first-to-last)
#endif

namespace tvcs {
namespace {

constexpr int kThreads = 256;

// native 4-wide vector (the nontemporal load builtin needs a clang vector type)
typedef float f4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ inline f4 load_a(const f4 *p) {
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

__device__ inline bool any_active(const ImgState *st, int nact) {
    if (st == nullptr) return true;
    int a = 0;
    for (int i = 0; i < nact; ++i) a |= st[i].active;
    return a != 0;
}

__device__ inline double dot4(f4 a, const double (&x)[4], double acc) {
    acc = fma((double)a.x, x[0], acc);
    acc = fma((double)a.y, x[1], acc);
    acc = fma((double)a.z, x[2], acc);
    return fma((double)a.w, x[3], acc);
}

// stw (one image, non-null): workgroup 0 first applies the stop rule of the
// previous iteration to stw from its nparts norm partials (as k_stop_rule would
// after the inverse row pass).  The other workgroups may read the flag before or
// after that update: when the rule stops the image, some of them still write R,
// which no later pass of a stopped image reads.
template <int NV, int ROWS, bool NT>
__global__ __launch_bounds__(kThreads) void k_gemv_rows(
    const float *__restrict__ A, int m, int N, const float *__restrict__ U, int ldu,
    const float *__restrict__ F, int ldf, float *__restrict__ R, int ldr,
    const ImgState *st, int nact, ImgState *stw, const double *parts, int nparts) {
    if (stw && blockIdx.x == 0) {
        if (threadIdx.x < 64 && stw->active) stop_rule(stw, parts, nparts, nullptr);
        __syncthreads();
    }
    if (!any_active(st, nact)) return;
    // Workgroups take row pairs from the last to the first (TVCS_GEMV_ROWS_REVERSE):
    // measured 0.4 % faster per 500-iteration solve at n = 128 (A of 256 MiB, about
    // the Infinity Cache's size), presumably from what the cache still holds of A.
    const int row0 = (TVCS_GEMV_ROWS_REVERSE ? (int)(gridDim.x - 1 - blockIdx.x) : (int)blockIdx.x) * ROWS;
    const int N4 = N >> 2;
    const f4 *rowp[ROWS];
#pragma unroll
    for (int r = 0; r < ROWS; ++r) {
        const int row = min(row0 + r, m - 1);   // ragged tail: re-read a valid row
        rowp[r] = reinterpret_cast<const f4 *>(A + (size_t)row * N);
    }
    double acc[ROWS][NV];
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[r][v] = 0.0;

#pragma unroll TVCS_GEMV_UNROLL
    for (int j = threadIdx.x; j < N4; j += kThreads) {
        f4 a[ROWS];
#pragma unroll
        for (int r = 0; r < ROWS; ++r) a[r] = load_a<NT>(rowp[r] + j);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const f4 x = reinterpret_cast<const f4 *>(U + (size_t)v * ldu)[j];
            const double xd[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int r = 0; r < ROWS; ++r) acc[r][v] = dot4(a[r], xd, acc[r][v]);
        }
    }

    // reduce over the 64 lanes of each wave, then over the 4 waves
    __shared__ double red[kThreads / 64][ROWS * NV];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < ROWS; ++r)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double x = acc[r][v];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
            if (lane == 0) red[wave][r * NV + v] = x;
        }
    __syncthreads();
    if (threadIdx.x < ROWS * NV) {
        const int r = threadIdx.x / NV, v = threadIdx.x % NV;
        const int row = row0 + r;
        if (row < m) {
            double x = (red[0][threadIdx.x] + red[1][threadIdx.x]) +
                       (red[2][threadIdx.x] + red[3][threadIdx.x]);
            if (F) x -= (double)F[(size_t)v * ldf + row];
            R[(size_t)v * ldr + row] = (float)x;
        }
    }
}

// Row chunks are visited by gridDim.y slots: slot s takes chunks s, s + slots, ...
// (counted from the last chunk when TVCS_COLS_REVERSE), accumulating all of them
// before it writes its partial sums.  A workgroup has RS row phases of 256 threads:
// phase p takes rows p, p + RS, ... of each chunk for the same columns, and the
// phases' sums are added in phase order at the end.  The chunking, the slots and
// the phases depend on (m, N) only.
template <int NV, bool NT>
__global__ __launch_bounds__(kThreads * TVCS_COLS_RS) void k_gemv_cols(
    const float *__restrict__ A, int m, int N, const float *__restrict__ Rv, int ldr,
    float *__restrict__ P, long long chunk_stride, int rows_per_chunk, int nrowchunk,
    const ImgState *__restrict__ st, int nact) {
    constexpr int VEC = TVCS_COLS_VEC, RS = TVCS_COLS_RS;
    if (!any_active(st, nact)) return;
    extern __shared__ double rs[];           // rows_per_chunk x NV coefficients, then 256 x 4
    const int N4 = N >> 2;
    const int tl = threadIdx.x & (kThreads - 1), phase = threadIdx.x / kThreads;
    // the workgroup covers VEC * 256 consecutive float4 columns; thread t owns
    // columns t, t + 256, ... so each wave still reads contiguous 1 KiB pieces
    const int jb = blockIdx.x * kThreads * VEC + tl;
    double acc[VEC][NV][4];
#pragma unroll
    for (int c = 0; c < VEC; ++c)
#pragma unroll
        for (int v = 0; v < NV; ++v) acc[c][v][0] = acc[c][v][1] = acc[c][v][2] = acc[c][v][3] = 0.0;
    for (int idx = blockIdx.y; idx < nrowchunk; idx += gridDim.y) {
        const int chunk = TVCS_COLS_REVERSE ? nrowchunk - 1 - idx : idx;
        const int i0 = chunk * rows_per_chunk;
        const int rows = min(rows_per_chunk, m - i0);
        if (TVCS_COLS_R_LDS) {
            __syncthreads();   // the previous chunk's coefficients are no longer read
            for (int t = threadIdx.x; t < rows * NV; t += kThreads * RS) {
                const int i = t / NV, v = t % NV;
                rs[t] = Rv[(size_t)v * ldr + i0 + i];
            }
            __syncthreads();
        }
        const f4 *col = reinterpret_cast<const f4 *>(A + (size_t)i0 * N);
#pragma unroll 8
        for (int i = phase; i < rows; i += RS) {
            f4 a[VEC];
#pragma unroll
            for (int c = 0; c < VEC; ++c) {
                const int j4 = jb + c * kThreads;
                a[c] = j4 < N4 ? load_a<NT>(col + (size_t)i * N4 + j4) : f4{0, 0, 0, 0};
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                // the row's coefficient: staged in LDS, or read where it is used (one
                // address for the whole workgroup, no barrier before the A stream)
                const double r = TVCS_COLS_R_LDS ? rs[i * NV + v] : (double)Rv[(size_t)v * ldr + i0 + i];
#pragma unroll
                for (int c = 0; c < VEC; ++c) {
                    acc[c][v][0] = fma((double)a[c].x, r, acc[c][v][0]);
                    acc[c][v][1] = fma((double)a[c].y, r, acc[c][v][1]);
                    acc[c][v][2] = fma((double)a[c].z, r, acc[c][v][2]);
                    acc[c][v][3] = fma((double)a[c].w, r, acc[c][v][3]);
                }
            }
        }
    }
    if (RS > 1) {   // phase 0 adds the other phases' sums, one (c, v) at a time
        double *buf = rs + (TVCS_COLS_R_LDS ? rows_per_chunk * NV : 0);
#pragma unroll
        for (int c = 0; c < VEC; ++c)
#pragma unroll
            for (int v = 0; v < NV; ++v)
                for (int p = 1; p < RS; ++p) {
                    __syncthreads();
                    if (phase == p)
                        for (int e = 0; e < 4; ++e) buf[e * kThreads + tl] = acc[c][v][e];
                    __syncthreads();
                    if (phase == 0)
                        for (int e = 0; e < 4; ++e) acc[c][v][e] += buf[e * kThreads + tl];
                }
        if (phase != 0) return;
    }
#pragma unroll
    for (int c = 0; c < VEC; ++c) {
        const int j4 = jb + c * kThreads;
        if (j4 >= N4) continue;
#pragma unroll
        for (int v = 0; v < NV; ++v)
            reinterpret_cast<f4 *>(P + blockIdx.y * chunk_stride + (size_t)v * N)[j4] =
                f4{(float)acc[c][v][0], (float)acc[c][v][1], (float)acc[c][v][2], (float)acc[c][v][3]};
    }
}

template <int NV>
void rows_dispatch(const float *A, int m, int N, const float *U, int ldu, const float *F,
                   int ldf, float *R, int ldr, const ImgState *st, int nact, ImgState *stw,
                   const double *parts, int nparts, hipStream_t s) {
    constexpr int ROWS = NV <= 2 ? TVCS_GEMV_ROWS : 2;
    const int grid = (m + ROWS - 1) / ROWS;
    if ((size_t)m * N * sizeof(float) > TVCS_GEMV_NT_BYTES)
        hipLaunchKernelGGL((k_gemv_rows<NV, ROWS, true>), dim3(grid), dim3(kThreads), 0, s, A, m,
                           N, U, ldu, F, ldf, R, ldr, st, nact, stw, parts, nparts);
    else
        hipLaunchKernelGGL((k_gemv_rows<NV, ROWS, false>), dim3(grid), dim3(kThreads), 0, s, A, m,
                           N, U, ldu, F, ldf, R, ldr, st, nact, stw, parts, nparts);
}

// ---- one image, both products in one pass over A --------------------------------
constexpr int kFusedThreadsMax = 1024;   // up to 16 waves: four per SIMD

#ifndef TVCS_FUSED_DPP
#define TVCS_FUSED_DPP 1   // the per-row wave sums through DPP moves (0: shuffles)
#endif
#ifndef TVCS_FUSED_ROWS
#define TVCS_FUSED_ROWS 3  // rows held in registers (ROWS - 1 in flight while one is used)
#endif
#ifndef TVCS_FUSED_ACC64
#define TVCS_FUSED_ACC64 1 // a band's share of g summed in FP64 (0: FP32)
#endif
#ifndef TVCS_FUSED_U64
#define TVCS_FUSED_U64 1   // u held in LDS as FP64 (converted once instead of per row)
#endif
#ifndef TVCS_FUSED_XSUM
#define TVCS_FUSED_XSUM 0  // the waves' sums of a row added by 16-lane DPP steps (0: serially)
#endif
#ifndef TVCS_FUSED_INTERLEAVE
#define TVCS_FUSED_INTERLEAVE 0   // workgroups take rows b, b + nb, ... instead of a band
#endif
#ifndef TVCS_FUSED_STEADY
#define TVCS_FUSED_STEADY 0   // 1: every trip of the row loop issues its loads (no branch around them)
#endif
// A double through two DPP moves of its 32-bit halves.  Rows the row mask leaves out
// keep whatever the destination registers held: no zero is written there first, so
// callers use those lanes' results only where the mask wrote every lane they read.
template <int CTRL, int ROWS>
__device__ inline double dpp_f64(double x) {
    const unsigned long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, ROWS, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// The sum of x over a 64-lane wave (every lane gets it): pairs and quads by quad
// permutes, 8 and 16 lanes by the half-row and row mirrors, then rows 0 + 1 and
// 2 + 3 by the row-15 broadcast and all four by the row-31 broadcast into lane 63
// (rows 0 and 2 take undefined values at the broadcasts; lane 63 reads only rows the
// masks wrote).
__device__ inline double wave_sum_dpp(double x) {
    x += dpp_f64<0xB1, 0xF>(x);    // quad_perm [1, 0, 3, 2]
    x += dpp_f64<0x4E, 0xF>(x);    // quad_perm [2, 3, 0, 1]
    x += dpp_f64<0x141, 0xF>(x);   // row_half_mirror
    x += dpp_f64<0x140, 0xF>(x);   // row_mirror
    x += dpp_f64<0x142, 0xA>(x);   // row_bcast:15 into rows 1 and 3
    x += dpp_f64<0x143, 0xC>(x);   // row_bcast:31 into rows 2 and 3
    const unsigned long long b = __double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)b, 63);
    const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Rows [band * rpb, min(m, (band + 1) * rpb)) of A, band = blockIdx.x.  Thread t of
// T = blockDim.x owns the float4 column groups t, t + T, ..., t + (G - 1) T (only
// the last may fall past the row: it then reads a valid group and contributes
// zero); u sits in LDS (as FP64: 128 KiB at n^2 = 16384, converted once instead of
// once per row), rows are loaded two rows ahead, a_i . u is reduced
// over the workgroup (wave shuffles, then the waves' sums in a fixed order through
// LDS, one barrier per row; the LDS slot alternates with the row so no second
// barrier is needed), r_i = a_i . u - f_i is rounded to FP32 (as the two-pass path
// stores it; F null: f = 0; Rout non-null: r_i goes to Rout[i]), and r_i a_i is
// added to the thread's FP64 share of g.  The band's partial g (FP32) goes to
// P[band * N ..].  (The previous iteration's stop rule,
// which k_gemv_rows applies in its workgroup 0, is applied by k_sum_bands here:
// with one workgroup per CU, a late workgroup 0 would hold up the whole pass.)
template <int G, bool NT>
__global__ __launch_bounds__(kFusedThreadsMax) void k_gemv_fused(
    const float *__restrict__ A, int m, int N, int rpb, const float *__restrict__ U,
    const float *__restrict__ F, float *__restrict__ P, const ImgState *st, int rev,
    float *__restrict__ Rout) {
    if (!any_active(st, 1)) return;
    const int T = blockDim.x, t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = T >> 6;
    const int N4 = N >> 2;
    const int jl = t + (G - 1) * T;            // the last group
    const bool last_ok = jl < N4;
    const int jlc = last_ok ? jl : N4 - 1;     // a valid group to read instead
    auto col = [&](int k) { return k == G - 1 ? jlc : t + k * T; };
    // u in LDS (the registers go to a third row in flight); a thread reads only its
    // own groups, so the one barrier of the first row orders these stores
    using u4 = std::conditional_t<TVCS_FUSED_U64 != 0, double4, f4>;
    __shared__ u4 us[kFusedN / 4];
    __shared__ double red[2][kFusedThreadsMax / 64];
    // TVCS_FUSED_INTERLEAVE: workgroup b takes rows b, b + nb, b + 2 nb, ... (the
    // workgroups then read neighbouring rows at the same time); else the band of rpb
    // consecutive rows from b rpb
    const int nb = gridDim.x, b = blockIdx.x;
    const int r0 = TVCS_FUSED_INTERLEAVE ? b : b * rpb;
    const int r1 = TVCS_FUSED_INTERLEAVE ? m : min(m, r0 + rpb);
    const int rstep = TVCS_FUSED_INTERLEAVE ? nb : 1;
    using acc_t = std::conditional_t<TVCS_FUSED_ACC64 != 0, double, float>;
    acc_t gs[G][4];
    auto load = [&](f4 (&a)[G], int row) {
        const f4 *rp = reinterpret_cast<const f4 *>(A + (size_t)row * N);
#pragma unroll
        for (int k = 0; k < G; ++k) a[k] = load_a<NT>(rp + col(k));
    };
    auto row_term = [&](f4 (&a)[G], int row, int idx) {
        double d = 0.0;
#pragma unroll
        for (int k = 0; k < G; ++k) {
            const u4 x = us[t + k * T];
            const double xd[4] = {(double)x.x, (double)x.y, (double)x.z, (double)x.w};
            d = dot4(a[k], xd, d);
        }
        if (TVCS_FUSED_DPP) {
            d = wave_sum_dpp(d);
        } else {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
        }
        const int slot = idx & 1;
        if (lane == 0) red[slot][wave] = d;
        __syncthreads();
        double tot;
        if (TVCS_FUSED_XSUM) {   // lanes 0..15 of every wave add the 16 sums alike
            double v = lane < nw ? red[slot][lane & 15] : 0.0;
            v += dpp_f64<0xB1, 0xF>(v);
            v += dpp_f64<0x4E, 0xF>(v);
            v += dpp_f64<0x141, 0xF>(v);
            v += dpp_f64<0x140, 0xF>(v);
            const unsigned long long b = __double_as_longlong(v);
            const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)b, 0);
            const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 0);
            tot = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
        } else {
            tot = red[slot][0];
            for (int w = 1; w < nw; ++w) tot += red[slot][w];   // fixed order
        }
        const double r = (double)(float)(F ? tot - (double)F[row] : tot);
        if (Rout && t == 0) Rout[row] = (float)r;
        // keep the FP64 copies of the row from living across the barrier (they are
        // cheaper to convert again than the registers they would hold)
#pragma unroll
        for (int k = 0; k < G; ++k) asm volatile("" : "+v"(a[k]));
        const acc_t ra = (acc_t)r;
#pragma unroll
        for (int k = 0; k < G; ++k) {
            gs[k][0] = fma((acc_t)a[k].x, ra, gs[k][0]);
            gs[k][1] = fma((acc_t)a[k].y, ra, gs[k][1]);
            gs[k][2] = fma((acc_t)a[k].z, ra, gs[k][2]);
            gs[k][3] = fma((acc_t)a[k].w, ra, gs[k][3]);
        }
    };
    // R rows in registers: rows i + 1 .. i + R - 1 are in flight while row i is
    // used.  rev: the band's rows last to first (the solve alternates the direction
    // from one iteration to the next, so that each pass starts on the rows the
    // previous one read last, which the Infinity Cache may still hold)
    constexpr int R = TVCS_FUSED_ROWS;
    const int cnt = r1 > r0 ? (r1 - r0 + rstep - 1) / rstep : 0;
    auto row_of = [&](int i) { return r0 + rstep * (rev ? cnt - 1 - i : i); };
    f4 rows[R][G];
#pragma unroll
    for (int k = 0; k < R - 1; ++k)
        if (k < cnt) load(rows[k], row_of(k));
    // u after the first rows' loads, so that those are in flight meanwhile
#pragma unroll
    for (int k = 0; k < G; ++k) {
        const f4 x = reinterpret_cast<const f4 *>(U)[col(k)];
        const bool ok = k < G - 1 || last_ok;
        us[t + k * T] = u4{ok ? x.x : 0.f, ok ? x.y : 0.f, ok ? x.z : 0.f, ok ? x.w : 0.f};
#pragma unroll
        for (int c = 0; c < 4; ++c) gs[k][c] = 0;
    }
    // TVCS_FUSED_STEADY: every trip issues all R of its loads, one past the band's
    // end re-reading its last row.  The memory counter retires loads in issue order
    // and the compiler sizes each wait by the path that issues fewest loads, so with
    // the loads under a condition a row's first use also waits for the rows issued
    // after it; without it two rows stay in flight, yet the pass measured slower.
    for (int i = 0; i < cnt; i += R) {
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const int nx = i + k + R - 1;
            if (TVCS_FUSED_STEADY)
                load(rows[(k + R - 1) % R], row_of(min(nx, cnt - 1)));
            else if (nx < cnt)
                load(rows[(k + R - 1) % R], row_of(nx));
            if (i + k < cnt) row_term(rows[k], row_of(i + k), i + k);
        }
    }
    float *out = P + (size_t)blockIdx.x * N;
#pragma unroll
    for (int k = 0; k < G; ++k)
        if (k < G - 1 || last_ok)
            reinterpret_cast<f4 *>(out)[t + k * T] =
                f4{(float)gs[k][0], (float)gs[k][1], (float)gs[k][2], (float)gs[k][3]};
}

// g = the sum of the nb band partials P[b * N ..] in a fixed order: a workgroup
// takes 16 float4 columns; thread t (column group t % 16, subset q = t / 16) adds
// bands q, q + 16, ... in FP64, all its loads in flight at once (each load of a
// wave reads 256 contiguous bytes of 4 band rows); then the 16 subtotals are added
// pairwise through LDS.
// stw (one image, non-null): an extra last workgroup applies the previous
// iteration's stop rule from its nparts norm partials (alone, so that its latency
// overlaps the sums instead of adding to one workgroup's); the other workgroups
// may read the flag before or after, and when the rule stops the image some of
// them still write g, which no later pass of a stopped image reads.
// nm.parts non-null: nm.nblk workgroups before the others (dispatched first: each
// takes longer than a workgroup of sums) write the partial sums of the BB step
// length's norms (device_bb.h) for the image whose A p the pass just wrote.
constexpr int kSumCols4 = 16;   // float4 columns per workgroup
__global__ __launch_bounds__(256) void k_sum_bands(const float *__restrict__ P, int nb, int N,
                                                   float *__restrict__ out,
                                                   const ImgState *st, ImgState *stw,
                                                   const double *parts, int nparts, BBNorms nm) {
    const int N4 = N >> 2;
    const int nsum = (N4 + kSumCols4 - 1) / kSumCols4;   // workgroups of sums
    const int nn = nm.parts ? nm.nblk : 0;               // norm-partials workgroups
    if ((int)blockIdx.x < nn) {
        if (any_active(st, 1)) bb_norms_block(nm, 0, blockIdx.x);
        return;
    }
    const int bx = (int)blockIdx.x - nn;
    if (bx >= nsum) {   // the stop-rule workgroup (the rule reads the flag itself)
        if (stw && threadIdx.x < 64) stop_rule(stw, parts, nparts, nullptr);
        return;
    }
    // the partials are loaded before the image's flag is read (in bounds either way),
    // so that one memory round trip covers both
    constexpr int kSub = 256 / kSumCols4;                 // 16 subsets of bands
    constexpr int kPer = kFusedMaxBands / kSub;           // bands per subset
    const int t = threadIdx.x, c = t % kSumCols4, q = t / kSumCols4;
    const int j = bx * kSumCols4 + c;   // float4 group
    const int jc = j < N4 ? j : N4 - 1;
    f4 v[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        const int b = q + kSub * i;
        v[i] = b < nb ? reinterpret_cast<const f4 *>(P + (size_t)b * N)[jc]
                      : f4{0.f, 0.f, 0.f, 0.f};
    }
    if (!any_active(st, 1)) return;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
        acc[0] += (double)v[i].x;
        acc[1] += (double)v[i].y;
        acc[2] += (double)v[i].z;
        acc[3] += (double)v[i].w;
    }
    __shared__ double red[kSub][kSumCols4][4];
#pragma unroll
    for (int k = 0; k < 4; ++k) red[q][c][k] = acc[k];
    __syncthreads();
    for (int w = kSub / 2; w > 0; w >>= 1) {
        if (q < w)
#pragma unroll
            for (int k = 0; k < 4; ++k) red[q][c][k] += red[q + w][c][k];
        __syncthreads();
    }
    if (q == 0 && j < N4)
        reinterpret_cast<f4 *>(out)[j] = f4{(float)red[0][c][0], (float)red[0][c][1],
                                            (float)red[0][c][2], (float)red[0][c][3]};
}

// Row chunks of the A^T r product: aim for ~TVCS_COLS_TARGET_WG chunk x column
// block pairs; keep chunks >= 16 rows so partial-sum traffic stays a few percent
// of the A stream, and a chunk's coefficients (rows x nv doubles, nv <= 8) within
// 64 KiB of LDS.  Independent of nv, so the order of the sums does not depend on
// how many vectors share a pass.
int cols_rowchunks(int m, int N) {
    const int nv = 8;
    const int colblocks = (N / 4 + kThreads - 1) / kThreads;   // of 1024 columns
    int nchunk = (TVCS_COLS_TARGET_WG + colblocks - 1) / colblocks;
    nchunk = std::max(1, std::min(nchunk, (m + 15) / 16));
    nchunk = std::max(nchunk, (m * nv + 8191) / 8192);
    // rows per chunk is ceil(m / nchunk); recompute nchunk so none is empty
    const int rpc = (m + nchunk - 1) / nchunk;
    return (m + rpc - 1) / rpc;
}

template <int NV>
void cols_dispatch(const float *A, int m, int N, const float *R, int ldr, float *P,
                   long long chunk_stride, const ImgState *st, int nact, hipStream_t s) {
    const int nrc = cols_rowchunks(m, N);          // the same chunks for every NV
    const int rpc = (m + nrc - 1) / nrc;
    const int slots = gemv_cols_chunks(m, N);
    const int colblocks = (N / 4 + kThreads * TVCS_COLS_VEC - 1) / (kThreads * TVCS_COLS_VEC);
    const size_t lds =
        sizeof(double) * ((TVCS_COLS_R_LDS ? rpc * NV : 0) + (TVCS_COLS_RS > 1 ? 4 * kThreads : 0));
    const dim3 block(kThreads * TVCS_COLS_RS);
    if ((size_t)m * N * sizeof(float) > TVCS_COLS_NT_BYTES)
        hipLaunchKernelGGL((k_gemv_cols<NV, true>), dim3(colblocks, slots), block, lds, s, A, m, N,
                           R, ldr, P, chunk_stride, rpc, nrc, st, nact);
    else
        hipLaunchKernelGGL((k_gemv_cols<NV, false>), dim3(colblocks, slots), block, lds, s, A, m,
                           N, R, ldr, P, chunk_stride, rpc, nrc, st, nact);
}

}  // namespace

// Partial sums per column of the A^T r product: one per slot (TVCS_COLS_SLOTS > 0)
// or one per row chunk.
int gemv_cols_chunks(int m, int N) {
    const int nrc = cols_rowchunks(m, N);
    return TVCS_COLS_SLOTS > 0 ? std::min(TVCS_COLS_SLOTS, nrc) : nrc;
}

void launch_gemv_rows(const float *A, int m, int N, const float *U, int ldu, const float *F,
                      int ldf, float *R, int ldr, int nv, const ImgState *st, int nact,
                      hipStream_t s, ImgState *stw, const double *parts, int nparts) {
    if (stw && (nv != 1 || nact != 1 || st != stw || !parts || nparts < 1))
        fail(TVCS_EINVAL, "gemv_rows: the stop rule is folded in for one image only");
    switch (nv) {
        case 1: rows_dispatch<1>(A, m, N, U, ldu, F, ldf, R, ldr, st, nact, stw, parts, nparts, s); break;
        case 2: rows_dispatch<2>(A, m, N, U, ldu, F, ldf, R, ldr, st, nact, stw, parts, nparts, s); break;
        case 4: rows_dispatch<4>(A, m, N, U, ldu, F, ldf, R, ldr, st, nact, stw, parts, nparts, s); break;
        case 8: rows_dispatch<8>(A, m, N, U, ldu, F, ldf, R, ldr, st, nact, stw, parts, nparts, s); break;
        default: fail(TVCS_EINVAL, "gemv_rows: nv must be 1, 2, 4 or 8");
    }
}

void launch_gemv_cols(const float *A, int m, int N, const float *R, int ldr, float *P,
                      long long chunk_stride, int nv, const ImgState *st, int nact,
                      hipStream_t s) {
    switch (nv) {
        case 1: cols_dispatch<1>(A, m, N, R, ldr, P, chunk_stride, st, nact, s); break;
        case 2: cols_dispatch<2>(A, m, N, R, ldr, P, chunk_stride, st, nact, s); break;
        case 4: cols_dispatch<4>(A, m, N, R, ldr, P, chunk_stride, st, nact, s); break;
        case 8: cols_dispatch<8>(A, m, N, R, ldr, P, chunk_stride, st, nact, s); break;
        default: fail(TVCS_EINVAL, "gemv_cols: nv must be 1, 2, 4 or 8");
    }
}

int fused_bands(int m, int N) {
    if (N > kFusedN || (N & 3)) return 0;
    const int rpb = (m + kFusedMaxBands - 1) / kFusedMaxBands;
    return (m + rpb - 1) / rpb;
}

template <int G>
void fused_dispatch(const float *A, int m, int N, int rpb, int nb, int T, const float *U,
                    const float *F, float *P, const ImgState *st, int rev, float *R,
                    hipStream_t s) {
    if ((size_t)m * N * sizeof(float) > TVCS_GEMV_NT_BYTES)
        hipLaunchKernelGGL((k_gemv_fused<G, true>), dim3(nb), dim3(T), 0, s, A, m, N, rpb, U, F,
                           P, st, rev, R);
    else
        hipLaunchKernelGGL((k_gemv_fused<G, false>), dim3(nb), dim3(T), 0, s, A, m, N, rpb, U, F,
                           P, st, rev, R);
}

void launch_gemv_fused(const float *A, int m, int N, const float *U, const float *F, float *P,
                       float *g_out, const ImgState *st, int rev, hipStream_t s, ImgState *stw,
                       const double *parts, int nparts, float *r_out, const BBNorms *norms) {
    const int nb = fused_bands(m, N);
    if (nb < 1) fail(TVCS_EINVAL, "gemv_fused: n^2 must be a multiple of 4 and at most 16384");
    if (stw && (st != stw || !parts || nparts < 1 || !g_out))
        fail(TVCS_EINVAL, "gemv_fused: the folded stop rule needs the image state, its partials "
                          "and the partial-sum pass");
    if (norms && (!g_out || !r_out || norms->P != U || norms->AP != r_out || norms->n * norms->n != N ||
                  norms->m != m))
        fail(TVCS_EINVAL, "gemv_fused: the BB norms are those of U and r_out, with the partial-sum "
                          "pass");
    const int rpb = (m + nb - 1) / nb;
    // G float4 groups per thread, T threads (a multiple of 64, at most 1024)
    const int N4 = N / 4;
    const int G = (N4 + kFusedThreadsMax - 1) / kFusedThreadsMax;
    const int T = ((N4 + G - 1) / G + 63) / 64 * 64;
    switch (G) {
        case 1: fused_dispatch<1>(A, m, N, rpb, nb, T, U, F, P, st, rev, r_out, s); break;
        case 2: fused_dispatch<2>(A, m, N, rpb, nb, T, U, F, P, st, rev, r_out, s); break;
        case 3: fused_dispatch<3>(A, m, N, rpb, nb, T, U, F, P, st, rev, r_out, s); break;
        default: fused_dispatch<4>(A, m, N, rpb, nb, T, U, F, P, st, rev, r_out, s);
    }
    if (g_out) launch_sum_bands(P, nb, N, g_out, st, s, stw, parts, nparts, norms);
}

void launch_sum_bands(const float *P, int nb, int N, float *g_out, const ImgState *st,
                      hipStream_t s, ImgState *stw, const double *parts, int nparts,
                      const BBNorms *norms) {
    if (nb < 1 || nb > kFusedMaxBands) fail(TVCS_EINVAL, "sum_bands: 1 to 256 band partials");
    const int nsum = (N / 4 + kSumCols4 - 1) / kSumCols4;
    const BBNorms nm = norms ? *norms : BBNorms{};
    hipLaunchKernelGGL(k_sum_bands, dim3(nsum + (stw ? 1 : 0) + (norms ? nm.nblk : 0)), dim3(256),
                       0, s, P, nb, N, g_out, st, stw, parts, nparts, nm);
}

}  // namespace tvcs
