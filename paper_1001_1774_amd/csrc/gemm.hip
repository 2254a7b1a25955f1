// A u and A^T r on MFMA for low-precision storage of A, shared by a batch of
// images (the two products of every iteration, g_k = A^T (A u^k - f), eq. (line)).
//
// Storage (built once per A by lowp_convert):
//   BF16        X_hi = bf16(A)                      (m_p x N)  and  XT_hi = X_hi^T (N x m_p)
//   BF16_SPLIT  X_hi = bf16(A), X_lo = bf16(A - X_hi), and both transposes
//   FP8         Q = E4M3(A_ij / s_i), s_i = max_j |A_ij| / 448 (FP32), and Q^T
// Both orientations are stored so that each product is a GEMM whose operands are
// contiguous along the reduction dimension; the HBM bytes per product are the same
// as for one copy (each product streams one copy once).  m_p = m and N_p = n^2
// rounded up to 256 (zero rows of A, and zero columns for sides whose n^2 is not a
// multiple of 256, e.g. 450; the forward product's batch operand is zero there and
// the adjoint does not store those rows).  Both copies are stored in MFMA fragment order: the 16 x 32
// block (rows 16 t .. +15, k 32 u .. +31) is 512 contiguous elements laid out as
// the A operand of v_mfma_f32_16x16x32_bf16 expects them (lane l holds row l % 16,
// k 8 (l / 16) .. +7), blocks ordered row-tile major.  A wave's operand load is then
// one contiguous 1 KiB read (512 B for fp8) instead of 16 rows x 64 B, and a wave
// streams each of its row tiles sequentially.
//
// GEMM: C[b][row] = sum_k X[row][k] Y[b][k] with X the streamed matrix (A or A^T)
// and Y the small batch operand.  A bf16-only copy of U (or R) would add fresh
// relative noise of ~2^-9 to every product in every iteration, which puts a floor
// under the relative change of the iterates and keeps the stop rule (eq. (stop))
// from firing.  Each image's products therefore take one of two forms, chosen per
// iteration by ImgState::mode:
//   fresh      Y = Y_hi + Y_lo, Y_hi = bf16(v), Y_lo = bf16(v - Y_hi) of v = u (or
//              s o r): r = A Y - f and g = A^T Y from scratch, carrying only the
//              fixed rounding of A's storage plus at most 2^-16 of v;
//   increment  Y = bf16(v - v~), one part, where v~ is the vector the current r (g)
//              was computed from: r += A Y, v~ += Y (and g += A^T Y).  What the
//              rounding drops stays in v - v~ and is applied by the next
//              increment, so it does not accumulate; it is at most 2^-8 of the
//              change since the last product, which vanishes as the iterates
//              converge.
// Fresh products run while an image's relative change exceeds 2^-8 and every 64th
// iteration (FP32 sums of increments add rounding relative to the sizes of the
// increments, which are large early on).  A group of images runs the Y_lo MFMAs
// only if one of its active images is fresh; an image in increment mode then has
// Y_lo = 0, whose MFMA adds exact zeros, so its bits do not depend on the group.
// Y is written in the same fragment order as X
// (16 images x 32 k per 1 KiB block).  A workgroup (4 waves) owns 4*RT*16
// consecutive rows of X and all 16*NT images of its group; each wave streams its
// RT 16-row tiles of X straight from HBM into registers (every X element is used
// by exactly one wave, so it never goes through LDS), while the workgroup stages
// the Y blocks of each step in LDS (double-buffered, moved through registers).
// The loop is software-pipelined: X of step t + 1 and Y of step t + 2 are in
// flight while step t runs v_mfma_f32_16x16x32_bf16 with FP32 accumulation:
// X Y_hi, plus X_lo Y_hi for split storage (X_lo Y_lo, at most 2^-16 of the product,
// is left out), plus X Y_lo for fresh products.  FP8 X is widened to bf16 in registers (exact); the row
// scale folds into vectors: (A u)_i = s_i sum_j q_ij u_j and
// (A^T r)_j = sum_i q_ij (s_i r_i).
// The forward product splits its reduction (length N) into KS slices whose FP32
// partial results are added in a fixed order by k_reduce_r; workgroups are
// ordered so that each XCD works on one K slice and its Y slice stays in that
// XCD's L2.  No order of summation depends on the batch, the image group or the
// tile shape, so an image's products are the same bits in any batch.
#include "device_stop.h"
#include "tvcs_internal.h"

#include <algorithm>

// Tile shapes are chosen at run time per product and batch (lowp_autotune) among
// rt in {2, 4} row tiles per wave, image groups of 16 nt images (nt <= 16; 256-image
// groups with 2 row tiles per wave only) and two tables of k tiles per pipeline step
// (kKF below).
#ifndef TVCS_Y_KMAJOR
#define TVCS_Y_KMAJOR 1        // batch operand blocks k-tile major, hi/lo interleaved
#endif
#ifndef TVCS_X_GROUP
#define TVCS_X_GROUP 16        // row tiles per group in the fragment order of A and A^T
#endif
// X prefetch distance (steps in flight ahead of the one computed) of tiles with 2 row
// tiles per wave and 1 k tile per step, per storage format (a step is 1 KiB of FP8
// per wave, 4 VGPRs a register set; 2 KiB of bf16, 8 VGPRs; 4 KiB of split bf16).
// Tiles with 4 row tiles per wave, or several k tiles per step, take distance 1:
// their accumulators leave no room for more register sets at 2 waves per SIMD.
#ifndef TVCS_GEMM_DEPTH_FP8
#define TVCS_GEMM_DEPTH_FP8 3
#endif
#ifndef TVCS_GEMM_DEPTH_BF16
#define TVCS_GEMM_DEPTH_BF16 2
#endif
#ifndef TVCS_GEMM_DEPTH_SPLIT
#define TVCS_GEMM_DEPTH_SPLIT 1
#endif
// ... and of FP8 tiles with 4 row tiles per wave (a register set is 8 VGPRs)
#ifndef TVCS_GEMM_DEPTH_FP8_RT4
#define TVCS_GEMM_DEPTH_FP8_RT4 3
#endif
#ifndef TVCS_FWD_TARGET_WG
#define TVCS_FWD_TARGET_WG 256 // K slices of the forward product grow until this many tiles
#endif
#ifndef TVCS_ADJ_SPLIT
#define TVCS_ADJ_SPLIT 2       // K slices of the adjoint product (partial sums added later)
#endif

namespace tvcs {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;
typedef unsigned char u8;
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
// Row tiles per group of the streamed matrix's fragment order: the blocks of a
// group's kXGroup row tiles for one k tile are adjacent, so one workgroup step
// (up to 16 row tiles x KF k tiles) reads one contiguous span of HBM.
constexpr int kXGroup = TVCS_X_GROUP;
// Batch operand order: k-tile major with hi and lo blocks interleaved (one step's
// Y blocks of a workgroup are then adjacent), or image-tile major in two arrays.
constexpr bool kYKMajor = TVCS_Y_KMAJOR != 0;
static_assert(kMPad % (16 * kXGroup) == 0 && 16 * kXGroup <= 256,
              "row counts (m_p, and N_p) must be whole groups");
constexpr int KMAX = 128;        // longest reduction step; every K slice is a multiple of it
// 32-wide k tiles per pipeline step by image tiles per group (1, 2, 4, 8, 16), two
// tables.  With one part of the batch operand a step moves NT * KF Y blocks over the
// four waves, so NT * KF is a multiple of 4.  Table 0 holds the measured defaults
// (longer steps for small groups, whose X stream dominates; one k tile for large
// groups, whose accumulators fill the registers), table 1 the neighbours.
constexpr int kKF[2][5] = {{4, 4, 4, 1, 1}, {4, 2, 1, 2, 1}};
constexpr int log2_nt(int nt) { return nt == 1 ? 0 : nt == 2 ? 1 : nt == 4 ? 2 : nt == 8 ? 3 : 4; }
constexpr int kRowsRT4 = 4 * 4 * 16;   // rows per workgroup with 4 row tiles per wave

enum { M_BF16 = 0, M_SPLIT = 1, M_FP8 = 2 };

int mode_of(int storage) {
    switch (storage) {
        case TVCS_A_BF16: return M_BF16;
        case TVCS_A_BF16_SPLIT: return M_SPLIT;
        case TVCS_A_FP8_ROWSCALE: return M_FP8;
    }
    fail(TVCS_EINVAL, "not a low-precision storage format");
}

__device__ inline u16 bf16_rne(float x) {   // finite inputs
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
__device__ inline float bf16_f32(u16 h) { return __uint_as_float((unsigned)h << 16); }

__device__ inline bool any_active(const ImgState *st, int nact) {
    if (st == nullptr) return true;
    int a = 0;
    for (int i = 0; i < nact; ++i) a |= st[i].active;
    return a != 0;
}

// the products of image b this iteration are fresh (parity < 0: outside the loop;
// b >= B: padding images, whose operands are zero)
__device__ inline bool fresh_of(const ImgState *st, int b, int B, int parity) {
    return parity < 0 || st == nullptr || b >= B || st[b].mode[parity] != 0;
}

// some active image of the group takes fresh products (two-part batch operand)
__device__ inline bool any_fresh(const ImgState *st, int nact, int parity) {
    if (st == nullptr || parity < 0) return true;
    int a = 0;
    for (int i = 0; i < nact; ++i) a |= st[i].active & st[i].mode[parity];
    return a != 0;
}

// 8 E4M3 codes -> 8 bf16 (every E4M3 value is exact in bf16): the packed conversion
// with scale 1, two codes per instruction
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ inline bf16x8 fp8x8_to_bf16(u32x2 q) {
    const bf16x2 a = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8((int)q.x, 1.0f, false);
    const bf16x2 b = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8((int)q.x, 1.0f, true);
    const bf16x2 c = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8((int)q.y, 1.0f, false);
    const bf16x2 d = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8((int)q.y, 1.0f, true);
    return bf16x8{a[0], a[1], b[0], b[1], c[0], c[1], d[0], d[1]};
}

// X fragments of one reduction step held in registers (FP8 stays packed until use)
template <int MODE, int RT, int KF>
struct XRegs {
    bf16x8 h[RT][KF];
    bf16x8 l[MODE == M_SPLIT ? RT : 1][MODE == M_SPLIT ? KF : 1];
};
template <int RT, int KF>
struct XRegs<M_FP8, RT, KF> {
    u32x2 q[RT][KF];
};

template <int MODE, int RT, int KF>
__device__ inline void load_x(XRegs<MODE, RT, KF> &x, const void *Xhi, const void *Xlo,
                              const long long (&xoff)[RT], int kt0) {
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
        for (int s = 0; s < KF; ++s) {
            const long long o = xoff[rt] + (long long)(kt0 + s) * (kXGroup * 512);
            if constexpr (MODE == M_FP8) {
                x.q[rt][s] = __builtin_nontemporal_load(
                    reinterpret_cast<const u32x2 *>((const u8 *)Xhi + o));
            } else {
                x.h[rt][s] = __builtin_nontemporal_load(
                    reinterpret_cast<const bf16x8 *>((const u16 *)Xhi + o));
                if constexpr (MODE == M_SPLIT)
                    x.l[rt][s] = __builtin_nontemporal_load(
                        reinterpret_cast<const bf16x8 *>((const u16 *)Xlo + o));
            }
        }
}

// Y (the batch operand) is stored in the same fragment order as X: image tile t
// (16 images), k tile u (32) is the 512-element block (t * ktiles + u), so the Y
// fragments of one step are whole 1 KiB blocks.  Per step the workgroup needs
// PARTS (hi, and lo for fresh products) x NT x KF blocks; wave w moves blocks w,
// w + 4, ... through registers into LDS, where every fragment read is one
// contiguous 1 KiB (no bank conflicts).
template <int MODE, int RT, int NT, int KF, int PARTS>
__device__ inline void gemm_body(const void *__restrict__ Xhi, const void *__restrict__ Xlo,
                                 long long xkt, const u16 *__restrict__ Yhi,
                                 const u16 *__restrict__ Ylo, long long yimg, long long ytile,
                                 int M, int mstore, int kspan, int ks, int rb,
                                 float *__restrict__ out, long long split_stride, long long ldo,
                                 u16 (*ys)[2 * NT * KF][512]) {
    constexpr int NB = NT * KF;           // Y blocks per step and part
    constexpr int YPW = PARTS * NB / 4;   // Y blocks moved per wave and step
    static_assert(PARTS * NB % 4 == 0, "the four waves share the Y blocks evenly");

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int row_wave = rb * (4 * RT * 16) + wave * RT * 16;
    const int kt_begin = (ks * kspan) >> 5;
    // the last K slice may be shorter (slices are multiples of 4 k tiles, so of KF)
    const int steps = min(kspan, (int)(xkt << 5) - ks * kspan) / (32 * KF);

    f32x4 acc[RT][NT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    long long xoff[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
    {
        const int tile = min((row_wave >> 4) + rt, (M >> 4) - 1);
        xoff[rt] = (((long long)(tile / kXGroup) * xkt) * kXGroup + tile % kXGroup) * 512 + lane * 8;
    }

    // this wave's Y blocks: j = wave + 4 q -> part j / NB, image tile (j % NB) / KF, k tile j % KF
    const u16 *ysrc[YPW];
#pragma unroll
    for (int q = 0; q < YPW; ++q) {
        const int j = wave + 4 * q, part = j / NB, r = j % NB;
        ysrc[q] = (part ? Ylo : Yhi) + (long long)(r / KF) * yimg +
                  (long long)(kt_begin + r % KF) * ytile + lane * 8;
    }
    // two register sets for Y with one k tile per step: the set filled in stage t - 1
    // is stored to LDS in stage t while stage t's own Y load is already in flight
    // (steps of several k tiles, 256-image groups and split storage keep one set:
    // the second would leave too few registers for two waves per SIMD)
    constexpr int YS = (KF == 1 && NT <= 8 && MODE != M_SPLIT) ? 2 : 1;
    u32x4 yr[YS][YPW];
    auto load_y = [&](int set, int t) {
#pragma unroll
        for (int q = 0; q < YPW; ++q)
            yr[set][q] = *reinterpret_cast<const u32x4 *>(ysrc[q] + (long long)t * KF * ytile);
    };
    auto store_y = [&](int set, int buf) {
#pragma unroll
        for (int q = 0; q < YPW; ++q)
            *reinterpret_cast<u32x4 *>(&ys[buf][wave + 4 * q][lane * 8]) = yr[set][q];
    };
    // One step: per k tile, the Y fragments of YC image tiles at a time are read from
    // LDS before their MFMAs (one LDS round trip waited for per chunk, not per image
    // tile).  Every accumulator sees X Y_hi, then X_lo Y_hi (split storage), then
    // X Y_lo (fresh products), in this order whatever the path.
    constexpr int YC = MODE == M_SPLIT ? (NT < 4 ? NT : 4) : (NT < 8 ? NT : 8);
    static_assert(NT % YC == 0, "whole chunks of image tiles");
    auto compute = [&](const XRegs<MODE, RT, KF> &x, int buf) {
#pragma unroll
        for (int s = 0; s < KF; ++s) {
            bf16x8 xc[RT];
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) {
                if constexpr (MODE == M_FP8)
                    xc[rt] = fp8x8_to_bf16(x.q[rt][s]);
                else
                    xc[rt] = x.h[rt][s];
            }
#pragma unroll
            for (int p = 0; p < PARTS; ++p)
#pragma unroll
                for (int c0 = 0; c0 < NT; c0 += YC) {
                    bf16x8 y[YC];
#pragma unroll
                    for (int c = 0; c < YC; ++c)
                        y[c] = *reinterpret_cast<const bf16x8 *>(
                            &ys[buf][p * NB + (c0 + c) * KF + s][lane * 8]);
                    // the RT accumulators of an image tile are updated in turn, so RT - 1
                    // independent MFMAs separate two that share an accumulator
#pragma unroll
                    for (int c = 0; c < YC; ++c)
#pragma unroll
                        for (int rt = 0; rt < RT; ++rt)
                            acc[rt][c0 + c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                xc[rt], y[c], acc[rt][c0 + c], 0, 0, 0);
                    if constexpr (MODE == M_SPLIT) {
                        if (p == 0) {
#pragma unroll
                            for (int c = 0; c < YC; ++c)
#pragma unroll
                                for (int rt = 0; rt < RT; ++rt)
                                    acc[rt][c0 + c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                        x.l[rt][s], y[c], acc[rt][c0 + c], 0, 0, 0);
                        }
                    }
                }
        }
    };

    // Software pipeline: the X fragments of steps t + 1 .. t + D and the Y blocks of
    // steps t + 1 and t + 2 are in flight while step t computes (Y is double-buffered
    // in LDS: step t reads buffer t & 1).  Each stage issues its Y load before its X
    // load: memory waits retire in issue order, so storing Y(t + 1), loaded a stage
    // earlier, then waits for nothing issued after it, and the X loads keep their
    // full distance.  X rotates through D + 1 register sets and Y through 2, and the
    // loop is unrolled by D + 1 (even, or doubled) so that every set index is a
    // constant (the accumulators never change registers).  Loads past the last step
    // re-read the last step (in bounds, results unused), which keeps the body
    // branch-free; scheduling barriers keep the compiler from reordering the loads.
    constexpr int D = KF > 1 ? 1
                    : RT > 2 ? (MODE == M_FP8 ? TVCS_GEMM_DEPTH_FP8_RT4 : 1)
                    : MODE == M_FP8 ? TVCS_GEMM_DEPTH_FP8
                    : MODE == M_SPLIT ? TVCS_GEMM_DEPTH_SPLIT : TVCS_GEMM_DEPTH_BF16;
    static_assert(D >= 1 && D <= 8, "prefetch distance 1 .. 8");
    constexpr int U = (D + 1) % 2 == 0 ? D + 1 : 2 * (D + 1);   // unroll: both rotations close
    const int last = steps - 1;
    XRegs<MODE, RT, KF> x[D + 1];
    // step t (= j mod the unroll) from X set j % (D + 1); step t + D is loaded into the
    // set step t - 1 used; Y(t + 2) into Y set t & 1, whose Y(t) went to LDS in stage t - 1
    auto stage = [&](int j, int t) {
        if constexpr (YS == 2) {
            load_y(j & 1, min(t + 2, last));
            load_x(x[(j + D) % (D + 1)], Xhi, Xlo, xoff, kt_begin + min(t + D, last) * KF);
            __builtin_amdgcn_sched_barrier(0);
            compute(x[j % (D + 1)], t & 1);
            store_y((j + 1) & 1, (t + 1) & 1);   // Y(t + 1), loaded in stage t - 1
        } else {
            load_x(x[(j + D) % (D + 1)], Xhi, Xlo, xoff, kt_begin + min(t + D, last) * KF);
            __builtin_amdgcn_sched_barrier(0);
            compute(x[j % (D + 1)], t & 1);
            store_y(0, (t + 1) & 1);
            load_y(0, min(t + 2, last));
        }
        __syncthreads();
    };
    load_y(0, 0);
    store_y(0, 0);
    load_y(YS - 1, min(1, last));
#pragma unroll
    for (int j = 0; j < D; ++j) load_x(x[j], Xhi, Xlo, xoff, kt_begin + min(j, last) * KF);
    __syncthreads();
    int t = 0;
    for (; t + U <= steps; t += U) {
#pragma unroll
        for (int j = 0; j < U; ++j) stage(j, t + j);
    }
#pragma unroll
    for (int j = 0; j < U - 1; ++j)
        if (t + j < steps) stage(j, t + j);
    // lane holds rows 4*(lane/16) .. +3 of its 16-row tile, image lane % 16 of its tile
    float *o = out + ks * split_stride;
    const int lr = lane & 15;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int row = row_wave + rt * 16 + 4 * (lane >> 4);
        if (row >= mstore) continue;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int img = nt * 16 + lr;
            *reinterpret_cast<f32x4 *>(o + img * ldo + row) = acc[rt][nt];
        }
    }
}

// One launch: the group's images are nact states at st (null: all active, fresh);
// parity selects each image's mode (< 0: fresh).  The whole workgroup takes the
// two-part path if any active image of the group is fresh.
template <int MODE, int RT, int NT, int KF>
__global__ __launch_bounds__(kThreads) void k_gemm(
    const void *__restrict__ Xhi, const void *__restrict__ Xlo, long long xkt,
    const u16 *__restrict__ Yhi, const u16 *__restrict__ Ylo, long long yimg, long long ytile,
    int M, int mstore, int kspan,
    int RB, int KS, float *__restrict__ out, long long split_stride, long long ldo,
    const ImgState *__restrict__ st, int nact, int parity) {
    if (!any_active(st, nact)) return;
    // XCD-aware order: consecutive tiles (same K slice, neighbouring rows) on one XCD
    const int total = RB * KS;
    const int nloc = (total + 7) / 8;
    const int L = (blockIdx.x & 7) * nloc + (blockIdx.x >> 3);
    if (L >= total) return;
    const int ks = L / RB, rb = L % RB;
    __shared__ __attribute__((aligned(16))) u16 ys[2][2 * NT * KF][512];
    if (any_fresh(st, nact, parity))
        gemm_body<MODE, RT, NT, KF, 2>(Xhi, Xlo, xkt, Yhi, Ylo, yimg, ytile, M, mstore, kspan, ks,
                                       rb, out, split_stride, ldo, ys);
    else
        gemm_body<MODE, RT, NT, KF, 1>(Xhi, Xlo, xkt, Yhi, Ylo, yimg, ytile, M, mstore, kspan, ks,
                                       rb, out, split_stride, ldo, ys);
}

// ---- conversions ---------------------------------------------------------------
// per-row scale of the fp8 format: s_i = max_j |A_ij| / 448 (1 for empty rows)
__global__ __launch_bounds__(256) void k_fp8_scale(const float *__restrict__ A, int m, int N,
                                                  float *__restrict__ scale) {
    const int i = blockIdx.x;
    if (i >= m) {
        if (threadIdx.x == 0) scale[i] = 1.f;
        return;
    }
    const float *a = A + (size_t)i * N;
    float mx = 0.f;
    for (int j = threadIdx.x; j < N; j += 256) mx = fmaxf(mx, fabsf(a[j]));
    __shared__ float red[256];
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float s = red[0] / 448.0f;
        scale[i] = s > 0.f ? s : 1.f;
    }
}

__device__ inline unsigned fp8_pack4(float a, float b, float c, float d) {
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false);   // bytes 0, 1
    return (unsigned)__builtin_amdgcn_cvt_pk_fp8_f32(c, d, w, true);   // bytes 2, 3
}

// Fragment-ordered copy of A (TRANS = false: rows i < m_p, reduction over columns;
// TRANS = true: rows j < N of A^T, reduction over i < m_p).  Each thread writes one
// lane's 8 consecutive elements of a block; rows i >= m are zero.
template <int MODE, bool TRANS>
__global__ void k_frag(const float *__restrict__ A, int m, int N, int Np, int mp,
                       const float *__restrict__ scale, void *__restrict__ hi,
                       void *__restrict__ lo) {
    const size_t R = TRANS ? (size_t)Np : (size_t)mp, K = TRANS ? (size_t)mp : (size_t)Np;
    const size_t chunks = R * K / 8, ktiles = K / 32;
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < chunks;
         c += (size_t)gridDim.x * blockDim.x) {
        const size_t f = c >> 6;
        const int lane = (int)(c & 63);
        // block f = ((t / G) * ktiles + u) * G + t % G for row tile t, k tile u
        const size_t g = f / (ktiles * kXGroup), rem = f % (ktiles * kXGroup);
        const size_t t = g * kXGroup + rem % kXGroup, u = rem / kXGroup;
        const size_t r = t * 16 + (lane & 15), k0 = u * 32 + 8 * (lane >> 4);
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const size_t i = TRANS ? k0 + j : r, col = TRANS ? r : k0 + j;   // A[i][col]
            v[j] = (i < (size_t)m && col < (size_t)N) ? A[i * N + col] : 0.f;
            if (MODE == M_FP8) v[j] = fminf(fmaxf(v[j] / scale[i], -448.f), 448.f);
        }
        if (MODE == M_FP8) {
            const unsigned w0 = fp8_pack4(v[0], v[1], v[2], v[3]), w1 = fp8_pack4(v[4], v[5], v[6], v[7]);
            reinterpret_cast<u32x2 *>(hi)[c] = u32x2{w0, w1};
        } else {
            u16 h[8], l[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                h[j] = bf16_rne(v[j]);
                l[j] = bf16_rne(v[j] - bf16_f32(h[j]));   // exact in FP32
            }
            reinterpret_cast<uint4 *>(hi)[c] = *reinterpret_cast<const uint4 *>(h);
            if (MODE == M_SPLIT) reinterpret_cast<uint4 *>(lo)[c] = *reinterpret_cast<const uint4 *>(l);
        }
    }
}

// Batch operand Y of a product, in fragment order, from V (Bp rows of length kv,
// FP32; columns kv .. K-1 are zero), each column optionally multiplied by scale[k]
// first (FP64 product, FP32 result: v = s o r for the FP8 adjoint).  Per image b:
//   fresh (fresh_of): hi = bf16(v), lo = bf16(v - hi); Vt = hi + lo (exact in FP32)
//   increment:        hi = bf16(v - Vt), lo = 0;        Vt += hi
// where Vt (Bp x kv, may be null outside the loop) is the vector the product
// results belong to.  Block (image tile t, k tile u) of part p sits at
// (p ? lo : hi) + t * yimg + u * ytile; lane l of a block holds image 16 t + l % 16,
// columns 32 u + 8 (l / 16) .. +7.
// A workgroup takes one image tile and 128 columns (4 k tiles): thread i handles
// image 16 t + i / 16, columns 8 (i % 16) .. +7, so 16 threads read 512 contiguous
// bytes of one image (16-byte loads when rows are 16-byte aligned), and each block
// the workgroup writes is written whole by it.
// stw (the forward product's split of U): the workgroups also apply the previous
// iteration's stop rule to images < B first, one image per workgroup in turn (the
// products read the flags after this pass; the rule writes mode[parity ^ 1], which
// this iteration does not read).
__global__ __launch_bounds__(256) void k_split_frag(
    const float *__restrict__ V, int kv, int K, int Bp, const float *__restrict__ scale,
    u16 *__restrict__ hi, u16 *__restrict__ lo, long long yimg, long long ytile, ImgState *stw,
    const double *parts, int nparts, int B, float *__restrict__ Vt, const ImgState *mst,
    int parity) {
    const int bid = blockIdx.y * gridDim.x + blockIdx.x, nblk = gridDim.x * gridDim.y;
    if (stw && threadIdx.x < 64)
        for (int b = bid; b < B; b += nblk)
            if (stw[b].active)
                stop_rule(stw + b, parts + (size_t)b * nparts * 2, nparts, nullptr,
                          parity >= 0 ? parity ^ 1 : -1);
    const int it = blockIdx.y, i = threadIdx.x;
    const int b = it * 16 + (i >> 4);
    const int k0 = blockIdx.x * 128 + 8 * (i & 15);
    const bool fresh = fresh_of(mst, b, B, parity);
    const size_t row = (size_t)b * kv;
    float x[8], base[8];
    if ((kv & 3) == 0 && k0 + 8 <= kv) {   // whole aligned chunk: 16-byte loads
        const float4 a0 = *reinterpret_cast<const float4 *>(V + row + k0);
        const float4 a1 = *reinterpret_cast<const float4 *>(V + row + k0 + 4);
        x[0] = a0.x; x[1] = a0.y; x[2] = a0.z; x[3] = a0.w;
        x[4] = a1.x; x[5] = a1.y; x[6] = a1.z; x[7] = a1.w;
        if (scale) {
            const float4 s0 = *reinterpret_cast<const float4 *>(scale + k0);
            const float4 s1 = *reinterpret_cast<const float4 *>(scale + k0 + 4);
            const float sc[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
#pragma unroll
            for (int j = 0; j < 8; ++j) x[j] = (float)((double)x[j] * (double)sc[j]);
        }
        if (!fresh) {
            const float4 t0 = *reinterpret_cast<const float4 *>(Vt + row + k0);
            const float4 t1 = *reinterpret_cast<const float4 *>(Vt + row + k0 + 4);
            base[0] = t0.x; base[1] = t0.y; base[2] = t0.z; base[3] = t0.w;
            base[4] = t1.x; base[5] = t1.y; base[6] = t1.z; base[7] = t1.w;
        }
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = k0 + j;
            x[j] = 0.f;
            base[j] = 0.f;
            if (k < kv) {
                x[j] = V[row + k];
                if (scale) x[j] = (float)((double)x[j] * (double)scale[k]);
                if (!fresh) base[j] = Vt[row + k];
            }
        }
    }
    u16 h[8], w[8];
    float nt[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (fresh) {
            h[j] = bf16_rne(x[j]);
            w[j] = bf16_rne(x[j] - bf16_f32(h[j]));          // exact in FP32
            nt[j] = bf16_f32(h[j]) + bf16_f32(w[j]);         // exact
        } else {
            h[j] = bf16_rne(x[j] - base[j]);
            w[j] = 0;
            nt[j] = base[j] + bf16_f32(h[j]);
        }
    }
    if (Vt) {
        if ((kv & 3) == 0 && k0 + 8 <= kv) {
            *reinterpret_cast<float4 *>(Vt + row + k0) = make_float4(nt[0], nt[1], nt[2], nt[3]);
            *reinterpret_cast<float4 *>(Vt + row + k0 + 4) = make_float4(nt[4], nt[5], nt[6], nt[7]);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (k0 + j < kv) Vt[row + k0 + j] = nt[j];
        }
    }
    const int u = k0 >> 5, l = (i >> 4) + 16 * ((k0 >> 3) & 3);
    const size_t o = (size_t)it * yimg + (size_t)u * ytile + (size_t)l * 8;
    *reinterpret_cast<uint4 *>(hi + o) = *reinterpret_cast<const uint4 *>(h);
    *reinterpret_cast<uint4 *>(lo + o) = *reinterpret_cast<const uint4 *>(w);
}

// R[b][i] = s_i * sum_ks P[ks][b][i] - F[b][i] for fresh products, or
// R[b][i] + s_i * sum_ks P[ks][b][i] for increments (FP64 sum, fixed order), i < m
__global__ void k_reduce_r(const float *__restrict__ P, int KS, long long split_stride, int mp,
                           const float *__restrict__ F, const float *__restrict__ scale, int m,
                           float *__restrict__ R, const ImgState *__restrict__ mst, int parity,
                           int B) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= m) return;
    double acc = 0.0;
    for (int k = 0; k < KS; ++k) acc += (double)P[k * split_stride + (size_t)b * mp + i];
    if (scale) acc *= (double)scale[i];
    float *r = R + (size_t)b * m + i;
    if (fresh_of(mst, b, B, parity)) {
        if (F) acc -= (double)F[(size_t)b * m + i];
    } else {
        acc += (double)*r;
    }
    *r = (float)acc;
}

// Arguments of one product launch (k_gemm's parameters)
struct GemmArgs {
    const void *Xhi, *Xlo;
    long long ldx;
    const u16 *Yhi, *Ylo;
    long long yimg, ytile;
    int M, mstore, kspan, RB, KS;   // rows of X (whole groups), rows written, ...
    float *out;
    long long split_stride, ldo;
    const ImgState *st;
    int nact, parity;
};

template <int MODE, int RT, int NT, int KF>
void launch_gemm(const GemmArgs &a, hipStream_t s) {
    const int total = a.RB * a.KS;
    hipLaunchKernelGGL((k_gemm<MODE, RT, NT, KF>), dim3(((total + 7) / 8) * 8), dim3(kThreads), 0, s,
                       a.Xhi, a.Xlo, a.ldx >> 5, a.Yhi, a.Ylo, a.yimg, a.ytile, a.M, a.mstore,
                       a.kspan, a.RB, a.KS, a.out, a.split_stride, a.ldo, a.st, a.nact, a.parity);
}

template <int MODE, int RT, int NT>
void launch_nt(int kfv, const GemmArgs &a, hipStream_t s) {
    constexpr int K0 = kKF[0][log2_nt(NT)], K1 = kKF[1][log2_nt(NT)];
    if (kfv == 0 || K0 == K1)
        launch_gemm<MODE, RT, NT, K0>(a, s);
    else
        launch_gemm<MODE, RT, NT, K1>(a, s);
}

template <int MODE, int RT>
void gemm_dispatch(int NT, int kfv, const GemmArgs &a, hipStream_t s) {
    switch (NT) {
        case 1: launch_nt<MODE, RT, 1>(kfv, a, s); break;
        case 2: launch_nt<MODE, RT, 2>(kfv, a, s); break;
        case 4: launch_nt<MODE, RT, 4>(kfv, a, s); break;
        case 8: launch_nt<MODE, RT, 8>(kfv, a, s); break;
        case 16:   // 2 row tiles per wave only (the accumulators of 4 do not fit)
            if constexpr (RT == 2) {
                launch_nt<MODE, 2, 16>(kfv, a, s);
                break;
            }
            fail(TVCS_EUNSUPPORTED, "MFMA product: 256-image groups take 2 row tiles per wave");
        default: fail(TVCS_EUNSUPPORTED, "MFMA product: image groups of 16, 32, 64, 128 or 256");
    }
}

// one image group of nt tiles with the tile shape c (c.nt is the largest group size)
void gemm_any(const TileCfg &c, int mode, int NT, GemmArgs a, hipStream_t s) {
    const int RT = NT == 16 ? 2 : c.rt;
    a.RB = (a.M + 4 * RT * 16 - 1) / (4 * RT * 16);
    switch (mode * 2 + (RT == 4)) {
        case M_BF16 * 2: gemm_dispatch<M_BF16, 2>(NT, c.kfv, a, s); break;
        case M_BF16 * 2 + 1: gemm_dispatch<M_BF16, 4>(NT, c.kfv, a, s); break;
        case M_SPLIT * 2: gemm_dispatch<M_SPLIT, 2>(NT, c.kfv, a, s); break;
        case M_SPLIT * 2 + 1: gemm_dispatch<M_SPLIT, 4>(NT, c.kfv, a, s); break;
        case M_FP8 * 2: gemm_dispatch<M_FP8, 2>(NT, c.kfv, a, s); break;
        default: gemm_dispatch<M_FP8, 4>(NT, c.kfv, a, s);
    }
}

size_t elem_bytes(int mode) { return mode == M_FP8 ? 1 : 2; }

// K slices of the forward product.  Depends on (m, N) only, so the order of every
// sum, and with it each image's result, is the same for every batch size and tile
// choice.  The RB x KS tiles of a launch run in rounds of 256 (one per CU; two per
// CU with twice the tiles at 2 row tiles per wave), and a tile's time is about its
// slice length plus a fixed cost (pipeline fill, partial results) of ~2 quanta of
// KMAX: the slice count is the smallest of 1 .. 64 (slices of at least 4 quanta)
// whose rounds x (length + 2) is within 3 % of the best.  At n = 256, m = 13107
// (RB = 52): 9 slices of 57 quanta in 2 nearly full rounds of 468 tiles, where 8
// leave 96 CUs idle in the second round.  The last slice may be shorter.
// TVCS_FWD_BALANCE 0: powers of two until RB x KS >= TVCS_FWD_TARGET_WG.
#ifndef TVCS_FWD_BALANCE
#define TVCS_FWD_BALANCE 1
#endif
#ifndef TVCS_SPLIT_FIXED
#define TVCS_SPLIT_FIXED 2   // fixed cost of a tile in the slice-count model, in quanta of KMAX
#endif
// Slice count of a reduction of length K over RB row blocks of 256, at most maxk
// slices of at least 4 quanta: the smallest whose rounds x (length + 2) is within
// 3 % of the best (see above).
void balanced_split(int RB, int K, int maxk, int &KS, int &kspan) {
    const int kq = K / KMAX;   // k quanta (the reduction step of every KF)
    constexpr int kMaxSlices = 64;
    maxk = std::min(maxk, kMaxSlices);
    long long cost[kMaxSlices + 1];
    int span[kMaxSlices + 1], nsl[kMaxSlices + 1];
    long long best = -1;
    int last = 1;
    for (int k = 1; k <= maxk; ++k) {
        span[k] = (kq + k - 1) / k;                 // quanta per slice
        if (k > 1 && span[k] < 4) break;
        nsl[k] = (kq + span[k] - 1) / span[k];      // slices actually used
        const long long rounds = ((long long)RB * nsl[k] + 255) / 256;
        cost[k] = rounds * (span[k] + TVCS_SPLIT_FIXED);
        if (best < 0 || cost[k] < best) best = cost[k];
        last = k;
    }
    for (int k = 1; k <= last; ++k)
        if (cost[k] * 100 <= best * 103) {
            KS = nsl[k];
            kspan = span[k] * KMAX;
            return;
        }
}

void fwd_split(const LowpA &L, int &KS, int &kspan) {
    const int RB = L.mp / kRowsRT4;
    if (!TVCS_FWD_BALANCE) {
        KS = 1;
        while (RB * KS < TVCS_FWD_TARGET_WG && (L.Np / (KS * 2)) % KMAX == 0 &&
               L.Np / (KS * 2) >= 4 * KMAX)
            KS *= 2;
        kspan = L.Np / KS;
        return;
    }
    balanced_split(RB, L.Np, 64, KS, kspan);
}

int fwd_splits(const LowpA &L) {
    int KS, kspan;
    fwd_split(L, KS, kspan);
    return KS;
}

// Element strides of the batch operand (K columns, Bp images) between image tiles
// and between k tiles of one part.
void y_strides(long long K, int Bp, long long &yimg, long long &ytile) {
    if (kYKMajor) {
        yimg = 1024;
        ytile = (long long)(Bp / 16) * 1024;
    } else {
        yimg = (K / 32) * 512;
        ytile = 512;
    }
}

// Default image tiles per group before the autotuner has run: 16 (256 images, A
// streamed once for them) for split storage, 8 for BF16 and FP8.
int nt_default(int mode) { return mode == M_SPLIT ? 16 : 8; }

// Cover the padded batch with image groups of 16 * nt, nt in {ntmax, ..., 2, 1};
// groups holding only padding images are skipped.  fn(first image, nt, real images).
template <class Fn>
void for_each_group(int Bp, int B, int ntmax, Fn &&fn) {
    int tiles = Bp / 16, img0 = 0;
    while (tiles > 0) {
        int nt = ntmax;
        while (nt > tiles) nt >>= 1;
        const int nact = std::min(16 * nt, B - img0);
        if (nact > 0) fn(img0, nt, nact);
        img0 += 16 * nt;
        tiles -= nt;
    }
}

int grid1d(size_t count) { return (int)std::min<size_t>((count + 255) / 256, 16384); }

}  // namespace

// K slices of the adjoint product: TVCS_ADJ_SPLIT, or with TVCS_ADJ_BALANCE the
// balanced count of at most TVCS_ADJ_SPLIT_MAX slices (the shrink pass adds the
// slices' partials per pixel, so they stay few; measured: 1 slice instead of 2 at
// n = 256 makes the adjoint 6-7 % faster, while 3-4 slices at n = 128 are slower
// than 2, the model's fixed cost per tile being too small for such short tiles).
// Depends on (m, N) only.
#ifndef TVCS_ADJ_BALANCE
#define TVCS_ADJ_BALANCE 1
#endif
#ifndef TVCS_ADJ_SPLIT_MAX
#define TVCS_ADJ_SPLIT_MAX 2
#endif
void adj_split(const LowpA &L, int &KS, int &kspan) {
    if (!TVCS_ADJ_BALANCE) {
        KS = 1;
        while (KS < TVCS_ADJ_SPLIT && (L.mp / (KS * 2)) % KMAX == 0) KS *= 2;
        kspan = L.mp / KS;
        return;
    }
    balanced_split(L.Np / kRowsRT4, L.mp, TVCS_ADJ_SPLIT_MAX, KS, kspan);
}

int lowp_adj_splits(const LowpA &L) {
    int KS, kspan;
    adj_split(L, KS, kspan);
    return KS;
}

size_t lowp_storage_bytes(const LowpA &L0) {
    LowpA L = L0;
    L.mp = ((L.m + kMPad - 1) / kMPad) * kMPad;
    L.Np = ((L.N + kMPad - 1) / kMPad) * kMPad;
    const int mode = mode_of(L.storage);
    const size_t one = (size_t)L.mp * L.Np * elem_bytes(mode);
    const size_t copies = mode == M_SPLIT ? 4 : 2;
    return copies * one + (mode == M_FP8 ? sizeof(float) * L.mp : 0) + 256 * 8;
}

void lowp_bind_storage(LowpA &L, void *base) {
    L.mp = ((L.m + kMPad - 1) / kMPad) * kMPad;
    L.Np = ((L.N + kMPad - 1) / kMPad) * kMPad;
    const int mode = mode_of(L.storage);
    const size_t one = (size_t)L.mp * L.Np * elem_bytes(mode);
    char *p = static_cast<char *>(base);
    auto take = [&](size_t b) {
        void *r = p;
        p += (b + 255) / 256 * 256;
        return r;
    };
    L.X_hi = take(one);
    L.XT_hi = take(one);
    L.X_lo = L.XT_lo = nullptr;
    L.scale = nullptr;
    if (mode == M_SPLIT) {
        L.X_lo = take(one);
        L.XT_lo = take(one);
    }
    if (mode == M_FP8) L.scale = static_cast<float *>(take(sizeof(float) * L.mp));
}

void lowp_convert(LowpA &L, const float *A32, hipStream_t s) {
    const int mode = mode_of(L.storage);
    const int grid = grid1d((size_t)L.mp * L.Np / 8);
    if (mode == M_FP8)
        hipLaunchKernelGGL(k_fp8_scale, dim3(L.mp), dim3(256), 0, s, A32, L.m, L.N, L.scale);
#define TVCS_FRAG(MODEV)                                                                     \
    hipLaunchKernelGGL((k_frag<MODEV, false>), dim3(grid), dim3(256), 0, s, A32, L.m, L.N,    \
                       L.Np, L.mp, L.scale, L.X_hi, L.X_lo);                                  \
    hipLaunchKernelGGL((k_frag<MODEV, true>), dim3(grid), dim3(256), 0, s, A32, L.m, L.N, L.Np, \
                       L.mp, L.scale, L.XT_hi, L.XT_lo);
    if (mode == M_FP8) {
        TVCS_FRAG(M_FP8)
    } else if (mode == M_SPLIT) {
        TVCS_FRAG(M_SPLIT)
    } else {
        TVCS_FRAG(M_BF16)
    }
#undef TVCS_FRAG
}

size_t lowp_work_bytes(const LowpA &L, int Bp) {
    const size_t u = (size_t)Bp * L.Np * sizeof(u16), r = (size_t)Bp * L.mp * sizeof(u16);
    return 2 * u + 2 * r + (size_t)fwd_splits(L) * Bp * L.mp * sizeof(float) +
           (size_t)Bp * (L.N + L.m) * sizeof(float) + 6 * 256;
}

void lowp_work_bind(LowpWork &W, const LowpA &L, int Bp, void *base) {
    char *p = static_cast<char *>(base);
    auto take = [&](size_t b) {
        void *r = p;
        p += (b + 255) / 256 * 256;
        return r;
    };
    const size_t u = (size_t)Bp * L.Np * sizeof(u16), r = (size_t)Bp * L.mp * sizeof(u16);
    if (kYKMajor) {   // one array per operand, hi and lo blocks interleaved
        W.Ubf_hi = take(2 * u);
        W.Ubf_lo = (u16 *)W.Ubf_hi + 512;
        W.Rbf_hi = take(2 * r);
        W.Rbf_lo = (u16 *)W.Rbf_hi + 512;
    } else {
        W.Ubf_hi = take(u);
        W.Ubf_lo = take(u);
        W.Rbf_hi = take(r);
        W.Rbf_lo = take(r);
    }
    W.Rpart = static_cast<float *>(take((size_t)fwd_splits(L) * Bp * L.mp * sizeof(float)));
    W.Ut = static_cast<float *>(take((size_t)Bp * L.N * sizeof(float)));
    W.St = static_cast<float *>(take((size_t)Bp * L.m * sizeof(float)));
    W.Bp = Bp;
    W.fwd = TileCfg{4, nt_default(mode_of(L.storage)), 0};
    W.adj = TileCfg{2, nt_default(mode_of(L.storage)), 0};
}

int tile_kf(int nt, int kfv) { return kKF[kfv ? 1 : 0][log2_nt(nt)]; }

bool tile_valid(const TileCfg &c) {
    const bool nt_ok = c.nt == 1 || c.nt == 2 || c.nt == 4 || c.nt == 8 || c.nt == 16;
    return nt_ok && (c.rt == 2 || (c.rt == 4 && c.nt < 16)) && (c.kfv == 0 || c.kfv == 1);
}

// Autotuner: for each product, time every candidate tile shape on this matrix and
// padded batch (HIP events) and keep the fastest.  Candidates: 2 or 4 row tiles per
// wave, both k-tile tables, and image groups of the whole padded batch (up to 256)
// or of a half or a quarter of it.  The cost of a candidate is three increment-form
// launches plus one fresh launch (about a fifth of the iterations are fresh), after
// one warm-up launch.  The inputs are hashed values of unit size (MFMA clocks depend
// on the operands' bits), and each increment launch follows a move of its input by
// 2^-10 of its size, as between two iterations, so its operand is never zero.  st (Bp
// states) is overwritten, and so are U, R and G (scratch of the workspace's sizes).
void lowp_autotune(const LowpA &L, LowpWork &W, int Bp, float *U, float *R, float *G,
                   ImgState *st, hipStream_t s) {
    hipEvent_t e0, e1;
    TVCS_HIP(hipEventCreate(&e0));
    TVCS_HIP(hipEventCreate(&e1));
    launch_init_state(st, Bp, 0.0, 1 << 30, s, 0);   // active, increment form
    launch_fill_hash(U, (size_t)Bp * L.N, 1u, 1.0f, false, s);
    launch_fill_hash(R, (size_t)Bp * L.m, 2u, 1.0f, false, s);
    unsigned seed = 16;
    // product(parity): 0 increment, -1 fresh; moved / count: its input
    auto cost = [&](auto &&product, float *moved, size_t count) {
        product(0);
        float total = 0.f, ms = 0.f;
        for (int i = 0; i < 4; ++i) {
            if (i < 3) launch_fill_hash(moved, count, seed++, 1.0f / 1024.0f, true, s);
            TVCS_HIP(hipEventRecord(e0, s));
            product(i < 3 ? 0 : -1);
            TVCS_HIP(hipEventRecord(e1, s));
            TVCS_HIP(hipEventSynchronize(e1));
            TVCS_HIP(hipEventElapsedTime(&ms, e0, e1));
            total += ms;
        }
        return total;
    };
    int ntop = 1;
    while (2 * ntop <= std::min(Bp / 16, 16)) ntop *= 2;
    float best_f = 1e30f, best_a = 1e30f;
    TileCfg bf = W.fwd, ba = W.adj;
    for (int nt = ntop; nt >= std::max(1, ntop / 4); nt /= 2)
        for (int rt : {2, 4})
            for (int kfv : {0, 1}) {
                const TileCfg c{rt, nt, kfv};
                if (!tile_valid(c)) continue;
                // skip a table that gives this group size (and the smaller groups a
                // batch may end with) the same steps as table 0
                bool same = kfv == 1;
                for (int t = nt; t >= 1 && same; t /= 2) same = tile_kf(t, 0) == tile_kf(t, 1);
                if (same) continue;
                W.fwd = W.adj = c;
                const float tf = cost(
                    [&](int par) {
                        lowp_apply_A(L, W, Bp, U, nullptr, R, st, s, nullptr, nullptr, 0, par);
                    },
                    U, (size_t)Bp * L.N);
                const float ta = cost([&](int par) { lowp_apply_At(L, W, Bp, R, G, st, s, par); },
                                      R, (size_t)Bp * L.m);
                if (tf < best_f) {
                    best_f = tf;
                    bf = c;
                }
                if (ta < best_a) {
                    best_a = ta;
                    ba = c;
                }
            }
    W.fwd = bf;
    W.adj = ba;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

void lowp_apply_A(const LowpA &L, LowpWork &W, int B, const float *U, const float *F, float *R,
                  const ImgState *st, hipStream_t s, ImgState *stw, const double *parts,
                  int nparts, int parity) {
    const int mode = mode_of(L.storage);
    const int Bp = ((B + kBTile - 1) / kBTile) * kBTile;
    if (Bp > W.Bp) fail(TVCS_EINVAL, "MFMA workspace too small for the batch");
    long long yimg, ytile;
    y_strides(L.Np, Bp, yimg, ytile);
    if (stw && (st != stw || !parts || nparts < 1))
        fail(TVCS_EINVAL, "MFMA product: the folded stop rule needs the image states and partials");
    if (parity >= 0 && !st) fail(TVCS_EINVAL, "MFMA product: increments need the image states");
    // outside the loop (parity < 0) every product is fresh and the tracked vectors
    // of a running loop (the request loop's other slots) are left alone
    hipLaunchKernelGGL(k_split_frag, dim3(L.Np / 128, Bp / 16), dim3(256), 0, s, U, L.N, L.Np, Bp,
                       nullptr, (u16 *)W.Ubf_hi, (u16 *)W.Ubf_lo, yimg, ytile, stw, parts, nparts, B,
                       parity >= 0 ? W.Ut : nullptr, st, parity);
    int KS, kspan;
    fwd_split(L, KS, kspan);
    const long long split_stride = (long long)Bp * L.mp;
    for_each_group(Bp, B, W.fwd.nt, [&](int img0, int nt, int nact) {
        const GemmArgs a{L.X_hi, L.X_lo, L.Np, (const u16 *)W.Ubf_hi + (img0 / 16) * yimg,
                         (const u16 *)W.Ubf_lo + (img0 / 16) * yimg, yimg, ytile, L.mp, L.mp,
                         kspan, 0, KS, W.Rpart + (size_t)img0 * L.mp, split_stride, L.mp,
                         st ? st + img0 : nullptr, nact, parity};
        gemm_any(W.fwd, mode, nt, a, s);
    });
    hipLaunchKernelGGL(k_reduce_r, dim3((L.m + 255) / 256, Bp), dim3(256), 0, s, W.Rpart, KS,
                       split_stride, L.mp, F, L.scale, L.m, R, st, parity, B);
}

void lowp_apply_At(const LowpA &L, LowpWork &W, int B, const float *R, float *G,
                   const ImgState *st, hipStream_t s, int parity) {
    const int mode = mode_of(L.storage);
    const int Bp = ((B + kBTile - 1) / kBTile) * kBTile;
    if (Bp > W.Bp) fail(TVCS_EINVAL, "MFMA workspace too small for the batch");
    long long yimg, ytile;
    y_strides(L.mp, Bp, yimg, ytile);
    if (parity >= 0 && !st) fail(TVCS_EINVAL, "MFMA product: increments need the image states");
    hipLaunchKernelGGL(k_split_frag, dim3(L.mp / 128, Bp / 16), dim3(256), 0, s, R, L.m, L.mp, Bp,
                       L.scale, (u16 *)W.Rbf_hi, (u16 *)W.Rbf_lo, yimg, ytile, nullptr, nullptr, 0, B,
                       parity >= 0 ? W.St : nullptr, st, parity);
    int KS, kspan;
    adj_split(L, KS, kspan);
    const long long split_stride = (long long)Bp * L.N;
    for_each_group(Bp, B, W.adj.nt, [&](int img0, int nt, int nact) {
        const GemmArgs a{L.XT_hi, L.XT_lo, L.mp, (const u16 *)W.Rbf_hi + (img0 / 16) * yimg,
                         (const u16 *)W.Rbf_lo + (img0 / 16) * yimg, yimg, ytile, L.Np, L.N,
                         kspan, 0, KS, G + (size_t)img0 * L.N, split_stride, L.N,
                         st ? st + img0 : nullptr, nact, parity};
        gemm_any(W.adj, mode, nt, a, s);
    });
}

}  // namespace tvcs
