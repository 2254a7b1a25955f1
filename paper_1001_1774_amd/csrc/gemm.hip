// A u and A^T r on MFMA for low-precision storage of A, shared by a batch of
// images (the two products of every iteration, g_k = A^T (A u^k - f), eq. (line)).
//
// Storage (built once per A by lowp_convert):
//   BF16        X_hi = bf16(A)                      (m_p x N)  and  XT_hi = X_hi^T (N x m_p)
//   BF16_SPLIT  X_hi = bf16(A), X_lo = bf16(A - X_hi), and both transposes
//   FP8         Q = E4M3(A_ij / s_i), s_i = max_j |A_ij| / 448 (FP32), and Q^T
// Both orientations are stored so that each product is a GEMM whose operands are
// contiguous along the reduction dimension; the HBM bytes per product are the same
// as for one copy (each product streams one copy once).  m_p = m rounded up to
// 256 with zero rows.
//
// GEMM: C[b][row] = sum_k X[row][k] Y[b][k] with X the streamed matrix (A or A^T)
// and Y the small batch operand (U or R in bf16).  A workgroup (4 waves) owns
// 4*RT*16 consecutive rows of X and all Bp = 16*NT images; each wave streams
// its RT 16-row tiles of X straight from HBM into registers (every X element
// is used by exactly one wave, so it never goes through LDS) and multiplies
// them with the Y tile that the workgroup stages in LDS, with
// v_mfma_f32_16x16x32_bf16 and FP32 accumulation.  Split storage adds the
// products X_hi Y_lo and X_lo Y_hi (X_lo Y_lo, of relative size 2^-18, is left
// out).  FP8 X is widened to bf16 in registers (exact) and multiplied with Y_hi;
// the row scale folds into vectors: (A u)_i = s_i sum_j q_ij u_j and
// (A^T r)_j = sum_i q_ij (s_i r_i).
// The forward product splits its reduction (length N) into KS slices whose FP32
// partial results are added in a fixed order by k_reduce_r; workgroups are
// ordered so that each XCD works on one K slice and its Y slice stays in that
// XCD's L2.
#include "tvcs_internal.h"

#include <algorithm>

namespace tvcs {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;
typedef unsigned char u8;
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;
constexpr int KT = 64;           // reduction step per loop iteration
constexpr int YLD = KT + 8;      // LDS row stride (bf16 elements), padded against bank conflicts
constexpr int kFwdRT = 4;        // forward: 4 x 16 rows per wave, 256 per workgroup
constexpr int kAdjRT = 2;        // adjoint: 2 x 16 rows per wave, 128 per workgroup

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

// 8 E4M3 codes -> 8 bf16 (every E4M3 value is exact in bf16)
__device__ inline bf16x8 fp8x8_to_bf16(u32x2 q) {
    bf16x8 r;
    const unsigned w[2] = {q.x, q.y};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[h], false);   // bytes 0, 1
        const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[h], true);    // bytes 2, 3
        const float f[4] = {lo[0], lo[1], hi[0], hi[1]};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const u16 b = (u16)(__float_as_uint(f[j]) >> 16);   // exact: low 16 bits are 0
            r[4 * h + j] = __builtin_bit_cast(__bf16, b);
        }
    }
    return r;
}

template <int MODE, int RT, int NT>
__global__ __launch_bounds__(kThreads) void k_gemm(
    const void *__restrict__ Xhi, const void *__restrict__ Xlo, long long ldx,
    const u16 *__restrict__ Yhi, const u16 *__restrict__ Ylo, long long ldy, int M, int kspan,
    int RB, int KS, float *__restrict__ out, long long split_stride, long long ldo,
    const ImgState *__restrict__ st, int nact) {
    if (!any_active(st, nact)) return;
    // XCD-aware order: consecutive tiles (same K slice, neighbouring rows) on one XCD
    const int total = RB * KS;
    const int nloc = (total + 7) / 8;
    const int L = (blockIdx.x & 7) * nloc + (blockIdx.x >> 3);
    if (L >= total) return;
    const int ks = L / RB, rb = L % RB;

    constexpr int NY = (MODE == M_SPLIT) ? 2 : 1;
    __shared__ u16 ys[NY][NT * 16][YLD];

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    const int row_wave = rb * (4 * RT * 16) + wave * RT * 16;
    const int k_begin = ks * kspan, k_end = k_begin + kspan;

    f32x4 acc[RT][NT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    long long xoff[RT];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) xoff[rt] = (long long)min(row_wave + rt * 16 + lr, M - 1) * ldx;

    for (int k0 = k_begin; k0 < k_end; k0 += KT) {
        // this wave's X fragments: row (tile rt, lane lr), k = k0 + 32 s + lk .. +7
        bf16x8 xh[RT][2], xl[RT][2];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const long long o = xoff[rt] + k0 + 32 * s + lk;
                if (MODE == M_FP8) {
                    xh[rt][s] = fp8x8_to_bf16(
                        __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>((const u8 *)Xhi + o)));
                } else {
                    xh[rt][s] = __builtin_nontemporal_load(
                        reinterpret_cast<const bf16x8 *>((const u16 *)Xhi + o));
                    if (MODE == M_SPLIT)
                        xl[rt][s] = __builtin_nontemporal_load(
                            reinterpret_cast<const bf16x8 *>((const u16 *)Xlo + o));
                }
            }
        // stage the Y tile (NT*16 images x KT) in LDS
        __syncthreads();
        for (int t = threadIdx.x; t < NT * 16 * (KT / 8); t += kThreads) {
            const int yr = t / (KT / 8), yc = (t % (KT / 8)) * 8;
            *reinterpret_cast<uint4 *>(&ys[0][yr][yc]) =
                *reinterpret_cast<const uint4 *>(Yhi + yr * ldy + k0 + yc);
            if (MODE == M_SPLIT)
                *reinterpret_cast<uint4 *>(&ys[NY - 1][yr][yc]) =
                    *reinterpret_cast<const uint4 *>(Ylo + yr * ldy + k0 + yc);
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const bf16x8 yh = *reinterpret_cast<const bf16x8 *>(&ys[0][nt * 16 + lr][32 * s + lk]);
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
                    acc[rt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[rt][s], yh, acc[rt][nt], 0, 0, 0);
                if (MODE == M_SPLIT) {
                    const bf16x8 yl =
                        *reinterpret_cast<const bf16x8 *>(&ys[NY - 1][nt * 16 + lr][32 * s + lk]);
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt) {
                        acc[rt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh[rt][s], yl, acc[rt][nt], 0, 0, 0);
                        acc[rt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl[rt][s], yh, acc[rt][nt], 0, 0, 0);
                    }
                }
            }
    }
    // lane holds rows 4*(lane/16) .. +3 of its 16-row tile, image lane % 16 of its tile
    float *o = out + ks * split_stride;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int row = row_wave + rt * 16 + 4 * (lane >> 4);
        if (row >= M) continue;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int img = nt * 16 + lr;
            *reinterpret_cast<f32x4 *>(o + img * ldo + row) = acc[rt][nt];
        }
    }
}

// ---- conversions ---------------------------------------------------------------
// rows >= m are zero
__global__ void k_to_bf16(const float *__restrict__ A, int m, int N, int mp, u16 *__restrict__ hi,
                          u16 *__restrict__ lo) {
    const size_t total = (size_t)mp * N;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t i = e / N;
        const float a = i < (size_t)m ? A[e] : 0.f;
        const u16 h = bf16_rne(a);
        hi[e] = h;
        if (lo) lo[e] = bf16_rne(a - bf16_f32(h));   // a - hi is exact in FP32
    }
}

// per-row scale and E4M3 codes, one workgroup per row
__global__ __launch_bounds__(256) void k_to_fp8(const float *__restrict__ A, int m, int N,
                                               u8 *__restrict__ Q, float *__restrict__ scale) {
    const int i = blockIdx.x;
    u8 *q = Q + (size_t)i * N;
    if (i >= m) {
        for (int j = threadIdx.x; j < N; j += 256) q[j] = 0;
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
    float s = red[0] / 448.0f;
    if (!(s > 0.f)) s = 1.f;
    for (int j = threadIdx.x; j < N; j += 256) {
        const float x = fminf(fmaxf(a[j] / s, -448.f), 448.f);
        const int packed = __builtin_amdgcn_cvt_pk_fp8_f32(x, 0.f, 0, false);
        q[j] = (u8)(packed & 0xFF);
    }
    if (threadIdx.x == 0) scale[i] = s;
}

// XT[j][i] = X[i][j], X rows x cols, 64 x 64 tiles through LDS
template <class T>
__global__ __launch_bounds__(256) void k_transpose(const T *__restrict__ X, int rows, int cols,
                                                   T *__restrict__ XT) {
    __shared__ T tile[64][65];
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    for (int t = threadIdx.x; t < 64 * 64; t += 256) {
        const int r = t / 64, c = t % 64;
        if (r0 + r < rows && c0 + c < cols) tile[r][c] = X[(size_t)(r0 + r) * cols + c0 + c];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 64 * 64; t += 256) {
        const int c = t / 64, r = t % 64;
        if (r0 + r < rows && c0 + c < cols) XT[(size_t)(c0 + c) * rows + r0 + r] = tile[r][c];
    }
}

// per-iteration: U (Bp x N, FP32) -> bf16 hi (and lo)
__global__ void k_split_vec(const float *__restrict__ U, size_t count, u16 *__restrict__ hi,
                            u16 *__restrict__ lo) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count;
         e += (size_t)gridDim.x * blockDim.x) {
        const float x = U[e];
        const u16 h = bf16_rne(x);
        hi[e] = h;
        if (lo) lo[e] = bf16_rne(x - bf16_f32(h));
    }
}

// R[b][i] = s_i * sum_ks P[ks][b][i] - F[b][i]  (FP64 sum, fixed order), i < m
__global__ void k_reduce_r(const float *__restrict__ P, int KS, long long split_stride, int mp,
                           const float *__restrict__ F, const float *__restrict__ scale, int m,
                           float *__restrict__ R) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= m) return;
    double acc = 0.0;
    for (int k = 0; k < KS; ++k) acc += (double)P[k * split_stride + (size_t)b * mp + i];
    if (scale) acc *= (double)scale[i];
    if (F) acc -= (double)F[(size_t)b * m + i];
    R[(size_t)b * m + i] = (float)acc;
}

// Y operand of the adjoint: bf16(s_i r_i) hi (and lo), rows padded to mp with zeros
__global__ void k_split_r(const float *__restrict__ R, int m, int mp, const float *__restrict__ scale,
                          u16 *__restrict__ hi, u16 *__restrict__ lo) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= mp) return;
    float x = 0.f;
    if (i < m) {
        x = R[(size_t)b * m + i];
        if (scale) x = (float)((double)x * (double)scale[i]);
    }
    const u16 h = bf16_rne(x);
    hi[(size_t)b * mp + i] = h;
    if (lo) lo[(size_t)b * mp + i] = bf16_rne(x - bf16_f32(h));
}

template <int MODE, int RT>
void gemm_dispatch(int NT, const void *Xhi, const void *Xlo, long long ldx, const u16 *Yhi,
                   const u16 *Ylo, long long ldy, int M, int kspan, int RB, int KS, float *out,
                   long long split_stride, long long ldo, const ImgState *st, int nact,
                   hipStream_t s) {
    const int total = RB * KS;
    const dim3 grid(((total + 7) / 8) * 8);
#define TVCS_GEMM_CASE(NTV)                                                                    \
    case NTV:                                                                                  \
        hipLaunchKernelGGL((k_gemm<MODE, RT, NTV>), grid, dim3(kThreads), 0, s, Xhi, Xlo, ldx, \
                           Yhi, Ylo, ldy, M, kspan, RB, KS, out, split_stride, ldo, st, nact); \
        break;
    switch (NT) {
        TVCS_GEMM_CASE(1)
        TVCS_GEMM_CASE(2)
        TVCS_GEMM_CASE(4)
        TVCS_GEMM_CASE(8)
        default: fail(TVCS_EUNSUPPORTED, "MFMA product: padded batch must be 16, 32, 64 or 128");
    }
#undef TVCS_GEMM_CASE
}

template <int RT>
void gemm_any(int mode, int NT, const void *Xhi, const void *Xlo, long long ldx, const u16 *Yhi,
              const u16 *Ylo, long long ldy, int M, int kspan, int RB, int KS, float *out,
              long long split_stride, long long ldo, const ImgState *st, int nact, hipStream_t s) {
    switch (mode) {
        case M_BF16:
            gemm_dispatch<M_BF16, RT>(NT, Xhi, Xlo, ldx, Yhi, Ylo, ldy, M, kspan, RB, KS, out,
                                      split_stride, ldo, st, nact, s);
            break;
        case M_SPLIT:
            gemm_dispatch<M_SPLIT, RT>(NT, Xhi, Xlo, ldx, Yhi, Ylo, ldy, M, kspan, RB, KS, out,
                                       split_stride, ldo, st, nact, s);
            break;
        default:
            gemm_dispatch<M_FP8, RT>(NT, Xhi, Xlo, ldx, Yhi, Ylo, ldy, M, kspan, RB, KS, out,
                                     split_stride, ldo, st, nact, s);
    }
}

size_t elem_bytes(int mode) { return mode == M_FP8 ? 1 : 2; }

// K slices of the forward product: enough workgroups to fill the chip, slices a
// multiple of KT long
int fwd_splits(const LowpA &L) {
    const int RB = L.mp / (4 * kFwdRT * 16);
    int KS = 1;
    while (RB * KS < 512 && (L.N / (KS * 2)) % KT == 0 && L.N / (KS * 2) >= 8 * KT) KS *= 2;
    return KS;
}

// Cover the padded batch with image groups of 16 * nt, nt in {8, 4, 2, 1}; groups
// holding only padding images are skipped.  fn(first image, nt, real images).
template <class Fn>
void for_each_group(int Bp, int B, Fn &&fn) {
    int tiles = Bp / 16, img0 = 0;
    while (tiles > 0) {
        int nt = 8;
        while (nt > tiles) nt >>= 1;
        const int nact = std::min(16 * nt, B - img0);
        if (nact > 0) fn(img0, nt, nact);
        img0 += 16 * nt;
        tiles -= nt;
    }
}

int grid1d(size_t count) { return (int)std::min<size_t>((count + 255) / 256, 16384); }

}  // namespace

size_t lowp_storage_bytes(const LowpA &L0) {
    LowpA L = L0;
    L.mp = ((L.m + kMPad - 1) / kMPad) * kMPad;
    const int mode = mode_of(L.storage);
    const size_t one = (size_t)L.mp * L.N * elem_bytes(mode);
    const size_t copies = mode == M_SPLIT ? 4 : 2;
    return copies * one + (mode == M_FP8 ? sizeof(float) * L.mp : 0) + 256 * 8;
}

void lowp_bind_storage(LowpA &L, void *base) {
    L.mp = ((L.m + kMPad - 1) / kMPad) * kMPad;
    L.Np = L.N;
    const int mode = mode_of(L.storage);
    const size_t one = (size_t)L.mp * L.N * elem_bytes(mode);
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
    const dim3 tgrid((L.N + 63) / 64, (L.mp + 63) / 64);
    if (mode == M_FP8) {
        hipLaunchKernelGGL(k_to_fp8, dim3(L.mp), dim3(256), 0, s, A32, L.m, L.N, (u8 *)L.X_hi,
                           L.scale);
        hipLaunchKernelGGL(k_transpose<u8>, tgrid, dim3(256), 0, s, (const u8 *)L.X_hi, L.mp, L.N,
                           (u8 *)L.XT_hi);
        return;
    }
    const size_t total = (size_t)L.mp * L.N;
    hipLaunchKernelGGL(k_to_bf16, dim3(grid1d(total)), dim3(256), 0, s, A32, L.m, L.N, L.mp,
                       (u16 *)L.X_hi, (u16 *)L.X_lo);
    hipLaunchKernelGGL(k_transpose<u16>, tgrid, dim3(256), 0, s, (const u16 *)L.X_hi, L.mp, L.N,
                       (u16 *)L.XT_hi);
    if (mode == M_SPLIT)
        hipLaunchKernelGGL(k_transpose<u16>, tgrid, dim3(256), 0, s, (const u16 *)L.X_lo, L.mp,
                           L.N, (u16 *)L.XT_lo);
}

size_t lowp_work_bytes(const LowpA &L, int Bp) {
    const size_t u = (size_t)Bp * L.N * sizeof(u16), r = (size_t)Bp * L.mp * sizeof(u16);
    return 2 * u + 2 * r + (size_t)fwd_splits(L) * Bp * L.mp * sizeof(float) + 4 * 256;
}

void lowp_work_bind(LowpWork &W, const LowpA &L, int Bp, void *base) {
    char *p = static_cast<char *>(base);
    auto take = [&](size_t b) {
        void *r = p;
        p += (b + 255) / 256 * 256;
        return r;
    };
    const size_t u = (size_t)Bp * L.N * sizeof(u16), r = (size_t)Bp * L.mp * sizeof(u16);
    W.Ubf_hi = take(u);
    W.Ubf_lo = take(u);
    W.Rbf_hi = take(r);
    W.Rbf_lo = take(r);
    W.Rpart = static_cast<float *>(take((size_t)fwd_splits(L) * Bp * L.mp * sizeof(float)));
    W.Bp = Bp;
}

void lowp_apply_A(const LowpA &L, LowpWork &W, int B, const float *U, const float *F, float *R,
                  const ImgState *st, hipStream_t s) {
    const int mode = mode_of(L.storage);
    const int Bp = ((B + kBTile - 1) / kBTile) * kBTile;
    if (Bp > W.Bp) fail(TVCS_EINVAL, "MFMA workspace too small for the batch");
    const size_t cnt = (size_t)Bp * L.N;
    hipLaunchKernelGGL(k_split_vec, dim3(grid1d(cnt)), dim3(256), 0, s, U, cnt, (u16 *)W.Ubf_hi,
                       mode == M_SPLIT ? (u16 *)W.Ubf_lo : nullptr);
    const int KS = fwd_splits(L);
    const int RB = L.mp / (4 * kFwdRT * 16);
    const long long split_stride = (long long)Bp * L.mp;
    for_each_group(Bp, B, [&](int img0, int nt, int nact) {
        gemm_any<kFwdRT>(mode, nt, L.X_hi, L.X_lo, L.N, (const u16 *)W.Ubf_hi + (size_t)img0 * L.N,
                         (const u16 *)W.Ubf_lo + (size_t)img0 * L.N, L.N, L.mp, L.N / KS, RB, KS,
                         W.Rpart + (size_t)img0 * L.mp, split_stride, L.mp,
                         st ? st + img0 : nullptr, nact, s);
    });
    hipLaunchKernelGGL(k_reduce_r, dim3((L.m + 255) / 256, Bp), dim3(256), 0, s, W.Rpart, KS,
                       split_stride, L.mp, F, L.scale, L.m, R);
}

void lowp_apply_At(const LowpA &L, LowpWork &W, int B, const float *R, float *G,
                   const ImgState *st, hipStream_t s) {
    const int mode = mode_of(L.storage);
    const int Bp = ((B + kBTile - 1) / kBTile) * kBTile;
    if (Bp > W.Bp) fail(TVCS_EINVAL, "MFMA workspace too small for the batch");
    hipLaunchKernelGGL(k_split_r, dim3((L.mp + 255) / 256, Bp), dim3(256), 0, s, R, L.m, L.mp,
                       L.scale, (u16 *)W.Rbf_hi, mode == M_SPLIT ? (u16 *)W.Rbf_lo : nullptr);
    const int rows_per_wg = 4 * kAdjRT * 16;
    const int RB = (L.N + rows_per_wg - 1) / rows_per_wg;
    for_each_group(Bp, B, [&](int img0, int nt, int nact) {
        gemm_any<kAdjRT>(mode, nt, L.XT_hi, L.XT_lo, L.mp, (const u16 *)W.Rbf_hi + (size_t)img0 * L.mp,
                         (const u16 *)W.Rbf_lo + (size_t)img0 * L.mp, L.mp, L.N, L.mp, RB, 1,
                         G + (size_t)img0 * L.N, 0, L.N, st ? st + img0 : nullptr, nact, s);
    });
}

}  // namespace tvcs
