// Internal declarations shared by the library's HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "tvcs.h"

namespace tvcs {

struct Error {
    int code;
    std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg);

#define TVCS_HIP(call)                                                                 \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            ::tvcs::fail(TVCS_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Per-image loop state kept on the device.  `active` predicates every per-image
// kernel: once an image meets the stop rule (or maxit), its kernels return at
// entry, so no extra iterations touch it.
struct ImgState {
    int iters;      // u-updates performed
    int active;     // 1 while the image still iterates
    int status;     // TVCS_OK / TVCS_MAXIT / TVCS_ENONFINITE
    int maxit;      // iteration cap of this image
    double rel;     // last ||u^{k+1}-u^k|| / ||u^k||
    double du2;     // last ||u^{k+1}-u^k||^2
    double u2;      // last ||u^k||^2
    double tol;     // stop tolerance of this image (0: run maxit iterations)
    // Products of MFMA storage: mode[k & 1] != 0 makes iteration k compute A u and
    // A^T r afresh from a two-part bf16 batch operand; 0 makes it add A d to the
    // previous r (and A^T e to the previous g) with d the one-part bf16 difference
    // between u and the point the previous r belongs to (see gemm.hip).  The stop
    // rule of iteration j sets mode[j & 1], the mode of iteration j + 2.
    int mode[2];
    int fresh;      // iterations so far whose products were fresh (counted by the stop rule)
    int pad_;
};

// Fresh (two-part) products while the relative change of the iterates exceeds this
// (bf16 rounding errs by at most 2^-8 of a value: the one-part increment then drops
// at most 2^-8 of a change of at most 2^-8 of u, the size of what the two-part split
// itself drops), and every kFreshEvery-th iteration, which bounds how long FP32 sums
// of increments run.
constexpr double kFreshTheta = 0.00390625;   // 2^-8
constexpr int kFreshEvery = 64;

// Largest image side the FFT kernels handle (LDS twiddle table length).
constexpr int kMaxN = 512;

// Image sides: even, 8 <= n <= kMaxN, no prime factor other than 2, 3 and 5
// (the FFTs are radix 2/3/4/5; two real rows share one complex transform).
bool is_pow2(int n);
bool supported_side(int n);
int even_divisor_at_most(int n, int want);   // largest even divisor of n <= want (>= 2)

// ---------------------------------------------------------------------------
// FP32 dense products (gemv.hip).  A is m x N row-major FP32.
//   rows: R[v*ldr + i] = sum_j A[i*N + j] U[v*ldu + j] - F[v*ldf + i], v < nv
//   cols: P[c*chunk_stride + v*N + j] = sum_{i in chunk c} A[i*N + j] R[v*ldr + i]
// Both return at entry when `active` is given and none of its `nact` flags is set.
// ---------------------------------------------------------------------------
// stw, parts, nparts (one image, nv = nact = 1, stw == active): workgroup 0 first
// applies the previous iteration's stop rule to stw from the inverse row pass's
// nparts norm partials (launch_fft_rows_inv with stop_pass = false)
void launch_gemv_rows(const float *A, int m, int N, const float *U, int ldu, const float *F,
                      int ldf, float *R, int ldr, int nv, const ImgState *active, int nact,
                      hipStream_t s, ImgState *stw = nullptr, const double *parts = nullptr,
                      int nparts = 0);
int gemv_cols_chunks(int m, int N);   // row chunks of the A^T r partial sums
// The partial sums of the BB step length's norms (device_bb.h): nblk blocks per
// image, 3 doubles each in parts (||p||^2, ||D p||^2 over the block's pixels of P,
// ||A p||^2 over its rows of AP, row stride ldap)
struct BBNorms {
    const float *P;
    const float *AP;
    double *parts;
    int n, m, ldap, nblk;
};
BBNorms bb_norms(int n, int m, const float *P, const float *AP, int ldap, double *parts);
// One image, both products in one pass (n^2 <= kFusedN): g = A^T (A U - F) into g_out
// (N floats; null: only the band partials), through nb = fused_bands(m, N) band
// partials in P (nb x N floats); rev (0/1) reverses the order of each band's rows
// (alternated per iteration); stw as for launch_gemv_rows (applied by the
// partial-sum kernel, so only with g_out); F null: f = 0; r_out (m floats, or null)
// receives A U - F as the pass rounds it; norms (non-null, with g_out and r_out):
// extra workgroups of the partial-sum kernel write the BB norm partials of U and
// r_out.  fused_bands is 0 where the pass does not apply.  launch_sum_bands: g_out =
// the fixed-order sum of the nb partials.
constexpr int kFusedN = 16384;
constexpr int kFusedMaxBands = 256;
int fused_bands(int m, int N);
void launch_gemv_fused(const float *A, int m, int N, const float *U, const float *F, float *P,
                       float *g_out, const ImgState *st, int rev, hipStream_t s,
                       ImgState *stw = nullptr, const double *parts = nullptr, int nparts = 0,
                       float *r_out = nullptr, const BBNorms *norms = nullptr);
void launch_sum_bands(const float *P, int nb, int N, float *g_out, const ImgState *st,
                      hipStream_t s, ImgState *stw = nullptr, const double *parts = nullptr,
                      int nparts = 0, const BBNorms *norms = nullptr);
// chunk c of vector v goes to P[c*chunk_stride + v*N + j]
void launch_gemv_cols(const float *A, int m, int N, const float *R, int ldr, float *P,
                      long long chunk_stride, int nv, const ImgState *active, int nact,
                      hipStream_t s);

// ---------------------------------------------------------------------------
// Reductions and small kernels (util.hip)
// ---------------------------------------------------------------------------
// out[v*ldo + j] = sum_c P[c*chunk_stride + v*N + j]  (fixed order, FP64 accumulate)
void launch_sum_partials(const float *P, int nchunk, long long chunk_stride, int nv, int N,
                         float *out, int ldo, hipStream_t s);
void launch_fill(float *x, size_t count, float value, hipStream_t s);
// x = scale * (hashed index in [-1, 1)), or x += that with add (measurement inputs)
void launch_fill_hash(float *x, size_t count, unsigned seed, float scale, bool add, hipStream_t s);
// fresh: the mode of the first two iterations (1: fresh products; 0 only for timing
// the increment form of the products)
void launch_init_state(ImgState *st, int B, double tol, int maxit, hipStream_t s,
                       int fresh = 1);
// Power-iteration step for lambda_max(A^T A): rq = v.w, v <- w/||w||; st->rel = rq,
// st->iters counts steps, st->active cleared once |rq - rq_prev| <= rtol rq.
void launch_power_normalize(float *v, const float *w, int N, ImgState *st, double rtol,
                            hipStream_t s);
// dst[i] = (float)src[i], nearest-even
void launch_round_f64_f32(const double *src, float *dst, size_t count, hipStream_t s);

// ---------------------------------------------------------------------------
// Shrinkage and right-hand side (device_shrink.h, consumed by the fused
// shrink + forward row-FFT pass in fft.hip)
//   FTVCS: q = s(D u);  IADM: q = s(2 D u - q_old) - D u + q_old
//   rhs = D^T (q - D u) - c tau g (right side for the increment u^{k+1} - u^k),
//   g = sum over `nchunk` partials of A^T r
// ---------------------------------------------------------------------------
struct ShrinkArgs {
    int n, B;
    const float *U;        // B x N
    // partial sums of A^T r: chunk c of image b at
    //   G + (b / gnv) * g_group_stride + c * g_chunk_stride + (b % gnv) * N
    const float *G;
    int gnv;
    long long g_group_stride;
    int nchunk;
    long long g_chunk_stride;
    const float2 *Qold;    // B x N pairs (q1, q2) (IADM)
    float2 *Qnew;          // B x N pairs (IADM)
    double beta, c, ctau;  // c = mu/(beta tau), ctau = c*tau = mu/beta
    const ImgState *st;
    // MFMA storage: the running g (B x N FP32).  Iterations in increment mode add
    // the partials to it, fresh ones replace it; null: g is the partials' sum alone
    float *Gacc;
    int parity;            // iteration parity (selects ImgState::mode)
    // IADM with inner steps on the u-subproblem: q = w^{k+1} - lambda^k / beta is
    // held fixed (read from Qold, nothing written) after the first inner step
    int frozen;
    // partial DCT: g is the inverse row DCT of T (the column pass's output,
    // column-major per image), computed in the pass; G is then unused
    const float *T;
    const float4 *dtab;
};
// q is held as FP32 pairs (q1, q2) per pixel; the arithmetic on it is FP64
void launch_init_q(int n, int B, const float *U, const double *lam0, double beta, float2 *Q,
                   hipStream_t s);
// lambda^K = beta (D u^K - q^{K-1}); q^{K-1} is in Q0 when the image's iteration count
// is even and in Q1 when it is odd (the fields alternate every iteration).
void launch_lambda_out(int n, int B, const float *U, const float2 *Q0, const float2 *Q1,
                       const ImgState *st, double beta, double *lam, hipStream_t s);
// obj[b] = TV(u_b) + mu/2 ||r_b||^2
void launch_objective(int n, int m, int B, const float *U, const float *R, int ldr, double mu,
                      double *obj, hipStream_t s);

// ---------------------------------------------------------------------------
// FFT solve of (D^T D + c I) u = rhs under periodic BC (fft.hip)
// Spectrum S: B x (n/2+1) x n complex FP32, k2-major ([b][k2][r]).
// inv_d: (n/2+1) x n FP64, 1 / (n^2 (4 sin^2(pi k1/n) + 4 sin^2(pi k2/n) + c)).
// ---------------------------------------------------------------------------
// tw[t] = exp(-2 pi i t / L), L = 512 for power-of-two n, else L = n (kMaxN entries)
void launch_twiddles(int n, float2 *tw, hipStream_t s);
void launch_denominators(int n, double c, double *inv_d, hipStream_t s);
void launch_fft_cols_solve(int n, int B, float2 *S, const double *inv_d, const float2 *tw,
                           const ImgState *st, hipStream_t s);
// inverse row pass, u += increment, and the stop rule of every image (the last
// workgroup of an image sums the norm partials; counters: one zeroed int per image)
// T, dtab (partial DCT): also write the DCT-II of the new rows of u to T, as
// launch_dct_rows_fwd does (null: not)
// stop_pass = false: no k_stop_rule after the pass (the caller applies the rule
// later, e.g. folded into the next A u product); stop_parts(n, B) partials per image.
// parity: the iteration's parity (the stop rule sets ImgState::mode[parity]; < 0: not)
// dir: the increment is a search direction (IADM with inner steps): written to dir
// (B x N) instead of added to U, parts receive (sum of its squares, 0) per block; use
// with stop_pass = false and T null
void launch_fft_rows_inv(int n, int B, const float2 *S, float *U, double *parts,
                         const float2 *tw, ImgState *st, int *counters, hipStream_t s,
                         float *T = nullptr, const float4 *dtab = nullptr,
                         bool stop_pass = true, int parity = -1, float *dir = nullptr);
int stop_parts(int n, int B);
// shrinkage + right-hand side fused with the forward row FFT
void launch_shrink_rows(const ShrinkArgs &a, bool iadm, float2 *S, const float2 *tw,
                        hipStream_t s);

// ---------------------------------------------------------------------------
// IADM with inner BB / non-monotone line-search steps on its u-subproblem (bb.hip)
// ---------------------------------------------------------------------------
constexpr int kBBMemory = 5;          // accepted values the non-monotone test looks back over
constexpr double kBBSigma = 1e-4;     // sufficient-decrease constant of that test
struct BBState {                      // per image, rewritten at the first inner step
    double phis[kBBMemory];           // the last accepted Phi(v) - Phi(v_0), circular
    double phi;                       // Phi(v) - Phi(v_0) at the current inner iterate
    double prev_pMp, prev_pHp;        // p'M p and p'H p of the previous direction
    double alpha;                     // the step length of the current inner step
    int nphi, pad_;
};
int bb_blocks(int n);                 // partial sums per image of the BB reductions
// Inner step j of the B images (k_bb_partials, k_bb_apply): squared norms of p, D p
// and A p, the step length, U += a P (B x N) and R += a AP (B x m, row stride ldr;
// skipped for R null); with G non-null also G += a H (B x N: the gradient
// A^T (A v - f) carried instead of r, H = A^T A p); j == 0 first saves U into Uk, and
// the last step (last) leaves the stop-rule partials of U against Uk.  parts:
// B x bb_blocks(n) x 5 doubles (the norm partials first, bb_norms(n, m, P, AP, ldr,
// parts), which norms_done says are already there); bs: 2 B states (the state
// alternates between the halves with the parity of j).
void launch_bb_step(int n, int m, int B, float *U, const float *P, float *R, const float *AP,
                    int ldr, float *Uk, double *parts, BBState *bs, const ImgState *st, int j,
                    bool last, double beta, double mu, double tau, double sigma, hipStream_t s,
                    float *G = nullptr, const float *H = nullptr, bool norms_done = false);
// the stop rule for the outer step from Uk to U, from the partials the last inner
// step left in parts (at parts + 3 B bb_blocks(n), 2 doubles per block)
void launch_bb_stop(int n, int B, double *parts, ImgState *st, int parity, hipStream_t s);

// ---------------------------------------------------------------------------
// MFMA products for bf16 / split-bf16 / fp8 storage (gemm.hip)
// ---------------------------------------------------------------------------
struct LowpA {
    int storage;                 // TVCS_A_BF16 / _BF16_SPLIT / _FP8_ROWSCALE
    int m, N, mp, Np;            // logical and padded sizes (mp, Np multiples of kMPad)
    void *X_hi, *X_lo;           // m_p x N_p (row products, K = N_p contiguous)
    void *XT_hi, *XT_lo;         // N_p x m_p (column products, K = m_p contiguous)
    float *scale;                // m_p row scales (fp8)
};
constexpr int kMPad = 256;       // row padding of A (and K padding of A^T)
constexpr int kBTile = 16;       // batch granularity of the MFMA products

size_t lowp_storage_bytes(const LowpA &L);          // bytes for the formats of L.storage
void lowp_bind_storage(LowpA &L, void *base);        // fills mp, Np and the pointers
void lowp_convert(LowpA &L, const float *A32, hipStream_t s);
// Tile shape of one MFMA product: rt 16-row tiles of the streamed matrix per wave;
// image groups of up to 16 * nt images (nt in 1, 2, 4, 8, 16; A is streamed once per
// group); kfv picks the table of 32-wide k tiles per pipeline step (tile_kf).  No
// choice changes the order of any sum, so results are the same bits for all.
struct TileCfg {
    int rt, nt, kfv;
};
int tile_kf(int nt, int kfv);                        // k tiles per step of an nt group
bool tile_valid(const TileCfg &c);
// R[b*ldr + i] = (A u_b)_i - F[b*ldf + i] for b < B (B padded to kBTile in workspace)
struct LowpWork {
    void *Ubf_hi, *Ubf_lo;       // Bp x N   bf16 copies of U
    void *Rbf_hi, *Rbf_lo;       // Bp x m_p bf16 copies of (scaled) R
    float *Rpart;                // ksplit x Bp x m_p
    float *Ut;                   // Bp x N: the point the current R belongs to
    float *St;                   // Bp x m: the vector the current g belongs to (s o r)
    int Bp;
    TileCfg fwd, adj;            // tile shapes of the two products (autotuned)
};
size_t lowp_work_bytes(const LowpA &L, int B);
void lowp_work_bind(LowpWork &W, const LowpA &L, int B, void *base);
// stw, parts, nparts (stw == st): the pass that splits U also applies the previous
// iteration's stop rule to every image first, as launch_gemv_rows does for one image.
// parity >= 0 (inside the iteration loop): image b's products follow
// st[b].mode[parity] (fresh, or the increment form that updates R in place);
// parity < 0: fresh products for every image.
void lowp_apply_A(const LowpA &L, LowpWork &W, int B, const float *U, const float *F, float *R,
                  const ImgState *st, hipStream_t s, ImgState *stw = nullptr,
                  const double *parts = nullptr, int nparts = 0, int parity = -1);
// K slices of the adjoint product: G holds that many partial sums, [slice][Bp][N]
int lowp_adj_splits(const LowpA &L);
// G[(k*Bp + b)*N + j] = slice k of (A^T r_b)_j
// (parity as for lowp_apply_A; in increment mode G receives the partials of the
// increment of g, which the shrink pass adds to the running g)
void lowp_apply_At(const LowpA &L, LowpWork &W, int B, const float *R, float *G,
                   const ImgState *st, hipStream_t s, int parity = -1);
// pick the tile shape of each product by timing the candidates on this batch; st
// holds Bp image states, U, R and G are workspace arrays (all overwritten)
void lowp_autotune(const LowpA &L, LowpWork &W, int Bp, float *U, float *R, float *G,
                   ImgState *st, hipStream_t s);

// ---------------------------------------------------------------------------
// Partial-DCT operator (dct.hip): A = rows of the orthonormal 2-D DCT-II.
// T is a B x N work array (column-major half transforms); selT[k_c * n + k_r] is
// the position of coefficient k_r * n + k_c among the kept ones, or -1 when it is
// not kept.  Positions count the kept coefficients in k_c-major order (the order
// the column pass visits them); F and R are held in that order on the device.
// ---------------------------------------------------------------------------
int dct_lines(int n);                                // lines per workgroup of the passes
void launch_dct_table(int n, float4 *tab, hipStream_t s);
// dst[b*m + j] = src[b*m + perm[j]] for b < B (measurement order -> pass order)
void launch_dct_permute(int m, int B, const int *perm, const float *src, float *dst,
                        hipStream_t s);
// R[b*ldr + i] = (C u_b)[sel_i] - F[b*ldf + i] (F may be null); with `adjoint`, T is
// left holding the inverse column transform of the zero-filled residual, ready for
// launch_dct_adjoint(..., from_R = false, ...)
void launch_dct_forward(int n, int B, const float *U, float *T, const int *selT, const float *F,
                        int ldf, float *R, int ldr, bool adjoint, const float2 *tw,
                        const float4 *tab, const ImgState *st, hipStream_t s);
// the row pass alone (T from U), and the column pass alone (continuing from T)
void launch_dct_rows_fwd(int n, int B, const float *U, float *T, const float2 *tw,
                         const float4 *tab, const ImgState *st, hipStream_t s);
// stw, parts, nparts (stw == st): the first workgroup of each image first applies
// the previous iteration's stop rule to it, as launch_gemv_rows does for one image
void launch_dct_cols_fwd(int n, int B, float *T, const int *selT, const float *F, int ldf,
                         float *R, int ldr, bool adjoint, const float2 *tw, const float4 *tab,
                         const ImgState *st, hipStream_t s, ImgState *stw = nullptr,
                         const double *parts = nullptr, int nparts = 0);
// G[b*ldg + p] = (A^T r_b)_p; from_R: scatter R first, else continue from T
void launch_dct_adjoint(int n, int B, const float *R, int ldr, float *T, const int *selT,
                        bool from_R, float *G, int ldg, const float2 *tw, const float4 *tab,
                        const ImgState *st, hipStream_t s);

// achievable HBM read bandwidth (GB/s) and dense bf16 MFMA rate (TFLOP/s)
void measure_peaks(size_t bytes, int reps, double *read_gbs, double *mfma_tflops);

}  // namespace tvcs
