// The solver context behind a tvcs_handle: device storage of A, workspaces for a
// batch, the captured iteration graph, and the product/iteration plan.  Shared by
// the C entry points (api.cpp) and the serving loop (server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "tvcs_internal.h"

namespace tvcs {

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    void ensure(size_t b) {
        if (b <= bytes && p) return;
        release();
        if (b == 0) return;
        if (hipMalloc(&p, b) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            fail(TVCS_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
        }
        bytes = b;
    }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

constexpr int kGraphIters = 10;   // iterations per captured graph (even: q ping-pong)
#ifndef TVCS_FUSED_PASS
#define TVCS_FUSED_PASS 1         // one image, FP32 A, n^2 <= 16384: A u and A^T r in one pass
#endif
#ifndef TVCS_FUSED_REV
#define TVCS_FUSED_REV 1          // the one-pass product alternates its row order per iteration
#endif
#ifndef TVCS_BB_FUSED
#define TVCS_BB_FUSED 1           // inner BB steps of one image: A p and A^T A p in one pass
#endif
#ifndef TVCS_FOLD_STOP
#define TVCS_FOLD_STOP 1          // stop rule folded into the next A u pass (one image FP32; DCT, MFMA)
#endif
constexpr int kPowerIters = 100;
// inner steps on the u-subproblem requested by the solve flags (1: the IADM u-step)
inline int bb_inner(unsigned flags) {
    const int j = (int)((flags >> TVCS_BB_SHIFT) & 0xFu);
    return j > 1 ? j : 1;
}
constexpr double kPowerRtol = 1e-10;

}  // namespace tvcs

using namespace tvcs;

struct tvcs_ctx {
    int m = 0, n = 0, N = 0, storage = TVCS_A_FP32;
    int device = -1;              // the device current when the handle was created
    hipStream_t user = nullptr;   // caller's stream (may be null)
    hipStream_t work = nullptr;   // internal stream all work and captures run on
    hipEvent_t ev_in = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;

    DevBuf A32;            // FP32 storage
    DevBuf selT, dperm, dtab;   // partial DCT: coefficient -> position, position ->
                                // measurement index, DCT table
    LowpA lowp{};          // low-precision storage
    DevBuf lowp_mem;
    DevBuf tw;             // FFT twiddles
    DevBuf invd;           // FFT denominators for invd_c
    double invd_c = -1.0;
    double lmax = 0.0, tau_user = 0.0;

    // workspace for a batch of up to `cap` images (Bp padded)
    int cap = 0, capP = 0;
    int gnv = 1;           // largest images-per-pass of the FP32 products
    DevBuf U, F, R, P, RHS, Q0, Q1, S, parts, state, obj, lowp_work, lamb, counters;
    DevBuf Gacc;           // MFMA storage: the running g of the product increments (B x N)
    DevBuf adm_F, adm_U;   // request loop: f and A^T f of newly admitted slots (capP rows)
    DevBuf bb_Uk, bb_P, bb_AP, bb_parts, bb_state;   // IADM with inner BB steps
    DevBuf bb_H;           // A^T A p of the one-pass inner steps (one image)
    DevBuf DT;             // partial DCT: the half-transformed images between passes
    DevBuf PF;             // one image, FP32 A, n^2 <= kFusedN: band partials of g, then g
    LowpWork lw{};
    bool tiles_forced = false;   // tile shapes set by tvcs_set_tiles instead of the autotuner
    TileCfg forced_fwd{}, forced_adj{};
    ImgState *host_state = nullptr;   // pinned mirror for polling: two halves of cap images
    int host_state_cap = 0;
    hipEvent_t ev_poll[2] = {nullptr, nullptr};   // copies into the two halves

    // graph cache
    hipGraphExec_t exec = nullptr;
    int g_B = -1;
    unsigned g_flags = 0;
    double g_beta = 0, g_c = 0, g_ctau = 0;

    ~tvcs_ctx() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (host_state) (void)hipHostFree(host_state);
        for (hipEvent_t e : ev_poll)
            if (e) (void)hipEventDestroy(e);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_t0) (void)hipEventDestroy(ev_t0);
        if (ev_t1) (void)hipEventDestroy(ev_t1);
        if (work) (void)hipStreamDestroy(work);
    }

    bool lowprec() const {
        return storage == TVCS_A_BF16 || storage == TVCS_A_BF16_SPLIT ||
               storage == TVCS_A_FP8_ROWSCALE;
    }
    bool dct() const { return storage == TVCS_A_PARTIAL_DCT; }
    // FP32 A with n^2 <= kFusedN: a single image takes both products in one pass over A
    bool fused() const { return TVCS_FUSED_PASS && storage == TVCS_A_FP32 && fused_bands(m, N) > 0; }
    double tau() const { return tau_user > 0 ? tau_user : 1.9 / lmax; }

    // padded batch: FP32 products take 1, 2, 4 or 8 vectors per pass of A
    int padded(int B) const {
        if (dct()) return B;
        if (lowprec()) return ((B + kBTile - 1) / kBTile) * kBTile;
        if (B <= 2) return B;
        if (B <= 4) return 4;
        return ((B + 7) / 8) * 8;
    }

    void ensure_workspace(int B) {
        if (B <= cap) return;
        // a batch whose workspace cannot fit the device is refused before anything
        // is freed, so the current workspace stays usable
        size_t free_b = 0, total_b = 0;
        TVCS_HIP(hipMemGetInfo(&free_b, &total_b));
        if (workspace_bytes(B) > total_b)
            fail(TVCS_ENOMEM, "the workspace of " + std::to_string(B) + " images (" +
                                  std::to_string(workspace_bytes(B)) +
                                  " bytes) exceeds the device memory");
        if (exec) {
            TVCS_HIP(hipGraphExecDestroy(exec));
            exec = nullptr;
        }
        // until every buffer below is allocated the workspace counts as empty, so a
        // grow that fails part-way (ENOMEM) makes the next call allocate again
        cap = capP = 0;
        const int Bp = padded(B);
        const size_t Nn = (size_t)N, mm = (size_t)m, h = (size_t)(n / 2 + 1);
        gnv = (lowprec() || dct()) ? Bp : std::min(Bp, 8);
        const int nchunk = partial_count(Bp);
        U.ensure(sizeof(float) * Bp * Nn);
        F.ensure(sizeof(float) * Bp * mm);
        R.ensure(sizeof(float) * Bp * mm);
        P.ensure(sizeof(float) * (size_t)nchunk * Bp * Nn);
        RHS.ensure(sizeof(float) * Bp * Nn);
        Q0.ensure(sizeof(float2) * B * Nn);
        Q1.ensure(sizeof(float2) * B * Nn);
        S.ensure(sizeof(float2) * B * h * n);
        parts.ensure(sizeof(double) * 2 * B * (size_t)n);   // >= n / rows-per-block
        state.ensure(sizeof(ImgState) * Bp);   // Bp: the autotuner times whole groups
        obj.ensure(sizeof(double) * B);
        counters.ensure(sizeof(int) * B);
        if (dct()) DT.ensure(sizeof(float) * Bp * Nn);
        if (fused()) PF.ensure(sizeof(float) * (size_t)(fused_bands(m, N) + 1) * Nn);
        launch_fill(counters.as<float>(), (size_t)B, 0.f, work);   // all-zero bits
        if (lowprec()) {
            Gacc.ensure(sizeof(float) * B * Nn);
            lowp_work.ensure(lowp_work_bytes(lowp, Bp));
            lowp_work_bind(lw, lowp, Bp, lowp_work.p);
        }
        if (host_state_cap < B) {
            if (host_state) TVCS_HIP(hipHostFree(host_state));
            host_state = nullptr;
            host_state_cap = 0;
            TVCS_HIP(hipHostMalloc((void **)&host_state, sizeof(ImgState) * 2 * B));
            host_state_cap = B;
        }
        // padded images must hold zeros (their products are computed and ignored)
        launch_fill(U.as<float>(), (size_t)Bp * Nn, 0.f, work);
        launch_fill(F.as<float>(), (size_t)Bp * mm, 0.f, work);
        // the adjoint writes all its K slices: P is sized for them
        if (lowprec()) {
            if (tiles_forced) {
                lw.fwd = forced_fwd;
                lw.adj = forced_adj;
            } else {
                lowp_autotune(lowp, lw, Bp, U.as<float>(), R.as<float>(), P.as<float>(),
                              state.as<ImgState>(), work);
                launch_fill(U.as<float>(), (size_t)Bp * Nn, 0.f, work);   // padding: zeros
            }
        }
        cap = B;
        capP = Bp;
    }

    // tile shapes of the two MFMA products as {rt, images per group, k tiles per step}
    // of each (zeros for other storage)
    void tiles_out(int *t) const {
        for (int i = 0; i < 6; ++i) t[i] = 0;
        if (!lowprec()) return;
        const TileCfg c[2] = {lw.fwd, lw.adj};
        for (int k = 0; k < 2; ++k) {
            t[3 * k] = c[k].nt == 16 ? 2 : c[k].rt;
            t[3 * k + 1] = 16 * c[k].nt;
            t[3 * k + 2] = tile_kf(c[k].nt, c[k].kfv);
        }
    }

    // vectors per pass and row chunks of the FP32 products for a padded batch Bp.
    // The chunking (the order of the A^T r sums) is that of the widest pass for
    // every batch, so an image's g_k does not depend on the batch it is in.
    int pass_nv(int Bp) const { return std::min(Bp, 8); }
    int chunks(int /*Bp*/) const { return gemv_cols_chunks(m, N); }
    // partial sums of A^T r the shrink pass adds (one for the DCT: its adjoint is whole)
    int partial_count(int Bp) const {
        return dct() ? 1 : lowprec() ? lowp_adj_splits(lowp) : chunks(Bp);
    }

    // device bytes of the workspace ensure_workspace(B) allocates
    size_t workspace_bytes(int B) const {
        const int Bp = padded(B);
        const size_t Nn = (size_t)N, mm = (size_t)m, h = (size_t)(n / 2 + 1);
        const int nchunk = partial_count(Bp);
        size_t b = sizeof(float) * Bp * (2 * Nn + 2 * mm) + sizeof(float) * (size_t)nchunk * Bp * Nn +
                   2 * sizeof(float2) * B * Nn + sizeof(float2) * B * h * n +
                   sizeof(double) * 2 * B * (size_t)n + sizeof(ImgState) * Bp + sizeof(double) * B +
                   sizeof(int) * B;
        if (lowprec()) b += lowp_work_bytes(lowp, Bp) + sizeof(float) * B * Nn;
        if (dct()) b += sizeof(float) * Bp * Nn;
        if (fused()) b += sizeof(float) * (size_t)(fused_bands(m, N) + 1) * Nn;
        return b;
    }

    // device bytes of the request loop's admission buffers for B slots
    size_t admission_bytes(int B) const {
        return sizeof(float) * (size_t)padded(B) * ((size_t)m + (size_t)N);
    }

    // bytes of A one product streams: one copy of the stored matrix (MFMA storage
    // keeps A and A^T; a product reads one of them)
    size_t a_copy_bytes() const {
        if (dct()) return 0;
        if (!lowprec()) return A32.bytes;
        const size_t el = storage == TVCS_A_FP8_ROWSCALE ? 1 : storage == TVCS_A_BF16_SPLIT ? 4 : 2;
        return el * (size_t)lowp.mp * (size_t)N;
    }

    // device bytes of A's storage and the FFT tables
    size_t storage_bytes() const {
        return A32.bytes + lowp_mem.bytes + selT.bytes + dperm.bytes + dtab.bytes + tw.bytes +
               invd.bytes;
    }

    // B measurement vectors (host or device memory, in the caller's order) into
    // rows first .. first+B-1 of F; the partial DCT keeps them in its pass order
    // (staged through the same rows of R, which every iteration rewrites)
    void load_measurements(const float *Fin, int first, int B) {
        float *dst = (dct() ? R : F).as<float>() + (size_t)first * m;
        TVCS_HIP(hipMemcpyAsync(dst, Fin, sizeof(float) * (size_t)B * m, hipMemcpyDefault, work));
        if (dct())
            launch_dct_permute(m, B, dperm.as<int>(), dst, F.as<float>() + (size_t)first * m,
                               work);
    }

    // give the batch workspace back (the next call re-allocates what it needs)
    void release_workspace() {
        if (exec) {
            TVCS_HIP(hipGraphExecDestroy(exec));
            exec = nullptr;
        }
        for (DevBuf *b : {&U, &F, &R, &P, &RHS, &Q0, &Q1, &S, &parts, &state, &obj, &lowp_work, &lamb,
                          &counters, &DT, &Gacc, &adm_F, &adm_U, &bb_Uk, &bb_P, &bb_AP, &bb_parts,
                          &bb_state, &bb_H, &PF})
            b->release();
        cap = capP = 0;
    }

    void ensure_denominators(double c) {
        const size_t cnt = (size_t)(n / 2 + 1) * n;
        invd.ensure(sizeof(double) * cnt);
        if (c != invd_c) {
            launch_denominators(n, c, invd.as<double>(), work);
            invd_c = c;
        }
    }

    // R = A U - F for the first Bp images (F may be null).  parity >= 0: inside the
    // iteration loop (MFMA storage: per-image fresh or increment products)
    void apply_A(int Bp, int B, const float *Uin, const float *Fin, float *Rout,
                 const ImgState *st, int parity = -1) {
        if (dct()) {
            launch_dct_forward(n, B, Uin, DT.as<float>(), selT.as<int>(), Fin, m, Rout, m, false,
                               tw.as<float2>(), dtab.as<float4>(), st, work);
            return;
        }
        if (lowprec()) {
            lowp_apply_A(lowp, lw, B, Uin, Fin, Rout, st, work, nullptr, nullptr, 0, parity);
            return;
        }
        const int nv = pass_nv(Bp);
        for (int g = 0; g * nv < Bp; ++g) {
            const int real = std::max(0, std::min(nv, B - g * nv));
            if (real == 0) continue;
            launch_gemv_rows(A32.as<float>(), m, N, Uin + (size_t)g * nv * N, N,
                             Fin ? Fin + (size_t)g * nv * m : nullptr, m,
                             Rout + (size_t)g * nv * m, m, nv, st ? st + g * nv : nullptr,
                             real, work);
        }
    }

    // partial sums of A^T Rin into P (layout described by shrink_args)
    void apply_At(int Bp, int B, const float *Rin, const ImgState *st, int parity = -1) {
        if (dct()) {
            launch_dct_adjoint(n, B, Rin, m, DT.as<float>(), selT.as<int>(), true, P.as<float>(), N,
                               tw.as<float2>(), dtab.as<float4>(), st, work);
            return;
        }
        if (lowprec()) {
            lowp_apply_At(lowp, lw, B, Rin, P.as<float>(), st, work, parity);
            return;
        }
        const int nv = pass_nv(Bp), nchunk = chunks(Bp);
        const long long cs = (long long)nv * N;
        for (int g = 0; g * nv < Bp; ++g) {
            const int real = std::max(0, std::min(nv, B - g * nv));
            if (real == 0) continue;
            launch_gemv_cols(A32.as<float>(), m, N, Rin + (size_t)g * nv * m, m,
                             P.as<float>() + (size_t)g * nchunk * cs, cs, nv,
                             st ? st + g * nv : nullptr, real, work);
        }
    }

    // out = A^T Rin (full sums) for the first Bp images
    void apply_At_full(int Bp, int B, const float *Rin, float *out, const ImgState *st) {
        if (dct()) {
            launch_dct_adjoint(n, B, Rin, m, DT.as<float>(), selT.as<int>(), true, out, N,
                               tw.as<float2>(), dtab.as<float4>(), st, work);
            return;
        }
        apply_At(Bp, B, Rin, st);
        if (lowprec()) {
            launch_sum_partials(P.as<float>(), lowp_adj_splits(lowp), (long long)Bp * N, Bp, N,
                                out, N, work);
            return;
        }
        const int nv = pass_nv(Bp), nchunk = chunks(Bp);
        const long long cs = (long long)nv * N;
        for (int g = 0; g * nv < Bp; ++g)
            launch_sum_partials(P.as<float>() + (size_t)g * nchunk * cs, nchunk, cs, nv, N,
                                out + (size_t)g * nv * N, N, work);
    }

    // partial DCT: the row pass of C u for the first B images (the iteration loop
    // expects it in DT on entry; call after any change of U outside the loop)
    void seed_dct_rows(int B) {
        if (dct())
            launch_dct_rows_fwd(n, B, U.as<float>(), DT.as<float>(), tw.as<float2>(),
                                dtab.as<float4>(), nullptr, work);
    }

    ShrinkArgs shrink_args(int B, int Bp) const {
        ShrinkArgs a{};
        a.n = n;
        a.B = B;
        a.U = U.as<float>();
        a.G = P.as<float>();
        if (lowprec() || dct()) {
            a.gnv = Bp;
            a.g_group_stride = 0;
            a.nchunk = partial_count(Bp);
            a.g_chunk_stride = (long long)Bp * N;
        } else {
            const int nv = pass_nv(Bp), nchunk = chunks(Bp);
            a.gnv = nv;
            a.g_chunk_stride = (long long)nv * N;
            a.g_group_stride = (long long)nchunk * nv * N;
            a.nchunk = nchunk;
        }
        a.st = state.as<ImgState>();
        a.Gacc = lowprec() ? Gacc.as<float>() : nullptr;
        a.parity = 0;
        return a;
    }

    // One image with FP32 A, or any batch with the partial DCT or MFMA storage: the
    // stop rule of an iteration is applied by the next iteration's first pass (its
    // first workgroup per image; for MFMA storage the split of U) (fold_prev), and
    // only the last iteration of a captured graph ends with its own stop-rule pass
    // (stop_here).
    bool fold_stop(int B) const {
        return TVCS_FOLD_STOP && (dct() || lowprec() || (B == 1 && pass_nv(padded(B)) == 1));
    }

    void enqueue_iteration(int B, int parity, bool iadm, double beta, double c, double ctau,
                           bool fold_prev = false, bool stop_here = true) {
        const int Bp = padded(B);
        ImgState *st = state.as<ImgState>();
        if (dct()) {
            // forward and adjoint share the column pass: r = (C u)[sel] - f and the
            // zero-filled residual's inverse column transform in one kernel; the row
            // pass of C u came from the previous iteration's inverse row FFT (or
            // seed_dct_rows before the first)
            launch_dct_cols_fwd(n, B, DT.as<float>(), selT.as<int>(), F.as<float>(), m,
                                R.as<float>(), m, true, tw.as<float2>(), dtab.as<float4>(), st,
                                work, fold_prev ? st : nullptr,
                                fold_prev ? parts.as<double>() : nullptr,
                                fold_prev ? stop_parts(n, B) : 0);
            // the inverse row transform (g = A^T r) is computed by the shrink pass
        } else if (fold_prev && lowprec()) {
            lowp_apply_A(lowp, lw, B, U.as<float>(), F.as<float>(), R.as<float>(), st, work, st,
                         parts.as<double>(), stop_parts(n, B), parity);
            apply_At(Bp, B, R.as<float>(), st, parity);
        } else if (fused() && B == 1) {
            const int nb = fused_bands(m, N);
            launch_gemv_fused(A32.as<float>(), m, N, U.as<float>(), F.as<float>(), PF.as<float>(),
                              PF.as<float>() + (size_t)nb * N, st, parity & TVCS_FUSED_REV, work,
                              fold_prev ? st : nullptr,
                              fold_prev ? parts.as<double>() : nullptr,
                              fold_prev ? stop_parts(n, B) : 0);
        } else if (fold_prev) {
            launch_gemv_rows(A32.as<float>(), m, N, U.as<float>(), N, F.as<float>(), m,
                             R.as<float>(), m, 1, st, 1, work, st, parts.as<double>(),
                             stop_parts(n, B));
            apply_At(Bp, B, R.as<float>(), st);
        } else {
            apply_A(Bp, B, U.as<float>(), F.as<float>(), R.as<float>(), st, parity);
            apply_At(Bp, B, R.as<float>(), st, parity);
        }
        ShrinkArgs a = shrink_args(B, Bp);
        a.parity = parity;
        if (fused() && B == 1) {   // g whole, after the band partials
            a.G = PF.as<float>() + (size_t)fused_bands(m, N) * N;
            a.gnv = 1;
            a.nchunk = 1;
            a.g_chunk_stride = N;
            a.g_group_stride = N;
        }
        if (dct()) {
            a.T = DT.as<float>();
            a.dtab = dtab.as<float4>();
        }
        a.beta = beta;
        a.c = c;
        a.ctau = ctau;
        a.Qold = parity ? Q1.as<float2>() : Q0.as<float2>();
        a.Qnew = parity ? Q0.as<float2>() : Q1.as<float2>();
        const float2 *twp = tw.as<float2>();
        float2 *Sp = S.as<float2>();
        launch_shrink_rows(a, iadm, Sp, twp, work);
        launch_fft_cols_solve(n, B, Sp, invd.as<double>(), twp, st, work);
        launch_fft_rows_inv(n, B, Sp, U.as<float>(), parts.as<double>(), twp, st,
                            counters.as<int>(), work, dct() ? DT.as<float>() : nullptr,
                            dct() ? dtab.as<float4>() : nullptr, stop_here, parity);
    }

    // buffers of IADM with inner steps for a batch of B (FP32 storage)
    void ensure_bb(int B) {
        const int Bp = padded(B);
        const size_t Nn = (size_t)N;
        bb_Uk.ensure(sizeof(float) * B * Nn);
        if (bb_P.bytes < sizeof(float) * Bp * Nn) {
            bb_P.ensure(sizeof(float) * Bp * Nn);
            launch_fill(bb_P.as<float>(), (size_t)Bp * Nn, 0.f, work);   // padded rows stay 0
        }
        bb_AP.ensure(sizeof(float) * Bp * (size_t)m);
        bb_parts.ensure(sizeof(double) * 5 * B * (size_t)bb_blocks(n));
        bb_state.ensure(sizeof(BBState) * 2 * B);
        if (bb_fused(B)) bb_H.ensure(sizeof(float) * Nn);
    }
    bool bb_fused(int B) const { return TVCS_BB_FUSED && fused() && B == 1; }

    // One outer iteration of IADM whose u-step is `inner` steps on the u-subproblem
    // of (ALP) (bb.hip): r = A u - f, then per inner step A^T r, the direction p (shrink
    // pass with q held fixed after the first step, FFT solve into bb_P), A p, the step
    // length and v += a p, r += a A p (one pass, which at the first step also saves u
    // and at the last adds up the stop-rule norms); the stop rule compares u with the
    // u saved first.
    // With MFMA storage every product is fresh (two-part batch operand, no running g):
    // directions do not shrink the way the increments of the plain iteration do.
    // fold_prev / stop_here as for enqueue_iteration (one-pass products only: the
    // previous outer step's stop rule is then applied by the first band sum).
    void enqueue_iteration_bb(int B, int parity, int inner, double mu, double beta, double c,
                              double ctau, double tau, bool fold_prev, bool stop_here) {
        const int Bp = padded(B);
        ImgState *st = state.as<ImgState>();
        float *Up = U.as<float>(), *Pd = bb_P.as<float>(), *AP = bb_AP.as<float>();
        // one image with the one-pass product: g = A^T (A u - f) is carried (g += a A^T A p)
        // and each pass reads A once for A p and A^T A p; the row order alternates
        // from one pass to the next, ending reversed before the last inner step's
        // plain A p, which reads forward; the norms of the step length are added up by
        // extra workgroups of the band sums
        const bool one = bb_fused(B);
        const int nb = one ? fused_bands(m, N) : 0;
        float *Gb = one ? PF.as<float>() + (size_t)nb * N : nullptr;
        float *Hb = one ? bb_H.as<float>() : nullptr;
        double *bparts = bb_parts.as<double>();
        const int nblk = bb_blocks(n);
        fold_prev = fold_prev && one;
        if (one)
            launch_gemv_fused(A32.as<float>(), m, N, Up, F.as<float>(), PF.as<float>(), Gb, st,
                              inner & 1, work, fold_prev ? st : nullptr,
                              fold_prev ? bparts + (size_t)3 * nblk : nullptr,
                              fold_prev ? nblk : 0);
        else
            apply_A(Bp, B, Up, F.as<float>(), R.as<float>(), st);
        const float2 *twp = tw.as<float2>();
        float2 *Sp = S.as<float2>();
        for (int j = 0; j < inner; ++j) {
            if (!one) apply_At(Bp, B, R.as<float>(), st);
            ShrinkArgs a = shrink_args(B, Bp);
            if (one) {   // g whole
                a.G = Gb;
                a.gnv = 1;
                a.nchunk = 1;
                a.g_chunk_stride = N;
                a.g_group_stride = N;
            }
            a.beta = beta;
            a.c = c;
            a.ctau = ctau;
            a.parity = parity;
            a.Gacc = nullptr;   // g is the sum of this step's (fresh) partials
            // the first step computes q^k from q^{k-1} into Qnew; later ones read it
            a.Qnew = parity ? Q0.as<float2>() : Q1.as<float2>();
            a.Qold = j == 0 ? (parity ? Q1.as<float2>() : Q0.as<float2>()) : a.Qnew;
            a.frozen = j > 0;
            launch_shrink_rows(a, true, Sp, twp, work);
            launch_fft_cols_solve(n, B, Sp, invd.as<double>(), twp, st, work);
            launch_fft_rows_inv(n, B, Sp, Up, parts.as<double>(), twp, st, counters.as<int>(), work,
                                nullptr, nullptr, false, parity, Pd);
            const bool fwd_only = !one || j == inner - 1;
            if (fwd_only) {
                apply_A(Bp, B, Pd, nullptr, AP, st);
            } else {
                const BBNorms nm = bb_norms(n, m, Pd, AP, m, bparts);
                launch_gemv_fused(A32.as<float>(), m, N, Pd, nullptr, PF.as<float>(), Hb, st,
                                  (inner - 1 - j) & 1, work, nullptr, nullptr, 0, AP, &nm);
            }
            launch_bb_step(n, m, B, Up, Pd, one ? nullptr : R.as<float>(), AP, m,
                           bb_Uk.as<float>(), bparts, bb_state.as<BBState>(), st, j,
                           j == inner - 1, beta, mu, tau, kBBSigma, work,
                           fwd_only ? nullptr : Gb, Hb, !fwd_only);
        }
        // no product-form bookkeeping: every product of this path is fresh
        if (!one || stop_here) launch_bb_stop(n, B, bparts, st, -1, work);
    }

    void build_graph(int B, unsigned flags, double beta, double c, double ctau) {
        if (exec && g_B == B && g_flags == flags && g_beta == beta && g_c == c && g_ctau == ctau)
            return;
        if (exec) {
            TVCS_HIP(hipGraphExecDestroy(exec));
            exec = nullptr;
        }
        hipGraph_t graph = nullptr;
        const int inner = bb_inner(flags);
        if (inner > 1) ensure_bb(B);
        TVCS_HIP(hipStreamBeginCapture(work, hipStreamCaptureModeRelaxed));
        try {
            const bool fold = fold_stop(B);
            for (int i = 0; i < kGraphIters; ++i) {
                if (inner > 1)
                    enqueue_iteration_bb(B, i & 1, inner, ctau * beta, beta, c, ctau,
                                         ctau * beta / (beta * c), TVCS_FOLD_STOP && i > 0,
                                         !TVCS_FOLD_STOP || i == kGraphIters - 1);
                else
                    enqueue_iteration(B, i & 1, (flags & TVCS_IADM) != 0, beta, c, ctau,
                                      fold && i > 0, !fold || i == kGraphIters - 1);
            }
        } catch (...) {
            (void)hipStreamEndCapture(work, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        TVCS_HIP(hipStreamEndCapture(work, &graph));
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            exec = nullptr;
            fail(TVCS_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        g_B = B;
        g_flags = flags;
        g_beta = beta;
        g_c = c;
        g_ctau = ctau;
    }

    void begin_call() {
        if (user) {
            TVCS_HIP(hipEventRecord(ev_in, user));
            TVCS_HIP(hipStreamWaitEvent(work, ev_in, 0));
        } else {
            TVCS_HIP(hipStreamSynchronize(nullptr));
        }
    }

    void estimate_lambda_max() {
        if (dct()) {   // A A^T = I: the nonzero eigenvalues of A^T A are all 1
            lmax = 1.0;
            return;
        }
        ensure_workspace(1);
        const int Bp = padded(1);
        ImgState *st = state.as<ImgState>();
        launch_init_state(st, 1, 0.0, kPowerIters, work);
        float *v = U.as<float>();
        launch_fill(v, (size_t)N, (float)(1.0 / std::sqrt((double)N)), work);
        for (int it = 0; it < kPowerIters; ++it) {
            apply_A(Bp, 1, v, nullptr, R.as<float>(), st);
            apply_At_full(Bp, 1, R.as<float>(), RHS.as<float>(), st);
            launch_power_normalize(v, RHS.as<float>(), N, st, kPowerRtol, work);
        }
        ImgState hs;
        TVCS_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, work));
        TVCS_HIP(hipStreamSynchronize(work));
        TVCS_HIP(hipGetLastError());
        lmax = hs.rel;
        if (!(lmax > 0) || !std::isfinite(lmax))
            fail(TVCS_ENONFINITE, "power iteration gave a non-positive lambda_max");
    }

    size_t device_bytes() const {
        return A32.bytes + lowp_mem.bytes + selT.bytes + dperm.bytes + dtab.bytes + DT.bytes +
               tw.bytes + invd.bytes + U.bytes + F.bytes + R.bytes +
               P.bytes + RHS.bytes + Q0.bytes + Q1.bytes + S.bytes + parts.bytes + state.bytes +
               obj.bytes + lowp_work.bytes + lamb.bytes + counters.bytes + Gacc.bytes + adm_F.bytes +
               adm_U.bytes + bb_Uk.bytes + bb_P.bytes + bb_AP.bytes + bb_parts.bytes +
               bb_state.bytes + bb_H.bytes + PF.bytes;
    }
};

namespace tvcs {
// error-to-code wrapper used by every C entry point
extern thread_local std::string g_last_error;
template <class F>
int guarded(F &&fn) {
    try {
        g_last_error.clear();
        return fn();
    } catch (const Error &e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return TVCS_ENOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return TVCS_EDEVICE;
    }
}
}  // namespace tvcs
