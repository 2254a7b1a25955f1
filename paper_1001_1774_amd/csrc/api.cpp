// C ABI and host orchestration of the reconstruction loop.
//
// One iteration of Alg. 1 (FTVCS) or Alg. 2 (IADM) is the kernel sequence
//   r = A u - f            (FP32 GEMV, or MFMA GEMM for low-precision storage)
//   g = A^T r              (partial sums per row chunk, added by the next kernel)
//   q, rhs                 (fused differences + shrinkage + D^T + c (u - tau g))
//   S = FFT_rows(rhs); S = IFFT_cols(FFT_cols(S) / d); u = IFFT_rows(S)
//   stop rule              (FP64 norms; per-image `active` flag)
// captured once into a hipGraph of P iterations and replayed.  Every kernel reads
// its image's `active` flag at entry, so images that have met the stop rule (eq.
// (stop)) or maxit are skipped on the device and the host only polls a few
// bytes between replays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "tvcs_internal.h"

namespace tvcs {

static thread_local std::string g_last_error;

[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }

namespace {

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
constexpr int kPowerIters = 100;
constexpr double kPowerRtol = 1e-10;

}  // namespace
}  // namespace tvcs

using namespace tvcs;

struct tvcs_ctx {
    int m = 0, n = 0, N = 0, storage = TVCS_A_FP32;
    hipStream_t user = nullptr;   // caller's stream (may be null)
    hipStream_t work = nullptr;   // internal stream all work and captures run on
    hipEvent_t ev_in = nullptr, ev_t0 = nullptr, ev_t1 = nullptr;

    DevBuf A32;            // FP32 storage
    LowpA lowp{};          // low-precision storage
    DevBuf lowp_mem;
    DevBuf tw;             // FFT twiddles
    DevBuf invd;           // FFT denominators for invd_c
    double invd_c = -1.0;
    double lmax = 0.0, tau_user = 0.0;

    // workspace for a batch of up to `cap` images (Bp padded)
    int cap = 0, capP = 0;
    int gnv = 1;           // largest images-per-pass of the FP32 products
    DevBuf U, F, R, P, RHS, Q0, Q1, S, parts, state, obj, lowp_work, lamb;
    LowpWork lw{};
    ImgState *host_state = nullptr;   // pinned mirror for polling
    int host_state_cap = 0;

    // graph cache
    hipGraphExec_t exec = nullptr;
    int g_B = -1;
    unsigned g_flags = 0;
    double g_beta = 0, g_c = 0, g_ctau = 0;

    ~tvcs_ctx() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (host_state) (void)hipHostFree(host_state);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_t0) (void)hipEventDestroy(ev_t0);
        if (ev_t1) (void)hipEventDestroy(ev_t1);
        if (work) (void)hipStreamDestroy(work);
    }

    bool lowprec() const { return storage != TVCS_A_FP32; }
    double tau() const { return tau_user > 0 ? tau_user : 1.9 / lmax; }

    // padded batch: FP32 products take 1, 2, 4 or 8 vectors per pass of A
    int padded(int B) const {
        if (lowprec()) return ((B + kBTile - 1) / kBTile) * kBTile;
        if (B <= 2) return B;
        if (B <= 4) return 4;
        return ((B + 7) / 8) * 8;
    }

    void ensure_workspace(int B) {
        if (B <= cap) return;
        if (exec) {
            TVCS_HIP(hipGraphExecDestroy(exec));
            exec = nullptr;
        }
        const int Bp = padded(B);
        const size_t Nn = (size_t)N, mm = (size_t)m, h = (size_t)(n / 2 + 1);
        gnv = lowprec() ? Bp : std::min(Bp, 8);
        // chunks grow with the vectors per pass, so this bounds every smaller call
        const int nchunk = lowprec() ? 1 : gemv_cols_chunks(m, N, gnv);
        U.ensure(sizeof(float) * Bp * Nn);
        F.ensure(sizeof(float) * Bp * mm);
        R.ensure(sizeof(float) * Bp * mm);
        P.ensure(sizeof(float) * (size_t)nchunk * Bp * Nn);
        RHS.ensure(sizeof(float) * Bp * Nn);
        Q0.ensure(sizeof(double) * 2 * B * Nn);
        Q1.ensure(sizeof(double) * 2 * B * Nn);
        S.ensure(sizeof(float2) * B * h * n);
        parts.ensure(sizeof(double) * 2 * B * (size_t)n);   // >= n / rows-per-block
        state.ensure(sizeof(ImgState) * B);
        obj.ensure(sizeof(double) * B);
        if (lowprec()) {
            lowp_work.ensure(lowp_work_bytes(lowp, Bp));
            lowp_work_bind(lw, lowp, Bp, lowp_work.p);
        }
        if (host_state_cap < B) {
            if (host_state) TVCS_HIP(hipHostFree(host_state));
            host_state = nullptr;
            TVCS_HIP(hipHostMalloc((void **)&host_state, sizeof(ImgState) * B));
            host_state_cap = B;
        }
        cap = B;
        capP = Bp;
        // padded images must hold zeros (their products are computed and ignored)
        launch_fill(U.as<float>(), (size_t)Bp * Nn, 0.f, work);
        launch_fill(F.as<float>(), (size_t)Bp * mm, 0.f, work);
    }

    // vectors per pass and row chunks of the FP32 products for a padded batch Bp
    int pass_nv(int Bp) const { return std::min(Bp, 8); }
    int chunks(int Bp) const { return gemv_cols_chunks(m, N, pass_nv(Bp)); }

    void ensure_denominators(double c) {
        const size_t cnt = (size_t)(n / 2 + 1) * n;
        invd.ensure(sizeof(double) * cnt);
        if (c != invd_c) {
            launch_denominators(n, c, invd.as<double>(), work);
            invd_c = c;
        }
    }

    // R = A U - F for the first Bp images (F may be null)
    void apply_A(int Bp, int B, const float *Uin, const float *Fin, float *Rout,
                 const ImgState *st) {
        if (lowprec()) {
            lowp_apply_A(lowp, lw, B, Uin, Fin, Rout, st, work);
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
    void apply_At(int Bp, int B, const float *Rin, const ImgState *st) {
        if (lowprec()) {
            lowp_apply_At(lowp, lw, B, Rin, P.as<float>(), st, work);
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
        apply_At(Bp, B, Rin, st);
        if (lowprec()) {
            TVCS_HIP(hipMemcpyAsync(out, P.p, sizeof(float) * (size_t)Bp * N,
                                    hipMemcpyDeviceToDevice, work));
            return;
        }
        const int nv = pass_nv(Bp), nchunk = chunks(Bp);
        const long long cs = (long long)nv * N;
        for (int g = 0; g * nv < Bp; ++g)
            launch_sum_partials(P.as<float>() + (size_t)g * nchunk * cs, nchunk, cs, nv, N,
                                out + (size_t)g * nv * N, N, work);
    }

    ShrinkArgs shrink_args(int B, int Bp) const {
        ShrinkArgs a{};
        a.n = n;
        a.B = B;
        a.U = U.as<float>();
        a.G = P.as<float>();
        if (lowprec()) {
            a.gnv = Bp;
            a.g_group_stride = 0;
            a.nchunk = 1;
            a.g_chunk_stride = 0;
        } else {
            const int nv = pass_nv(Bp), nchunk = chunks(Bp);
            a.gnv = nv;
            a.g_chunk_stride = (long long)nv * N;
            a.g_group_stride = (long long)nchunk * nv * N;
            a.nchunk = nchunk;
        }
        a.RHS = RHS.as<float>();
        a.st = state.as<ImgState>();
        return a;
    }

    void enqueue_iteration(int B, int parity, bool iadm, double beta, double c, double ctau) {
        const int Bp = padded(B);
        ImgState *st = state.as<ImgState>();
        apply_A(Bp, B, U.as<float>(), F.as<float>(), R.as<float>(), st);
        apply_At(Bp, B, R.as<float>(), st);
        ShrinkArgs a = shrink_args(B, Bp);
        a.beta = beta;
        a.c = c;
        a.ctau = ctau;
        a.Qold = parity ? Q1.as<double>() : Q0.as<double>();
        a.Qnew = parity ? Q0.as<double>() : Q1.as<double>();
        launch_shrink_rhs(a, iadm, work);
        const float2 *twp = tw.as<float2>();
        float2 *Sp = S.as<float2>();
        launch_fft_rows_fwd(n, B, RHS.as<float>(), Sp, twp, st, work);
        launch_fft_cols_solve(n, B, Sp, invd.as<double>(), twp, st, work);
        launch_fft_rows_inv(n, B, Sp, U.as<float>(), parts.as<double>(), twp, st, work);
        launch_finalize(st, parts.as<double>(), fft_row_parts(n, B), B, work);
    }

    void build_graph(int B, unsigned flags, double beta, double c, double ctau) {
        if (exec && g_B == B && g_flags == flags && g_beta == beta && g_c == c && g_ctau == ctau)
            return;
        if (exec) {
            TVCS_HIP(hipGraphExecDestroy(exec));
            exec = nullptr;
        }
        hipGraph_t graph = nullptr;
        TVCS_HIP(hipStreamBeginCapture(work, hipStreamCaptureModeRelaxed));
        try {
            for (int i = 0; i < kGraphIters; ++i)
                enqueue_iteration(B, i & 1, (flags & TVCS_IADM) != 0, beta, c, ctau);
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
        return A32.bytes + lowp_mem.bytes + tw.bytes + invd.bytes + U.bytes + F.bytes + R.bytes +
               P.bytes + RHS.bytes + Q0.bytes + Q1.bytes + S.bytes + parts.bytes + state.bytes +
               obj.bytes + lowp_work.bytes + lamb.bytes;
    }
};

namespace {

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

bool pow2_in_range(int n) { return n >= 8 && n <= kMaxN && (n & (n - 1)) == 0; }

int solve_impl(tvcs_ctx *h, const float *Fin, int B, double mu, double beta, double tol,
               int maxit, unsigned flags, float *Uout, double *lam, tvcs_stats *stats) {
    if (!h) fail(TVCS_EINVAL, "null handle");
    if (!Fin || !Uout) fail(TVCS_EINVAL, "f and u must not be NULL");
    if (B < 1) fail(TVCS_EINVAL, "batch size must be >= 1");
    if (!(mu > 0) || !(beta > 0) || !std::isfinite(mu) || !std::isfinite(beta))
        fail(TVCS_EINVAL, "mu and beta must be positive and finite");
    if (!(tol >= 0) || !std::isfinite(tol)) fail(TVCS_EINVAL, "tol must be >= 0");
    if (maxit < 1) fail(TVCS_EINVAL, "maxit must be >= 1");
    if (flags & ~(TVCS_IADM | TVCS_U0_ZERO | TVCS_OBJECTIVE | TVCS_WARM_START))
        fail(TVCS_EINVAL, "unknown flag bits");
    if ((flags & TVCS_U0_ZERO) && (flags & TVCS_WARM_START))
        fail(TVCS_EINVAL, "TVCS_U0_ZERO and TVCS_WARM_START exclude each other");
    const bool iadm = (flags & TVCS_IADM) != 0;

    h->begin_call();
    h->ensure_workspace(B);
    const int Bp = h->padded(B);
    const int N = h->N, m = h->m;
    const double tau = h->tau();
    const double c = mu / (beta * tau), ctau = mu / beta;
    TVCS_HIP(hipEventRecord(h->ev_t0, h->work));

    TVCS_HIP(hipMemcpyAsync(h->F.p, Fin, sizeof(float) * (size_t)B * m, hipMemcpyDefault,
                            h->work));
    h->ensure_denominators(c);
    ImgState *st = h->state.as<ImgState>();
    launch_init_state(st, B, tol, maxit, h->work);
    float *U = h->U.as<float>();
    const double *lam0 = nullptr;
    if (flags & TVCS_WARM_START) {
        TVCS_HIP(hipMemcpyAsync(U, Uout, sizeof(float) * (size_t)B * N, hipMemcpyDefault,
                                h->work));
        if (iadm && lam) {
            h->lamb.ensure(sizeof(double) * 2 * (size_t)B * N);
            TVCS_HIP(hipMemcpyAsync(h->lamb.p, lam, sizeof(double) * 2 * (size_t)B * N,
                                    hipMemcpyDefault, h->work));
            lam0 = h->lamb.as<double>();
        }
    } else if (flags & TVCS_U0_ZERO) {
        launch_fill(U, (size_t)B * N, 0.f, h->work);
    } else {
        h->apply_At_full(Bp, B, h->F.as<float>(), U, nullptr);   // u^0 = A^T f
    }
    if (iadm) launch_init_q(h->n, B, U, lam0, beta, h->Q0.as<double>(), h->work);

    h->build_graph(B, flags & TVCS_IADM, beta, c, ctau);
    const int launches = (maxit + kGraphIters - 1) / kGraphIters;
    for (int i = 0; i < launches; ++i) {
        TVCS_HIP(hipGraphLaunch(h->exec, h->work));
        if (tol > 0 && i + 1 < launches) {
            TVCS_HIP(hipMemcpyAsync(h->host_state, st, sizeof(ImgState) * B,
                                    hipMemcpyDeviceToHost, h->work));
            TVCS_HIP(hipStreamSynchronize(h->work));
            bool any = false;
            for (int b = 0; b < B; ++b) any |= h->host_state[b].active != 0;
            if (!any) break;
        }
    }

    if (iadm && lam) {
        // lambda^K = beta (D u^K - q^{K-1}); q^{K-1} sits in Q0 or Q1 by the image's
        // iteration parity
        h->lamb.ensure(sizeof(double) * 2 * (size_t)B * N);
        launch_lambda_out(h->n, B, U, h->Q0.as<double>(), h->Q1.as<double>(), st, beta,
                          h->lamb.as<double>(), h->work);
        TVCS_HIP(hipMemcpyAsync(lam, h->lamb.p, sizeof(double) * 2 * (size_t)B * N,
                                hipMemcpyDefault, h->work));
    }
    if (flags & TVCS_OBJECTIVE) {
        h->apply_A(Bp, B, U, h->F.as<float>(), h->R.as<float>(), nullptr);
        launch_objective(h->n, m, B, U, h->R.as<float>(), m, mu, h->obj.as<double>(), h->work);
    }
    TVCS_HIP(hipMemcpyAsync(Uout, U, sizeof(float) * (size_t)B * N, hipMemcpyDefault, h->work));
    TVCS_HIP(hipMemcpyAsync(h->host_state, st, sizeof(ImgState) * B, hipMemcpyDeviceToHost,
                            h->work));
    std::vector<double> objv(B, 0.0);
    if (flags & TVCS_OBJECTIVE)
        TVCS_HIP(hipMemcpyAsync(objv.data(), h->obj.p, sizeof(double) * B, hipMemcpyDeviceToHost,
                                h->work));
    TVCS_HIP(hipEventRecord(h->ev_t1, h->work));
    TVCS_HIP(hipStreamSynchronize(h->work));
    TVCS_HIP(hipGetLastError());
    float ms = 0.f;
    TVCS_HIP(hipEventElapsedTime(&ms, h->ev_t0, h->ev_t1));

    int rc = TVCS_OK;
    for (int b = 0; b < B; ++b) {
        const ImgState &s = h->host_state[b];
        if (s.status == TVCS_ENONFINITE)
            rc = TVCS_ENONFINITE;
        else if (s.status == TVCS_MAXIT && rc == TVCS_OK)
            rc = TVCS_MAXIT;
        if (stats) {
            stats[b].iters = s.iters;
            stats[b].status = s.status;
            stats[b].rel_change = s.rel;
            stats[b].objective = objv[b];
            stats[b].tau = tau;
            stats[b].ms = ms;
        }
    }
    if (rc == TVCS_ENONFINITE) g_last_error = "an iterate became NaN or Inf";
    return rc;
}

tvcs_ctx *create_impl(const void *A, int a_is_fp64, int m, int n, int storage, void *stream) {
    if (!A) fail(TVCS_EINVAL, "A must not be NULL");
    if (m < 1) fail(TVCS_EINVAL, "m must be >= 1");
    if (!pow2_in_range(n))
        fail(TVCS_EUNSUPPORTED, "n must be a power of two in [8, 512], got " + std::to_string(n));
    if (storage < TVCS_A_FP32 || storage > TVCS_A_FP8_ROWSCALE)
        fail(TVCS_EINVAL, "unknown storage format");
    std::unique_ptr<tvcs_ctx> h(new tvcs_ctx());
    h->m = m;
    h->n = n;
    h->N = n * n;
    h->storage = storage;
    h->user = static_cast<hipStream_t>(stream);
    TVCS_HIP(hipStreamCreateWithFlags(&h->work, hipStreamNonBlocking));
    TVCS_HIP(hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming));
    TVCS_HIP(hipEventCreate(&h->ev_t0));
    TVCS_HIP(hipEventCreate(&h->ev_t1));
    h->begin_call();

    const size_t cnt = (size_t)m * h->N;
    // A as FP32 on the device (rounded to nearest if given in FP64)
    DevBuf staging;
    float *A32dev = nullptr;
    if (a_is_fp64) {
        DevBuf a64;
        a64.ensure(sizeof(double) * cnt);
        TVCS_HIP(hipMemcpyAsync(a64.p, A, sizeof(double) * cnt, hipMemcpyDefault, h->work));
        (storage == TVCS_A_FP32 ? h->A32 : staging).ensure(sizeof(float) * cnt);
        A32dev = (storage == TVCS_A_FP32 ? h->A32 : staging).as<float>();
        launch_round_f64_f32(a64.as<double>(), A32dev, cnt, h->work);
        TVCS_HIP(hipStreamSynchronize(h->work));
    } else {
        (storage == TVCS_A_FP32 ? h->A32 : staging).ensure(sizeof(float) * cnt);
        A32dev = (storage == TVCS_A_FP32 ? h->A32 : staging).as<float>();
        TVCS_HIP(hipMemcpyAsync(A32dev, A, sizeof(float) * cnt, hipMemcpyDefault, h->work));
    }
    if (storage != TVCS_A_FP32) {
        h->lowp.storage = storage;
        h->lowp.m = m;
        h->lowp.N = h->N;
        h->lowp_mem.ensure(lowp_storage_bytes(h->lowp));
        lowp_bind_storage(h->lowp, h->lowp_mem.p);
        lowp_convert(h->lowp, A32dev, h->work);
        TVCS_HIP(hipStreamSynchronize(h->work));
        staging.release();
    }
    h->tw.ensure(sizeof(float2) * kMaxN);
    launch_twiddles(h->tw.as<float2>(), h->work);
    h->estimate_lambda_max();
    return h.release();
}

}  // namespace

extern "C" {

tvcs_handle tvcs_create(const float *A, int m, int n) {
    return tvcs_create_ex(A, 0, m, n, TVCS_A_FP32, nullptr);
}

tvcs_handle tvcs_create_ex(const void *A, int a_is_fp64, int m, int n, int storage,
                           void *stream) {
    tvcs_ctx *out = nullptr;
    const int rc = guarded([&] {
        out = create_impl(A, a_is_fp64, m, n, storage, stream);
        return TVCS_OK;
    });
    return rc == TVCS_OK ? out : nullptr;
}

int tvcs_set_stream(tvcs_handle h, void *stream) {
    return guarded([&] {
        if (!h) fail(TVCS_EINVAL, "null handle");
        h->user = static_cast<hipStream_t>(stream);
        return TVCS_OK;
    });
}

int tvcs_set_tau(tvcs_handle h, double tau) {
    return guarded([&] {
        if (!h) fail(TVCS_EINVAL, "null handle");
        if (!std::isfinite(tau)) fail(TVCS_EINVAL, "tau must be finite");
        h->tau_user = tau > 0 ? tau : 0.0;
        return TVCS_OK;
    });
}

double tvcs_get_tau(tvcs_handle h) {
    if (!h) {
        g_last_error = "null handle";
        return -1.0;
    }
    return h->tau();
}

double tvcs_lambda_max(tvcs_handle h) {
    if (!h) {
        g_last_error = "null handle";
        return -1.0;
    }
    return h->lmax;
}

size_t tvcs_device_bytes(tvcs_handle h) { return h ? h->device_bytes() : 0; }

int tvcs_solve(tvcs_handle h, const float *f, double mu, double beta, double tol, int maxit,
               unsigned flags, float *u, double *lambda, tvcs_stats *st) {
    return guarded([&] { return solve_impl(h, f, 1, mu, beta, tol, maxit, flags, u, lambda, st); });
}

int tvcs_solve_batch(tvcs_handle h, const float *F, int B, double mu, double beta, double tol,
                     int maxit, unsigned flags, float *U, double *lambda, tvcs_stats *st) {
    return guarded([&] { return solve_impl(h, F, B, mu, beta, tol, maxit, flags, U, lambda, st); });
}

int tvcs_time_products(tvcs_handle h, int B, int reps, float *ms_forward, float *ms_adjoint) {
    return guarded([&] {
        if (!h) fail(TVCS_EINVAL, "null handle");
        if (B < 1 || reps < 1) fail(TVCS_EINVAL, "B and reps must be >= 1");
        h->begin_call();
        h->ensure_workspace(B);
        const int Bp = h->padded(B);
        float *U = h->U.as<float>(), *F = h->F.as<float>(), *R = h->R.as<float>();
        // warm-up launch of each, then the timed runs
        h->apply_A(Bp, B, U, F, R, nullptr);
        h->apply_At(Bp, B, R, nullptr);
        TVCS_HIP(hipEventRecord(h->ev_t0, h->work));
        for (int i = 0; i < reps; ++i) h->apply_A(Bp, B, U, F, R, nullptr);
        TVCS_HIP(hipEventRecord(h->ev_t1, h->work));
        TVCS_HIP(hipEventSynchronize(h->ev_t1));
        float ms = 0.f;
        TVCS_HIP(hipEventElapsedTime(&ms, h->ev_t0, h->ev_t1));
        if (ms_forward) *ms_forward = ms / reps;
        TVCS_HIP(hipEventRecord(h->ev_t0, h->work));
        for (int i = 0; i < reps; ++i) h->apply_At(Bp, B, R, nullptr);
        TVCS_HIP(hipEventRecord(h->ev_t1, h->work));
        TVCS_HIP(hipEventSynchronize(h->ev_t1));
        TVCS_HIP(hipEventElapsedTime(&ms, h->ev_t0, h->ev_t1));
        if (ms_adjoint) *ms_adjoint = ms / reps;
        TVCS_HIP(hipGetLastError());
        return TVCS_OK;
    });
}

void tvcs_destroy(tvcs_handle h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->work);
    delete h;
}

const char *tvcs_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
