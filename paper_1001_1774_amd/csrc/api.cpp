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

#include "solver.h"

namespace tvcs {

thread_local std::string g_last_error;

[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }

}  // namespace tvcs


namespace {

int solve_impl(tvcs_ctx *h, const float *Fin, int B, double mu, double beta, double tol,
               int maxit, unsigned flags, float *Uout, double *lam, tvcs_stats *stats) {
    if (!h) fail(TVCS_EINVAL, "null handle");
    if (!Fin || !Uout) fail(TVCS_EINVAL, "f and u must not be NULL");
    if (B < 1) fail(TVCS_EINVAL, "batch size must be >= 1");
    if (!(mu > 0) || !(beta > 0) || !std::isfinite(mu) || !std::isfinite(beta))
        fail(TVCS_EINVAL, "mu and beta must be positive and finite");
    if (!(tol >= 0) || !std::isfinite(tol)) fail(TVCS_EINVAL, "tol must be >= 0");
    if (maxit < 1) fail(TVCS_EINVAL, "maxit must be >= 1");
    if (flags & ~(TVCS_IADM | TVCS_U0_ZERO | TVCS_OBJECTIVE | TVCS_WARM_START | TVCS_BB_STEPS(15)))
        fail(TVCS_EINVAL, "unknown flag bits");
    if ((flags & TVCS_U0_ZERO) && (flags & TVCS_WARM_START))
        fail(TVCS_EINVAL, "TVCS_U0_ZERO and TVCS_WARM_START exclude each other");
    const bool iadm = (flags & TVCS_IADM) != 0;
    if (bb_inner(flags) > 1) {
        if (!iadm) fail(TVCS_EINVAL, "inner steps on the u-subproblem need TVCS_IADM");
        if (h->dct())
            fail(TVCS_EUNSUPPORTED, "inner steps on the u-subproblem take a stored matrix A");
    }

    h->begin_call();
    h->ensure_workspace(B);
    const int Bp = h->padded(B);
    const int N = h->N, m = h->m;
    const double tau = h->tau();
    const double c = mu / (beta * tau), ctau = mu / beta;
    TVCS_HIP(hipEventRecord(h->ev_t0, h->work));

    h->load_measurements(Fin, 0, B);
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
    if (iadm) launch_init_q(h->n, B, U, lam0, beta, h->Q0.as<float2>(), h->work);
    h->seed_dct_rows(B);

    h->build_graph(B, flags & (TVCS_IADM | TVCS_BB_STEPS(15)), beta, c, ctau);
    const int launches = (maxit + kGraphIters - 1) / kGraphIters;
    if (tol > 0) {
        // The state after launch i is copied into one half of the pinned mirror and
        // read while launch i + 1 runs, so the device never waits for the host; a
        // launch queued after every image has stopped finds them all inactive and
        // each of its kernels returns at once.
        for (hipEvent_t &e : h->ev_poll)
            if (!e) TVCS_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        for (int i = 0; i < launches; ++i) {
            TVCS_HIP(hipGraphLaunch(h->exec, h->work));
            if (i + 1 == launches) break;
            TVCS_HIP(hipMemcpyAsync(h->host_state + (size_t)(i & 1) * B, st,
                                    sizeof(ImgState) * B, hipMemcpyDeviceToHost, h->work));
            TVCS_HIP(hipEventRecord(h->ev_poll[i & 1], h->work));
            if (i == 0) continue;
            TVCS_HIP(hipEventSynchronize(h->ev_poll[(i - 1) & 1]));
            const ImgState *prev = h->host_state + (size_t)((i - 1) & 1) * B;
            bool any = false;
            for (int b = 0; b < B; ++b) any |= prev[b].active != 0;
            if (!any) break;
        }
    } else {
        for (int i = 0; i < launches; ++i) TVCS_HIP(hipGraphLaunch(h->exec, h->work));
    }

    if (iadm && lam) {
        // lambda^K = beta (D u^K - q^{K-1}); q^{K-1} sits in Q0 or Q1 by the image's
        // iteration parity
        h->lamb.ensure(sizeof(double) * 2 * (size_t)B * N);
        launch_lambda_out(h->n, B, U, h->Q0.as<float2>(), h->Q1.as<float2>(), st, beta,
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
            // with inner steps every product is fresh (two-part batch operand)
            stats[b].fresh_iters = !h->lowprec() ? 0 : bb_inner(flags) > 1 ? s.iters : s.fresh;
            h->tiles_out(stats[b].tiles);
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
    if (!supported_side(n))
        fail(TVCS_EUNSUPPORTED, "n must be even, in [8, 512], with no prime factor other than "
                                 "2, 3 and 5, got " + std::to_string(n));
    if (storage == TVCS_A_PARTIAL_DCT)
        fail(TVCS_EINVAL, "the partial-DCT operator is created with tvcs_create_dct");
    if (storage < TVCS_A_FP32 || storage > TVCS_A_FP8_ROWSCALE)
        fail(TVCS_EINVAL, "unknown storage format");
    if (storage != TVCS_A_FP32 && n < 16)
        fail(TVCS_EUNSUPPORTED, "low-precision storage needs n >= 16");
    std::unique_ptr<tvcs_ctx> h(new tvcs_ctx());
    h->m = m;
    h->n = n;
    h->N = n * n;
    h->storage = storage;
    TVCS_HIP(hipGetDevice(&h->device));
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
    launch_twiddles(n, h->tw.as<float2>(), h->work);
    h->estimate_lambda_max();
    return h.release();
}

tvcs_ctx *create_dct_impl(const int *rows, int m, int n, void *stream) {
    if (!rows) fail(TVCS_EINVAL, "rows must not be NULL");
    if (!supported_side(n))
        fail(TVCS_EUNSUPPORTED, "n must be even, in [8, 512], with no prime factor other than "
                                 "2, 3 and 5, got " + std::to_string(n));
    const int N = n * n;
    if (m < 1 || m > N) fail(TVCS_EINVAL, "m must be in [1, n*n]");
    // which[k_c * n + k_r] = i for rows[i] = k_r * n + k_c, -1 if not measured
    std::vector<int> which((size_t)N, -1);
    for (int i = 0; i < m; ++i) {
        const int p = rows[i];
        if (p < 0 || p >= N)
            fail(TVCS_EINVAL, "rows[" + std::to_string(i) + "] = " + std::to_string(p) +
                                  " is outside [0, n*n)");
        int &slot = which[(size_t)(p % n) * n + p / n];
        if (slot >= 0) fail(TVCS_EINVAL, "coefficient " + std::to_string(p) + " is repeated");
        slot = i;
    }
    // positions in the column pass's order (k_c-major): selT[q] = position of
    // coefficient q, perm[position] = measurement index
    std::vector<int> selT((size_t)N, -1), perm((size_t)m);
    for (int q = 0, j = 0; q < N; ++q)
        if (which[q] >= 0) {
            selT[q] = j;
            perm[j++] = which[q];
        }
    std::unique_ptr<tvcs_ctx> h(new tvcs_ctx());
    h->m = m;
    h->n = n;
    h->N = N;
    h->storage = TVCS_A_PARTIAL_DCT;
    TVCS_HIP(hipGetDevice(&h->device));
    h->user = static_cast<hipStream_t>(stream);
    TVCS_HIP(hipStreamCreateWithFlags(&h->work, hipStreamNonBlocking));
    TVCS_HIP(hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming));
    TVCS_HIP(hipEventCreate(&h->ev_t0));
    TVCS_HIP(hipEventCreate(&h->ev_t1));
    h->begin_call();
    h->selT.ensure(sizeof(int) * (size_t)N);
    TVCS_HIP(hipMemcpyAsync(h->selT.p, selT.data(), sizeof(int) * (size_t)N, hipMemcpyHostToDevice,
                            h->work));
    h->dperm.ensure(sizeof(int) * (size_t)m);
    TVCS_HIP(hipMemcpyAsync(h->dperm.p, perm.data(), sizeof(int) * (size_t)m,
                            hipMemcpyHostToDevice, h->work));
    h->dtab.ensure(sizeof(float4) * (size_t)n);
    launch_dct_table(n, h->dtab.as<float4>(), h->work);
    h->tw.ensure(sizeof(float2) * kMaxN);
    launch_twiddles(n, h->tw.as<float2>(), h->work);
    h->estimate_lambda_max();
    TVCS_HIP(hipStreamSynchronize(h->work));   // the host tables go out of scope
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

tvcs_handle tvcs_create_dct(const int *rows, int m, int n, void *stream) {
    tvcs_ctx *out = nullptr;
    const int rc = guarded([&] {
        out = create_dct_impl(rows, m, n, stream);
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

int tvcs_solve_continuation(tvcs_handle h, const float *F, int B, double mu,
                            const double *betas, int nbeta, double tol, int maxit,
                            unsigned flags, float *U, tvcs_stats *st) {
    return guarded([&] {
        if (!betas || nbeta < 1) fail(TVCS_EINVAL, "betas must hold nbeta >= 1 values");
        for (int k = 0; k < nbeta; ++k)
            if (!(betas[k] > 0) || !std::isfinite(betas[k]))
                fail(TVCS_EINVAL, "every beta must be positive and finite");
        if (flags & TVCS_IADM)
            fail(TVCS_EINVAL, "continuation in beta is defined for FTVCS (Algorithm 1)");
        if (flags & ~(TVCS_U0_ZERO | TVCS_OBJECTIVE | TVCS_WARM_START))
            fail(TVCS_EINVAL, "unknown flag bits");
        if (B < 1) fail(TVCS_EINVAL, "batch size must be >= 1");
        std::vector<tvcs_stats> stage((size_t)B);
        std::vector<int> total((size_t)B, 0);
        std::vector<float> ms((size_t)B, 0.f);
        int rc = TVCS_OK;
        for (int k = 0; k < nbeta; ++k) {
            // first stage: the caller's start; later stages: warm start from U
            unsigned f = k == 0 ? (flags & (TVCS_U0_ZERO | TVCS_WARM_START)) : TVCS_WARM_START;
            if (k == nbeta - 1) f |= flags & TVCS_OBJECTIVE;
            const int r = solve_impl(h, F, B, mu, betas[k], tol, maxit, f, U, nullptr,
                                     stage.data());
            if (r < 0) return r;
            if (r == TVCS_MAXIT) rc = TVCS_MAXIT;
            for (int b = 0; b < B; ++b) {
                total[b] += stage[b].iters;
                ms[b] += stage[b].ms;
            }
        }
        if (st)
            for (int b = 0; b < B; ++b) {
                st[b] = stage[b];
                st[b].iters = total[b];
                st[b].ms = ms[b];
            }
        return rc;
    });
}

int tvcs_time_products(tvcs_handle h, int B, int reps, int form, float *ms_forward,
                       float *ms_adjoint) {
    return guarded([&] {
        if (!h) fail(TVCS_EINVAL, "null handle");
        if (B < 1 || reps < 1) fail(TVCS_EINVAL, "B and reps must be >= 1");
        if (form != 0 && form != 1) fail(TVCS_EINVAL, "form must be 0 (fresh) or 1 (increment)");
        h->begin_call();
        h->ensure_workspace(B);
        const int Bp = h->padded(B);
        float *U = h->U.as<float>(), *F = h->F.as<float>(), *R = h->R.as<float>();
        ImgState *st = h->state.as<ImgState>();
        // inputs like a solve's: u and f of unit size with hashed (nonzero, unstructured)
        // entries, since MFMA clocks depend on the operands' bits.  One fresh pair of
        // products sets the vectors the increments are taken from; u then moves by
        // 2^-10 of its size, so the increment operands are nonzero (after the warm-up
        // launch, the rounding residuals of that move), and every image takes the
        // requested form (mode slot 0, parity 0)
        launch_fill_hash(U, (size_t)B * h->N, 1u, 1.0f, false, h->work);
        launch_fill_hash(F, (size_t)B * h->m, 2u, 1.0f, false, h->work);
        launch_init_state(st, B, 0.0, 1, h->work, 1);
        h->apply_A(Bp, B, U, F, R, st, 0);
        h->apply_At(Bp, B, R, st, 0);
        launch_fill_hash(U, (size_t)B * h->N, 3u, 1.0f / 1024.0f, true, h->work);
        launch_init_state(st, B, 0.0, 1, h->work, form ? 0 : 1);
        // warm-up launch of each, then the timed runs.  In the increment form each
        // timed launch follows (outside its timed span) a move of its input by 2^-10
        // of its size, as between two iterations: otherwise the increments of
        // repeated launches on one input round to zero after a few launches.
        const bool incr = form == 1 && h->lowprec();
        h->apply_A(Bp, B, U, F, R, st, 0);
        h->apply_At(Bp, B, R, st, 0);
        auto timed = [&](auto &&op, float *moved, size_t count) {
            float total = 0.f, ms = 0.f;
            if (!incr) {
                TVCS_HIP(hipEventRecord(h->ev_t0, h->work));
                for (int i = 0; i < reps; ++i) op();
                TVCS_HIP(hipEventRecord(h->ev_t1, h->work));
                TVCS_HIP(hipEventSynchronize(h->ev_t1));
                TVCS_HIP(hipEventElapsedTime(&total, h->ev_t0, h->ev_t1));
                return total / reps;
            }
            for (int i = 0; i < reps; ++i) {
                launch_fill_hash(moved, count, 16u + (unsigned)i, 1.0f / 1024.0f, true, h->work);
                TVCS_HIP(hipEventRecord(h->ev_t0, h->work));
                op();
                TVCS_HIP(hipEventRecord(h->ev_t1, h->work));
                TVCS_HIP(hipEventSynchronize(h->ev_t1));
                TVCS_HIP(hipEventElapsedTime(&ms, h->ev_t0, h->ev_t1));
                total += ms;
            }
            return total / reps;
        };
        const float msf = timed([&] { h->apply_A(Bp, B, U, F, R, st, 0); }, U, (size_t)B * h->N);
        if (ms_forward) *ms_forward = msf;
        const float msa = timed([&] { h->apply_At(Bp, B, R, st, 0); }, R, (size_t)B * h->m);
        if (ms_adjoint) *ms_adjoint = msa;
        TVCS_HIP(hipGetLastError());
        return TVCS_OK;
    });
}

int tvcs_time_fused(tvcs_handle h, int reps, float *ms_pass, float *ms_sum) {
    return guarded([&] {
        if (!h) fail(TVCS_EINVAL, "null handle");
        if (reps < 1) fail(TVCS_EINVAL, "reps must be >= 1");
        if (!h->fused())
            fail(TVCS_EUNSUPPORTED, "the one-pass product takes FP32 storage with n*n <= 16384");
        h->begin_call();
        h->ensure_workspace(1);
        float *U = h->U.as<float>(), *F = h->F.as<float>(), *PF = h->PF.as<float>();
        ImgState *st = h->state.as<ImgState>();
        const int nb = fused_bands(h->m, h->N);
        float *G = PF + (size_t)nb * h->N;
        launch_fill_hash(U, (size_t)h->N, 1u, 1.0f, false, h->work);
        launch_fill_hash(F, (size_t)h->m, 2u, 1.0f, false, h->work);
        launch_init_state(st, 1, 0.0, 1, h->work, 1);
        auto timed = [&](auto &&op) {
            op();   // warm-up
            float total = 0.f;
            TVCS_HIP(hipEventRecord(h->ev_t0, h->work));
            for (int i = 0; i < reps; ++i) op();
            TVCS_HIP(hipEventRecord(h->ev_t1, h->work));
            TVCS_HIP(hipEventSynchronize(h->ev_t1));
            TVCS_HIP(hipEventElapsedTime(&total, h->ev_t0, h->ev_t1));
            return total / reps;
        };
        // the row order alternates from launch to launch, as in the solve loop; the
        // band sum is timed behind its pass (the difference of the two loops), where
        // it reads partials the pass has just written, not ones already in cache
        int rev = 0;
        const float mp = timed([&] {
            launch_gemv_fused(h->A32.as<float>(), h->m, h->N, U, F, PF, nullptr, st,
                              rev & TVCS_FUSED_REV, h->work);
            rev ^= 1;
        });
        const float mboth = timed([&] {
            launch_gemv_fused(h->A32.as<float>(), h->m, h->N, U, F, PF, G, st,
                              rev & TVCS_FUSED_REV, h->work);
            rev ^= 1;
        });
        if (ms_pass) *ms_pass = mp;
        if (ms_sum) *ms_sum = std::max(0.f, mboth - mp);
        TVCS_HIP(hipGetLastError());
        return TVCS_OK;
    });
}

int tvcs_set_tiles(tvcs_handle h, const int *tiles) {
    return guarded([&] {
        if (!h) fail(TVCS_EINVAL, "null handle");
        if (!h->lowprec()) fail(TVCS_EUNSUPPORTED, "tile shapes exist for MFMA storage only");
        TileCfg c[2];
        if (tiles) {
            for (int k = 0; k < 2; ++k) {
                const int rt = tiles[3 * k], img = tiles[3 * k + 1], kf = tiles[3 * k + 2];
                c[k] = TileCfg{rt, img / 16, -1};
                if (img % 16 != 0) fail(TVCS_EINVAL, "images per group: 16, 32, 64, 128 or 256");
                if (img >= 16 && img <= 256)
                    for (int v = 1; v >= 0; --v)
                        if (tile_kf(c[k].nt, v) == kf) c[k].kfv = v;
                if (c[k].kfv < 0 || !tile_valid(c[k]))
                    fail(TVCS_EINVAL, "no such tile shape (rt 2 or 4, 4 not with 256 images; "
                                      "k tiles per step from the shape's two tables)");
            }
        }
        h->begin_call();
        if (h->exec) {   // the captured iterations hold the old shapes
            TVCS_HIP(hipGraphExecDestroy(h->exec));
            h->exec = nullptr;
        }
        h->tiles_forced = tiles != nullptr;
        if (tiles) {
            h->forced_fwd = c[0];
            h->forced_adj = c[1];
            if (h->capP) {
                h->lw.fwd = c[0];
                h->lw.adj = c[1];
            }
        } else if (h->capP) {
            lowp_autotune(h->lowp, h->lw, h->capP, h->U.as<float>(), h->R.as<float>(),
                          h->P.as<float>(), h->state.as<ImgState>(), h->work);
            launch_fill(h->U.as<float>(), (size_t)h->capP * h->N, 0.f, h->work);
        }
        TVCS_HIP(hipStreamSynchronize(h->work));
        return TVCS_OK;
    });
}

int tvcs_get_tiles(tvcs_handle h, int *tiles) {
    return guarded([&] {
        if (!h || !tiles) fail(TVCS_EINVAL, "null argument");
        h->tiles_out(tiles);
        return TVCS_OK;
    });
}

int tvcs_measure_peaks(size_t bytes, int reps, double *read_gbs, double *mfma_tflops) {
    return guarded([&] {
        if (bytes < ((size_t)1 << 20) || reps < 1)
            fail(TVCS_EINVAL, "bytes must be >= 1 MiB and reps >= 1");
        measure_peaks(bytes, reps, read_gbs, mfma_tflops);
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
