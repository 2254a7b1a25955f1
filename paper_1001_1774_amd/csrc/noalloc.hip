// tvcs_solve_noalloc: the single-image solve of tvcs_solve (FP32 storage of A)
// for callers that cannot allocate device memory.  Every per-solve buffer (u, f,
// r, the A^T r partial sums (or, for n^2 <= 16384, the band partials of the
// one-pass product and g), the two q fields, the half spectrum, the stop-rule
// partials, the FFT denominators, the image state) lives in one file-scope device
// array of kScratchBytes; the iteration's kernels are launched directly (no
// captured graph, no pinned host memory).  The array's device address is taken
// once per device with hipGetSymbolAddress.  Calls on one GPU share its array:
// calls that overlap on one GPU race, and each call rewrites every part of the
// array it reads before reading it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <mutex>

#include "solver.h"

namespace {

constexpr size_t kScratchBytes = 32u << 20;   // 32 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// the device address of this device's array (taken on the first call on the device)
unsigned char *scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices) fail(TVCS_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            fail(TVCS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = p;
    }
    return static_cast<unsigned char *>(g_scratch_ptr[device]);
}

// carve the per-solve buffers out of the array, 256-byte aligned
struct Carve {
    unsigned char *base;
    size_t used = 0;
    template <class T>
    T *take(size_t count) {
        T *p = reinterpret_cast<T *>(base + used);
        used += (count * sizeof(T) + 255) / 256 * 256;
        return p;
    }
};

struct Work {
    float *U, *F, *R, *P;
    float2 *Q0, *Q1, *S;
    double *parts, *invd, *obj;
    ImgState *st;
    int *counters;
};

Work carve(unsigned char *base, int n, int m, int nchunk, size_t &bytes) {
    const size_t N = (size_t)n * n, h = (size_t)(n / 2 + 1);
    Carve c{base};
    Work w;
    w.U = c.take<float>(N);
    w.F = c.take<float>(m);
    w.R = c.take<float>(m);
    w.P = c.take<float>((size_t)nchunk * N);
    w.Q0 = c.take<float2>(N);
    w.Q1 = c.take<float2>(N);
    w.S = c.take<float2>(h * n);
    w.parts = c.take<double>(2 * (size_t)n);
    w.invd = c.take<double>(h * n);
    w.obj = c.take<double>(1);
    w.st = c.take<ImgState>(1);
    w.counters = c.take<int>(1);
    bytes = c.used;
    return w;
}

int solve_noalloc_impl(tvcs_ctx *h, const float *f, double mu, double beta, double tol,
                       int maxit, unsigned flags, float *u, tvcs_stats *stats) {
    if (!h) fail(TVCS_EINVAL, "null handle");
    if (!f || !u) fail(TVCS_EINVAL, "f and u must not be NULL");
    if (!(mu > 0) || !(beta > 0) || !std::isfinite(mu) || !std::isfinite(beta))
        fail(TVCS_EINVAL, "mu and beta must be positive and finite");
    if (!(tol >= 0) || !std::isfinite(tol)) fail(TVCS_EINVAL, "tol must be >= 0");
    if (maxit < 1) fail(TVCS_EINVAL, "maxit must be >= 1");
    if (flags & ~(TVCS_IADM | TVCS_U0_ZERO | TVCS_OBJECTIVE | TVCS_WARM_START))
        fail(TVCS_EINVAL, "unknown flag bits");
    if ((flags & TVCS_U0_ZERO) && (flags & TVCS_WARM_START))
        fail(TVCS_EINVAL, "TVCS_U0_ZERO and TVCS_WARM_START exclude each other");
    if (h->storage != TVCS_A_FP32)
        fail(TVCS_EUNSUPPORTED, "tvcs_solve_noalloc takes handles with FP32 storage of A");
    int dev = -1;
    TVCS_HIP(hipGetDevice(&dev));
    if (dev != h->device)
        fail(TVCS_EINVAL, "the current device is not the one the handle was created on");
    const int n = h->n, m = h->m, N = h->N;
    const int nchunk = gemv_cols_chunks(m, N);
    // the one-pass product (as tvcs_solve takes it for one image): nb band partials
    // of g, then g, in the partial-sum buffer
    const int nb = TVCS_FUSED_PASS ? fused_bands(m, N) : 0;
    const int pslots = std::max(nchunk, nb > 0 ? nb + 1 : 0);
    size_t need = 0;
    (void)carve(nullptr, n, m, pslots, need);
    if (need > kScratchBytes)
        fail(TVCS_EINVAL, "tvcs_solve_noalloc: this problem's workspace is " +
                              std::to_string(need) + " bytes, beyond the " +
                              std::to_string(kScratchBytes) + "-byte scratch array");
    size_t used = 0;
    const Work w = carve(scratch_on(dev), n, m, pslots, used);
    const bool iadm = (flags & TVCS_IADM) != 0;
    const double tau = h->tau();
    const double c = mu / (beta * tau), ctau = mu / beta;
    hipStream_t s = h->work;
    const auto t0 = std::chrono::steady_clock::now();

    h->begin_call();
    TVCS_HIP(hipMemcpyAsync(w.F, f, sizeof(float) * m, hipMemcpyDefault, s));
    launch_denominators(n, c, w.invd, s);
    launch_init_state(w.st, 1, tol, maxit, s);
    launch_fill(reinterpret_cast<float *>(w.counters), 1, 0.f, s);   // all-zero bits
    if (flags & TVCS_WARM_START) {
        TVCS_HIP(hipMemcpyAsync(w.U, u, sizeof(float) * N, hipMemcpyDefault, s));
    } else if (flags & TVCS_U0_ZERO) {
        launch_fill(w.U, (size_t)N, 0.f, s);
    } else {   // u^0 = A^T f
        launch_gemv_cols(h->A32.as<float>(), m, N, w.F, m, w.P, N, 1, nullptr, 1, s);
        launch_sum_partials(w.P, nchunk, N, 1, N, w.U, N, s);
    }
    if (iadm) launch_init_q(n, 1, w.U, nullptr, beta, w.Q0, s);

    ShrinkArgs a{};
    a.n = n;
    a.B = 1;
    a.U = w.U;
    a.G = nb > 0 ? w.P + (size_t)nb * N : w.P;
    a.gnv = 1;
    a.g_chunk_stride = N;
    a.g_group_stride = nb > 0 ? (long long)N : (long long)nchunk * N;
    a.nchunk = nb > 0 ? 1 : nchunk;
    a.beta = beta;
    a.c = c;
    a.ctau = ctau;
    a.st = w.st;
    a.Gacc = nullptr;
    const float2 *tw = h->tw.as<float2>();
    ImgState hs{};
    for (int k = 0; k < maxit; ++k) {
        const int parity = k & 1;
        if (nb > 0) {
            launch_gemv_fused(h->A32.as<float>(), m, N, w.U, w.F, w.P, w.P + (size_t)nb * N, w.st,
                              parity & TVCS_FUSED_REV, s);
        } else {
            launch_gemv_rows(h->A32.as<float>(), m, N, w.U, N, w.F, m, w.R, m, 1, w.st, 1, s);
            launch_gemv_cols(h->A32.as<float>(), m, N, w.R, m, w.P, N, 1, w.st, 1, s);
        }
        a.Qold = parity ? w.Q1 : w.Q0;
        a.Qnew = parity ? w.Q0 : w.Q1;
        a.parity = parity;
        launch_shrink_rows(a, iadm, w.S, tw, s);
        launch_fft_cols_solve(n, 1, w.S, w.invd, tw, w.st, s);
        launch_fft_rows_inv(n, 1, w.S, w.U, w.parts, tw, w.st, w.counters, s, nullptr, nullptr,
                            true, parity);
        // with a tolerance, look at the stop flag every 10 iterations (the kernels of
        // a stopped image return at entry meanwhile)
        if (tol > 0 && (k + 1) % 10 == 0 && k + 1 < maxit) {
            TVCS_HIP(hipMemcpyAsync(&hs, w.st, sizeof(ImgState), hipMemcpyDeviceToHost, s));
            TVCS_HIP(hipStreamSynchronize(s));
            if (!hs.active) break;
        }
    }
    if (flags & TVCS_OBJECTIVE) {
        launch_gemv_rows(h->A32.as<float>(), m, N, w.U, N, w.F, m, w.R, m, 1, nullptr, 1, s);
        launch_objective(n, m, 1, w.U, w.R, m, mu, w.obj, s);
    }
    double objv = 0.0;
    TVCS_HIP(hipMemcpyAsync(u, w.U, sizeof(float) * N, hipMemcpyDefault, s));
    TVCS_HIP(hipMemcpyAsync(&hs, w.st, sizeof(ImgState), hipMemcpyDeviceToHost, s));
    if (flags & TVCS_OBJECTIVE)
        TVCS_HIP(hipMemcpyAsync(&objv, w.obj, sizeof(double), hipMemcpyDeviceToHost, s));
    TVCS_HIP(hipStreamSynchronize(s));
    TVCS_HIP(hipGetLastError());
    const float ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    int rc = hs.status == TVCS_ENONFINITE ? TVCS_ENONFINITE
             : hs.status == TVCS_MAXIT    ? TVCS_MAXIT
                                          : TVCS_OK;
    if (stats) {
        stats->iters = hs.iters;
        stats->status = hs.status;
        stats->rel_change = hs.rel;
        stats->objective = objv;
        stats->tau = tau;
        stats->ms = ms;
        stats->fresh_iters = 0;
        for (int i = 0; i < 6; ++i) stats->tiles[i] = 0;
    }
    if (rc == TVCS_ENONFINITE) g_last_error = "an iterate became NaN or Inf";
    return rc;
}

}  // namespace

extern "C" {

int tvcs_solve_noalloc(tvcs_handle h, const float *f, double mu, double beta, double tol,
                       int maxit, unsigned flags, float *u, tvcs_stats *st) {
    return guarded([&] { return solve_noalloc_impl(h, f, mu, beta, tol, maxit, flags, u, st); });
}

}  // extern "C"
