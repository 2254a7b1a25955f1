/*
 * tvcs.h -- C ABI of the MI355X (gfx950) library for total-variation image
 * reconstruction from dense random projections.
 *
 * The library solves, for an n x n image u (row-major, pixel r*n + c) observed
 * through a dense m x n^2 matrix A as f = A u + noise (Sec. 1, eq. (obser)),
 *
 *     min_u  sum_i ||D_i u||_2 + mu/2 ||A u - f||_2^2             (eq. (tv))
 *
 * with the alternating minimisation of Algorithm 1 (FTVCS: shrinkage eq.
 * (shrink), linearised-proximal u-step eq. (eqnorm)) or the accelerated
 * inexact ADM of Algorithm 2 (IADM: eqs. (iadmw), (eqnorm11), (udlamb)).
 * D_i are forward differences with periodic boundary conditions, so each
 * u-step is solved exactly by a forward and an inverse 2-D FFT (Sec. 2.1).
 * Every iteration costs two dense products (A u, A^T r), one shrinkage and
 * two FFTs, all of them hand-written HIP kernels.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * - Pointers may be host or device memory of the calling process (the library
 *   copies with hipMemcpyDefault).  Input buffers are only read during the call;
 *   output buffers are written before the call returns.
 * - All calls are synchronous for the host: they return after the device work
 *   they enqueue has finished.  Work is ordered after everything already
 *   enqueued on the handle's stream (see tvcs_set_stream).
 * - Return codes: TVCS_OK (0) on success, TVCS_MAXIT (1) when a tolerance was
 *   given and not met within maxit iterations (outputs are still valid), and a
 *   negative TVCS_E* code on error, with a message from tvcs_last_error().
 * - One call per handle at a time; different handles are independent.
 */
#ifndef TVCS_H
#define TVCS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes -------------------------------------------------------- */
#define TVCS_OK            0
#define TVCS_MAXIT         1   /* tol > 0 was not met within maxit: outputs valid   */
#define TVCS_EINVAL       -1   /* bad argument (NULL, size, non-positive parameter) */
#define TVCS_ENOMEM       -2   /* device allocation failed / HBM budget exceeded    */
#define TVCS_EDEVICE      -3   /* HIP runtime error                                 */
#define TVCS_ENONFINITE   -4   /* NaN or Inf appeared in an iterate                 */
#define TVCS_EUNSUPPORTED -5   /* image side or storage format not supported        */

/* ---- solve flags --------------------------------------------------------- */
/* Algorithm 2 (IADM) instead of Algorithm 1 (FTVCS). */
#define TVCS_IADM     0x1u
/* Start from u^0 = 0 instead of u^0 = A^T f.  (Alg. 1 and 2 print "u^0 = f",
 * which has the wrong length; A^T f is the default reading.) */
#define TVCS_U0_ZERO  0x2u
/* Compute stats.objective (one extra product with A and a TV sum). */
#define TVCS_OBJECTIVE 0x4u
/* Warm start: on entry u holds u^0 and, with TVCS_IADM and a non-NULL lambda,
 * lambda holds lambda^0 (otherwise lambda^0 = 0).  Used to continue a run, e.g.
 * across the stages of a continuation in beta (Sec. 3.1). */
#define TVCS_WARM_START 0x8u
/* IADM (with TVCS_IADM) whose u-step is J inner steps (2 <= J <= 15) on the
 * u-subproblem of (ALP) instead of one: the acceleration the concluding remarks
 * (Sec. 4) suggest, a gradient method with Barzilai-Borwein step lengths and a
 * non-monotone line search.  With q = w^{k+1} - lambda^k / beta fixed, the
 * subproblem is Phi(v) = beta/2 ||q - D v||^2 + mu/2 ||A v - f||^2; each step goes
 * along p = -M^{-1} grad Phi (M = beta D^T D + (mu / tau) I, one FFT solve), the
 * first with length 1 (the IADM step), later ones with the BB length
 * p'M p / p'H p of the previous direction (H = beta D^T D + mu A^T A), halved until
 * Phi(v + a p) <= max of the last 5 accepted values + 1e-4 a grad'p (Phi along the
 * line is an exact quadratic).  Each inner step costs two products with A (A^T r
 * and A p; r is carried).  The stop rule compares outer iterates; stats.iters
 * counts outer iterations.  Any stored A (with bf16, split bf16 or FP8 storage
 * every product is computed afresh from a two-part batch operand, and
 * stats.fresh_iters equals stats.iters); TVCS_EUNSUPPORTED for the partial DCT. */
#define TVCS_BB_SHIFT 8
#define TVCS_BB_STEPS(J) (((unsigned)(J) & 0xFu) << TVCS_BB_SHIFT)

/* ---- storage of A on the device ------------------------------------------ */
/* A is first rounded to FP32 (nearest-even), then to the storage format.    */
#define TVCS_A_FP32          0  /* FP32, 4 bytes/entry; FP32 GEMV kernels           */
#define TVCS_A_BF16          1  /* bf16(A), 2 bytes/entry; MFMA with FP32 accumulate.
                                   For this and the next two formats an image's
                                   products are computed afresh (batch operand v split
                                   into bf16 hi + lo) while its relative change
                                   exceeds 2^-8 and every 64th iteration, and
                                   otherwise as increments: r += A bf16(u - u~) and
                                   g += A^T bf16(v - v~) for v the residual, u~ and v~
                                   being the vectors the current r and g belong to */
#define TVCS_A_BF16_SPLIT    2  /* hi = bf16(A), lo = bf16(A - hi); hi*x_hi +
                                   hi*x_lo + lo*x_hi on MFMA, 4 bytes/entry          */
#define TVCS_A_FP8_ROWSCALE  3  /* s_i = max_j |A_ij| / 448 (FP32), q_ij = OCP E4M3
                                   nearest-even of A_ij / s_i; 1 byte/entry + 4/row  */
#define TVCS_A_PARTIAL_DCT   4  /* no stored matrix: A = m rows of the orthonormal
                                   2-D DCT-II, applied as fast transforms; only
                                   through tvcs_create_dct                          */

typedef struct tvcs_ctx *tvcs_handle;

/* Per-image results of a solve. */
typedef struct {
    int    iters;       /* u-updates performed (eq. (stop) is tested after each) */
    int    status;      /* TVCS_OK, TVCS_MAXIT or TVCS_ENONFINITE for this image */
    double rel_change;  /* last ||u^{k+1} - u^k|| / ||u^k||, FP64                */
    double objective;   /* sum_i ||D_i u|| + mu/2 ||A u - f||^2 at the returned u
                           with the stored A (only with TVCS_OBJECTIVE, else 0)  */
    double tau;         /* step parameter tau used                               */
    float  ms;          /* device time of the whole solve call, milliseconds     */
    int    fresh_iters; /* bf16, split bf16 and FP8 storage: iterations whose two
                           products were computed afresh from a two-part batch
                           operand; the others added the one-part increment form
                           (see TVCS_A_BF16); 0 for FP32 and the partial DCT     */
    int    tiles[6];    /* bf16, split bf16 and FP8 storage: the tile shapes of the
                           two MFMA products, {rows of A per wave / 16, images per
                           group, 32-wide k tiles per pipeline step} of the forward
                           product (A u), then of the adjoint (A^T r); zeros
                           otherwise (see tvcs_set_tiles)                        */
} tvcs_stats;

/*
 * tvcs_create: copy a dense FP32 A (m x n*n, row-major: column r*n + c
 * multiplies pixel (r, c)) to the device in TVCS_A_FP32 storage, and estimate
 * lambda_max(A^T A) for the default step tau = 1.9 / lambda_max (Thm. 1 needs
 * 0 < tau < 2 / lambda_max).  The caller keeps ownership of A and may free it
 * when the call returns.  Uses the default stream.
 * Image sides: n even, 8 <= n <= 512, with no prime factor other than 2, 3 and 5
 * (e.g. 128, 450, 512); the FFTs are radix 2/3/4/5.
 * Returns NULL on error (see tvcs_last_error): m < 1, n not such a side
 * (TVCS_EUNSUPPORTED), A NULL, or out of device memory.
 */
tvcs_handle tvcs_create(const float *A, int m, int n);

/*
 * tvcs_create_ex: as tvcs_create, with
 *   a_is_fp64  0: A holds float, 1: A holds double (rounded to FP32 first);
 *   storage    one of TVCS_A_*;
 *   stream     a hipStream_t (may be NULL for the default stream) on which all
 *              work of this handle is ordered.
 * Storage formats other than FP32 also keep a transposed copy of A so that
 * both products read their reduction dimension contiguously (2x the bytes of
 * the format; the HBM traffic per product is unchanged), and need n >= 16
 * (TVCS_EUNSUPPORTED otherwise); m and n*n are padded with zero rows and
 * columns to multiples of 256 in the stored copies.
 */
tvcs_handle tvcs_create_ex(const void *A, int a_is_fp64, int m, int n, int storage,
                           void *stream);

/*
 * tvcs_create_dct: the partial-DCT measurement operator of Sec. 3.2, A = P C with
 * C the orthonormal 2-D DCT-II of n x n images (C[k_r n + k_c][r n + c] =
 * w_{k_r} w_{k_c} cos(pi k_r (2r+1) / 2n) cos(pi k_c (2c+1) / 2n), w_0 = sqrt(1/n),
 * w_k = sqrt(2/n)) and P the selection of the m coefficients rows[0..m-1]
 * (host int array of flat indices k_r * n + k_c, distinct, any order; f[i]
 * measures coefficient rows[i]).  A u and A^T r are computed as fast transforms
 * in FP32 (no matrix is stored).  A A^T = I, so lambda_max(A^T A) = 1 exactly and
 * the default tau is 1.9, the value of the partial-DCT experiments.  The caller
 * keeps ownership of rows.  Storage is TVCS_A_PARTIAL_DCT.
 * Returns NULL on error (see tvcs_last_error): rows NULL, m < 1 or m > n*n, an
 * index outside [0, n*n) or repeated, n not an image side tvcs_create accepts,
 * or out of device memory.
 */
tvcs_handle tvcs_create_dct(const int *rows, int m, int n, void *stream);

/* Set the stream the handle's work is ordered on (hipStream_t or NULL). */
int tvcs_set_stream(tvcs_handle h, void *stream);

/* Set tau explicitly (> 0), or restore the automatic 1.9 / lambda_max (<= 0). */
int tvcs_set_tau(tvcs_handle h, double tau);

/* Current tau and the power-iteration estimate of lambda_max(A^T A) for the
 * stored A (FP64 norms, start vector 1/sqrt(N), up to 100 steps or relative
 * Rayleigh-quotient change < 1e-10; exactly 1 for the partial DCT).  Return a
 * negative value on error. */
double tvcs_get_tau(tvcs_handle h);
double tvcs_lambda_max(tvcs_handle h);

/* Bytes of device memory held by the handle (A storage and workspaces). */
size_t tvcs_device_bytes(tvcs_handle h);

/*
 * tvcs_solve: reconstruct one image.
 *   f      m observations (FP32);
 *   mu     fidelity weight > 0;  beta  penalty parameter > 0;
 *   tol    stop when ||u^{k+1} - u^k|| <= tol ||u^k|| (eq. (stop), FP64 norms,
 *          inclusive); tol = 0 runs exactly maxit iterations; tol < 0 is EINVAL;
 *   maxit  iteration cap >= 1;
 *   flags  TVCS_IADM | TVCS_U0_ZERO | TVCS_OBJECTIVE | TVCS_WARM_START;
 *   u      n*n output (FP32, caller-owned); input u^0 with TVCS_WARM_START;
 *   lambda optional 2*n*n output (FP64, planar: horizontal then vertical
 *          component) of the IADM multiplier after the last iteration; NULL to
 *          skip; ignored without TVCS_IADM; input lambda^0 with TVCS_WARM_START;
 *   st     optional stats (NULL to skip).
 * Returns TVCS_OK, TVCS_MAXIT, or an error code.
 */
int tvcs_solve(tvcs_handle h, const float *f, double mu, double beta, double tol, int maxit,
               unsigned flags, float *u, double *lambda, tvcs_stats *st);

/*
 * tvcs_solve_batch: reconstruct B images that share A, in one run of the loop.
 *   F  B x m observations (image-major); U  B x n*n outputs; lambda  optional
 *   B x 2*n*n (FP64); st  optional array of B stats.
 * Each image stops on its own by eq. (stop); an image that has stopped is not
 * updated any more, so its result and iteration count equal those of a solve
 * of that image alone (up to the products' rounding, which does not depend on
 * the image's slot).  FP32 storage applies A to up to 8 images per pass of A;
 * the other storage formats use MFMA GEMMs over the whole batch.  With FP32
 * storage and n*n <= 16384 a single image (B = 1, and tvcs_solve) takes both
 * products in one pass over A, g = sum_i a_i (a_i . u - f_i) (see
 * tvcs_time_fused): the same sums in another order, so its result agrees with the
 * same image's in a batch to rounding, not bit for bit.
 * Returns TVCS_OK if every image met tol (or tol = 0), else TVCS_MAXIT, or an
 * error code (TVCS_ENONFINITE if any image became non-finite).
 */
int tvcs_solve_batch(tvcs_handle h, const float *F, int B, double mu, double beta, double tol,
                     int maxit, unsigned flags, float *U, double *lambda, tvcs_stats *st);

/*
 * tvcs_solve_noalloc: tvcs_solve for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  It allocates nothing: no device or pinned memory and no graph.
 * Its buffers come from one static device array of 32 MiB per GPU, which holds
 * u, f, r, the A^T r partial sums (the band partials of the one-pass product for
 * n*n <= 16384), the IADM fields, the FFT spectrum and denominators and the loop
 * state of one image, and it launches the iteration's kernels one by one.
 *   Arguments as for tvcs_solve, without lambda; st->fresh_iters is 0.
 *   Handles: FP32 storage only (TVCS_EUNSUPPORTED otherwise), used on the device
 *   that was current when the handle was created (TVCS_EINVAL otherwise).
 *   Sizes: TVCS_EINVAL when the workspace exceeds the 32 MiB array (e.g. n = 128,
 *   m = 4096 needs 17.3 MB; n = 512 does not fit).
 * Results are those of tvcs_solve: the same kernels in the same order.  Every call
 * on one GPU shares that GPU's array: calls that overlap on one GPU (from several
 * threads or handles) race and must be serialised by the caller.
 */
int tvcs_solve_noalloc(tvcs_handle h, const float *f, double mu, double beta, double tol,
                       int maxit, unsigned flags, float *u, tvcs_stats *st);

/*
 * tvcs_solve_continuation: Algorithm 1 (FTVCS) with continuation in beta, as the
 * paper runs it (Sec. 3.1): one FTVCS run per value of betas[0..nbeta-1] (an
 * increasing sequence, e.g. 2^4, 2^5, 2^6, 2^7), each stage warm-started from the
 * previous stage's u and ended by eq. (stop) with tolerance tol (0: exactly maxit
 * iterations per stage) or by maxit.
 *   F, B, mu, U   as for tvcs_solve_batch (U is also the warm start of the first
 *                 stage with TVCS_WARM_START)
 *   flags         TVCS_U0_ZERO, TVCS_WARM_START (first stage only) and
 *                 TVCS_OBJECTIVE (after the last stage); TVCS_IADM is rejected
 *                 (Algorithm 2 keeps beta fixed)
 *   st            optional B stats: iters counts all stages, the other fields are
 *                 the last stage's (ms: sum over stages)
 * Returns TVCS_OK if every stage of every image met tol (or tol = 0), TVCS_MAXIT if
 * some stage stopped at maxit (the next stage still runs), or an error code
 * (TVCS_EINVAL for NULL betas, nbeta < 1 or a beta that is not positive and finite).
 */
int tvcs_solve_continuation(tvcs_handle h, const float *F, int B, double mu,
                            const double *betas, int nbeta, double tol, int maxit,
                            unsigned flags, float *U, tvcs_stats *st);

/*
 * tvcs_set_tiles / tvcs_get_tiles: tile shapes of the MFMA products (bf16, split
 * bf16 and FP8 storage).  By default an autotuner picks each product's shape when a
 * workspace is set up for a batch (the first solve of a larger batch, a request
 * loop's slots): it times every candidate on the handle's matrix and padded batch
 * and keeps the fastest.  Candidates: 2 or 4 sixteen-row tiles of A per wave;
 * groups of the whole padded batch (at most 256 images, A streamed once per group),
 * half or a quarter of it; and two tables of k tiles per pipeline step.  No shape
 * changes the order of any sum, so every shape gives the same bits; a forced shape
 * changes only the speed.  The shapes apply to solves, the request loop and
 * tvcs_time_products.
 *   tiles   six ints as in tvcs_stats.tiles: {rt, images, kf} of the forward product,
 *           then of the adjoint, used from the next call on; NULL: autotune again
 *           (now if a workspace exists, else at its set-up).  rt is 2 or 4 (2 with
 *           256 images); images 16, 32, 64, 128 or 256 (batches that are not a
 *           multiple end with smaller groups); kf is that group size's entry in one
 *           of the two tables ({4, 4, 4, 1, 1} and {4, 2, 1, 2, 1} for 16 .. 256
 *           images).
 * Returns TVCS_OK, TVCS_EINVAL for a shape that does not exist, TVCS_EUNSUPPORTED
 * for FP32 storage and the partial DCT.  tvcs_get_tiles writes the shapes in use
 * (zeros for those formats, and before the first workspace the defaults).
 */
int tvcs_set_tiles(tvcs_handle h, const int *tiles);
int tvcs_get_tiles(tvcs_handle h, int *tiles);

/*
 * tvcs_time_products: measurement helper.  Average device time in milliseconds
 * of one forward product (r = A u - f, all images of a batch of B) and of one
 * adjoint product (A^T r, including its partial-sum reduction), over `reps`
 * launches of each timed with HIP events on the stream the solver launches them
 * on, with the launch configuration a solve of B images uses.  The inputs are
 * deterministic hashed values of unit size, not zeros (MFMA clocks depend on the
 * operands' bits); the workspace contents are overwritten.  Either output may
 * be NULL.
 *   form  0: the fresh products every storage format computes (for bf16, split
 *         bf16 and FP8 storage: from a two-part bf16 batch operand);
 *         1: the increment form of those three formats' products (one-part batch
 *         operand; the form most iterations take once the iterates change by
 *         less than 2^-8 per iteration); each timed launch follows a move of its
 *         input by 2^-10 of its size, outside the timed span, as between two
 *         iterations.  The same as 0 for FP32 and the DCT.
 */
int tvcs_time_products(tvcs_handle h, int B, int reps, int form, float *ms_forward,
                       float *ms_adjoint);

/*
 * tvcs_time_fused: measurement helper for the one-pass product a single image
 * takes with FP32 storage and n*n <= 16384: g = A^T (A u - f) as the sum over the
 * rows of A of a_i (a_i . u - f_i) (eq. (line)), each row read once.  The pass
 * (k_gemv_fused) gives each of up to 256 workgroups a band of consecutive rows;
 * the workgroup keeps whole rows in registers, reduces a_i . u across its
 * threads, and adds r_i a_i to its FP64 share of g, then writes the band's partial
 * g; a second kernel (k_sum_bands) adds the partials in a fixed order.  Average
 * device milliseconds per launch of the pass (`reps` launches back to back, the
 * row order alternating as in a solve) and of the sum (the time of `reps` pass +
 * sum pairs less that of the passes alone, so the sum reads freshly written
 * partials), timed with HIP events on the solver's stream, on hashed inputs of
 * unit size; the workspace contents are overwritten.  Either output may be NULL.
 * Returns TVCS_EUNSUPPORTED for handles that do not take the pass (other storage,
 * n*n > 16384).
 */
int tvcs_time_fused(tvcs_handle h, int reps, float *ms_pass, float *ms_sum);

/*
 * tvcs_measure_peaks: measurement helper, independent of any handle.  Achievable
 * HBM read bandwidth in GB/s (a streaming read of a `bytes`-byte device buffer with
 * 16-byte loads; use >= 1 GiB so that caches do not serve it) and dense bf16 MFMA
 * throughput in TFLOP/s (independent chains of v_mfma_f32_16x16x32_bf16 on every
 * CU), each averaged over `reps` launches timed with HIP events.  Allocates and
 * frees `bytes` of device memory.  Either output may be NULL.  Returns TVCS_EINVAL
 * if bytes < 1 MiB or reps < 1.
 */
int tvcs_measure_peaks(size_t bytes, int reps, double *read_gbs, double *mfma_tflops);

/* ---- continuous-batching request loop ------------------------------------ */
typedef struct tvcs_server *tvcs_server_handle;

/*
 * tvcs_server_create: a request loop over encoding matrices registered with
 * tvcs_server_add_matrix (the batched solve of Sec. 2 applied to a stream of
 * reconstruction requests).  Each matrix gets `slots` image slots (1..1024): its
 * batch.  A matrix's slots are allocated when its first request is admitted, and
 * only if the device bytes of all registered matrices and allocated slot groups
 * stay within hbm_budget (0: no limit); a group with no request in flight gives its
 * slots back when another matrix's requests wait for room.  A matrix that has
 * waited for room for a few rounds makes the other groups stop admitting, finish
 * the requests they hold and give their slots back, so no matrix waits longer
 * than about one request's iteration cap.  mu, beta and flags (0 or TVCS_IADM)
 * apply to every request; each request has its own tol and maxit.  Returns NULL on
 * error (see tvcs_last_error).
 */
tvcs_server_handle tvcs_server_create(size_t hbm_budget, int slots, double mu, double beta,
                                      unsigned flags);

/* Register a matrix.  The server borrows h: it must outlive the server and must not
 * be used for tvcs_solve / tvcs_solve_batch while the server runs.  Returns the
 * matrix id (>= 0) or a negative error code. */
int tvcs_server_add_matrix(tvcs_server_handle s, tvcs_handle h);

/* Queue a reconstruction of f (m floats of that matrix, host or device; copied before
 * the call returns) with its own stop tolerance tol >= 0 (eq. (stop); 0: exactly
 * maxit iterations) and cap maxit >= 1.  Returns a request id >= 0, or a negative
 * error code. */
long long tvcs_server_submit(tvcs_server_handle s, int matrix, const float *f, double tol,
                             int maxit);

/*
 * tvcs_server_step: one scheduling round.  Every matrix whose previous replay has
 * ended retires the requests that met their stop rule or cap, admits queued
 * requests into its free slots (u^0 = A^T f computed for the new slots only) and,
 * if it holds requests, starts the next replay of its captured iteration graph (10
 * iterations) on its own stream.  Matrices do not wait for each other: the call
 * returns as soon as one running replay has ended.  Requests submitted between
 * rounds join the running batches at their matrix's next replay.  A request's
 * iterates do not depend on its slot, on the other requests or on when it was
 * admitted.  Returns the number of requests queued or in flight after the round,
 * or a negative error code (TVCS_ENOMEM if queued requests can never fit the
 * budget).
 */
int tvcs_server_step(tvcs_server_handle s);

/* Result of a request: returns 1 and fills u (n*n floats, host or device; NULL to
 * skip) and st (may be NULL; st->ms is the time from admission to retirement) once it
 * has finished, after which the request id is forgotten; 0 if it has not finished;
 * TVCS_EINVAL for an unknown id. */
int tvcs_server_result(tvcs_server_handle s, long long request, float *u, tvcs_stats *st);

/* Requests queued or in flight. */
int tvcs_server_pending(tvcs_server_handle s);

/* Device bytes counted against the budget (registered matrices and slot groups). */
size_t tvcs_server_device_bytes(tvcs_server_handle s);

/* Bytes of A the replays launched so far stream: 10 iterations x 2 products x one
 * copy of the stored matrix per replay (the A^T copy of the MFMA formats has the
 * same size).  Divided by wall time, the request loop's A-stream rate, to be set
 * against the HBM roofline.  Returns a negative value for a NULL server. */
double tvcs_server_a_bytes(tvcs_server_handle s);

/* Release the server (not the registered handles).  NULL is ignored. */
void tvcs_server_destroy(tvcs_server_handle s);

/* Release the handle and all its device memory.  NULL is ignored. */
void tvcs_destroy(tvcs_handle h);

/* Message of the last error on the calling thread ("" if none). */
const char *tvcs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TVCS_H */
