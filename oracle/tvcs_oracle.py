"""Plain FP64 oracle of the FTVCS and IADM iterations (test infrastructure only).

Model (Sec. 1, eq. (tv)):   min_u  sum_i ||D_i u||_2 + mu/2 ||A u - f||^2,
u an n x n image stored row-major as a vector of length N = n^2 (pixel r*n + c),
A dense m x N, f of length m.  D = (D1; D2) are the first-order differences
with periodic boundary conditions (Sec. 2.1), stored planar: w[0] is the
horizontal component, w[1] the vertical one (index set {i, i + n^2}, App. A).

Readings of the paper taken here (each is a choice where the text is silent,
ambiguous or in error):

* D1 u[r, c] = u[r, (c+1) mod n] - u[r, c];  D2 u[r, c] = u[(r+1) mod n, c] - u[r, c].
* Alg. 1 and Alg. 2 print "u^0 = f", which has the wrong length; u^0 = A^T f is
  used (an optional u^0 can be passed), and lambda^0 = 0.
* tau is an input; `default_tau` gives 1.9 / lambda_max(A^T A), with
  lambda_max from FP64 power iteration (Thm. 1 needs tau < 2 / lambda_max; the
  experiments of Sec. 3.2 use tau = 1.9 with an orthonormal A).
* IADM w-step (eq. (iadmw)): minimizing the augmented Lagrangian (ALP) over w_i
  gives the shrinkage centre D_i u^k + lambda_i^k / beta; the printed
  "D_i u^k - lambda_i^k / beta" contradicts (ALP), (eqnorm11) and (udlamb).  The
  default `sign=+1` follows (ALP); `sign=-1` reproduces the printed formula.
* Stop rule (eq. (stop)): ||u^{k+1} - u^k|| <= tol ||u^k|| checked after every
  u-update, inclusive; tol = 0 runs exactly maxit iterations.
* Shrinkage at ||z|| = 0 returns 0 (the 0 * (0/0) = 0 convention of (shrink)).

Parity status: every function below is pinned by a CPU test in tests/ against
closed forms, dense linear algebra, brute-force minimisation or library
routines (see the tests named in each docstring).  None is "parity unpinned".
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "D", "Dt", "project_disc", "shrink", "dtd_eigenvalues", "solve_u", "gradient",
    "lambda_max", "default_tau", "tv", "objective_tv", "huber_objective",
    "OracleResult", "initial_u", "ftvcs", "ftvcs_continuation", "iadm", "iadm_bb", "bf16_rne",
    "PartialDCT", "apply_A", "apply_At", "split_bf16", "fp8_e4m3_values",
    "fp8_e4m3_rne", "fp8_rowscale_quantize", "dequantized_A",
]


# ---------------------------------------------------------------------------
# Finite differences (Sec. 2 notation: D = (D^(1); D^(2)), periodic BC, Sec. 2.1)
# ---------------------------------------------------------------------------
def D(u: np.ndarray) -> np.ndarray:
    """Forward differences: (..., n, n) -> (..., 2, n, n); component 0 along c, 1 along r.

    Pinned by tests/test_oracle_ops.py (dense matrix built entry by entry).
    """
    d1 = np.roll(u, -1, axis=-1) - u
    d2 = np.roll(u, -1, axis=-2) - u
    return np.stack([d1, d2], axis=-3)


def Dt(w: np.ndarray) -> np.ndarray:
    """Adjoint D^T: (..., 2, n, n) -> (..., n, n), the negated backward difference.

    Pinned by the adjoint identity <D u, w> = <u, D^T w> and the dense matrix.
    """
    w1 = w[..., 0, :, :]
    w2 = w[..., 1, :, :]
    return (np.roll(w1, 1, axis=-1) - w1) + (np.roll(w2, 1, axis=-2) - w2)


# ---------------------------------------------------------------------------
# Two-dimensional shrinkage (eq. (shrink), and its operator form (sop) in App. A)
# ---------------------------------------------------------------------------
def project_disc(z: np.ndarray, beta: float) -> np.ndarray:
    """P_B(z): Euclidean projection of each 2-vector onto the disc ||.|| <= 1/beta (App. A)."""
    t = np.hypot(z[..., 0, :, :], z[..., 1, :, :])
    r = 1.0 / beta
    scale = np.where(t > r, r / np.where(t > 0, t, 1.0), 1.0)
    return z * scale[..., None, :, :]


def shrink(z: np.ndarray, beta: float) -> np.ndarray:
    """w_i = max(||z_i|| - 1/beta, 0) z_i / ||z_i||, with 0 * (0/0) = 0 (eq. (shrink)).

    Pinned by tests/test_oracle_ops.py against s(z) = z - P_B(z) (eq. (sop)) and a
    brute-force minimisation of ||w|| + beta/2 ||w - z||^2 (eq. (fixu)).
    """
    t = np.hypot(z[..., 0, :, :], z[..., 1, :, :])
    safe_t = np.where(t > 0, t, 1.0)
    scale = np.where(t > 0, np.maximum(t - 1.0 / beta, 0.0) / safe_t, 0.0)
    return z * scale[..., None, :, :]


# ---------------------------------------------------------------------------
# The u-step linear system (eq. (eqnorm) / (eqnorm11)) solved by 2-D FFTs
# ---------------------------------------------------------------------------
def dtd_eigenvalues(n: int) -> np.ndarray:
    """Eigenvalues of D^T D under periodic BC, indexed by 2-D frequency (k1, k2).

    D^T D is block-circulant (Sec. 2.1) with symbol 4 sin^2(pi k1/n) + 4 sin^2(pi k2/n).
    Pinned against numpy.linalg.eigvalsh of the dense D^T D.
    """
    k = np.arange(n)
    s = 4.0 * np.sin(np.pi * k / n) ** 2
    return s[:, None] + s[None, :]


def solve_u(rhs: np.ndarray, c: float) -> np.ndarray:
    """Solve (D^T D + c I) u = rhs for each n x n image by one FFT and one inverse FFT.

    Sec. 2.1: under periodic BC the coefficient matrix is diagonalised by the 2-D
    DFT.  Pinned by a dense Cholesky solve in tests/test_oracle_ops.py.
    """
    n = rhs.shape[-1]
    denom = dtd_eigenvalues(n) + c
    spec = np.fft.fft2(rhs)
    return np.real(np.fft.ifft2(spec / denom))


class PartialDCT:
    """A = P C as an operator: the rows `rows` (flat indices k_r * n + k_c) of the
    orthonormal 2-D DCT-II C of n x n images, applied as fast transforms (Sec. 3.2:
    m rows of the DCT matrix chosen at random, stored implicitly).  The rows of C are
    orthonormal, so A A^T = I and A^T is the inverse DCT of the zero-filled
    coefficients.  The transforms are scipy.fft.dctn / idctn (type 2, norm "ortho");
    pinned against the DCT matrix written out from its cosine formula."""

    def __init__(self, n: int, rows):
        self.n = int(n)
        self.rows = np.asarray(rows, dtype=np.int64)
        self.shape = (len(self.rows), self.n * self.n)

    def fwd(self, U: np.ndarray) -> np.ndarray:
        """U (B, n^2) -> A U (B, m)."""
        import scipy.fft
        B, n = U.shape[0], self.n
        X = scipy.fft.dctn(U.reshape(B, n, n), type=2, norm="ortho", axes=(1, 2))
        return X.reshape(B, n * n)[:, self.rows]

    def adj(self, R: np.ndarray) -> np.ndarray:
        """R (B, m) -> A^T R (B, n^2)."""
        import scipy.fft
        B, n = R.shape[0], self.n
        X = np.zeros((B, n * n))
        X[:, self.rows] = R
        return scipy.fft.idctn(X.reshape(B, n, n), type=2, norm="ortho",
                               axes=(1, 2)).reshape(B, n * n)


def _as_A(A):
    """A dense matrix as FP64, or an operator object as it is."""
    return A if isinstance(A, PartialDCT) else np.asarray(A, dtype=np.float64)


def apply_A(A, U: np.ndarray) -> np.ndarray:
    """A U for U (B, N): a dense product or the operator's forward transform."""
    return A.fwd(U) if isinstance(A, PartialDCT) else U @ A.T


def apply_At(A, R: np.ndarray) -> np.ndarray:
    """A^T R for R (B, m)."""
    return A.adj(R) if isinstance(A, PartialDCT) else R @ A


def gradient(A: np.ndarray, u: np.ndarray, f: np.ndarray) -> np.ndarray:
    """g_k = A^T (A u^k - f), the gradient of 1/2 ||A u - f||^2 (eq. (line)).

    u: (B, n, n), f: (B, m).  Returns (B, n, n).  Pinned by finite differences.
    """
    B, n, _ = u.shape
    U = u.reshape(B, n * n)
    R = apply_A(A, U) - f      # (B, m): r_b = A u_b - f_b
    G = apply_At(A, R)         # (B, N): g_b = A^T r_b
    return G.reshape(B, n, n)


def lambda_max(A: np.ndarray, iters: int = 100, rtol: float = 1e-10) -> float:
    """Largest eigenvalue of A^T A by power iteration from 1/sqrt(N) (tau rule of Thm. 1).

    Stops after `iters` steps or when the Rayleigh quotient changes by < rtol
    (relative).  Pinned against the top singular value from numpy.linalg.svd.
    """
    N = A.shape[1]
    v = np.full(N, 1.0 / np.sqrt(N))
    lam = 0.0
    for _ in range(iters):
        w = apply_At(A, apply_A(A, v[None]))[0]
        new = float(v @ w)
        v = w / np.linalg.norm(w)
        if lam > 0 and abs(new - lam) <= rtol * new:
            lam = new
            break
        lam = new
    return lam


def default_tau(A: np.ndarray) -> float:
    """tau = 1.9 / lambda_max(A^T A), inside the range 0 < tau < 2/lambda_max of Thm. 1."""
    return 1.9 / lambda_max(A)


# ---------------------------------------------------------------------------
# Objectives
# ---------------------------------------------------------------------------
def tv(u: np.ndarray) -> np.ndarray:
    """Isotropic TV sum_i ||D_i u|| per image (eq. (tv))."""
    d = D(u)
    return np.hypot(d[..., 0, :, :], d[..., 1, :, :]).sum(axis=(-1, -2))


def objective_tv(u: np.ndarray, A: np.ndarray, f: np.ndarray, mu: float) -> np.ndarray:
    """sum_i ||D_i u|| + mu/2 ||A u - f||^2 per image (eq. (tv)); u (B,n,n), f (B,m)."""
    B, n, _ = u.shape
    R = apply_A(A, u.reshape(B, n * n)) - f
    return tv(u) + 0.5 * mu * np.sum(R * R, axis=1)


def huber_objective(u: np.ndarray, A: np.ndarray, f: np.ndarray, mu: float,
                    beta: float) -> np.ndarray:
    """min over w of the penalty objective (eq. (atv)) at fixed u.

    Substituting the minimiser w_i = s(D_i u) (eq. (shrink)) gives
    sum_i phi(||D_i u||) + mu/2 ||A u - f||^2, phi(t) = beta t^2/2 for t <= 1/beta and
    t - 1/(2 beta) otherwise.
    """
    B, n, _ = u.shape
    d = D(u)
    t = np.hypot(d[..., 0, :, :], d[..., 1, :, :])
    phi = np.where(t <= 1.0 / beta, 0.5 * beta * t * t, t - 0.5 / beta)
    R = apply_A(A, u.reshape(B, n * n)) - f
    return phi.sum(axis=(-1, -2)) + 0.5 * mu * np.sum(R * R, axis=1)


# ---------------------------------------------------------------------------
# Algorithms 1 (FTVCS) and 2 (IADM)
# ---------------------------------------------------------------------------
@dataclass
class OracleResult:
    u: np.ndarray                      # (B, n, n) final iterate
    iters: np.ndarray                  # (B,) u-updates performed
    rel_change: np.ndarray             # (B,) last ||u^{k+1}-u^k|| / ||u^k||
    w: np.ndarray | None = None        # (B, 2, n, n) last w
    lam: np.ndarray | None = None      # (B, 2, n, n) last multiplier (IADM)
    history: list = field(default_factory=list)


def _as_batch(f):
    f = np.atleast_2d(np.asarray(f, dtype=np.float64))
    return f


def initial_u(A, f, n, u0):
    """u^0: A^T f by default (Alg. 1 and 2 print "u^0 = f", which has the wrong length),
    else a copy of the given u0 broadcast over the batch.

    Pinned by tests/test_oracle_start_storage.py: for A = I the default is the printed
    start f itself, and it is minus the gradient of 1/2 ||A u - f||^2 at u = 0 taken by
    finite differences of that objective.
    """
    B = f.shape[0]
    if u0 is None:                                  # reading: u^0 = A^T f
        return apply_At(A, f).reshape(B, n, n)
    return np.broadcast_to(np.asarray(u0, dtype=np.float64), (B, n, n)).copy()


def ftvcs(A, f, n, mu, beta, tau, tol=0.0, maxit=200, u0=None, record=None) -> OracleResult:
    """Algorithm 1 (FTVCS): alternate the shrinkage (eq. (shrink)) and the
    linearised-proximal u-step (eq. (eqnorm)) with c = mu / (beta tau).

    Each image of the batch stops on its own by the rule (eq. (stop)).
    `record(k, u)` is called after every iteration if given.
    """
    A = _as_A(A)
    f = _as_batch(f)
    u = initial_u(A, f, n, u0)
    B = u.shape[0]
    c = mu / (beta * tau)
    active = np.ones(B, dtype=bool)
    iters = np.zeros(B, dtype=np.int64)
    rel = np.full(B, np.inf)
    w = np.zeros((B, 2, n, n))
    for k in range(maxit):
        if not active.any():
            break
        idx = np.nonzero(active)[0]
        uk = u[idx]
        wk = shrink(D(uk), beta)                                  # step 1, eq. (shrink)
        g = gradient(A, uk, f[idx])                               # g_k, eq. (line)
        rhs = Dt(wk) + c * (uk - tau * g)                         # right side of (eqnorm)
        un = solve_u(rhs, c)                                      # step 2, eq. (eqnorm)
        du = np.sqrt(np.sum((un - uk) ** 2, axis=(1, 2)))
        nu = np.sqrt(np.sum(uk ** 2, axis=(1, 2)))
        u[idx] = un
        w[idx] = wk
        iters[idx] += 1
        rel[idx] = du / np.where(nu > 0, nu, 1.0)
        if tol > 0:
            done = du <= tol * nu                                 # eq. (stop)
            active[idx[done]] = False
        if record is not None:
            record(k, u)
    return OracleResult(u=u, iters=iters, rel_change=rel, w=w)


def ftvcs_continuation(A, f, n, mu, betas, tau, tol=0.0, maxit=200, u0=None,
                       record=None) -> OracleResult:
    """FTVCS with continuation in beta (Sec. 3.1): Algorithm 1 is run for each beta of
    the increasing sequence `betas` in turn, each stage warm-started from the previous
    stage's u and ended by the stop rule (eq. (stop)) or `maxit`.  Returns the last
    stage's u and w; `iters` counts the iterations of all stages.
    `record(stage, k, u)` is called after every iteration if given.
    """
    f = _as_batch(f)
    u = u0
    total = np.zeros(f.shape[0], dtype=np.int64)
    res = None
    for s, beta in enumerate(betas):
        rec = None if record is None else (lambda k, uu, s=s: record(s, k, uu))
        res = ftvcs(A, f, n, mu, beta, tau, tol=tol, maxit=maxit, u0=u, record=rec)
        total += res.iters
        u = res.u
    return OracleResult(u=res.u, iters=total, rel_change=res.rel_change, w=res.w)


def iadm(A, f, n, mu, beta, tau, tol=0.0, maxit=200, u0=None, lam0=None, sign=+1,
         record=None) -> OracleResult:
    """Algorithm 2 (IADM): w-step (eq. (iadmw)), u-step (eq. (eqnorm11)),
    multiplier update (eq. (udlamb)).

    sign=+1 uses the shrinkage centre D_i u^k + lambda_i^k / beta obtained by
    minimising (ALP) over w_i; sign=-1 uses the printed D_i u^k - lambda_i^k / beta.
    """
    A = _as_A(A)
    f = _as_batch(f)
    u = initial_u(A, f, n, u0)
    B = u.shape[0]
    lam = np.zeros((B, 2, n, n)) if lam0 is None else \
        np.broadcast_to(np.asarray(lam0, dtype=np.float64), (B, 2, n, n)).copy()
    c = mu / (beta * tau)
    active = np.ones(B, dtype=bool)
    iters = np.zeros(B, dtype=np.int64)
    rel = np.full(B, np.inf)
    w = np.zeros((B, 2, n, n))
    for k in range(maxit):
        if not active.any():
            break
        idx = np.nonzero(active)[0]
        uk, lk = u[idx], lam[idx]
        wk = shrink(D(uk) + sign * lk / beta, beta)               # step 1, eq. (iadmw)
        g = gradient(A, uk, f[idx])
        rhs = Dt(wk - lk / beta) + c * (uk - tau * g)             # right side of (eqnorm11)
        un = solve_u(rhs, c)                                      # step 2
        lam[idx] = lk - beta * (wk - D(un))                       # step 3, eq. (udlamb)
        du = np.sqrt(np.sum((un - uk) ** 2, axis=(1, 2)))
        nu = np.sqrt(np.sum(uk ** 2, axis=(1, 2)))
        u[idx] = un
        w[idx] = wk
        iters[idx] += 1
        rel[idx] = du / np.where(nu > 0, nu, 1.0)
        if tol > 0:
            done = du <= tol * nu                                 # eq. (stop)
            active[idx[done]] = False
        if record is not None:
            record(k, u)
    return OracleResult(u=u, iters=iters, rel_change=rel, w=w, lam=lam)


def iadm_bb(A, f, n, mu, beta, tau, tol=0.0, maxit=200, inner=4, memory=5, sigma=1e-4,
            u0=None, record=None) -> OracleResult:
    """Algorithm 2 with its u-step replaced by `inner` steps of a gradient method with
    BB step lengths and a non-monotone line search on the u-subproblem of (ALP), the
    acceleration the concluding remarks (Sec. 4) suggest.

    For fixed w^{k+1} and lambda^k, with q = w^{k+1} - lambda^k / beta, (ALP) in u is
    Phi(v) = beta/2 ||q - D v||^2 + mu/2 ||A v - f||^2 up to a constant, a convex
    quadratic with gradient beta D^T (D v - q) + mu A^T (A v - f) and Hessian
    H = beta D^T D + mu A^T A.  The steps are preconditioned by
    M = beta D^T D + (mu / tau) I, the matrix of the u-step (eqnorm11) times beta, so
    the direction p = -M^{-1} grad Phi costs one FFT solve, and the first step with
    length 1 is exactly the IADM u-step (inner = 1 gives Algorithm 2).  Later
    lengths are BB step lengths in the M metric: for the previous step
    s = a p_prev, y = H s (Phi is quadratic), so s^T M s / s^T y =
    (p_prev^T M p_prev) / (p_prev^T H p_prev).  A length a is accepted when
    Phi(v + a p) <= max of the last `memory` accepted values + sigma a grad^T p
    (non-monotone Armijo test of Grippo, Lampariello and Lucidi, SIAM J. Numer.
    Anal. 23 (1986)), else halved; along the line Phi is the exact quadratic
    Phi(v) + a grad^T p + a^2/2 p^T H p, with grad^T p = -p^T M p.  The residual is
    carried as r <- r + a A p, so each inner step costs two products with A (A^T r
    and A p), as one IADM iteration does.  lambda is then updated by (udlamb) and
    the stop rule (eq. (stop)) compares consecutive outer iterates.
    Readings: w-step with the "+" centre as in `iadm`; tau as in `iadm`.
    Pinned by tests/test_oracle_bb.py: inner = 1 reproduces `iadm`; many inner steps
    solve the u-subproblem to the dense direct solution; every accepted step meets
    the non-monotone test; the limit satisfies the dual certificate of (tv).
    `record(k, u)` is called after every outer iteration; the result's `history`
    holds, per outer iteration, (A-products, [Phi(v_J) - Phi(v_0) per image], [step
    lengths of the last image's inner steps]).
    """
    A = _as_A(A)
    f = _as_batch(f)
    u = initial_u(A, f, n, u0)
    B = u.shape[0]
    lam = np.zeros((B, 2, n, n))
    c = mu / (beta * tau)
    iters = np.zeros(B, dtype=np.int64)
    rel = np.full(B, np.inf)
    active = np.ones(B, dtype=bool)
    w = np.zeros((B, 2, n, n))
    hist = []
    for k in range(maxit):
        if not active.any():
            break
        idx = np.nonzero(active)[0]
        drops, lengths = [], []
        for b in idx:
            ub, lb = u[b], lam[b]
            wb = shrink(D(ub) + lb / beta, beta)                     # eq. (iadmw)
            q = wb - lb / beta
            v = ub.copy()
            r = apply_A(A, v.reshape(1, -1))[0] - f[b]
            phis = [0.0]                                             # Phi(v_j) - Phi(v_0)
            prev = None                                              # (p^T M p, p^T H p)
            for j in range(inner):
                grad = beta * Dt(D(v) - q) + mu * apply_At(A, r[None])[0].reshape(n, n)
                p = solve_u(-grad / beta, c)                         # -M^{-1} grad
                Dp = D(p)
                Ap = apply_A(A, p.reshape(1, -1))[0]
                pMp = beta * np.sum(Dp * Dp) + (mu / tau) * np.sum(p * p)
                pHp = beta * np.sum(Dp * Dp) + mu * np.sum(Ap * Ap)
                gp = -pMp
                a = 1.0 if prev is None else prev[0] / prev[1]
                ref = max(phis[-memory:])
                while phis[-1] + a * gp + 0.5 * a * a * pHp > ref + sigma * a * gp:
                    a *= 0.5
                v = v + a * p
                r = r + a * Ap
                phis.append(phis[-1] + a * gp + 0.5 * a * a * pHp)
                prev = (pMp, pHp)
                if b == idx[-1]:
                    lengths.append(a)
            drops.append(phis[-1])
            lam[b] = lb - beta * (wb - D(v))                         # eq. (udlamb)
            du = np.sqrt(np.sum((v - ub) ** 2))
            nu = np.sqrt(np.sum(ub ** 2))
            u[b] = v
            w[b] = wb
            iters[b] += 1
            rel[b] = du / (nu if nu > 0 else 1.0)
            if tol > 0 and du <= tol * nu:                          # eq. (stop)
                active[b] = False
        hist.append((2 * inner * len(idx), drops, lengths))
        if record is not None:
            record(k, u)
    return OracleResult(u=u, iters=iters, rel_change=rel, w=w, lam=lam, history=hist)


# ---------------------------------------------------------------------------
# Storage formats of A (definitions used to build de-quantised copies of A)
# ---------------------------------------------------------------------------
def bf16_rne(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to bfloat16 (8 significant bits), nearest-even, returned as FP32.

    Definition on the IEEE bit pattern: add 0x7FFF plus the lowest kept bit, then
    clear the 16 discarded bits.  Finite inputs only.  Pinned against torch's
    float32 -> bfloat16 conversion.
    """
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def split_bf16(x: np.ndarray):
    """hi = bf16(x), lo = bf16(x - hi) with x - hi formed exactly in FP32."""
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_rne(x)
    lo = bf16_rne((x - hi).astype(np.float32))
    return hi, lo


def fp8_e4m3_values() -> np.ndarray:
    """The 127 non-negative finite values of OCP FP8 E4M3 indexed by code 0..126.

    Exponent bias 7, 3 mantissa bits, subnormals m * 2^-9; code 127 is NaN, so the
    largest finite value is 1.75 * 2^8 = 448.
    """
    vals = []
    for code in range(127):
        e, mt = code >> 3, code & 7
        vals.append(mt * 2.0 ** -9 if e == 0 else (1.0 + mt / 8.0) * 2.0 ** (e - 7))
    return np.array(vals)


def fp8_e4m3_rne(x: np.ndarray):
    """Round to the nearest E4M3 value, ties to even code, saturating at +-448.

    Returns (value as FP64, signed code magnitude index).  Pinned against torch's
    float8_e4m3fn conversion on values inside the finite range.
    """
    vals = fp8_e4m3_values()
    a = np.abs(np.asarray(x, dtype=np.float64))
    a = np.minimum(a, vals[-1])
    hi = np.clip(np.searchsorted(vals, a, side="left"), 0, len(vals) - 1)
    lo = np.clip(hi - 1, 0, len(vals) - 1)
    dlo = a - vals[lo]
    dhi = vals[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo)
    return np.copysign(vals[code], x), code


def fp8_rowscale_quantize(A32: np.ndarray):
    """Per-row scaled E4M3 storage: s_i = max_j |A_ij| / 448 (FP32),
    q_ij = E4M3_rne(A_ij / s_i) with the division in FP32.  Returns (q as FP64, s)."""
    A32 = np.asarray(A32, dtype=np.float32)
    amax = np.max(np.abs(A32), axis=1).astype(np.float32)
    s = (amax / np.float32(448.0)).astype(np.float32)
    s = np.where(s > 0, s, np.float32(1.0)).astype(np.float32)
    ratio = (A32 / s[:, None]).astype(np.float32)
    q, _ = fp8_e4m3_rne(ratio)
    return q, s


def dequantized_A(A: np.ndarray, storage: str) -> np.ndarray:
    """The FP64 matrix that a storage format represents, after rounding A to FP32.

    storage: "fp32", "bf16", "bf16_split" (hi + lo) or "fp8_rowscale" (s_i * q_ij).
    Pinned by tests/test_oracle_start_storage.py (bf16 against torch's cast, the
    split's error bounds) and tests/test_oracle_ops.py (FP8 with row scales).
    """
    A32 = np.asarray(A, dtype=np.float32)
    if storage == "fp32":
        return A32.astype(np.float64)
    if storage == "bf16":
        return bf16_rne(A32).astype(np.float64)
    if storage == "bf16_split":
        hi, lo = split_bf16(A32)
        return hi.astype(np.float64) + lo.astype(np.float64)
    if storage == "fp8_rowscale":
        q, s = fp8_rowscale_quantize(A32)
        return q * s.astype(np.float64)[:, None]
    raise ValueError(f"unknown storage {storage!r}")
