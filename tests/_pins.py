"""Independent reference computations used to pin the oracle.

Nothing here imports the oracle: the finite-difference operator is built entry by
entry as a dense matrix, and the minimisers come from general-purpose convex
solvers (scipy L-BFGS, and the primal-dual method of Chambolle and Pock, J. Math.
Imaging Vis. 40 (2011)).
"""
from __future__ import annotations

import numpy as np
import scipy.optimize


def dense_D(n: int):
    """Dense forward-difference matrices D1, D2 (N x N), periodic, pixel r*n + c."""
    N = n * n
    D1 = np.zeros((N, N))
    D2 = np.zeros((N, N))
    for r in range(n):
        for c in range(n):
            i = r * n + c
            D1[i, i] -= 1.0
            D1[i, r * n + (c + 1) % n] += 1.0
            D2[i, i] -= 1.0
            D2[i, ((r + 1) % n) * n + c] += 1.0
    return D1, D2


def huber_value_grad(u, A, f, mu, beta, D1, D2):
    """Psi(u) = sum_i phi(||D_i u||) + mu/2 ||Au - f||^2 and its gradient (dense)."""
    a, b = D1 @ u, D2 @ u
    t = np.hypot(a, b)
    small = t <= 1.0 / beta
    phi = np.where(small, 0.5 * beta * t * t, t - 0.5 / beta)
    # d phi / d(a, b) = beta (a, b) on the disc, (a, b)/t outside
    sc = np.where(small, beta, 1.0 / np.where(t > 0, t, 1.0))
    r = A @ u - f
    val = phi.sum() + 0.5 * mu * r @ r
    grad = D1.T @ (sc * a) + D2.T @ (sc * b) + mu * (A.T @ r)
    return val, grad


def lbfgs_huber(A, f, n, mu, beta, u0=None):
    D1, D2 = dense_D(n)
    x0 = np.zeros(n * n) if u0 is None else u0.ravel().copy()
    res = scipy.optimize.minimize(
        huber_value_grad, x0, args=(A, f, mu, beta, D1, D2), jac=True, method="L-BFGS-B",
        options=dict(maxiter=200000, maxfun=400000, ftol=1e-16, gtol=1e-12, maxcor=50))
    return res.x, res.fun


def tv_objective(u, A, f, mu, D1, D2):
    a, b = D1 @ u, D2 @ u
    r = A @ u - f
    return np.hypot(a, b).sum() + 0.5 * mu * r @ r


def chambolle_pock_tv(A, f, n, mu, iters=40000):
    """min_u sum_i ||D_i u|| + mu/2 ||A u - f||^2 by the Chambolle-Pock primal-dual
    method with K = D, F = the (2,1)-norm, G(u) = mu/2 ||Au - f||^2 (prox by a dense
    solve).  Returns (u, objective)."""
    D1, D2 = dense_D(n)
    N = n * n
    K = np.vstack([D1, D2])
    L2 = np.linalg.norm(K, 2) ** 2
    sig = tau = 0.99 / np.sqrt(L2)
    M = np.eye(N) + tau * mu * (A.T @ A)
    Minv = np.linalg.inv(M)
    Atf = tau * mu * (A.T @ f)
    u = np.zeros(N)
    ubar = u.copy()
    p = np.zeros(2 * N)
    for _ in range(iters):
        p = p + sig * (K @ ubar)
        p1, p2 = p[:N], p[N:]
        nrm = np.maximum(1.0, np.hypot(p1, p2))
        p = np.concatenate([p1 / nrm, p2 / nrm])
        un = Minv @ (u - tau * (K.T @ p) + Atf)
        ubar = 2 * un - u
        u = un
    return u, tv_objective(u, A, f, mu, D1, D2)


def shrink_bruteforce(z, beta):
    """argmin_w ||w|| + beta/2 ||w - z||^2 over R^2 by Nelder-Mead from several starts."""
    def obj(w):
        return np.hypot(w[0], w[1]) + 0.5 * beta * ((w[0] - z[0]) ** 2 + (w[1] - z[1]) ** 2)
    best = None
    for start in (np.zeros(2), np.asarray(z, float), 0.5 * np.asarray(z, float)):
        r = scipy.optimize.minimize(obj, start, method="Nelder-Mead",
                                    options=dict(xatol=1e-12, fatol=1e-15, maxiter=20000))
        if best is None or r.fun < best.fun:
            best = r
    return best.x, best.fun, obj
