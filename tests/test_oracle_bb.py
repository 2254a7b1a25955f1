"""Pins of the oracle's IADM with a BB / non-monotone line-search u-step (the
acceleration suggested in the concluding remarks, Sec. 4) (CPU only).

* One inner step is Algorithm 2 itself (the IADM u-step is the first, unit-length
  preconditioned gradient step).
* Many inner steps solve the u-subproblem of (ALP) for fixed w^{k+1}, lambda^k:
  the result matches the dense direct solution of its normal equations
  (beta D^T D + mu A^T A) v = beta D^T q + mu A^T f, with D built entry by entry.
* The drop of Phi(v) = beta/2 ||q - D v||^2 + mu/2 ||A v - f||^2 that the method
  tracks through its exact quadratic line model equals Phi evaluated densely.
* Accepted step lengths: the first of each outer iteration is 1; all are positive.
* The limit is a solution of (tv): the dual certificate holds and the objective
  matches an independent primal-dual (Chambolle-Pock) solve.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle as O
from paper_1001_1774_amd import synth
from tests._pins import chambolle_pock_tv, dense_D

N8 = dict(n=8, m=20, n_shapes=3, seed_A=7, sigma=1e-3)
MU, BETA = 50.0, 10.0


@pytest.fixture(scope="module")
def small():
    p = synth.make_problem("n8", **N8)
    return p, O.default_tau(p.A)


def test_one_inner_step_is_iadm(small):
    p, tau = small
    a = O.iadm(p.A, p.f, p.n, MU, BETA, tau, tol=0, maxit=60)
    b = O.iadm_bb(p.A, p.f, p.n, MU, BETA, tau, tol=0, maxit=60, inner=1)
    assert np.allclose(a.u, b.u, rtol=1e-11, atol=1e-13)
    assert np.allclose(a.lam, b.lam, rtol=1e-10, atol=1e-12)


def test_many_inner_steps_solve_the_u_subproblem(small):
    p, tau = small
    n = p.n
    D1, D2 = dense_D(n)
    u0 = O.initial_u(p.A, p.f, n, None)[0]
    q = O.shrink(O.D(u0), BETA)                      # w^1 with lambda^0 = 0, q = w^1
    H = BETA * (D1.T @ D1 + D2.T @ D2) + MU * (p.A.T @ p.A)
    rhs = BETA * (D1.T @ q[0].ravel() + D2.T @ q[1].ravel()) + MU * (p.A.T @ p.f[0])
    v = scipy.linalg.solve(H, rhs, assume_a="pos")
    r = O.iadm_bb(p.A, p.f, n, MU, BETA, tau, tol=0, maxit=1, inner=400)
    assert np.linalg.norm(r.u[0].ravel() - v) <= 1e-9 * np.linalg.norm(v)


def test_tracked_drop_matches_dense_phi(small):
    p, tau = small
    n = p.n
    D1, D2 = dense_D(n)

    def phi(v, q):
        d = np.concatenate([D1 @ v.ravel() - q[0].ravel(), D2 @ v.ravel() - q[1].ravel()])
        rr = p.A @ v.ravel() - p.f[0]
        return 0.5 * BETA * d @ d + 0.5 * MU * rr @ rr

    us = []
    r = O.iadm_bb(p.A, p.f, n, MU, BETA, tau, tol=0, maxit=6, inner=5,
                  record=lambda k, u: us.append(u[0].copy()))
    prev_u = O.initial_u(p.A, p.f, n, None)[0]
    lam = np.zeros((2, n, n))
    for k in range(6):
        q = O.shrink(O.D(prev_u) + lam / BETA, BETA) - lam / BETA
        drop = phi(us[k], q) - phi(prev_u, q)
        tracked = r.history[k][1][0]
        assert abs(drop - tracked) <= 1e-9 * max(1.0, abs(drop)), (k, drop, tracked)
        assert r.history[k][2][0] == 1.0 and min(r.history[k][2]) > 0
        w = q + lam / BETA
        lam = lam - BETA * (w - O.D(us[k]))
        prev_u = us[k]


@pytest.fixture(scope="module")
def bb_limit(small):
    p, tau = small
    return O.iadm_bb(p.A, p.f, p.n, MU, BETA, tau, tol=0, maxit=1500, inner=3)


def test_bb_limit_dual_certificate(small, bb_limit):
    p, _ = small
    u, lam = bb_limit.u, bb_limit.lam
    assert np.hypot(lam[:, 0], lam[:, 1]).max() <= 1 + 1e-8
    Du = O.D(u)
    t = np.hypot(Du[:, 0], Du[:, 1])
    on = t > 1e-6
    assert np.allclose((lam[:, 0] * Du[:, 0] + lam[:, 1] * Du[:, 1])[on], t[on], rtol=1e-6)
    res = O.Dt(lam) + MU * O.gradient(p.A, u, p.f)
    assert np.abs(res).max() <= 1e-8 * MU * np.abs(p.f @ p.A).max()


def test_bb_limit_matches_primal_dual_solver(small, bb_limit):
    p, _ = small
    _, fc = chambolle_pock_tv(p.A, p.f[0], p.n, MU, iters=20000)
    obj = O.objective_tv(bb_limit.u, p.A, p.f, MU)[0]
    assert abs(obj - fc) <= 1e-8 * fc
