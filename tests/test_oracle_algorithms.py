"""Pins of the oracle's Algorithms 1 (FTVCS) and 2 (IADM) (CPU only).

The limits are checked against optimality certificates (complete proofs of
optimality for these convex problems) and against independent solvers; the
iterates are checked against the descent bound that Thm. 1's step-size range
implies, and against special cases with closed-form answers.
"""
import numpy as np
import pytest
import scipy.linalg

import oracle as O
from paper_1001_1774_amd import synth
from tests._pins import chambolle_pock_tv, dense_D, lbfgs_huber

N8 = dict(n=8, m=20, n_shapes=3, seed_A=7, sigma=1e-3)
MU, BETA = 50.0, 10.0


@pytest.fixture(scope="module")
def small():
    p = synth.make_problem("n8", **N8)
    tau = O.default_tau(p.A)
    return p, tau


@pytest.fixture(scope="module")
def ftvcs_limit(small):
    p, tau = small
    return O.ftvcs(p.A, p.f, p.n, MU, BETA, tau, tol=0, maxit=5000)


@pytest.fixture(scope="module")
def iadm_limit(small):
    p, tau = small
    return O.iadm(p.A, p.f, p.n, MU, BETA, tau, tol=0, maxit=5000)


# --- FTVCS ------------------------------------------------------------------------
def test_ftvcs_descent_bound(small):
    """Psi(u^{k+1}) <= Psi(u^k) - mu (1/tau - lmax/2) ||u^{k+1} - u^k||^2 (0 < tau < 2/lmax).

    The w-step minimises (atv) exactly; the u-step minimises a majoriser of (atv) in u
    that is strongly convex with modulus mu/tau (eq. (eqline)).
    """
    p, tau = small
    lmax = O.lambda_max(p.A, iters=5000, rtol=1e-14)
    us = [O.initial_u(p.A, np.atleast_2d(p.f), p.n, None).copy()]
    O.ftvcs(p.A, p.f, p.n, 1e3, BETA, tau, tol=0, maxit=300,
            record=lambda k, u: us.append(u.copy()))
    psi = [O.huber_objective(u, p.A, p.f, 1e3, BETA)[0] for u in us]
    for k in range(len(us) - 1):
        d2 = np.sum((us[k + 1] - us[k]) ** 2)
        bound = psi[k] - 1e3 * (1.0 / tau - lmax / 2) * d2
        assert psi[k + 1] <= bound + 1e-9 * abs(psi[k]), k


def test_ftvcs_limit_satisfies_kkt(small, ftvcs_limit):
    """Fixed point (eq. (solution)) times beta: beta D^T P_B(D u*) + mu A^T (A u* - f) = 0."""
    p, _ = small
    u = ftvcs_limit.u
    res = BETA * O.Dt(O.project_disc(O.D(u), BETA)) + MU * O.gradient(p.A, u, p.f)
    scale = MU * np.abs(p.f @ p.A).max()
    assert np.abs(res).max() <= 1e-10 * scale
    # and w = s(D u*) at the fixed point
    assert np.allclose(ftvcs_limit.w, O.shrink(O.D(u), BETA), atol=1e-12)


def test_ftvcs_limit_matches_bruteforce(small, ftvcs_limit):
    p, _ = small
    ub, fb = lbfgs_huber(p.A, p.f[0], p.n, MU, BETA)
    psi = O.huber_objective(ftvcs_limit.u, p.A, p.f, MU, BETA)[0]
    assert abs(psi - fb) <= 1e-9 * abs(fb)
    # A u* is unique even when u* is not (m < N)
    assert np.allclose(p.A @ ftvcs_limit.u.ravel(), p.A @ ub, rtol=1e-5, atol=1e-6)


def test_ftvcs_zero_set_stabilises(small):
    """Thm. 2: w_i = 0 on L = {i : ||D_i u*|| <= 1/beta} after finitely many steps."""
    p, tau = small
    sets = []
    O.ftvcs(p.A, p.f, p.n, MU, BETA, tau, tol=0, maxit=1500,
            record=lambda k, u: sets.append(
                np.hypot(*O.shrink(O.D(u), BETA)[0]) == 0))
    last = sets[-1]
    assert last.any() and not last.all()
    assert all(np.array_equal(s, last) for s in sets[-700:])


def test_ftvcs_tikhonov_special_case(rng):
    """If every ||D_i u^k|| <= 1/beta then w == 0 and the limit solves
    (D^T D + mu/beta A^T A) u = mu/beta A^T f (eq. (foru) with w = 0)."""
    n, m = 8, 24
    A = rng.standard_normal((m, n * n)) / np.sqrt(m)
    f = (A @ rng.uniform(0, 1, n * n) + 1e-3 * rng.standard_normal(m))[None]
    mu, beta = 1.0, 0.1
    tau = O.default_tau(A)
    seen = []
    r = O.ftvcs(A, f, n, mu, beta, tau, tol=0, maxit=4000,
                record=lambda k, u: seen.append(np.abs(O.shrink(O.D(u), beta)).max()))
    assert max(seen) == 0.0
    D1, D2 = dense_D(n)
    H = D1.T @ D1 + D2.T @ D2 + mu / beta * (A.T @ A)
    ref = scipy.linalg.solve(H, mu / beta * (A.T @ f[0]), assume_a="pos")
    assert np.linalg.norm(r.u.ravel() - ref) <= 1e-8 * np.linalg.norm(ref)


def test_ftvcs_denoising_step(rng):
    """A = I, tau = 1: one step is (D^T D + mu/beta I) u = D^T s(D u^0) + mu/beta f,
    the alternating step for TV denoising (Sec. 1.2, eq. (atv) with A = I)."""
    n = 8
    A = np.eye(n * n)
    f = rng.uniform(0, 1, (1, n * n))
    u0 = rng.uniform(0, 1, (n, n))
    mu, beta = 20.0, 5.0
    r = O.ftvcs(A, f, n, mu, beta, 1.0, tol=0, maxit=1, u0=u0)
    D1, D2 = dense_D(n)
    a, b = D1 @ u0.ravel(), D2 @ u0.ravel()
    t = np.hypot(a, b)
    sc = np.where(t > 0, np.maximum(t - 1 / beta, 0) / np.where(t > 0, t, 1), 0)
    rhs = D1.T @ (sc * a) + D2.T @ (sc * b) + mu / beta * f[0]
    ref = np.linalg.solve(D1.T @ D1 + D2.T @ D2 + mu / beta * np.eye(n * n), rhs)
    assert np.allclose(r.u.ravel(), ref, rtol=1e-12, atol=1e-12)


def test_stop_rule_counts(small):
    """(eq. (stop)): the run stops at the first k with ||u^{k+1}-u^k|| <= tol ||u^k||."""
    p, tau = small
    rels = []
    prev = [O.initial_u(p.A, np.atleast_2d(p.f), p.n, None).copy()]

    def rec(k, u):
        rels.append(np.linalg.norm(u - prev[0]) / np.linalg.norm(prev[0]))
        prev[0] = u.copy()
    O.ftvcs(p.A, p.f, p.n, MU, BETA, tau, tol=0, maxit=400, record=rec)
    tol = 1e-3
    first = next(k for k, r in enumerate(rels) if r <= tol) + 1
    r = O.ftvcs(p.A, p.f, p.n, MU, BETA, tau, tol=tol, maxit=400)
    assert r.iters[0] == first
    assert r.rel_change[0] <= tol


def test_batch_equals_single(rng):
    p = synth.make_problem("b", n=16, m=60, batch=3, n_shapes=4, seed_A=3, sigma=[1e-3, 1e-2, 0])
    tau = O.default_tau(p.A)
    for alg in (O.ftvcs, O.iadm):
        rb = alg(p.A, p.f, p.n, 300.0, 10.0, tau, tol=1e-4, maxit=300)
        for b in range(3):
            rs = alg(p.A, p.f[b:b + 1], p.n, 300.0, 10.0, tau, tol=1e-4, maxit=300)
            assert rs.iters[0] == rb.iters[b]
            # BLAS may order the batched product's sums differently: FP64 rounding only
            assert np.allclose(rs.u[0], rb.u[b], rtol=1e-12, atol=1e-14)


# --- IADM -------------------------------------------------------------------------
def test_iadm_dual_certificate(small, iadm_limit):
    """Thm. 4 limit is a solution of (tv): lambda_i in d||D_i u*||, D^T lambda + mu A^T(Au*-f) = 0.

    These conditions certify optimality of u* for (tv) (convexity)."""
    p, _ = small
    u, lam = iadm_limit.u, iadm_limit.lam
    nl = np.hypot(lam[:, 0], lam[:, 1])
    assert nl.max() <= 1 + 1e-10
    Du = O.D(u)
    t = np.hypot(Du[:, 0], Du[:, 1])
    on = t > 1e-8
    assert np.allclose((lam[:, 0] * Du[:, 0] + lam[:, 1] * Du[:, 1])[on], t[on], rtol=1e-8)
    res = O.Dt(lam) + MU * O.gradient(p.A, u, p.f)
    assert np.abs(res).max() <= 1e-10 * MU * np.abs(p.f @ p.A).max()
    assert np.abs(iadm_limit.w - Du).max() <= 1e-12


def test_iadm_objective_matches_primal_dual_solver(small, iadm_limit):
    p, _ = small
    _, fc = chambolle_pock_tv(p.A, p.f[0], p.n, MU, iters=20000)
    obj = O.objective_tv(iadm_limit.u, p.A, p.f, MU)[0]
    assert obj <= fc + 1e-9 * fc
    assert abs(obj - fc) <= 1e-8 * fc


def test_iadm_printed_sign_fails(small, iadm_limit):
    """The printed w-step sign (eq. (iadmw)) does not reach a solution of (tv)."""
    p, tau = small
    with np.errstate(all="ignore"):
        r = O.iadm(p.A, p.f, p.n, MU, BETA, tau, tol=0, maxit=2000, sign=-1)
        obj = O.objective_tv(r.u, p.A, p.f, MU)[0]
    best = O.objective_tv(iadm_limit.u, p.A, p.f, MU)[0]
    assert not np.isfinite(obj) or obj > best * (1 + 1e-3)


def test_iadm_equals_ftvcs_when_lambda_frozen_at_zero(small):
    """With lambda^0 = 0 the first IADM iterate equals the first FTVCS iterate."""
    p, tau = small
    a = O.ftvcs(p.A, p.f, p.n, MU, BETA, tau, tol=0, maxit=1)
    b = O.iadm(p.A, p.f, p.n, MU, BETA, tau, tol=0, maxit=1)
    assert np.array_equal(a.u, b.u)


def test_iadm_step_optimality(small):
    """Each IADM step satisfies the optimality conditions of its two sub-problems
    (the proximal ADM form of App. B, with R_k = 0 and S_k = I/tau - A^T A):

    w-step (minimising (ALP) over w_i):  0 in d||w_i|| - lambda_i^k + beta (w_i - D_i u^k);
    u-step (eq. (linetv)) followed by (udlamb):
        D^T lambda^{k+1} + mu A^T (A u^k - f) + mu/tau (u^{k+1} - u^k) = 0.
    """
    p, tau = small
    for k in (0, 1, 7, 40):
        if k == 0:
            uk = O.initial_u(p.A, np.atleast_2d(p.f), p.n, None)
            lk = np.zeros((1, 2, p.n, p.n))
        else:
            prev = O.iadm(p.A, p.f, p.n, MU, BETA, tau, tol=0, maxit=k)
            uk, lk = prev.u, prev.lam
        nxt = O.iadm(p.A, p.f, p.n, MU, BETA, tau, tol=0, maxit=k + 1)
        w, u1, l1 = nxt.w, nxt.u, nxt.lam
        # w-step
        Du = O.D(uk)
        tw = np.hypot(w[:, 0], w[:, 1])
        nz = tw > 0
        resid = np.where(nz[:, None], w / np.where(nz, tw, 1)[:, None], 0) - lk + BETA * (w - Du)
        assert np.abs(resid[:, :, nz[0]]).max() <= 1e-10
        v = lk + BETA * Du
        assert np.all(np.hypot(v[:, 0], v[:, 1])[~nz] <= 1 + 1e-10)
        # u-step + multiplier update
        r = O.Dt(l1) + MU * O.gradient(p.A, uk, p.f) + MU / tau * (u1 - uk)
        assert np.abs(r).max() <= 1e-9 * MU * np.abs(p.f @ p.A).max(), k


def test_ftvcs_step_optimality(small):
    """Each FTVCS u-step minimises (eq. (eqline)) at fixed w^{k+1}:
    beta D^T (D u^{k+1} - w^{k+1}) + mu A^T (A u^k - f) + mu/tau (u^{k+1} - u^k) = 0."""
    p, tau = small
    for k in (0, 3, 50):
        uk = O.initial_u(p.A, np.atleast_2d(p.f), p.n, None) if k == 0 else \
            O.ftvcs(p.A, p.f, p.n, MU, BETA, tau, tol=0, maxit=k).u
        nxt = O.ftvcs(p.A, p.f, p.n, MU, BETA, tau, tol=0, maxit=k + 1)
        r = BETA * O.Dt(O.D(nxt.u) - nxt.w) + MU * O.gradient(p.A, uk, p.f) \
            + MU / tau * (nxt.u - uk)
        assert np.abs(r).max() <= 1e-9 * MU * np.abs(p.f @ p.A).max(), k


# --- FTVCS with continuation in beta (Sec. 3.1) ------------------------------------
BETAS = [2.0 ** 4, 2.0 ** 5, 2.0 ** 6, 2.0 ** 7]


def test_continuation_single_beta_is_ftvcs(small):
    p, tau = small
    a = O.ftvcs_continuation(p.A, p.f, p.n, MU, [BETA], tau, tol=1e-4, maxit=300)
    b = O.ftvcs(p.A, p.f, p.n, MU, BETA, tau, tol=1e-4, maxit=300)
    assert np.array_equal(a.u, b.u) and np.array_equal(a.iters, b.iters)


def test_continuation_descent_within_each_stage(small):
    """Within a stage beta is fixed, so the descent bound of Thm. 1's step range
    holds for that stage's Huber objective Psi_beta (the warm start only moves the
    starting point)."""
    p, tau = small
    lmax = O.lambda_max(p.A, iters=5000, rtol=1e-14)
    traj = {s: [] for s in range(len(BETAS))}
    start = {}

    def rec(s, k, u):
        traj[s].append(u.copy())
    res_prev = O.initial_u(p.A, np.atleast_2d(p.f), p.n, None).copy()
    for s, beta in enumerate(BETAS):   # the starting point of each stage
        start[s] = res_prev
        res_prev = O.ftvcs(p.A, p.f, p.n, MU, beta, tau, tol=1e-3, maxit=400, u0=res_prev).u
    out = O.ftvcs_continuation(p.A, p.f, p.n, MU, BETAS, tau, tol=1e-3, maxit=400, record=rec)
    assert np.array_equal(out.u, res_prev)
    for s, beta in enumerate(BETAS):
        us = [start[s]] + traj[s]
        psi = [O.huber_objective(u, p.A, p.f, MU, beta)[0] for u in us]
        for k in range(len(us) - 1):
            d2 = np.sum((us[k + 1] - us[k]) ** 2)
            assert psi[k + 1] <= psi[k] - MU * (1.0 / tau - lmax / 2) * d2 + 1e-9 * abs(psi[k])


def test_continuation_approaches_tv_optimum(small):
    """Each stage converges to the minimiser of (atv) for its beta, whose (tv) value
    approaches the optimum of (tv) as beta grows: the gap after the last stage is a
    fraction of the gap of the first stage alone (the independent optimum comes from
    a long Chambolle-Pock run)."""
    p, tau = small
    _, fc = chambolle_pock_tv(p.A, p.f[0], p.n, MU, iters=20000)
    first = O.ftvcs(p.A, p.f, p.n, MU, BETAS[0], tau, tol=0, maxit=3000)
    cont = O.ftvcs_continuation(p.A, p.f, p.n, MU, BETAS, tau, tol=0, maxit=3000)
    gap1 = O.objective_tv(first.u, p.A, p.f, MU)[0] - fc
    gap4 = O.objective_tv(cont.u, p.A, p.f, MU)[0] - fc
    assert gap1 > 0 and gap4 > -1e-9 * fc
    assert gap4 <= gap1 / 4
