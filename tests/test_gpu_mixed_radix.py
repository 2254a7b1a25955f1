"""GPU parity at image sides that are not powers of two (radix 2/3/4/5 FFTs).

The FFT solve, the shrink pass and the partial-DCT transforms take the mixed-radix
path for these sides; the bars are those of the power-of-two cases (FP32 path:
1e-5 after a fixed number of iterations, 2e-6 for one step), since the rounding of
a radix-3 or radix-5 stage is of the same order as a radix-4 stage's.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1001_1774_amd import synth
from tests._parity import rel

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    from paper_1001_1774_amd import tvcs
    tvcs.lib()
    return tvcs




def tau_for(A):
    return 1.9 / np.linalg.eigvalsh(A @ A.T).max()


@pytest.mark.parametrize("iadm", [False, True], ids=["ftvcs", "iadm"])
@pytest.mark.parametrize("n,K", [(10, 80), (12, 100), (30, 100), (90, 60), (100, 40)])
def test_dense_fixed_iterations(T, n, K, iadm):
    m = int(round(0.25 * n * n))
    p = synth.make_problem("p", n=n, m=m, n_shapes=max(3, min(20, n // 6)), seed_A=31 + n,
                           sigma=1e-3)
    tau = tau_for(p.A)
    say(f"case n={n} m={m} K={K} iadm={iadm}")
    alg = O.iadm if iadm else O.ftvcs
    ref = alg(p.A, p.f, n, p.mu, p.beta, tau, tol=0, maxit=K)
    with T.Solver(p.A, n) as s:
        s.tau = tau
        out = s.solve(p.f[0].astype(np.float32), mu=p.mu, beta=p.beta, maxit=K, iadm=iadm,
                      want_lambda=iadm)
    assert out["stats"]["iters"] == K
    e = rel(out["u"].cpu().numpy(), ref.u[0])
    say(f"  rel err u = {e:.3e}")
    assert e <= 1e-5
    if iadm:
        el = rel(out["lam"].cpu().numpy(), ref.lam[0])
        say(f"  rel err lambda = {el:.3e}")
        assert el <= 1e-4


@pytest.mark.parametrize("n", [24, 180])
def test_dense_one_step_from_warm_start(T, n):
    """One FTVCS step from a noisy u^k: the shrink pass and the FFT solve at one step."""
    m = min(n * n // 8, 2000)
    p = synth.make_problem("p", n=n, m=m, n_shapes=10, seed_A=77 + n, sigma=1e-3,
                           dtype=np.float32)
    A64 = p.A.astype(np.float64)
    rng = np.random.default_rng(n)
    u0 = (p.ubar[0] + 0.05 * rng.standard_normal((n, n))).astype(np.float32)
    tau = 1.9 / O.lambda_max(A64)
    with T.Solver(p.A, n) as s:
        s.tau = tau
        out = s.solve(p.f[0].astype(np.float32), mu=p.mu, beta=p.beta, maxit=1, u0=u0)
    ref = O.ftvcs(A64, p.f[:1].astype(np.float32).astype(np.float64), n, p.mu, p.beta, tau,
                  tol=0, maxit=1, u0=u0.astype(np.float64))
    e = rel(out["u"].cpu().numpy(), ref.u[0])
    say(f"  n={n}: one-step rel err {e:.3e}")
    assert e <= 2e-6


def test_dense_batch_equals_single(T):
    p = synth.make_problem("p", n=24, m=150, batch=5, n_shapes=6, seed_A=91,
                           sigma=[1e-3, 1e-2, 0.0, 1e-3, 5e-3])
    f32 = p.f.astype(np.float32)
    with T.Solver(p.A, p.n) as s:
        out = s.solve_batch(f32, mu=p.mu, beta=p.beta, tol=1e-4, maxit=600, iadm=True)
        U = out["u"].cpu().numpy()
        for b in (1, 4):
            # alone, the image takes the one-pass product (n*n <= 16384): the same
            # sums in another order, so the values agree to rounding
            alone = s.solve(f32[b], mu=p.mu, beta=p.beta, tol=1e-4, maxit=600, iadm=True)
            assert rel(alone["u"].cpu().numpy(), U[b].astype(np.float64)) <= 1e-5
            assert alone["stats"]["iters"] == out["stats"][b]["iters"]


@pytest.mark.parametrize("n", [12, 60, 450])
def test_dct_one_step(T, n):
    p = synth.make_dct_problem("d", n, 0.3, n_shapes=max(3, min(40, n // 6)))
    A = O.PartialDCT(n, p.rows)
    rng = np.random.default_rng(n)
    u0 = (p.ubar[0] + 0.05 * rng.standard_normal((n, n))).astype(np.float32)
    f32 = p.f[0].astype(np.float32)
    with T.Solver.partial_dct(p.rows, n) as s:
        out = s.solve(f32, mu=p.mu, beta=p.beta, maxit=1, u0=u0, objective=True)
    ref = O.ftvcs(A, f32.astype(np.float64)[None], n, p.mu, p.beta, p.tau, tol=0, maxit=1,
                  u0=u0.astype(np.float64))
    e = rel(out["u"].cpu().numpy(), ref.u[0])
    obj = O.objective_tv(out["u"].cpu().numpy().astype(np.float64)[None], A,
                         f32.astype(np.float64)[None], p.mu)[0]
    eo = abs(out["stats"]["objective"] - obj) / obj
    say(f"  n={n}: one-step rel err {e:.3e}, objective rel err {eo:.3e}")
    assert e <= 2e-6
    assert eo <= 1e-6


def test_dct_n450_b4_iadm(T):
    """The partial-DCT experiment's 450 x 450 size: 30 % of the coefficients, four
    images in one batch, 40 IADM iterations against the oracle."""
    p = synth.make_dct_problem("n450", 450, 0.3, batch=4)
    f32 = p.f.astype(np.float32)
    K = 40
    with T.Solver.partial_dct(p.rows, p.n) as s:
        out = s.solve_batch(f32, mu=p.mu, beta=p.beta, maxit=K, iadm=True)
        alone = s.solve(f32[2], mu=p.mu, beta=p.beta, maxit=K, iadm=True)
    U = out["u"].cpu().numpy()
    assert np.array_equal(alone["u"].cpu().numpy(), U[2])
    ref = O.iadm(O.PartialDCT(p.n, p.rows), f32.astype(np.float64), p.n, p.mu, p.beta, p.tau,
                 tol=0, maxit=K)
    for b in range(p.B):
        e = rel(U[b], ref.u[b])
        say(f"  image {b}: rel err {e:.3e}")
        assert e <= 1e-5
