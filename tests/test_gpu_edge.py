"""GPU parity at the degenerate ends of the problem: one measurement (m = 1), more
measurements than pixels (m > n^2), zero measurements (f = 0, whose exact iterates
are all zero), and ragged row counts for the padded low-precision storage (m = 1,
m = 257: one full 256-row block and one holding a single row).

Bars as in the main parity tests: FP32 path 1e-5 relative iterate error after a
fixed number of iterations, split storage 1e-4 against the FP64 oracle on the FP64 A,
each widened by the path factor S = sum_k ||u^{k+1} - u^k|| / ||u^K|| (from the
oracle's trajectory, per image) where the run's steps dwarf its final iterate: the
per-step rounding (log2(n) eps32 of the increment for the FP32 FFT solve, about
2^-17 of it for the split products) then accumulates to that many times the step
error relative to ||u^K||.  With one measurement the first steps flatten u^0 =
A^T f, a noise-like image, into a nearly flat one, and S reaches the hundreds.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1001_1774_amd import synth

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


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def tau_for(A):
    return 1.9 / np.linalg.eigvalsh(A @ A.T).max()


def oracle_with_path(alg, A, f, n, mu, beta, tau, K):
    """The oracle's iterates after K steps and the path factor S of each image."""
    f = np.atleast_2d(f)
    prev = [O.initial_u(A, f, n, None).reshape(f.shape[0], -1).copy()]
    path = [np.zeros(f.shape[0])]

    def rec(k, u):
        u = np.asarray(u).reshape(f.shape[0], -1)
        path[0] += np.linalg.norm(u - prev[0], axis=1)
        prev[0] = u.copy()
    r = alg(A, f, n, mu, beta, tau, tol=0, maxit=K, record=rec)
    return r, path[0] / np.linalg.norm(r.u.reshape(f.shape[0], -1), axis=1)


@pytest.mark.parametrize("iadm", [False, True], ids=["ftvcs", "iadm"])
@pytest.mark.parametrize("n,m", [(8, 1), (32, 1), (8, 100), (16, 400)])
def test_extreme_measurement_counts(T, n, m, iadm):
    """m = 1 (a single row of A) and m > n^2 (more rows than pixels)."""
    p = synth.make_problem("e", n=n, m=m, n_shapes=3, seed_A=5 + m, sigma=1e-3)
    tau = tau_for(p.A)
    K = 60
    say(f"case n={n} m={m} iadm={iadm}")
    alg = O.iadm if iadm else O.ftvcs
    ref, S = oracle_with_path(alg, p.A, p.f[:1].astype(np.float32).astype(np.float64), n,
                              p.mu, p.beta, tau, K)
    with T.Solver(p.A.astype(np.float32), n) as s:
        s.tau = tau
        out = s.solve(p.f[0].astype(np.float32), mu=p.mu, beta=p.beta, maxit=K, iadm=iadm)
    assert out["stats"]["iters"] == K
    e = rel(out["u"].cpu().numpy(), ref.u[0])
    bound = max(1e-5, 2.0 ** -24 * np.log2(n) * S[0])
    say(f"  rel err u = {e:.3e} (bound {bound:.2e}, S = {S[0]:.1f})")
    assert e <= bound


@pytest.mark.parametrize("storage", ["fp32", "bf16_split"])
@pytest.mark.parametrize("iadm", [False, True], ids=["ftvcs", "iadm"])
def test_zero_measurements_give_zero_iterates(T, storage, iadm):
    """f = 0: u^0 = A^T f = 0, every shrinkage of 0 is 0 and g = 0, so every iterate
    is exactly zero.  With tol > 0 the inclusive stop rule 0 <= tol * 0 holds after
    the first update; with tol = 0 the run takes maxit iterations."""
    p = synth.make_problem("z", n=32, m=307, batch=3, n_shapes=3, seed_A=9)
    F = np.zeros((3, p.m), np.float32)
    with T.Solver(p.A.astype(np.float32), p.n, storage=storage) as s:
        out = s.solve_batch(F, mu=p.mu, beta=p.beta, tol=1e-3, maxit=50, iadm=iadm,
                            want_lambda=iadm)
        assert np.all(out["u"].cpu().numpy() == 0.0)
        assert [st["iters"] for st in out["stats"]] == [1, 1, 1]
        assert all(st["status"] == T.TVCS_OK for st in out["stats"])
        if iadm:
            assert np.all(out["lam"].cpu().numpy() == 0.0)
        out = s.solve_batch(F, mu=p.mu, beta=p.beta, tol=0.0, maxit=20, iadm=iadm)
        assert np.all(out["u"].cpu().numpy() == 0.0)
        assert [st["iters"] for st in out["stats"]] == [20, 20, 20]


@pytest.mark.parametrize("m", [1, 257])
def test_ragged_rows_in_padded_storage(T, m):
    """Split storage pads A to whole 256-row blocks with zero rows: m = 1 (255 zero
    rows) and m = 257 (a second block with one real row)."""
    p = synth.make_problem("r", n=32, m=m, batch=3, n_shapes=4, seed_A=13 + m, sigma=1e-3)
    tau = tau_for(p.A)
    K = 40
    ref, S = oracle_with_path(O.ftvcs, p.A, p.f, p.n, p.mu, p.beta, tau, K)
    with T.Solver(p.A.astype(np.float32), p.n, storage="bf16_split") as s:
        s.tau = tau
        out = s.solve_batch(p.f.astype(np.float32), mu=p.mu, beta=p.beta, maxit=K)
    U = out["u"].cpu().numpy()
    for b in range(p.B):
        e = rel(U[b], ref.u[b])
        bound = max(1e-4, 2.0 ** -17 * S[b])
        say(f"  m={m} image {b}: rel err {e:.3e} (bound {bound:.2e}, S = {S[b]:.1f})")
        assert e <= bound
