"""FTVCS with continuation in beta (Sec. 3.1) through the C ABI, against the FP64
oracle's `ftvcs_continuation` (same tau): fixed iterations per stage to the FP32 bar,
the per-stage stop rule's iteration counts, and the native stage loop equal to stages
run one by one with warm starts (bitwise)."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1001_1774_amd import synth
from tests._parity import TOL_FP32, check, rel

pytestmark = pytest.mark.gpu

BETAS = [2.0 ** 4, 2.0 ** 5, 2.0 ** 6, 2.0 ** 7]


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


@pytest.fixture(scope="module")
def prob():
    p = synth.workload("n32_m307", batch=3, sigma=[1e-3, 1e-3, 1e-2])
    return p, O.default_tau(p.A)




def test_continuation_fixed_iterations_parity(T, prob):
    p, tau = prob
    K = 60
    ref = O.ftvcs_continuation(p.A, p.f, p.n, p.mu, BETAS, tau, tol=0, maxit=K)
    with T.Solver(p.A, p.n) as s:
        s.tau = tau
        out = s.solve_continuation(p.f.astype(np.float32), mu=p.mu, betas=BETAS, tol=0,
                                   maxit=K)
    U = out["u"].cpu().numpy()
    for b in range(p.B):
        assert out["stats"][b]["iters"] == len(BETAS) * K
        check(U[b], ref.u[b], TOL_FP32, f"image {b}", say)


def test_continuation_stop_rule(T, prob):
    """Each stage ends by eq. (stop) at tol = 1e-3; the total count matches the oracle's
    (a stage can differ by one iteration only if its relative change lands within
    FP32 rounding of tol)."""
    p, tau = prob
    ref = O.ftvcs_continuation(p.A, p.f, p.n, p.mu, BETAS, tau, tol=1e-3, maxit=400)
    with T.Solver(p.A, p.n) as s:
        s.tau = tau
        out = s.solve_continuation(p.f.astype(np.float32), mu=p.mu, betas=BETAS, tol=1e-3,
                                   maxit=400)
    it = np.array([st["iters"] for st in out["stats"]])
    say(f"  iters gpu {it.tolist()} oracle {ref.iters.tolist()}")
    assert out["rc"] == T.TVCS_OK
    assert np.all(np.abs(it - ref.iters) <= len(BETAS))
    U = out["u"].cpu().numpy()
    for b in range(p.B):
        e = rel(U[b], ref.u[b])
        assert e <= (1e-5 if it[b] == ref.iters[b] else 5e-3), (b, e)


def test_continuation_equals_warm_started_stages(T, prob):
    p, tau = prob
    F = p.f.astype(np.float32)
    with T.Solver(p.A, p.n) as s:
        s.tau = tau
        out = s.solve_continuation(F, mu=p.mu, betas=BETAS, tol=1e-3, maxit=400)
        u = None
        total = np.zeros(p.B, dtype=np.int64)
        for beta in BETAS:
            r = s.solve_batch(F, mu=p.mu, beta=beta, tol=1e-3, maxit=400, u0=u)
            u = r["u"]
            total += [st["iters"] for st in r["stats"]]
    assert np.array_equal(out["u"].cpu().numpy(), u.cpu().numpy())
    assert [st["iters"] for st in out["stats"]] == total.tolist()
