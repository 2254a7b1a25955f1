"""GPU parity at the degenerate ends of the problem: one measurement (m = 1), more
measurements than pixels (m > n^2), zero measurements (f = 0, whose exact iterates
are all zero), and ragged row counts for the padded low-precision storage (m = 1,
m = 257: one full 256-row block and one holding a single row).

Bars as in the main parity tests (tests/_parity.py): FP32 path 1e-5, split storage
1e-4 against the FP64 oracle on the FP64 A, for the norm-relative and the per-pixel
error after a fixed number of iterations.  With one measurement (m = 1) the first
steps flatten u^0 = A^T f, a noise-like image, into a nearly flat one: the steps are
hundreds of times the final iterate, and the rounding of each step (a fixed
fraction of it) is large next to ||u^K||.  These cases carry fixed bounds of their
own (DEGENERATE in tests/_parity.py).
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1001_1774_amd import synth
from tests._parity import bar_for, check, rel

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
@pytest.mark.parametrize("n,m", [(8, 1), (32, 1), (8, 100), (16, 400)])
def test_extreme_measurement_counts(T, n, m, iadm):
    """m = 1 (a single row of A) and m > n^2 (more rows than pixels)."""
    p = synth.make_problem("e", n=n, m=m, n_shapes=3, seed_A=5 + m, sigma=1e-3)
    tau = tau_for(p.A)
    K = 60
    say(f"case n={n} m={m} iadm={iadm}")
    alg = O.iadm if iadm else O.ftvcs
    ref = alg(p.A, p.f[:1].astype(np.float32).astype(np.float64), n, p.mu, p.beta, tau,
              tol=0, maxit=K)
    with T.Solver(p.A.astype(np.float32), n) as s:
        s.tau = tau
        out = s.solve(p.f[0].astype(np.float32), mu=p.mu, beta=p.beta, maxit=K, iadm=iadm)
    assert out["stats"]["iters"] == K
    check(out["u"].cpu().numpy(), ref.u[0], bar_for(n, m), "u", say)


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
    ref = O.ftvcs(p.A, p.f, p.n, p.mu, p.beta, tau, tol=0, maxit=K)
    with T.Solver(p.A.astype(np.float32), p.n, storage="bf16_split") as s:
        s.tau = tau
        out = s.solve_batch(p.f.astype(np.float32), mu=p.mu, beta=p.beta, maxit=K)
    U = out["u"].cpu().numpy()
    for b in range(p.B):
        check(U[b], ref.u[b], bar_for(p.n, m, "bf16_split"), f"m={m} image {b}", say)


@pytest.mark.parametrize("storage", ["fp32", "bf16"])
def test_batch_beyond_device_memory_is_refused(T, storage):
    """A batch whose workspace exceeds the device (2^27 images of 32 x 32: half a TB of
    iterates alone) is refused with TVCS_ENOMEM before any buffer is touched, and the
    handle keeps working: the next solve gives the same bits as before."""
    import torch
    p = synth.make_problem("big", n=32, m=307, batch=1, seed_A=81)
    with T.Solver(p.A.astype(np.float32), p.n, storage=storage) as s:
        f = p.f[0].astype(np.float32)
        u1 = s.solve(f, mu=p.mu, beta=p.beta, maxit=30, iadm=True)["u"].cpu().numpy()
        F = torch.from_numpy(f[None]).cuda()
        U = torch.empty(1, p.N, dtype=torch.float32, device="cuda")
        rc = T.tvcs_solve_batch(s.h, F, 1 << 27, p.mu, p.beta, 0.0, 30, T.TVCS_IADM, U)
        say(f"  {storage}: rc {rc}: {T.tvcs_last_error()}")
        assert rc == T.TVCS_ENOMEM
        u2 = s.solve(f, mu=p.mu, beta=p.beta, maxit=30, iadm=True)["u"].cpu().numpy()
        assert np.array_equal(u1, u2)
