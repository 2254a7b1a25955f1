"""GPU test of tvcs_solve_noalloc (the entry point that allocates nothing) through
the C ABI: its results equal tvcs_solve's on the same handle (the same kernels in
the same order: bitwise, same iteration count), on two calls in a row, the second
with a smaller problem, and a problem beyond its scratch array is refused."""
import sys

import numpy as np
import pytest

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


def run_both(T, p, flags, tol, maxit):
    import torch
    h = T.tvcs_create(p.A.astype(np.float32), p.m, p.n)
    assert h
    try:
        f = torch.from_numpy(p.f[0].astype(np.float32)).cuda()
        u_ref = torch.zeros(p.N, dtype=torch.float32, device="cuda")
        u_na = torch.full((p.N,), 7.0, dtype=torch.float32, device="cuda")
        st_ref, st_na = T.tvcs_stats(), T.tvcs_stats()
        rc_ref = T.tvcs_solve(h, f, p.mu, p.beta, tol, maxit, flags, u_ref, None, st_ref)
        rc_na = T.tvcs_solve_noalloc(h, f, p.mu, p.beta, tol, maxit, flags, u_na, st_na)
        assert rc_ref >= 0 and rc_na == rc_ref, (rc_ref, rc_na, T.tvcs_last_error())
        assert st_na.iters == st_ref.iters
        a, b = u_ref.cpu().numpy(), u_na.cpu().numpy()
        say(f"  n={p.n} m={p.m} flags={flags} tol={tol}: iters {st_na.iters}, "
            f"max |diff| {np.abs(a - b).max():.3e}")
        assert np.array_equal(a, b)
        # host pointers work as for tvcs_solve
        u_host = np.zeros(p.N, np.float32)
        assert T.tvcs_solve_noalloc(h, p.f[0].astype(np.float32), p.mu, p.beta, tol, maxit, flags,
                                    u_host, None) == rc_ref
        assert np.array_equal(u_host, a)
    finally:
        T.tvcs_destroy(h)


def test_noalloc_equals_solve_two_calls(T):
    big = synth.workload("n128_m4096")
    small = synth.make_problem("na64", n=64, m=1229, n_shapes=8, seed_A=77, sigma=1e-3)
    run_both(T, big, T.TVCS_IADM, 0.0, 120)       # first call: n = 128, m = 4096
    run_both(T, small, T.TVCS_IADM, 0.0, 60)      # second call: a smaller problem
    run_both(T, small, 0, 1e-3, 400)              # FTVCS with the stop rule


def test_noalloc_rejects_what_it_cannot_hold(T):
    import torch
    # n = 512, m = 26214: 26 row chunks of A^T r partial sums, a 33.1 MiB workspace
    # beyond the 32 MiB array (any values of A do: the call is refused before it
    # computes anything); A (27.5 GB) is made on the device
    n, m = 512, 26214
    A = torch.full((m, n * n), 1e-3, dtype=torch.float32, device="cuda")
    h = T.tvcs_create(A, m, n)
    del A
    torch.cuda.empty_cache()
    assert h
    try:
        f = torch.ones(m, dtype=torch.float32, device="cuda")
        u = torch.zeros(n * n, dtype=torch.float32, device="cuda")
        rc = T.tvcs_solve_noalloc(h, f, 1e3, 10.0, 0.0, 5, 0, u, None)
        assert rc == T.TVCS_EINVAL
        assert "scratch" in T.tvcs_last_error()
    finally:
        T.tvcs_destroy(h)
    q = synth.make_problem("na32", n=32, m=307, n_shapes=4, seed_A=79, sigma=1e-3)
    with T.Solver(q.A, q.n, storage="bf16") as s:
        f = torch.from_numpy(q.f[0].astype(np.float32)).cuda()
        u = torch.zeros(q.N, dtype=torch.float32, device="cuda")
        assert T.tvcs_solve_noalloc(s.h, f, q.mu, q.beta, 0.0, 5, 0, u, None) == \
            T.TVCS_EUNSUPPORTED
