"""GPU parity of IADM with inner BB / non-monotone line-search steps on its
u-subproblem (TVCS_BB_STEPS, the acceleration of the concluding remarks, Sec. 4)
against the oracle's iadm_bb (FP32 storage); batch invariance; the flag's limits.

BB iterations amplify rounding: in the FP64 oracle itself a relative perturbation
of 1e-7 in f grows to about 1e-2 in u after 30 to 60 outer iterations (n = 32,
J = 3: 1e-7 up to 20 iterations, 3e-4 at 22, 2e-2 at 30; C2: 2e-6 at 18, 1e-2 at
33), because long BB lengths (up to a few hundred) multiply the error of the
direction and the halvings of the line search switch on small differences.  The
bars below come from a rounding model of the FP32 path: the oracle's iteration
with every product, FFT solve and stored vector given a relative error of 1e-7
(FP32 storage and sums), four seeds; the bar is about three times the largest
model error, and 1e-5 (the FP32 bar of the plain iterations) where that is
smaller.  The counts include steps with halvings (n = 32, J = 8: outer iterations
4 and 5).  Longer runs are compared where the method goes: to the same fixed
point, at a rate like the oracle's."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1001_1774_amd import synth
from tests._parity import check

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


# (workload, inner steps J, outer iterations K, bar): model error max over 4 seeds
# 5.7e-7 (J = 8, K = 3), 7.8e-7 (C2, K = 4), 1.2e-5 (J = 8, K = 5), 2.6e-5 (J = 3,
# K = 15)
CASES = [("n32_m307", 8, 3, 1e-5), ("n128_m4096", 3, 4, 1e-5), ("n32_m307", 8, 5, 5e-5),
         ("n32_m307", 3, 15, 1e-4)]


@pytest.mark.parametrize("name,J,K,bar", CASES)
def test_bb_parity(T, name, J, K, bar):
    p = synth.workload(name)
    tau = O.default_tau(p.A)
    say(f"case {name} J={J} K={K}")
    ref = O.iadm_bb(p.A, p.f[:1], p.n, p.mu, p.beta, tau, tol=0, maxit=K, inner=J)
    with T.Solver(p.A.astype(np.float32), p.n) as s:
        s.tau = tau
        out = s.solve(p.f[0].astype(np.float32), mu=p.mu, beta=p.beta, maxit=K, iadm=True,
                      bb_steps=J, want_lambda=True)
    assert out["stats"]["iters"] == K
    check(out["u"].cpu().numpy(), ref.u[0], bar, "u", say)
    lam = out["lam"].cpu().numpy()
    el = float(np.linalg.norm(lam - ref.lam[0]) / np.linalg.norm(ref.lam[0]))
    say(f"  lambda rel err {el:.3e}")
    assert el <= 10 * bar   # beta (D u - q): a difference of close fields


# One-pass inner steps where that product gives each thread 2 and 3 float4 groups of
# columns (n = 80, 100; 100 also takes the mixed-radix FFTs), J = 3, K = 4: model error
# (4 seeds) 7.8e-7 and 7.7e-7, so the FP32 bar.
SIDE_CASES = [(80, 1600), (100, 2500)]


@pytest.mark.parametrize("n,m", SIDE_CASES)
def test_bb_parity_one_pass_sides(T, n, m):
    p = synth.make_problem(f"bbs{n}", n=n, m=m, batch=1, seed_A=50 + n, sigma=[1e-3])
    tau = O.default_tau(p.A)
    say(f"case n={n} m={m} J=3 K=4")
    ref = O.iadm_bb(p.A, p.f, p.n, p.mu, p.beta, tau, tol=0, maxit=4, inner=3)
    with T.Solver(p.A.astype(np.float32), p.n) as s:
        s.tau = tau
        out = s.solve(p.f[0].astype(np.float32), mu=p.mu, beta=p.beta, maxit=4, iadm=True,
                      bb_steps=3)
    assert out["stats"]["iters"] == 4
    check(out["u"].cpu().numpy(), ref.u[0], 1e-5, "u", say)


# n = 144 (N = 20736): the two-pass products, and 20 blocks of 1037 pixels per image in
# the step-length and update passes, so those passes also run the loop that follows
# each thread's first 4 pixels; J = 3, K = 4, the FP32 bar.
def test_bb_parity_two_pass_side_144(T):
    p = synth.make_problem("bbs144", n=144, m=2074, batch=1, seed_A=194, sigma=[1e-3])
    tau = O.default_tau(p.A)
    say("case n=144 m=2074 J=3 K=4")
    ref = O.iadm_bb(p.A, p.f, p.n, p.mu, p.beta, tau, tol=0, maxit=4, inner=3)
    with T.Solver(p.A.astype(np.float32), p.n) as s:
        s.tau = tau
        out = s.solve(p.f[0].astype(np.float32), mu=p.mu, beta=p.beta, maxit=4, iadm=True,
                      bb_steps=3)
    assert out["stats"]["iters"] == 4
    check(out["u"].cpu().numpy(), ref.u[0], 1e-5, "u", say)


def test_bb_batch_equals_single_and_stop_rule(T):
    """Per-image stopping against the oracle's counts (n = 32, tol 1e-3), for three
    images solved together (two-pass products) and for each solved alone (one-pass
    inner steps: A p and A^T A p from one read of A, g carried); and batch invariance
    where both take the two-pass products (n = 144): bit for bit, same counts."""
    p = synth.make_problem("bbb", n=32, m=307, batch=3, seed_A=31, sigma=[1e-3, 1e-2, 1e-3])
    tau = O.default_tau(p.A)
    F = p.f.astype(np.float32)
    ref = O.iadm_bb(p.A, p.f, p.n, p.mu, p.beta, tau, tol=1e-3, maxit=300, inner=3)
    lim = np.maximum(2, 0.25 * ref.iters)
    with T.Solver(p.A.astype(np.float32), p.n) as s:
        s.tau = tau
        rb = s.solve_batch(F, mu=p.mu, beta=p.beta, tol=1e-3, maxit=300, iadm=True, bb_steps=3)
        it = np.array([st["iters"] for st in rb["stats"]])
        one = np.array([s.solve(F[b], mu=p.mu, beta=p.beta, tol=1e-3, maxit=300, iadm=True,
                                bb_steps=3)["stats"]["iters"] for b in range(3)])
    say(f"  outer iterations batch {it.tolist()} alone {one.tolist()} oracle {ref.iters.tolist()}")
    assert np.all(np.abs(it - ref.iters) <= lim)
    assert np.all(np.abs(one - ref.iters) <= lim)
    q = synth.make_problem("bbb144", n=144, m=2074, batch=3, seed_A=35, sigma=[1e-3, 1e-2, 0])
    Fq = q.f.astype(np.float32)
    with T.Solver(q.A.astype(np.float32), q.n) as s:
        rb = s.solve_batch(Fq, mu=q.mu, beta=q.beta, tol=1e-3, maxit=100, iadm=True, bb_steps=3)
        for b in range(3):
            r1 = s.solve(Fq[b], mu=q.mu, beta=q.beta, tol=1e-3, maxit=100, iadm=True, bb_steps=3)
            assert r1["stats"]["iters"] == rb["stats"][b]["iters"]
            assert np.array_equal(r1["u"].cpu().numpy(), rb["u"][b].cpu().numpy())


def test_bb_reaches_the_oracle_fixed_point(T):
    """n = 32, J = 3, stop at a relative change of 1e-6: the oracle stops after about
    550 outer iterations at 2.7e-4 from its own limit (6000 iterations, change
    1.6e-9); the GPU run stops at a similar count, as close to that limit."""
    p = synth.workload("n32_m307")
    tau = O.default_tau(p.A)
    star = O.iadm_bb(p.A, p.f[:1], p.n, p.mu, p.beta, tau, tol=1e-9, maxit=6000, inner=3)
    ref = O.iadm_bb(p.A, p.f[:1], p.n, p.mu, p.beta, tau, tol=1e-6, maxit=3000, inner=3)
    with T.Solver(p.A.astype(np.float32), p.n) as s:
        s.tau = tau
        out = s.solve(p.f[0].astype(np.float32), mu=p.mu, beta=p.beta, tol=1e-6, maxit=3000,
                      iadm=True, bb_steps=3)
    u = out["u"].cpu().numpy().astype(np.float64)
    dg = float(np.linalg.norm(u - star.u[0]) / np.linalg.norm(star.u[0]))
    do = float(np.linalg.norm(ref.u[0] - star.u[0]) / np.linalg.norm(star.u[0]))
    it = out["stats"]["iters"]
    say(f"  distance to the limit: gpu {dg:.2e} after {it}, oracle {do:.2e} after {ref.iters[0]}")
    assert it < 3000
    assert 0.6 * ref.iters[0] <= it <= 1.6 * ref.iters[0]
    assert dg <= max(3 * do, 1e-5)


# MFMA storage: every product is fresh, its batch operand split into two bf16 parts
# (2^-17 of v left, about 7.6e-6 per product against ~1e-7 in FP32).  The same
# rounding model with that product error gives (max over 4 seeds): n = 32, J = 8,
# K = 3: 3.1e-5; n = 128, J = 3, K = 4: 4.7e-5 (bf16; split adds A's own 2^-16).
# Bars: about three times those; bf16 and FP8 against the oracle on the de-quantised A,
# split against the FP64 A.
LOWP_CASES = [("n32_m307", 8, 3, "bf16", 1e-4), ("n32_m307", 8, 3, "fp8_rowscale", 1e-4),
              ("n128_m4096", 3, 4, "bf16", 1.5e-4), ("n128_m4096", 3, 4, "bf16_split", 3e-4)]


@pytest.mark.parametrize("name,J,K,storage,bar", LOWP_CASES)
def test_bb_parity_mfma_storage(T, name, J, K, storage, bar):
    p = synth.workload(name)
    A_or = p.A if storage == "bf16_split" else O.dequantized_A(p.A, storage)
    tau = O.default_tau(A_or)
    say(f"case {name} J={J} K={K} {storage}")
    ref = O.iadm_bb(A_or, p.f[:1], p.n, p.mu, p.beta, tau, tol=0, maxit=K, inner=J)
    with T.Solver(p.A.astype(np.float32), p.n, storage=storage) as s:
        s.tau = tau
        out = s.solve(p.f[0].astype(np.float32), mu=p.mu, beta=p.beta, maxit=K, iadm=True,
                      bb_steps=J)
    assert out["stats"]["iters"] == K and out["stats"]["fresh_iters"] == K
    check(out["u"].cpu().numpy(), ref.u[0], bar, "u", say)


def test_bb_mfma_storage_batch_invariance_and_limit(T):
    """bf16 storage, n = 32, J = 3: three images solved together equal each solved
    alone (bitwise, same outer counts); at tol 1e-5 the first image stops near the
    oracle's limit on the de-quantised A, as the oracle itself does."""
    p = synth.make_problem("bbm", n=32, m=307, batch=3, seed_A=33, sigma=[1e-3, 1e-2, 1e-3])
    A_or = O.dequantized_A(p.A, "bf16")
    tau = O.default_tau(A_or)
    F = p.f.astype(np.float32)
    with T.Solver(p.A.astype(np.float32), p.n, storage="bf16") as s:
        s.tau = tau
        rb = s.solve_batch(F, mu=p.mu, beta=p.beta, tol=1e-5, maxit=3000, iadm=True, bb_steps=3)
        for b in range(3):
            r1 = s.solve(F[b], mu=p.mu, beta=p.beta, tol=1e-5, maxit=3000, iadm=True, bb_steps=3)
            assert r1["stats"]["iters"] == rb["stats"][b]["iters"]
            assert np.array_equal(r1["u"].cpu().numpy(), rb["u"][b].cpu().numpy())
    star = O.iadm_bb(A_or, p.f[:1], p.n, p.mu, p.beta, tau, tol=1e-9, maxit=6000, inner=3)
    ref = O.iadm_bb(A_or, p.f[:1], p.n, p.mu, p.beta, tau, tol=1e-5, maxit=3000, inner=3)
    u = rb["u"][0].cpu().numpy().astype(np.float64)
    dg = float(np.linalg.norm(u - star.u[0]) / np.linalg.norm(star.u[0]))
    do = float(np.linalg.norm(ref.u[0] - star.u[0]) / np.linalg.norm(star.u[0]))
    it = rb["stats"][0]["iters"]
    say(f"  distance to the limit: gpu {dg:.2e} after {it}, oracle {do:.2e} after {ref.iters[0]}")
    assert it < 3000
    assert dg <= max(3 * do, 1e-4)


def test_bb_flag_limits(T):
    import torch
    p = synth.workload("n32_m307")
    f = torch.from_numpy(p.f[0].astype(np.float32)).cuda()
    with T.Solver(p.A.astype(np.float32), p.n) as s:
        with pytest.raises(T.TvcsError) as ei:
            s.solve(f, mu=p.mu, beta=p.beta, maxit=5, iadm=False, bb_steps=3)
        assert ei.value.code == T.TVCS_EINVAL
        one = s.solve(f, mu=p.mu, beta=p.beta, maxit=20, iadm=True, bb_steps=1)["u"]
        plain = s.solve(f, mu=p.mu, beta=p.beta, maxit=20, iadm=True)["u"]
        assert np.array_equal(one.cpu().numpy(), plain.cpu().numpy())
    q = synth.make_dct_problem("bbdct", 16, 0.3)
    with T.Solver.partial_dct(q.rows, q.n) as s:
        with pytest.raises(T.TvcsError) as ei:
            s.solve(q.f[0].astype(np.float32), mu=q.mu, beta=q.beta, maxit=5, iadm=True,
                    bb_steps=3)
        assert ei.value.code == T.TVCS_EUNSUPPORTED
