"""GPU parity of the batched MFMA path (BF16, split BF16, FP8 storage of A).

Bars: split storage must stay within 1e-4 relative iterate error of the FP64
oracle on the FP64 A after a fixed number of iterations.  Plain BF16 and FP8
storage must stay within 1e-4 of the oracle run on the de-quantised A they
represent (FP64 arithmetic): what remains is the rounding of the batch operand
(two bf16 parts in fresh products, the one-part increment otherwise, whose rounding
is carried to the next increment) and the products' FP32 accumulation.  Their error
against the FP64-A oracle is set by the storage format itself; it is reported
(relative error and PSNR), not bounded tightly.
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


@pytest.fixture(scope="module")
def batch64():
    # n = 64, m = 819 (20 %), 20 images with 10-40 shapes, two noise levels
    sig = [1e-3 if i % 2 == 0 else 1e-2 for i in range(20)]
    return synth.make_problem("b64", n=64, m=819, batch=20, seed_A=31, sigma=sig)


@pytest.mark.parametrize("iadm", [False, True], ids=["ftvcs", "iadm"])
def test_split_batch_parity_vs_fp64(T, batch64, iadm):
    p = batch64
    tau = tau_for(p.A)
    K = 150
    say(f"case split n=64 m=819 B=20 K={K} iadm={iadm}")
    ref = (O.iadm if iadm else O.ftvcs)(p.A, p.f, p.n, p.mu, p.beta, tau, tol=0, maxit=K)
    with T.Solver(p.A, p.n, storage="bf16_split") as s:
        s.tau = tau
        out = s.solve_batch(p.f.astype(np.float32), mu=p.mu, beta=p.beta, maxit=K, iadm=iadm)
    U = out["u"].cpu().numpy()
    errs = [rel(U[b], ref.u[b]) for b in range(p.B)]
    say(f"  max rel err {max(errs):.3e}  median {np.median(errs):.3e}  ms {out['stats'][0]['ms']:.1f}")
    assert all(st["iters"] == K for st in out["stats"])
    assert max(errs) <= 1e-4


@pytest.mark.parametrize("storage", ["bf16", "fp8_rowscale"])
def test_lowp_against_dequantised_oracle(T, batch64, storage):
    p = batch64
    Aq = O.dequantized_A(p.A, storage)
    tau = tau_for(Aq)
    K = 100
    say(f"case {storage} n=64 m=819 B=20 K={K}")
    ref_q = O.iadm(Aq, p.f, p.n, p.mu, p.beta, tau, tol=0, maxit=K)
    ref_64 = O.iadm(p.A, p.f, p.n, p.mu, p.beta, tau, tol=0, maxit=K)
    with T.Solver(p.A, p.n, storage=storage) as s:
        s.tau = tau
        say(f"  lambda_max gpu {s.lambda_max:.5f} dequantised {1.9 / tau:.5f}")
        assert abs(s.lambda_max - 1.9 / tau) <= 5e-3 * (1.9 / tau)
        out = s.solve_batch(p.f.astype(np.float32), mu=p.mu, beta=p.beta, maxit=K, iadm=True)
    U = out["u"].cpu().numpy()
    eq = max(rel(U[b], ref_q.u[b]) for b in range(p.B))
    e64 = max(rel(U[b], ref_64.u[b]) for b in range(p.B))
    psnr = min(20 * np.log10(np.abs(ref_64.u[b]).max() / np.sqrt(np.mean((U[b] - ref_64.u[b]) ** 2)))
               for b in range(p.B))
    say(f"  max rel err vs dequantised-A oracle {eq:.3e}; vs FP64-A oracle {e64:.3e} "
        f"(min PSNR {psnr:.1f} dB)")
    assert eq <= 1e-4
    assert e64 <= 0.2


def test_lowp_batch_invariance(T, batch64):
    """An image gives the same bits alone and in any slot of a batch."""
    p = batch64
    tau = tau_for(p.A)
    F = p.f.astype(np.float32)
    with T.Solver(p.A, p.n, storage="bf16_split") as s:
        s.tau = tau
        rb = s.solve_batch(F, mu=p.mu, beta=p.beta, tol=1e-3, maxit=200, iadm=True)
        for b in (0, 7, 19):
            r1 = s.solve(F[b], mu=p.mu, beta=p.beta, tol=1e-3, maxit=200, iadm=True)
            assert r1["stats"]["iters"] == rb["stats"][b]["iters"]
            assert np.array_equal(r1["u"].cpu().numpy(), rb["u"][b].cpu().numpy()), b
        # a different batch composition: the image in another slot
        perm = np.roll(np.arange(p.B), 5)
        rp = s.solve_batch(F[perm], mu=p.mu, beta=p.beta, tol=1e-3, maxit=200, iadm=True)
        for slot in (0, 3, 12):
            b = perm[slot]
            assert np.array_equal(rp["u"][slot].cpu().numpy(), rb["u"][b].cpu().numpy())


@pytest.mark.parametrize("storage", ["bf16", "fp8_rowscale"])
def test_lowp_storage_reaches_tolerance(T, batch64, storage):
    """With the batch operand split hi + lo, plain BF16 / FP8 storage converges: the
    stop rule fires at tol = 1e-3 well before the cap, at the iteration the oracle on
    the de-quantised A stops (+-1)."""
    p = batch64
    Aq = O.dequantized_A(p.A, storage)
    tau = tau_for(Aq)
    ref = O.iadm(Aq, p.f, p.n, p.mu, p.beta, tau, tol=1e-3, maxit=1000)
    with T.Solver(p.A, p.n, storage=storage) as s:
        s.tau = tau
        out = s.solve_batch(p.f.astype(np.float32), mu=p.mu, beta=p.beta, tol=1e-3, maxit=1000,
                            iadm=True)
    it = np.array([st["iters"] for st in out["stats"]])
    say(f"  {storage}: iters {it.tolist()}\n  oracle {ref.iters.tolist()}")
    assert out["rc"] == T.TVCS_OK and it.max() < 1000
    assert np.all(np.abs(it - ref.iters) <= 1)


def test_lowp_stop_rule_per_image(T, batch64):
    p = batch64
    tau = tau_for(p.A)
    ref = O.ftvcs(p.A, p.f, p.n, p.mu, p.beta, tau, tol=1e-3, maxit=300)
    with T.Solver(p.A, p.n, storage="bf16_split") as s:
        s.tau = tau
        out = s.solve_batch(p.f.astype(np.float32), mu=p.mu, beta=p.beta, tol=1e-3, maxit=300)
    it_gpu = np.array([st["iters"] for st in out["stats"]])
    say(f"  iters gpu {it_gpu.tolist()}\n  iters ref {ref.iters.tolist()}")
    assert np.all(np.abs(it_gpu - ref.iters) <= 1)
    assert len(set(it_gpu.tolist())) > 1     # images really stop at different counts


@pytest.mark.parametrize("B", [1, 16, 33, 130, 300])
def test_lowp_batch_sizes(T, B):
    """Padded batches (1 -> 16, 33 -> 48, 130 -> 144, 300 -> 304: image groups of
    256, 32 and 16) run and agree with the oracle."""
    p = synth.make_problem("bs", n=32, m=307, batch=B, seed_A=41, n_shapes=6)
    tau = tau_for(p.A)
    ref = O.ftvcs(p.A, p.f, p.n, p.mu, p.beta, tau, tol=0, maxit=40)
    with T.Solver(p.A, p.n, storage="bf16_split") as s:
        s.tau = tau
        out = s.solve_batch(p.f.astype(np.float32), mu=p.mu, beta=p.beta, maxit=40)
    U = out["u"].cpu().numpy()
    e = max(rel(U[b], ref.u[b]) for b in range(B))
    say(f"  B={B}: max rel err {e:.3e}")
    assert e <= 1e-4


@pytest.mark.parametrize("storage", ["bf16", "bf16_split", "fp8_rowscale"])
def test_lowp_256_image_groups_are_batch_invariant(T, storage):
    """A batch of 272 images runs as one 256-image group (split storage) or two
    128-image groups (BF16, FP8), and one 16-image group; an image gives the same
    bits there as alone (a 16-image group), in each storage."""
    p = synth.make_problem("g256", n=32, m=307, batch=272, seed_A=43, n_shapes=6)
    F = p.f.astype(np.float32)
    with T.Solver(p.A, p.n, storage=storage) as s:
        rb = s.solve_batch(F, mu=p.mu, beta=p.beta, maxit=30, iadm=True)
        for b in (0, 137, 255, 271):
            r1 = s.solve(F[b], mu=p.mu, beta=p.beta, maxit=30, iadm=True)
            assert np.array_equal(r1["u"].cpu().numpy(), rb["u"][b].cpu().numpy()), b
    say(f"  {storage}: images 0, 137, 255, 271 equal alone and in the batch of 272")
