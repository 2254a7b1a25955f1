"""GPU parity at the full workload sizes, in the launch configuration bench.py times.

* n = 256, m = 13107, 64 images sharing A, split bf16 storage: sampled images after a
  fixed number of IADM iterations against the FP64 oracle on the FP64 A (bar 1e-4),
  and one of them solved alone against its slot in the batch (bitwise).
* n = 512, m = 26214, 128 images sharing A, FP8-E4M3 with row scales: the oracle can
  only afford a few rows of the de-quantised A, so each image measures one row
  (f_b = e_{i_b}); from u^0 = 0 one FTVCS step gives g = -A^T e_i = -(row i of A),
  so u^1 = (D^T D + c I)^{-1} (c tau a_i), which the oracle computes one image at a
  time from that row alone.  This runs the adjoint product, the batch-operand split,
  the shrink pass and the FFT solve at full size with all 128 images in flight.  The
  image alone equals its slot in the batch (bitwise).
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




def test_n256_m13107_b64_split_sampled_images(T):
    import torch
    sig = [1e-3 if i % 2 == 0 else 1e-2 for i in range(64)]
    p = synth.workload("n256_m13107_b64", sigma=sig)            # FP64 A (6.9 GB)
    K, sample = 10, [0, 45]
    F = torch.from_numpy(p.f.astype(np.float32)).cuda()
    say(f"case n=256 m=13107 B=64 split, K={K}, images {sample}")
    with T.Solver(p.A.astype(np.float32), p.n, storage="bf16_split") as s:
        tau = s.tau
        out = s.solve_batch(F, mu=p.mu, beta=p.beta, maxit=K, iadm=True)
        alone = s.solve(F[45], mu=p.mu, beta=p.beta, maxit=K, iadm=True)
    U = out["u"].cpu().numpy()
    assert np.array_equal(alone["u"].cpu().numpy(), U[45])
    ref = O.iadm(p.A, p.f[sample], p.n, p.mu, p.beta, tau, tol=0, maxit=K)
    for j, b in enumerate(sample):
        e = rel(U[b], ref.u[j])
        say(f"  image {b}: rel err {e:.3e}")
        assert e <= 1e-4


def test_n512_m26214_b128_fp8_first_step(T):
    import torch
    p = synth.workload("n512_m26214_b128", dtype=np.float32)    # FP32 A (27.5 GB)
    m, n, B = p.m, p.n, p.B
    rows = np.array([(b * 205 + 17) % m for b in range(B)])
    rows[-1] = m - 1                                             # the last row of A
    assert len(set(rows.tolist())) == B
    F = np.zeros((B, m), np.float32)
    F[np.arange(B), rows] = 1.0
    Fd = torch.from_numpy(F).cuda()
    sample = [0, 63, B - 1]
    say(f"case n=512 m=26214 B=128 fp8, one FTVCS step from u0 = 0, images {sample}")
    with T.Solver(p.A, n, storage="fp8_rowscale") as s:
        tau = s.tau
        out = s.solve_batch(Fd, mu=p.mu, beta=p.beta, maxit=1, u0_zero=True)
        alone = s.solve(Fd[63], mu=p.mu, beta=p.beta, maxit=1, u0_zero=True)
    U = out["u"].cpu().numpy()
    assert np.array_equal(alone["u"].cpu().numpy(), U[63])
    c = p.mu / (p.beta * tau)
    for b in sample:
        a_i = O.dequantized_A(p.A[rows[b]:rows[b] + 1], "fp8_rowscale")[0]
        ref = O.solve_u(c * tau * a_i.reshape(n, n), c)
        e = rel(U[b], ref)
        say(f"  image {b} (row {rows[b]}): rel err {e:.3e}")
        assert e <= 1e-4
