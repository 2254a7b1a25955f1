"""GPU parity at the full n = 256 workload in the configuration bench.py times.

n = 256, m = 13107, 64 images sharing A (noise 1e-3 on even images, 1e-2 on odd
ones), split bf16 storage, IADM for the 300 iterations the benchmark times:
sampled images of both noise levels against the FP64 oracle on the FP64 A (bar
1e-4, norm and per-pixel; tests/_parity.py), and one of them solved alone against
its slot in the batch (bitwise).  The n = 512 workload is in test_gpu_fullsize_c5.py.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1001_1774_amd import synth
from tests._parity import TOL_LOWP, rel

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
    K, sample = 300, [0, 45]
    F = torch.from_numpy(p.f.astype(np.float32)).cuda()
    say(f"case n=256 m=13107 B=64 split, K={K}, images {sample}")
    with T.Solver(p.A.astype(np.float32), p.n, storage="bf16_split") as s:
        tau = s.tau
        out = s.solve_batch(F, mu=p.mu, beta=p.beta, maxit=K, iadm=True)
        alone = s.solve(F[45], mu=p.mu, beta=p.beta, maxit=K, iadm=True)
    U = out["u"].cpu().numpy()
    assert np.array_equal(alone["u"].cpu().numpy(), U[45])
    say(f"  fresh iterations {[out['stats'][b]['fresh_iters'] for b in sample]} of {K}")

    def progress(k, u):
        if (k + 1) % 50 == 0:
            say(f"  oracle iteration {k + 1}")
    ref = O.iadm(p.A, p.f[sample], p.n, p.mu, p.beta, tau, tol=0, maxit=K, record=progress)
    for j, b in enumerate(sample):
        e = rel(U[b], ref.u[j])
        say(f"  image {b} (sigma {sig[b]:g}): rel err {e:.3e}")
        assert e <= TOL_LOWP
