"""MFMA storage at a side whose n^2 is not a multiple of the 256-row groups of the
stored copies: n = 450 (n^2 = 202500, padded to 202752 with zero columns of A and
zero rows of A^T; the paper's largest images are of this size class, Sec. 3.2,
Table 2).  Parity of split storage against the FP64 oracle on the FP64 A and of FP8
storage against the oracle on the de-quantised A, 16 images, at the bar of the
MFMA formats (1e-4, norm and per-pixel); batch invariance and tile-shape
invariance (bitwise) on the padded path."""
import os
import sys
import threading

import numpy as np
import pytest

import oracle as O
from paper_1001_1774_amd import synth
from tests._parity import TOL_LOWP, check

pytestmark = pytest.mark.gpu
K = 20


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
    # m = 20250 measurements of 450 x 450 images (10 %), 16 images, two noise levels
    return synth.make_problem("p450", n=450, m=20250, batch=16, seed_A=45,
                              sigma=[1e-3, 1e-2] * 8)


@pytest.fixture(scope="module")
def tau(prob):
    return O.default_tau(prob.A)


def dequantized(A, storage):
    """The oracle's de-quantised A, in row blocks of 256 on a few threads."""
    out = np.empty(A.shape, np.float64)
    blocks = list(range(0, A.shape[0], 256))
    lock = threading.Lock()

    def work():
        while True:
            with lock:
                if not blocks:
                    return
                i = blocks.pop()
            out[i:i + 256] = O.dequantized_A(A[i:i + 256], storage)
    ths = [threading.Thread(target=work) for _ in range(min(16, len(os.sched_getaffinity(0))))]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    return out


@pytest.mark.parametrize("storage,sample", [("bf16_split", [0, 5, 10, 15]),
                                            ("fp8_rowscale", [0, 15])])
def test_parity_450(T, prob, tau, storage, sample):
    p = prob
    say(f"case n=450 m=20250 B=16 K={K} {storage}")
    A_or = p.A if storage == "bf16_split" else dequantized(p.A, storage)
    ref = O.iadm(A_or, p.f[sample], p.n, p.mu, p.beta, tau, tol=0, maxit=K)
    del A_or
    with T.Solver(p.A.astype(np.float32), p.n, storage=storage) as s:
        s.tau = tau
        out = s.solve_batch(p.f.astype(np.float32), mu=p.mu, beta=p.beta, maxit=K, iadm=True)
        say(f"  tiles {s.tiles}")
    U = out["u"].cpu().numpy()
    assert all(st["iters"] == K for st in out["stats"])
    for j, b in enumerate(sample):
        check(U[b], ref.u[j], TOL_LOWP, f"image {b}", say)


def test_padded_path_is_batch_and_tile_invariant(T, prob, tau):
    p = prob
    F = p.f.astype(np.float32)
    with T.Solver(p.A.astype(np.float32), p.n, storage="bf16_split") as s:
        s.tau = tau
        base = s.solve_batch(F, mu=p.mu, beta=p.beta, maxit=K, iadm=True)["u"].cpu().numpy()
        for b in (3, 11):
            one = s.solve_batch(F[b:b + 1], mu=p.mu, beta=p.beta, maxit=K, iadm=True)
            assert np.array_equal(one["u"].cpu().numpy()[0], base[b]), b
        for shape in [(2, 16, 4, 4, 16, 4), (4, 64, 1, 2, 128, 2)]:
            s.tiles = shape
            out = s.solve_batch(F, mu=p.mu, beta=p.beta, maxit=K, iadm=True)["u"].cpu().numpy()
            same = np.array_equal(out, base)
            say(f"  shape {shape}: bitwise equal {same}")
            assert same, shape
