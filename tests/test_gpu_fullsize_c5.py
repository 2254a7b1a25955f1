"""GPU parity at the largest workload in the configuration bench.py times: n = 512
(262144 pixels), m = 26214 (10 %), 128 images sharing A, IADM, from u^0 = A^T f.

The oracle runs on the de-quantised A, the FP64 matrix the storage format represents
(Sec. 3.2 sizes: 512^2 images), built row block by row block from the same FP64
blocks the GPU's FP32 copy comes from and held whole in host memory (55 GB).  Two
sampled images are compared after K iterations; the bar is 1e-4 for the norm and the
per-pixel error (tests/_parity.py).  K is long enough for the products to run in
both forms: fresh while the iterates still move by more than 2^-8 per iteration,
increments after that (stats["fresh_iters"] counts the fresh ones).
"""
import os
import sys
import threading
import time

import numpy as np
import pytest

import oracle as O
from paper_1001_1774_amd import synth
from tests._parity import TOL_LOWP, check

pytestmark = pytest.mark.gpu

K = 80
SAMPLE = [5, 100]


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
def c5():
    t0 = time.time()
    p = synth.workload("n512_m26214_b128", dtype=np.float32)   # FP32 A (27.5 GB), FP64 f
    say(f"  n512_m26214_b128 generated in {time.time() - t0:.1f}s")
    return p


def dequantized(A32, storage):
    """O.dequantized_A applied to blocks of rows (the formats are row-local), in
    parallel threads, into one FP64 array."""
    m = A32.shape[0]
    out = np.empty(A32.shape, np.float64)
    blk = 256
    nxt = [0]
    lock = threading.Lock()

    def work():
        while True:
            with lock:
                i = nxt[0]
                nxt[0] += blk
            if i >= m:
                return
            out[i:i + blk] = O.dequantized_A(A32[i:i + blk], storage)
    try:
        nt = max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        nt = 8
    ths = [threading.Thread(target=work) for _ in range(nt)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    return out


@pytest.mark.parametrize("storage", ["fp8_rowscale", "bf16"])
def test_n512_m26214_b128_iadm(T, c5, storage):
    import torch
    p = c5
    say(f"case n=512 m=26214 B=128 {storage} IADM K={K}, images {SAMPLE}")
    F = torch.from_numpy(p.f.astype(np.float32)).cuda()
    with T.Solver(p.A, p.n, storage=storage) as s:
        tau = s.tau
        t0 = time.time()
        out = s.solve_batch(F, mu=p.mu, beta=p.beta, maxit=K, iadm=True)
        say(f"  GPU solve {time.time() - t0:.1f}s; fresh iterations "
            f"{[out['stats'][b]['fresh_iters'] for b in SAMPLE]} of {K}")
        alone = s.solve(F[SAMPLE[1]], mu=p.mu, beta=p.beta, maxit=K, iadm=True)
    U = out["u"].cpu().numpy()
    assert np.array_equal(alone["u"].cpu().numpy(), U[SAMPLE[1]])
    for b in SAMPLE:
        fr = out["stats"][b]["fresh_iters"]
        assert 2 <= fr < K, fr          # both forms ran
    t0 = time.time()
    Aq = dequantized(p.A, storage)
    say(f"  de-quantised A in {time.time() - t0:.1f}s")
    t0 = time.time()

    def progress(k, u):
        if (k + 1) % 10 == 0:
            say(f"  oracle iteration {k + 1} ({time.time() - t0:.0f}s)")
    ref = O.iadm(Aq, p.f[SAMPLE].astype(np.float32).astype(np.float64), p.n, p.mu, p.beta,
                 tau, tol=0, maxit=K, record=progress)
    say(f"  oracle {time.time() - t0:.1f}s")
    del Aq
    for j, b in enumerate(SAMPLE):
        check(U[b], ref.u[j], TOL_LOWP, f"image {b}", say)
