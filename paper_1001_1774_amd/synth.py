"""Seeded synthetic inputs for TV/L2 reconstruction from dense random projections.

This module only *draws* inputs: piecewise-constant test images, the dense
Gaussian encoding matrix A, and the noisy observation f = A u_bar + noise of
the observation model (Sec. 1, eq. (obser), additive Gaussian noise).  It holds
none of the reconstruction method's arithmetic, so both the GPU library's tests
and the FP64 oracle can take their inputs from here without sharing any solver
code.

Recipe (the paper's phantom and natural images are not available, so these
stand in for them at the same sizes, sampling ratios and noise level):

* image: zeros, then K shapes painted in order, each overwriting its pixels.
  A shape is a rectangle or a disk with probability 1/2 each, with value
  v ~ U[0, 1].  Rectangle sides ~ U{ceil(n/16) .. ceil(n/2)}, placed fully
  inside; disk radius ~ U[n/16, n/4], centre in [r, n - r]^2, holding the
  pixels whose centres (r + 1/2, c + 1/2) lie inside.  Optionally a linear
  ramp a*c/(n-1) + b*r/(n-1), a, b ~ U[-1/4, 1/4].
* A: i.i.d. N(0, 1/m), generated in FP64 in blocks of 1024 rows, block b from
  PCG64(SeedSequence([seed_A, b])), then rounded to the requested dtype.
* f = A_64 u_bar + sigma * N(0, 1) with the FP64 A (rows regenerated per block).
* seeds: image i -> 1774 + i, noise of image i -> 10**6 + i.
"""
from __future__ import annotations

import math
import os
import threading
from dataclasses import dataclass, field

import numpy as np

ROW_BLOCK = 1024
IMAGE_SEED0 = 1774
NOISE_SEED0 = 10**6


def _threads() -> int:
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:  # pragma: no cover
        return max(1, min(16, os.cpu_count() or 1))


def image(n: int, seed: int, n_shapes: int | None = None, ramp: bool = False) -> np.ndarray:
    """Piecewise-constant n x n test image in FP64 (row-major, pixel r*n + c)."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    if n_shapes is None:
        n_shapes = int(rng.integers(10, 41))
    u = np.zeros((n, n), dtype=np.float64)
    lo, hi = math.ceil(n / 16), math.ceil(n / 2)
    rr, cc = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5, indexing="ij")
    for _ in range(n_shapes):
        is_rect = rng.random() < 0.5
        v = rng.random()
        if is_rect:
            h = int(rng.integers(lo, hi + 1))
            w = int(rng.integers(lo, hi + 1))
            r0 = int(rng.integers(0, n - h + 1))
            c0 = int(rng.integers(0, n - w + 1))
            u[r0:r0 + h, c0:c0 + w] = v
        else:
            rad = rng.uniform(n / 16, n / 4)
            cy = rng.uniform(rad, n - rad)
            cx = rng.uniform(rad, n - rad)
            u[(rr - cy) ** 2 + (cc - cx) ** 2 <= rad * rad] = v
    if ramp:
        a = rng.uniform(-0.25, 0.25)
        b = rng.uniform(-0.25, 0.25)
        u += a * (cc - 0.5) / (n - 1) + b * (rr - 0.5) / (n - 1)
    return u


def _block_rows(m: int, N: int, seed_A: int, blk: int) -> np.ndarray:
    r0 = blk * ROW_BLOCK
    rows = min(ROW_BLOCK, m - r0)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed_A, blk])))
    x = rng.standard_normal((rows, N))
    x *= 1.0 / math.sqrt(m)
    return x


def gaussian_matrix(m: int, N: int, seed_A: int, dtype=np.float64,
                    ubar: np.ndarray | None = None):
    """Dense A (m x N, row-major) with i.i.d. N(0, 1/m) entries, in `dtype`.

    If `ubar` (B x N, FP64) is given, also returns A_64 @ ubar.T (m x B), computed
    block by block from the FP64 rows before they are rounded to `dtype`.
    """
    A = np.empty((m, N), dtype=dtype)
    Au = None if ubar is None else np.empty((m, ubar.shape[0]), dtype=np.float64)
    nblk = (m + ROW_BLOCK - 1) // ROW_BLOCK
    nxt = [0]
    lock = threading.Lock()

    def worker():
        while True:
            with lock:
                b = nxt[0]
                nxt[0] += 1
            if b >= nblk:
                return
            x = _block_rows(m, N, seed_A, b)
            r0 = b * ROW_BLOCK
            A[r0:r0 + x.shape[0]] = x
            if Au is not None:
                Au[r0:r0 + x.shape[0]] = x @ ubar.T

    ths = [threading.Thread(target=worker) for _ in range(min(_threads(), nblk))]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    return A if ubar is None else (A, Au)


def noise(m: int, index: int, sigma: float) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(NOISE_SEED0 + index)))
    return sigma * rng.standard_normal(m)


@dataclass
class Problem:
    """One seeded reconstruction workload: B images sharing one A."""
    name: str
    n: int
    m: int
    A: np.ndarray              # m x n^2, dtype as requested
    ubar: np.ndarray           # B x n x n, FP64 ground truth
    f: np.ndarray              # B x m, FP64 observations (from the FP64 A)
    sigma: np.ndarray          # B noise levels
    mu: float = 1e3
    beta: float = 10.0
    seed_A: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.n * self.n

    @property
    def B(self) -> int:
        return self.ubar.shape[0]


def make_problem(name: str, n: int, ratio: float | None = None, m: int | None = None,
                 batch: int = 1, n_shapes: int | None = None, ramp: bool = False,
                 sigma=1e-3, seed_A: int = 1001, image_index0: int = 0,
                 dtype=np.float64, mu: float = 1e3, beta: float = 10.0) -> Problem:
    N = n * n
    if m is None:
        m = int(round(ratio * N))
    # a scalar, or one noise level per image (raises if the shapes disagree)
    sig = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (batch,)).copy()
    ubar = np.stack([image(n, IMAGE_SEED0 + image_index0 + i, n_shapes, ramp)
                     for i in range(batch)])
    A, Au = gaussian_matrix(m, N, seed_A, dtype=dtype, ubar=ubar.reshape(batch, N))
    f = Au.T.copy()
    for i in range(batch):
        f[i] += noise(m, image_index0 + i, sig[i])
    return Problem(name=name, n=n, m=m, A=A, ubar=ubar, f=f, sigma=sig, mu=mu, beta=beta,
                   seed_A=seed_A, meta=dict(image_index0=image_index0, n_shapes=n_shapes,
                                            ramp=ramp))


@dataclass
class DctProblem:
    """Seeded inputs for the partial-DCT operator: `rows` are the m selected flat
    indices k_r * n + k_c of the orthonormal 2-D DCT-II of n x n images."""
    name: str
    n: int
    m: int
    rows: np.ndarray
    ubar: np.ndarray
    f: np.ndarray
    sigma: np.ndarray
    mu: float
    beta: float
    tau: float
    seed_sel: int

    @property
    def N(self) -> int:
        return self.n * self.n

    @property
    def B(self) -> int:
        return self.f.shape[0]


def make_dct_problem(name: str, n: int, ratio: float, batch: int = 1, seed_sel: int = 1006,
                     n_shapes: int | None = None, sigma=1e-3, image_index0: int = 0,
                     mu: float = 500.0, beta: float = 2.0 ** 6, tau: float = 1.9) -> DctProblem:
    """m = round(ratio n^2) DCT coefficients: the DC term and m - 1 others chosen
    uniformly at random without replacement (seed `seed_sel`), f = (DCT2 ubar)[rows]
    + sigma N(0, 1).  Defaults follow the partial-DCT experiments: mu = 500,
    beta = 2^6, tau = 1.9."""
    import scipy.fft
    N = n * n
    m = int(round(ratio * N))
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed_sel, 0xDC7])))
    # the DC coefficient is always kept: TV and the other DCT rows both vanish on
    # constant images, so without it the image mean could not be recovered
    rest = 1 + rng.choice(N - 1, size=m - 1, replace=False)
    rows = np.sort(np.concatenate([[0], rest])).astype(np.int64)
    sig = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (batch,)).copy()
    ubar = np.stack([image(n, IMAGE_SEED0 + image_index0 + i, n_shapes)
                     for i in range(batch)])
    X = scipy.fft.dctn(ubar, type=2, norm="ortho", axes=(1, 2)).reshape(batch, N)
    f = X[:, rows].copy()
    for i in range(batch):
        f[i] += noise(m, image_index0 + i, sig[i])
    return DctProblem(name=name, n=n, m=m, rows=rows, ubar=ubar, f=f, sigma=sig, mu=mu,
                      beta=beta, tau=tau, seed_sel=seed_sel)


# Named workloads (sizes of the paper's dense-A experiment range, Sec. 3.1).
WORKLOADS = {
    # n = 32, m = 307 (30 %), 6 shapes: the small case the oracle runs in seconds.
    "n32_m307": dict(n=32, m=307, n_shapes=6, seed_A=1001),
    # n = 128, m = 4096 (25 %), 20 shapes plus a ramp: single image, FP32 A of 256 MiB.
    "n128_m4096": dict(n=128, m=4096, n_shapes=20, ramp=True, seed_A=1002),
    # n = 256, m = 13107 (20 %), 10-40 shapes, 64 images sharing A.
    "n256_m13107_b64": dict(n=256, m=13107, batch=64, seed_A=1003),
    # n = 512, m = 26214 (10 %), 128 images sharing A.
    "n512_m26214_b128": dict(n=512, m=26214, batch=128, seed_A=1005),
}


def workload(name: str, **over) -> Problem:
    kw = dict(WORKLOADS[name])
    kw.update(over)
    return make_problem(name, **kw)
