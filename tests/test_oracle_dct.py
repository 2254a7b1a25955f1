"""Pins of the oracle's partial-DCT operator (Sec. 3.2: m rows of the 2-D DCT matrix
chosen at random, applied as fast transforms) and of the algorithms run on it (CPU)."""
import numpy as np
import pytest

import oracle as O
from paper_1001_1774_amd import synth


def dct_matrix_1d(n):
    """Orthonormal DCT-II written out from its cosine formula:
    C[k, j] = w_k cos(pi (2 j + 1) k / (2 n)), w_0 = sqrt(1/n), w_k = sqrt(2/n)."""
    C = np.empty((n, n))
    for k in range(n):
        w = np.sqrt(1.0 / n) if k == 0 else np.sqrt(2.0 / n)
        for j in range(n):
            C[k, j] = w * np.cos(np.pi * (2 * j + 1) * k / (2 * n))
    return C


def dense_partial_dct(n, rows):
    C1 = dct_matrix_1d(n)
    # coefficient (kr, kc) of pixel (r, c): C1[kr, r] C1[kc, c], row-major on both sides
    return np.kron(C1, C1)[rows]


@pytest.mark.parametrize("n", [4, 6, 8, 10])
def test_operator_equals_the_written_out_matrix(n):
    rng = np.random.default_rng(n)
    rows = np.sort(rng.choice(n * n, size=(n * n) // 3, replace=False))
    op = O.PartialDCT(n, rows)
    A = dense_partial_dct(n, rows)
    U = rng.standard_normal((3, n * n))
    R = rng.standard_normal((3, len(rows)))
    assert np.abs(op.fwd(U) - U @ A.T).max() <= 1e-13
    assert np.abs(op.adj(R) - R @ A).max() <= 1e-13


def test_rows_are_orthonormal():
    rng = np.random.default_rng(3)
    n = 16
    rows = rng.choice(n * n, size=77, replace=False)
    op = O.PartialDCT(n, rows)
    R = rng.standard_normal((2, 77))
    assert np.abs(op.fwd(op.adj(R)) - R).max() <= 1e-13       # A A^T = I
    assert abs(O.lambda_max(op) - 1.0) <= 1e-10


@pytest.mark.parametrize("alg", ["ftvcs", "iadm"])
def test_algorithms_on_the_operator_equal_the_dense_matrix(alg):
    p = synth.make_dct_problem("d8", n=8, ratio=0.4, batch=2, seed_sel=5)
    A = dense_partial_dct(8, p.rows)
    op = O.PartialDCT(8, p.rows)
    run = getattr(O, alg)
    a = run(op, p.f, p.n, 50.0, 2.0 ** 6, 1.9, tol=0, maxit=60)
    b = run(A, p.f, p.n, 50.0, 2.0 ** 6, 1.9, tol=0, maxit=60)
    assert np.abs(a.u - b.u).max() <= 1e-11


def test_dct_problem_measurements():
    """f = A ubar + noise with A the partial DCT; the selected rows are distinct."""
    p = synth.make_dct_problem("d16", n=16, ratio=0.3, batch=2, seed_sel=9, sigma=0.0)
    assert len(np.unique(p.rows)) == p.m == round(0.3 * 256)
    assert p.rows[0] == 0                      # the DC coefficient is always measured
    A = dense_partial_dct(16, p.rows)
    assert np.abs(p.f - p.ubar.reshape(2, -1) @ A.T).max() <= 1e-12
