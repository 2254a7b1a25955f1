"""Pins of the oracle's start point and of its de-quantised storage formats (CPU only).

* initial_u: Alg. 1 and Alg. 2 start from "u^0 = f", which has the right length
  only when m = n^2.  The reading u^0 = A^T f must reduce to the printed start for
  A = I, and it is the negative gradient of the data term 1/2 ||A u - f||^2 at
  u = 0 (one unit gradient step from zero), which finite differences of that
  objective give without using A^T.  The zero start and the warm start return
  what the caller passes.
* dequantized_A("bf16"): elementwise the bfloat16 rounding that torch's cast
  performs; ("bf16_split"): hi is that rounding, lo is a bfloat16 value, and
  hi + lo is within 2^-16 (relative) of the FP32 entry (a bfloat16 value has 8
  significant bits, so rounding to it errs by at most half a unit in the 8th bit,
  2^-8 of the value: the remainder x - hi is at most 2^-8 |x|, and rounding it errs
  by at most 2^-8 of it); entries that bfloat16 holds exactly give lo = 0.
"""
import numpy as np
import pytest

import oracle as O


def test_initial_u_is_the_printed_start_for_identity(rng):
    n = 6
    f = rng.standard_normal((2, n * n))
    u0 = O.initial_u(np.eye(n * n), f, n, None)
    assert u0.shape == (2, n, n)
    assert np.array_equal(u0.reshape(2, n * n), f)


def test_initial_u_is_minus_gradient_of_data_term_at_zero(rng):
    n, m = 4, 11
    A = rng.standard_normal((m, n * n))
    f = rng.standard_normal((1, m))

    def h(x):
        r = A @ x - f[0]
        return 0.5 * r @ r
    eps = 1e-5
    fd = np.array([(h(eps * e) - h(-eps * e)) / (2 * eps) for e in np.eye(n * n)])
    u0 = O.initial_u(A, f, n, None).ravel()
    # h is quadratic: central differences are exact up to rounding
    assert np.allclose(u0, -fd, rtol=1e-8, atol=1e-9)


def test_initial_u_zero_and_warm_start(rng):
    n, m = 5, 9
    A = rng.standard_normal((m, n * n))
    f = rng.standard_normal((3, m))
    z = O.initial_u(A, f, n, np.zeros((n, n)))
    assert z.shape == (3, n, n) and not z.any()
    w = rng.standard_normal((3, n, n))
    got = O.initial_u(A, f, n, w)
    assert np.array_equal(got, w) and got is not w
    got[0, 0, 0] += 1.0                      # a copy: the caller's start is not changed
    assert got[0, 0, 0] != w[0, 0, 0]


def test_algorithms_start_from_initial_u(rng):
    """Zero iterations of either algorithm return the start point: A^T f, 0 or u0."""
    n, m = 4, 7
    A = rng.standard_normal((m, n * n))
    f = rng.standard_normal((1, m))
    for alg in (O.ftvcs, O.iadm):
        r = alg(A, f, n, 10.0, 5.0, 0.1, tol=0, maxit=0)
        assert np.array_equal(r.u.reshape(1, -1), f @ A)
        r0 = alg(A, f, n, 10.0, 5.0, 0.1, tol=0, maxit=0, u0=np.zeros((n, n)))
        assert not r0.u.any()


def test_dequantized_bf16_matches_torch(rng):
    torch = pytest.importorskip("torch")
    A = (rng.standard_normal((40, 64)) / np.sqrt(40)).astype(np.float32)
    A[0, :4] = [1.0, -0.5, 2.0 ** -20, 0.0]          # exact in bf16
    ref = torch.from_numpy(A).to(torch.bfloat16).to(torch.float64).numpy()
    got = O.dequantized_A(A, "bf16")
    assert got.dtype == np.float64 and np.array_equal(got, ref)
    # from FP64 input: rounded to FP32 first, then to bf16
    A64 = rng.standard_normal((8, 16))
    ref64 = torch.from_numpy(A64.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(O.dequantized_A(A64, "bf16"), ref64)


def test_dequantized_split_properties(rng):
    torch = pytest.importorskip("torch")
    A = (rng.standard_normal((60, 128)) / np.sqrt(60)).astype(np.float32)
    A[0, :3] = [1.0, -0.75, 2.0 ** -30]                # exact in bf16: lo must be 0
    got = O.dequantized_A(A, "bf16_split")
    hi = torch.from_numpy(A).to(torch.bfloat16).to(torch.float64).numpy()
    lo = got - hi
    # lo is a bfloat16 value
    lo32 = lo.astype(np.float32)
    assert np.array_equal(lo32.astype(np.float64), lo)
    assert not np.any(lo32.view(np.uint32) & 0xFFFF)
    err = np.abs(A.astype(np.float64) - got)
    assert np.all(err <= 2.0 ** -16 * np.abs(A.astype(np.float64)))
    assert np.array_equal(lo[0, :3], [0.0, 0.0, 0.0])
    # lo is the remainder x - hi rounded to 8 significant bits: the split errs by at
    # most 2^-8 of what bf16 alone leaves (the point of storing lo)
    assert np.all(err <= 2.0 ** -8 * np.abs(A.astype(np.float64) - hi))


def test_dequantized_fp32_is_the_fp32_rounding(rng):
    A = rng.standard_normal((7, 9))
    got = O.dequantized_A(A, "fp32")
    assert np.array_equal(got, A.astype(np.float32).astype(np.float64))
    with pytest.raises(ValueError):
        O.dequantized_A(A, "int4")
