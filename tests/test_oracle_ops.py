"""Pins of the oracle's building blocks (CPU only)."""
import os

import numpy as np
import pytest
import scipy.linalg

import oracle as O
from tests._pins import dense_D, shrink_bruteforce

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#", ndmin=2)


# --- finite differences (Sec. 2 notation, periodic BC) ----------------------------
@pytest.mark.parametrize("n", [3, 4, 5, 8])
def test_D_matches_dense_matrix(n, rng):
    D1, D2 = dense_D(n)
    u = rng.standard_normal((n, n))
    d = O.D(u)
    assert np.allclose(d[0].ravel(), D1 @ u.ravel(), atol=1e-14)
    assert np.allclose(d[1].ravel(), D2 @ u.ravel(), atol=1e-14)
    w = rng.standard_normal((2, n, n))
    assert np.allclose(O.Dt(w).ravel(), D1.T @ w[0].ravel() + D2.T @ w[1].ravel(), atol=1e-13)


def test_D_adjoint_and_constants(rng):
    n = 16
    u = rng.standard_normal((3, n, n))
    w = rng.standard_normal((3, 2, n, n))
    lhs = np.sum(O.D(u) * w, axis=(1, 2, 3))
    rhs = np.sum(u * O.Dt(w), axis=(1, 2))
    assert np.allclose(lhs, rhs, rtol=1e-12)
    assert np.abs(O.D(np.full((n, n), 3.7))).max() == 0.0
    # horizontal component is along columns: a column ramp has zero vertical difference
    ramp = np.tile(np.arange(n, dtype=float), (n, 1))
    d = O.D(ramp)
    assert np.abs(d[1]).max() == 0.0 and d[0][0, 0] == 1.0


# --- eigenvalues of D^T D and the FFT solve of (eqnorm) -----------------------------
def test_dtd_eigenvalues_golden_n4():
    assert np.allclose(O.dtd_eigenvalues(4), _golden("dtd_eig_n4.txt"), atol=1e-14)


@pytest.mark.parametrize("n", [4, 6, 8, 10, 12])
def test_dtd_eigenvalues_match_dense(n):
    D1, D2 = dense_D(n)
    ev = np.sort(np.linalg.eigvalsh(D1.T @ D1 + D2.T @ D2))
    assert np.allclose(np.sort(O.dtd_eigenvalues(n).ravel()), ev, atol=1e-11)


@pytest.mark.parametrize("n,c", [(4, 0.3), (8, 5.0), (16, 474.0), (16, 1e-3), (6, 2.0),
                                 (10, 0.7), (12, 40.0), (18, 3.0)])
def test_solve_u_matches_dense_cholesky(n, c, rng):
    D1, D2 = dense_D(n)
    H = D1.T @ D1 + D2.T @ D2 + c * np.eye(n * n)
    rhs = rng.standard_normal((2, n, n))
    cf = scipy.linalg.cho_factor(H)
    for b in range(2):
        ref = scipy.linalg.cho_solve(cf, rhs[b].ravel())
        got = O.solve_u(rhs[b], c).ravel()
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref) * max(1.0, 1.0 / c)


def test_solve_u_matches_library_real_fft(rng):
    """The real-input FFT pair gives the same solve (rfft2/irfft2 as the library routine)."""
    n, c = 32, 17.0
    rhs = rng.standard_normal((n, n))
    k = np.arange(n)
    lam = (2 - 2 * np.cos(2 * np.pi * k / n))
    d = lam[:, None] + lam[None, : n // 2 + 1] + c
    ref = np.fft.irfft2(np.fft.rfft2(rhs) / d, s=(n, n))
    assert np.allclose(O.solve_u(rhs, c), ref, rtol=1e-12, atol=1e-14)


# --- shrinkage (eq. (shrink), (sop), (fixu)) --------------------------------------
def test_shrink_golden():
    for beta, z1, z2, w1, w2 in _golden("shrink_cases.txt"):
        z = np.array([z1, z2]).reshape(2, 1, 1)
        w = O.shrink(z, beta).ravel()
        assert np.allclose(w, [w1, w2], atol=1e-15), (beta, z1, z2, w)


def test_shrink_equals_identity_minus_projection(rng):
    beta = 3.0
    z = rng.standard_normal((2, 32, 32)) * 0.5
    z[:, 0, 0] = 0.0
    z[:, 0, 1] = [1.0 / beta, 0.0]       # exactly on the circle
    assert np.allclose(O.shrink(z, beta), z - O.project_disc(z, beta), atol=1e-15)


def test_shrink_is_the_minimiser_of_fixu(rng):
    for beta in (0.7, 4.0, 10.0):
        for _ in range(12):
            z = rng.standard_normal(2) * rng.choice([0.05, 0.3, 2.0])
            w = O.shrink(z.reshape(2, 1, 1), beta).ravel()
            wb, fb, obj = shrink_bruteforce(z, beta)
            assert obj(w) <= fb + 1e-12
            assert np.allclose(w, wb, atol=1e-5)
            # optimality: 0 in d||w|| + beta (w - z)
            if np.hypot(*w) > 0:
                assert np.allclose(w / np.hypot(*w) + beta * (w - z), 0, atol=1e-12)
            else:
                assert beta * np.hypot(*z) <= 1 + 1e-12


# --- gradient and step-size ------------------------------------------------------
def test_gradient_by_finite_differences(rng):
    n, m = 4, 7
    A = rng.standard_normal((m, n * n))
    f = rng.standard_normal((1, m))
    u = rng.standard_normal((1, n, n))
    g = O.gradient(A, u, f).ravel()

    def h(x):
        r = A @ x - f[0]
        return 0.5 * r @ r
    x = u.ravel()
    fd = np.array([(h(x + 1e-6 * e) - h(x - 1e-6 * e)) / 2e-6 for e in np.eye(n * n)])
    assert np.allclose(g, fd, rtol=1e-7, atol=1e-7)


def test_lambda_max_against_svd(rng):
    for m, N in [(20, 64), (77, 256), (307, 1024)]:
        A = rng.standard_normal((m, N)) / np.sqrt(m)
        ref = np.linalg.svd(A, compute_uv=False)[0] ** 2
        lam = O.lambda_max(A, iters=2000, rtol=1e-13)
        assert abs(lam - ref) <= 1e-6 * ref
        assert O.default_tau(A) * ref < 2.0


# --- storage formats ---------------------------------------------------------------
def test_bf16_rne_matches_torch(rng):
    torch = pytest.importorskip("torch")
    x = np.concatenate([rng.standard_normal(20000).astype(np.float32),
                        np.float32([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 0.0, 3e-39])])
    ref = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    assert np.array_equal(O.bf16_rne(x), ref)


def test_split_bf16_properties(rng):
    x = rng.standard_normal(50000).astype(np.float32)
    hi, lo = O.split_bf16(x)
    assert np.array_equal(O.bf16_rne(hi), hi) and np.array_equal(O.bf16_rne(lo), lo)
    err = np.abs(x.astype(np.float64) - hi - lo)
    assert np.all(err <= 2.0 ** -16 * np.abs(x))


def test_fp8_e4m3_table_and_torch(rng):
    torch = pytest.importorskip("torch")
    v = O.fp8_e4m3_values()
    assert v[-1] == 448.0 and v[1] == 2.0 ** -9 and v[8] == 2.0 ** -6 and len(v) == 127
    assert np.all(np.diff(v) > 0)
    x = np.concatenate([rng.standard_normal(20000) * 40, rng.uniform(-448, 448, 5000),
                        [300.0, 17.0, 0.5 * 2 ** -9, 1.5 * 2 ** -9, 448.0, -448.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).float().numpy()
    got, _ = O.fp8_e4m3_rne(x)
    assert np.array_equal(got.astype(np.float32), ref)
    sat, _ = O.fp8_e4m3_rne(np.array([500.0, -1e6]))
    assert np.array_equal(sat, [448.0, -448.0])


def test_fp8_rowscale(rng):
    A = (rng.standard_normal((50, 300)) / np.sqrt(50)).astype(np.float32)
    q, s = O.fp8_rowscale_quantize(A)
    assert np.allclose(np.abs(q).max(axis=1), 448.0)
    deq = q * s[:, None]
    rel = np.abs(deq - A) / np.abs(A).max(axis=1, keepdims=True)
    assert rel.max() <= 2.0 ** -4 * 1.0001      # half an ulp at the top binade / 448
    assert np.allclose(O.dequantized_A(A, "fp8_rowscale"), deq)
