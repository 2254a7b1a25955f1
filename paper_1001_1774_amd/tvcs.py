"""Thin ctypes binding of the C ABI in include/tvcs.h (argument marshalling only).

Every function here has the name and arguments of its C counterpart; arrays may
be torch tensors (device or host) or numpy arrays, and are passed by pointer.
All arithmetic of the reconstruction runs in the HIP kernels of libtvcs.so; if
the library is not built, loading it raises instead of falling back to anything.

torch is imported before the library is loaded so that both use the same HIP
runtime, and device tensors allocated by torch can be handed to the library.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

# the in-tree build; TVCS_LIBRARY may name another build of the same sources
LIB_PATH = os.environ.get("TVCS_LIBRARY") or os.path.join(
    os.path.dirname(os.path.abspath(__file__)), "libtvcs.so")

TVCS_OK = 0
TVCS_MAXIT = 1
TVCS_EINVAL = -1
TVCS_ENOMEM = -2
TVCS_EDEVICE = -3
TVCS_ENONFINITE = -4
TVCS_EUNSUPPORTED = -5

TVCS_IADM = 0x1
TVCS_U0_ZERO = 0x2
TVCS_OBJECTIVE = 0x4
TVCS_WARM_START = 0x8
TVCS_BB_SHIFT = 8


def TVCS_BB_STEPS(j):
    """Solve flag: IADM with j inner BB / line-search steps on its u-subproblem."""
    return (int(j) & 0xF) << TVCS_BB_SHIFT

TVCS_A_FP32 = 0
TVCS_A_BF16 = 1
TVCS_A_BF16_SPLIT = 2
TVCS_A_FP8_ROWSCALE = 3
TVCS_A_PARTIAL_DCT = 4

STORAGE = {"fp32": TVCS_A_FP32, "bf16": TVCS_A_BF16, "bf16_split": TVCS_A_BF16_SPLIT,
           "fp8_rowscale": TVCS_A_FP8_ROWSCALE}


class tvcs_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("status", ctypes.c_int),
                ("rel_change", ctypes.c_double), ("objective", ctypes.c_double),
                ("tau", ctypes.c_double), ("ms", ctypes.c_float),
                ("fresh_iters", ctypes.c_int), ("tiles", ctypes.c_int * 6)]


class TvcsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tvcs error {code}: {msg}")
        self.code = code


_lib = None
_lock = threading.Lock()

_SIGS = {
    "tvcs_create": (ctypes.c_void_p, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    "tvcs_create_ex": (ctypes.c_void_p, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
    "tvcs_create_dct": (ctypes.c_void_p, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_void_p]),
    "tvcs_set_stream": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "tvcs_set_tau": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_double]),
    "tvcs_get_tau": (ctypes.c_double, [ctypes.c_void_p]),
    "tvcs_lambda_max": (ctypes.c_double, [ctypes.c_void_p]),
    "tvcs_device_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "tvcs_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_uint,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "tvcs_solve_batch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_uint, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "tvcs_solve_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                          ctypes.c_uint, ctypes.c_void_p, ctypes.c_void_p]),
    "tvcs_solve_continuation": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                               ctypes.c_double, ctypes.c_void_p, ctypes.c_int,
                                               ctypes.c_double, ctypes.c_int, ctypes.c_uint,
                                               ctypes.c_void_p, ctypes.c_void_p]),
    "tvcs_measure_peaks": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_void_p]),
    "tvcs_time_products": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
    "tvcs_time_fused": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "tvcs_set_tiles": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "tvcs_get_tiles": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "tvcs_destroy": (None, [ctypes.c_void_p]),
    "tvcs_server_create": (ctypes.c_void_p, [ctypes.c_size_t, ctypes.c_int, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_uint]),
    "tvcs_server_add_matrix": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "tvcs_server_submit": (ctypes.c_longlong, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                               ctypes.c_double, ctypes.c_int]),
    "tvcs_server_step": (ctypes.c_int, [ctypes.c_void_p]),
    "tvcs_server_result": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_void_p,
                                          ctypes.c_void_p]),
    "tvcs_server_pending": (ctypes.c_int, [ctypes.c_void_p]),
    "tvcs_server_device_bytes": (ctypes.c_size_t, [ctypes.c_void_p]),
    "tvcs_server_a_bytes": (ctypes.c_double, [ctypes.c_void_p]),
    "tvcs_server_destroy": (None, [ctypes.c_void_p]),
    "tvcs_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load libtvcs.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is not built: run `python -m "
                                   "paper_1001_1774_amd.build` (hipcc, gfx950)")
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGS.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def _ptr(x, dtype=None):
    """Pointer to the data of a contiguous torch tensor or numpy array (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        if dtype is not None and x.dtype != dtype:
            raise TypeError(f"expected {dtype}, got {x.dtype}")
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return ctypes.c_void_p(x.data_ptr())
    if isinstance(x, np.ndarray):
        if dtype is not None:
            want = {torch.float32: np.float32, torch.float64: np.float64}[dtype]
            if x.dtype != want:
                raise TypeError(f"expected {want}, got {x.dtype}")
        if not x.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return ctypes.c_void_p(x.ctypes.data)
    if isinstance(x, (int, ctypes.c_void_p)):
        return x
    raise TypeError(f"unsupported buffer type {type(x)}")


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


# --- the C entry points, same names --------------------------------------------------
def tvcs_create(A, m, n):
    return lib().tvcs_create(_ptr(A, torch.float32), m, n)


def tvcs_create_ex(A, a_is_fp64, m, n, storage, stream=None):
    dt = torch.float64 if a_is_fp64 else torch.float32
    return lib().tvcs_create_ex(_ptr(A, dt), int(a_is_fp64), m, n, int(storage), _stream(stream))


def tvcs_create_dct(rows, m, n, stream=None):
    """rows: C-contiguous int32 numpy array of m flat coefficient indices."""
    if not (isinstance(rows, np.ndarray) and rows.dtype == np.int32 and rows.flags["C_CONTIGUOUS"]):
        raise TypeError("rows must be a C-contiguous int32 numpy array")
    return lib().tvcs_create_dct(ctypes.c_void_p(rows.ctypes.data), int(m), int(n),
                                 _stream(stream))


def tvcs_set_stream(h, stream):
    return lib().tvcs_set_stream(h, _stream(stream))


def tvcs_set_tau(h, tau):
    return lib().tvcs_set_tau(h, float(tau))


def tvcs_get_tau(h):
    return lib().tvcs_get_tau(h)


def tvcs_lambda_max(h):
    return lib().tvcs_lambda_max(h)


def tvcs_device_bytes(h):
    return lib().tvcs_device_bytes(h)


def tvcs_solve(h, f, mu, beta, tol, maxit, flags, u, lam=None, st=None):
    return lib().tvcs_solve(h, _ptr(f, torch.float32), mu, beta, tol, maxit, flags,
                            _ptr(u, torch.float32), _ptr(lam, torch.float64),
                            ctypes.byref(st) if st is not None else None)


def tvcs_solve_noalloc(h, f, mu, beta, tol, maxit, flags, u, st=None):
    return lib().tvcs_solve_noalloc(h, _ptr(f, torch.float32), mu, beta, tol, maxit, flags,
                                    _ptr(u, torch.float32),
                                    ctypes.byref(st) if st is not None else None)


def tvcs_solve_batch(h, F, B, mu, beta, tol, maxit, flags, U, lam=None, st=None):
    return lib().tvcs_solve_batch(h, _ptr(F, torch.float32), B, mu, beta, tol, maxit, flags,
                                  _ptr(U, torch.float32), _ptr(lam, torch.float64),
                                  st if st is not None else None)


def tvcs_solve_continuation(h, F, B, mu, betas, nbeta, tol, maxit, flags, U, st=None):
    """betas: a float64 numpy array (host) of nbeta values."""
    return lib().tvcs_solve_continuation(h, _ptr(F, torch.float32), B, mu,
                                         _ptr(betas, torch.float64), nbeta, tol, maxit, flags,
                                         _ptr(U, torch.float32), st if st is not None else None)


def tvcs_time_products(h, B, reps, form=0, ms_forward=None, ms_adjoint=None):
    """form 0: fresh products, 1: their increment form (MFMA storage);
    ms_forward / ms_adjoint: ctypes.c_float objects (or None)."""
    return lib().tvcs_time_products(h, B, reps, form,
                                    ctypes.byref(ms_forward) if ms_forward is not None else None,
                                    ctypes.byref(ms_adjoint) if ms_adjoint is not None else None)


def tvcs_time_fused(h, reps, ms_pass=None, ms_sum=None):
    """ms_pass / ms_sum: ctypes.c_float objects (or None)."""
    return lib().tvcs_time_fused(h, reps,
                                 ctypes.byref(ms_pass) if ms_pass is not None else None,
                                 ctypes.byref(ms_sum) if ms_sum is not None else None)


def tvcs_set_tiles(h, tiles=None):
    """tiles: six ints {rt, images, kf} of the forward then the adjoint product, or
    None (autotune)."""
    arr = (ctypes.c_int * 6)(*tiles) if tiles is not None else None
    return lib().tvcs_set_tiles(h, arr)


def tvcs_get_tiles(h, tiles):
    """tiles: a (ctypes.c_int * 6) array filled with the shapes in use."""
    return lib().tvcs_get_tiles(h, tiles)


def tvcs_measure_peaks(nbytes, reps, read_gbs=None, mfma_tflops=None):
    """read_gbs / mfma_tflops: ctypes.c_double objects (or None)."""
    return lib().tvcs_measure_peaks(nbytes, reps,
                                    ctypes.byref(read_gbs) if read_gbs is not None else None,
                                    ctypes.byref(mfma_tflops) if mfma_tflops is not None else None)


def measure_peaks(nbytes=2 << 30, reps=10):
    """(HBM read GB/s, bf16 MFMA TFLOP/s) measured on the current device."""
    a, b = ctypes.c_double(), ctypes.c_double()
    rc = tvcs_measure_peaks(nbytes, reps, a, b)
    if rc < 0:
        raise TvcsError(rc, tvcs_last_error())
    return a.value, b.value


def tvcs_destroy(h):
    lib().tvcs_destroy(h)


def tvcs_last_error():
    return lib().tvcs_last_error().decode()


def tvcs_server_create(hbm_budget, slots, mu, beta, flags):
    return lib().tvcs_server_create(int(hbm_budget), int(slots), float(mu), float(beta),
                                    int(flags))


def tvcs_server_add_matrix(s, h):
    return lib().tvcs_server_add_matrix(s, h)


def tvcs_server_submit(s, matrix, f, tol, maxit):
    return lib().tvcs_server_submit(s, int(matrix), _ptr(f, torch.float32), float(tol),
                                    int(maxit))


def tvcs_server_step(s):
    return lib().tvcs_server_step(s)


def tvcs_server_result(s, request, u=None, st=None):
    return lib().tvcs_server_result(s, int(request), _ptr(u, torch.float32),
                                    ctypes.byref(st) if st is not None else None)


def tvcs_server_pending(s):
    return lib().tvcs_server_pending(s)


def tvcs_server_device_bytes(s):
    return lib().tvcs_server_device_bytes(s)


def tvcs_server_a_bytes(s):
    return lib().tvcs_server_a_bytes(s)


def tvcs_server_destroy(s):
    lib().tvcs_server_destroy(s)


# --- a small convenience wrapper -------------------------------------------------------
class Solver:
    """Owns a handle: ``Solver(A, n, storage="fp32")``, then ``solve`` / ``solve_batch``.

    A is m x n^2 (numpy or torch, float32 or float64).  Results are torch tensors on
    ``device`` (default cuda:0).
    """

    def __init__(self, A, n, storage="fp32", device="cuda", stream=None):
        if isinstance(A, np.ndarray):
            A = np.ascontiguousarray(A)
            is64 = A.dtype == np.float64
            if not is64:
                A = A.astype(np.float32, copy=False)
        else:
            A = A.contiguous()
            is64 = A.dtype == torch.float64
            if not is64:
                A = A.float()
        self.m, self.n, self.N = int(A.shape[0]), int(n), int(n) * int(n)
        if A.shape[1] != self.N:
            raise ValueError(f"A has {A.shape[1]} columns, expected n^2 = {self.N}")
        self.device = torch.device(device)
        self.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
        self.h = tvcs_create_ex(A, is64, self.m, self.n, self.storage, stream)
        if not self.h:
            raise TvcsError(-1, tvcs_last_error())

    @classmethod
    def partial_dct(cls, rows, n, device="cuda", stream=None):
        """The partial-DCT operator: f[i] measures coefficient rows[i] = k_r * n + k_c
        of the orthonormal 2-D DCT-II of the n x n image (no matrix is stored)."""
        rows = np.ascontiguousarray(np.asarray(rows), dtype=np.int32)
        self = cls.__new__(cls)
        self.m, self.n, self.N = int(rows.shape[0]), int(n), int(n) * int(n)
        self.device = torch.device(device)
        self.storage = TVCS_A_PARTIAL_DCT
        self.h = tvcs_create_dct(rows, self.m, self.n, stream)
        if not self.h:
            raise TvcsError(-1, tvcs_last_error())
        return self

    def close(self):
        if getattr(self, "h", None):
            tvcs_destroy(self.h)
            self.h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def tau(self):
        return tvcs_get_tau(self.h)

    @tau.setter
    def tau(self, value):
        rc = tvcs_set_tau(self.h, value)
        if rc < 0:
            raise TvcsError(rc, tvcs_last_error())

    @property
    def lambda_max(self):
        return tvcs_lambda_max(self.h)

    def _as_dev(self, x, dtype):
        t = torch.as_tensor(x).to(self.device, dtype)
        return t.contiguous()

    def solve_batch(self, F, mu=1e3, beta=10.0, tol=0.0, maxit=500, iadm=False, objective=False,
                    u0=None, lam0=None, want_lambda=False, u0_zero=False, bb_steps=1):
        F = self._as_dev(F, torch.float32)
        if F.dim() == 1:
            F = F[None]
        B = F.shape[0]
        flags = (TVCS_IADM if iadm else 0) | (TVCS_OBJECTIVE if objective else 0) | \
            (TVCS_U0_ZERO if u0_zero else 0) | (TVCS_BB_STEPS(bb_steps) if bb_steps > 1 else 0)
        if u0 is not None:
            U = self._as_dev(u0, torch.float32).reshape(B, self.N).clone()
            flags |= TVCS_WARM_START
        else:
            U = torch.empty(B, self.N, dtype=torch.float32, device=self.device)
        lam = None
        if iadm and (want_lambda or lam0 is not None):
            lam = (self._as_dev(lam0, torch.float64).reshape(B, 2 * self.N).clone()
                   if lam0 is not None else
                   torch.zeros(B, 2 * self.N, dtype=torch.float64, device=self.device))
        st = (tvcs_stats * B)()
        rc = tvcs_solve_batch(self.h, F, B, mu, beta, tol, maxit, flags, U, lam, st)
        if rc < 0:
            raise TvcsError(rc, tvcs_last_error())
        stats = [dict(iters=s.iters, status=s.status, rel_change=s.rel_change,
                      objective=s.objective, tau=s.tau, ms=s.ms,
                      fresh_iters=s.fresh_iters, tiles=tuple(s.tiles)) for s in st]
        out = dict(u=U.reshape(B, self.n, self.n), stats=stats, rc=rc)
        if lam is not None:
            out["lam"] = lam.reshape(B, 2, self.n, self.n)
        return out

    def solve_continuation(self, F, mu=1e3, betas=(16.0, 32.0, 64.0, 128.0), tol=1e-3,
                           maxit=500, objective=False, u0=None, u0_zero=False):
        """FTVCS with continuation in beta (one warm-started stage per beta)."""
        F = self._as_dev(F, torch.float32)
        if F.dim() == 1:
            F = F[None]
        B = F.shape[0]
        flags = (TVCS_OBJECTIVE if objective else 0) | (TVCS_U0_ZERO if u0_zero else 0)
        if u0 is not None:
            U = self._as_dev(u0, torch.float32).reshape(B, self.N).clone()
            flags |= TVCS_WARM_START
        else:
            U = torch.empty(B, self.N, dtype=torch.float32, device=self.device)
        b = np.ascontiguousarray(np.asarray(betas, dtype=np.float64))
        st = (tvcs_stats * B)()
        rc = tvcs_solve_continuation(self.h, F, B, mu, b, len(b), tol, maxit, flags, U, st)
        if rc < 0:
            raise TvcsError(rc, tvcs_last_error())
        stats = [dict(iters=s.iters, status=s.status, rel_change=s.rel_change,
                      objective=s.objective, tau=s.tau, ms=s.ms,
                      fresh_iters=s.fresh_iters, tiles=tuple(s.tiles)) for s in st]
        return dict(u=U.reshape(B, self.n, self.n), stats=stats, rc=rc)

    @property
    def tiles(self):
        """The MFMA products' tile shapes: (rt, images, kf) of the forward product, then
        of the adjoint (zeros for FP32 storage and the partial DCT)."""
        t = (ctypes.c_int * 6)()
        rc = tvcs_get_tiles(self.h, t)
        if rc < 0:
            raise TvcsError(rc, tvcs_last_error())
        return tuple(t)

    @tiles.setter
    def tiles(self, value):
        rc = tvcs_set_tiles(self.h, None if value is None else [int(x) for x in value])
        if rc < 0:
            raise TvcsError(rc, tvcs_last_error())

    def time_products(self, B=1, reps=20, increment=False):
        """Average ms per launch of the forward and adjoint products (HIP events);
        increment=True times the one-part increment form of the MFMA products."""
        a, b = ctypes.c_float(), ctypes.c_float()
        rc = tvcs_time_products(self.h, B, reps, 1 if increment else 0, a, b)
        if rc < 0:
            raise TvcsError(rc, tvcs_last_error())
        return a.value, b.value

    def time_fused(self, reps=20):
        """Average ms per launch of the one-pass product of one image and of its
        band-partial sum (FP32 storage, n*n <= 16384; TvcsError otherwise)."""
        a, b = ctypes.c_float(), ctypes.c_float()
        rc = tvcs_time_fused(self.h, reps, a, b)
        if rc < 0:
            raise TvcsError(rc, tvcs_last_error())
        return a.value, b.value

    def solve(self, f, **kw):
        r = self.solve_batch(f, **kw)
        r["u"] = r["u"][0]
        r["stats"] = r["stats"][0]
        if "lam" in r:
            r["lam"] = r["lam"][0]
        return r
