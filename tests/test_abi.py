"""The C ABI: the library loads and exports every declared symbol; the header is
plain C; argument errors are reported before any device work (CPU only)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tvcs.h")
LIB = os.path.join(ROOT, "paper_1001_1774_amd", "libtvcs.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tvcs_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for want in ("tvcs_create", "tvcs_create_ex", "tvcs_solve", "tvcs_solve_batch",
                 "tvcs_destroy", "tvcs_last_error", "tvcs_set_tau"):
        assert want in names


def test_header_is_plain_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "tvcs.h"\nint main(void){ tvcs_stats s; (void)s; '
                   'return TVCS_OK + (int)sizeof(tvcs_handle); }\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only",
                    f"-I{os.path.dirname(HEADER)}", str(src)], check=True)


@pytest.fixture(scope="module")
def clib():
    if not os.path.exists(LIB):
        pytest.fail("libtvcs.so not built (python -m paper_1001_1774_amd.build)")
    import torch  # noqa: F401  same HIP runtime as the binding
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(clib):
    for name in declared_functions():
        assert hasattr(clib, name), name


def test_argument_errors_without_device(clib):
    from paper_1001_1774_amd import tvcs as T
    A = np.zeros((4, 64), np.float32)
    # NULL A, bad m, unsupported n: rejected before any HIP call
    assert not T.tvcs_create(None, 4, 8)
    assert "NULL" in T.tvcs_last_error()
    assert not T.tvcs_create(A, 0, 8)
    assert "m must be" in T.tvcs_last_error()
    for n in (7, 4, 1024, 98, 450 * 2, 15, 6):
        assert not T.tvcs_create(np.zeros((4, n * n), np.float32), 4, n)
        assert "prime factor" in T.tvcs_last_error()
    assert not T.tvcs_create_ex(A, 0, 4, 8, 9, None)
    assert "storage" in T.tvcs_last_error()
    assert not T.tvcs_create_ex(A, 0, 4, 8, T.TVCS_A_BF16, None)
    assert "n >= 16" in T.tvcs_last_error()
    # NULL handle
    u = np.zeros(64, np.float32)
    f = np.zeros(4, np.float32)
    assert T.tvcs_solve(None, f, 1.0, 1.0, 0.0, 1, 0, u) == T.TVCS_EINVAL
    assert T.tvcs_set_tau(None, 1.0) == T.TVCS_EINVAL
    # continuation: betas and flags are checked before any device work
    betas = np.array([16.0, 32.0])
    U = np.zeros((1, 64), np.float32)
    assert T.tvcs_solve_continuation(None, f, 1, 1.0, None, 2, 0.0, 1, 0, U) == T.TVCS_EINVAL
    assert "betas" in T.tvcs_last_error()
    assert T.tvcs_solve_continuation(None, f, 1, 1.0, betas, 0, 0.0, 1, 0, U) == T.TVCS_EINVAL
    assert T.tvcs_solve_continuation(None, f, 1, 1.0, np.array([16.0, -1.0]), 2, 0.0, 1, 0,
                                     U) == T.TVCS_EINVAL
    assert "positive" in T.tvcs_last_error()
    assert T.tvcs_solve_continuation(None, f, 1, 1.0, betas, 2, 0.0, 1, T.TVCS_IADM,
                                     U) == T.TVCS_EINVAL
    assert "FTVCS" in T.tvcs_last_error()
    assert T.tvcs_solve_continuation(None, f, 1, 1.0, betas, 2, 0.0, 1, 0, U) == T.TVCS_EINVAL
    assert "null handle" in T.tvcs_last_error()
    assert T.tvcs_measure_peaks(1024, 1) == T.TVCS_EINVAL
    assert T.tvcs_measure_peaks(1 << 30, 0) == T.TVCS_EINVAL
    # partial DCT: the coefficient list is checked on the host first
    assert not T.tvcs_create_ex(A, 0, 4, 8, T.TVCS_A_PARTIAL_DCT, None)
    assert "tvcs_create_dct" in T.tvcs_last_error()
    assert not T.lib().tvcs_create_dct(None, 4, 8, None)
    assert "rows" in T.tvcs_last_error()
    rows = np.array([0, 5, 63], np.int32)
    assert not T.tvcs_create_dct(rows, 3, 14)
    assert "prime factor" in T.tvcs_last_error()
    assert not T.tvcs_create_dct(rows, 0, 8)
    assert "m must be" in T.tvcs_last_error()
    assert not T.tvcs_create_dct(np.zeros(65, np.int32), 65, 8)
    assert "m must be" in T.tvcs_last_error()
    assert not T.tvcs_create_dct(np.array([0, 64], np.int32), 2, 8)
    assert "outside" in T.tvcs_last_error()
    assert not T.tvcs_create_dct(np.array([3, -1], np.int32), 2, 8)
    assert "outside" in T.tvcs_last_error()
    assert not T.tvcs_create_dct(np.array([7, 9, 7], np.int32), 3, 8)
    assert "repeated" in T.tvcs_last_error()
    with pytest.raises(TypeError):
        T.tvcs_create_dct(np.array([1, 2], np.int64), 2, 8)
    assert T.tvcs_get_tau(None) < 0
    T.tvcs_destroy(None)


def test_stats_struct_layout(tmp_path):
    """The binding's tvcs_stats has the C struct's size and field offsets."""
    from paper_1001_1774_amd import tvcs as T
    fields = [f[0] for f in T.tvcs_stats._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "tvcs.h"\n'
                   'int main(void){ printf("%zu", sizeof(tvcs_stats));'
                   + "".join(f' printf(" %zu", offsetof(tvcs_stats, {f}));' for f in fields)
                   + " return 0; }\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", f"-I{os.path.dirname(HEADER)}", str(src), "-o", str(exe)],
                   check=True)
    c = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True,
                                         text=True).stdout.split()]
    py = [ctypes.sizeof(T.tvcs_stats)] + [getattr(T.tvcs_stats, f).offset for f in fields]
    assert py == c
