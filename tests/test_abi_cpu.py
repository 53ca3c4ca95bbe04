"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/lobpcg.h declares, validates arguments, and its host FP64
dense kernels agree with LAPACK (scipy) and with the paper's scale-invariance
requirement for Cholesky (Section 2.2)."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.linalg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lobpcg.h")

L = pytest.importorskip("paper_0705_2626_amd")
from paper_0705_2626_amd.lobpcg import _Op, _Precond as PC  # noqa: E402


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lobpcg_[a-z_A-Z0-9]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings():
    for s in (0, 1, -1, -2, -3, -4, -5, -6, -7):
        assert L.status_string(s)
    assert L.status_string(99) == "unknown status"


def ws(dims, levels, m, prec, B=None):
    lib = L.lib()
    n = ctypes.c_size_t(0)
    A = L.Op(*dims).c()
    T = L.Precond(levels).c()
    s = lib.lobpcg_workspace_bytes(ctypes.byref(A), ctypes.byref(B) if B is not None else None, ctypes.byref(T),
                                   m, prec, ctypes.byref(n))
    return s, n.value


def test_workspace_bytes_scales_with_problem():
    s1, n1 = ws((64, 64, 64), 4, 8, L.FP64)
    s2, n2 = ws((64, 64, 64), 4, 8, L.MIXED)
    s3, n3 = ws((128, 64, 64), 4, 8, L.FP64)
    assert s1 == s2 == s3 == L.OK
    N, m = 64 ** 3, 8
    assert n1 >= 11 * N * m * 8 and n2 >= 11 * N * m * (8 + 4)
    assert n3 - n1 >= 11 * N * m * 8     # the N x m blocks double with N


@pytest.mark.parametrize("dims,levels,m,prec,want", [
    ((4, 4, 4), None, 0, 0, L.ERR_ARG),            # m < 1
    ((3, 3, 3), None, 10, 0, L.ERR_ARG),           # 3m > N
    ((16, 16, 16), None, 129, 0, L.ERR_ARG),       # beyond the supported block size
    ((16, 16, 16), 6, 4, 0, L.ERR_ARG),            # too many levels for the grid
    ((16, 16, 16), 2, 4, 7, L.ERR_ARG),            # bad precision
    ((0, 16, 16), None, 4, 0, L.ERR_ARG),          # empty grid
])
def test_workspace_bytes_rejects_bad_arguments(dims, levels, m, prec, want):
    s, _ = ws(dims, levels, m, prec)
    assert s == want


def test_B_must_be_a_positive_diagonal_or_a_dominant_mass7_of_the_grid():
    """B: a DIAG descriptor of A's grid, or MASS7 with b0 > 6 |b1| (then
    symmetric positive definite); the diagonal array is not read by the
    workspace query, so a placeholder address is enough here."""
    fake = 256
    diag = _Op(8, 8, 8, L.OP_DIAG, None, None, None, fake)
    s0, n0 = ws((8, 8, 8), None, 2, L.FP64)
    s, n = ws((8, 8, 8), None, 2, L.FP64, B=diag)
    assert s == s0 == L.OK
    assert n - n0 >= 5 * 512 * 2 * 8                 # B X (twice), B W, B P and a spare
    s0m, n0m = ws((8, 8, 8), None, 2, L.MIXED)
    sm, nm = ws((8, 8, 8), None, 2, L.MIXED, B=diag)
    assert s0m == sm == L.OK
    assert nm - n0m >= 5 * 512 * 2 * (8 + 4)         # the B-blocks in both precisions
    assert ws((8, 8, 8), None, 2, L.FP64, B=L.Op(8, 8, 8).c())[0] == L.ERR_ARG          # not a B kind
    assert ws((8, 8, 8), None, 2, L.FP64, B=_Op(8, 8, 4, L.OP_DIAG, None, None, None, fake))[0] == L.ERR_ARG
    assert ws((8, 8, 8), None, 2, L.FP64, B=_Op(8, 8, 8, L.OP_DIAG, None, None, None, None))[0] == L.ERR_ARG
    assert ws((8, 8, 8), None, 2, L.FP64, B=L.Mass7(8, 8, 8, 0.6, 1.0 / 12.0).c())[0] == L.OK
    assert ws((8, 8, 8), None, 2, L.MIXED, B=L.Mass7(8, 8, 8, 1.0, -0.1).c())[0] == L.OK
    for b0, b1 in ((0.5, 1.0 / 12.0), (0.6, -0.1), (0.0, 0.0), (float("nan"), 0.0)):   # not dominant
        assert ws((8, 8, 8), None, 2, L.FP64, B=L.Mass7(8, 8, 8, b0, b1).c())[0] == L.ERR_ARG
    assert ws((8, 8, 8), None, 2, L.FP64, B=L.Mass7(8, 8, 7, 0.5, 0.01).c())[0] == L.ERR_ARG


def test_setup_rejects_small_or_missing_workspace():
    lib = L.lib()
    A, T = L.Op(8, 8, 8).c(), L.Precond(2).c()
    h = ctypes.c_void_p()
    s = lib.lobpcg_setup(ctypes.byref(h), ctypes.byref(A), None, ctypes.byref(T), 2, 0, None, 0, None)
    assert s == L.ERR_WORKSPACE
    s = lib.lobpcg_setup(ctypes.byref(h), ctypes.byref(A), None, ctypes.byref(T), 2, 0, ctypes.c_void_p(256), 16,
                         None)
    assert s == L.ERR_WORKSPACE
    assert not h.value


def test_vcycle_parameters_validated():
    lib = L.lib()
    A = L.Op(16, 16, 16).c()
    n = ctypes.c_size_t(0)
    for T in (PC(1, 3, 2, 1, 20, 2 / 3), PC(1, 3, 2, 2, 0, 2 / 3), PC(1, 3, 2, 2, 20, 2.5),
              PC(5, 3, 2, 2, 20, 2 / 3)):
        assert lib.lobpcg_workspace_bytes(ctypes.byref(A), None, ctypes.byref(T), 4, 0, ctypes.byref(n)) == L.ERR_ARG


# ---------------------------------------------------------------- host dense kernels

def test_dense_chol_factor_and_scale_invariance():
    rng = np.random.default_rng(3)
    V = rng.standard_normal((60, 7))
    G = V.T @ V
    s, R = L.lobpcg_dense_chol(G)
    assert s == L.OK
    np.testing.assert_allclose(R.T @ R, G, rtol=1e-13, atol=1e-13)
    assert np.allclose(R, np.triu(R))
    d = np.array([1e-15, 1.0, 1e9, 3e-7, 7.0, 1e-30, 2e4])
    s2, R2 = L.lobpcg_dense_chol(G * np.outer(d, d))
    assert s2 == L.OK
    np.testing.assert_allclose(R2, R * d[None, :], rtol=1e-12, atol=0)


@pytest.mark.parametrize("G", [np.ones((3, 3)), np.diag([1.0, 0.0, 1.0]), np.array([[1.0, 2.0], [2.0, 1.0]]),
                               np.array([[1.0, np.nan], [np.nan, 1.0]])])
def test_dense_chol_rejects_non_pd(G):
    s, _ = L.lobpcg_dense_chol(G)
    assert s == L.ERR_CHOL


@pytest.mark.parametrize("n,m,seed", [(12, 4, 0), (48, 16, 1), (96, 32, 2), (24, 8, 3), (1, 1, 4)])
def test_dense_rr_matches_lapack(n, m, seed):
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((3 * n, n))
    B = V.T @ V
    A = rng.standard_normal((n, n))
    A = A + A.T
    s, th, C = L.lobpcg_dense_rr(A, B, m)
    assert s == L.OK
    ref = scipy.linalg.eigh(A, B, eigvals_only=True)[:m]
    np.testing.assert_allclose(th, ref, rtol=1e-10, atol=1e-11 * np.abs(ref).max())
    np.testing.assert_allclose(C.T @ B @ C, np.eye(m), atol=1e-10)
    np.testing.assert_allclose(A @ C, B @ C * th, atol=1e-9 * np.abs(A).max())


def test_dense_rr_multiple_eigenvalues():
    """A pencil with a 5-fold eigenvalue: values exact, the eigenspace spanned."""
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((20, 20)))
    w = np.array([0.5] * 5 + list(np.linspace(1, 3, 15)))
    A = Q @ np.diag(w) @ Q.T
    s, th, C = L.lobpcg_dense_rr(A, np.eye(20), 6)
    assert s == L.OK
    np.testing.assert_allclose(th, w[:6], atol=1e-13)
    # the first five vectors span Q[:, :5]
    P = Q[:, :5] @ Q[:, :5].T
    np.testing.assert_allclose(P @ C[:, :5], C[:, :5], atol=1e-12)


def test_dense_rr_scale_invariant_in_B():
    """Badly scaled gramB (columns converging at different rates) still works."""
    rng = np.random.default_rng(6)
    V = rng.standard_normal((30, 10))
    B0 = V.T @ V
    A0 = rng.standard_normal((10, 10))
    A0 = A0 + A0.T
    d = np.logspace(-12, 3, 10)
    s, th, C = L.lobpcg_dense_rr(A0 * np.outer(d, d), B0 * np.outer(d, d), 4)
    assert s == L.OK
    np.testing.assert_allclose(th, scipy.linalg.eigh(A0, B0, eigvals_only=True)[:4], rtol=1e-9)


def test_dense_rr_rejects_indefinite_B():
    s, _, _ = L.lobpcg_dense_rr(np.eye(3), np.diag([1.0, -1.0, 1.0]), 2)
    assert s == L.ERR_RR
