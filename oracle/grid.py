"""ctypes wrappers over the oracle's C grid loops (test infrastructure only).

A block of k grid vectors is a float64 array of shape (N, k) in column-major
(Fortran) order, so that each vector is contiguous; 1-D arrays are one vector.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        i, d, p = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        L.or_laplace7.argtypes = [i, i, i, i, p, p]
        L.or_varcoef7.argtypes = [i, i, i, i, p, p, p, p, p]
        L.or_restrict.argtypes = [i, i, i, i, i, i, i, p, p]
        L.or_prolong_add.argtypes = [i, i, i, i, i, i, i, p, p]
        L.or_jacobi.argtypes = [i, i, i, i, d, d, p, p, p]
        L.or_eig_grad_faces.argtypes = [i, i, i, i, p, p, p, p, p]
        for f in (L.or_laplace7, L.or_varcoef7, L.or_restrict, L.or_prolong_add, L.or_jacobi,
                  L.or_eig_grad_faces):
            f.restype = None
        _lib = L
    return _lib


def _colmajor(u):
    u = np.asarray(u, dtype=np.float64)
    if u.ndim == 1:
        u = u[:, None]
    return np.asfortranarray(u)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _shape_back(out, u):
    return out[:, 0] if np.ndim(u) == 1 else out


def laplace7(dims, u):
    """A u for the 7-point Laplacian (Section 4)."""
    nx, ny, nz = dims
    uc = _colmajor(u)
    assert uc.shape[0] == nx * ny * nz
    out = np.empty_like(uc, order="F")
    lib().or_laplace7(nx, ny, nz, uc.shape[1], _ptr(uc), _ptr(out))
    return _shape_back(out, u)


def varcoef7(dims, kx, ky, kz, u):
    """A u for -div(k grad u) with face coefficients kx, ky, kz."""
    nx, ny, nz = dims
    uc = _colmajor(u)
    kx, ky, kz = (np.ascontiguousarray(a, dtype=np.float64) for a in (kx, ky, kz))
    assert kx.size == nz * ny * (nx + 1) and ky.size == nz * (ny + 1) * nx and kz.size == (nz + 1) * ny * nx
    out = np.empty_like(uc, order="F")
    lib().or_varcoef7(nx, ny, nz, uc.shape[1], _ptr(kx), _ptr(ky), _ptr(kz), _ptr(uc), _ptr(out))
    return _shape_back(out, u)


def mass7(dims, b0, b1, u):
    """B u for a 7-point mass-type operator: (B u)_p = b0 u_p + b1 * (sum of u
    over the up to six axis neighbours of p inside the grid).  It is
    symmetric, and positive definite when b0 > 6 |b1| (strict diagonal
    dominance): a stand-in for a consistent finite-element mass matrix, the
    kind of B the generalized problem of Section 2.1.1 is written for.
    Plain numpy on a zero-padded copy of the grid."""
    nx, ny, nz = dims
    uc = _colmajor(u)
    k = uc.shape[1]
    g = np.zeros((nz + 2, ny + 2, nx + 2, k))
    g[1:-1, 1:-1, 1:-1] = np.stack([uc[:, j].reshape(nz, ny, nx) for j in range(k)], axis=3)
    nb = (g[1:-1, 1:-1, :-2] + g[1:-1, 1:-1, 2:] + g[1:-1, :-2, 1:-1] + g[1:-1, 2:, 1:-1]
          + g[:-2, 1:-1, 1:-1] + g[2:, 1:-1, 1:-1])
    out = b0 * g[1:-1, 1:-1, 1:-1] + b1 * nb
    res = np.asfortranarray(np.stack([out[..., j].ravel() for j in range(k)], axis=1))
    return _shape_back(res, u)


def gershgorin_mass7(b0, b1):
    """||B||_inf bound b0 + 6 |b1|."""
    return abs(b0) + 6.0 * abs(b1)


def restrict(fine, coarse, r):
    uc = _colmajor(r)
    out = np.empty((coarse[0] * coarse[1] * coarse[2], uc.shape[1]), order="F")
    lib().or_restrict(*fine, *coarse, uc.shape[1], _ptr(uc), _ptr(out))
    return _shape_back(out, r)


def prolong_add(fine, coarse, e, x):
    """x + P e (returns a new array)."""
    ec = _colmajor(e)
    xc = np.array(_colmajor(x), order="F", copy=True)
    lib().or_prolong_add(*fine, *coarse, ec.shape[1], _ptr(ec), _ptr(xc))
    return _shape_back(xc, x)


def jacobi(dims, scale, omega, x, b):
    """x + omega/(6 scale) (b - scale*L7 x); x None means a zero guess."""
    bc = _colmajor(b)
    out = np.empty_like(bc, order="F")
    xc = None if x is None else _colmajor(x)
    lib().or_jacobi(*dims, bc.shape[1], float(scale), float(omega),
                    None if xc is None else _ptr(xc), _ptr(bc), _ptr(out))
    return _shape_back(out, b)


def eig_grad_faces(dims, X, gbar):
    """Face gradients sum_i gbar_i (x_i[p]-x_i[q])^2/(x_i,x_i), as (gkx, gky, gkz)."""
    nx, ny, nz = dims
    Xc = _colmajor(X)
    g = np.ascontiguousarray(gbar, dtype=np.float64)
    assert g.size == Xc.shape[1]
    gkx = np.empty((nz, ny, nx + 1)); gky = np.empty((nz, ny + 1, nx)); gkz = np.empty((nz + 1, ny, nx))
    lib().or_eig_grad_faces(nx, ny, nz, Xc.shape[1], _ptr(Xc), _ptr(g), _ptr(gkx), _ptr(gky), _ptr(gkz))
    return gkx, gky, gkz


def eig_grad_faces_B(dims, X, gbar, BX):
    """The face gradients for A x = lambda B x with B independent of k:
    d lambda_i / d k_f = (x_i[p]-x_i[q])^2 / (x_i, B x_i), i.e. the sums of
    eig_grad_faces with each weight gbar_i rescaled from (x_i, x_i) to
    (x_i, B x_i).  BX: B applied to the columns of X."""
    X = np.asarray(X, dtype=np.float64)
    BX = np.asarray(BX, dtype=np.float64)
    xx = np.einsum("pi,pi->i", X, X)
    xbx = np.einsum("pi,pi->i", X, BX)
    return eig_grad_faces(dims, X, np.asarray(gbar, dtype=np.float64) * xx / xbx)


def coarsen(dims):
    """Grid of the next coarser level: each axis halves, rounding down."""
    return tuple(n // 2 for n in dims)


def gershgorin_laplace7():
    """||A|| bound max_p sum_q |A_pq| = 12 for the 7-point Laplacian."""
    return 12.0


def gershgorin_varcoef7(dims, kx, ky, kz):
    """||A||_inf = max_p sum_q |A_pq|: the diagonal is the sum of the six face
    coefficients of p, and each face to an interior neighbour adds its
    coefficient once more off the diagonal (boundary faces only add to the
    diagonal)."""
    nx, ny, nz = dims
    kx, ky, kz = (np.asarray(a).reshape(s) for a, s in
                  zip((kx, ky, kz), ((nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx))))
    diag = kx[:, :, :-1] + kx[:, :, 1:] + ky[:, :-1, :] + ky[:, 1:, :] + kz[:-1] + kz[1:]
    off = np.zeros_like(diag)
    off[:, :, 1:] += kx[:, :, 1:-1]
    off[:, :, :-1] += kx[:, :, 1:-1]
    off[:, 1:, :] += ky[:, 1:-1, :]
    off[:, :-1, :] += ky[:, 1:-1, :]
    off[1:] += kz[1:-1]
    off[:-1] += kz[1:-1]
    return float((diag + off).max())


def laplace7_rows(dims, U, points):
    """(A U)[p, :] for the listed grid points only (for sampled checks of
    blocks too large to apply the whole operator to).  U: (N, k), any order."""
    nx, ny, nz = dims
    U = np.asarray(U)
    out = np.empty((len(points), U.shape[1]))
    for r, p in enumerate(points):
        p = int(p)
        x, y, z = p % nx, (p // nx) % ny, p // (nx * ny)
        s = 6.0 * U[p].astype(np.float64)
        for dx, dy, dz in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
            a, b, c = x + dx, y + dy, z + dz
            if 0 <= a < nx and 0 <= b < ny and 0 <= c < nz:
                s = s - U[a + nx * (b + ny * c)].astype(np.float64)
        out[r] = s
    return out
