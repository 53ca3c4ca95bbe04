"""Closed-form spectrum of the Dirichlet 7-point Laplacian (Section 4.1).

The paper compares its computed eigenvalues with
  lambda_{i,j,k} = 4 [sin^2(i pi / (2(nx+1))) + sin^2(j pi / (2(ny+1))) + sin^2(k pi / (2(nz+1)))],
1 <= i <= nx, 1 <= j <= ny, 1 <= k <= nz.  The matching eigenvectors are the
products of discrete sines sin(i pi (x+1)/(nx+1)) sin(j pi (y+1)/(ny+1))
sin(k pi (z+1)/(nz+1)) (the standard Kronecker-sum eigenvectors).
"""
import numpy as np


def eig1d(n):
    i = np.arange(1, n + 1)
    return 4.0 * np.sin(i * np.pi / (2.0 * (n + 1))) ** 2


def smallest(nx, ny, nz, m):
    """The m smallest eigenvalues (with multiplicity), ascending, with their (i,j,k)."""
    # only the lowest m modes per axis can be among the m smallest
    ax, ay, az = eig1d(nx)[: min(nx, m)], eig1d(ny)[: min(ny, m)], eig1d(nz)[: min(nz, m)]
    lam = ax[None, None, :] + ay[None, :, None] + az[:, None, None]
    order = np.argsort(lam, axis=None, kind="stable")[:m]
    kk, jj, ii = np.unravel_index(order, lam.shape)
    return lam.ravel()[order], np.stack([ii + 1, jj + 1, kk + 1], axis=1)


def mode(nx, ny, nz, i, j, k):
    """Unnormalised sine eigenvector, flat in grid order p = x + nx*(y + ny*z)."""
    sx = np.sin(i * np.pi * np.arange(1, nx + 1) / (nx + 1))
    sy = np.sin(j * np.pi * np.arange(1, ny + 1) / (ny + 1))
    sz = np.sin(k * np.pi * np.arange(1, nz + 1) / (nz + 1))
    return (sz[:, None, None] * sy[None, :, None] * sx[None, None, :]).ravel()


def norm_bound(nx, ny, nz):
    """Largest eigenvalue lambda_{nx,ny,nz}."""
    return eig1d(nx)[-1] + eig1d(ny)[-1] + eig1d(nz)[-1]
