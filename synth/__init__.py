"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and the bench.

This module only draws numbers: it holds none of the eigensolver's arithmetic.
Both implementations receive the arrays made here, so that the random start
vectors and coefficient fields are identical on both sides.

Workload recipe (the paper's own test problems are synthetic too: the 7-point
Dirichlet Laplacian on an nx x ny x nz grid, Section 4):

* start block X0: i.i.d. uniform[-1, 1] in float64, drawn with
  ``numpy.random.default_rng(seed)`` in grid-point-major order (row p is grid
  point p = x + nx*(y + ny*z), column j is start vector j).  The paper says the
  initial approximations are chosen randomly (Section 4.1) and its drivers use
  seed 2 (Appendix B), which is the default here.
* face coefficients of -div(k grad u): k_f = exp(g_f), with g a Gaussian
  random field of standard deviation ``sigma`` and squared-exponential
  correlation length ``corr`` cells, sampled on the (nx+2)x(ny+2)x(nz+2) node
  grid including the boundary layer and averaged onto each face's two nodes.
"""
import numpy as np

__all__ = ["x0_uniform", "gaussian_field_faces", "face_shapes", "sample_faces", "random_block"]


def x0_uniform(N, m, seed=2):
    """Start block X0, shape (N, m) float64, C-contiguous (point-major)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(N, m))


def random_block(N, k, seed, dtype=np.float64):
    """Generic seeded test block, shape (N, k), uniform[-1, 1]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(N, k)).astype(dtype)


def face_shapes(nx, ny, nz):
    """Array shapes (z, y, x order) of the x-, y- and z-face coefficient arrays.

    x-face (z, y, i) sits between grid x-indices i-1 and i, for i = 0..nx; the
    faces i = 0 and i = nx touch the Dirichlet boundary.  Likewise for y and z.
    """
    return (nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)


def gaussian_field_faces(nx, ny, nz, sigma=0.5, corr=8.0, seed=2):
    """Lognormal face coefficients (kx, ky, kz), float64, C-contiguous.

    g: white noise on the node grid (including one boundary layer on each
    side), smoothed with a Gaussian filter of std corr/sqrt(2) cells so that
    its covariance is proportional to exp(-r^2 / (2 corr^2)), then shifted and
    scaled to zero mean and standard deviation sigma.  Node (a, b, c) of the
    padded grid is interior point (a-1, b-1, c-1).  A face takes the mean of g
    over its two nodes and k_f = exp(g_f).
    """
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(size=(nz + 2, ny + 2, nx + 2))
    g = gaussian_filter(g, sigma=corr / np.sqrt(2.0), mode="reflect")
    g = (g - g.mean()) / g.std() * sigma
    # x-faces: between padded nodes (c, b, i) and (c, b, i+1), interior rows only
    gx = 0.5 * (g[1:-1, 1:-1, :-1] + g[1:-1, 1:-1, 1:])
    gy = 0.5 * (g[1:-1, :-1, 1:-1] + g[1:-1, 1:, 1:-1])
    gz = 0.5 * (g[:-1, 1:-1, 1:-1] + g[1:, 1:-1, 1:-1])
    kx, ky, kz = (np.ascontiguousarray(np.exp(a)) for a in (gx, gy, gz))
    assert (kx.shape, ky.shape, kz.shape) == face_shapes(nx, ny, nz)
    return kx, ky, kz


def sample_faces(n_total, count, seed):
    """`count` distinct flat face indices out of n_total, seeded."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_total, size=count, replace=False))
