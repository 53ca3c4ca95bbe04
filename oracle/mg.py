"""Geometric-multigrid V-cycle preconditioner T (test infrastructure only).

The paper applies hypre's multigrid preconditioners and only requires that T
be linear, symmetric and positive definite (Section 2.1.1).  This is the
reading of the multigrid used here, a plain V(nu_pre, nu_post) cycle:

* level l has grid floor(n/2^l) per axis; coarse node I sits on fine node 2I+1;
* level operator A_l = 4^-l * L7 (the 7-point stencil rediscretised on the
  coarser grid, in units of the finest spacing);
* smoother: weighted Jacobi x <- x + omega D_l^-1 (b - A_l x), D_l = 6*4^-l;
* restriction R = P^T/8 (full weighting), prolongation P trilinear;
* coarsest level: `coarse_sweeps` Jacobi sweeps from a zero guess.

Equal pre/post sweep counts make T symmetric; every piece is a polynomial in
a symmetric matrix or a Galerkin-type product, so T is SPD as required.
"""
from . import grid


class VCycle:
    def __init__(self, dims, levels, nu_pre=2, nu_post=2, coarse_sweeps=20, omega=2.0 / 3.0):
        self.levels = [tuple(dims)]
        for _ in range(levels - 1):
            self.levels.append(grid.coarsen(self.levels[-1]))
        if min(min(d) for d in self.levels) < 1:
            raise ValueError("grid too small for %d levels" % levels)
        self.nu_pre, self.nu_post, self.coarse_sweeps, self.omega = nu_pre, nu_post, coarse_sweeps, omega

    def _smooth(self, l, x, b, sweeps):
        s = 4.0 ** (-l)
        for _ in range(sweeps):
            x = grid.jacobi(self.levels[l], s, self.omega, x, b)
        return x

    def _cycle(self, l, b):
        dims = self.levels[l]
        if l == len(self.levels) - 1:
            x = self._smooth(l, None, b, self.coarse_sweeps)
            return x if x is not None else 0.0 * b
        x = self._smooth(l, None, b, self.nu_pre)
        if x is None:
            x = 0.0 * b
        r = b - 4.0 ** (-l) * grid.laplace7(dims, x)
        e = self._cycle(l + 1, grid.restrict(dims, self.levels[l + 1], r))
        x = grid.prolong_add(dims, self.levels[l + 1], e, x)
        x = self._smooth(l, x, b, self.nu_post)
        return x

    def __call__(self, b):
        """T b for a block b of shape (N, k) (or one vector)."""
        return self._cycle(0, b)
