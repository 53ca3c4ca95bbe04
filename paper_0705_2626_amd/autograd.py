"""Eigenvalue gradients through torch.autograd.

EigSmallest maps the face coefficients k of -div(k grad u) to the m smallest
eigenvalues, solving with LOBPCG (FP64) in the forward pass; the backward pass
is one launch of the library's Hellmann-Feynman adjoint kernel,
d lambda_i / d k_f = (x_i[p] - x_i[q])^2 / (x_i, B x_i) (B = I unless the
solver context has a B, which does not depend on k), contracted with the
incoming gradient.  The derivative is undefined where lambda_i is a multiple
eigenvalue; a warning is raised when two returned eigenvalues are closer than
1e-8 ||A||.
"""
import warnings

import torch

from . import lobpcg as L


class EigSmallest(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kx, ky, kz, solver, X0, tol, maxit):
        A = L.Op(*solver.A.dims, kx, ky, kz)
        r = L.lobpcg_solve(solver, X0, tol, maxit, A=A, hist=False)
        if r.status != L.OK:
            warnings.warn("EigSmallest: LOBPCG did not converge (%s)" % L.status_string(r.status))
        lam = torch.tensor(r.lam, dtype=torch.float64, device=kx.device)
        gaps = (lam[1:] - lam[:-1]).abs()
        if gaps.numel() and float(gaps.min()) < 1e-8 * float(lam.abs().max()):
            warnings.warn("EigSmallest: nearly multiple eigenvalues; their gradient is not defined")
        ctx.save_for_backward(r.X)
        ctx.solver = solver
        ctx.result = r
        return lam

    @staticmethod
    def backward(ctx, gbar):
        (X,) = ctx.saved_tensors
        gkx, gky, gkz = L.lobpcg_eig_grad_k(ctx.solver, X, gbar.detach().double().cpu().numpy())
        return gkx, gky, gkz, None, None, None, None


def eig_smallest(kx, ky, kz, solver, X0, tol=1e-10, maxit=500):
    """The m smallest eigenvalues of -div(k grad u), differentiable in k."""
    return EigSmallest.apply(kx, ky, kz, solver, X0, tol, maxit)
