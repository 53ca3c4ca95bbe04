"""Block LOBPCG for the 7-point 3-D Laplacian on AMD MI355X (gfx950).

The solver, its kernels and its C ABI live in liblobpcg.so (sources in csrc/,
header include/lobpcg.h); this package is the thin Python binding.
"""
from .lobpcg import *  # noqa: F401,F403
from .lobpcg import (Context, Diag, LobpcgError, Mass7, Op, Precond, SolveResult, lib, lobpcg_apply_A,  # noqa: F401
                     lobpcg_apply_T, lobpcg_combine, lobpcg_dense_chol, lobpcg_dense_rr, lobpcg_eig_grad_k,
                     lobpcg_get_stats, lobpcg_gram, lobpcg_residual, lobpcg_set_option, lobpcg_setup,
                     lobpcg_solve, lobpcg_update, lobpcg_workspace_bytes, status_string)
