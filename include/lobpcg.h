/*
 * lobpcg.h -- C ABI of liblobpcg.so, block LOBPCG for the 7-point 3-D
 * Laplacian (and -div(k grad u)) on one AMD MI355X (gfx950).
 *
 * Method: Knyazev, Argentati, Lashuk, Ovtchinnikov, "Block Locally Optimal
 * Preconditioned Eigenvalue Xolvers (BLOPEX) in hypre and PETSc".  The solver
 * computes the m smallest eigenpairs of A x = lambda B x (Section 2.1.1) with
 * the algorithm of Section 2.2 and soft locking (Section 2.3).  A, B and the
 * preconditioner T are matrix-free (Section 2.2 and Appendix A): here they are
 * described by small descriptors and applied by the library's own kernels.
 *
 * Conventions shared by every entry point
 *  - Grid point (x, y, z) of an nx x ny x nz grid is p = x + nx*(y + ny*z).
 *  - A block of k grid vectors is an N x k array stored point-major: element
 *    (p, j) at offset p*k + j (a C-contiguous (N, k) tensor).  Device blocks
 *    must be 16-byte aligned.
 *  - "d_" pointers are device memory, "h_" pointers host memory.  The caller
 *    owns all memory; the library never allocates or frees device memory
 *    (it carves the caller's workspace) and only allocates small host and
 *    pinned-host buffers inside its context.
 *  - All kernels run on the stream given to lobpcg_setup.  Every entry point
 *    that returns host results synchronises that stream before returning.
 *  - Errors are returned as a status code (below); nothing is thrown across
 *    the ABI.  On an error the outputs are unspecified unless stated.
 *  - Calls on one context must not overlap (a context is not thread-safe).
 */
#ifndef LOBPCG_H
#define LOBPCG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status codes */
enum {
    LOBPCG_OK = 0,              /* converged: every residual norm <= tol            */
    LOBPCG_NOT_CONVERGED = 1,   /* maxit reached; outputs hold the last iterate     */
    LOBPCG_ERR_ARG = -1,        /* bad dimension, pointer, tolerance or mismatch    */
    LOBPCG_ERR_UNSUPPORTED = -2,/* a combination this version does not provide      */
    LOBPCG_ERR_WORKSPACE = -3,  /* workspace too small or misaligned               */
    LOBPCG_ERR_CHOL = -4,       /* Cholesky of X0^T X0 or W^T W failed (steps 3, 11)*/
    LOBPCG_ERR_RR = -5,         /* Rayleigh-Ritz failed even without P (step 24)    */
    LOBPCG_ERR_NONFINITE = -6,  /* NaN or Inf in the input or the iteration         */
    LOBPCG_ERR_HIP = -7         /* a HIP runtime call failed                        */
};

/* ---------------------------------------------------------------- descriptors */
enum { LOBPCG_OP_LAPLACE7 = 0, LOBPCG_OP_VARCOEF7 = 1, LOBPCG_OP_DIAG = 2, LOBPCG_OP_MASS7 = 3 };
enum { LOBPCG_PC_NONE = 0, LOBPCG_PC_GMG_V = 1 };
enum { LOBPCG_FP64 = 0, LOBPCG_MIXED = 1 };     /* solver precision           */
enum { LOBPCG_F64 = 0, LOBPCG_F32 = 1 };        /* element type of one block  */

/* Operator A (or B).  LAPLACE7: the 7-point finite-difference Laplacian with
 * homogeneous Dirichlet boundary, diagonal 6 and off-diagonals -1 (Section 4).
 * VARCOEF7: -div(k grad u) with one coefficient per cell face,
 *   (A u)_p = sum over the six faces f of p of k_f (u_p - u_q),
 * q the neighbour across f (u_q = 0 beyond the boundary).  Face arrays are
 * device FP64, C order: kx (nz, ny, nx+1), ky (nz, ny+1, nx), kz (nz+1, ny, nx);
 * face i along an axis lies between grid indices i-1 and i. */
typedef struct lobpcg_op {
    int nx, ny, nz;
    int kind;
    const double *kx, *ky, *kz;     /* VARCOEF7 only, else NULL */
    const double *diag;             /* DIAG only: N positive FP64 entries (device), */
                                    /* B = diag(diag), e.g. a lumped mass matrix    */
    double b0, b1;                  /* MASS7 only: (B u)_p = b0 u_p + b1 (sum of u  */
                                    /* over the axis neighbours of p in the grid),  */
                                    /* b0 > 6 |b1| (symmetric positive definite);   */
                                    /* a consistent-mass-like B with off-diagonals  */
} lobpcg_op;

/* Preconditioner T (Section 2.1.1 requires it linear, symmetric, positive
 * definite).  GMG_V: a geometric-multigrid V(nu_pre, nu_post) cycle on the
 * constant-coefficient 7-point operator: level l has floor(n/2^l) points per
 * axis (coarse node I on fine node 2I+1), level operator 4^-l L7, weighted
 * Jacobi smoothing with weight omega, full-weighting restriction P^T/8,
 * trilinear prolongation P, and coarse_sweeps Jacobi sweeps from zero on the
 * coarsest level.  nu_pre must equal nu_post (symmetry). */
typedef struct lobpcg_precond {
    int kind;
    int levels;
    int nu_pre, nu_post, coarse_sweeps;
    double omega;
} lobpcg_precond;

typedef struct lobpcg_ctx lobpcg_ctx;   /* opaque */

/* ---------------------------------------------------------------- solver */

/* Device workspace needed by lobpcg_setup for this problem, in bytes.
 * B: NULL (B = I), or a DIAG or MASS7 operator of A's dimensions
 * (A x = lambda B x, Section 2.1.1, with the B-orthonormalisation and the
 * B X, B W, B P recurrences of Section 2.2).  m: block
 * size, 1 <= m <= 128 and 3m <= N (blocks of more than 32 columns run through
 * a general path of the block kernels: slower per column).  Pure host code:
 * callable without a GPU. */
int lobpcg_workspace_bytes(const lobpcg_op *A, const lobpcg_op *B, const lobpcg_precond *T,
                           int m, int precision, size_t *bytes);

/* Create a context: the set-up phase that Section 4's timing tables report
 * apart from the solve (operator, preconditioner hierarchy, and room for the
 * 6m vectors that Section 2.2 keeps so that A X and A P need no extra A
 * products).  d_workspace: caller-owned device memory of
 * at least lobpcg_workspace_bytes bytes, 256-byte aligned, kept alive until
 * lobpcg_destroy.  stream: a hipStream_t (NULL = the default stream).
 * Errors: ARG (as lobpcg_workspace_bytes), WORKSPACE (too small, misaligned
 * or NULL), HIP (the pinned host staging could not be allocated). */
int lobpcg_setup(lobpcg_ctx **ctx, const lobpcg_op *A, const lobpcg_op *B, const lobpcg_precond *T,
                 int m, int precision, void *d_workspace, size_t ws_bytes, void *stream);

/* Solve for the m smallest eigenpairs (Section 2.2, steps 1-37, no
 * constraints; see lobpcg_solve_constrained for steps 2 and 10).  B must be
 * NULL or an operator of the kind given to setup (a DIAG array or the MASS7
 * coefficients may differ between calls); with B, X is B-orthonormal and rho_j = ||A x_j - lambda_j B x_j|| /
 * (||A|| ||B x_j||) (for B = I the definition below).  A must have the dimensions and kind given to setup (its
 * face arrays may differ between calls); T must equal setup's.
 *   d_X0         N x m FP64 start block (linearly independent columns)
 *   tol          stop when every rho_j = ||A x_j - lambda_j x_j|| / (||A|| ||x_j||)
 *                is <= tol; ||A|| is the operator's infinity norm
 *   maxit        number of passes through the main loop
 *   h_lambda     [m] out: Ritz values, ascending
 *   d_X          N x m FP64 out: Ritz vectors, orthonormal
 *   h_hist       [maxit x m] out or NULL: rho_j of every column per iteration
 *   h_iters      out: iterations performed (rows of h_hist written)
 *   h_final_resid [m] out or NULL: rho_j recomputed with an explicit A X
 * precision MIXED: FP32 iterations until the residuals stop falling or reach
 * the switch tolerance, then FP64 iterations (FP32 preconditioner) to tol. */
int lobpcg_solve(lobpcg_ctx *ctx, const lobpcg_op *A, const lobpcg_op *B, const lobpcg_precond *T,
                 const double *d_X0, int m, double tol, int maxit, double *h_lambda, double *d_X,
                 double *h_hist, int *h_iters, double *h_final_resid);

/* lobpcg_solve with constraints (hard locking, Section 2.3): the eigenpairs
 * are sought in the B-orthogonal complement of span(Y), imposed on X0 (step
 * 2) and on every preconditioned residual block (step 10) as
 * V - Y (Y^T B Y)^-1 (Y^T B V) (B = I without B).
 *   d_Y   N x ny FP64, point-major, full column rank, 1 <= ny <= 128,
 *         3m + ny <= N; caller-owned, read during the call only
 * As printed, step 7 does not project the residual: it goes to zero only when
 * span(Y) is invariant under A, as for previously computed eigenvectors (the
 * intended use: repeated calls with the converged X appended to Y give the
 * next eigenpairs).  In a MIXED context the FP32 iterations project their
 * residual blocks in FP64 (up-cast, project, down-cast) and the FP64 finish
 * applies step 2 again to the iterate it starts from.  With B, B Y is formed
 * once per call (in pieces of at most m columns) for Y^T B Y, and B V for
 * every projected block.  A rank-deficient Y (Cholesky of Y^T B Y fails)
 * gives ERR_ARG.  Other arguments and outputs as lobpcg_solve. */
int lobpcg_solve_constrained(lobpcg_ctx *ctx, const lobpcg_op *A, const lobpcg_op *B, const lobpcg_precond *T,
                             const double *d_Y, int ny, const double *d_X0, int m, double tol, int maxit,
                             double *h_lambda, double *d_X, double *h_hist, int *h_iters,
                             double *h_final_resid);

/* Hellmann-Feynman eigenvalue adjoint for VARCOEF7: for
 * lambda_i = (x_i, A x_i) / (x_i, B x_i) and A = sum_f k_f (e_p - e_q)(e_p - e_q)^T
 * (B = I, or the context's B, which does not depend on k),
 * d lambda_i / d k_f = (x_i[p] - x_i[q])^2 / (x_i, B x_i).  Writes the
 * vector-Jacobian product g_f = sum_i h_gbar[i] d lambda_i / d k_f into the
 * three device FP64 face arrays (shapes as in lobpcg_op).  d_X: N x m FP64. */
int lobpcg_eig_grad_k(lobpcg_ctx *ctx, const double *d_X, const double *h_gbar, int m,
                      double *d_gkx, double *d_gky, double *d_gkz);

/* Release a context made by lobpcg_setup (its host and pinned-host buffers;
 * the caller's workspace is left alone).  NULL is a no-op. */
void lobpcg_destroy(lobpcg_ctx *ctx);
/* A static, human-readable name of a status code above, including the
 * failure modes Section 2.2 names (Cholesky of steps 3 and 11 failing,
 * Rayleigh-Ritz of step 24 failing); "unknown status" for other values. */
const char *lobpcg_status_string(int status);

/* ---------------------------------------------------------------- options and statistics */
enum {
    LOBPCG_OPT_SWITCH_TOL = 0,      /* MIXED: FP32 phase ends at max rho <= this (default 3e-7) */
    LOBPCG_OPT_STALL_WINDOW = 1,    /* MIXED: ... or when max rho fell by less than a    */
    LOBPCG_OPT_STALL_FACTOR = 2,    /*        factor STALL_FACTOR (default 0.95) over    */
                                    /*        STALL_WINDOW (default 10) iterations       */
    LOBPCG_OPT_PROFILE = 3,         /* 1: time each step class with HIP events          */
    LOBPCG_OPT_REACTIVATE = 4,      /* 1 (default): see lobpcg_solve's stopping rule    */
    LOBPCG_OPT_KERNELS = 5,         /* kernel variants, 0 = default; results agree to  */
                                    /* rounding.  Bit 0: the FP32 update of steps      */
                                    /* 25-33 on the fragment kernel (register loads)   */
                                    /* instead of the LDS-pipelined one; bit 1: the    */
                                    /* V-cycle on the active columns as stored, not    */
                                    /* rounded up to the 16-byte vector width; bit 2:  */
                                    /* the multi-column-tile Gram kernel also for      */
                                    /* narrow single-block Grams; bit 3: up to four    */
                                    /* Gram tiles per wave (default two); bit 4: the   */
                                    /* same for FP32 blocks only; bit 5: Gram operands */
                                    /* loaded per tile group rather than staged once   */
                                    /* per row chunk through LDS (bits 3-4 apply to    */
                                    /* that kernel and to products with more operand   */
                                    /* blocks than the LDS-staged kernel holds); bit   */
                                    /* 6: the LDS-pipelined update stores P, AP and W  */
                                    /* per MFMA fragment also when they have at most   */
                                    /* 16 columns (default: as compact rows)           */
    LOBPCG_OPT_FP32_EXPLICIT_GRAM = 6,/* MIXED: 1 (default) FP32 iterations compute   */
                                    /* X^T X, X^T AX, W^T W, P^T P rather than taking  */
                                    /* I and Lambda for them as the paper's form does  */
    LOBPCG_OPT_FOLD_CHOLQR = 7,     /* 1 (default): the Cholesky-QR factors of steps   */
                                    /* 11 and 14-15 are folded into the Gram matrices  */
                                    /* and the update coefficients (W_J R^-1 and       */
                                    /* P_J R^-1 are never formed; same algebra, fewer  */
                                    /* passes); 0: applied to the blocks               */
    LOBPCG_OPT_LOCK_GAP = 9,        /* soft locking by clusters: a column below tol    */
                                    /* stays active while an unconverged active column */
                                    /* has a Ritz value within this relative distance  */
                                    /* of its own (0 <= value < 1)                     */
    LOBPCG_OPT_NWANT = 10,          /* a block wider than the wanted set (Section      */
                                    /* 2.1.3's advice when the spectrum clusters at    */
                                    /* the block edge): the solve ends as soon as the  */
                                    /* first NWANT columns (the smallest Ritz pairs)   */
                                    /* have rho_j <= tol, the rest being guard         */
                                    /* columns; 0 (default) = m.  In the mixed solver  */
                                    /* the FP32 phase's switch and stall tests also    */
                                    /* look at the wanted columns only                 */
    LOBPCG_OPT_FP32_EXPLICIT_ABOVE = 11,/* MIXED, with FP32_EXPLICIT_GRAM: an FP32       */
                                    /* iteration takes the explicit form only while    */
                                    /* more than this many columns are active, the     */
                                    /* paper's form after (X then changes little per   */
                                    /* iteration; the Gram step reads neither AX nor   */
                                    /* the X-X tiles); default m/4 rounded down, 0:    */
                                    /* always the explicit form                        */
    LOBPCG_OPT_FP64_EXPLICIT_GRAM = 8 /* 1: FP64 iterations compute the block diagonal */
                                    /* of gramB and X^T AX too (the variant Section    */
                                    /* 2.2 reports testing in MATLAB: better           */
                                    /* attainable accuracy; it keeps long runs on      */
                                    /* clustered spectra from losing orthogonality);   */
                                    /* 0 (default): the paper's form                   */
};
int lobpcg_set_option(lobpcg_ctx *ctx, int key, double value);

enum {
    LOBPCG_STEP_RESIDUAL = 0,   /* step 7 and the norms of step 8          */
    LOBPCG_STEP_PRECOND = 1,    /* step 9                                  */
    LOBPCG_STEP_ORTHO = 2,      /* steps 3, 11, 14-15 (Gram, Cholesky, apply)*/
    LOBPCG_STEP_APPLY_A = 3,    /* step 12 and explicit A X                */
    LOBPCG_STEP_GRAM = 4,       /* steps 17-23                             */
    LOBPCG_STEP_RR = 5,         /* step 24 (host FP64)                     */
    LOBPCG_STEP_UPDATE = 6,     /* steps 25-33                             */
    LOBPCG_STEP_OTHER = 7,      /* precision casts, phase switch, copies   */
    LOBPCG_NSTEP = 8
};
typedef struct lobpcg_stats {
    int iters_total, iters_fp32, iters_fp64;
    int restarts;               /* iterations run without P after a failure */
    int status;
    double solve_ms;            /* host wall time of the last lobpcg_solve  */
    double step_ms[LOBPCG_NSTEP];   /* summed HIP-event times (OPT_PROFILE)  */
    int step_calls[LOBPCG_NSTEP];
    double step_bytes[LOBPCG_NSTEP];/* algorithmic HBM bytes of the step's   */
                                    /* kernels: each operand the arithmetic  */
                                    /* needs read once, each result written  */
                                    /* once (always counted)                 */
} lobpcg_stats;
int lobpcg_get_stats(const lobpcg_ctx *ctx, lobpcg_stats *stats);

/* ---------------------------------------------------------------- the steps one by one
 * The solver's building blocks, exposed for testing and timing.  They use
 * the context's workspace as scratch (so they may overwrite solver state)
 * and its dimensions: N = nx*ny*nz of setup's operator, k <= m unless said.
 * dtype selects FP64 or FP32 elements; FP32 requires a MIXED context. */

/* d_out = A d_in for an N x k block (the block product of step 12). */
int lobpcg_apply_A(lobpcg_ctx *ctx, const lobpcg_op *A, int dtype, const void *d_in, void *d_out, int k);

/* d_out = T d_in for an N x k block (step 9); T is setup's preconditioner. */
int lobpcg_apply_T(lobpcg_ctx *ctx, int dtype, const void *d_in, void *d_out, int k);

/* Gram products of steps 17-23 for S = [S_0 .. S_{n-1}] and AS = [AS_0 ..],
 * n <= 3 blocks of widths w_i (sum K <= 3m), all N x w_i of type dtype:
 * h_SS = S^T S and h_SAS = S^T AS, K x K row-major FP64 on the host, upper
 * triangle (entries (a, b), a <= b) computed, the strict lower triangle
 * mirrored from it.  Accumulation is FP64 across row chunks.  paper_form = 1
 * (needs AS and n >= 2) computes only the entries the paper's form of steps
 * 17-23 does not take as known -- S^T S off the block diagonal, S^T AS outside
 * the S_0-S_0 block -- and returns zero for the others. */
int lobpcg_gram(lobpcg_ctx *ctx, int dtype, int n, const void *const *d_S, const void *const *d_AS,
                const int *w, int paper_form, double *h_SS, double *h_SAS);

/* Multivector combination used by steps 3-4, 11, 14-15 and 25-33:
 * d_out (N x kout) = sum_i in_i[:, cols_i] C_i (+ d_add if not NULL), with
 * n <= 3 inputs of widths ld_i, column selections cols_i[0..k_i-1] (NULL =
 * all ld_i columns, k_i = ld_i) and h_C the stacked (sum k_i) x kout
 * row-major FP64 coefficients.  d_out must not alias an input. */
int lobpcg_combine(lobpcg_ctx *ctx, int dtype, int n, const void *const *d_in, const int *ld,
                   const int *const *cols, const int *k, const double *h_C, int kout,
                   const void *d_add, void *d_out);

/* Steps 25-33 fused with step 7 of the next iteration (the solver's update):
 * with C = [C_X; C_W; C_P] ((m + nW + nP) x m row-major FP64 on the host),
 *   P'  = W C_W + P C_P,    AP' = AW C_W + AP C_P       (step 27-30 form)
 *   X'  = X C_X + P',       AX' = AX C_X + AP'          (steps 31-33)
 *   W'  = AX'_j - theta_j X'_j for j in J               (step 7)
 * for d_X, d_AX (N x m), d_W, d_AW (N x nW), and P, AP: the columns
 * h_Pcols[0..nP) of d_P, d_AP (N x ldP), or with h_Pcols NULL all of them
 * (ldP = nP); nP = 0 drops the P terms (d_P, d_AP may then be NULL).  d_Xn,
 * d_AXn (N x m) receive X', AX';
 * d_Pn, d_APn, d_Wn (N x nJ) receive the columns h_J[0..nJ) of P', AP', W'
 * packed (column jj = column h_J[jj]); h_rho[j] = ||AX'_j - theta_j X'_j|| /
 * (norm_A ||X'_j||) for all m columns.  Outputs must not alias inputs
 * (ARG).  1 <= nW, nJ <= m, 0 <= nP <= m, nP <= ldP <= m, h_J distinct in
 * [0, m), h_Pcols in [0, ldP). */
int lobpcg_update(lobpcg_ctx *ctx, int dtype, const void *d_X, const void *d_AX, const void *d_W,
                  const void *d_AW, int nW, const void *d_P, const void *d_AP, int ldP, const int *h_Pcols, int nP,
                  const double *h_C, const double *h_theta, const int *h_J, int nJ, double norm_A, void *d_Xn,
                  void *d_AXn, void *d_Pn, void *d_APn, void *d_Wn, double *h_rho);

/* Step 7 and the norms of step 8: for the m columns of d_X, d_AX (N x m)
 * and Ritz values h_lambda, writes W_J = AX_J - X_J Lambda_J packed as
 * N x nJ (column jj = column h_J[jj]) and h_rho[j] = ||AX_j - lambda_j X_j|| /
 * (norm_A ||X_j||) for all j. */
int lobpcg_residual(lobpcg_ctx *ctx, int dtype, const void *d_X, const void *d_AX, int m,
                    const double *h_lambda, const int *h_J, int nJ, double norm_A, void *d_W,
                    double *h_rho);

/* lobpcg_residual without a context, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): it calls no allocating routine, takes every input and output
 * in device memory, synchronises nothing and only enqueues kernels on
 * `stream` (a hipStream_t, NULL = the default stream).  Its kernels' scratch
 * (per-workgroup partial sums and their reduction, 2 MiB + 2 KiB) is a
 * fixed array in the library's device memory, one per GPU, kept until the
 * process ends; calls that overlap on one GPU race on it (serialise them,
 * e.g. on one stream).  Nothing in the scratch needs clearing between calls.
 *   dtype      LOBPCG_F64 or LOBPCG_F32 for X, AX and W
 *   N, m       N x m point-major blocks d_X, d_AX (16-byte aligned), 1 <= m <= 128
 *   d_lambda   [m] FP64 Ritz values
 *   d_jpos     [m] packed column of j in W, or -1 (column not written)
 *   nJ, d_W    W (N x nJ) receives AX_j - lambda_j X_j in column d_jpos[j]
 *              (d_W may be NULL when nJ = 0)
 *   d_rho      [m] FP64 out: ||AX_j - lambda_j X_j|| / (norm_A ||X_j||)
 * Errors (checked before anything is enqueued): ARG for a bad type, size,
 * pointer or m > 128; HIP when a launch fails.  Results are valid once the
 * stream has reached the call. */
int lobpcg_residual_noalloc(int dtype, long long N, const void *d_X, const void *d_AX, int m,
                            const double *d_lambda, const int *d_jpos, int nJ, double norm_A, void *d_W,
                            double *d_rho, void *stream);

/* Host FP64 dense kernels (no GPU needed). */
/* Scale-invariant Cholesky G = R^T R (Section 2.2: the factorisation must be
 * invariant under column scaling): R = Rh D, D = diag(G)^(1/2), Rh^T Rh =
 * D^-1 G D^-1.  G, R: n x n row-major; R upper triangular.  Returns
 * LOBPCG_ERR_CHOL if G is not numerically positive definite. */
int lobpcg_dense_chol(int n, const double *G, double *R);
/* Step 24: the m smallest eigenpairs of gramA C = gramB C Theta (n x n,
 * row-major, symmetric, gramB positive definite), ascending, with
 * C^T gramB C = I.  C: n x m row-major.  LOBPCG_ERR_RR if gramB is not
 * positive definite or the eigensolver fails. */
int lobpcg_dense_rr(int n, int m, const double *gramA, const double *gramB, double *theta, double *C);

#ifdef __cplusplus
}
#endif
#endif /* LOBPCG_H */
