"""Block LOBPCG oracle, FP64 (test infrastructure only).

Follows the algorithm of Section 2.2 (steps 1-37), for B = I or a given SPD
B, with optional constraints Y (steps 2 and 10: hard locking) and soft
locking as described
in Section 2.3: only the active columns J get residuals, preconditioned
residuals W_J and directions P_J, while all m columns of X take part in every
Rayleigh-Ritz procedure.

Readings of the paper taken here (each is listed with its reason in the
design notes of the repository):
* residual norm: rho_j = ||A x_j - lambda_j x_j||_2 / (||A|| ||x_j||_2), with
  ||A|| the Gershgorin bound of the operator;
* "for k = 0, ..., MaxIterations" is read as maxit passes of the loop;
* a column leaves J when rho_j <= tol and stays out while other columns are
  active; the loop ends only when every column has rho_j <= tol.  If J
  empties while a soft-locked column has drifted back above tol (this
  happens inside degenerate eigenvalue groups, where the condition that makes
  locked vectors keep improving, Section 2.3, does not hold), those columns
  are made active again;
* Cholesky is made scale invariant by an explicit diagonal scaling (the
  paper requires scale invariance, Section 2.2, and explicit column scaling
  is the fix it names);
* if the Cholesky factorisation of P_J^T P_J or the Rayleigh-Ritz problem with
  P fails, that iteration proceeds without P (a restart); failure without P is
  an error.
"""
import numpy as np
import scipy.linalg

OK, NOT_CONVERGED = 0, 1
ERR_CHOL, ERR_RR, ERR_NONFINITE = -4, -5, -6


class CholeskyFailure(Exception):
    pass


def chol_scaled(G):
    """Scale-invariant Cholesky G = R^T R, R upper triangular (Section 2.2).

    With d = sqrt(diag G): G = D Gh D, Gh = R_h^T R_h, and R = R_h D, so the
    factor of a column-scaled Gram matrix is the column-scaled factor.
    """
    G = 0.5 * (G + G.T)
    d = np.sqrt(np.diag(G)) if np.all(np.diag(G) > 0) else None
    if d is None or not np.all(np.isfinite(d)):
        raise CholeskyFailure("non-positive or non-finite diagonal")
    Gh = G / np.outer(d, d)
    try:
        L = np.linalg.cholesky(Gh)
    except np.linalg.LinAlgError as e:
        raise CholeskyFailure(str(e))
    return L.T * d[None, :]


def right_solve_upper(V, R):
    """V R^{-1} for upper-triangular R."""
    return scipy.linalg.solve_triangular(R, V.T, trans="T", lower=False).T


def orthonormalize(V, *others):
    """Cholesky orthonormalisation: R = chol(V^T V); V R^-1 (and others R^-1)."""
    R = chol_scaled(V.T @ V)
    return (right_solve_upper(V, R),) + tuple(right_solve_upper(O, R) for O in others)


def rayleigh_ritz(gramA, gramB, m):
    """Step 24: gramA C = gramB C Theta; the m smallest, C gramB-orthonormal."""
    theta, C = scipy.linalg.eigh(gramA, gramB)
    return theta[:m], C[:, :m]


class Result:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def b_orthonormalize(V, BV, *others):
    """B-orthonormalisation (steps 3, 11, 14-15): R = chol(V^T BV);
    V R^-1, BV R^-1 (and others R^-1)."""
    R = chol_scaled(V.T @ BV)
    return (right_solve_upper(V, R), right_solve_upper(BV, R)) + tuple(right_solve_upper(O, R) for O in others)


def lobpcg(apply_A, X0, tol, maxit, normA, apply_T=None, callback=None, reactivate=True, Y=None, apply_B=None,
           explicit_gram=False, lock_gap=0.0, nwant=None):
    """Smallest eigenpairs of A x = lambda B x (Section 2.1.1).

    apply_A, apply_T, apply_B: functions on (N, k) blocks (apply_B None: B = I).
    X0: (N, m) start block.
    Y: optional (N, l) constraint vectors of full column rank: the
    eigenvectors are sought in the B-orthogonal complement of span(Y), which
    steps 2 and 10 impose on X0 and on every preconditioned residual block
    (hard locking, Section 2.3).
    Returns Result(status, lam, X, hist, iters, resid) where hist[k] holds
    rho_j = ||A x_j - lambda_j B x_j|| / (||A|| ||B x_j||) of every column at
    iteration k and resid the explicit final rho_j.
    explicit_gram: the variant of Section 2.2 that computes the block diagonal
    of gramB (X^T B X, W^T B W, P_J^T B P_J) instead of taking identities, and
    with it the X block of gramA (X^T A X instead of Lambda), so that the
    Rayleigh-Ritz procedure sees the basis as it is after rounding.
    lock_gap: soft locking by clusters (a reading, off at 0): a column whose
    residual is below tol stays in J while a column of J that is still above
    tol has a Ritz value within the relative distance lock_gap of its own, so
    that the members of a cluster leave J together.
    nwant: a block wider than the wanted set (Section 2.1.3 advises a few
    columns more than the eigenpairs sought when the spectrum clusters at
    the block edge; a reading of how such a run ends): the iteration also
    ends once the nwant smallest Ritz pairs (the first nwant columns) have
    rho_j <= tol; the other columns are guard vectors, iterated like the rest
    while unconverged.  None: nwant = m.
    """
    X0 = np.asfortranarray(np.asarray(X0, dtype=np.float64))
    N, m = X0.shape
    if not np.all(np.isfinite(X0)):
        return Result(status=ERR_NONFINITE, lam=None, X=None, hist=np.zeros((0, m)), iters=0, resid=None)
    T = apply_T if apply_T is not None else (lambda V: V)
    Bop = apply_B if apply_B is not None else (lambda V: V)
    if Y is not None:
        Y = np.asfortranarray(np.asarray(Y, dtype=np.float64))
        BY = Bop(Y)
        YtBY = Y.T @ BY

        def constrain(V):
            # steps 2 and 10: V - Y (Y^T BY)^-1 ((BY)^T V)
            return V - Y @ np.linalg.solve(YtBY, BY.T @ V)
        X0 = np.asfortranarray(constrain(X0))                  # step 2
    else:
        constrain = None

    def rho_of(X, AX, BX, lam):
        Rr = AX - BX * lam[None, :]
        return np.linalg.norm(Rr, axis=0) / (normA * np.linalg.norm(BX, axis=0)), Rr

    # step 3: B-orthonormalise X, then AX = A X
    try:
        X, BX = b_orthonormalize(X0, Bop(X0))
    except CholeskyFailure:
        return Result(status=ERR_CHOL, lam=None, X=None, hist=np.zeros((0, m)), iters=0, resid=None)
    AX = apply_A(X)
    # step 4: initial Ritz vectors from X^T A X
    H = X.T @ AX
    lam, Z = np.linalg.eigh(0.5 * (H + H.T))
    X, AX, BX = X @ Z, AX @ Z, BX @ Z
    # step 5
    J = np.arange(m)
    P = AP = BP = None
    hist, status, k = [], NOT_CONVERGED, 0
    nw = m if nwant is None else int(nwant)
    for k in range(maxit):                                     # step 6
        rho, Rr = rho_of(X, AX, BX, lam)                       # step 7 (all columns)
        hist.append(rho)
        if not np.all(np.isfinite(rho)):
            status = ERR_NONFINITE
            break
        if nw < m and np.all(rho[:nw] <= tol):                 # the wanted pairs have converged
            status = OK
            break
        above = rho[J] > tol                                   # step 8
        if lock_gap > 0.0:
            U = J[above]
            for i, j in enumerate(J):
                if not above[i] and np.any(np.abs(lam[U] - lam[j]) <= lock_gap * np.abs(lam[U])):
                    above[i] = True
        J = J[above]
        if J.size == 0 and reactivate:
            J = np.flatnonzero(rho > tol)
        if callback is not None:
            callback(k, lam, rho, J)
        if J.size == 0:
            status = OK
            break
        W = T(np.asfortranarray(Rr[:, J]))                     # step 9
        if constrain is not None:                              # step 10
            W = np.asfortranarray(constrain(W))
        try:                                                   # step 11
            W, BW = b_orthonormalize(W, Bop(W))
        except CholeskyFailure:
            status = ERR_CHOL
            break
        AW = apply_A(W)                                        # step 12
        use_p = False
        if P is not None:                                      # steps 13-16
            try:
                PJ, BPJ, APJ = b_orthonormalize(P[:, J], BP[:, J], AP[:, J])
                use_p = True
            except CholeskyFailure:
                use_p = False
        C = None
        if explicit_gram:
            gXX, gXA, gWW = X.T @ BX, X.T @ AX, W.T @ BW
            gPP = PJ.T @ BPJ if use_p else None
        else:
            gXX, gXA, gWW = np.eye(m), np.diag(lam), np.eye(J.size)
            gPP = np.eye(J.size)
        for with_p in ([True, False] if use_p else [False]):
            if with_p:                                         # steps 18-19
                gramA = np.block([[gXA, X.T @ AW, X.T @ APJ],
                                  [AW.T @ X, W.T @ AW, W.T @ APJ],
                                  [APJ.T @ X, APJ.T @ W, PJ.T @ APJ]])
                gramB = np.block([[gXX, X.T @ BW, X.T @ BPJ],
                                  [BW.T @ X, gWW, W.T @ BPJ],
                                  [BPJ.T @ X, BPJ.T @ W, gPP]])
            else:                                              # steps 21-22
                gramA = np.block([[gXA, X.T @ AW], [AW.T @ X, W.T @ AW]])
                gramB = np.block([[gXX, X.T @ BW], [BW.T @ X, gWW]])
            # the lower blocks are the transposes of the upper ones
            gramA = np.triu(gramA) + np.triu(gramA, 1).T
            gramB = np.triu(gramB) + np.triu(gramB, 1).T
            try:
                theta, C = rayleigh_ritz(gramA, gramB, m)      # step 24
                use_p = with_p
                break
            except np.linalg.LinAlgError:
                C = None
        if C is None:
            status = ERR_RR
            break
        j = J.size
        CX, CW = C[:m], C[m:m + j]
        if use_p:                                              # steps 26-28
            CP = C[m + j:]
            P = W @ CW + PJ @ CP
            AP = AW @ CW + APJ @ CP
            BP = BW @ CW + BPJ @ CP
        else:                                                  # steps 30-32
            P = W @ CW
            AP = AW @ CW
            BP = BW @ CW
        X = X @ CX + P
        AX = AX @ CX + AP
        BX = BX @ CX + BP
        lam = theta
    else:
        k = maxit
    iters = len(hist)
    # explicit final residuals with a fresh A X and B X
    resid, _ = rho_of(X, apply_A(X), Bop(X), lam)
    return Result(status=status, lam=lam, X=X, hist=np.array(hist).reshape(-1, m), iters=iters,
                  resid=resid, J=J)


def laplace7_solver(dims, m, X0, tol, maxit, levels=None, nu_pre=2, nu_post=2, coarse_sweeps=20,
                    omega=2.0 / 3.0, callback=None, Y=None, bdiag=None, explicit_gram=False, bmass=None,
                    lock_gap=0.0, nwant=None):
    """LOBPCG on the 7-point Laplacian with optional V-cycle preconditioning,
    constraints Y and B = diag(bdiag) (a lumped mass) or B = the 7-point
    mass-type operator with coefficients bmass = (b0, b1)."""
    from . import grid, mg
    A = lambda V: grid.laplace7(dims, V)
    T = None
    if levels:
        T = mg.VCycle(dims, levels, nu_pre, nu_post, coarse_sweeps, omega)
    Bop = None
    if bdiag is not None:
        d = np.asarray(bdiag, dtype=np.float64).reshape(-1)
        Bop = lambda V: d[:, None] * V
    elif bmass is not None:
        b0, b1 = bmass
        Bop = lambda V: grid.mass7(dims, b0, b1, V)
    return lobpcg(A, X0, tol, maxit, grid.gershgorin_laplace7(), apply_T=T, callback=callback, Y=Y, apply_B=Bop,
                  explicit_gram=explicit_gram, lock_gap=lock_gap, nwant=nwant)


def varcoef_solver(dims, kx, ky, kz, m, X0, tol, maxit, levels=None, callback=None):
    """LOBPCG on -div(k grad u), preconditioned by the constant-coefficient V-cycle."""
    from . import grid, mg
    A = lambda V: grid.varcoef7(dims, kx, ky, kz, V)
    T = mg.VCycle(dims, levels) if levels else None
    return lobpcg(A, X0, tol, maxit, grid.gershgorin_varcoef7(dims, kx, ky, kz), apply_T=T,
                  callback=callback)
