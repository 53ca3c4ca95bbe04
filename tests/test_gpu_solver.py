"""Whole-solver parity on the GPU (through the C ABI) against the FP64 CPU
oracle, the closed-form spectrum (Section 4.1) and the invariants of the
method, for the FP64 and the mixed-precision forms, the variable-coefficient
operator and the eigenvalue adjoint.

Eigenvalues are unique and compared one by one.  Eigenvectors are compared
where the eigenvalue is simple (up to sign); vectors of degenerate groups are
checked by their residuals only.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import closed_form, grid
from oracle import lobpcg as olob

L = pytest.importorskip("paper_0705_2626_amd")
pytestmark = pytest.mark.gpu

DEV = "cuda"


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def solve(dims, m, levels, prec, tol, maxit, seed=2, A=None):
    N = int(np.prod(dims))
    X0 = synth.x0_uniform(N, m, seed=seed)
    ctx = L.lobpcg_setup(A or L.Op(*dims), L.Precond(levels), m, prec)
    r = L.lobpcg_solve(ctx, dev(X0), tol, maxit)
    return ctx, r, X0


def active_sets(hist, tol):
    """The active set J of every iteration, replayed from a residual history
    with the soft-locking rule both implementations follow: J keeps the
    columns above tol; if it empties while some column is above tol again,
    those columns are active again."""
    J, out = np.arange(hist.shape[1]), []
    for rho in hist:
        J = J[rho[J] > tol]
        if J.size == 0:
            J = np.flatnonzero(rho > tol)
        out.append(tuple(J.tolist()))
    return out


def group_histories(hist, groups):
    """Per group of equal eigenvalues, the root sum of squares of its columns'
    residual norms: unlike a single column's norm, it does not depend on how
    the group's Ritz vectors are rotated within the group."""
    return np.stack([np.sqrt((hist[:, g] ** 2).sum(axis=1)) for g in groups], axis=1)


def test_fp64_unpreconditioned_n16_matches_oracle():
    """Plain FP64 LOBPCG, n=16, m=4, no preconditioner, tol 1e-8.

    lambda_2..4 is a triple eigenvalue.  Within such a group the Ritz vectors
    are fixed only up to a rotation, which rounding chooses: the oracle run
    from X0 perturbed by 1e-15 (relative) splits the group's residual among
    its three columns differently after about 40 iterations, while the
    group's root sum of squares stays within 1e-8.  So the histories are
    compared per group (the simple lambda_1 alone, the triple by its root
    sum of squares) at 1e-6 relative, up to the first iteration at which the
    active sets differ (a column of the group crossing tol in one run and
    not the other).  After that iteration the runs take different steps;
    the iteration counts must then agree within 2 plus the oracle's own
    spread over rounding-level perturbations of X0."""
    dims, m, tol = (16, 16, 16), 4, 1e-8
    ctx, r, X0 = solve(dims, m, None, L.FP64, tol, 500)
    ref = olob.laplace7_solver(dims, m, X0, tol, 500)
    exact, _ = closed_form.smallest(*dims, m)
    assert r.status == L.OK and ref.status == olob.OK
    np.testing.assert_allclose(r.lam, exact, rtol=1e-10)
    # two runs that each stop at rho <= tol (possibly one iteration apart)
    # agree to the accuracy that tolerance buys: relative 1e-10 in FP64
    np.testing.assert_allclose(r.lam, ref.lam, rtol=1e-10)
    assert r.resid.max() <= tol
    Jg, Jo = active_sets(r.hist, tol), active_sets(ref.hist, tol)
    k = min(len(Jg), len(Jo))
    kd = next((i for i in range(k) if Jg[i] != Jo[i]), None)
    upto = k if kd is None else kd + 1      # the histories of iteration kd still agree
    groups = [[0], [1, 2, 3]]
    np.testing.assert_allclose(group_histories(r.hist[:upto], groups), group_histories(ref.hist[:upto], groups),
                               rtol=1e-6, atol=1e-14)
    if kd is None:
        assert abs(r.iters - ref.iters) <= 2, (r.iters, ref.iters)
    else:
        rng = np.random.default_rng(11)
        counts = [olob.laplace7_solver(dims, m, X0 * (1 + 1e-15 * rng.standard_normal(X0.shape)), tol, 500).iters
                  for _ in range(3)]
        lo, hi = min(counts + [ref.iters]), max(counts + [ref.iters])
        assert lo - 2 <= r.iters <= hi + 2, (r.iters, ref.iters, counts, kd)


def test_cluster_locking_matches_oracle():
    """Soft locking by clusters (LOBPCG_OPT_LOCK_GAP) against the oracle's
    lock_gap on 16^3 without preconditioner: the same active sets (the triple
    lambda_2..4 leaves J in one iteration), histories per group at 1e-6 up
    to the first lock (a locked column's residual is no longer reduced by
    the iteration and drifts with rounding: the oracle run from X0 perturbed
    by 1e-15 departs from its own history by 1e-6 some 30 iterations after
    the first lock), eigenvalues at 1e-10."""
    dims, m, tol, gap = (16, 16, 16), 4, 1e-8, 1e-3
    N = 4096
    X0 = synth.x0_uniform(N, m, seed=2)
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(None), m, L.FP64)
    L.lobpcg_set_option(ctx, L.OPT_LOCK_GAP, gap)
    r = L.lobpcg_solve(ctx, dev(X0), tol, 500)
    ref = olob.laplace7_solver(dims, m, X0, tol, 500, lock_gap=gap)
    exact, _ = closed_form.smallest(*dims, m)
    assert r.status == L.OK and ref.status == olob.OK
    np.testing.assert_allclose(r.lam, exact, rtol=1e-10)
    np.testing.assert_allclose(r.lam, ref.lam, rtol=1e-10)
    assert r.resid.max() <= tol

    def sets(hist):
        J, out = np.arange(m), []
        for rho in hist:
            above = rho[J] > tol
            for i, j in enumerate(J):
                if not above[i] and np.any(rho[J] > tol):
                    # the replay has no Ritz values: a converged column of the
                    # triple stays while another column of the triple is above
                    above[i] = j in (1, 2, 3) and np.any(rho[[a for a in J if a in (1, 2, 3)]] > tol)
            J = J[above]
            out.append(tuple(J.tolist()))
        return out
    Jg, Jo = sets(r.hist), sets(ref.hist)
    k = min(len(Jg), len(Jo))
    first_lock = next(i for i in range(k) if len(Jg[i]) < m or len(Jo[i]) < m)
    groups = [[0], [1, 2, 3]]
    np.testing.assert_allclose(group_histories(r.hist[:first_lock + 1], groups),
                               group_histories(ref.hist[:first_lock + 1], groups), rtol=1e-6, atol=1e-14)
    # the triple leaves J together in both runs
    for Js in (Jg, Jo):
        assert len({next(i for i, J in enumerate(Js) if j not in J) for j in (1, 2, 3)}) == 1
    assert abs(r.iters - ref.iters) <= 2, (r.iters, ref.iters)


@pytest.mark.parametrize("dims,m,levels", [((24, 20, 16), 6, 3), ((32, 32, 32), 8, 3), ((33, 31, 30), 10, 4)])
def test_fp64_multigrid_matches_oracle(dims, m, levels):
    tol = 1e-9
    ctx, r, X0 = solve(dims, m, levels, L.FP64, tol, 200)
    ref = olob.laplace7_solver(dims, m, X0, tol, 200, levels=levels)
    exact, _ = closed_form.smallest(*dims, m)
    assert r.status == L.OK and ref.status == olob.OK
    # |dlambda| <= (rho ||A||)^2 / gap: 5e-9 relative covers the closely
    # clustered non-cubic spectra at rho = 1e-9 (gaps down to 2e-4)
    np.testing.assert_allclose(r.lam, exact, rtol=5e-9)
    np.testing.assert_allclose(ref.lam, exact, rtol=5e-9)
    np.testing.assert_allclose(r.lam, ref.lam, rtol=5e-9)
    assert r.resid.max() <= tol
    assert abs(r.iters - ref.iters) <= 1, (r.iters, ref.iters)
    k = min(8, r.iters)
    np.testing.assert_allclose(r.hist[:k], ref.hist[:k], rtol=1e-6)


def test_fp64_eigenvectors_match_sine_modes():
    dims, m = (24, 20, 16), 6
    ctx, r, _ = solve(dims, m, 3, L.FP64, 1e-10, 200)
    lam, ijk = closed_form.smallest(*dims, m)
    X = r.X.cpu().numpy()
    for i in range(m):
        v = closed_form.mode(*dims, *ijk[i])
        c = abs(v @ X[:, i]) / (np.linalg.norm(v) * np.linalg.norm(X[:, i]))
        assert 1 - c < 1e-12
    # orthonormal
    np.testing.assert_allclose(X.T @ X, np.eye(m), atol=1e-12)


def test_mixed_precision_reaches_fp64_accuracy():
    dims, m, levels, tol = (32, 32, 32), 8, 3, 1e-8
    ctx, r, X0 = solve(dims, m, levels, L.MIXED, tol, 200)
    st = L.lobpcg_get_stats(ctx)
    ref = olob.laplace7_solver(dims, m, X0, tol, 200, levels=levels)
    assert r.status == L.OK
    assert st["iters_fp32"] > 0 and st["iters_fp64"] > 0
    np.testing.assert_allclose(r.lam, ref.lam, rtol=1e-6)
    exact, _ = closed_form.smallest(*dims, m)
    np.testing.assert_allclose(r.lam, exact, rtol=1e-6)
    assert r.resid.max() <= tol


@pytest.mark.parametrize("above", [0, 2, 8, 16])
def test_mixed_explicit_gram_threshold(above):
    """The FP32 iterations' Gram form by active count (explicit while more
    than `above` columns are active, the paper's form after; 0: always
    explicit, 16 = m: never): every setting reaches the FP64 eigenpairs of
    the closed form and every explicit residual <= tol.  Out-of-range values
    are rejected."""
    dims, m, levels, tol = (32, 30, 28), 16, 3, 1e-8
    N = int(np.prod(dims))
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(levels), m, L.MIXED)
    L.lobpcg_set_option(ctx, L.OPT_FP32_EXPLICIT_ABOVE, above)
    r = L.lobpcg_solve(ctx, dev(synth.x0_uniform(N, m, seed=3)), tol, 300)
    st = L.lobpcg_get_stats(ctx)
    exact, _ = closed_form.smallest(*dims, m)
    assert r.status == L.OK and st["iters_fp32"] > 0
    np.testing.assert_allclose(r.lam, exact, rtol=1e-9)
    assert r.resid.max() <= tol
    for v in (-1, m + 1, 2.5):
        with pytest.raises(L.LobpcgError):
            L.lobpcg_set_option(ctx, L.OPT_FP32_EXPLICIT_ABOVE, v)


def test_mixed_precision_non_cubic_degenerate_edge():
    """m=10 on a cube cuts a degenerate eigenvalue group: values still right."""
    dims, m, levels, tol = (16, 16, 16), 10, 3, 1e-8
    ctx, r, X0 = solve(dims, m, levels, L.MIXED, tol, 300)
    exact, _ = closed_form.smallest(*dims, m)
    assert r.status == L.OK
    np.testing.assert_allclose(r.lam, exact, rtol=1e-9)
    assert r.resid.max() <= tol


def test_varcoef_fp64_matches_oracle():
    dims, m, tol = (12, 10, 8), 4, 1e-10
    kx, ky, kz = synth.gaussian_field_faces(*dims, sigma=0.5, corr=4.0, seed=2)
    A = L.Op(*dims, dev(kx), dev(ky), dev(kz))
    ctx, r, X0 = solve(dims, m, 2, L.FP64, tol, 300, A=A)
    ref = olob.varcoef_solver(dims, kx, ky, kz, m, X0, tol, 300, levels=2)
    assert r.status == L.OK and ref.status == olob.OK
    np.testing.assert_allclose(r.lam, ref.lam, rtol=1e-9)
    assert abs(r.iters - ref.iters) <= 1
    # simple eigenvalues: vectors agree up to sign
    X, Xr = r.X.cpu().numpy(), ref.X
    for i in range(m):
        c = abs(X[:, i] @ Xr[:, i]) / (np.linalg.norm(X[:, i]) * np.linalg.norm(Xr[:, i]))
        assert 1 - c < 1e-10


def test_adjoint_on_solver_output_matches_oracle_and_euler_identity():
    dims, m = (16, 14, 12), 5
    kx, ky, kz = synth.gaussian_field_faces(*dims, sigma=0.5, corr=8.0, seed=5)
    A = L.Op(*dims, dev(kx), dev(ky), dev(kz))
    ctx, r, X0 = solve(dims, m, 2, L.FP64, 1e-11, 300, A=A)
    assert r.status == L.OK
    X = r.X.cpu().numpy()
    gbar = np.array([1.0, -0.5, 0.25, 2.0, 0.0])
    got = [t.cpu().numpy() for t in L.lobpcg_eig_grad_k(ctx, r.X, gbar)]
    ref = grid.eig_grad_faces(dims, X, gbar)
    for a, b in zip(got, ref):
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-14 * np.abs(b).max())
    # Euler: sum_f k_f dlambda_i/dk_f = lambda_i
    for i in range(m):
        e = np.zeros(m); e[i] = 1
        g = [t.cpu().numpy() for t in L.lobpcg_eig_grad_k(ctx, r.X, e)]
        s = np.sum(kx * g[0]) + np.sum(ky * g[1]) + np.sum(kz * g[2])
        assert s == pytest.approx(r.lam[i], rel=1e-12)


def test_autograd_directional_finite_difference():
    """d/dt lambda(k + t v) at t=0 by central differences of warm-started GPU
    solves, against the autograd gradient contracted with v."""
    from paper_0705_2626_amd.autograd import eig_smallest
    dims, m = (10, 9, 8), 3
    kx, ky, kz = synth.gaussian_field_faces(*dims, sigma=0.5, corr=4.0, seed=6)
    K = [dev(a).requires_grad_(True) for a in (kx, ky, kz)]
    N = int(np.prod(dims))
    solver = L.lobpcg_setup(L.Op(*dims, *[k.detach() for k in K]), L.Precond(2), m, L.FP64)
    X0 = dev(synth.x0_uniform(N, m))
    lam = eig_smallest(*K, solver, X0, 1e-12, 500)
    w = torch.tensor([1.0, 0.3, -0.7], dtype=torch.float64, device=DEV)
    (lam * w).sum().backward()
    rng = np.random.default_rng(1)
    V = [dev(rng.uniform(-1, 1, a.shape)) for a in (kx, ky, kz)]
    dirderiv = sum(float((k.grad * v).sum()) for k, v in zip(K, V))
    h = 1e-5
    vals = []
    for sgn in (1, -1):
        Kp = [(k.detach() + sgn * h * v) for k, v in zip(K, V)]
        Ap = L.Op(*dims, *Kp)
        r = L.lobpcg_solve(solver, X0, 1e-12, 500, A=Ap)
        assert r.status == L.OK
        vals.append(float(np.dot(r.lam, w.cpu().numpy())))
    fd = (vals[0] - vals[1]) / (2 * h)
    assert fd == pytest.approx(dirderiv, rel=1e-5)


def face_rayleigh_quotients(dims, k, X):
    """lambda_i = sum_f k_f (x_i[p] - x_i[q])^2 / (x_i, x_i), the face-sum
    form of the Rayleigh quotient (a sum of non-negative terms), evaluated on
    the host in extended precision (numpy longdouble), so that its rounding
    stays far below the finite-difference signal."""
    nx, ny, nz = dims
    kx, ky, kz = (np.asarray(a, dtype=np.longdouble) for a in k)
    Xh = X.cpu().numpy().astype(np.longdouble)
    out = []
    for i in range(Xh.shape[1]):
        g = np.zeros((nz + 2, ny + 2, nx + 2), dtype=np.longdouble)
        g[1:-1, 1:-1, 1:-1] = Xh[:, i].reshape(nz, ny, nx)
        e = (np.sum(kx * np.diff(g[1:-1, 1:-1, :], axis=2) ** 2) + np.sum(ky * np.diff(g[1:-1, :, 1:-1], axis=1) ** 2)
             + np.sum(kz * np.diff(g[:, 1:-1, 1:-1], axis=0) ** 2))
        out.append(e / np.sum(Xh[:, i] ** 2))
    return np.array(out)


def test_per_face_finite_differences_through_eig_smallest():
    """The adjoint of EigSmallest against central differences (relative step
    h = 1e-6) of single face coefficients, on 200 seeded faces of a
    12 x 11 x 10 grid (lognormal k), for each of the m = 4 eigenvalues.
    Here one face moves lambda by about lambda / #faces, a difference of
    some 1e6 units in the last place of lambda, so the quotient resolves
    1e-5 (at n = 96 it would not).  lambda(k +- h k_f e_f) is the Rayleigh
    quotient, in extended precision, of a warm-started solve to rho <= 1e-12
    (its error is quadratic in the vector's: about (rho ||A||)^2 / gap).  A face where a mode
    is nearly flat (x_p close to x_q, e.g. across a symmetry plane of the
    mode) has a derivative close to zero; the relative error is taken
    against max(|g_f|, 1e-2 * the median |g| of the sampled faces)."""
    from paper_0705_2626_amd.autograd import EigSmallest

    dims, m, h = (12, 11, 10), 4, 1e-6
    N = int(np.prod(dims))
    kx, ky, kz = synth.gaussian_field_faces(*dims, sigma=0.5, corr=4.0, seed=3)
    shapes = [a.shape for a in (kx, ky, kz)]
    sizes = [a.size for a in (kx, ky, kz)]
    K = [dev(a).requires_grad_(True) for a in (kx, ky, kz)]
    solver = L.lobpcg_setup(L.Op(*dims, *[k.detach() for k in K]), L.Precond(2), m, L.FP64)
    # warm starts from an iterate already at rho ~ 1e-11: with the Cholesky-QR
    # factors folded into the Gram matrices, X^T W R^-1 carries the rounding
    # of X^T W amplified by the condition of R (W is then nearly rank
    # deficient), and on some faces the residuals drift up instead of down;
    # with the factors applied to the blocks (the printed form) they converge
    L.lobpcg_set_option(solver, L.OPT_FOLD_CHOLQR, 0)
    X0 = dev(synth.x0_uniform(N, m, seed=4))
    lam = EigSmallest.apply(*K, solver, X0, 1e-12, 500)
    assert np.all(np.diff(lam.detach().cpu().numpy()) > 1e-4)     # simple eigenvalues
    grads = []
    for i in range(m):
        g = torch.autograd.grad(lam[i], K, retain_graph=True)
        grads.append(np.concatenate([gi.detach().cpu().numpy().ravel() for gi in g]))
    X = L.lobpcg_solve(solver, X0, 1e-12, 500, hist=False).X
    flat = np.concatenate([kx.ravel(), ky.ravel(), kz.ravel()])
    faces = synth.sample_faces(flat.size, 200, seed=5)
    floor = [1e-2 * np.median(np.abs(grads[i][faces])) for i in range(m)]
    worst = 0.0
    for f in faces:
        vals = []
        for sgn in (1.0, -1.0):
            kp = flat.copy()
            kp[f] *= 1.0 + sgn * h
            parts = np.split(kp, np.cumsum(sizes)[:-1])
            Kp = [dev(a.reshape(sh)) for a, sh in zip(parts, shapes)]
            Ap = L.Op(*dims, *Kp)
            r = L.lobpcg_solve(solver, X, 1e-12, 200, A=Ap, hist=False)
            assert r.status == L.OK
            vals.append(face_rayleigh_quotients(dims, [a.reshape(sh) for a, sh in zip(parts, shapes)], r.X))
        fd = np.asarray((vals[0] - vals[1]) / (2.0 * h * flat[f]), dtype=np.float64)
        for i in range(m):
            g = grads[i][f]
            worst = max(worst, abs(fd[i] - g) / max(abs(g), floor[i]))
    print("per-face central differences: largest relative error %.2e" % worst)
    assert worst < 1e-5


def test_error_paths():
    dims, m = (8, 8, 8), 3
    N = 512
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(2), m, L.FP64)
    X0 = synth.x0_uniform(N, m)
    X0[:, 2] = X0[:, 1]
    r = L.lobpcg_solve(ctx, dev(X0), 1e-8, 50, raise_on_error=False)
    assert r.status == L.ERR_CHOL
    X0 = synth.x0_uniform(N, m)
    X0[7, 1] = np.nan
    r = L.lobpcg_solve(ctx, dev(X0), 1e-8, 50, raise_on_error=False)
    assert r.status == L.ERR_NONFINITE
    r = L.lobpcg_solve(ctx, dev(synth.x0_uniform(N, m)), 1e-8, 2)
    assert r.status == L.NOT_CONVERGED and r.iters == 2
    with pytest.raises(L.LobpcgError):
        L.lobpcg_solve(ctx, dev(synth.x0_uniform(N, m)), -1.0, 10)
    for v in (128, -4, 1000):       # out of range
        with pytest.raises(L.LobpcgError):
            L.lobpcg_set_option(ctx, L.OPT_KERNELS, v)


@pytest.mark.parametrize("variant,prec", [(4, L.FP64), (8, L.FP64), (32, L.FP64), (1, L.MIXED), (64, L.MIXED)])
@pytest.mark.parametrize("m", [6, 12])
def test_kernel_variants_give_the_same_solution(variant, prec, m):
    """The default Gram and update kernels and the other variants agree."""
    dims = (20, 18, 16)
    N = int(np.prod(dims))
    X0 = dev(synth.x0_uniform(N, m))
    res = []
    for v in (0, variant):
        ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(3), m, prec)
        L.lobpcg_set_option(ctx, L.OPT_KERNELS, v)
        res.append(L.lobpcg_solve(ctx, X0, 1e-9, 200))
    assert res[0].status == res[1].status == L.OK
    np.testing.assert_allclose(res[0].lam, res[1].lam, rtol=1e-10)
    assert abs(res[0].iters - res[1].iters) <= 1


@pytest.mark.parametrize("prec", [L.FP64, L.MIXED])
def test_folded_and_applied_cholqr_agree(prec):
    """Steps 11 and 14-15 with R^-1 applied to W_J, P_J (as printed) and folded
    into the Gram matrices and coefficients (the default) give the same
    eigenpairs."""
    dims, m, levels = (24, 20, 18), 8, 3
    N = int(np.prod(dims))
    X0 = dev(synth.x0_uniform(N, m))
    res = []
    for fold in (0, 1):
        ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(levels), m, prec)
        L.lobpcg_set_option(ctx, L.OPT_FOLD_CHOLQR, fold)
        res.append(L.lobpcg_solve(ctx, X0, 1e-9, 200))
    exact, _ = closed_form.smallest(*dims, m)
    for r in res:
        assert r.status == L.OK and r.resid.max() <= 1e-9
        np.testing.assert_allclose(r.lam, exact, rtol=5e-9)
    assert abs(res[0].iters - res[1].iters) <= 2


def test_solver_is_deterministic():
    dims, m = (20, 20, 20), 6
    _, r1, _ = solve(dims, m, 3, L.MIXED, 1e-8, 100)
    _, r2, _ = solve(dims, m, 3, L.MIXED, 1e-8, 100)
    assert np.array_equal(r1.lam, r2.lam)
    assert torch.equal(r1.X, r2.X)
    assert r1.iters == r2.iters


def test_soft_locking_reduces_active_work():
    """Columns converge at different rates; the run still ends with every
    explicit residual below tol."""
    dims, m = (16, 16, 16), 8
    ctx, r, _ = solve(dims, m, 3, L.FP64, 1e-9, 200)
    assert r.status == L.OK and r.resid.max() <= 1e-9
    H = r.hist
    # some column dropped below tol before the last iteration
    first_below = [int(np.argmax(H[:, j] <= 1e-9)) if np.any(H[:, j] <= 1e-9) else H.shape[0] for j in range(m)]
    assert min(first_below) < H.shape[0] - 1


def test_soft_lock_demo_m10_matches_oracle():
    """Section 2.3's demonstration: m=10, stopping at residual norm 1e-1
    (rho = 1e-1 / ||A||, ||A|| = 12): the GPU's residual history follows the
    oracle's, and every column that is soft-locked before the end still
    improves while the others converge."""
    dims, m = (16, 16, 16), 10
    tol = 1e-1 / 12.0
    ctx, r, X0 = solve(dims, m, None, L.FP64, tol, 200)
    ref = olob.laplace7_solver(dims, m, X0, tol, 200)
    assert r.status == L.OK and ref.status == olob.OK
    assert r.iters == ref.iters
    np.testing.assert_allclose(r.hist, ref.hist[:r.iters], rtol=1e-6)
    H = r.hist
    locked = [j for j in range(m) if H[-1, j] <= tol and np.argmax(H[:, j] <= tol) < H.shape[0] - 1]
    assert len(locked) >= 2
    for j in locked:
        k = int(np.argmax(H[:, j] <= tol))
        assert H[-1, j] <= H[k, j]


# ---------------------------------------------------------------- blocks wider than 32 columns

def test_wide_block_fp64_matches_oracle():
    """m=36: the Gram products in several launches, the block updates through
    the wide kernel (inputs in 32-column pieces, outputs in column chunks)."""
    dims, m, levels, tol = (18, 17, 16), 36, 3, 1e-8
    ctx, r, X0 = solve(dims, m, levels, L.FP64, tol, 200)
    ref = olob.laplace7_solver(dims, m, X0, tol, 200, levels=levels)
    exact, _ = closed_form.smallest(*dims, m)
    assert r.status == L.OK and ref.status == olob.OK
    # |dlambda| <= (rho ||A||)^2 / gap with gap >= 0.03 to lambda_37
    np.testing.assert_allclose(r.lam, exact, rtol=1e-9)
    np.testing.assert_allclose(r.lam, ref.lam, rtol=1e-9)
    assert r.resid.max() <= tol
    assert abs(r.iters - ref.iters) <= 1, (r.iters, ref.iters)
    k = min(8, r.iters)
    np.testing.assert_allclose(r.hist[:k], ref.hist[:k], rtol=1e-6)
    X = r.X.cpu().numpy()
    np.testing.assert_allclose(X.T @ X, np.eye(m), atol=1e-10)


def test_wide_block_mixed_reaches_fp64_accuracy():
    dims, m, levels, tol = (24, 24, 24), 50, 3, 1e-8
    ctx, r, X0 = solve(dims, m, levels, L.MIXED, tol, 300)
    st = L.lobpcg_get_stats(ctx)
    exact, _ = closed_form.smallest(*dims, m)
    assert r.status == L.OK
    assert st["iters_fp32"] > 0 and st["iters_fp64"] > 0
    np.testing.assert_allclose(r.lam, exact, rtol=1e-6)
    assert r.resid.max() <= tol


def test_explicit_gram_fp64_matches_oracle():
    """The variant of Section 2.2 with the block diagonal of gramB (and X^T AX)
    computed: m=40 on 20 x 18 x 16 to rho 1e-9, a run on which the paper's
    form loses orthogonality after about 45 iterations (a spurious Ritz value
    below lambda_1 appears) while the explicit form converges."""
    dims, m, levels, tol = (20, 18, 16), 40, 3, 1e-9
    N = int(np.prod(dims))
    X0 = synth.x0_uniform(N, m, seed=2)
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(levels), m, L.FP64)
    L.lobpcg_set_option(ctx, L.OPT_FP64_EXPLICIT_GRAM, 1)
    r = L.lobpcg_solve(ctx, dev(X0), tol, 200)
    ref = olob.laplace7_solver(dims, m, X0, tol, 200, levels=levels, explicit_gram=True)
    exact, _ = closed_form.smallest(*dims, m)
    assert r.status == L.OK and ref.status == olob.OK
    np.testing.assert_allclose(r.lam, exact, rtol=1e-10)
    np.testing.assert_allclose(r.lam, ref.lam, rtol=1e-10)
    assert r.resid.max() <= tol
    assert abs(r.iters - ref.iters) <= 1, (r.iters, ref.iters)
    assert active_sets(r.hist, tol) == active_sets(ref.hist, tol)
    # the histories agree at 1e-6 over the first 8 iterations; later the
    # columns of the close pair lambda_39, lambda_40 (relative gap 1.8e-3),
    # whose split between the two Ritz vectors is ill-determined until they
    # converge, amplify rounding differences steadily (the oracle's own runs
    # from X0 perturbed by 1e-15 drift the same way, from 7e-8 at iteration
    # 8 to 1.3e-6 at iteration 16)
    k = min(8, r.iters)
    np.testing.assert_allclose(r.hist[:k], ref.hist[:k], rtol=1e-6, atol=1e-14)


@pytest.mark.parametrize("prec", [L.FP64, L.MIXED])
def test_wanted_pairs_with_guard_columns_match_oracle(prec):
    """A block of 7 columns for 4 wanted pairs (LOBPCG_OPT_NWANT): the solve
    ends when the first 4 have converged, as the oracle's run with nwant = 4
    does (same iteration count in FP64; eigenvalues and residuals of the
    wanted pairs against the oracle and the closed form).  nwant out of
    range is rejected."""
    dims, m, nw, levels, tol = (12, 11, 10), 7, 4, 2, 1e-9
    N = int(np.prod(dims))
    X0 = synth.x0_uniform(N, m, seed=5)
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(levels), m, prec)
    L.lobpcg_set_option(ctx, L.OPT_NWANT, nw)
    r = L.lobpcg_solve(ctx, dev(X0), tol, 500)
    ref = olob.laplace7_solver(dims, m, X0, tol, 500, levels=levels, nwant=nw)
    exact, _ = closed_form.smallest(*dims, m)
    assert r.status == L.OK and ref.status == olob.OK
    assert r.resid[:nw].max() <= tol
    np.testing.assert_allclose(r.lam[:nw], exact[:nw], rtol=1e-10)
    np.testing.assert_allclose(r.lam[:nw], ref.lam[:nw], rtol=1e-10)
    if prec == L.FP64:
        assert r.iters == ref.iters
        assert active_sets(r.hist, tol) == active_sets(ref.hist, tol)
        np.testing.assert_allclose(r.hist, ref.hist, rtol=1e-6, atol=1e-14)
    ctx_all = L.lobpcg_setup(L.Op(*dims), L.Precond(levels), m, prec)
    full = L.lobpcg_solve(ctx_all, dev(X0), tol, 500)
    assert r.iters < full.iters
    for v in (-1, m + 1, 2.5):
        with pytest.raises(L.LobpcgError):
            L.lobpcg_set_option(ctx, L.OPT_NWANT, v)


def test_block_of_98_fp64():
    """The widest block of the paper's block-size study (m = 98) on a 16^3
    grid: a Rayleigh-Ritz basis of 294 vectors."""
    dims, m, levels, tol = (16, 16, 16), 98, 3, 1e-8
    ctx, r, X0 = solve(dims, m, levels, L.FP64, tol, 300)
    exact, _ = closed_form.smallest(*dims, m)
    assert r.status == L.OK
    assert r.resid.max() <= tol
    # |dlambda| <= (rho ||A||)^2 / gap, gaps >= 1e-3 here
    np.testing.assert_allclose(r.lam, exact, rtol=1e-10, atol=2e-11)
    X = r.X.cpu().numpy()
    np.testing.assert_allclose(X.T @ X, np.eye(m), atol=1e-10)


def test_hundred_constraints_give_the_next_eigenpairs():
    """Y = the 100 lowest sine modes of a 12 x 10 x 8 grid (more columns than
    one Gram launch takes): the solve returns lambda_101..104."""
    dims, ny, m, tol = (12, 10, 8), 100, 4, 1e-9
    N = int(np.prod(dims))
    lam, ijk = closed_form.smallest(*dims, ny + m + 1)
    assert lam[ny] - lam[ny - 1] > 1e-3 and lam[ny + m] - lam[ny + m - 1] > 1e-3
    Y = sine_block(dims, ijk[:ny])
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(2), m, L.FP64)
    r = L.lobpcg_solve(ctx, dev(synth.x0_uniform(N, m, seed=3)), tol, 300, Y=dev(Y))
    assert r.status == L.OK
    np.testing.assert_allclose(r.lam, lam[ny:ny + m], rtol=1e-9)
    assert np.abs(Y.T @ r.X.cpu().numpy()).max() < 1e-10


def test_one_column_with_sixty_four_constraints():
    """m = 1 with 64 constraint vectors: the projection's (1 + 64) x 1
    coefficients exceed 3 m^2 entries, the size of an update's coefficient
    slot (regression test for the slot size), and the 64-column Y takes the
    general (wide) block product."""
    dims, ny, m, tol = (12, 10, 8), 64, 1, 1e-9
    N = int(np.prod(dims))
    lam, ijk = closed_form.smallest(*dims, ny + m + 1)
    assert lam[ny] - lam[ny - 1] > 5e-3 and lam[ny + 1] - lam[ny] > 5e-3
    Y = sine_block(dims, ijk[:ny])
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(2), m, L.FP64)
    # a single vector converging to lambda_65 (relative gap 6e-3 to
    # lambda_66) takes some hundreds of iterations, in the oracle too
    for seed in (3, 4):     # twice on one context: the ring slots are reused
        X0 = synth.x0_uniform(N, m, seed=seed)
        r = L.lobpcg_solve(ctx, dev(X0), tol, 1000, Y=dev(Y))
        ref = olob.laplace7_solver(dims, m, X0, tol, 1000, levels=2, Y=Y)
        assert r.status == L.OK and ref.status == olob.OK
        np.testing.assert_allclose(r.lam, lam[ny:ny + m], rtol=1e-9)
        np.testing.assert_allclose(r.lam, ref.lam, rtol=1e-9)
        assert r.resid.max() <= tol
        assert np.abs(Y.T @ r.X.cpu().numpy()).max() < 1e-10


# ---------------------------------------------------------------- constraints Y (steps 2 and 10)

def sine_block(dims, ijk):
    V = np.stack([closed_form.mode(*dims, *t) for t in ijk], axis=1)
    return V / np.linalg.norm(V, axis=0)


@pytest.mark.parametrize("mix", [False, True])
def test_constraints_match_oracle(mix):
    """Y = the exact eigenvectors of the 6 smallest eigenvalues (or a random,
    non-orthonormal basis of their span): GPU and oracle find eigenvalues
    7..12, with vectors orthogonal to Y."""
    dims, m, levels, tol = (24, 20, 16), 6, 3, 1e-9
    N = int(np.prod(dims))
    lam, ijk = closed_form.smallest(*dims, 2 * m)
    Y = sine_block(dims, ijk[:m])
    if mix:
        Y = Y @ np.random.default_rng(7).standard_normal((m, m))
    X0 = synth.x0_uniform(N, m, seed=5)
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(levels), m, L.FP64)
    r = L.lobpcg_solve(ctx, dev(X0), tol, 200, Y=dev(Y))
    ref = olob.laplace7_solver(dims, m, X0, tol, 200, levels=levels, Y=Y)
    assert r.status == L.OK and ref.status == olob.OK
    np.testing.assert_allclose(r.lam, lam[m:], rtol=5e-9)
    np.testing.assert_allclose(r.lam, ref.lam, rtol=5e-9)
    assert r.resid.max() <= tol
    assert np.abs(Y.T @ r.X.cpu().numpy()).max() < 1e-8 * np.abs(Y).max() * np.sqrt(N)
    assert abs(r.iters - ref.iters) <= 2, (r.iters, ref.iters)


@pytest.mark.parametrize("mix", [False, True])
def test_constraints_in_mixed_precision(mix):
    """Constraints in the mixed solver: Y = the exact eigenvectors of the 6
    smallest eigenvalues (or a random basis of their span); eigenvalues 7..12
    within 1e-6 of the FP64 oracle's and of the closed form, every explicit
    FP64 residual <= tol, X orthogonal to Y."""
    dims, m, levels, tol = (24, 20, 16), 6, 3, 1e-8
    N = int(np.prod(dims))
    lam, ijk = closed_form.smallest(*dims, 2 * m)
    Y = sine_block(dims, ijk[:m])
    if mix:
        Y = Y @ np.random.default_rng(7).standard_normal((m, m))
    X0 = synth.x0_uniform(N, m, seed=5)
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(levels), m, L.MIXED)
    r = L.lobpcg_solve(ctx, dev(X0), tol, 300, Y=dev(Y))
    st = L.lobpcg_get_stats(ctx)
    ref = olob.laplace7_solver(dims, m, X0, tol, 300, levels=levels, Y=Y)
    assert r.status == L.OK and ref.status == olob.OK
    assert st["iters_fp32"] > 0 and st["iters_fp64"] > 0
    np.testing.assert_allclose(r.lam, ref.lam, rtol=1e-6)
    np.testing.assert_allclose(r.lam, lam[m:], rtol=1e-6)
    assert r.resid.max() <= tol
    assert np.abs(Y.T @ r.X.cpu().numpy()).max() < 1e-10 * np.abs(Y).max() * np.sqrt(N)


def test_constraints_repeated_calls_give_successive_eigenpairs():
    """Hard locking as intended: each call appends its converged vectors to Y
    and the next call finds the next block of the spectrum."""
    dims, m, tol = (20, 18, 16), 4, 1e-10
    N = int(np.prod(dims))
    lam, _ = closed_form.smallest(*dims, 3 * m)
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(3), m, L.FP64)
    Y = None
    found = []
    for call in range(3):
        r = L.lobpcg_solve(ctx, dev(synth.x0_uniform(N, m, seed=20 + call)), tol, 300, Y=Y)
        assert r.status == L.OK
        found.append(r.lam)
        Y = r.X.clone() if Y is None else torch.cat([Y, r.X], dim=1).contiguous()
    np.testing.assert_allclose(np.concatenate(found), lam, rtol=1e-9)
    G = (Y.T @ Y).cpu().numpy()
    np.testing.assert_allclose(G, np.eye(3 * m), atol=1e-9)


def test_constraints_error_paths():
    dims, m = (12, 10, 8), 3
    N = int(np.prod(dims))
    X0 = dev(synth.x0_uniform(N, m))
    Y = synth.random_block(N, 2, seed=1)
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(None), m, L.FP64)
    r = L.lobpcg_solve(ctx, X0, 1e-8, 10, Y=dev(np.hstack([Y, Y[:, :1]])), raise_on_error=False)
    assert r.status == L.ERR_ARG          # rank-deficient constraints
    r = L.lobpcg_solve(ctx, X0, 1e-8, 10, Y=dev(synth.random_block(N, 129, seed=2)), raise_on_error=False)
    assert r.status == L.ERR_ARG          # more than 128 constraint vectors


# ---------------------------------------------------------------- B != I (a positive diagonal)

def lumped_mass(N, seed):
    return np.random.default_rng(seed).uniform(0.5, 2.0, N)


def test_diagonal_B_matches_oracle():
    """A x = lambda B x with a seeded lumped-mass-like B = diag(d): GPU and
    oracle agree, X is B-orthonormal, every explicit residual <= tol."""
    dims, m, levels, tol = (20, 18, 16), 6, 3, 1e-9
    N = int(np.prod(dims))
    d = lumped_mass(N, 21)
    X0 = synth.x0_uniform(N, m, seed=8)
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(levels), m, L.FP64, B=L.Diag(*dims, dev(d)))
    r = L.lobpcg_solve(ctx, dev(X0), tol, 300)
    ref = olob.laplace7_solver(dims, m, X0, tol, 300, levels=levels, bdiag=d)
    assert r.status == L.OK and ref.status == olob.OK
    np.testing.assert_allclose(r.lam, ref.lam, rtol=5e-9)
    assert r.resid.max() <= tol
    X = r.X.cpu().numpy()
    np.testing.assert_allclose(X.T @ (d[:, None] * X), np.eye(m), atol=1e-10)
    assert abs(r.iters - ref.iters) <= 2, (r.iters, ref.iters)


def test_scalar_B_scales_the_closed_form():
    dims, m, c = (24, 20, 16), 6, 2.5
    N = int(np.prod(dims))
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(3), m, L.FP64, B=L.Diag(*dims, dev(np.full(N, c))))
    r = L.lobpcg_solve(ctx, dev(synth.x0_uniform(N, m)), 1e-10, 300)
    exact, _ = closed_form.smallest(*dims, m)
    assert r.status == L.OK
    np.testing.assert_allclose(r.lam, exact / c, rtol=1e-9)


def test_B_adjoint_matches_oracle():
    """The eigenvalue adjoint for A(k) x = lambda B x with a diagonal B: the
    face gradients (x_p - x_q)^2 / (x, B x) of the solved (B-orthonormal)
    eigenvectors match the oracle's element by element, also through
    EigSmallest, and satisfy Euler's identity sum_f k_f d lambda_i / d k_f =
    lambda_i (A is linear in k, B does not depend on it)."""
    from paper_0705_2626_amd.autograd import EigSmallest

    dims, m, tol = (12, 10, 8), 3, 1e-11
    N = int(np.prod(dims))
    kx, ky, kz = synth.gaussian_field_faces(*dims, sigma=0.5, corr=4.0, seed=2)
    d = lumped_mass(N, 19)
    K = [dev(a).requires_grad_(True) for a in (kx, ky, kz)]
    ctx = L.lobpcg_setup(L.Op(*dims, *[k.detach() for k in K]), L.Precond(2), m, L.FP64,
                         B=L.Diag(*dims, dev(d)))
    X0 = dev(synth.x0_uniform(N, m, seed=4))
    lam = EigSmallest.apply(*K, ctx, X0, tol, 500)
    r = L.lobpcg_solve(ctx, X0, tol, 500, hist=False)
    assert r.status == L.OK
    X = r.X.cpu().numpy()
    gbar = np.array([0.7, -1.3, 0.4])
    got = [g.cpu().numpy() for g in L.lobpcg_eig_grad_k(ctx, r.X, gbar)]
    ref = grid.eig_grad_faces_B(dims, X, gbar, d[:, None] * X)
    for a, b in zip(got, ref):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-13 * np.abs(b).max())
    euler = sum(np.sum(k * g) for k, g in zip((kx, ky, kz), got))
    assert euler == pytest.approx(float(gbar @ r.lam), rel=1e-9)
    auto = torch.autograd.grad(lam @ torch.tensor(gbar, device=lam.device), K)
    for a, b in zip(auto, ref):
        np.testing.assert_allclose(a.cpu().numpy(), b, rtol=0, atol=1e-9 * np.abs(b).max())


@pytest.mark.parametrize("prec", [L.FP64, L.MIXED])
@pytest.mark.parametrize("kind", ["diag", "mass7"])
def test_B_applied_and_folded_cholqr_agree(kind, prec):
    """With B, steps 11 and 14-15 as printed (R^-1 of W_J^T B W_J and
    P_J^T B P_J applied to W_J, B W_J, P_J, A P_J and B P_J) and folded (the
    default) give the oracle's eigenpairs, with X B-orthonormal and every
    explicit residual <= tol; with the mass-type B also under constraints
    (Y = the 3 smallest sine modes, B-eigenvectors: the next closed-form
    pairs)."""
    dims, m, levels, tol = (20, 18, 16), 6, 3, 1e-9 if prec == L.FP64 else 1e-8
    N = int(np.prod(dims))
    X0 = synth.x0_uniform(N, m, seed=8)
    if kind == "diag":
        d = lumped_mass(N, 21)
        Bd, kw, Bapply = L.Diag(*dims, dev(d)), {"bdiag": d}, (lambda V: d[:, None] * V)
    else:
        b0, b1 = 0.6, 1.0 / 12.0
        Bd, kw, Bapply = L.Mass7(*dims, b0, b1), {"bmass": (b0, b1)}, (lambda V: grid.mass7(dims, b0, b1, V))
    ref = olob.laplace7_solver(dims, m, X0, tol, 300, levels=levels, **kw)
    assert ref.status == olob.OK
    rt = 5e-9 if prec == L.FP64 else 1e-6
    iters = []
    for fold in (0, 1):
        ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(levels), m, prec, B=Bd)
        L.lobpcg_set_option(ctx, L.OPT_FOLD_CHOLQR, fold)
        r = L.lobpcg_solve(ctx, dev(X0), tol, 300)
        assert r.status == L.OK and r.resid.max() <= tol
        np.testing.assert_allclose(r.lam, ref.lam, rtol=rt)
        X = r.X.cpu().numpy()
        np.testing.assert_allclose(X.T @ Bapply(X), np.eye(m), atol=1e-10)
        iters.append(r.iters)
    if prec == L.FP64:
        assert abs(iters[0] - iters[1]) <= 2, iters
    if kind == "mass7":
        mu, ijk = closed_form.smallest(*dims, m + 3)
        Y = sine_block(dims, ijk[:3])
        ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(levels), m, prec, B=Bd)
        L.lobpcg_set_option(ctx, L.OPT_FOLD_CHOLQR, 0)
        r = L.lobpcg_solve(ctx, dev(synth.x0_uniform(N, m, seed=9)), tol, 300, Y=dev(Y))
        assert r.status == L.OK and r.resid.max() <= tol
        np.testing.assert_allclose(r.lam, mu[3:] / (b0 + b1 * (6.0 - mu[3:])), rtol=rt)
        assert np.abs(Y.T @ Bapply(r.X.cpu().numpy())).max() < 1e-9 * np.sqrt(N)


@pytest.mark.parametrize("prec", [L.FP64, L.MIXED])
def test_diagonal_B_with_constraints_matches_dense_pencil(prec):
    """Constraints with B = diag(d) (steps 2 and 10 B-orthogonal): Y spans the
    B-eigenvectors 0 and 2 of the pencil (A, B) (randomly mixed; a dense
    generalized eigensolve on 8 x 7 x 6 points); the solve finds eigenpairs 1,
    3 and 4, as the oracle does, with X B-orthogonal to Y and B-orthonormal."""
    dims, m, tol = (8, 7, 6), 3, 1e-9
    N = int(np.prod(dims))
    d = lumped_mass(N, 13)
    A = grid.laplace7(dims, np.eye(N))
    s = 1.0 / np.sqrt(d)
    mu, Z = np.linalg.eigh(s[:, None] * A * s[None, :])
    V = s[:, None] * Z                                  # B-orthonormal eigenvectors
    assert np.all(np.diff(mu[:6]) > 1e-6)
    Y = V[:, [0, 2]] @ np.random.default_rng(14).standard_normal((2, 2))
    X0 = synth.x0_uniform(N, m, seed=6)
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(None), m, prec, B=L.Diag(*dims, dev(d)))
    r = L.lobpcg_solve(ctx, dev(X0), tol, 500, Y=dev(Y))
    ref = olob.laplace7_solver(dims, m, X0, tol, 500, bdiag=d, Y=Y)
    assert r.status == L.OK and ref.status == olob.OK
    rt = 1e-9 if prec == L.FP64 else 1e-6
    np.testing.assert_allclose(r.lam, mu[[1, 3, 4]], rtol=rt)
    np.testing.assert_allclose(r.lam, ref.lam, rtol=rt)
    assert r.resid.max() <= tol
    X = r.X.cpu().numpy()
    assert np.abs(Y.T @ (d[:, None] * X)).max() < 1e-9
    np.testing.assert_allclose(X.T @ (d[:, None] * X), np.eye(m), atol=1e-10)
    if prec == L.FP64:
        assert abs(r.iters - ref.iters) <= 2, (r.iters, ref.iters)


@pytest.mark.parametrize("prec", [L.FP64, L.MIXED])
@pytest.mark.parametrize("ny", [3, 7])
def test_mass7_B_with_constraints_gives_the_next_closed_form_pairs(prec, ny):
    """Constraints with the 7-point mass-type B: the sine modes are the
    B-eigenvectors too, so with Y spanning the ny smallest modes (randomly
    mixed; 7 > m takes B Y in two pieces) the solve gives the next m
    eigenvalues mu / (b0 + b1 (6 - mu)); X is B-orthogonal to Y and
    B-orthonormal, every explicit residual <= tol."""
    dims, m, levels, tol = (20, 18, 16), 5, 3, 1e-9 if prec == L.FP64 else 1e-8
    b0, b1 = 1.0, -0.1
    N = int(np.prod(dims))
    mu, ijk = closed_form.smallest(*dims, ny + m)
    Y = sine_block(dims, ijk[:ny]) @ np.random.default_rng(ny).standard_normal((ny, ny))
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(levels), m, prec, B=L.Mass7(*dims, b0, b1))
    r = L.lobpcg_solve(ctx, dev(synth.x0_uniform(N, m, seed=9)), tol, 300, Y=dev(Y))
    assert r.status == L.OK
    lam = mu[ny:] / (b0 + b1 * (6.0 - mu[ny:]))
    np.testing.assert_allclose(r.lam, lam, rtol=1e-9 if prec == L.FP64 else 1e-6)
    assert r.resid.max() <= tol
    X = r.X.cpu().numpy()
    BX = grid.mass7(dims, b0, b1, X)
    assert np.abs(Y.T @ BX).max() < 1e-9 * np.abs(Y).max() * np.sqrt(N)
    np.testing.assert_allclose(X.T @ BX, np.eye(m), atol=1e-10)


@pytest.mark.parametrize("b0,b1", [(0.6, 1.0 / 12.0), (1.0, -0.1)])
def test_mass7_B_fp64_matches_oracle_and_closed_form(b0, b1):
    """A x = lambda B x with the 7-point mass-type B: eigenvalues mu / (b0 +
    b1 (6 - mu)) of the closed-form mu, the oracle's iteration within 2,
    X B-orthonormal, every explicit residual ||Ax - lambda Bx|| / (||A|| ||Bx||)
    <= tol."""
    dims, m, levels, tol = (20, 18, 16), 6, 3, 1e-9
    N = int(np.prod(dims))
    X0 = synth.x0_uniform(N, m, seed=8)
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(levels), m, L.FP64, B=L.Mass7(*dims, b0, b1))
    r = L.lobpcg_solve(ctx, dev(X0), tol, 300)
    ref = olob.laplace7_solver(dims, m, X0, tol, 300, levels=levels, bmass=(b0, b1))
    mu, _ = closed_form.smallest(*dims, m)
    assert r.status == L.OK and ref.status == olob.OK
    np.testing.assert_allclose(r.lam, mu / (b0 + b1 * (6.0 - mu)), rtol=5e-9)
    np.testing.assert_allclose(r.lam, ref.lam, rtol=5e-9)
    assert r.resid.max() <= tol
    X = r.X.cpu().numpy()
    np.testing.assert_allclose(X.T @ grid.mass7(dims, b0, b1, X), np.eye(m), atol=1e-10)
    assert abs(r.iters - ref.iters) <= 2, (r.iters, ref.iters)


@pytest.mark.parametrize("kind", ["diag", "mass7"])
def test_B_in_mixed_precision_reaches_fp64_accuracy(kind):
    """The mixed solver with B (FP32 iterations with FP32 B X, B W, B P
    recurrences, then the FP64 finish from the FP32 iterate): eigenvalues
    within 1e-6 of the FP64 oracle's, every explicit FP64 residual <= tol, X
    B-orthonormal."""
    dims, m, levels, tol = (32, 30, 28), 8, 3, 1e-8
    N = int(np.prod(dims))
    X0 = synth.x0_uniform(N, m, seed=2)
    if kind == "diag":
        d = lumped_mass(N, 21)
        Bd, kw, Bapply = L.Diag(*dims, dev(d)), {"bdiag": d}, (lambda V: d[:, None] * V)
    else:
        b0, b1 = 1.0, -0.1
        Bd, kw, Bapply = L.Mass7(*dims, b0, b1), {"bmass": (b0, b1)}, (lambda V: grid.mass7(dims, b0, b1, V))
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(levels), m, L.MIXED, B=Bd)
    r = L.lobpcg_solve(ctx, dev(X0), tol, 300)
    st = L.lobpcg_get_stats(ctx)
    ref = olob.laplace7_solver(dims, m, X0, tol, 300, levels=levels, **kw)
    assert r.status == L.OK and ref.status == olob.OK
    assert st["iters_fp32"] > 0 and st["iters_fp64"] > 0
    np.testing.assert_allclose(r.lam, ref.lam, rtol=1e-6)
    assert r.resid.max() <= tol
    X = r.X.cpu().numpy()
    np.testing.assert_allclose(X.T @ Bapply(X), np.eye(m), atol=1e-9)
