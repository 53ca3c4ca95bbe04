"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Every oracle function is checked here against something other than itself:
the closed-form spectrum of Section 4.1 (and its sine eigenvectors),
brute-force dense eigensolves built independently by Kronecker sums or by
face assembly, algebraic identities (symmetry, adjointness, the energy and
Euler identities), and textbook multigrid error propagation.
"""
import os

import numpy as np
import pytest

import synth
from oracle import closed_form, grid, lobpcg, mg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- helpers (independent constructions)

def second_diff(n):
    """1-D Dirichlet second-difference matrix tridiag(-1, 2, -1)."""
    return 2.0 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)


def dense_laplace7(nx, ny, nz):
    """7-point Laplacian as a Kronecker sum (grid order p = x + nx*(y + ny*z))."""
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    return (np.kron(Iz, np.kron(Iy, second_diff(nx))) + np.kron(Iz, np.kron(second_diff(ny), Ix))
            + np.kron(second_diff(nz), np.kron(Iy, Ix)))


def dense_varcoef_by_faces(nx, ny, nz, kx, ky, kz):
    """A = sum over faces f of k_f (e_p - e_q)(e_p - e_q)^T, assembled face by face."""
    N = nx * ny * nz
    A = np.zeros((N, N))
    pid = lambda x, y, z: x + nx * (y + ny * z)

    def add(k, a, b):
        if a is not None:
            A[a, a] += k
        if b is not None:
            A[b, b] += k
        if a is not None and b is not None:
            A[a, b] -= k
            A[b, a] -= k

    for z in range(nz):
        for y in range(ny):
            for i in range(nx + 1):
                add(kx[z, y, i], pid(i - 1, y, z) if i > 0 else None, pid(i, y, z) if i < nx else None)
    for z in range(nz):
        for i in range(ny + 1):
            for x in range(nx):
                add(ky[z, i, x], pid(x, i - 1, z) if i > 0 else None, pid(x, i, z) if i < ny else None)
    for i in range(nz + 1):
        for y in range(ny):
            for x in range(nx):
                add(kz[i, y, x], pid(x, y, i - 1) if i > 0 else None, pid(x, y, i) if i < nz else None)
    return A


def energy_by_differences(dims, kx, ky, kz, u):
    """u^T A u = sum_f k_f (u_p - u_q)^2 via zero-padded numpy differences."""
    nx, ny, nz = dims
    g = np.zeros((nz + 2, ny + 2, nx + 2))
    g[1:-1, 1:-1, 1:-1] = u.reshape(nz, ny, nx)
    dx = np.diff(g[1:-1, 1:-1, :], axis=2)
    dy = np.diff(g[1:-1, :, 1:-1], axis=1)
    dz = np.diff(g[:, 1:-1, 1:-1], axis=0)
    return np.sum(kx * dx ** 2) + np.sum(ky * dy ** 2) + np.sum(kz * dz ** 2)


def lognormal_faces(dims, seed):
    return synth.gaussian_field_faces(*dims, sigma=0.5, corr=2.0, seed=seed)


# ---------------------------------------------------------------- closed form (Section 4.1)

@pytest.mark.parametrize("dims", [(6, 7, 8), (5, 5, 5), (3, 4, 9)])
def test_closed_form_equals_dense_eigvalsh(dims):
    N = int(np.prod(dims))
    ref = np.linalg.eigvalsh(dense_laplace7(*dims))
    lam, _ = closed_form.smallest(*dims, N)
    np.testing.assert_allclose(lam, ref, rtol=1e-13, atol=1e-13)


def test_closed_form_hand_values():
    rows = np.loadtxt(os.path.join(GOLDEN, "worked_values.txt"))
    for nx, ny, nz, idx, val in rows:
        lam, _ = closed_form.smallest(int(nx), int(ny), int(nz), int(idx) + 1)
        # the typed values carry at least nine significant digits
        assert abs(lam[int(idx)] / val - 1) < 5e-9, (nx, idx, lam[int(idx)], val)


def test_closed_form_golden_file_current():
    rows = np.loadtxt(os.path.join(GOLDEN, "laplace7_smallest.txt"))
    for nx, ny, nz, idx, val, i, j, k in rows:
        lam, ijk = closed_form.smallest(int(nx), int(ny), int(nz), int(idx) + 1)
        assert lam[int(idx)] == pytest.approx(val, rel=1e-15)


# ---------------------------------------------------------------- stencils

@pytest.mark.parametrize("dims", [(6, 7, 8), (4, 4, 4), (1, 3, 5)])
def test_laplace7_matches_kronecker_sum(dims):
    N = int(np.prod(dims))
    U = synth.random_block(N, 3, seed=11)
    np.testing.assert_allclose(grid.laplace7(dims, U), dense_laplace7(*dims) @ U, rtol=0, atol=1e-13)


@pytest.mark.parametrize("dims,ijk", [((16, 16, 16), (1, 1, 1)), ((16, 16, 16), (3, 5, 16)),
                                      ((9, 12, 7), (2, 11, 4))])
def test_laplace7_sine_modes(dims, ijk):
    v = closed_form.mode(*dims, *ijk)
    lam = sum(closed_form.eig1d(n)[i - 1] for n, i in zip(dims, ijk))
    np.testing.assert_allclose(grid.laplace7(dims, v), lam * v, rtol=0, atol=1e-13)


def test_varcoef7_with_unit_k_is_laplace7():
    dims = (7, 6, 5)
    kx, ky, kz = (np.ones(s) for s in synth.face_shapes(*dims))
    U = synth.random_block(210, 4, seed=3)
    np.testing.assert_allclose(grid.varcoef7(dims, kx, ky, kz, U), grid.laplace7(dims, U), rtol=0, atol=1e-14)


def test_varcoef7_matches_face_assembly():
    dims = (3, 4, 5)
    kx, ky, kz = lognormal_faces(dims, 5)
    A = dense_varcoef_by_faces(*dims, kx, ky, kz)
    U = synth.random_block(60, 3, seed=4)
    np.testing.assert_allclose(grid.varcoef7(dims, kx, ky, kz, U), A @ U, rtol=0, atol=1e-13)


def test_varcoef7_energy_and_symmetry():
    dims = (9, 8, 7)
    kx, ky, kz = lognormal_faces(dims, 6)
    u, v = synth.random_block(504, 2, seed=7).T
    Au, Av = grid.varcoef7(dims, kx, ky, kz, u), grid.varcoef7(dims, kx, ky, kz, v)
    assert u @ Au == pytest.approx(energy_by_differences(dims, kx, ky, kz, u), rel=1e-13)
    assert u @ Av == pytest.approx(v @ Au, rel=1e-13)


def test_gershgorin_bounds():
    dims = (5, 6, 7)
    kx, ky, kz = lognormal_faces(dims, 8)
    A = dense_varcoef_by_faces(*dims, kx, ky, kz)
    assert grid.gershgorin_varcoef7(dims, kx, ky, kz) == pytest.approx(np.abs(A).sum(axis=1).max(), rel=1e-14)
    assert grid.gershgorin_laplace7() == np.abs(dense_laplace7(*dims)).sum(axis=1).max()


# ---------------------------------------------------------------- multigrid pieces

@pytest.mark.parametrize("level", [0, 1, 3])
def test_jacobi_damps_sine_mode_exactly(level):
    dims, ijk, om = (11, 10, 9), (2, 7, 9), 2.0 / 3.0
    v = closed_form.mode(*dims, *ijk)
    lam = sum(closed_form.eig1d(n)[i - 1] for n, i in zip(dims, ijk))
    out = grid.jacobi(dims, 4.0 ** -level, om, v, np.zeros_like(v))
    np.testing.assert_allclose(out, (1 - om * lam / 6.0) * v, rtol=0, atol=1e-14)


def test_jacobi_first_sweep_from_zero():
    b = synth.random_block(60, 2, seed=1)
    np.testing.assert_allclose(grid.jacobi((3, 4, 5), 0.25, 0.5, None, b), b * 0.5 / (6 * 0.25), rtol=1e-15)


@pytest.mark.parametrize("fine", [(8, 8, 8), (9, 7, 6), (5, 10, 11)])
def test_restriction_is_prolongation_transpose_over_8(fine):
    coarse = grid.coarsen(fine)
    x = synth.random_block(int(np.prod(fine)), 1, seed=2)[:, 0]
    y = synth.random_block(int(np.prod(coarse)), 1, seed=3)[:, 0]
    lhs = grid.restrict(fine, coarse, x) @ y
    rhs = x @ grid.prolong_add(fine, coarse, y, np.zeros_like(x)) / 8.0
    assert lhs == pytest.approx(rhs, rel=1e-14)


def test_prolongation_reproduces_linear_functions():
    fine = (13, 11, 9)
    coarse = grid.coarsen(fine)
    a, bx, by, bz = 0.3, 1.1, -0.7, 0.45
    f = lambda x, y, z: a + bx * x + by * y + bz * z
    Z, Y, X = np.meshgrid(*(2 * np.arange(n) + 1 for n in coarse[::-1]), indexing="ij")
    ec = f(X, Y, Z).ravel()
    xf = grid.prolong_add(fine, coarse, ec, np.zeros(int(np.prod(fine)))).reshape(fine[::-1])
    Zf, Yf, Xf = np.meshgrid(*(np.arange(n) for n in fine[::-1]), indexing="ij")
    want = f(Xf, Yf, Zf)
    # interior: every fine node with both interpolation partners inside the coarse grid
    inner = tuple(slice(1, 2 * c) for c in coarse[::-1])
    np.testing.assert_allclose(xf[inner], want[inner], rtol=0, atol=1e-13)


def test_restriction_weights_sum_to_one():
    fine = (15, 13, 11)
    coarse = grid.coarsen(fine)
    bc = grid.restrict(fine, coarse, np.ones(int(np.prod(fine))))
    np.testing.assert_allclose(bc, 1.0, rtol=1e-15)


# ---------------------------------------------------------------- V-cycle

@pytest.mark.parametrize("dims,levels", [((16, 16, 16), 3), ((15, 13, 12), 3), ((8, 8, 8), 4)])
def test_vcycle_symmetric_positive(dims, levels):
    T = mg.VCycle(dims, levels)
    N = int(np.prod(dims))
    B = synth.random_block(N, 4, seed=9)
    TB = T(B)
    G = B.T @ TB
    np.testing.assert_allclose(G, G.T, rtol=1e-12, atol=1e-14)
    assert np.all(np.linalg.eigvalsh(0.5 * (G + G.T)) > 0)


def test_vcycle_single_level_is_jacobi_polynomial():
    dims, ijk, om = (8, 8, 8), (3, 1, 2), 2.0 / 3.0
    v = closed_form.mode(*dims, *ijk)
    lam = sum(closed_form.eig1d(n)[i - 1] for n, i in zip(dims, ijk))
    out = mg.VCycle(dims, 1, coarse_sweeps=20, omega=om)(v)
    np.testing.assert_allclose(out, (1 - (1 - om * lam / 6) ** 20) / lam * v, rtol=0, atol=1e-13)


def interp_1d(nf):
    nc = nf // 2
    P = np.zeros((nf, nc))
    for I in range(nc):
        P[2 * I + 1, I] = 1.0
        P[2 * I, I] = 0.5
        if 2 * I + 2 < nf:
            P[2 * I + 2, I] = 0.5
    return P


@pytest.mark.parametrize("dims", [(7, 7, 7), (8, 6, 7)])
def test_vcycle_two_grid_error_propagation(dims):
    """Two-level V(2,2): E = I - T A = S^2 (I - P T_c R A) S^2 (textbook form)."""
    om = 2.0 / 3.0
    nx, ny, nz = dims
    A = dense_laplace7(*dims)
    N = A.shape[0]
    S = np.eye(N) - om / 6.0 * A
    P = np.kron(interp_1d(nz), np.kron(interp_1d(ny), interp_1d(nx)))
    R = P.T / 8.0
    Ac = dense_laplace7(nx // 2, ny // 2, nz // 2) / 4.0
    Sc = np.eye(Ac.shape[0]) - om / (6.0 / 4.0) * Ac
    Tc = (np.eye(Ac.shape[0]) - np.linalg.matrix_power(Sc, 20)) @ np.linalg.inv(Ac)
    E = S @ S @ (np.eye(N) - P @ Tc @ R @ A) @ S @ S
    T_ref = (np.eye(N) - E) @ np.linalg.inv(A)
    T_or = mg.VCycle(dims, 2)(np.eye(N))
    np.testing.assert_allclose(T_or, T_ref, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- dense building blocks

def test_chol_scaled_factor_and_scale_invariance():
    rng = np.random.default_rng(0)
    V = rng.standard_normal((50, 6))
    G = V.T @ V
    R = lobpcg.chol_scaled(G)
    np.testing.assert_allclose(R.T @ R, G, rtol=1e-13, atol=1e-13)
    assert np.allclose(R, np.triu(R))
    d = np.array([1e-12, 1.0, 1e8, 3e-5, 7.0, 1e-20])
    R2 = lobpcg.chol_scaled(G * np.outer(d, d))
    np.testing.assert_allclose(R2, R * d[None, :], rtol=1e-12, atol=0)


@pytest.mark.parametrize("G", [np.array([[1.0, 1.0], [1.0, 1.0]]), np.array([[1.0, 0.0], [0.0, 0.0]]),
                               np.array([[1.0, 2.0], [2.0, 1.0]]), np.array([[np.nan, 0], [0, 1.0]])])
def test_chol_scaled_rejects_non_pd(G):
    with pytest.raises(lobpcg.CholeskyFailure):
        lobpcg.chol_scaled(G)


def test_rayleigh_ritz_solves_pencil():
    rng = np.random.default_rng(1)
    V = rng.standard_normal((40, 9))
    Bm = V.T @ V
    Am = rng.standard_normal((9, 9)); Am = Am + Am.T
    theta, C = lobpcg.rayleigh_ritz(Am, Bm, 4)
    np.testing.assert_allclose(Am @ C, Bm @ C * theta, atol=1e-11)
    np.testing.assert_allclose(C.T @ Bm @ C, np.eye(4), atol=1e-12)
    # smallest four of the full pencil, via the standard problem for L^-1 A L^-T
    L = np.linalg.cholesky(Bm)
    Li = np.linalg.inv(L)
    np.testing.assert_allclose(theta, np.linalg.eigvalsh(Li @ Am @ Li.T)[:4], rtol=1e-11)


# ---------------------------------------------------------------- LOBPCG (Section 2.2)

def test_lobpcg_unpreconditioned_n16_closed_form():
    dims, m = (16, 16, 16), 4
    r = lobpcg.laplace7_solver(dims, m, synth.x0_uniform(4096, m), 1e-8, 500)
    assert r.status == lobpcg.OK
    lam, _ = closed_form.smallest(*dims, m)
    np.testing.assert_allclose(r.lam, lam, rtol=1e-10)
    assert r.resid.max() <= 1e-8


@pytest.mark.parametrize("dims,m,levels", [((6, 7, 8), 5, None), ((8, 8, 8), 6, 2)])
def test_lobpcg_matches_dense_bruteforce(dims, m, levels):
    N = int(np.prod(dims))
    ref = np.linalg.eigvalsh(dense_laplace7(*dims))[:m]
    r = lobpcg.laplace7_solver(dims, m, synth.x0_uniform(N, m, seed=3), 1e-11, 1000, levels=levels)
    assert r.status == lobpcg.OK
    np.testing.assert_allclose(r.lam, ref, rtol=1e-12)


def test_lobpcg_varcoef_matches_dense_bruteforce():
    dims, m = (5, 6, 7), 4
    kx, ky, kz = lognormal_faces(dims, 12)
    A = dense_varcoef_by_faces(*dims, kx, ky, kz)
    w, V = np.linalg.eigh(A)
    r = lobpcg.varcoef_solver(dims, kx, ky, kz, m, synth.x0_uniform(210, m, seed=4), 1e-11, 1000)
    assert r.status == lobpcg.OK
    np.testing.assert_allclose(r.lam, w[:m], rtol=1e-12)
    # simple eigenvalues: vectors equal up to sign
    for i in range(m):
        c = abs(r.X[:, i] @ V[:, i]) / np.linalg.norm(r.X[:, i])
        assert c == pytest.approx(1.0, abs=1e-10)


def test_lobpcg_mg_eigenpairs_against_sine_modes():
    dims, m = (24, 20, 16), 6
    N = int(np.prod(dims))
    r = lobpcg.laplace7_solver(dims, m, synth.x0_uniform(N, m), 1e-9, 200, levels=3)
    assert r.status == lobpcg.OK
    lam, ijk = closed_form.smallest(*dims, m)
    np.testing.assert_allclose(r.lam, lam, rtol=1e-10)
    assert r.resid.max() <= 1e-9
    # distinct eigenvalues here: each Ritz vector is a sine mode up to sign
    assert np.min(np.diff(lam)) > 1e-3
    for i in range(m):
        v = closed_form.mode(*dims, *ijk[i])
        c = abs(v @ r.X[:, i]) / (np.linalg.norm(v) * np.linalg.norm(r.X[:, i]))
        assert 1 - c < 1e-12


def test_lobpcg_ritz_values_never_increase():
    """X lies in every trial subspace, so each Ritz value is non-increasing (Section 2.1.3)."""
    lams = []
    r = lobpcg.laplace7_solver((12, 12, 12), 6, synth.x0_uniform(1728, 6), 1e-9, 300, levels=2,
                               callback=lambda k, lam, rho, J: lams.append(np.array(lam)))
    assert r.status == lobpcg.OK
    L = np.array(lams)
    assert np.all(np.diff(L, axis=0) <= 1e-13 * np.abs(L[1:]))


def test_lobpcg_soft_locked_pairs_keep_improving():
    """Section 2.3: a soft-locked pair whose Ritz value is below the next
    eigenvalue still improves through the Rayleigh-Ritz procedure."""
    dims, m = (16, 16, 16), 4
    lam_ex, _ = closed_form.smallest(*dims, m)
    errs, locked_at = [], {}

    def cb(k, lam, rho, J):
        errs.append(np.array(lam) - lam_ex)
        for j in range(m):
            if j not in J and j not in locked_at:
                locked_at[j] = k

    lobpcg.lobpcg(lambda V: grid.laplace7(dims, V), synth.x0_uniform(4096, m), 1e-4, 500, 12.0,
                  callback=cb, reactivate=False)
    assert 0 in locked_at and locked_at[0] < len(errs) - 2
    e0 = np.array(errs)[locked_at[0]:, 0]
    assert np.all(np.diff(e0) <= 1e-15) and e0[-1] < e0[0]


def test_lobpcg_explicit_gram_variant():
    """Section 2.2's variant with the block diagonal of gramB computed: on a
    short run it gives the paper's form's eigenvalues (closed form) in the same
    number of iterations; on a long run with m=40 where the paper's form loses
    orthogonality (a spurious Ritz value below lambda_1), it converges to the
    closed form."""
    dims, m = (12, 10, 8), 6
    X0 = synth.x0_uniform(960, m)
    exact, _ = closed_form.smallest(*dims, m)
    a = lobpcg.laplace7_solver(dims, m, X0, 1e-10, 200, levels=2)
    b = lobpcg.laplace7_solver(dims, m, X0, 1e-10, 200, levels=2, explicit_gram=True)
    assert a.status == b.status == lobpcg.OK
    np.testing.assert_allclose(b.lam, exact, rtol=1e-12)
    assert abs(a.iters - b.iters) <= 1
    dims, m = (20, 18, 16), 40
    X0 = synth.x0_uniform(5760, m)
    exact, _ = closed_form.smallest(*dims, m)
    c = lobpcg.laplace7_solver(dims, m, X0, 1e-9, 120, levels=3, explicit_gram=True)
    assert c.status == lobpcg.OK and c.iters < 60
    np.testing.assert_allclose(c.lam, exact, rtol=1e-11)
    assert c.resid.max() <= 1e-9


def test_lobpcg_error_paths():
    dims, m = (6, 6, 6), 3
    X0 = synth.x0_uniform(216, m)
    X0[:, 2] = X0[:, 1]
    assert lobpcg.laplace7_solver(dims, m, X0, 1e-8, 50).status == lobpcg.ERR_CHOL
    X0 = synth.x0_uniform(216, m)
    X0[5, 0] = np.nan
    assert lobpcg.laplace7_solver(dims, m, X0, 1e-8, 50).status == lobpcg.ERR_NONFINITE
    r = lobpcg.laplace7_solver(dims, m, synth.x0_uniform(216, m), 1e-8, 2)
    assert r.status == lobpcg.NOT_CONVERGED and r.iters == 2 and r.lam.shape == (m,)


# ---------------------------------------------------------------- eigenvalue adjoint

def test_adjoint_euler_identity():
    """A is linear in k, so sum_f k_f d lambda/d k_f equals the Rayleigh quotient."""
    dims = (9, 8, 7)
    kx, ky, kz = lognormal_faces(dims, 13)
    X = synth.random_block(504, 3, seed=14)
    for i in range(3):
        g = np.zeros(3); g[i] = 1.0
        gkx, gky, gkz = grid.eig_grad_faces(dims, X, g)
        s = np.sum(kx * gkx) + np.sum(ky * gky) + np.sum(kz * gkz)
        x = X[:, i]
        assert s == pytest.approx(x @ grid.varcoef7(dims, kx, ky, kz, x) / (x @ x), rel=1e-13)


def test_adjoint_matches_dense_finite_differences():
    dims = (3, 4, 3)
    kx, ky, kz = lognormal_faces(dims, 15)
    shapes = synth.face_shapes(*dims)
    sizes = [int(np.prod(s)) for s in shapes]
    kflat = np.concatenate([kx.ravel(), ky.ravel(), kz.ravel()])

    def eigs(kf):
        a, b, c = np.split(kf, np.cumsum(sizes)[:2])
        return np.linalg.eigh(dense_varcoef_by_faces(*dims, a.reshape(shapes[0]), b.reshape(shapes[1]),
                                                     c.reshape(shapes[2])))

    w, V = eigs(kflat)
    gbar = np.array([0.7, -1.3, 0.4])
    gk = np.concatenate([a.ravel() for a in grid.eig_grad_faces(dims, V[:, :3], gbar)])
    h = 1e-6
    fd = np.empty_like(kflat)
    for f in range(kflat.size):
        kp, km = kflat.copy(), kflat.copy()
        kp[f] += h; km[f] -= h
        fd[f] = gbar @ (eigs(kp)[0][:3] - eigs(km)[0][:3]) / (2 * h)
    # rounding floor of the central difference: about eps*||A||/h = 2e-9
    np.testing.assert_allclose(gk, fd, rtol=1e-6, atol=1e-8)


def test_adjoint_with_B_matches_dense_finite_differences():
    """A(k) x = lambda B x with a fixed diagonal B (seeded, in [0.5, 2]): the
    gradient (x_p - x_q)^2 / (x, B x) of eig_grad_faces_B against central
    differences of the pencil's eigenvalues (dense, through the congruent
    standard problem) in every face coefficient."""
    dims = (3, 4, 3)
    N = int(np.prod(dims))
    kx, ky, kz = lognormal_faces(dims, 17)
    d = np.random.default_rng(18).uniform(0.5, 2.0, N)
    s = 1.0 / np.sqrt(d)
    shapes = synth.face_shapes(*dims)
    sizes = [int(np.prod(t)) for t in shapes]
    kflat = np.concatenate([kx.ravel(), ky.ravel(), kz.ravel()])

    def eigs(kf):
        a, b, c = np.split(kf, np.cumsum(sizes)[:2])
        A = dense_varcoef_by_faces(*dims, a.reshape(shapes[0]), b.reshape(shapes[1]), c.reshape(shapes[2]))
        w, Z = np.linalg.eigh(s[:, None] * A * s[None, :])
        return w, s[:, None] * Z

    w, V = eigs(kflat)
    X = V[:, :3] * np.array([1.0, -2.5, 0.3])        # not B-normalised: the formula divides by (x, B x)
    gbar = np.array([0.7, -1.3, 0.4])
    gk = np.concatenate([a.ravel() for a in grid.eig_grad_faces_B(dims, X, gbar, d[:, None] * X)])
    h = 1e-6
    fd = np.empty_like(kflat)
    for f in range(kflat.size):
        kp, km = kflat.copy(), kflat.copy()
        kp[f] += h; km[f] -= h
        fd[f] = gbar @ (eigs(kp)[0][:3] - eigs(km)[0][:3]) / (2 * h)
    np.testing.assert_allclose(gk, fd, rtol=1e-6, atol=1e-8)
    # with B = I it is eig_grad_faces
    for a, b in zip(grid.eig_grad_faces_B(dims, X, gbar, X), grid.eig_grad_faces(dims, X, gbar)):
        np.testing.assert_allclose(a, b, rtol=1e-14, atol=0)


def test_adjoint_scale_invariance():
    """lambda(c k) = c lambda(k), so the gradient does not change under k -> c k."""
    dims = (5, 5, 6)
    kx, ky, kz = lognormal_faces(dims, 16)
    A = dense_varcoef_by_faces(*dims, kx, ky, kz)
    A2 = dense_varcoef_by_faces(*dims, 3 * kx, 3 * ky, 3 * kz)
    w, V = np.linalg.eigh(A)
    w2, V2 = np.linalg.eigh(A2)
    np.testing.assert_allclose(w2[:2], 3 * w[:2], rtol=1e-13)
    g1 = grid.eig_grad_faces(dims, V[:, :2], np.ones(2))
    g2 = grid.eig_grad_faces(dims, V2[:, :2], np.ones(2))
    for a, b in zip(g1, g2):
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-13)


def test_laplace7_rows_matches_full_operator():
    dims = (7, 5, 6)
    U = synth.random_block(210, 3, seed=21)
    pts = np.array([0, 1, 6, 34, 35, 100, 209])
    np.testing.assert_allclose(grid.laplace7_rows(dims, U, pts), grid.laplace7(dims, U)[pts], rtol=0, atol=1e-14)


# ---------------------------------------------------------------- constraints Y (steps 2 and 10)

def test_constraints_give_the_next_eigenpairs():
    """Hard locking: with Y = the exact eigenvectors of the m smallest
    eigenvalues, LOBPCG in span(Y)^perp finds eigenvalues m+1 .. 2m (closed
    form, Section 4.1) and its vectors stay orthogonal to Y."""
    dims, m = (12, 10, 8), 4
    N = int(np.prod(dims))
    lam, ijk = closed_form.smallest(*dims, 2 * m)
    assert np.all(np.diff(lam) > 1e-6)            # simple spectrum here
    Y = np.stack([closed_form.mode(*dims, *t) for t in ijk[:m]], axis=1)
    Y /= np.linalg.norm(Y, axis=0)
    X0 = synth.x0_uniform(N, m, seed=3)
    r = lobpcg.laplace7_solver(dims, m, X0, 1e-10, 300, levels=2, Y=Y)
    assert r.status == lobpcg.OK
    np.testing.assert_allclose(r.lam, lam[m:], rtol=1e-9)
    assert np.abs(Y.T @ r.X).max() < 1e-9
    # without the constraints the same start finds the m smallest instead
    r0 = lobpcg.laplace7_solver(dims, m, X0, 1e-10, 300, levels=2)
    np.testing.assert_allclose(r0.lam, lam[:m], rtol=1e-9)


def test_constraints_match_dense_projected_eigenproblem():
    """Y spanning an invariant subspace that is not the lowest one, given by a
    non-orthonormal basis (a random mix of the exact eigenvectors 0, 2 and 5
    of a dense solve, N = 72): the constrained problem's m smallest eigenvalues
    are those of indices 1, 3, 4 (brute force), and the vectors stay orthogonal
    to Y.  The mix makes the (Y^T Y)^-1 of steps 2 and 10 matter."""
    dims, m = (6, 4, 3), 3
    N = int(np.prod(dims))
    lam, V = np.linalg.eigh(dense_laplace7(*dims))
    assert np.all(np.diff(lam[:6]) > 1e-8)
    Y = V[:, [0, 2, 5]] @ np.random.default_rng(12).standard_normal((3, 3))
    r = lobpcg.laplace7_solver(dims, m, synth.x0_uniform(N, m, seed=4), 1e-11, 500, Y=Y)
    assert r.status == lobpcg.OK
    np.testing.assert_allclose(r.lam, lam[[1, 3, 4]], rtol=1e-10)
    assert np.abs(Y.T @ r.X).max() < 1e-10


# ---------------------------------------------------------------- B != I (general SPD B)

def test_scalar_B_scales_the_spectrum():
    """A x = lambda (c I) x: the eigenvalues are the closed form divided by c,
    and X is B-orthonormal (X^T B X = I)."""
    dims, m, c = (12, 10, 8), 4, 2.5
    N = int(np.prod(dims))
    lam, _ = closed_form.smallest(*dims, m)
    r = lobpcg.laplace7_solver(dims, m, synth.x0_uniform(N, m, seed=3), 1e-10, 300, levels=2,
                               bdiag=np.full(N, c))
    assert r.status == lobpcg.OK
    np.testing.assert_allclose(r.lam, lam / c, rtol=1e-9)
    np.testing.assert_allclose(c * r.X.T @ r.X, np.eye(m), atol=1e-10)


def test_diagonal_B_matches_dense_generalized_eigenproblem():
    """Lumped-mass-like B = diag(d), d in [0.5, 2] (seeded): the eigenvalues of
    the pencil (A, B) by brute force through the congruent standard problem
    D^-1/2 A D^-1/2 (N = 72); X is B-orthonormal; with constraints Y spanning
    B-eigenvectors 0 and 2 (randomly mixed) the next ones are 1, 3, 4."""
    dims, m = (6, 4, 3), 3
    N = int(np.prod(dims))
    d = np.random.default_rng(13).uniform(0.5, 2.0, N)
    A = dense_laplace7(*dims)
    s = 1.0 / np.sqrt(d)
    mu, Z = np.linalg.eigh(s[:, None] * A * s[None, :])
    V = s[:, None] * Z                                  # B-orthonormal eigenvectors
    assert np.all(np.diff(mu[:6]) > 1e-6)
    r = lobpcg.laplace7_solver(dims, m, synth.x0_uniform(N, m, seed=5), 1e-11, 500, bdiag=d)
    assert r.status == lobpcg.OK
    np.testing.assert_allclose(r.lam, mu[:m], rtol=1e-10)
    np.testing.assert_allclose(r.X.T @ (d[:, None] * r.X), np.eye(m), atol=1e-10)
    Y = V[:, [0, 2]] @ np.random.default_rng(14).standard_normal((2, 2))
    r = lobpcg.laplace7_solver(dims, m, synth.x0_uniform(N, m, seed=6), 1e-11, 500, bdiag=d, Y=Y)
    assert r.status == lobpcg.OK
    np.testing.assert_allclose(r.lam, mu[[1, 3, 4]], rtol=1e-10)
    assert np.abs(Y.T @ (d[:, None] * r.X)).max() < 1e-10


def dense_mass7_by_neighbours(nx, ny, nz, b0, b1):
    """B[p, p] = b0 and B[p, q] = b1 for the axis neighbours q of p, entered
    point by point."""
    N = nx * ny * nz
    B = np.zeros((N, N))
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                p = x + nx * (y + ny * z)
                B[p, p] = b0
                for dx, dy, dz in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
                    a, b, c = x + dx, y + dy, z + dz
                    if 0 <= a < nx and 0 <= b < ny and 0 <= c < nz:
                        B[p, a + nx * (b + ny * c)] = b1
    return B


@pytest.mark.parametrize("b0,b1", [(0.6, 1.0 / 12.0), (1.0, -0.1)])
def test_mass7_matches_neighbour_assembly(b0, b1):
    dims = (5, 4, 3)
    N = 60
    U = np.random.default_rng(31).standard_normal((N, 3))
    np.testing.assert_allclose(grid.mass7(dims, b0, b1, U), dense_mass7_by_neighbours(*dims, b0, b1) @ U,
                               rtol=0, atol=1e-14)


@pytest.mark.parametrize("b0,b1", [(0.6, 1.0 / 12.0), (1.0, -0.1)])
def test_mass7_B_closed_form(b0, b1):
    """B = b0 I + b1 (6 I - L7) shares the sine eigenvectors of L7, so the
    pencil (L7, B) has eigenvalues mu / (b0 + b1 (6 - mu)) for the closed-form
    mu; the map is increasing while b0 > 6 |b1|, so the smallest eigenvalues
    of the pencil are those of the smallest mu.  X comes out B-orthonormal."""
    dims, m = (12, 10, 8), 4
    N = int(np.prod(dims))
    mu, _ = closed_form.smallest(*dims, m)
    want = mu / (b0 + b1 * (6.0 - mu))
    r = lobpcg.laplace7_solver(dims, m, synth.x0_uniform(N, m, seed=3), 1e-10, 300, levels=2, bmass=(b0, b1))
    assert r.status == lobpcg.OK
    np.testing.assert_allclose(r.lam, want, rtol=1e-9)
    np.testing.assert_allclose(r.X.T @ grid.mass7(dims, b0, b1, r.X), np.eye(m), atol=1e-10)


def test_mass7_B_matches_dense_generalized_eigenproblem():
    """The pencil (A, B) with A = -div(k grad u) (lognormal k) and the
    7-point mass-type B, N = 72: eigenvalues of the dense generalized
    problem (scipy.linalg.eigh(A, B)) with B assembled neighbour by
    neighbour."""
    import scipy.linalg
    dims, m, b0, b1 = (6, 4, 3), 3, 0.6, 1.0 / 12.0
    N = int(np.prod(dims))
    kx, ky, kz = lognormal_faces(dims, seed=8)
    A = dense_varcoef_by_faces(*dims, kx, ky, kz)
    B = dense_mass7_by_neighbours(*dims, b0, b1)
    mu = scipy.linalg.eigh(A, B, eigvals_only=True)
    assert np.all(np.diff(mu[:m + 1]) > 1e-6)
    Aop = lambda V: grid.varcoef7(dims, kx, ky, kz, V)
    Bop = lambda V: grid.mass7(dims, b0, b1, V)
    r = lobpcg.lobpcg(Aop, synth.x0_uniform(N, m, seed=9), 1e-11, 500,
                      grid.gershgorin_varcoef7(dims, kx, ky, kz), apply_B=Bop)
    assert r.status == lobpcg.OK
    np.testing.assert_allclose(r.lam, mu[:m], rtol=1e-10)


def test_wanted_pairs_with_guard_columns():
    """A block of 7 columns for the 4 wanted pairs (three guard columns): the
    run ends when the first 4 have converged, their Ritz values agree with the
    closed form, and it takes no more iterations than converging all 7.  With
    nwant = m it is the plain run, iteration for iteration."""
    dims, m, nw, tol = (12, 11, 10), 7, 4, 1e-9
    N = int(np.prod(dims))
    X0 = synth.x0_uniform(N, m, seed=5)
    exact, _ = closed_form.smallest(*dims, m)
    r = lobpcg.laplace7_solver(dims, m, X0, tol, 500, levels=2, nwant=nw)
    assert r.status == lobpcg.OK
    assert r.hist[-1][:nw].max() <= tol and r.resid[:nw].max() <= 1.01 * tol
    np.testing.assert_allclose(r.lam[:nw], exact[:nw], rtol=1e-12)
    full = lobpcg.laplace7_solver(dims, m, X0, tol, 500, levels=2)
    same = lobpcg.laplace7_solver(dims, m, X0, tol, 500, levels=2, nwant=m)
    assert full.status == lobpcg.OK and same.iters == full.iters
    assert np.array_equal(same.lam, full.lam) and np.array_equal(same.hist, full.hist)
    assert r.iters <= full.iters
    # the runs agree up to the wanted set's exit
    np.testing.assert_array_equal(r.hist, full.hist[:r.iters])


def test_cluster_locking_keeps_groups_together():
    """Soft locking by clusters (lock_gap): on 16^3 without preconditioner
    the triple lambda_2..4 leaves the active set in one iteration (with the
    paper's rule its columns leave one by one), the eigenvalues still match
    the closed form, and at lock_gap = 0 the run is the paper's."""
    dims, m, tol = (16, 16, 16), 4, 1e-8
    N = 4096
    X0 = synth.x0_uniform(N, m, seed=2)
    exact, _ = closed_form.smallest(*dims, m)
    sets = {}
    for gap in (0.0, 1e-3):
        Js = []
        r = lobpcg.laplace7_solver(dims, m, X0, tol, 500, lock_gap=gap,
                                   callback=lambda k, lam, rho, J: Js.append(tuple(J.tolist())))
        assert r.status == lobpcg.OK
        np.testing.assert_allclose(r.lam, exact, rtol=1e-10)
        sets[gap] = Js
    def leave(Js, j):
        return next(k for k, J in enumerate(Js) if j not in J)
    assert len({leave(sets[1e-3], j) for j in (1, 2, 3)}) == 1
    assert len({leave(sets[0.0], j) for j in (1, 2, 3)}) > 1
    r0 = lobpcg.laplace7_solver(dims, m, X0, tol, 500)
    assert r0.iters == len(sets[0.0])
