"""Kernel parity on the GPU: every step's kernel, called through the C ABI,
against the FP64 CPU oracle on the same seeded inputs.

Sizes span several workgroups, ragged grid tails (dimensions that are not
multiples of anything) and ragged column counts (1, 3, 5, 7 ...).  FP64
results must agree to rounding (about 1e-14 relative to the data); FP32
kernels are compared with the oracle applied to the same FP32 values, to a
bound of a few FP32 units in the last place times the number of terms.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import grid, mg

L = pytest.importorskip("paper_0705_2626_amd")
pytestmark = pytest.mark.gpu

DEV = "cuda"
EPS32 = 2.0 ** -24


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def host(t):
    return t.double().cpu().numpy()


_ctx_cache = {}


def ctx_for(dims, m, levels=None, prec=L.FP64):
    key = (dims, m, levels, prec)
    if key not in _ctx_cache:
        _ctx_cache[key] = L.lobpcg_setup(L.Op(*dims), L.Precond(levels), m, prec)
    return _ctx_cache[key]


# ---------------------------------------------------------------- stencils (step 12)

@pytest.mark.parametrize("dims", [(16, 16, 16), (13, 11, 9), (40, 7, 5), (3, 50, 2)])
@pytest.mark.parametrize("k", [1, 3, 4, 8, 32, 33])
def test_laplace7_fp64(dims, k):
    N = int(np.prod(dims))
    ctx = ctx_for(dims, 32 if 96 <= N else max(1, N // 3))
    if k > 3 * ctx.m:
        pytest.skip("block wider than the context allows")
    U = synth.random_block(N, k, seed=k)
    out = host(L.lobpcg_apply_A(ctx, dev(U)))
    ref = grid.laplace7(dims, U)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-14 * 12)


# column counts that are and are not multiples of the 16-byte vector width
@pytest.mark.parametrize("dims,k", [((16, 16, 16), 32), ((13, 11, 9), 5), ((40, 7, 5), 8), ((9, 9, 9), 2),
                                    ((17, 15, 13), 23), ((16, 9, 11), 31), ((8, 8, 8), 3), ((13, 11, 9), 7)])
def test_laplace7_fp32(dims, k):
    N = int(np.prod(dims))
    ctx = ctx_for(dims, min(32, N // 3), prec=L.MIXED)
    U = synth.random_block(N, k, seed=5).astype(np.float32)
    out = host(L.lobpcg_apply_A(ctx, dev(U, torch.float32)))
    ref = grid.laplace7(dims, U.astype(np.float64))
    np.testing.assert_allclose(out, ref, rtol=0, atol=16 * EPS32 * 12)


@pytest.mark.parametrize("dims,k", [((12, 10, 8), 8), ((9, 7, 11), 3), ((16, 16, 16), 1)])
def test_varcoef7_fp64(dims, k):
    N = int(np.prod(dims))
    kx, ky, kz = synth.gaussian_field_faces(*dims, sigma=0.5, corr=4.0, seed=7)
    A = L.Op(*dims, dev(kx), dev(ky), dev(kz))
    ctx = L.lobpcg_setup(A, L.Precond(None), 8, L.FP64)
    U = synth.random_block(N, k, seed=9)
    out = host(L.lobpcg_apply_A(ctx, dev(U), A=A))
    ref = grid.varcoef7(dims, kx, ky, kz, U)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-14 * np.abs(ref).max())


def test_laplace7_full_size_sampled_fp32():
    """The n=256, m=32 FP32 block of the mixed-precision benchmark: sampled rows,
    including the grid's corners, edges and its last point."""
    dims, k = (256, 256, 256), 32
    nx, ny, nz = dims
    N = nx * ny * nz
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(None), k, L.MIXED)
    g = torch.Generator(device=DEV).manual_seed(3)
    U = torch.rand((N, k), generator=g, device=DEV, dtype=torch.float32) * 2 - 1
    out = L.lobpcg_apply_A(ctx, U)
    pts = np.concatenate([[0, nx - 1, nx * (ny - 1), N - 1, N // 2], synth.sample_faces(N, 300, 4)])
    # the sampled points and their six neighbours, copied to the host
    need = set()
    for p in pts:
        x, y, z = p % nx, (p // nx) % ny, p // (nx * ny)
        need.add(int(p))
        for dx, dy, dz in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
            a, b, c = x + dx, y + dy, z + dz
            if 0 <= a < nx and 0 <= b < ny and 0 <= c < nz:
                need.add(int(a + nx * (b + ny * c)))
    idx = np.array(sorted(need))
    sparse = np.zeros((N, k))
    sparse[idx] = U[torch.from_numpy(idx).to(DEV)].cpu().numpy().astype(np.float64)
    ref = grid.laplace7_rows(dims, sparse, pts)
    got = out[torch.from_numpy(pts).to(DEV)].double().cpu().numpy()
    del ctx, U, out
    np.testing.assert_allclose(got, ref, rtol=0, atol=16 * EPS32 * 12)


# ---------------------------------------------------------------- multigrid (step 9)

@pytest.mark.parametrize("dims,levels,k", [((16, 16, 16), 3, 4), ((15, 13, 12), 3, 1), ((24, 20, 16), 4, 7),
                                           ((32, 32, 32), 3, 8), ((9, 9, 9), 1, 2)])
def test_vcycle_fp64(dims, levels, k):
    N = int(np.prod(dims))
    ctx = ctx_for(dims, 8, levels)
    B = synth.random_block(N, k, seed=13)
    out = host(L.lobpcg_apply_T(ctx, dev(B)))
    ref = mg.VCycle(dims, levels)(B)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("dims,levels,k", [((16, 16, 16), 3, 4), ((24, 20, 16), 4, 6), ((33, 17, 9), 2, 3)])
def test_vcycle_fp32(dims, levels, k):
    N = int(np.prod(dims))
    ctx = ctx_for(dims, 8, levels, L.MIXED)
    B = synth.random_block(N, k, seed=14).astype(np.float32)
    out = host(L.lobpcg_apply_T(ctx, dev(B, torch.float32)))
    ref = mg.VCycle(dims, levels)(B.astype(np.float64))
    np.testing.assert_allclose(out, ref, rtol=0, atol=2e-5 * np.abs(ref).max())


# An FP32 cycle on 3 or more columns, not a multiple of 4, runs on the count
# rounded up to a multiple of 4 (the extra columns zero); each column's
# arithmetic is the same either way, so the results are identical to the
# cycle on the columns as stored (kernel variant bit 1).  FP64 blocks in a
# mixed context take the FP32 cycle with the precision changes in its first
# and last sweeps; FP64 cycles and 1-2 columns are not rounded up.
@pytest.mark.parametrize("prec,blk", [(L.FP64, torch.float64), (L.MIXED, torch.float32),
                                      (L.MIXED, torch.float64)])
@pytest.mark.parametrize("k", [1, 3, 5, 7, 21, 23])
def test_vcycle_rounded_up_columns(prec, blk, k):
    dims, levels = (26, 19, 21), 3
    N = int(np.prod(dims))
    B = synth.random_block(N, k, seed=16 + k)
    if blk == torch.float32:
        B = B.astype(np.float32)
    outs = []
    for v in (0, 2):
        ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(levels), 24, prec)
        L.lobpcg_set_option(ctx, L.OPT_KERNELS, v)
        outs.append(L.lobpcg_apply_T(ctx, dev(B, blk)))
    assert torch.equal(outs[0], outs[1])
    ref = mg.VCycle(dims, levels)(B.astype(np.float64))
    tol = 1e-13 if prec == L.FP64 else 2e-5
    np.testing.assert_allclose(host(outs[0]), ref, rtol=0, atol=tol * np.abs(ref).max())


def test_vcycle_large_coarsest_grid_uses_global_sweeps():
    """A coarsest level too big for one workgroup's LDS (20^3 > 2048 points)."""
    dims, levels, k = (40, 40, 40), 2, 3
    ctx = ctx_for(dims, 4, levels)
    B = synth.random_block(64000, k, seed=15)
    out = host(L.lobpcg_apply_T(ctx, dev(B)))
    ref = mg.VCycle(dims, levels)(B)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


# ---------------------------------------------------------------- Gram products (steps 17-23, 3, 11, 14)

# variant 0: the kernel chosen by shape (one row per thread for a single block
# of at most 8 columns, else the LDS-staged MFMA kernel), 4: always an MFMA
# kernel, 32: the direct-load MFMA kernel, 40: the same with up to four tiles
# per wave
@pytest.mark.parametrize("variant", [0, 4, 32, 40])
@pytest.mark.parametrize("N,widths", [(4096, (8, 3, 3)), (33 * 17 * 9, (32, 32, 32)), (1000, (4,)),
                                      (70001, (16, 16)), (5003, (5, 7, 2)), (200000, (32, 17, 17)),
                                      (300007, (1,)), (12345, (32, 1, 1)), (50021, (32, 31, 31))])
def test_gram_fp64(N, widths, variant):
    dims = (N, 1, 1)
    ctx = ctx_for(dims, 32)
    L.lobpcg_set_option(ctx, L.OPT_KERNELS, variant)
    S = [synth.random_block(N, w, seed=20 + i) for i, w in enumerate(widths)]
    AS = [synth.random_block(N, w, seed=40 + i) for i, w in enumerate(widths)]
    SS, SAS = L.lobpcg_gram(ctx, [dev(s) for s in S], [dev(a) for a in AS])
    Sf, ASf = np.hstack(S), np.hstack(AS)
    refB, refA = Sf.T @ Sf, Sf.T @ ASf
    iu = np.triu_indices(Sf.shape[1])
    np.testing.assert_allclose(SS[iu], refB[iu], rtol=0, atol=1e-13 * N)
    np.testing.assert_allclose(SAS[iu], refA[iu], rtol=0, atol=1e-13 * N)
    np.testing.assert_allclose(SS, SS.T)      # lower triangle mirrored


@pytest.mark.parametrize("variant", [0, 4, 32, 48])
@pytest.mark.parametrize("N,widths", [(4096, (8, 3, 3)), (70001, (32, 32, 32)), (5003, (5, 7, 2)),
                                      (99999, (32, 1, 1)), (77777, (2,)), (3001, (17, 9)), (129, (33,)),
                                      (50021, (32, 31, 31)), (1000003, (32, 16, 16))])
def test_gram_fp32(N, widths, variant):
    ctx = ctx_for((N, 1, 1), 32, None, L.MIXED)
    L.lobpcg_set_option(ctx, L.OPT_KERNELS, variant)
    S = [synth.random_block(N, w, seed=60 + i).astype(np.float32) for i, w in enumerate(widths)]
    AS = [synth.random_block(N, w, seed=80 + i).astype(np.float32) for i, w in enumerate(widths)]
    SS, SAS = L.lobpcg_gram(ctx, [dev(s, torch.float32) for s in S], [dev(a, torch.float32) for a in AS])
    Sf, ASf = np.hstack(S).astype(np.float64), np.hstack(AS).astype(np.float64)
    iu = np.triu_indices(Sf.shape[1])
    # FP32 partial sums over at most 64-row chunks: error <= 64 eps32 sum |s||a|
    bound = 64 * EPS32 * (np.abs(Sf).T @ np.abs(ASf))
    assert np.all(np.abs(SAS - Sf.T @ ASf)[iu] <= bound[iu] + 1e-30)
    boundB = 64 * EPS32 * (np.abs(Sf).T @ np.abs(Sf))
    assert np.all(np.abs(SS - Sf.T @ Sf)[iu] <= boundB[iu] + 1e-30)


@pytest.mark.parametrize("prec", [L.FP64, L.MIXED])
@pytest.mark.parametrize("N,widths", [(4096, (8, 3, 3)), (70001, (32, 32, 32)), (5003, (5, 7, 2)),
                                      (99999, (32, 1, 1)), (20000, (16, 5)), (3001, (7, 1))])
def test_gram_paper_form(N, widths, prec):
    """Steps 17-23 in the paper's form: S^T S off the block diagonal and S^T AS
    outside the S_0-S_0 block are computed, every other entry is zero."""
    ctx = ctx_for((N, 1, 1), 32, None, L.MIXED)
    npdt, tdt = (np.float64, torch.float64) if prec == L.FP64 else (np.float32, torch.float32)
    S = [synth.random_block(N, w, seed=120 + i).astype(npdt) for i, w in enumerate(widths)]
    AS = [synth.random_block(N, w, seed=140 + i).astype(npdt) for i, w in enumerate(widths)]
    SS, SAS = L.lobpcg_gram(ctx, [dev(s, tdt) for s in S], [dev(a, tdt) for a in AS], paper_form=True)
    Sf, ASf = np.hstack(S).astype(np.float64), np.hstack(AS).astype(np.float64)
    blk = np.concatenate([np.full(w, b) for b, w in enumerate(widths)])
    wantB = blk[:, None] != blk[None, :]
    wantA = ~((blk[:, None] == 0) & (blk[None, :] == 0))
    if prec == L.FP64:
        tolB = tolA = 1e-13 * N
    else:
        tolB = 64 * EPS32 * (np.abs(Sf).T @ np.abs(Sf)).max()
        tolA = 64 * EPS32 * (np.abs(Sf).T @ np.abs(ASf)).max()
    np.testing.assert_allclose(SS[wantB], (Sf.T @ Sf)[wantB], rtol=0, atol=tolB)
    np.testing.assert_array_equal(SS[~wantB], 0.0)
    iu = np.triu(np.ones_like(wantA), 0) & wantA
    np.testing.assert_allclose(SAS[iu], (Sf.T @ ASf)[iu], rtol=0, atol=tolA)
    np.testing.assert_array_equal(SAS[~wantA], 0.0)
    np.testing.assert_array_equal(SAS, SAS.T)


def test_gram_single_block_without_AS():
    N = 12345
    ctx = ctx_for((N, 1, 1), 8)
    S = synth.random_block(N, 8, seed=3)
    SS, SAS = L.lobpcg_gram(ctx, [dev(S)])
    assert SAS is None
    np.testing.assert_allclose(SS, S.T @ S, rtol=0, atol=1e-13 * N)


def test_gram_is_deterministic():
    N = 300001
    ctx = ctx_for((N, 1, 1), 16)
    S = dev(synth.random_block(N, 16, seed=4))
    a = L.lobpcg_gram(ctx, [S, S], [S, S])
    b = L.lobpcg_gram(ctx, [S, S], [S, S])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ---------------------------------------------------------------- combinations (steps 3-4, 11, 14-15, 27-32)

# shapes: narrow (one point per thread), wide with 16-byte fragment loads,
# wide with a column map, ragged k (not a multiple of 4) and tiny N
@pytest.mark.parametrize("N,ks,kout,use_cols", [(5000, (8,), 8, False), (4099, (8, 3, 3), 8, False),
                                                (70001, (32, 32, 32), 32, False), (1234, (6, 5), 4, True),
                                                (9999, (7,), 7, True), (3001, (5, 2), 3, True), (3, (1,), 1, False),
                                                (777, (30, 9), 17, False), (2049, (12, 4), 12, True)])
@pytest.mark.parametrize("prec", [L.FP64, L.MIXED])
def test_combine(N, ks, kout, use_cols, prec):
    ctx = ctx_for((N, 1, 1), min(32, N // 3), None, L.MIXED)
    dtype = torch.float64 if prec == L.FP64 else torch.float32
    rng = np.random.default_rng(N + kout)
    ld = [k + (3 if use_cols else 0) for k in ks]
    ins = [synth.random_block(N, l, seed=i + 100).astype(np.float32 if prec == L.MIXED else np.float64)
           for i, l in enumerate(ld)]
    cols = [np.sort(rng.choice(l, size=k, replace=False)) for l, k in zip(ld, ks)] if use_cols else None
    C = rng.standard_normal((sum(ks), kout))
    add = synth.random_block(N, kout, seed=99).astype(ins[0].dtype)
    out = host(L.lobpcg_combine(ctx, [dev(x, dtype) for x in ins], C, kout, cols=cols, add=dev(add, dtype)))
    sel = [x.astype(np.float64)[:, c] if cols else x.astype(np.float64) for x, c in zip(ins, cols or [None] * len(ins))]
    ref = np.hstack(sel) @ (C.astype(np.float32).astype(np.float64) if prec == L.MIXED else C) + add
    tol = 1e-14 if prec == L.FP64 else 4 * sum(ks) * EPS32
    np.testing.assert_allclose(out, ref, rtol=0, atol=tol * (np.abs(np.hstack(sel)) @ np.abs(C)).max())


# blocks wider than 32 columns: the inputs go to the kernels in pieces of at
# most 32 columns and the outputs in chunks of 32 (or 16) columns
@pytest.mark.parametrize("N,ks,kout,use_cols", [(20011, (50,), 50, False), (9001, (64, 40, 33), 64, True),
                                                (5003, (100, 100, 100), 100, False), (3001, (33, 7), 40, False),
                                                (777, (128,), 3, True), (4099, (5, 70), 128, False)])
@pytest.mark.parametrize("prec", [L.FP64, L.MIXED])
def test_combine_wide(N, ks, kout, use_cols, prec):
    ctx = ctx_for((N, 1, 1), min(128, N // 3), None, L.MIXED)
    dtype = torch.float64 if prec == L.FP64 else torch.float32
    rng = np.random.default_rng(N + kout)
    ld = [k + (3 if use_cols and k + 3 <= 128 else 0) for k in ks]
    ins = [synth.random_block(N, l, seed=i + 200).astype(np.float32 if prec == L.MIXED else np.float64)
           for i, l in enumerate(ld)]
    cols = [np.sort(rng.choice(l, size=k, replace=False)) for l, k in zip(ld, ks)] if use_cols else None
    C = rng.standard_normal((sum(ks), kout))
    add = synth.random_block(N, kout, seed=98).astype(ins[0].dtype)
    out = host(L.lobpcg_combine(ctx, [dev(x, dtype) for x in ins], C, kout, cols=cols, add=dev(add, dtype)))
    sel = [x.astype(np.float64)[:, c] if cols else x.astype(np.float64) for x, c in zip(ins, cols or [None] * len(ins))]
    ref = np.hstack(sel) @ (C.astype(np.float32).astype(np.float64) if prec == L.MIXED else C) + add
    tol = 1e-14 if prec == L.FP64 else 4 * sum(ks) * EPS32
    np.testing.assert_allclose(out, ref, rtol=0, atol=tol * (np.abs(np.hstack(sel)) @ np.abs(C)).max())


@pytest.mark.parametrize("N,widths", [(20011, (50, 50, 50)), (5003, (100, 100, 100)), (3001, (97, 45, 13)),
                                      (9001, (128,)), (7777, (40, 33))])
@pytest.mark.parametrize("prec", [L.FP64, L.MIXED])
@pytest.mark.parametrize("paper", [False, True])
def test_gram_wide(N, widths, prec, paper):
    """Gram products wider than one launch's tables: the tiles are spread over
    several launches."""
    if paper and len(widths) < 2:
        pytest.skip("the paper's form needs two blocks")
    ctx = ctx_for((N, 1, 1), min(128, N // 3), None, L.MIXED)
    npdt, tdt = (np.float64, torch.float64) if prec == L.FP64 else (np.float32, torch.float32)
    S = [synth.random_block(N, w, seed=220 + i).astype(npdt) for i, w in enumerate(widths)]
    AS = [synth.random_block(N, w, seed=240 + i).astype(npdt) for i, w in enumerate(widths)]
    SS, SAS = L.lobpcg_gram(ctx, [dev(x, tdt) for x in S], [dev(a, tdt) for a in AS], paper_form=paper)
    Sf, ASf = np.hstack(S).astype(np.float64), np.hstack(AS).astype(np.float64)
    blk = np.concatenate([np.full(w, b) for b, w in enumerate(widths)])
    wantB = blk[:, None] != blk[None, :] if paper else np.ones((len(blk), len(blk)), bool)
    wantA = ~((blk[:, None] == 0) & (blk[None, :] == 0)) if paper else np.ones_like(wantB)
    if prec == L.FP64:
        tolB = 1e-13 * N * np.ones_like(SS)
        tolA = 1e-13 * N * np.ones_like(SS)
    else:
        tolB = 64 * EPS32 * (np.abs(Sf).T @ np.abs(Sf)) + 1e-30
        tolA = 64 * EPS32 * (np.abs(Sf).T @ np.abs(ASf)) + 1e-30
    assert np.all(np.abs(SS - Sf.T @ Sf)[wantB] <= tolB[wantB])
    np.testing.assert_array_equal(SS[~wantB], 0.0)
    iu = np.triu(np.ones_like(wantA), 0) & wantA
    assert np.all(np.abs(SAS - Sf.T @ ASf)[iu] <= tolA[iu])
    np.testing.assert_array_equal(SAS[~wantA], 0.0)
    np.testing.assert_array_equal(SAS, SAS.T)


# ---------------------------------------------------------------- the fused update (steps 25-33 and 7)

def update_reference(X, AX, W, AW, P, AP, C, theta, J, norm_A):
    """Steps 25-33 and 7 as plain FP64 matrix algebra."""
    m, nW = X.shape[1], W.shape[1]
    CX, CW, CP = C[:m], C[m:m + nW], C[m + nW:]
    Pn = W @ CW + (P @ CP if P is not None else 0.0)
    APn = AW @ CW + (AP @ CP if P is not None else 0.0)
    Xn, AXn = X @ CX + Pn, AX @ CX + APn
    R = AXn - Xn * theta[None, :]
    rho = np.linalg.norm(R, axis=0) / (norm_A * np.linalg.norm(Xn, axis=0))
    return Xn, AXn, Pn[:, J], APn[:, J], R[:, J], rho


# shapes: the LDS-pipelined FP32 kernel (m a multiple of 4, at most 32
# columns: W and P widths that are and are not multiples of 4, with and
# without P, ragged last groups of 16 points, a grid of fewer points than one
# workgroup pass), the fragment kernel (m = 30), the narrow kernel (m = 8) and
# the wide kernel (m = 48)
# (N, m, nW, nP, nJ, ldP): ldP > nP takes P as a column list of a wider
# block (the solver's active directions)
UPDATE_SHAPES = [(5003, 32, 32, 32, 32, 32), (70001, 32, 20, 20, 20, 20), (4099, 32, 23, 23, 21, 23),
                 (777, 32, 32, 0, 32, 0), (3001, 12, 7, 5, 7, 5), (37, 12, 5, 5, 4, 5), (2049, 30, 17, 17, 15, 17),
                 (1000, 8, 5, 3, 5, 3), (3000, 48, 40, 40, 33, 40), (9001, 32, 21, 21, 21, 24),
                 (4097, 32, 26, 26, 20, 31), (4097, 32, 13, 13, 13, 16),
                 # several 16-point groups per wave (the steady state of the
                 # FP32 update's load pipeline), narrow and wide W and P
                 (600011, 32, 13, 13, 11, 16), (600011, 32, 24, 24, 20, 28), (1200007, 16, 9, 9, 9, 12),
                 # few active columns (P, AP and W leave as compact rows)
                 (600011, 32, 1, 1, 1, 1), (70001, 32, 3, 3, 3, 8), (600011, 32, 6, 6, 6, 6),
                 (4099, 16, 2, 0, 2, 0), (1003, 20, 4, 2, 3, 4)]


def update_inputs(N, m, nW, nP, nJ, ldP, npdt):
    rng = np.random.default_rng(N + 7 * m + nW + ldP)
    blk = lambda w, s: synth.random_block(N, w, seed=s).astype(npdt)
    X, AX, W, AW = blk(m, 1), blk(m, 2), blk(nW, 3), blk(nW, 4)
    P, AP = (blk(ldP, 5), blk(ldP, 6)) if nP else (None, None)
    Pcols = np.sort(rng.choice(ldP, size=nP, replace=False)) if ldP > nP else None
    C = rng.standard_normal((m + nW + nP, m)) / np.sqrt(m)
    theta = np.sort(rng.uniform(0.01, 2.0, m))
    J = np.sort(rng.choice(m, size=nJ, replace=False))
    return X, AX, W, AW, P, AP, Pcols, C, theta, J


@pytest.mark.parametrize("N,m,nW,nP,nJ,ldP", UPDATE_SHAPES)
@pytest.mark.parametrize("prec", [L.FP64, L.MIXED])
def test_update(N, m, nW, nP, nJ, ldP, prec):
    ctx = ctx_for((N, 1, 1), m, None, L.MIXED)
    npdt = np.float64 if prec == L.FP64 else np.float32
    dtype = torch.float64 if prec == L.FP64 else torch.float32
    X, AX, W, AW, P, AP, Pcols, C, theta, J = update_inputs(N, m, nW, nP, nJ, ldP, npdt)
    d = lambda a: dev(a, dtype) if a is not None else None
    got = L.lobpcg_update(ctx, d(X), d(AX), d(W), d(AW), d(P), d(AP), C, theta, J, 12.0, Pcols=Pcols)
    f64 = lambda a: a.astype(np.float64) if a is not None else None
    if Pcols is not None:
        P, AP = P[:, Pcols], AP[:, Pcols]
    # the FP32 kernels multiply by the coefficients rounded to FP32
    Cr = C.astype(np.float32).astype(np.float64) if prec == L.MIXED else C
    ref = update_reference(f64(X), f64(AX), f64(W), f64(AW), f64(P), f64(AP), Cr, theta, J, 12.0)
    K = C.shape[0]
    S = np.hstack([f64(X), f64(W)] + ([f64(P)] if nP else []))
    scale = (np.abs(S) @ np.abs(Cr)).max()
    tol = (1e-14 if prec == L.FP64 else 4 * K * EPS32) * scale
    names = ["X'", "AX'", "P'_J", "AP'_J", "W'_J"]
    for name, g, r in zip(names, got[:5], ref[:5]):
        assert g.shape == r.shape, name
        # W' = AX' - theta X' adds the error of X' times theta <= 2
        np.testing.assert_allclose(host(g), r, rtol=0, atol=3 * tol, err_msg=name)
    np.testing.assert_allclose(got[5], ref[5], rtol=1e-12 if prec == L.FP64 else 1e-4)


@pytest.mark.parametrize("N,m,nW,nP,nJ,ldP", [s for s in UPDATE_SHAPES if s[1] % 4 == 0 and 8 < s[1] <= 32])
def test_update_kernels_agree(N, m, nW, nP, nJ, ldP):
    """The LDS-pipelined FP32 update, the same with P, AP and W stored per
    MFMA fragment (kernel variant bit 6) and the fragment kernel (bit 0) take
    the same products in the same order: identical blocks."""
    X, AX, W, AW, P, AP, Pcols, C, theta, J = update_inputs(N, m, nW, nP, nJ, ldP, np.float32)
    d = lambda a: dev(a, torch.float32) if a is not None else None
    res = []
    for v in (0, 1, 64):
        ctx = L.lobpcg_setup(L.Op(N, 1, 1), L.Precond(None), m, L.MIXED)
        L.lobpcg_set_option(ctx, L.OPT_KERNELS, v)
        res.append(L.lobpcg_update(ctx, d(X), d(AX), d(W), d(AW), d(P), d(AP), C, theta, J, 12.0, Pcols=Pcols))
    for r in res[1:]:
        for a, b in zip(res[0][:5], r[:5]):
            assert torch.equal(a, b)
        np.testing.assert_allclose(res[0][5], r[5], rtol=1e-13)


def test_update_argument_errors():
    """lobpcg_update rejects bad sizes, repeated or out-of-range active
    columns, P column lists out of range and outputs that alias inputs,
    before launching anything."""
    N, m = 3001, 12
    ctx = ctx_for((N, 1, 1), m, None, L.MIXED)
    X, AX, W, AW, P, AP, Pcols, C, theta, J = update_inputs(N, m, 7, 5, 7, 8, np.float64)
    d = lambda a: dev(a) if a is not None else None
    dX, dAX, dW, dAW, dP, dAP = d(X), d(AX), d(W), d(AW), d(P), d(AP)
    ok = L.lobpcg_update(ctx, dX, dAX, dW, dAW, dP, dAP, C, theta, J, 12.0, Pcols=Pcols)
    assert ok[5].shape == (m,)
    bad = [dict(J=[0, 0, 1]), dict(J=[m]), dict(Pcols=[0, 1, 2, 3, 8]), dict(Pcols=[-1, 1, 2, 3, 4]),
           dict(norm_A=0.0)]
    for b in bad:
        kw = dict(J=J, Pcols=Pcols, norm_A=12.0)
        kw.update(b)
        with pytest.raises(L.LobpcgError):
            L.lobpcg_update(ctx, dX, dAX, dW, dAW, dP, dAP, C, theta, kw["J"], kw["norm_A"], Pcols=kw["Pcols"])
    # an output aliasing an input, through the C ABI directly
    lib = L.lib()
    Cn = np.ascontiguousarray(C)
    th = np.ascontiguousarray(theta)
    Jn = np.ascontiguousarray(J, dtype=np.int32)
    pc = np.ascontiguousarray(Pcols, dtype=np.int32)
    rho = np.zeros(m)
    outs = [torch.empty_like(dX), torch.empty_like(dAX)] + [torch.empty((N, len(J)), dtype=dX.dtype, device=DEV)
                                                            for _ in range(3)]
    for k in range(5):
        o = [t.data_ptr() for t in outs]
        o[k] = dW.data_ptr()
        s = lib.lobpcg_update(ctx.h, L.F64, dX.data_ptr(), dAX.data_ptr(), dW.data_ptr(), dAW.data_ptr(), 7,
                              dP.data_ptr(), dAP.data_ptr(), 8, pc.ctypes.data, 5, Cn.ctypes.data, th.ctypes.data,
                              Jn.ctypes.data, len(J), 12.0, *o, rho.ctypes.data)
        assert s == L.ERR_ARG


# ---------------------------------------------------------------- residual and norms (steps 7-8)

@pytest.mark.parametrize("N,m,J", [(4096, 4, [0, 1, 2, 3]), (70001, 32, list(range(0, 32, 3))), (999, 7, [6]),
                                   (5000, 8, [])])
@pytest.mark.parametrize("prec", [L.FP64, L.MIXED])
def test_residual(N, m, J, prec):
    ctx = ctx_for((N, 1, 1), m, None, L.MIXED)
    npdt = np.float64 if prec == L.FP64 else np.float32
    dtype = torch.float64 if prec == L.FP64 else torch.float32
    X = synth.random_block(N, m, seed=1).astype(npdt)
    AX = synth.random_block(N, m, seed=2).astype(npdt)
    lam = np.linspace(0.1, 2.0, m)
    W, rho = L.lobpcg_residual(ctx, dev(X, dtype), dev(AX, dtype), lam, J, 12.0)
    R = AX.astype(np.float64) - X.astype(np.float64) * lam[None, :]
    ref_rho = np.linalg.norm(R, axis=0) / (12.0 * np.linalg.norm(X.astype(np.float64), axis=0))
    np.testing.assert_allclose(rho, ref_rho, rtol=1e-12)
    if J:
        np.testing.assert_allclose(host(W), R[:, J], rtol=0, atol=(1e-15 if prec == L.FP64 else 1e-7) * 3)


# ---------------------------------------------------------------- eigenvalue adjoint

@pytest.mark.parametrize("dims,m", [((12, 10, 8), 4), ((7, 9, 5), 3), ((32, 32, 32), 8)])
def test_eig_grad_faces(dims, m):
    N = int(np.prod(dims))
    kx, ky, kz = synth.gaussian_field_faces(*dims, seed=3)
    A = L.Op(*dims, dev(kx), dev(ky), dev(kz))
    ctx = L.lobpcg_setup(A, L.Precond(None), m, L.FP64)
    X = synth.random_block(N, m, seed=5)
    gbar = np.linspace(-1, 2, m)
    got = [host(t) for t in L.lobpcg_eig_grad_k(ctx, dev(X), gbar)]
    ref = grid.eig_grad_faces(dims, X, gbar)
    for a, b in zip(got, ref):
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-13 * np.abs(b).max())
