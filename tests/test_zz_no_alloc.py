"""The allocation-free residual entry point against the context-based one.

lobpcg_residual_noalloc keeps its kernels' scratch in a fixed device array
instead of a context's workspace; called twice in a row (the second call
with a smaller problem, so that the scratch holds the first call's sums), it
must give the same W and residual norms as lobpcg_residual on the same
inputs: the same kernels with the same summation order.
"""
import ctypes

import numpy as np
import pytest
import torch

import synth

L = pytest.importorskip("paper_0705_2626_amd")
pytestmark = pytest.mark.gpu


def context_residual(dims, m, dt, X, AX, lam, J):
    ctx = L.lobpcg_setup(L.Op(*dims), L.Precond(None), m, L.MIXED if dt == L.F32 else L.FP64)
    N = X.shape[0]
    tdt = torch.float32 if dt == L.F32 else torch.float64
    W = torch.zeros((N, max(len(J), 1)), dtype=tdt, device="cuda")
    rho = np.zeros(m)
    Jh = np.asarray(J, dtype=np.int32)
    s = L.lib().lobpcg_residual(ctx.h, dt, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(AX.data_ptr()), m,
                                lam.ctypes.data_as(ctypes.c_void_p), Jh.ctypes.data_as(ctypes.c_void_p), len(J),
                                12.0, ctypes.c_void_p(W.data_ptr()), rho.ctypes.data_as(ctypes.c_void_p))
    assert s == L.OK
    return W, rho


def noalloc_residual(m, dt, X, AX, lam, J):
    N = X.shape[0]
    tdt = torch.float32 if dt == L.F32 else torch.float64
    W = torch.zeros((N, max(len(J), 1)), dtype=tdt, device="cuda")
    jpos = -np.ones(m, dtype=np.int32)
    for i, j in enumerate(J):
        jpos[j] = i
    d_lam = torch.from_numpy(lam).cuda()
    d_jpos = torch.from_numpy(jpos).cuda()
    d_rho = torch.zeros(m, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream()
    s = L.lib().lobpcg_residual_noalloc(dt, N, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(AX.data_ptr()), m,
                                        ctypes.c_void_p(d_lam.data_ptr()), ctypes.c_void_p(d_jpos.data_ptr()),
                                        len(J), 12.0, ctypes.c_void_p(W.data_ptr()),
                                        ctypes.c_void_p(d_rho.data_ptr()), ctypes.c_void_p(st.cuda_stream))
    assert s == L.OK
    torch.cuda.synchronize()
    return W, d_rho.cpu().numpy()


@pytest.mark.parametrize("dt", [0, 1])
def test_noalloc_residual_matches_context_residual_twice(dt):
    cases = [((40, 36, 32), 24, [0, 3, 5, 6, 10, 11, 17, 23]),    # 46080 points: many workgroups
             ((9, 7, 5), 5, [1, 4])]                              # then a smaller one
    tdt = torch.float32 if dt == L.F32 else torch.float64
    for dims, m, J in cases:
        N = int(np.prod(dims))
        X = torch.from_numpy(synth.random_block(N, m, seed=1)).to(device="cuda", dtype=tdt)
        AX = torch.from_numpy(synth.random_block(N, m, seed=2)).to(device="cuda", dtype=tdt)
        lam = np.linspace(0.1, 0.9, m)
        Wc, rc = context_residual(dims, m, dt, X, AX, lam, J)
        Wn, rn = noalloc_residual(m, dt, X, AX, lam, J)
        np.testing.assert_allclose(rn, rc, rtol=1e-15, atol=0)
        assert torch.equal(Wn, Wc)


def test_noalloc_residual_rejects_bad_arguments():
    X = torch.zeros((64, 4), dtype=torch.float64, device="cuda")
    d_lam = torch.zeros(4, dtype=torch.float64, device="cuda")
    d_jpos = torch.full((4,), -1, dtype=torch.int32, device="cuda")
    d_rho = torch.zeros(4, dtype=torch.float64, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    lib = L.lib()
    assert lib.lobpcg_residual_noalloc(0, 64, p(X), p(X), 129, p(d_lam), p(d_jpos), 0, 12.0, None, p(d_rho), None) \
        == L.ERR_ARG                                             # wider than the scratch holds
    assert lib.lobpcg_residual_noalloc(0, 64, p(X), p(X), 4, p(d_lam), p(d_jpos), 2, 12.0, None, p(d_rho), None) \
        == L.ERR_ARG                                             # nJ > 0 without W
    assert lib.lobpcg_residual_noalloc(2, 64, p(X), p(X), 4, p(d_lam), p(d_jpos), 0, 12.0, None, p(d_rho), None) \
        == L.ERR_ARG                                             # bad element type
    assert lib.lobpcg_residual_noalloc(0, 64, p(X), p(X), 4, p(d_lam), p(d_jpos), 0, 0.0, None, p(d_rho), None) \
        == L.ERR_ARG                                             # norm_A <= 0
