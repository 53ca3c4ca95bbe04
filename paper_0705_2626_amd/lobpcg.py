"""Python binding of liblobpcg.so (argument marshalling only).

Every entry point has the name of the C function it calls.  Device memory
comes from PyTorch tensors on the ROCm device; the library runs all of its
kernels on the stream the context was created with (PyTorch's current
stream by default).  Nothing here computes: if the shared library is not
built, the first call raises.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblobpcg.so")

OK, NOT_CONVERGED = 0, 1
ERR_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_CHOL, ERR_RR, ERR_NONFINITE, ERR_HIP = -1, -2, -3, -4, -5, -6, -7
OP_LAPLACE7, OP_VARCOEF7, OP_DIAG, OP_MASS7 = 0, 1, 2, 3
PC_NONE, PC_GMG_V = 0, 1
FP64, MIXED = 0, 1
F64, F32 = 0, 1
OPT_SWITCH_TOL, OPT_STALL_WINDOW, OPT_STALL_FACTOR, OPT_PROFILE, OPT_REACTIVATE, OPT_KERNELS = 0, 1, 2, 3, 4, 5
OPT_FP32_EXPLICIT_GRAM = 6
OPT_FOLD_CHOLQR = 7
OPT_FP64_EXPLICIT_GRAM = 8
OPT_LOCK_GAP = 9
OPT_NWANT = 10
OPT_FP32_EXPLICIT_ABOVE = 11
STEP_NAMES = ["residual", "precond", "ortho", "apply_A", "gram", "rr_host", "update", "other"]


class LobpcgError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s: %s (%d)" % (where, status_string(status), status))


class _Op(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("kind", ctypes.c_int),
                ("kx", ctypes.c_void_p), ("ky", ctypes.c_void_p), ("kz", ctypes.c_void_p),
                ("diag", ctypes.c_void_p), ("b0", ctypes.c_double), ("b1", ctypes.c_double)]


class _Precond(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("levels", ctypes.c_int), ("nu_pre", ctypes.c_int),
                ("nu_post", ctypes.c_int), ("coarse_sweeps", ctypes.c_int), ("omega", ctypes.c_double)]


NSTEP = 8


class _Stats(ctypes.Structure):
    _fields_ = [("iters_total", ctypes.c_int), ("iters_fp32", ctypes.c_int), ("iters_fp64", ctypes.c_int),
                ("restarts", ctypes.c_int), ("status", ctypes.c_int), ("solve_ms", ctypes.c_double),
                ("step_ms", ctypes.c_double * NSTEP), ("step_calls", ctypes.c_int * NSTEP),
                ("step_bytes", ctypes.c_double * NSTEP)]


_lib = None


def lib():
    """The loaded shared library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblobpcg.so is not built (run __graft_entry__.build()); "
                               "there is no fallback implementation")
        L = ctypes.CDLL(LIB_PATH)
        i, d, p, sz = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
        P = ctypes.POINTER
        sig = {
            "lobpcg_workspace_bytes": (i, [P(_Op), P(_Op), P(_Precond), i, i, P(sz)]),
            "lobpcg_setup": (i, [P(p), P(_Op), P(_Op), P(_Precond), i, i, p, sz, p]),
            "lobpcg_solve": (i, [p, P(_Op), P(_Op), P(_Precond), p, i, d, i, p, p, p, p, p]),
            "lobpcg_solve_constrained": (i, [p, P(_Op), P(_Op), P(_Precond), p, i, p, i, d, i, p, p, p, p, p]),
            "lobpcg_eig_grad_k": (i, [p, p, p, i, p, p, p]),
            "lobpcg_destroy": (None, [p]),
            "lobpcg_status_string": (ctypes.c_char_p, [i]),
            "lobpcg_set_option": (i, [p, i, d]),
            "lobpcg_get_stats": (i, [p, P(_Stats)]),
            "lobpcg_apply_A": (i, [p, P(_Op), i, p, p, i]),
            "lobpcg_apply_T": (i, [p, i, p, p, i]),
            "lobpcg_gram": (i, [p, i, i, p, p, p, i, p, p]),
            "lobpcg_combine": (i, [p, i, i, p, p, p, p, p, i, p, p]),
            "lobpcg_update": (i, [p, i, p, p, p, p, i, p, p, i, p, i, p, p, p, i, d, p, p, p, p, p, p]),
            "lobpcg_residual": (i, [p, i, p, p, i, p, p, i, d, p, p]),
            "lobpcg_residual_noalloc": (i, [i, ctypes.c_longlong, p, p, i, p, p, i, d, p, p, p]),
            "lobpcg_dense_chol": (i, [i, p, p]),
            "lobpcg_dense_rr": (i, [i, i, p, p, p, p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def status_string(s):
    return lib().lobpcg_status_string(int(s)).decode()


def _check(s, where, allow=(OK,)):
    if s not in allow:
        raise LobpcgError(s, where)
    return s


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Op:
    """Operator descriptor: the 7-point Laplacian, or -div(k grad u) with
    FP64 device face arrays kx (nz,ny,nx+1), ky (nz,ny+1,nx), kz (nz+1,ny,nx)."""

    def __init__(self, nx, ny, nz, kx=None, ky=None, kz=None):
        self.dims = (int(nx), int(ny), int(nz))
        self.k = None
        if kx is not None:
            self.k = tuple(t.contiguous() for t in (kx, ky, kz))
            shapes = ((nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx))
            for t, shp in zip(self.k, shapes):
                if t.dtype != torch.float64 or not t.is_cuda:
                    raise ValueError("face arrays must be float64 device tensors")
                if t.numel() != shp[0] * shp[1] * shp[2]:
                    raise ValueError("face array of %d entries, expected shape %s" % (t.numel(), shp))

    @property
    def N(self):
        return self.dims[0] * self.dims[1] * self.dims[2]

    def c(self):
        o = _Op(*self.dims, OP_LAPLACE7 if self.k is None else OP_VARCOEF7, None, None, None, None)
        if self.k is not None:
            o.kx, o.ky, o.kz = (t.data_ptr() for t in self.k)
        return o


class Diag:
    """B = diag(d) for A x = lambda B x: d an (N,) positive float64 device
    tensor on the grid of A (e.g. a lumped mass matrix)."""

    def __init__(self, nx, ny, nz, d):
        self.dims = (int(nx), int(ny), int(nz))
        if not isinstance(d, torch.Tensor) or d.dtype != torch.float64 or not d.is_cuda:
            raise ValueError("the diagonal must be a float64 device tensor")
        if d.numel() != self.dims[0] * self.dims[1] * self.dims[2]:
            raise ValueError("the diagonal must have N entries")
        self.d = d.contiguous()

    def c(self):
        return _Op(*self.dims, OP_DIAG, None, None, None, self.d.data_ptr())


class Mass7:
    """B = the 7-point mass-type operator on the grid of A: (B u)_p = b0 u_p
    + b1 (sum of u over the axis neighbours of p), b0 > 6 |b1|."""

    def __init__(self, nx, ny, nz, b0, b1):
        self.dims = (int(nx), int(ny), int(nz))
        self.b0, self.b1 = float(b0), float(b1)

    def c(self):
        return _Op(*self.dims, OP_MASS7, None, None, None, None, self.b0, self.b1)


class Precond:
    """Multigrid V-cycle descriptor (levels=0 or None: no preconditioner)."""

    def __init__(self, levels=None, nu_pre=2, nu_post=2, coarse_sweeps=20, omega=2.0 / 3.0):
        self.levels, self.nu_pre, self.nu_post, self.coarse_sweeps, self.omega = \
            levels, nu_pre, nu_post, coarse_sweeps, omega

    def c(self):
        if not self.levels:
            return _Precond(PC_NONE, 0, 0, 0, 0, 0.0)
        return _Precond(PC_GMG_V, self.levels, self.nu_pre, self.nu_post, self.coarse_sweeps, self.omega)


def _bref(B):
    return ctypes.byref(B.c()) if B is not None else None


def lobpcg_workspace_bytes(A, T, m, precision, B=None):
    n = ctypes.c_size_t(0)
    _check(lib().lobpcg_workspace_bytes(ctypes.byref(A.c()), _bref(B), ctypes.byref(T.c()), int(m),
                                        int(precision), ctypes.byref(n)), "lobpcg_workspace_bytes")
    return n.value


class Context:
    """A solver context with its device workspace (a uint8 tensor it owns)."""

    def __init__(self, A, T, m, precision, device="cuda", stream=None, B=None):
        self.A, self.T, self.m, self.precision, self.B = A, T, int(m), int(precision), B
        nbytes = lobpcg_workspace_bytes(A, T, m, precision, B)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.h = ctypes.c_void_p()
        _check(lib().lobpcg_setup(ctypes.byref(self.h), ctypes.byref(A.c()), _bref(B), ctypes.byref(T.c()), self.m,
                                  self.precision, ctypes.c_void_p(self._ws_ptr), ctypes.c_size_t(nbytes),
                                  ctypes.c_void_p(self.stream.cuda_stream)), "lobpcg_setup")

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:
            _lib.lobpcg_destroy(h)
            self.h = None

    @property
    def N(self):
        return self.A.N


def lobpcg_setup(A, T, m, precision=FP64, device="cuda", stream=None, B=None):
    """Context for A x = lambda x, or A x = lambda B x with B a Diag or a Mass7 (FP64 or mixed)."""
    return Context(A, T, m, precision, device, stream, B)


def lobpcg_set_option(ctx, key, value):
    _check(lib().lobpcg_set_option(ctx.h, int(key), float(value)), "lobpcg_set_option")


def lobpcg_get_stats(ctx):
    s = _Stats()
    _check(lib().lobpcg_get_stats(ctx.h, ctypes.byref(s)), "lobpcg_get_stats")
    return {"iters_total": s.iters_total, "iters_fp32": s.iters_fp32, "iters_fp64": s.iters_fp64,
            "restarts": s.restarts, "status": s.status, "solve_ms": s.solve_ms,
            "step_ms": dict(zip(STEP_NAMES, list(s.step_ms))),
            "step_calls": dict(zip(STEP_NAMES, list(s.step_calls))),
            "step_bytes": dict(zip(STEP_NAMES, list(s.step_bytes)))}


class SolveResult:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def lobpcg_solve(ctx, X0, tol, maxit, A=None, hist=True, raise_on_error=True, Y=None):
    """Smallest eigenpairs.  X0: (N, m) float64 device tensor; Y: optional
    (N, l) float64 device tensor of constraints (lobpcg_solve_constrained).
    Returns a SolveResult(status, lam, X, hist, iters, resid)."""
    A = A if A is not None else ctx.A
    N, m = ctx.N, ctx.m
    X0 = _blk(ctx, X0, "X0", m, torch.float64)
    X = torch.empty_like(X0)
    lam = np.zeros(m)
    H = np.zeros((max(maxit, 1), m)) if hist else None
    iters = ctypes.c_int(0)
    res = np.zeros(m)
    tail = (m, float(tol), int(maxit), _np_ptr(lam), _ptr(X), _np_ptr(H) if hist else None, ctypes.byref(iters),
            _np_ptr(res))
    if Y is None:
        s = lib().lobpcg_solve(ctx.h, ctypes.byref(A.c()), _bref(ctx.B), ctypes.byref(ctx.T.c()), _ptr(X0), *tail)
    else:
        Y = _blk(ctx, Y, "Y", dtype=torch.float64)
        s = lib().lobpcg_solve_constrained(ctx.h, ctypes.byref(A.c()), _bref(ctx.B), ctypes.byref(ctx.T.c()),
                                           _ptr(Y), int(Y.shape[1]), _ptr(X0), *tail)
    if raise_on_error:
        _check(s, "lobpcg_solve", allow=(OK, NOT_CONVERGED))
    return SolveResult(status=s, lam=lam, X=X, hist=H[:iters.value] if hist else None, iters=iters.value,
                       resid=res)


def lobpcg_eig_grad_k(ctx, X, gbar):
    """Face gradients sum_i gbar_i d lambda_i / d k_f as three float64 device tensors."""
    nx, ny, nz = ctx.A.dims
    X = _blk(ctx, X, "X", dtype=torch.float64)
    gb = np.ascontiguousarray(np.asarray(gbar, dtype=np.float64))
    gkx = torch.empty((nz, ny, nx + 1), dtype=torch.float64, device=X.device)
    gky = torch.empty((nz, ny + 1, nx), dtype=torch.float64, device=X.device)
    gkz = torch.empty((nz + 1, ny, nx), dtype=torch.float64, device=X.device)
    _check(lib().lobpcg_eig_grad_k(ctx.h, _ptr(X), _np_ptr(gb), int(X.shape[1]), _ptr(gkx), _ptr(gky), _ptr(gkz)),
           "lobpcg_eig_grad_k")
    return gkx, gky, gkz


def _blk(ctx, t, what, width=None, dtype=None):
    """Check that t is an (N, k) contiguous 16-byte-aligned device block."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError("%s must be a device tensor" % what)
    if t.dim() != 2 or t.shape[0] != ctx.N:
        raise ValueError("%s must have shape (%d, k), got %s" % (what, ctx.N, tuple(t.shape)))
    if width is not None and t.shape[1] != width:
        raise ValueError("%s must have %d columns" % (what, width))
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must be %s" % (what, dtype))
    if t.dtype not in (torch.float32, torch.float64):
        raise ValueError("%s must be float32 or float64" % what)
    t = t.contiguous()
    if t.data_ptr() % 16:
        t = t.clone()
    return t


def _dt(t):
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise ValueError("blocks must be float32 or float64")


def lobpcg_apply_A(ctx, X, A=None):
    A = A if A is not None else ctx.A
    X = _blk(ctx, X, "X")
    out = torch.empty_like(X)
    _check(lib().lobpcg_apply_A(ctx.h, ctypes.byref(A.c()), _dt(X), _ptr(X), _ptr(out), int(X.shape[1])),
           "lobpcg_apply_A")
    return out


def lobpcg_apply_T(ctx, X):
    X = _blk(ctx, X, "X")
    out = torch.empty_like(X)
    _check(lib().lobpcg_apply_T(ctx.h, _dt(X), _ptr(X), _ptr(out), int(X.shape[1])), "lobpcg_apply_T")
    return out


def lobpcg_gram(ctx, S, AS=None, paper_form=False):
    """(S^T S, S^T AS) for lists of (N, w_i) blocks, as float64 numpy arrays
    (paper_form: only the entries the paper's form of steps 17-23 computes)."""
    S = [_blk(ctx, s, "S", dtype=S[0].dtype) for s in S]
    n = len(S)
    dt = _dt(S[0])
    sp = (ctypes.c_void_p * 3)(*[s.data_ptr() for s in S])
    w = (ctypes.c_int * 3)(*[int(s.shape[1]) for s in S])
    K = sum(int(s.shape[1]) for s in S)
    SS = np.zeros((K, K))
    SAS = None
    ap = None
    if AS is not None:
        AS = [_blk(ctx, a, "AS", s.shape[1], S[0].dtype) for a, s in zip(AS, S)]
        ap = (ctypes.c_void_p * 3)(*[a.data_ptr() for a in AS])
        SAS = np.zeros((K, K))
    _check(lib().lobpcg_gram(ctx.h, dt, n, sp, ap, w, int(bool(paper_form)), _np_ptr(SS),
                             _np_ptr(SAS) if SAS is not None else None), "lobpcg_gram")
    return SS, SAS


def lobpcg_combine(ctx, ins, C, kout, cols=None, add=None):
    """out = sum_i ins[i][:, cols[i]] @ C_i (+ add), C stacked (sum k_i, kout)."""
    ins = [_blk(ctx, x, "input", dtype=ins[0].dtype) for x in ins]
    n = len(ins)
    N = ins[0].shape[0]
    ld = [int(x.shape[1]) for x in ins]
    cols = cols or [None] * n
    ks = [len(c) if c is not None else ld[i] for i, c in enumerate(cols)]
    keep = [np.ascontiguousarray(np.asarray(c, dtype=np.int32)) if c is not None else None for c in cols]
    colp = (ctypes.c_void_p * 3)(*[k.ctypes.data if k is not None else None for k in keep])
    Cn = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
    if Cn.shape != (sum(ks), kout):
        raise ValueError("C must have shape (%d, %d)" % (sum(ks), kout))
    if add is not None:
        add = _blk(ctx, add, "add", kout, ins[0].dtype)
    out = torch.empty((N, kout), dtype=ins[0].dtype, device=ins[0].device)
    _check(lib().lobpcg_combine(ctx.h, _dt(ins[0]), n, (ctypes.c_void_p * 3)(*[x.data_ptr() for x in ins]),
                                (ctypes.c_int * 3)(*ld), colp, (ctypes.c_int * 3)(*ks), _np_ptr(Cn), int(kout),
                                _ptr(add) if add is not None else None, _ptr(out)), "lobpcg_combine")
    return out


def lobpcg_update(ctx, X, AX, W, AW, P, AP, C, theta, J, norm_A, Pcols=None):
    """The fused update of steps 25-33 and 7: returns (X', AX', P'_J, AP'_J,
    W'_J, rho) for C = [C_X; C_W; C_P] of shape (m + nW + nP, m); P and AP
    may be None (no P terms); Pcols: the columns of P, AP that form the
    P block (nP = len(Pcols)), else all of them."""
    X = _blk(ctx, X, "X", ctx.m)
    AX = _blk(ctx, AX, "AX", ctx.m, X.dtype)
    W = _blk(ctx, W, "W", dtype=X.dtype)
    AW = _blk(ctx, AW, "AW", W.shape[1], X.dtype)
    nW = int(W.shape[1])
    if P is not None:
        P = _blk(ctx, P, "P", dtype=X.dtype)
        AP = _blk(ctx, AP, "AP", P.shape[1], X.dtype)
    ldP = int(P.shape[1]) if P is not None else 0
    pc = np.ascontiguousarray(np.asarray(Pcols, dtype=np.int32)) if (P is not None and Pcols is not None) else None
    nP = len(pc) if pc is not None else ldP
    m = ctx.m
    Cn = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
    if Cn.shape != (m + nW + nP, m):
        raise ValueError("C must have shape (%d, %d)" % (m + nW + nP, m))
    th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
    if th.shape != (m,):
        raise ValueError("theta must have %d entries" % m)
    Jn = np.ascontiguousarray(np.asarray(J, dtype=np.int32))
    nJ = len(Jn)
    N = X.shape[0]
    Xn, AXn = torch.empty_like(X), torch.empty_like(X)
    Pn, APn, Wn = (torch.empty((N, max(nJ, 1)), dtype=X.dtype, device=X.device) for _ in range(3))
    rho = np.zeros(m)
    _check(lib().lobpcg_update(ctx.h, _dt(X), _ptr(X), _ptr(AX), _ptr(W), _ptr(AW), nW,
                               _ptr(P) if P is not None else None, _ptr(AP) if P is not None else None, ldP,
                               _np_ptr(pc) if pc is not None else None, nP,
                               _np_ptr(Cn), _np_ptr(th), _np_ptr(Jn) if nJ else None, nJ, float(norm_A),
                               _ptr(Xn), _ptr(AXn), _ptr(Pn), _ptr(APn), _ptr(Wn), _np_ptr(rho)), "lobpcg_update")
    return Xn, AXn, Pn[:, :nJ], APn[:, :nJ], Wn[:, :nJ], rho


def lobpcg_residual(ctx, X, AX, lam, J, norm_A):
    """(W_J packed (N, |J|), rho (m,)) for step 7 and the norms of step 8."""
    X = _blk(ctx, X, "X", ctx.m)
    AX = _blk(ctx, AX, "AX", ctx.m, X.dtype)
    m = X.shape[1]
    Jn = np.ascontiguousarray(np.asarray(J, dtype=np.int32))
    W = torch.empty((X.shape[0], max(len(Jn), 1)), dtype=X.dtype, device=X.device)
    lamn = np.ascontiguousarray(np.asarray(lam, dtype=np.float64))
    rho = np.zeros(m)
    if lamn.shape != (m,):
        raise ValueError("lam must have %d entries" % m)
    _check(lib().lobpcg_residual(ctx.h, _dt(X), _ptr(X), _ptr(AX), int(m), _np_ptr(lamn),
                                 _np_ptr(Jn) if len(Jn) else None, len(Jn), float(norm_A), _ptr(W), _np_ptr(rho)),
           "lobpcg_residual")
    return W[:, :len(Jn)], rho


def lobpcg_dense_chol(G):
    G = np.ascontiguousarray(G, dtype=np.float64)
    R = np.zeros_like(G)
    s = lib().lobpcg_dense_chol(G.shape[0], _np_ptr(G), _np_ptr(R))
    return s, R


def lobpcg_dense_rr(gramA, gramB, m):
    A = np.ascontiguousarray(gramA, dtype=np.float64)
    B = np.ascontiguousarray(gramB, dtype=np.float64)
    n = A.shape[0]
    th = np.zeros(m)
    C = np.zeros((n, m))
    s = lib().lobpcg_dense_rr(n, int(m), _np_ptr(A), _np_ptr(B), _np_ptr(th), _np_ptr(C))
    return s, th, C
