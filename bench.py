"""Benchmark: LOBPCG time-to-residual on the 256^3 Laplacian, mixed vs FP64.

One "step" is one complete solve for the m=32 smallest eigenpairs of the
7-point Dirichlet Laplacian on a 256^3 grid (16,777,216 unknowns) with the
multigrid V(2,2) preconditioner (6 levels), from the seeded uniform[-1,1]
start block, to an explicit FP64 residual ||Ax - lambda x|| / (||A|| ||x||)
<= 1e-8 for every pair.  The headline value is the mixed-precision solve
time (FP32 iterations, FP64 refinement); the plain FP64 solve is timed beside
it.  The start block is resident in HBM before the timed region starts.
`value` is the mean over the K timed solves; each solve's time, their median
and the setup time are reported beside it.

Also reported:
  spmm          the 7-point block stencil (the "SpMM" of the metric) on the
                N x 32 FP32 block, timed with HIP events on the library's
                stream: algorithmic bytes 2*N*m*4 per launch / average launch
                time
  steps         one more mixed (and FP64) solve with HIP events around every
                step class on the library's stream: time, calls, the
                algorithmic bytes the library counts for the step's kernels
                (operands read once, results written once) and their ratio
  roofline      that ratio for the step class with the most time in the
                mixed solve, against 8 TB/s
  cpu_baseline  the FP64 CPU oracle on the host's cores: its setup plus one
                LOBPCG iteration at the same size, extrapolated to the
                iteration count of the FP64 GPU solve
Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]

Block-size study (Section 4, LOBPCG performance vs block size, m = 1..98 on
the 128^3 Laplacian to tol 1e-8): python bench.py --sweep-m 1,2,4,...,98
prints one JSON line per (m, precision) with the solve time, the iteration
counts and the time of each step class; the headline line is not printed.

Problem-size study: python bench.py --sweep-n 48,64,...,464 solves the n^3
Laplacian at m=8 (and m=32 up to n=256), mixed and FP64, one JSON line each.
Seed spread: python bench.py --seeds 2,3,4,5,6 solves the headline problem
from each start block, one JSON line each and a line of medians.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-residual 1e-8, 256^3 Laplacian m=32, FP64 vs mixed; SpMM HBM GB/s"
HBM_PEAK_GBPS = 8000.0

# Measured HBM bytes per launch of a step's kernels in the mixed solve, from
# two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) scaled by a 1 GiB copy;
# valid only while the kernel source is the one the counters were taken with.
TRAFFIC = {
    "update": {"bytes_per_launch": 16.763e9, "source": "paper_0705_2626_amd/csrc/k_update.hip",
               "sha1": "69c451f26724be4d2374ccf4b5c094a6fd724539", "profile": "profiles/lobpcg_mixed_n256_m32_hbm_traffic.md"},
}


def measured_traffic(step):
    t = TRAFFIC.get(step)
    if not t:
        return None
    import hashlib
    with open(os.path.join(ROOT, t["source"]), "rb") as f:
        if hashlib.sha1(f.read()).hexdigest() != t["sha1"]:
            return None
    return t["bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--m", type=int, default=32)
    ap.add_argument("--levels", type=int, default=6)
    ap.add_argument("--nu", type=int, default=2, help="pre- and post-smoothing sweeps of the V-cycle")
    ap.add_argument("--omega", type=float, default=2.0 / 3.0, help="weighted-Jacobi weight of the smoother")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=300)
    ap.add_argument("--spmm-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 1 GiB buffer three times (a plain copy kernel of known size, the "
                         "reference for scaling hardware byte counters)")
    ap.add_argument("--no-profile-steps", action="store_true",
                    help="skip the extra solve with per-step HIP-event timing (then the roofline is the stencil's)")
    ap.add_argument("--sweep-m", default=None,
                    help="comma-separated block sizes: the block-size study instead of the headline run")
    ap.add_argument("--sweep-n", default=None,
                    help="comma-separated grid sizes: the problem-size study instead of the headline run")
    ap.add_argument("--seeds", default=None,
                    help="comma-separated start-block seeds: the seed spread instead of the headline run")
    ap.add_argument("--cpu-baseline-full", action="store_true",
                    help="instead of the headline run: the FP64 oracle's full time to residual 1e-8 on the "
                         "host's physical cores, 16^3 m=4 without preconditioner (median of 3) and 128^3 m=16 "
                         "with the 5-level V-cycle; one JSON line")
    ap.add_argument("--adjoint-fd", action="store_true",
                    help="instead of the headline run: per-face central differences of lambda_1 at the 96^3 "
                         "variable-coefficient workload on 1000 seeded faces against the adjoint; one JSON line")
    ap.add_argument("--opt", action="append", default=[],
                    help="NAME=VALUE: a solver option (lobpcg_set_option, NAME without the OPT_ prefix, e.g. "
                         "LOCK_GAP=1e-3) set on every context of the run")
    args = ap.parse_args()
    if args.cpu_baseline_full:
        cpu_baseline_full()
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path (how it would shard is "
              "described with the design); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_0705_2626_amd as L
    import synth

    options = []
    for o in args.opt:
        name, val = o.split("=", 1)
        options.append((getattr(L, "OPT_" + name.upper()), float(val)))
    setup = L.lobpcg_setup

    def setup_with_options(*a, **k):
        ctx = setup(*a, **k)
        for key, val in options:
            L.lobpcg_set_option(ctx, key, val)
        return ctx
    L.lobpcg_setup = setup_with_options

    torch.cuda.init()
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.adjoint_fd:
        adjoint_fd(L, synth, torch, dev)
        return
    if args.sweep_m:
        sweep_block_size(args, L, synth, torch, dev)
        return
    if args.sweep_n:
        sweep_problem_size(args, L, synth, torch, dev)
        return
    if args.seeds:
        seed_spread(args, L, synth, torch, dev)
        return
    n, m, levels, tol = args.n, args.m, args.levels, args.tol
    dims = (n, n, n)
    N = n ** 3
    X0 = torch.from_numpy(synth.x0_uniform(N, m, seed=2)).to(dev)
    A, T = L.Op(*dims), L.Precond(levels, args.nu, args.nu, 20, args.omega)
    from oracle import closed_form  # closed form of the spectrum, used only to report accuracy
    exact_next, _ = closed_form.smallest(*dims, m + 1)
    exact = exact_next[:m]

    def run(prec, K, W):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        ctx = L.lobpcg_setup(A, T, m, prec, device=dev)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - ts
        res = None
        for _ in range(W):
            res = L.lobpcg_solve(ctx, X0, tol, args.maxit)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        results, marks = [], []
        for _ in range(K):
            results.append(L.lobpcg_solve(ctx, X0, tol, args.maxit, hist=False))
            marks.append(time.perf_counter())   # the solve returns after a stream sync
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / K
        each = [b - a for a, b in zip([t0] + marks[:-1], marks)]
        stats = L.lobpcg_get_stats(ctx)
        steps = None
        if not args.no_profile_steps:
            # one more solve with HIP events around every step class on the
            # library's stream; the library also counts each step's
            # algorithmic bytes, so achieved GB/s = bytes / event time
            L.lobpcg_set_option(ctx, L.OPT_PROFILE, 1)
            L.lobpcg_solve(ctx, X0, tol, args.maxit, hist=False)
            st = L.lobpcg_get_stats(ctx)
            steps = {}
            for k in st["step_ms"]:
                ms, by, calls = st["step_ms"][k], st["step_bytes"][k], st["step_calls"][k]
                steps[k] = {"ms": ms, "calls": calls, "GB": by / 1e9,
                            "GBps": (by / (ms * 1e-3) / 1e9) if ms > 0 and by > 0 else None}
            L.lobpcg_set_option(ctx, L.OPT_PROFILE, 0)
        for r in results:
            assert r.status == L.OK, L.status_string(r.status)
        r = results[-1]
        acc = {"max_rel_err_closed_form": float(np.max(np.abs(r.lam / exact - 1))),
               "max_resid": float(r.resid.max()), "iters": r.iters,
               "iters_fp32": stats["iters_fp32"], "iters_fp64": stats["iters_fp64"], "setup_s": setup_s,
               "solve_s_each": each, "solve_s_median": float(np.median(each))}
        del ctx
        torch.cuda.empty_cache()
        return dt, acc, steps, r

    t_mixed, acc_mixed, steps_mixed, r_mixed = run(L.MIXED, args.steps, args.warmup)
    fp64 = None
    if not args.no_fp64:
        t64, acc64, steps64, r64 = run(L.FP64, args.steps, args.warmup)
        fp64 = {"value": t64, "unit": "s", "ms_per_step": 1e3 * t64, **acc64}
        if steps64:
            fp64["steps"] = steps64
        lam_agree = float(np.max(np.abs(r_mixed.lam / r64.lam - 1)))
        gates = headline_gates(exact_next, r_mixed, r64, t_mixed, t64, tol)
        del r64
    else:
        lam_agree = None
        gates = None
    del r_mixed
    torch.cuda.empty_cache()

    # ---- stencil SpMM on the N x m FP32 block, HIP events on the library's stream
    ctx = L.lobpcg_setup(A, L.Precond(None), m, L.MIXED, device=dev)
    U = X0.float()
    V = torch.empty_like(U)
    lib = L.lib()
    import ctypes
    opc = A.c()
    for _ in range(3):
        lib.lobpcg_apply_A(ctx.h, ctypes.byref(opc), L.F32, ctypes.c_void_p(U.data_ptr()),
                           ctypes.c_void_p(V.data_ptr()), m)
    st = ctx.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(args.spmm_reps):
        s = lib.lobpcg_apply_A(ctx.h, ctypes.byref(opc), L.F32, ctypes.c_void_p(U.data_ptr()),
                               ctypes.c_void_p(V.data_ptr()), m)
        assert s == 0
    e1.record(st)
    e1.synchronize()
    spmm_ms = e0.elapsed_time(e1) / args.spmm_reps
    spmm_bytes = 2.0 * N * m * 4
    spmm_gbps = spmm_bytes / (spmm_ms * 1e-3) / 1e9
    del ctx, U, V
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC, "value": t_mixed, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * t_mixed, "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "7-point Dirichlet Laplacian %d^3 (N=%d), m=%d smallest eigenpairs, "
                               "GMG V(%d,%d) weighted Jacobi omega=%.4g, %d levels, tol %g after FP64 refinement, "
                               "X0 uniform[-1,1] seed 2" % (n, N, m, args.nu, args.nu, args.omega, levels, tol),
                   "n": n, "N": N, "m": m, "levels": levels, "nu": args.nu, "omega": args.omega, "tol": tol},
        "mixed": {"value": t_mixed, "unit": "s", **acc_mixed},
        "fp64": fp64,
        "speedup_mixed_vs_fp64": (fp64["value"] / t_mixed) if fp64 else None,
        "mixed_vs_fp64_max_rel_lambda_diff": lam_agree,
        "spmm": {"GBps": spmm_gbps, "dtype": "f32", "block": [N, m], "ms": spmm_ms},
        "gates": ({name: {"pass": ok, "value": v, "limit": lim} for name, ok, v, lim in gates}
                  if gates is not None else None),
    }
    if steps_mixed:
        out["mixed"]["steps"] = steps_mixed
        # the dominant step class of the headline (mixed) solve
        kern = {"precond": "V-cycle kernels (stencil7 Jacobi/residual, restrict, prolong_add)",
                "gram": "gramy_kernel / gram_rows_kernel (steps 17-23)",
                "update": "mvl_kernel (FP32) / mvf_kernel (FP64), fused Ritz update + residual (steps 25-33, 7)",
                "ortho": "Cholesky-QR Grams and multivector products (steps 11, 14-15)",
                "apply_A": "stencil7 A*W (step 12)", "residual": "residual_kernel (step 7)"}
        name = max(kern, key=lambda k: steps_mixed[k]["ms"])
        d = steps_mixed[name]
        tr = measured_traffic(name)
        out["roofline"] = {"bound": "hbm", "achieved": d["GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                           "frac": d["GBps"] / HBM_PEAK_GBPS, "traffic": tr, "step": name, "kernel": kern[name],
                           "ms": d["ms"], "calls": d["calls"], "algorithmic_GB": d["GB"],
                           "algorithmic_bytes_per_launch": d["GB"] * 1e9 / max(d["calls"], 1)}
    else:
        out["roofline"] = {"bound": "hbm", "achieved": spmm_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                           "frac": spmm_gbps / HBM_PEAK_GBPS, "traffic": None, "kernel": "stencil7 f32 N x 32"}

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(dims, m, levels, X0.cpu().numpy(),
                                           fp64["iters"] if fp64 else acc_mixed["iters"])
    print(json.dumps(out), flush=True)
    if gates is not None and not all(ok for _, ok, _, _ in gates):
        print("headline gates failed: " + ", ".join("%s %.3g > %.3g" % (nm, v, lim)
                                                    for nm, ok, v, lim in gates if not ok), file=sys.stderr)
        sys.exit(1)


def degenerate_groups(exact, rel=1e-12):
    """Index lists of the groups of equal closed-form eigenvalues among the
    first len(exact) (ascending)."""
    groups, cur = [], [0]
    for j in range(1, len(exact)):
        if exact[j] - exact[cur[0]] <= rel * exact[j]:
            cur.append(j)
        else:
            groups.append(cur)
            cur = [j]
    groups.append(cur)
    return groups


def tall_gram(A, B, chunk=1 << 16):
    """A^T B for tall device blocks (N, a), (N, b) as a sum of batched
    products over row chunks: the library's single product with N = 16.7M
    inner terms runs on a handful of workgroups and takes seconds."""
    import torch

    N = A.shape[0]
    nc = N // chunk
    out = torch.zeros((A.shape[1], B.shape[1]), dtype=A.dtype, device=A.device)
    if nc:
        Ab = A[:nc * chunk].reshape(nc, chunk, A.shape[1]).transpose(1, 2).contiguous()
        Bb = B[:nc * chunk].reshape(nc, chunk, B.shape[1]).contiguous()
        out += torch.bmm(Ab, Bb).sum(0)
        del Ab, Bb
    if nc * chunk < N:
        out += A[nc * chunk:].T.contiguous() @ B[nc * chunk:].contiguous()
    return out


def headline_gates(exact, r_mixed, r64, t_mixed, t64, tol, norm_A=12.0):
    """Acceptance checks of the headline problem (Section 2.2's iteration
    judged by Section 4.1's closed form), as a list of
    (name, passed, value, limit).

    exact: the closed-form eigenvalues lambda_1..lambda_{m+1} (one beyond the
    block, for the gaps).  r_mixed, r64: solve results (lam, X on the device,
    resid = explicit FP64 residual norms rho_j).  t_mixed, t64: solve times.
      - every explicit residual <= tol, in both solves;
      - mixed eigenvalues within 1e-6 (relative) of the closed form;
      - FP64 eigenvalues within the a-posteriori bound (rho_j ||A||)^2 / gap_j
        of the closed form (gap_j: distance to the nearest other eigenvalue);
      - mixed and FP64 eigenvalues within 1e-6 (relative) of each other;
      - for every complete group of equal eigenvalues G (the block edge of
        the headline problem falls between groups), the sine of the largest
        principal angle between the mixed and the FP64 span of G is at most
        (||R_G^mixed|| + ||R_G^fp64||) / delta_G (Davis-Kahan for each
        solve against the exact invariant subspace, then the triangle
        inequality; ||R_G|| <= ||A|| (sum rho_j^2)^(1/2), delta_G the
        distance from G's eigenvalue to the rest of the spectrum);
      - X^T X = I to 1e-9 in both solves;
      - the mixed solve faster than the FP64 one.
    """
    import torch

    m = len(r_mixed.lam)
    lam_ex = np.asarray(exact[:m])
    out = []

    def gate(name, value, limit):
        out.append((name, bool(value <= limit), float(value), float(limit)))

    gate("mixed_max_resid", float(np.max(r_mixed.resid)), tol)
    gate("fp64_max_resid", float(np.max(r64.resid)), tol)
    gate("mixed_vs_closed_form_rel", float(np.max(np.abs(r_mixed.lam / lam_ex - 1))), 1e-6)
    worst = 0.0
    for j in range(m):
        others = np.abs(np.asarray(exact) - lam_ex[j])
        gap = others[others > 1e-12 * lam_ex[j]].min()
        bound = (norm_A * r64.resid[j]) ** 2 / gap
        worst = max(worst, abs(r64.lam[j] - lam_ex[j]) / max(bound, 1e-300))
    gate("fp64_vs_closed_form_over_bound", worst, 1.0)
    gate("mixed_vs_fp64_rel", float(np.max(np.abs(r_mixed.lam / r64.lam - 1))), 1e-6)
    groups = degenerate_groups(np.asarray(exact))
    complete = [g for g in groups if g[-1] < m]
    worst = 0.0
    for g in complete:
        Qm, Q64 = r_mixed.X[:, g].contiguous(), r64.X[:, g].contiguous()
        E = Qm - Q64 @ tall_gram(Q64, Qm)
        s = float(torch.linalg.eigvalsh(tall_gram(E, E).cpu()).max().clamp(min=0.0).sqrt())
        lam_g = lam_ex[g[0]]
        outside = [exact[j] for j in range(len(exact)) if j not in g]
        delta = min(abs(v - lam_g) for v in outside)
        bound = norm_A * (np.sqrt(np.sum(np.asarray(r_mixed.resid)[g] ** 2)) +
                          np.sqrt(np.sum(np.asarray(r64.resid)[g] ** 2))) / delta
        worst = max(worst, s / bound)
    gate("principal_angles_over_bound", worst, 1.0)
    for name, r in (("mixed", r_mixed), ("fp64", r64)):
        G = tall_gram(r.X, r.X).cpu().numpy()
        gate(name + "_orthonormality", float(np.abs(G - np.eye(m)).max()), 1e-9)
    gate("mixed_over_fp64_time", t_mixed / t64, 1.0)
    return out


def face_rayleigh_quotient(dims, k, x):
    """sum_f k_f (x_p - x_q)^2 / (x, x) for one vector, in numpy longdouble."""
    nx, ny, nz = dims
    g = np.zeros((nz + 2, ny + 2, nx + 2), dtype=np.longdouble)
    g[1:-1, 1:-1, 1:-1] = np.asarray(x, dtype=np.longdouble).reshape(nz, ny, nx)
    kx, ky, kz = (np.asarray(a, dtype=np.longdouble) for a in k)
    e = (np.sum(kx * np.diff(g[1:-1, 1:-1, :], axis=2) ** 2) + np.sum(ky * np.diff(g[1:-1, :, 1:-1], axis=1) ** 2)
         + np.sum(kz * np.diff(g[:, 1:-1, 1:-1], axis=0) ** 2))
    return e / np.sum(g ** 2)


def adjoint_fd(L, synth, torch, dev):
    """Per-face central differences (relative step 1e-6) of lambda_1 of
    -div(k grad u) on 96^3 (lognormal k, sigma 0.5, correlation 8 cells, m = 8,
    5-level V-cycle) on 1000 seeded faces, against the Hellmann-Feynman
    adjoint.  Each lambda(k +- h k_f e_f) is the face-sum Rayleigh quotient
    (extended precision on the host) of a warm-started FP64 solve to 1e-12.
    One face moves lambda_1 by only a few thousand units in its last place, so
    this is a report, not a gate."""
    n, m, h = 96, 8, 1e-6
    dims = (n, n, n)
    N = n ** 3
    kx, ky, kz = synth.gaussian_field_faces(n, n, n, sigma=0.5, corr=8.0, seed=2)
    shapes, sizes = [a.shape for a in (kx, ky, kz)], [a.size for a in (kx, ky, kz)]
    flat = np.concatenate([kx.ravel(), ky.ravel(), kz.ravel()])
    K = [torch.from_numpy(a).to(dev) for a in (kx, ky, kz)]
    ctx = L.lobpcg_setup(L.Op(n, n, n, *K), L.Precond(5), m, L.FP64, device=dev)
    L.lobpcg_set_option(ctx, L.OPT_FOLD_CHOLQR, 0)
    t0 = time.perf_counter()
    r = L.lobpcg_solve(ctx, torch.from_numpy(synth.x0_uniform(N, m, seed=2)).to(dev), 1e-12, 500, hist=False)
    e1 = np.zeros(m)
    e1[0] = 1.0
    g = np.concatenate([t.cpu().numpy().ravel() for t in L.lobpcg_eig_grad_k(ctx, r.X, e1)])
    faces = synth.sample_faces(flat.size, 1000, seed=3)
    errs, iters = [], []
    for f in faces:
        vals = []
        for sgn in (1.0, -1.0):
            kp = flat.copy()
            kp[f] *= 1.0 + sgn * h
            parts = [a.reshape(sh) for a, sh in zip(np.split(kp, np.cumsum(sizes)[:-1]), shapes)]
            Ap = L.Op(n, n, n, *[torch.from_numpy(a).to(dev) for a in parts])
            rp = L.lobpcg_solve(ctx, r.X, 1e-12, 200, A=Ap, hist=False, raise_on_error=False)
            iters.append(rp.iters)
            vals.append(face_rayleigh_quotient(dims, parts, rp.X[:, 0].cpu().numpy()))
        fd = float((vals[0] - vals[1]) / (2.0 * h * flat[f]))
        errs.append(abs(fd - g[f]) / abs(g[f]))
    errs = np.array(errs)
    print(json.dumps({"adjoint_fd": "per-face central differences of lambda_1", "n": n, "m": m, "faces": len(faces),
                      "h": h, "lambda_1": float(r.lam[0]), "median_rel_err": float(np.median(errs)),
                      "p90_rel_err": float(np.percentile(errs, 90)), "max_rel_err": float(errs.max()),
                      "median_grad": float(np.median(np.abs(g[faces]))), "warm_start_iters_median":
                      float(np.median(iters)), "wall_s": time.perf_counter() - t0}), flush=True)


def levels_for(n):
    """V-cycle depth of the size studies: halve while the coarsest grid keeps
    at least 6 points per axis (128 -> 5 levels, 256 -> 6, 464 -> 7)."""
    levels = 1
    while (n >> levels) >= 6:
        levels += 1
    return levels


def timed_solve(L, torch, A, T, m, prec, X0, tol, maxit, dev):
    """(setup s, solve s, result, stats) for one solve after a 2-iteration
    warm-up solve on the same context."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = L.lobpcg_setup(A, T, m, prec, device=dev)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    L.lobpcg_solve(ctx, X0, tol, 2, hist=False, raise_on_error=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = L.lobpcg_solve(ctx, X0, tol, maxit, hist=False, raise_on_error=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = L.lobpcg_get_stats(ctx)
    del ctx
    return setup, dt, r, st


def sweep_problem_size(args, L, synth, torch, dev):
    """Time to tol vs grid size (n^3 unknowns) at m = 8, and m = 32 up to
    n = 256, mixed and FP64."""
    from oracle import closed_form  # closed form of the spectrum, used only to report accuracy
    for n in [int(v) for v in args.sweep_n.split(",")]:
        dims = (n, n, n)
        N = n ** 3
        levels = levels_for(n)
        A, T = L.Op(*dims), L.Precond(levels, args.nu, args.nu, 20, args.omega)
        for m in ((8, 32) if n <= 256 else (8,)):
            X0 = torch.from_numpy(synth.x0_uniform(N, m, seed=2)).to(dev)
            exact, _ = closed_form.smallest(*dims, m)
            for prec, name in ((L.MIXED, "mixed"), (L.FP64, "fp64")):
                setup, dt, r, st = timed_solve(L, torch, A, T, m, prec, X0, args.tol, args.maxit, dev)
                ok = r.status in (L.OK, L.NOT_CONVERGED)
                print(json.dumps({"sweep": "problem_size", "n": n, "N": N, "m": m, "levels": levels,
                                  "precision": name, "status": L.status_string(r.status), "setup_s": setup,
                                  "time_s": dt, "iters": r.iters, "iters_fp32": st["iters_fp32"],
                                  "iters_fp64": st["iters_fp64"], "ms_per_iter": dt * 1e3 / max(r.iters, 1),
                                  "unknown_iters_per_s": N * m * r.iters / dt,
                                  "max_rel_err_closed_form":
                                      float(np.max(np.abs(r.lam - exact) / exact)) if ok else None,
                                  "max_resid": float(r.resid.max()) if ok else None}), flush=True)
                del r
                torch.cuda.empty_cache()
            del X0


def seed_spread(args, L, synth, torch, dev):
    """The headline problem from several start blocks: the spread of
    iteration counts and times that Section 4 reports across random starts."""
    n, m, levels = args.n, args.m, args.levels
    dims = (n, n, n)
    N = n ** 3
    A, T = L.Op(*dims), L.Precond(levels, args.nu, args.nu, 20, args.omega)
    times = {"mixed": [], "fp64": []}
    iters = {"mixed": [], "fp64": []}
    for seed in [int(v) for v in args.seeds.split(",")]:
        X0 = torch.from_numpy(synth.x0_uniform(N, m, seed=seed)).to(dev)
        for prec, name in ((L.MIXED, "mixed"), (L.FP64, "fp64")):
            setup, dt, r, st = timed_solve(L, torch, A, T, m, prec, X0, args.tol, args.maxit, dev)
            times[name].append(dt)
            iters[name].append(r.iters)
            print(json.dumps({"sweep": "seeds", "n": n, "m": m, "seed": seed, "precision": name,
                              "status": L.status_string(r.status), "setup_s": setup, "time_s": dt,
                              "iters": r.iters, "iters_fp32": st["iters_fp32"], "iters_fp64": st["iters_fp64"],
                              "max_resid": float(r.resid.max()) if r.resid is not None else None}), flush=True)
            del r
            torch.cuda.empty_cache()
        del X0
    print(json.dumps({"sweep": "seeds", "summary": True,
                      "median_time_s": {k: float(np.median(v)) for k, v in times.items()},
                      "min_max_time_s": {k: [min(v), max(v)] for k, v in times.items()},
                      "min_max_iters": {k: [min(v), max(v)] for k, v in iters.items()}}), flush=True)


def sweep_block_size(args, L, synth, torch, dev):
    """Solve time vs block size on the 128^3 Laplacian (5-level V-cycle), FP64
    and mixed, one solve per (m, precision) after an untimed short solve."""
    from oracle import closed_form  # closed form of the spectrum, used only to report accuracy
    n = 128 if args.n == 256 else args.n
    levels = 5 if args.levels == 6 else args.levels
    dims = (n, n, n)
    N = n ** 3
    A, T = L.Op(*dims), L.Precond(levels, args.nu, args.nu, 20, args.omega)
    for m in [int(v) for v in args.sweep_m.split(",")]:
        X0 = torch.from_numpy(synth.x0_uniform(N, m, seed=2)).to(dev)
        exact, _ = closed_form.smallest(*dims, m)
        for prec, name in ((L.FP64, "fp64"), (L.MIXED, "mixed")):
            ctx = L.lobpcg_setup(A, T, m, prec, device=dev)
            L.lobpcg_solve(ctx, X0, args.tol, 2, hist=False, raise_on_error=False)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = L.lobpcg_solve(ctx, X0, args.tol, 1000, hist=False, raise_on_error=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            st = L.lobpcg_get_stats(ctx)
            L.lobpcg_set_option(ctx, L.OPT_PROFILE, 1)
            L.lobpcg_solve(ctx, X0, args.tol, 1000, hist=False, raise_on_error=False)
            sp = L.lobpcg_get_stats(ctx)
            ok = r.status in (L.OK, L.NOT_CONVERGED)
            line = {"sweep": "block_size", "n": n, "m": m, "precision": name, "status": L.status_string(r.status),
                    "time_s": dt, "iters": r.iters, "iters_fp32": st["iters_fp32"], "iters_fp64": st["iters_fp64"],
                    "ms_per_iter": dt * 1e3 / max(r.iters, 1),
                    "max_rel_err_closed_form": float(np.max(np.abs(r.lam - exact) / exact)) if ok else None,
                    "max_resid": float(r.resid.max()) if ok else None,
                    "step_ms": {k: round(v, 3) for k, v in sp["step_ms"].items()}}
            print(json.dumps(line), flush=True)
            del ctx, r
            torch.cuda.empty_cache()
        del X0


def physical_cores():
    """Physical cores among the CPUs this process may run on (lscpu's
    core/socket pairs of the allowed CPUs), and the allowed logical CPUs."""
    import subprocess
    allowed = os.sched_getaffinity(0)
    try:
        out = subprocess.run(["lscpu", "-p=cpu,core,socket"], capture_output=True, text=True, check=True).stdout
        pairs = set()
        for line in out.splitlines():
            if line.startswith("#"):
                continue
            cpu, core, sock = (int(v) for v in line.split(","))
            if cpu in allowed:
                pairs.add((core, sock))
        return len(pairs), len(allowed)
    except (OSError, ValueError, subprocess.CalledProcessError):
        return len(allowed), len(allowed)


_CPU_FULL_CHILD = r"""
import json, sys, time
import numpy as np
sys.path.insert(0, %r)
import synth
from oracle import lobpcg as olob
out = {}
for name, dims, m, levels, reps in (("16^3 m=4, no preconditioner", (16, 16, 16), 4, None, 3),
                                    ("128^3 m=16, 5-level V-cycle", (128, 128, 128), 16, 5, 1)):
    N = dims[0] * dims[1] * dims[2]
    X0 = synth.x0_uniform(N, m, seed=2)
    times, iters = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = olob.laplace7_solver(dims, m, X0, 1e-8, 500, levels=levels)
        times.append(time.perf_counter() - t0)
        iters.append(int(r.iters))
        assert r.status == olob.OK
    out[name] = {"seconds_each": times, "median_s": float(np.median(times)), "iterations": iters,
                 "max_resid": float(r.resid.max())}
    print(json.dumps({"done": name, **out[name]}), file=sys.stderr, flush=True)
print(json.dumps(out), flush=True)
"""


def cpu_baseline_full():
    """The oracle's full time to residual 1e-8 at 16^3 (m=4, median of 3) and
    128^3 (m=16, 5-level V-cycle), run in a child process whose OpenMP and
    BLAS thread counts are the physical cores available here."""
    import subprocess
    phys, logical = physical_cores()
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = str(phys)
    t0 = time.perf_counter()
    p = subprocess.run([sys.executable, "-u", "-c", _CPU_FULL_CHILD % ROOT], env=env, capture_output=True,
                       text=True)
    if p.returncode != 0:
        print(p.stderr, file=sys.stderr)
        sys.exit(p.returncode)
    res = json.loads(p.stdout.strip().splitlines()[-1])
    print(json.dumps({"metric": "FP64 oracle time to residual 1e-8 on the host", "unit": "s",
                      "cores": phys, "logical_cpus_allowed": logical,
                      "threads_env": {k: env[k] for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                                          "MKL_NUM_THREADS")},
                      "kind": "oracle", "results": res, "wall_s": time.perf_counter() - t0}), flush=True)


def cpu_baseline(dims, m, levels, X0, iters):
    """The FP64 oracle at the benchmark size: setup (steps 3-4) plus one loop
    iteration, timed, and extrapolated to `iters` iterations."""
    from oracle import lobpcg as olob

    marks = []
    t0 = time.perf_counter()

    def cb(k, lam, rho, J):
        marks.append(time.perf_counter())

    olob.laplace7_solver(dims, m, X0, 1e-300, 1, levels=levels, callback=cb)
    t_end = time.perf_counter()
    # the callback fires after the first residual: before it lie steps 3-4,
    # after it one loop iteration and the final explicit residual
    t_setup = marks[0] - t0
    t_iter = t_end - marks[0]
    est = t_setup + iters * t_iter
    phys, logical = physical_cores()
    threads = int(os.environ.get("OMP_NUM_THREADS", logical))
    return {"value": est, "unit": "s", "cores": threads, "physical_cores": phys, "kind": "oracle",
            "extrapolated": True,
            "threads_env": {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS")},
            "sample": "FP64 oracle at the same size (n=%d, m=%d): setup + 1 iteration (with the final explicit "
                      "residual) timed (%.1f s + %.1f s), extrapolated to %d iterations; the full solves at "
                      "16^3 and 128^3 are bench.py --cpu-baseline-full" % (dims[0], m, t_setup, t_iter, iters)}


if __name__ == "__main__":
    main()
