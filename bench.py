"""Benchmark: Hermitian FEAST contour-integration eigensolver on one MI355X.

Workload (the metric's configuration): generalized complex Hermitian pencil,
n = 4096, B = I + 0.1 C C^H / n, A = L U diag(lambda) U^H L^H with lambda ~ U[-10, 10]
(seed 0; 385 eigenvalues in [-1, 1]), M0 = 600, 8-node Gauss-Legendre half contour
(ellipse ratio 0.30), convergence at relative residual <= 1e-10 (fpm(3) = 10).
One step = one complete mfeast_zhegv call (factor all nodes, iterate the contour
solves and Rayleigh-Ritz to convergence) on inputs already resident in HBM,
starting from the library's seeded random block.  FP32 solves with the FP64
residual form (fpm(42) = 1) is the reported value; the plain complex FP64 form
(fpm(42) = 0) is timed beside it.

Prints ONE JSON line (rank 0).
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "converged eigenpairs/s + contour-solve TFLOP/s, FP32+IR vs FP64 at res≤1e-10"

# HBM bytes per launch unit from the rocprofv3 FETCH_SIZE / WRITE_SIZE passes (scaled by a
# plain copy's readings), measured on the pencil workload (n = 4096, M0 = 600, 8 nodes) and
# reported for that workload only, while the listed sources hash to the profiled ones
TRAFFIC = {
    "contour_solve": {"bytes": 14.05e9, "workload": "pencil",
                      "sources": ["paper_2002_04807_amd/csrc/gemm.hip", "paper_2002_04807_amd/csrc/solve.hip"],
                      "sha256_16": "99f5eb5a6d72f31e"},
    "reduced_eig": {"bytes": 1.48e9, "workload": "pencil",
                    "sources": ["paper_2002_04807_amd/csrc/eig.hip", "paper_2002_04807_amd/csrc/tri.hip"],
                    "sha256_16": "0ada7b7777fd1d85"},
}
PEAK = {"fp32_mfma": 157.3, "fp64_mfma": 78.6, "fp32_vector": 157.3, "fp64_vector": 78.6, "hbm": 8000.0}
N, M0, NE, EMIN, EMAX, SEED = 4096, 600, 8, -1.0, 1.0, 0
RES_BAR = 1e-10
# the classes of the contour step: shift-form and quadrature sums (other), LU, block solves
CONTOUR_CLASSES = ("lu_trailing_gemm", "lu_panel", "lu_rows", "contour_solve", "other")
# Issued MFMA work of the block solves per unit of algorithmic work: each 256-row panel
# step multiplies by the panel's full 256 x 256 inverse (16 panels at n = 4096: 136 x 256^2
# complex multiply-adds per right-hand side and triangle against n^2 / 2 = 128 x 256^2),
# and a complex multiply-add is three real products (6 flops) in the three-product
# scheme against the 8 flops counted
SOLVE_ISSUED_PER_ALG = (136.0 / 128.0) * (6.0 / 8.0)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--profile-steps", type=int, default=0,
                   help="only run this many FP32 steps (for rocprofv3 runs); no JSON extras")
    p.add_argument("--workload", default="pencil",
                   choices=("pencil", "sparse", "batched", "adjoint", "count", "general", "polynomial"),
                   help="pencil: the metric's n=4096 generalized complex Hermitian problem (default); "
                        "sparse: 64^3 Laplacian CSR with batched BiCGSTAB; batched: 128 independent "
                        "real problems; adjoint: forward and backward of the n=4096 tridiagonal workload; "
                        "count: stochastic eigenvalue-count estimate on the n=4096 pencil; general: "
                        "two-sided non-Hermitian FEAST on an n=4096 complex pencil; polynomial: quadratic "
                        "FEAST at n=4096")
    return p.parse_args()


def run_steps(mf, torch, h, At, Bt, fp32, steps, profile):
    dt = torch.complex128
    E = torch.zeros(M0, dtype=torch.float64, device=At.device)
    res = torch.zeros(M0, dtype=torch.float64, device=At.device)
    X = torch.zeros((M0, N), dtype=dt, device=At.device).mT
    outs, times, profs = [], [], []
    for _ in range(steps):
        fpm = mf.mfeast_init()
        fpm[41] = 1 if fp32 else 0   # fpm(42): FP32 solves + FP64 residual form, or plain FP64
        fpm[2] = 10                  # fpm(3): residual tolerance 1e-10 (the metric's bar)
        fpm[51] = 1 if profile else 0  # fpm(52): per-class device timing
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = mf.mfeast_zhegv(h, "F", N, At, N, Bt, N, fpm, EMIN, EMAX, M0, E, X, N, res)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        out["E"] = E[:out["m0"]].cpu().numpy().copy()
        out["res"] = res[:out["m0"]].cpu().numpy().copy()
        out["timing"] = h.timing()
        if profile:
            profs.append(h.profile())
        outs.append(out)
    return outs, times, profs


def accuracy(out, lam_in):
    import numpy as np
    M = out["M"]
    cnt = lam_in.size
    ok_count = (M == cnt)
    res = out["res"][:M]
    E = out["E"][:M]
    alpha = max(abs(EMIN), abs(EMAX))
    eig_err = float(np.max(np.abs(E - lam_in) / np.maximum(np.abs(lam_in), alpha))) if ok_count else None
    m_conv = int(np.sum(res <= RES_BAR)) if ok_count else 0
    return {"M": M, "exact_count": cnt, "count_exact": bool(ok_count), "max_rel_eig_err": eig_err,
            "max_res": float(res.max()) if M else None, "converged_pairs": m_conv, "loop": out["loop"],
            "info": out["info"]}


KERNELS = {
    # class -> (kernel, bound, peak key or None, what one launch processes)
    "bicgstab_vector": ("k_bi_sweep_c (+ column sums)", "hbm", "hbm", "one BiCGSTAB update sweep over the active tiles"),
    "bicgstab_spmv": ("k_bi_sweep_a / k_bi_sweep_b", "hbm", "hbm", "one shifted sparse product sweep"),
    "lu_panel": ("k_leaf + k_leaf_update (recursive panel)", "alu", "fp32_vector",
                 "one 64-column panel of every factored matrix"),
    "lu_rows": ("k_laswp + k_trsm_u12 (per panel), k_invert_diag, panel inverses", "alu", "fp32_vector",
                "one panel's row interchanges and U12 substitution, or the inverses after the last panel"),
    "orth": ("k_chol_diag / Newton-Schulz (B-orthonormalization)", "alu", "fp64_vector",
             "one B-orthonormalization pass"),
    "resid": ("residual norms, B^-1 products of the found-pair test", "hbm", "hbm", "one residual evaluation"),
    "other": ("shift-form, right-hand sides, quadrature sums", "hbm", "hbm", "one small-kernel group"),
    "lu_trailing_gemm": ("k_gemm (LU trailing update)", "mfma", "fp32_mfma", "one trailing update, all nodes"),
    "contour_solve": ("k_gemm (panel-inverse products and updates of the block solves)", "mfma", "fp32_mfma",
                      "one contour's block solves, all 8 nodes: the forward (L, U) and the "
                      "conjugate-transpose (U^H, L^H) sweeps, which run concurrently on two streams"),
    "rr_gemm": ("k_gemm (FP64 Rayleigh-Ritz)", "mfma", "fp64_mfma", "one FP64 product"),
    "reduced_eig": ("k_bj_sub + k_bj_upd (block Jacobi), k_trd_* (tridiagonal seeding solves)", "alu", "fp64_vector",
                    "one reduced eigensolve (48 m^3 flops per Jacobi sweep; 8 (4/3 + 2) m^3 for a tridiagonal one)"),
    "batched_factor": ("factorization graph: k_bt_shift_form + blocked LU + panel inverses of every size class",
                       "mfma", "fp32_mfma", "one replay: all problems and nodes (flops of the unpadded matrices)"),
}


def _source_unchanged(entry):
    import hashlib
    h = hashlib.sha256()
    try:
        for src in entry["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
    except OSError:
        return False
    return h.hexdigest()[:16] == entry["sha256_16"]


def roofline_of(prof, rank=0, workload=None):
    """Roofline of the kernel class with the largest device time in this call (rank 0; rank 1
    the next one): algorithmic flops (8 per complex multiply-add) or bytes per launch over
    the mean launch time, both from the library's HIP-event profile of the timed call.  The
    measured traffic is attached only for the workload it was taken on."""
    cands = sorted([c for c in KERNELS if prof.get(c, {}).get("ms", 0.0) > 0.0], key=lambda c: -prof[c]["ms"])
    if rank >= len(cands):
        return None
    cls = cands[rank]
    p = prof[cls]
    kernel, bound, peak_key, unit_desc = KERNELS[cls]
    peak = PEAK[peak_key]
    per_launch_s = p["ms"] / 1e3 / p["launches"]
    if bound == "hbm":
        work_per_launch = p["bytes"] / p["launches"]
        achieved = work_per_launch / per_launch_s / 1e9
        unit = "GB/s"
    else:
        work_per_launch = p["flops"] / p["launches"]
        achieved = work_per_launch / per_launch_s / 1e12
        unit = "TFLOP/s"
    tr = TRAFFIC.get(cls)
    traffic = (tr["bytes"] if tr is not None and tr["workload"] == workload and _source_unchanged(tr)
               else None)
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": traffic, "kernel": kernel, "kernel_class": cls,
            "unit_of_work": unit_desc, ("bytes_per_launch" if bound == "hbm" else "flops_per_launch"): work_per_launch,
            "launches_per_step": p["launches"], "avg_launch_us": per_launch_s * 1e6,
            "classes_ms_per_step": {c: round(prof[c]["ms"], 3) for c in prof}}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def classes_summary(prof, ms_per_step):
    """Per-class device milliseconds of one call, their sum, and what no class covers
    (host round trips between synchronized phases and launch gaps).  The forward and the
    conjugate-transpose solves overlap on two streams, so the sum can exceed the span."""
    total = sum(v["ms"] for v in prof.values())
    return {"classes_ms": {c: round(v["ms"], 3) for c, v in prof.items() if v["ms"] > 0},
            "classes_sum_ms": round(total, 3), "call_ms": round(ms_per_step, 3),
            "unattributed_ms": round(ms_per_step - total, 3)}


def cpu_baseline(A, B, lam_in, loops):
    """The oracle's own steps timed on a bounded sample: one node's complex128 LU, one
    forward and one conjugate-transpose solve with M0 right-hand sides, and one
    Rayleigh-Ritz step (A Q, B Q, Gram matrices, dense eigensolve), scaled to a whole
    call with the same node count and loop count as the GPU FP64 run."""
    import numpy as np
    import scipy.linalg as sla
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()])
    except Exception:
        cores = os.cpu_count()
    import oracle
    from oracle.feast import rayleigh_ritz, _Factored
    z, w = oracle.half_contour(EMIN, EMAX, NE)
    rng = np.random.default_rng(1)
    Y = (rng.standard_normal((N, M0)) + 1j * rng.standard_normal((N, M0)))
    BY = B @ Y
    t_lu = t_solve2 = 0.0
    for j in range(NE):
        t0 = time.perf_counter()
        fac = _Factored(z[j], A, B)
        t_lu += time.perf_counter() - t0
        t0 = time.perf_counter()
        fac.solve(BY)
        fac.solve_h(BY)
        t_solve2 += time.perf_counter() - t0
        del fac
    t0 = time.perf_counter()
    rayleigh_ritz(Y, A, B)
    t_rr = time.perf_counter() - t0
    iters = loops + 1
    t_est = t_lu + iters * (t_solve2 + t_rr)
    m = lam_in.size
    return {"value": m / t_est, "unit": "eigenpairs/s", "cores": int(cores), "cpu": _cpu_model(), "kind": "oracle",
            "sample": "the first subspace iteration's factorizations and solves: the 8 node LUs "
                      "(complex128, n=4096) with one forward and one conjugate solve of 600 right-hand "
                      "sides each, plus one Rayleigh-Ritz step (A Q, B Q, Grams, eigh 600), %.1f s; "
                      "scaled to %d loops: est. %.1f s per call (lu %.2f s, solves %.2f s, rr %.2f s)"
                      % (t_lu + t_solve2 + t_rr, iters, t_est, t_lu, t_solve2, t_rr)}


def _cores():
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [os.cpu_count()]))
    except Exception:
        return int(os.cpu_count() or 1)


def bench_sparse(args, mf, torch, np, gen):
    """64^3 Laplacian (CSR, n = 262144), [0, 0.08] (69 eigenvalues), M0 = 160, 16 trapezoidal
    nodes on a circle, BiCGSTAB to 1e-4 (at most 2000 iterations) in complex FP32, res <= 1e-10."""
    nx = 64
    v, c, p = gen.laplacian_3d_csr(nx)
    lam = gen.laplacian_3d_eigs(nx)
    emin, emax, m0 = 0.0, 0.08, 160
    exact = np.sort(lam[(lam >= emin) & (lam <= emax)])
    dev = torch.device("cuda:0")
    csr = (torch.tensor(v, device=dev), torch.tensor(p, device=dev), torch.tensor(c, device=dev))
    h = mf.Handle(0)

    def fpm_for(profile):
        f = mf.mfeast_init_ifeast()
        f[1], f[2], f[44], f[45], f[51] = 16, 10, 4, 2000, 1 if profile else 0
        return f

    for _ in range(args.warmup):
        mf.feast_csr(csr, emin, emax, m0, fpm=fpm_for(False), handle=h)
    times, outs = [], []
    for _ in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = mf.feast_csr(csr, emin, emax, m0, fpm=fpm_for(True), handle=h)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        outs.append(out)
    out = outs[-1]
    M = out["M"]
    res = out["res"].cpu().numpy()[:M]
    E = out["E"].cpu().numpy()[:M]
    ok = M == exact.size
    m_conv = int(np.sum(res <= RES_BAR)) if ok else 0
    t = float(np.median(times))
    result = {
        "metric": "converged eigenpairs/s (IFEAST, FP32 BiCGSTAB + FP64 outer residuals, res<=1e-10)",
        "value": m_conv / t, "unit": "eigenpairs/s", "n_gpus": 1, "steps": len(times), "warmup": args.warmup,
        "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 BiCGSTAB + f64 outer", "data": "synthetic",
        "config": {"workload": "3-D 7-point Laplacian 64^3 CSR, [0,0.08], M0=160, 16 trapezoidal nodes (circle), "
                               "BiCGSTAB 1e-4 / 2000 it", "n": int(len(p) - 1), "nnz": int(len(v))},
        "accuracy": {"M": M, "exact_count": int(exact.size), "max_abs_eig_err": float(np.max(np.abs(E - exact))) if ok
                     else None, "max_res": float(res.max()) if M else None, "loop": out["loop"],
                     "bicgstab_iterations_fpm60": out["fpm60"], "info": out["info"]},
        "roofline": roofline_of(out["profile"]),
    }
    if not args.no_cpu_baseline:
        # the oracle's BiCGSTAB on a sample: 4 columns of the node nearest the spectrum for 10
        # iterations, scaled to the column-iterations of the whole GPU call (fpm(60) x M0)
        import scipy.sparse as sp
        import oracle
        A = sp.csr_matrix((v, c, p))
        z, _ = oracle.half_contour(emin, emax, 16, rule=1, ratio_pct=100)
        rng = np.random.default_rng(0)
        ncol, nit = 16, 50
        b = rng.standard_normal((A.shape[0], ncol)) + 0j
        op = lambda q: z[-1] * q - A @ q  # noqa: E731
        t0 = time.perf_counter()
        oracle.bicgstab_block(op, b, 1e-30, nit)
        ts = time.perf_counter() - t0
        col_its = float(out["fpm60"]) * m0
        est = ts / float(ncol * nit) * col_its
        result["cpu_baseline"] = {"value": m_conv / est if est > 0 else None, "unit": "eigenpairs/s",
                                  "cores": _cores(), "cpu": _cpu_model(), "kind": "oracle",
                                  "sample": "oracle BiCGSTAB, %d columns x %d iterations (%.1f s) scaled to "
                                            "fpm(60) x M0 = %.0f column-iterations (outer steps not counted): "
                                            "est. %.0f s per call" % (ncol, nit, ts, col_its, est)}
    h.close()
    return result


def bench_batched(args, mf, torch, np, gen):
    """128 independent real symmetric problems, n ~ U{256..2048}, 24-48 eigenvalues each,
    M0 = ceil(1.5 count), 8 Gauss nodes, FP32 solves + FP64 residual form, res <= 1e-10."""
    t0 = time.perf_counter()
    probs = gen.batched_real_problems(128, seed=0)
    print("bench: batched inputs built in %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    As = [torch.from_numpy(p["A"]).to(dev) for p in probs]
    emins = [p["emin"] for p in probs]
    emaxs = [p["emax"] for p in probs]
    m0s = [p["m0"] for p in probs]
    fpm = mf.mfeast_init()
    fpm[2] = 10
    h = mf.Handle(0)
    for _ in range(args.warmup):
        mf.feast_batched(As, emins, emaxs, m0s, fpm=fpm, handle=h)
    times, last = [], None
    for _ in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ret, outs, _ = mf.feast_batched(As, emins, emaxs, m0s, fpm=fpm, handle=h)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        last = (ret, outs)
    ret, outs = last
    # one more call with per-class device timing (summed over the 128 problems' calls)
    h.set_profiling(True)
    mf.feast_batched(As, emins, emaxs, m0s, fpm=fpm, handle=h)
    torch.cuda.synchronize()
    prof = h.profile()
    h.set_profiling(False)
    roofline = roofline_of(prof)
    if roofline is not None:
        roofline["note"] = ("per-launch averages over all 128 problems' launches; the problems run on 8 "
                            "concurrent streams, so each launch shares the GPU with others")
    m_conv, exact_ok, max_err = 0, 0, 0.0
    for o, p in zip(outs, probs):
        c = p["count"]
        if o["M"] == c and o["info"] == 0:
            exact_ok += 1
            r = o["res"].cpu().numpy()[:c]
            m_conv += int(np.sum(r <= RES_BAR))
            lam = p["lam"][p["start"]:p["start"] + c]
            max_err = max(max_err, float(np.max(np.abs(o["E"].cpu().numpy()[:c] - lam))))
    t = float(np.median(times))
    sum_n3 = sum(float(p["A"].shape[0]) ** 3 for p in probs)
    result = {
        "metric": "converged eigenpairs/s over 128 independent problems (FP32+IR, res<=1e-10)",
        "value": m_conv / t, "unit": "eigenpairs/s", "n_gpus": 1, "steps": len(times), "warmup": args.warmup,
        "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 solves + f64 residual/RR", "data": "synthetic",
        "config": {"workload": "128 real symmetric problems, n~U{256..2048} (seed 0), 24-48 eigenvalues each, "
                               "M0=ceil(1.5 count), 8 Gauss nodes; all factorizations in one replayed graph "
                               "(padded size classes), iterations on 8 concurrent streams", "sum_n3": sum_n3},
        "accuracy": {"problems_exact": exact_ok, "problems": len(probs), "max_abs_eig_err": max_err,
                     "loops": np.bincount([o["loop"] for o in outs]).tolist(), "ret": ret},
        "lu_tflops": 8.0 * (8.0 / 3.0) * sum_n3 / t / 1e12,
        "lu_tflops_kind": "algorithmic LU flops of all problems and nodes over the whole call's wall time",
        "factor_graph_ms": prof.get("batched_factor", {}).get("ms"),
        "factor_graph_tflops": (prof["batched_factor"]["flops"] / prof["batched_factor"]["ms"] / 1e9
                                if prof.get("batched_factor", {}).get("ms") else None),
        "roofline": roofline,
        "roofline_next": roofline_of(prof, 1),
        "classes_ms_summed_over_problems": {c: round(v["ms"], 3) for c, v in prof.items() if v["ms"] > 0},
    }
    if not args.no_cpu_baseline:
        import oracle
        sample = sorted(range(len(probs)), key=lambda k: probs[k]["A"].shape[0])[::5]
        t0 = time.perf_counter()
        n3 = 0.0
        for k in sample:
            f = oracle.feastinit()
            f[2] = 10
            oracle.feast_dense(probs[k]["A"], None, probs[k]["emin"], probs[k]["emax"], probs[k]["m0"], f)
            n3 += float(probs[k]["A"].shape[0]) ** 3
        ts = time.perf_counter() - t0
        est = ts * sum_n3 / n3
        result["cpu_baseline"] = {"value": m_conv / est, "unit": "eigenpairs/s", "cores": _cores(), "cpu": _cpu_model(), "kind": "oracle",
                                  "sample": "oracle FEAST on %d of the 128 problems (n = %s, %.1f s), scaled by "
                                            "sum n^3: est. %.0f s for all" % (len(sample), [probs[k]["A"].shape[0]
                                                                                            for k in sample], ts, est)}
    h.close()
    return result


def bench_adjoint(args, mf, torch, np, gen):
    """n = 4096 tridiag(-1, 2 + v, -1), v ~ U[0,1] (seed 3), [0, 0.2] (2 eigenvalues), M0 = 16:
    forward mfeast_dsygv (FP32+IR) and backward mfeast_dsy_adjoint (FP32 LU + FP64 refinement)
    for L = sum lambda_i + sum_i sum_k c_k x_ik^2; one step = forward + backward."""
    from oracle import adjoint as adj
    n, emin, emax = 4096, 0.0, 0.2
    v, c, _ = gen.differentiation_problem(n, seed=3)
    dev = torch.device("cuda:0")
    A0 = (2.0 * torch.eye(n, dtype=torch.float64, device=dev) - torch.diag(torch.ones(n - 1, dtype=torch.float64,
          device=dev), 1) - torch.diag(torch.ones(n - 1, dtype=torch.float64, device=dev), -1))
    ct = torch.tensor(c, dtype=torch.float64, device=dev)

    def step():
        vt = torch.tensor(v, dtype=torch.float64, device=dev, requires_grad=True)
        E, X = mf.feast_eigh(A0 + torch.diag(vt), emin, emax, 16, precision=1)
        L = E.sum() + (ct[:, None] * X * X).sum()
        L.backward()
        return vt.grad

    for _ in range(args.warmup):
        step()
    times = []
    for _ in range(max(1, args.steps)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    # one more step with per-class device timing of the forward call and of the adjoint
    hp = mf.Handle(0)
    hp.set_profiling(True)
    vt = torch.tensor(v, dtype=torch.float64, device=dev, requires_grad=True)
    E, X = mf.feast_eigh(A0 + torch.diag(vt), emin, emax, 16, precision=1, handle=hp)
    prof_f = hp.profile()
    (E.sum() + (ct[:, None] * X * X).sum()).backward()
    torch.cuda.synchronize()
    prof_b = hp.profile()
    hp.close()
    prof = {c: {k: prof_f[c][k] + prof_b[c][k] for k in prof_f[c]} for c in prof_f}
    t0 = time.perf_counter()
    Lr, gr, lamS, _ = adj.loss_and_grad_v(v, c, emin, emax)
    t_cpu = time.perf_counter() - t0
    err = float(np.max(np.abs(g.cpu().numpy() - gr)) / np.max(np.abs(gr)))
    t = float(np.median(times))
    return {
        "metric": "gradient evaluations/s (forward FEAST + adjoint dL/dv, n=4096)", "value": 1.0 / t,
        "unit": "gradients/s", "n_gpus": 1, "steps": len(times), "warmup": args.warmup, "ms_per_step": t * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64 LU + f64 refinement",
        "data": "synthetic",
        "config": {"workload": "tridiag(-1,2+v,-1) n=4096 dense, v~U[0,1] seed 3, [0,0.2], M0=16, "
                               "L=sum lambda + sum c_k x_k^2", "pairs": int(lamS.size)},
        "accuracy": {"max_rel_grad_err_vs_oracle": err},
        "roofline": roofline_of(prof),
        "roofline_next": roofline_of(prof, 1),
        "classes_ms": {"forward": {c: round(p["ms"], 3) for c, p in prof_f.items() if p["ms"] > 0},
                       "adjoint": {c: round(p["ms"], 3) for c, p in prof_b.items() if p["ms"] > 0}},
        "cpu_baseline": {"value": 1.0 / t_cpu, "unit": "gradients/s", "cores": _cores(), "cpu": _cpu_model(), "kind": "oracle",
                         "sample": "the whole oracle gradient (dense eigh n=4096 + eigen-sum), %.1f s" % t_cpu},
    }


def bench_count(args, mf, torch, np, gen):
    """Stochastic eigenvalue count (fpm(14)=2) on the n = 4096 complex Hermitian pencil of the
    headline workload, [-1, 1], M0 = 600 probe vectors, 3 Gauss half-contour nodes, FP32 solves:
    one step = one estimate (3 node LUs, forward and conjugate-transpose solves, the trace)."""
    from oracle.stochastic import stochastic_count
    dev = torch.device("cuda:0")
    A, B, lam, _ = gen.prescribed_complex_pencil(N, seed=SEED)
    exact = int(((lam >= EMIN) & (lam <= EMAX)).sum())
    At = torch.from_numpy(np.asfortranarray(A)).to(dev)
    Bt = torch.from_numpy(np.asfortranarray(B)).to(dev)
    E = torch.zeros(M0, dtype=torch.float64, device=dev)
    res = torch.zeros(M0, dtype=torch.float64, device=dev)
    X = torch.zeros((M0, N), dtype=torch.complex128, device=dev).mT
    h = mf.Handle(0)

    def step(profile):
        fpm = mf.mfeast_init_stochastic()
        fpm[51] = 1 if profile else 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = mf.mfeast_zhegv(h, "F", N, At, N, Bt, N, fpm, EMIN, EMAX, M0, E, X, N, res)
        torch.cuda.synchronize()
        return out, time.perf_counter() - t0

    for _ in range(args.warmup):
        step(False)
    times = []
    for _ in range(max(1, args.steps)):
        out, t = step(False)
        times.append(t)
    est = float(E[0].item())
    out_p, _ = step(True)
    prof = h.profile()
    h.close()
    roofline = roofline_of(prof)
    roofline_next = roofline_of(prof, 1)
    for r in (roofline, roofline_next):
        if r is not None:
            r["unit_of_work"] = r["unit_of_work"].replace("8 nodes", "3 nodes")
    print("bench: count steps %s s, estimate %.3f (exact count %d)" % (["%.4f" % t for t in times], est, exact),
          file=sys.stderr, flush=True)
    t = float(np.median(times))
    result = {
        "metric": "stochastic eigenvalue-count estimates/s (fpm(14)=2)", "value": 1.0 / t, "unit": "estimates/s",
        "n_gpus": 1, "steps": len(times), "warmup": args.warmup, "ms_per_step": t * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64 solves + f64 accumulation", "data": "synthetic",
        "config": {"workload": "generalized complex Hermitian n=4096 (seed 0), [-1,1], 600 +-1 probes, "
                               "3-node Gauss half contour, FP32 solves", "n": N, "m0": M0, "nodes": 3},
        "accuracy": {"estimate": est, "M": out["M"], "info": out["info"], "exact_count": exact},
        "roofline": roofline,
        "roofline_next": roofline_next,
    }
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        est_ref, _ = stochastic_count(A, B, EMIN, EMAX, 64, ne=3, seed=0)
        t_cpu = time.perf_counter() - t0
        result["cpu_baseline"] = {"value": 1.0 / t_cpu, "unit": "estimates/s", "cores": _cores(), "cpu": _cpu_model(), "kind": "oracle",
                                  "sample": "the whole oracle estimate with 64 probes (3 complex128 LUs of n=4096 "
                                            "and their solves), %.1f s; 600 probes cost more" % t_cpu}
        fpm = mf.mfeast_init_stochastic()
        h2 = mf.Handle(0)
        mf.mfeast_zhegv(h2, "F", N, At, N, Bt, N, fpm, EMIN, EMAX, 64, E, X, N, res)
        torch.cuda.synchronize()
        h2.close()
        result["accuracy"]["parity_64_probes"] = {"gpu": float(E[0].item()), "oracle": est_ref}
    return result


def _match_err(E, lam_in, scale):
    """Largest distance from each computed eigenvalue to the nearest exact one, and whether
    the matching is one to one."""
    import numpy as np
    if E.size == 0 or lam_in.size == 0:
        return None, False
    d = np.abs(E[:, None] - lam_in[None, :])
    idx = np.argmin(d, axis=1)
    return float(np.max(d[np.arange(E.size), idx]) / scale), bool(np.unique(idx).size == E.size)


GN, GSEED, GEMID, GR = 4096, 0, 0.0 + 0.0j, 0.5


def bench_general(args, mf, torch, np, gen):
    """Non-hermitian FEAST (Section 3.3) on a complex general pencil: n = 4096,
    A = B V diag(lambda) V^-1 with lambda uniform on [-2, 2] + i[-2, 2], V = I + 0.3 G / sqrt(n),
    B = I + 0.1 C C^H / n (seed 0); the eigenvalues in the circle |z| <= 0.5 with right and left
    eigenvectors (two-sided, fpm(15)=0), M0 = 1.5 times the count, 16 trapezoidal nodes,
    FP32 solves with the FP64 residual form, res <= 1e-10.  One step = one mfeast_zgegv call."""
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    A, B, lam, _, _ = gen.prescribed_nonnormal(GN, GSEED, generalized=True)
    lam_in = lam[np.abs(lam - GEMID) <= GR]
    cnt = int(lam_in.size)
    m0 = int(math.ceil(1.5 * cnt))
    print("bench: general inputs built in %.1f s (%d eigenvalues inside, M0 %d)"
          % (time.perf_counter() - t0, cnt, m0), file=sys.stderr, flush=True)
    At = torch.from_numpy(np.asfortranarray(A)).to(dev)
    Bt = torch.from_numpy(np.asfortranarray(B)).to(dev)
    E = torch.zeros(m0, dtype=torch.complex128, device=dev)
    res = torch.zeros(2 * m0, dtype=torch.float64, device=dev)
    X = torch.zeros((2 * m0, GN), dtype=torch.complex128, device=dev).mT
    h = mf.Handle(0)

    def step(profile):
        fpm = mf.mfeast_init_general()
        fpm[41] = 1
        fpm[2] = 10
        fpm[51] = 1 if profile else 0
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out = mf.mfeast_zgegv(h, GN, At, GN, Bt, GN, fpm, GEMID, GR, m0, E, X, GN, res)
        torch.cuda.synchronize()
        return out, time.perf_counter() - t1

    for _ in range(args.warmup):
        step(False)
    times = []
    for _ in range(max(1, args.steps)):
        out, t = step(False)
        times.append(t)
    out_p, _ = step(True)
    prof = h.profile()
    timing = h.timing()
    h.close()
    M, mk = out["M"], out["m0"]
    r_all = res.cpu().numpy()
    rr, rl = r_all[:mk][:M], r_all[m0:m0 + mk][:M]
    err, one_to_one = _match_err(E.cpu().numpy()[:M], lam_in, abs(GEMID) + GR)
    conv = int(np.sum((rr <= RES_BAR) & (rl <= RES_BAR)))
    t = float(np.median(times))
    print("bench: general steps %s s, M %d of %d, loop %d" % (["%.3f" % x for x in times], M, cnt, out["loop"]),
          file=sys.stderr, flush=True)
    result = {
        "metric": "converged eigenpairs/s (right and left), non-Hermitian FEAST, FP32 solves + FP64 residual form",
        "value": conv / t, "unit": "eigenpairs/s", "n_gpus": 1, "steps": len(times), "warmup": args.warmup,
        "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 solves + c128 residual/RR", "data": "synthetic",
        "config": {"workload": "complex general pencil n=4096 (seed 0), circle |z|<=0.5, two-sided, "
                               "16 trapezoidal nodes, M0=1.5x count, res<=1e-10, FP32 solves",
                   "n": GN, "m0": m0, "nodes": 16, "seed": GSEED},
        "accuracy": {"M": M, "exact_count": cnt, "max_eig_err_over_alpha": err, "one_to_one": one_to_one,
                     "max_res_right": float(rr.max()) if M else None, "max_res_left": float(rl.max()) if M else None,
                     "loop": out["loop"], "info": out["info"], "m0_out": mk},
        "timing_split_s": {"factor": timing[0], "solve": timing[1], "a_x": timing[2], "b_x": timing[3],
                           "rest": timing[4], "total": timing[5], "reduced_eig": timing[7]},
        "time_split": classes_summary(prof, t * 1e3),
        "roofline": roofline_of(prof),
        "roofline_next": roofline_of(prof, 1),
    }
    for r in (result["roofline"], result["roofline_next"]):
        if r is not None:
            r["unit_of_work"] = r["unit_of_work"].replace("all 8 nodes: the forward (L, U) and the conjugate-transpose "
                                                          "(U^H, L^H) sweeps", "all 16 nodes: the right (conjugate-"
                                                          "transpose) and left (forward) sweeps")
            if r["kernel_class"] == "reduced_eig":
                r["kernel"] = ("nh_eigensolve: Newton-Schulz inverse and Hessenberg launches, k_nh_qr (windowed "
                               "single-shift QR in one workgroup), k_nh_trivec, GEMMs")
                r["traffic"] = None  # the measured traffic figure is the Hermitian eigensolver's
                r["unit_of_work"] = ("one profiled launch group of the reduced non-Hermitian eigensolves (about 58 "
                                     "per eigensolve: the Schur step counted at a nominal 100 m^3 flops, each "
                                     "GEMM at 8 m^3)")
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline_general(A, B, m0, out["loop"], conv)
    return result


def cpu_baseline_general(A, B, m0, loop, conv):
    """The oracle's steps for the non-Hermitian workload on a bounded sample: one node's
    complex128 LU (scipy, as the oracle), its right and left solves with M0 right-hand sides,
    and one two-sided Rayleigh-Ritz step (range bases by SVD, reduced products, scipy eig
    with left and right vectors), scaled to 16 nodes and the GPU run's loop count."""
    import numpy as np
    import scipy.linalg as sla
    from oracle import nonhermitian as nh
    z, w = nh.full_contour(GEMID, GR, 16)
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((GN, m0)) + 1j * rng.standard_normal((GN, m0))
    t0 = time.perf_counter()
    fac = sla.lu_factor(z[0] * B - A)
    t_lu = time.perf_counter() - t0
    t0 = time.perf_counter()
    Q = sla.lu_solve(fac, B @ Y)
    QL = sla.lu_solve(fac, B.conj().T @ Y, trans=2)
    t_solve = time.perf_counter() - t0
    del fac
    t0 = time.perf_counter()
    Qo = nh._range_basis(Q)
    QLo = nh._range_basis(QL)
    k = min(Qo.shape[1], QLo.shape[1])
    Qo, QLo = Qo[:, :k], QLo[:, :k]
    Aq = QLo.conj().T @ (A @ Qo)
    Bq = QLo.conj().T @ (B @ Qo)
    sla.eig(Aq, Bq, left=True, right=True)
    A.conj().T @ QLo
    B.conj().T @ QLo
    t_rr = time.perf_counter() - t0
    iters = loop + 1
    t_est = 16 * (t_lu + iters * t_solve) + iters * t_rr
    return {"value": conv / t_est, "unit": "eigenpairs/s", "cores": _cores(), "cpu": _cpu_model(), "kind": "oracle",
            "sample": "one node of 16: complex128 LU (n=4096), right and left solves of %d right-hand sides, and "
                      "one two-sided Rayleigh-Ritz step, %.1f s; scaled to 16 nodes and %d loops: est. %.1f s per "
                      "call (lu %.2f s, solves %.2f s, rr %.2f s)" % (m0, t_lu + t_solve + t_rr, iters, t_est,
                                                                      t_lu, t_solve, t_rr)}


PN, PDEG, PSEED, PEMID, PR = 4096, 2, 0, 0.0 + 0.0j, 0.3


def bench_polynomial(args, mf, torch, np, gen):
    """Polynomial FEAST (Section 3.4) on a quadratic problem: n = 4096, P(lambda) =
    L (lambda - S_2)(lambda - S_1) with S_t = V_t diag(D_t) V_t^-1 (D_t uniform on
    [-2, 2] + i[-2, 2], V_t = I + 0.3 G_t / sqrt(n)) and L = I + 0.1 C C^H / n (seed 0); the
    eigenvalues in |z| <= 0.3, M0 = 1.5 times the count, 16 trapezoidal nodes, FP32 solves
    with the FP64 residual form, res <= 1e-10.  One step = one mfeast_zgepev call."""
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    As, lam, _ = gen.prescribed_polynomial(PN, PDEG, PSEED, leading=True, vectors=False)
    lam_in = lam[np.abs(lam - PEMID) <= PR]
    cnt = int(lam_in.size)
    m0 = int(math.ceil(1.5 * cnt))
    print("bench: polynomial inputs built in %.1f s (%d eigenvalues inside, M0 %d)"
          % (time.perf_counter() - t0, cnt, m0), file=sys.stderr, flush=True)
    At = torch.stack([torch.from_numpy(a).mT for a in As]).contiguous().to(dev)
    E = torch.zeros(m0, dtype=torch.complex128, device=dev)
    res = torch.zeros(m0, dtype=torch.float64, device=dev)
    X = torch.zeros((m0, PN), dtype=torch.complex128, device=dev).mT
    h = mf.Handle(0)

    def step(profile):
        fpm = mf.mfeast_init_polynomial()
        fpm[41] = 1
        fpm[2] = 10
        fpm[51] = 1 if profile else 0
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        out = mf.mfeast_zgepev(h, PDEG, PN, At, PN, fpm, PEMID, PR, m0, E, X, PN, res)
        torch.cuda.synchronize()
        return out, time.perf_counter() - t1

    for _ in range(args.warmup):
        step(False)
    times = []
    for _ in range(max(1, args.steps)):
        out, t = step(False)
        times.append(t)
    out_p, _ = step(True)
    prof = h.profile()
    timing = h.timing()
    h.close()
    M = out["M"]
    rr = res.cpu().numpy()[:M]
    err, one_to_one = _match_err(E.cpu().numpy()[:M], lam_in, abs(PEMID) + PR)
    conv = int(np.sum(rr <= RES_BAR))
    t = float(np.median(times))
    print("bench: polynomial steps %s s, M %d of %d, loop %d" % (["%.3f" % x for x in times], M, cnt, out["loop"]),
          file=sys.stderr, flush=True)
    result = {
        "metric": "converged eigenpairs/s, polynomial (quadratic) FEAST, FP32 solves + FP64 residual form",
        "value": conv / t, "unit": "eigenpairs/s", "n_gpus": 1, "steps": len(times), "warmup": args.warmup,
        "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 solves + c128 residual/RR", "data": "synthetic",
        "config": {"workload": "quadratic matrix polynomial n=4096 (seed 0, leading coefficient), circle "
                               "|z|<=0.3, 16 trapezoidal nodes, M0=1.5x count, res<=1e-10, FP32 solves",
                   "n": PN, "degree": PDEG, "m0": m0, "nodes": 16, "seed": PSEED},
        "accuracy": {"M": M, "exact_count": cnt, "max_eig_err_over_alpha": err, "one_to_one": one_to_one,
                     "max_res": float(rr.max()) if M else None, "loop": out["loop"], "info": out["info"]},
        "timing_split_s": {"factor": timing[0], "solve": timing[1], "a_x": timing[2], "rest": timing[4],
                           "total": timing[5], "reduced_eig": timing[7]},
        "time_split": classes_summary(prof, t * 1e3),
        "roofline": roofline_of(prof),
        "roofline_next": roofline_of(prof, 1),
    }
    for r in (result["roofline"], result["roofline_next"]):
        if r is not None:
            r["unit_of_work"] = r["unit_of_work"].replace("all 8 nodes: the forward (L, U) and the conjugate-transpose "
                                                          "(U^H, L^H) sweeps, which run concurrently on two streams",
                                                          "all 16 nodes: the conjugate-transpose sweeps of P(z_j)^H")
            if r["kernel_class"] == "reduced_eig":
                r["kernel"] = ("nh_eigensolve on the companion pencil: Newton-Schulz inverse and Hessenberg "
                               "launches, k_nh_qr (windowed single-shift QR in one workgroup), k_nh_trivec, GEMMs")
                r["traffic"] = None  # the measured traffic figure is the Hermitian eigensolver's
                r["unit_of_work"] = ("one profiled launch group of the companion eigensolves of order 2 m (the "
                                     "Schur step counted at a nominal 100 (2m)^3 flops, each GEMM at 8 (2m)^3)")
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline_polynomial(As, m0, out["loop"], conv)
    return result


def cpu_baseline_polynomial(As, m0, loop, conv):
    """The oracle's steps for the polynomial workload on a bounded sample: forming P(z_j) and
    its complex128 LU for one node, one solve with M0 right-hand sides, and one
    Rayleigh-Ritz step (range basis, the p + 1 projected coefficients, scipy eig of the
    companion pencil), scaled to 16 nodes and the GPU run's loop count."""
    import numpy as np
    import scipy.linalg as sla
    from oracle import nonhermitian as nh
    from oracle import polynomial as po
    z, w = nh.full_contour(PEMID, PR, 16)
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((PN, m0)) + 1j * rng.standard_normal((PN, m0))
    t0 = time.perf_counter()
    fac = sla.lu_factor(po.poly_eval(As, z[0]))
    t_lu = time.perf_counter() - t0
    t0 = time.perf_counter()
    Q = sla.lu_solve(fac, Y)
    t_solve = time.perf_counter() - t0
    del fac
    t0 = time.perf_counter()
    Qo = nh._range_basis(Q)
    m = Qo.shape[1]
    Aq = [Qo.conj().T @ (Ak @ Qo) for Ak in As]
    L0 = np.zeros((2 * m, 2 * m), dtype=np.complex128)
    L1 = np.zeros_like(L0)
    L0[:m, m:] = np.eye(m)
    L1[:m, :m] = np.eye(m)
    L0[m:, :m] = -Aq[0]
    L0[m:, m:] = -Aq[1]
    L1[m:, m:] = Aq[2]
    sla.eig(L0, L1)
    t_rr = time.perf_counter() - t0
    iters = loop + 1
    t_est = 16 * (t_lu + iters * t_solve) + iters * t_rr
    return {"value": conv / t_est, "unit": "eigenpairs/s", "cores": _cores(), "cpu": _cpu_model(), "kind": "oracle",
            "sample": "one node of 16: P(z) and its complex128 LU (n=4096), one solve of %d right-hand sides, and "
                      "one Rayleigh-Ritz step with the companion eigensolve, %.1f s; scaled to 16 nodes and %d "
                      "loops: est. %.1f s per call (lu %.2f s, solves %.2f s, rr %.2f s)"
                      % (m0, t_lu + t_solve + t_rr, iters, t_est, t_lu, t_solve, t_rr)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: runs on one GPU only; --gpus %d is not supported "
              "(the contour nodes would shard across GPUs with one all-reduce of Q per iteration)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2002_04807_amd as mf
    from workloads import generators as gen

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.workload != "pencil":
        fn = {"sparse": bench_sparse, "batched": bench_batched, "adjoint": bench_adjoint,
              "count": bench_count, "general": bench_general, "polynomial": bench_polynomial}[args.workload]
        print(json.dumps(fn(args, mf, torch, np, gen)))
        return
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    A, B, lam, _ = gen.prescribed_complex_pencil(N, seed=SEED)
    lam_in = np.sort(lam[(lam >= EMIN) & (lam <= EMAX)])
    print("bench: inputs built in %.1f s (%d eigenvalues in the interval)" % (time.perf_counter() - t0, lam_in.size),
          file=sys.stderr, flush=True)
    At = torch.from_numpy(np.asfortranarray(A)).to(dev)
    Bt = torch.from_numpy(np.asfortranarray(B)).to(dev)
    h = mf.Handle(0)

    if args.profile_steps:
        # calibration for hardware traffic counters: one plain device copy of 256 MiB
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        outs, times, _ = run_steps(mf, torch, h, At, Bt, True, args.profile_steps, False)
        print("bench: profile run %s s, M=%s" % (["%.3f" % t for t in times], [o["M"] for o in outs]),
              file=sys.stderr, flush=True)
        h.close()
        return

    run_steps(mf, torch, h, At, Bt, True, args.warmup, False)
    outs, times, profs = run_steps(mf, torch, h, At, Bt, True, args.steps, True)
    print("bench: fp32+IR steps %s s" % ["%.3f" % t for t in times], file=sys.stderr, flush=True)
    acc = [accuracy(o, lam_in) for o in outs]
    t_step = float(np.median(times))
    m_conv = min(a["converged_pairs"] for a in acc)
    value = m_conv / t_step

    # contour-solve TFLOP/s from the device profile of the timed steps: algorithmic flops of
    # the factorizations and of every contour's solves (8 per complex multiply-add) over
    # the device time of shift-form, LU (panel, row operations, inverses, trailing update),
    # block solves and quadrature sums
    loops = outs[-1]["loop"] + 1
    f_alg = NE * (8.0 / 3.0) * N ** 3 + loops * (2 * NE) * 8.0 * N * N * M0
    prof = profs[-1]
    t_contour = sum(prof[c]["ms"] for c in CONTOUR_CLASSES) / 1e3
    contour_tflops = f_alg / t_contour / 1e12 if t_contour > 0 else None

    roofline = roofline_of(prof, workload="pencil")
    # the second-largest class's roofline is reported beside the first
    roofline_next = roofline_of(prof, 1, workload="pencil")

    if roofline is not None and roofline["kernel_class"] == "contour_solve":
        roofline["rate"] = ("effective: algorithmic flops (8 per complex multiply-add) over time; the kernel "
                            "issues Gauss's three real products per complex multiply-add and full panel inverses")
        roofline["issued_mfma_frac"] = roofline["frac"] * SOLVE_ISSUED_PER_ALG
    for r in (roofline, roofline_next):
        if r is not None and r["kernel_class"] == "rr_gemm":
            r["rate"] = ("effective: algorithmic flops (8 per complex multiply-add) over time; the complex FP64 "
                         "products issue Gauss's three real products per complex multiply-add")
            r["issued_mfma_frac"] = r["frac"] * 6.0 / 8.0
    result = {
        "metric": METRIC, "value": value, "unit": "eigenpairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_step * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64 solves + f64 residual/RR", "data": "synthetic",
        "config": {"workload": "generalized complex Hermitian n=4096, M0=600, 8-node Gauss half contour, "
                               "interval [-1,1], res<=1e-10, FP32+IR (fpm42=1)",
                   "n": N, "m0": M0, "nodes": NE, "seed": SEED},
        "contour_tflops": contour_tflops,
        "contour_tflops_kind": "effective (algorithmic flops; three-product complex FP32 MFMA)",
        "time_split": classes_summary(prof, float(np.median(times)) * 1e3),
        "accuracy": acc[-1],
        "roofline": roofline,
        "roofline_next": roofline_next,
    }

    if not args.no_fp64:
        run_steps(mf, torch, h, At, Bt, False, 1, False)
        outs64, times64, profs64 = run_steps(mf, torch, h, At, Bt, False, max(1, args.steps), True)
        print("bench: fp64 steps %s s" % ["%.3f" % t for t in times64], file=sys.stderr, flush=True)
        acc64 = [accuracy(o, lam_in) for o in outs64]
        t64 = float(np.median(times64))
        v64 = min(a["converged_pairs"] for a in acc64) / t64
        loops64 = outs64[-1]["loop"] + 1
        f64_alg = NE * (8.0 / 3.0) * N ** 3 + loops64 * (2 * NE) * 8.0 * N * N * M0
        p64 = profs64[-1]
        t64c = sum(p64[c]["ms"] for c in CONTOUR_CLASSES) / 1e3
        result["fp64_plain"] = {"value": v64, "ms_per_step": t64 * 1e3, "accuracy": acc64[-1],
                                "contour_tflops": f64_alg / t64c / 1e12 if t64c > 0 else None,
                                "time_split": classes_summary(p64, t64 * 1e3)}
        result["speedup_fp32ir_vs_fp64"] = value / v64 if v64 > 0 else None
        loops_cpu = outs64[-1]["loop"]
    else:
        loops_cpu = outs[-1]["loop"]

    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        result["cpu_baseline"] = cpu_baseline(A, B, lam_in, loops_cpu)
        print("bench: cpu baseline sample took %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)
    h.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
