#!/usr/bin/env python
"""Benchmark: systems solved per second on a shifted convection-diffusion sequence.

Workload: 3D 7-point upwind convection-diffusion, 64^3 grid (n = 262,144),
A(i) = K + sigma_i M with 5 log-spaced shifts in [1e-2, 1e1] times 4 N(0,1)
right-hand sides (20 systems), recycle dimension k = 20, true relative
residual 1e-8.  One step = the whole sequence: per shift the matrix setup
(sliced copy, C = A U, Ct = A^T Ut, bi-orthogonalisation), RBiCG on the first
right-hand side with the recycle-space update from its Lanczos vectors, and
RBiCGSTAB on the other three, solved together (the same iterates as three
separate solves, with the matrix and block reads shared).  The same sequence
is also timed with plain BiCGSTAB on the same kernels (the baseline the
metric compares against, its four right-hand sides per matrix solved
together), and both again one system at a time and with FP32 storage under
FP64 refinement.

Prints one JSON line.  Inputs are generated and uploaded before timing.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFLOPS = 78.6
K_BUCKETS = (0, 4, 8, 12, 16, 20, 24, 28, 32, 40, 48, 56, 64)


def k_bucket(k):
    """Template instantiation (recycle-dimension bucket) the library launches for k."""
    return next(b for b in K_BUCKETS if b >= k)


def counter_traffic(kernel):
    """Calibrated HBM bytes per dispatch of `kernel` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summaries in profiles/, or None when there is no
    summary for it or the kernel source has changed since the counters were taken."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_1406_2831_amd", "csrc", "kernels.hip")
    with open(src, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_hbm_counters.md"))):
        kv = {}
        with open(path) as f:
            for line in f:
                key, sep, val = line.partition(":")
                if sep and key.strip() in ("kernel", "kernels_hip_sha256", "fetch_kib_per_dispatch",
                                           "write_kib_per_dispatch", "fetch_scale", "write_scale"):
                    kv[key.strip()] = val.strip()
        if kv.get("kernel") != kernel or kv.get("kernels_hip_sha256") != digest:
            continue
        return 1024.0 * (float(kv["fetch_kib_per_dispatch"]) * float(kv["fetch_scale"])
                         + float(kv["write_kib_per_dispatch"]) * float(kv["write_scale"]))
    return None


def cpu_baseline(seq, rtol, systems):
    """The oracle (CPU FP64) on a bounded sample of the same sequence."""
    import oracle as o
    threads = os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        if info:
            threads = max(int(p.get("num_threads", 1)) for p in info)
    except Exception:
        pass
    t0 = time.perf_counter()
    res = o.run_sequence(seq, mode="rbicgstab", rtol=rtol, systems=systems)
    dt = time.perf_counter() - t0
    nr = seq.nrhs
    nshift = (systems + nr - 1) // nr
    return {"value": systems / dt, "unit": "systems/s", "cores": threads, "kind": "oracle",
            "sample": f"first {systems} systems of the sequence ({nshift} shift(s); per shift RBiCG on "
                      f"the first right-hand side, RBiCGSTAB on the others), {dt:.1f} s, "
                      f"iterations {res.iters}",
            "seconds": dt}


def adjoint_workload(args):
    """Gradients of L = c^T x, x = A(sigma)^-1 b, A = K + sigma M on a 3D 7-point
    grid (default 128^3, n = 2,097,152): one step = forward RBiCGSTAB solve with the
    recycle space + transposed RBiCGSTAB solve reusing it (swapped) + the gradient
    kernel (dL/db, dL/dsigma, dL/dK values).  The space comes from one RBiCG
    forward solve before timing.  After timing, directional derivatives are
    checked against central differences (step 1e-6, solves at rtol 1e-12)."""
    import numpy as np
    import torch
    import workloads as w
    from paper_1406_2831_amd.adjoint import ShiftedSystem, recycled_solve

    N = args.grid if args.grid != 64 else 128
    seq, c, bdirs = w.adjoint_problem(N=N, ndirs=args.fd_dirs)
    K, mdiag, sigma, b = seq.K, seq.mdiag, float(seq.sigmas[0]), seq.rhs[0]
    sysm = ShiftedSystem(K, mdiag, k_max=args.k, s_max=512, secant_max=args.secant_max)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    bt = dev(b).requires_grad_(True)
    sg = torch.tensor(sigma, dtype=torch.float64, device="cuda", requires_grad=True)
    kv = dev(K.val).requires_grad_(True)
    ct = dev(c)
    rtol = args.rtol

    def step(mode="rbicgstab"):
        for t in (bt, sg, kv):
            t.grad = None
        x = recycled_solve(sysm, bt, sg, kv, rtol, 20000, mode)
        (x * ct).sum().backward()
        return x

    x = step("rbicg")                       # builds and installs the recycle space
    k_used = sysm.ctx.blocks()[1]
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    fwd = sysm.ctx.solve(bt.detach(), rtol=rtol, mode="rbicgstab")[1]
    adj = sysm.ctx.solve(ct, rtol=rtol, mode="rbicgstab", transpose=True)[1]
    # the same with plain BiCGSTAB forward and adjoint (the non-recycling baseline)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step("bicgstab")
    torch.cuda.synchronize()
    dt0 = (time.perf_counter() - t0) / args.steps
    # finite-difference check of the gradient on random directions
    gb, gs, gk = bt.grad.cpu().numpy(), sg.grad.item(), kv.grad.cpu().numpy()
    step()
    gb, gs, gk = bt.grad.cpu().numpy(), sg.grad.item(), kv.grad.cpu().numpy()
    dirs = w.generator(3, 1, "dirs")
    h, fds, ans = 1e-6, [], []
    for i in range(args.fd_dirs):
        db, ds = bdirs[i], dirs.standard_normal()
        dk = dirs.standard_normal(K.nnz) * np.abs(K.val)
        vals = []
        for sgn in (1.0, -1.0):
            with torch.no_grad():
                xp, _ = sysm.solve(dev(b + sgn * h * db), sigma + sgn * h * ds, dev(K.val + sgn * h * dk),
                                   rtol=1e-12, max_it=50000)
                vals.append(float((xp * ct).sum().item()))
        fds.append((vals[0] - vals[1]) / (2 * h))
        ans.append(gb @ db + gs * ds + gk @ dk)
    fds, ans = np.array(fds), np.array(ans)
    fd_err = float(np.max(np.abs(fds - ans)) / np.sqrt(np.mean(ans ** 2)))
    out = {
        "metric": "gradient evaluations/s (forward + transposed recycled solve + gradients)",
        "value": 1.0 / dt, "unit": "gradients/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"adjoint of c^T x on 3d 7-point convection-diffusion {N}^3 "
                               f"(n={seq.n}), sigma={sigma}, k={args.k}, rtol={rtol}",
                   "n": seq.n, "nnz": int(K.nnz), "k_used": k_used},
        "forward_iters": fwd.iters, "adjoint_iters": adj.iters,
        "bicgstab_ms_per_step": dt0 * 1e3,
        "fd_check": {"directions": args.fd_dirs, "step": h, "max_err_over_rms": fd_err},
    }
    sysm.close()
    print(json.dumps(out), flush=True)


def batched_workload(args):
    """32 shifted 3D 7-point systems of uneven size (n from 40k to 500k, velocities
    U[-1,1]^3, sigma log-spaced in [1e-2, 1e1]), k = 16.  A first, untimed pass builds
    each system's recycle space by RBiCG; the timed step solves all 32 systems with
    their spaces in one batch (persistent tile-walking passes, tuned tiles, graph
    replay).  Also timed: the same solves one system at a time, and BiCGSTAB batched."""
    import numpy as np
    import torch
    import workloads as w
    from paper_1406_2831_amd.rbicgstab import Batch, Context
    from paper_1406_2831_amd.sequence import max_row_nnz

    k = 16
    systems = w.batched_systems(count=args.batch_count)
    ctxs, bs, shs = [], [], []
    gen_iters = []
    for (A, At, b, sh) in systems:
        ctx = Context(A.n, max_row_nnz(A, At), k, 256, "cuda", args.secant_max)
        ctx.setup(A, At)
        bt = torch.as_tensor(b, device="cuda")
        st = ctx.solve(bt, torch.zeros_like(bt), rtol=args.rtol, max_it=20000, mode="rbicg")[1]
        ctx.recycle("from_last_solve")
        gen_iters.append(st.iters)
        ctxs.append(ctx)
        bs.append(bt)
        shs.append(torch.as_tensor(sh, device="cuda"))
    k_used = [c.blocks()[1] for c in ctxs]
    ns = [c.n for c in ctxs]
    nnzs = [int(s[0].nnz) for s in systems]
    batch = Batch(ctxs, tune=True, graph=True)
    cfg = batch.config()
    xs = [torch.zeros_like(b) for b in bs]

    def run_batch(mode, precision="fp64"):
        for x in xs:
            x.zero_()
        sts = batch.solve(bs, xs, shs, rtol=args.rtol, max_it=20000, mode=mode, precision=precision)
        if any(s.status != 0 or s.rel_res_true > args.rtol for s in sts):
            print(f"batched {mode} {precision}: not every system converged", file=sys.stderr)
            sys.exit(1)
        return sts

    def run_single(mode):
        out = []
        for ctx, b, sh, x in zip(ctxs, bs, shs, xs):
            x.zero_()
            out.append(ctx.solve(b, x, shadow=sh, rtol=args.rtol, max_it=20000, mode=mode)[1])
        return out

    timed, errs = {}, {}
    x64 = None
    for key, fn, mode, prec in (("rbicgstab_batched", run_batch, "rbicgstab", "fp64"),
                                ("bicgstab_batched", run_batch, "bicgstab", "fp64"),
                                ("rbicgstab_batched_fp32_ir", run_batch, "rbicgstab", "fp32_ir"),
                                ("bicgstab_batched_fp32_ir", run_batch, "bicgstab", "fp32_ir"),
                                ("rbicgstab_single", run_single, "rbicgstab", "fp64"),
                                ("bicgstab_single", run_single, "bicgstab", "fp64")):
        call = (lambda: fn(mode, prec)) if fn is run_batch else (lambda: fn(mode))
        for _ in range(args.warmup):
            call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            sts = call()
        torch.cuda.synchronize()
        timed[key] = ((time.perf_counter() - t0) / args.steps, [s.iters for s in sts])
        if key == "rbicgstab_batched":
            x64 = [x.clone() for x in xs]
        elif prec == "fp32_ir":   # error of each FP32-storage result against the FP64 batch's
            errs[key] = [float(torch.linalg.norm(x - xr) / torch.linalg.norm(xr)) for x, xr in zip(xs, x64)]
    nsys = len(ctxs)
    # the three batched passes moved these algorithmic bytes in one tuned iteration
    byts = sum((80 * n + 8 * n * kk) + (12 * nz + 4 * (n + 1) + 32 * n + 16 * n * kk)
               + (12 * nz + 4 * (n + 1) + 24 * n + 8 * n * kk) for n, nz, kk in zip(ns, nnzs, k_used))
    ach = byts / (cfg["tuned_ms_per_iter"] * 1e-3) / 1e9 if cfg["tuned_ms_per_iter"] > 0 else None
    out = {
        "metric": "systems solved/s at rel.res 1e-8, batched RBiCGSTAB (32 uneven shifted systems)",
        "value": nsys / timed["rbicgstab_batched"][0], "unit": "systems/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": timed["rbicgstab_batched"][0] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{nsys} shifted 3d 7-point convection-diffusion systems, n {min(ns)}-{max(ns)} "
                               f"(sum {sum(ns)}), k={k}, rtol={args.rtol}; spaces from one RBiCG solve each",
                   "n": ns, "k_used": k_used},
        "tuned": cfg,
        "iters": {key: v[1] for key, v in timed.items()},
        "systems_per_s": {key: nsys / v[0] for key, v in timed.items()},
        "rbicg_iters_round1": gen_iters,
        "fp32_ir": {"err_vs_fp64": errs, "max_err_vs_fp64": max(max(v) for v in errs.values()),
                    "note": "FP32 storage under FP64 refinement; inner FP32 solves batched, "
                            "launched directly (no graph replay)"},
        "roofline": {"bound": "hbm", "kernel": "k_batch_update + k_batch_spmv1 + k_batch_spmv2 (one iteration)",
                     "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS if ach else None, "traffic": None,
                     "bytes_per_launch": byts, "us_per_launch": cfg["tuned_ms_per_iter"] * 1e3},
    }
    batch.close()
    for c in ctxs:
        c.close()
    print(json.dumps(out), flush=True)


def large_workload(args):
    """The 27-point nonsymmetric stencil on 160^3 (n = 4,096,000, nnz = 109,215,352),
    k = 30, first --large-shifts shifts x 5 right-hand sides of the 10-shift sequence:
    RBiCG (FP64) on the first right-hand side of each shift, then RBiCGSTAB with FP32
    storage under FP64 refinement on the others; BiCGSTAB (FP32-IR) on all as the
    baseline.  One step, no warm-up (each run takes seconds).  Also times the fused
    passes in FP32 and FP64 at this HBM-resident size."""
    import torch
    import workloads as w
    from paper_1406_2831_amd.sequence import GpuSequence

    N = args.grid if args.grid != 64 else 160
    seq = w.seq_3d27(N=N, nshift=10, nrhs=5, k=30)
    nsys = args.large_shifts * seq.nrhs
    # keep the first shifts only (the sequence's systems are shift-major)
    seq.sigmas = seq.sigmas[: args.large_shifts]
    seq.rhs, seq.shadows = seq.rhs[:nsys], seq.shadows[:nsys]
    gs = GpuSequence(seq, s_max=512, secant_max=args.secant_max)
    res, timed = {}, {}
    for key, mode, prec in (("rbicgstab_fp32_ir", "rbicgstab", "fp32_ir"),
                            ("bicgstab_fp32_ir", "bicgstab", "fp32_ir"),
                            ("rbicgstab_fp64", "rbicgstab", "fp64")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = gs.run(mode=mode, rtol=args.rtol, max_it=40000, precision=prec)
        torch.cuda.synchronize()
        timed[key] = time.perf_counter() - t0
        res[key] = r
        if any(s_ != 0 for s_ in r.status) or max(r.rel_res_true) > args.rtol:
            print(f"{key}: not every system converged: {r.status} {r.rel_res_true}", file=sys.stderr)
            sys.exit(1)
    k_last = int(res["rbicgstab_fp32_ir"].k_used[-1])
    gbs = lambda b, ms: b / (ms * 1e-3) / 1e9
    passes = {}
    for name, which, kk in (("spmv1_project_fp32", 5, k_last), ("update_fp32", 4, k_last),
                            ("spmv2_project_fp32", 6, k_last), ("spmv_fp32", 7, 0),
                            ("spmv1_project", 1, k_last), ("update", 0, k_last),
                            ("spmv2_project", 2, k_last), ("spmv", 3, 0)):
        ms, by = gs.ctx.time_pass(which, kk, 20)
        passes[name] = {"us": ms * 1e3, "gbs": gbs(by, ms), "bytes": by}
    dom = passes["spmv1_project_fp32"]
    out = {
        "metric": "systems solved/s at rel.res 1e-8 (FP64 true residual), RBiCGSTAB FP32-IR",
        "value": nsys / timed["rbicgstab_fp32_ir"], "unit": "systems/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": timed["rbicgstab_fp32_ir"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 storage / f64 refinement",
        "data": "synthetic",
        "config": {"workload": f"3d 27-point convection-diffusion {N}^3 (n={seq.n}, nnz={seq.K.nnz}), "
                               f"first {args.large_shifts} of 10 shifts x 5 rhs = {nsys} systems, k=30, "
                               f"rtol={args.rtol}", "n": seq.n, "nnz": int(seq.K.nnz)},
        "systems_per_s": {k_: nsys / v for k_, v in timed.items()},
        "iters": {k_: r.iters for k_, r in res.items()},
        "k_used": res["rbicgstab_fp32_ir"].k_used,
        "matvecs": {k_: r.total_matvecs for k_, r in res.items()},
        "passes": dict(passes, k=k_last),
        "roofline": {"bound": "hbm", "kernel": f"k_spmv1<float, {k_bucket(k_last)}>",
                     "achieved": dom["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dom["gbs"] / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": dom["bytes"], "us_per_launch": dom["us"]},
    }
    gs.close()
    print(json.dumps(out), flush=True)


def study_workload(args):
    """Choices of the recycle-space generation, measured on the sequence (GPU,
    multi-RHS RBiCGSTAB pipeline, one warm-up and one timed run per setting):
    the RBiCG cycle length s_max (the Ritz step runs every s_max stored vectors;
    Section 6.2 uses 25), the oblique-projector cap secant_max, and RBiCG's
    stopping rule (both residuals, as in Section 3, or the primary alone).
    Reports iterations, recycle dimensions, products and time per setting."""
    import torch
    import workloads as w
    from paper_1406_2831_amd.sequence import GpuSequence

    seq = w.seq_3d(N=args.grid, k=args.k)
    nsys = seq.num_systems
    settings = [("bicgstab", 512, 0.0, "both", "bicgstab")]
    settings += [(f"s_max={s_}", s_, 0.0, "both", "rbicgstab") for s_ in (25, 50, 128, 256, 512)]
    settings += [(f"secant_max={c_:g}", 512, c_, "both", "rbicgstab") for c_ in (10.0, 1e3, 1e4, float("inf"))]
    settings += [("stop=primary", 512, 0.0, "primary", "rbicgstab")]
    rows = {}
    for name, s_max, cap, stop, mode in settings:
        gs = GpuSequence(seq, s_max=s_max, secant_max=cap, keep_x=False)
        r = None
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = gs.run(mode=mode, rtol=args.rtol, multi_rhs=True, rbicg_stop=stop)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        gen = [sv == "rbicg" for sv in r.solver]
        rows[name] = {"systems_per_s": nsys / dt, "ms": dt * 1e3, "iters": r.iters, "k_used": r.k_used,
                      "matvecs": r.total_matvecs, "status": r.status,
                      "rbicgstab_iters": sum(i for i, g in zip(r.iters, gen) if not g),
                      "rbicg_iters": sum(i for i, g in zip(r.iters, gen) if g),
                      "ritz_ms": sum(r.ritz_ms), "ritz_m": r.ritz_m,
                      "converged": all(st == 0 for st in r.status) and max(r.rel_res_true) <= args.rtol}
        gs.close()
        del gs
        torch.cuda.empty_cache()
        print(f"[study] {name}: {rows[name]['systems_per_s']:.1f} systems/s, "
              f"rbicgstab iters {rows[name]['rbicgstab_iters']}, k {r.k_used}", file=sys.stderr, flush=True)
    print(json.dumps({"workload": f"recycle-space choices, 3d 7-point {args.grid}^3, 5 shifts x 4 rhs, "
                                  f"k={args.k}, rtol={args.rtol}", "settings": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=64, help="grid points per axis")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--k", type=int, default=20)
    ap.add_argument("--cpu-systems", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--time-reps", type=int, default=100)
    ap.add_argument("--calib-copy-mib", type=int, default=256,
                    help="size of the known-size copy used to calibrate HBM counters (0: skip)")
    ap.add_argument("--s-max", type=int, default=512,
                    help="Lanczos vectors stored per RBiCG cycle (the Ritz step runs every s_max vectors)")
    ap.add_argument("--no-hbm128", action="store_true",
                    help="skip the fused-pass timing at 128^3 (HBM-resident working set)")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the FP32-storage / FP64-refinement runs (reported beside the FP64 line)")
    ap.add_argument("--secant-max", type=float, default=0.0,
                    help="oblique-projector cap of the recycle setup (0: library default)")
    ap.add_argument("--workload", choices=("sequence", "adjoint", "batched", "large", "study"),
                    default="sequence",
                    help="sequence: the shifted 64^3 sequence (default); adjoint: gradients of "
                         "c^T x on the 128^3 problem through the transposed recycled solve; "
                         "batched: 32 shifted systems of uneven size solved together; large: the "
                         "27-point 160^3 sequence with FP32 storage under FP64 refinement; study: "
                         "cycle length, projector cap and RBiCG stopping rule on the sequence")
    ap.add_argument("--large-shifts", type=int, default=2,
                    help="large workload: shifts of the 10-shift sequence run (a stated subset)")
    ap.add_argument("--batch-count", type=int, default=32)
    ap.add_argument("--fd-dirs", type=int, default=16,
                    help="adjoint workload: finite-difference directions checked after timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}): the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    if args.workload == "adjoint":
        return adjoint_workload(args)
    if args.workload == "batched":
        return batched_workload(args)
    if args.workload == "large":
        return large_workload(args)
    if args.workload == "study":
        return study_workload(args)

    import numpy as np
    import torch
    import workloads as w
    from paper_1406_2831_amd.sequence import GpuSequence

    seq = w.seq_3d(N=args.grid, k=args.k)
    gs = GpuSequence(seq, s_max=args.s_max, secant_max=args.secant_max)
    nsys = seq.num_systems
    n, nnz = seq.n, int(seq.K.nnz)

    def run(mode, precision="fp64", multi=False):
        return gs.run(mode=mode, rtol=args.rtol, precision=precision, multi_rhs=multi)

    # variants of the same sequence: (key, solver mode, precision, multi-RHS)
    variants = [("rbicgstab", "rbicgstab", "fp64", True), ("bicgstab", "bicgstab", "fp64", True),
                ("rbicgstab_single", "rbicgstab", "fp64", False),
                ("bicgstab_single", "bicgstab", "fp64", False)]
    if not args.no_fp32:
        variants += [("rbicgstab_fp32_ir", "rbicgstab", "fp32_ir", False),
                     ("bicgstab_fp32_ir", "bicgstab", "fp32_ir", False)]
    for _ in range(args.warmup):
        for _key, mode, prec, multi in variants:
            run(mode, prec, multi)
    timed, results = {}, {}
    x64 = None
    for key, mode, prec, multi in variants:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            results[key] = run(mode, prec, multi)
        torch.cuda.synchronize()
        timed[key] = (time.perf_counter() - t0) / args.steps
        res = results[key]
        if any(s != 0 for s in res.status) or max(res.rel_res_true) > args.rtol:
            print(f"{key}: not every system converged: status {res.status}, "
                  f"iters {res.iters}, k {res.k_used}, solver {res.solver}, "
                  f"true residuals {res.rel_res_true}", file=sys.stderr)
            sys.exit(1)
        if key == "rbicgstab":
            x64 = [x.clone() for x in res.x]
        elif prec == "fp32_ir":
            # error of each FP32-storage result against the FP64 pipeline's; the
            # RBiCG systems run in FP64 in both pipelines and are left out
            res.err_vs_fp64 = [float(torch.linalg.norm(x - xr) / torch.linalg.norm(xr))
                               for x, xr, sv in zip(res.x, x64, res.solver) if sv != "rbicg"]
    rres = results["rbicgstab"]

    # parity at the benchmark's tolerance on a sampled system: the second system
    # (first RBiCGSTAB solve) of each pipeline against the oracle's BiCGSTAB at
    # rtol 1e-12 on the host; bound kappa * rtol with kappa ~ 4 / (pi h)^2
    sample = 1
    A0, _ = seq.matrix(seq.system(sample)[0])
    kappa = 4.0 / (np.pi / (args.grid + 1)) ** 2
    parity = {"system": sample, "bound": kappa * args.rtol, "kappa": kappa}
    if not args.no_cpu_baseline:
        import oracle as o
        xo, io = o.bicgstab(A0.to_scipy(), seq.rhs[sample], shadow=seq.shadows[sample], rtol=1e-12)
        for key in results:
            xg = results[key].x[sample].cpu().numpy()
            parity[key] = float(np.linalg.norm(xg - xo) / np.linalg.norm(xo))
        parity["within_bound"] = all(v <= parity["bound"] for k_, v in parity.items() if k_ in results)

    # where the headline pipeline's time and products go (last timed step)
    is_gen = [sv == "rbicg" for sv in rres.solver]
    ritz_ms = sum(rres.ritz_ms)
    phases = {
        "setup_and_install_ms": rres.setup_ms,
        "rbicg_ms": sum(ms for ms, g in zip(rres.ms, is_gen) if g) - ritz_ms,
        "ritz_ms": ritz_ms,
        "rbicgstab_ms": sum(ms for ms, g in zip(rres.ms, is_gen) if not g),
        "ritz_m": rres.ritz_m,
        "matvecs_setup": rres.setup_matvecs,
        "matvecs_rbicg_and_ritz": sum(mv for mv, g in zip(rres.matvecs, is_gen) if g),
        "matvecs_rbicgstab": sum(mv for mv, g in zip(rres.matvecs, is_gen) if not g),
        "note": "rbicg_ms excludes the Ritz steps, which run inside the RBiCG solve calls",
    }

    # end-to-end time per iteration against the byte model (one system at a time):
    # B_0 = 2 (12 nnz + 4 (n+1) + 16 n) + 128 n per BiCGSTAB iteration,
    # B_R(k) = B_0 + 16 n + 32 n k per RBiCGSTAB iteration (projections and x_c)
    spmv_b = 12 * nnz + 4 * (n + 1) + 16 * n
    B0 = 2 * spmv_b + 128 * n
    BR = lambda kk: 2 * spmv_b + 144 * n + 32 * n * kk
    r1, b1 = results["rbicgstab_single"], results["bicgstab_single"]
    it_b = sum(b1.iters)
    us_b = sum(b1.ms) * 1e3 / it_b
    stab = [(ms, it, kk) for ms, it, kk, sv in zip(r1.ms, r1.iters, r1.k_used, r1.solver) if sv == "rbicgstab"]
    it_r = sum(it for _, it, _ in stab)
    us_r = sum(ms for ms, _, _ in stab) * 1e3 / it_r
    br_avg = sum(BR(kk) * it for _, it, kk in stab) / it_r
    per_iter = {
        "bicgstab_us": us_b, "bicgstab_bytes": B0, "bicgstab_frac": B0 / (us_b * 1e-6) / 1e9 / HBM_PEAK_GBS,
        "rbicgstab_us": us_r, "rbicgstab_bytes": br_avg,
        "rbicgstab_frac": br_avg / (us_r * 1e-6) / 1e9 / HBM_PEAK_GBS,
        "note": "host wall time of the solve calls / iterations (prologue, true residual and polling included)",
    }

    # live per-kernel timing of the fused passes (outside the timed steps) with the
    # space the first matrix's RBiCG solve generates: the multi-RHS passes for that
    # matrix's other right-hand sides, the single-system passes (FP64 and FP32
    # storage) and a plain product.  (The space at the end of the sequence depends
    # on rounding through five Ritz steps; the first one does not.)
    gs.run(mode="rbicgstab", rtol=args.rtol, systems=1)
    k_last = int(gs.ctx.blocks()[1])
    nr = seq.nrhs - 1
    gbs = lambda b, ms: b / (ms * 1e-3) / 1e9
    passes = {}
    for name, which, kk in (("mspmv1_project", 8 + 4 * (nr - 1) + 1, k_last),
                            ("mupdate", 8 + 4 * (nr - 1), k_last),
                            ("mspmv2_project", 8 + 4 * (nr - 1) + 2, k_last),
                            ("spmv1_project", 1, k_last), ("update", 0, k_last),
                            ("spmv2_project", 2, k_last), ("spmv", 3, 0),
                            ("spmv1_project_fp32", 5, k_last), ("update_fp32", 4, k_last),
                            ("spmv2_project_fp32", 6, k_last), ("spmv_fp32", 7, 0)):
        ms, by = gs.ctx.time_pass(which, kk, args.time_reps)
        passes[name] = {"us": ms * 1e3, "gbs": gbs(by, ms), "frac": gbs(by, ms) / HBM_PEAK_GBS}

    # the kernel with the largest share of device time in the timed pipeline is the
    # Ritz step's Gram product kernel, whose interior 128 x 128 tile class
    # (kernel k_gemmt_mfma_dl) does most of its work (rocprofv3 kernel
    # statistics in profiles/): per Ritz step five symmetric X^T X (upper-triangle
    # tiles) and three X^T Y; each is timed live as that class's launch alone
    # (2 n 128^2 flops per tile) at the median m of the timed run's Ritz steps on
    # the context's stream (after everything that needs the RBiCG store)
    m_ritz = int(np.median([m for m in rres.ritz_m if m > 0]))
    reps = max(3, args.time_reps // 20)
    t_sym, f_sym = gs.ctx.time_pass(40, m_ritz, reps)
    t_gen, f_gen = gs.ctx.time_pass(41, m_ritz, reps)
    t_ts, f_ts = gs.ctx.time_pass(42, m_ritz, reps)
    gram_tflops = (5 * f_sym + 3 * f_gen) / ((5 * t_sym + 3 * t_gen) * 1e-3) / 1e12
    ritz_kernels = {
        "m": m_ritz, "n": n,
        "gemmt_sym": {"us": t_sym * 1e3, "tflops": f_sym / (t_sym * 1e-3) / 1e12, "flops": f_sym},
        "gemmt_gen": {"us": t_gen * 1e3, "tflops": f_gen / (t_gen * 1e-3) / 1e12, "flops": f_gen},
        "gemm_ts": {"us": t_ts * 1e3, "tflops": f_ts / (t_ts * 1e-3) / 1e12, "flops": f_ts},
    }

    def summary(key):
        r = results[key]
        return {"systems_per_s": nsys / timed[key], "ms_per_step": timed[key] * 1e3, "iters": r.iters,
                "matvecs": r.total_matvecs, "max_rel_res_true": max(r.rel_res_true)}

    out = {
        "metric": "systems solved/s + SpMV HBM GB/s at rel.res 1e-8, RBiCGSTAB vs BiCGSTAB",
        "value": nsys / timed["rbicgstab"],
        "unit": "systems/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": timed["rbicgstab"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3d 7-point convection-diffusion {args.grid}^3 (n={n}), "
                               f"5 shifts x 4 rhs = {nsys} systems, k={args.k}, rtol={args.rtol}; "
                               f"per shift RBiCG on rhs 1, RBiCGSTAB on rhs 2-4 solved together",
                   "n": n, "nnz": nnz, "systems": nsys, "k": args.k, "s_max": args.s_max},
        "rbicgstab": dict(summary("rbicgstab"), solver=rres.solver, k_used=rres.k_used),
        "bicgstab": summary("bicgstab"),
        "rbicgstab_over_bicgstab_time": timed["rbicgstab"] / timed["bicgstab"],
        "phases": phases,
        "single_rhs": {"rbicgstab": summary("rbicgstab_single"), "bicgstab": summary("bicgstab_single")},
        "per_iteration": per_iter,
        "spmv_gbs": passes["spmv"]["gbs"],
        "passes": dict(passes, k=k_last, multi_nrhs=nr),
        "ritz_kernels": ritz_kernels,
        "roofline": {"bound": "mfma", "kernel": "k_gemmt_mfma_dl (interior 128 x 128 tiles)",
                     "achieved": gram_tflops, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": gram_tflops / FP64_MFMA_PEAK_TFLOPS,
                     "traffic": counter_traffic(f"k_gemmt_mfma_dl tiles={m_ritz // 128} n={n}"),
                     "flops_per_launch": (5 * f_sym + 3 * f_gen) / 8,
                     "us_per_launch": (5 * t_sym + 3 * t_gen) / 8 * 1e3,
                     "mix": "interior-tile launches of 5 X^T X + 3 X^T Y per Ritz step"},
        "parity_sample": parity,
    }
    if not args.no_fp32:
        r32, b32 = results["rbicgstab_fp32_ir"], results["bicgstab_fp32_ir"]
        errs = r32.err_vs_fp64 + b32.err_vs_fp64
        out["fp32_ir"] = {
            "rbicgstab_systems_per_s": nsys / timed["rbicgstab_fp32_ir"],
            "rbicgstab_ms_per_step": timed["rbicgstab_fp32_ir"] * 1e3,
            "bicgstab_systems_per_s": nsys / timed["bicgstab_fp32_ir"],
            "bicgstab_ms_per_step": timed["bicgstab_fp32_ir"] * 1e3,
            "note": "the RBiCG system of each matrix runs in FP64 in both RBiCGSTAB pipelines; its time is "
                    "part of the FP32-IR systems/s and it is left out of the error lists",
            "rbicgstab_inner_iters": r32.iters, "bicgstab_inner_iters": b32.iters,
            "rbicgstab_matvecs": r32.total_matvecs, "bicgstab_matvecs": b32.total_matvecs,
            "max_rel_res_true_fp64": max(max(r32.rel_res_true), max(b32.rel_res_true)),
            "rbicgstab_err_vs_fp64": r32.err_vs_fp64, "bicgstab_err_vs_fp64": b32.err_vs_fp64,
            "max_err_vs_fp64": max(errs), "err_bound": kappa * args.rtol,
            "within_bound": max(errs) <= kappa * args.rtol}
    if not args.no_hbm128:
        out["hbm_resident_128"] = hbm_resident_passes(args)
        out["hbm_stream_reference"] = stream_references()
    if args.calib_copy_mib > 0:
        # a plain device-to-device copy of known size (outside the timed region):
        # the reference the HBM counters of a profiled run are calibrated with
        nel = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calib_copy_bytes"] = 2 * nel * 8
        del src, dst
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(seq, args.rtol, args.cpu_systems)
    gs.close()
    print(json.dumps(out), flush=True)


def stream_references(n=1 << 27, reps=10):
    """HBM rates of plain streams with the passes' work distribution (the library's
    streaming reference kernels over two 1 GiB buffers, four times the last-level
    cache): a read, a copy, and the update pass's seven-read / three-write mix, at
    the passes' grid of 1024 workgroups and at 4096."""
    import torch
    from paper_1406_2831_amd.rbicgstab import rbicgstab_time_stream
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.zeros(n, dtype=torch.float64, device="cuda")
    res = {}
    for grid in (1024, 4096):
        for kind, name in ((0, "read"), (1, "copy"), (2, "mix_7r_3w")):
            ms, by = rbicgstab_time_stream(kind, a, b, grid, reps)
            gbs = by / (ms * 1e-3) / 1e9
            res[f"{name}_grid{grid}"] = {"us": ms * 1e3, "gbs": gbs, "frac": gbs / HBM_PEAK_GBS}
    del a, b
    return res


def hbm_resident_passes(args, N=128, k=20):
    """The fused passes and whole iterations where the working set is far past the
    last-level cache: 3D 7-point operator at N^3 (n = 2,097,152 at 128), sigma = 1,
    the k lowest eigenpairs of the sigma = 0 operator as recycle space.  Per-pass
    rooflines (live HIP events) and the end-to-end time per iteration of BiCGSTAB
    and RBiCGSTAB runs of a fixed 100 iterations (no convergence test)."""
    import numpy as np
    import torch
    import workloads as w
    from paper_1406_2831_amd.rbicgstab import Context
    from paper_1406_2831_amd.sequence import max_row_nnz

    K = w.convdiff((N, N, N), w.VEL3, w.PECLET)
    mdiag = w.generator(3, 0, "M").uniform(0.5, 1.5, size=K.n)
    A = w.shifted(K, mdiag, 1.0)
    At = A.transpose()
    n, nnz = A.n, A.nnz
    ctx = Context(n, max_row_nnz(A, At), k, 0, "cuda", float("inf"))
    ctx.setup(A, At)
    # the exact eigenvectors of K (sigma = 0): a well-conditioned oblique projector for A
    _, U, Ut = w.separable_eigenpairs((N, N, N), w.VEL3, w.PECLET, k)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a.T), dtype=torch.float64, device="cuda")
    ctx.recycle("set", dev(U), dev(Ut))
    del U, Ut
    kk = ctx.blocks()[1]
    gbs = lambda b, ms: b / (ms * 1e-3) / 1e9
    passes = {}
    for name, which in (("update", 0), ("spmv1_project", 1), ("spmv2_project", 2), ("spmv", 3),
                        ("update_fp32", 4), ("spmv1_project_fp32", 5), ("spmv2_project_fp32", 6),
                        ("mupdate_3rhs", 8 + 4 * 2), ("mspmv1_project_3rhs", 8 + 4 * 2 + 1),
                        ("mspmv2_project_3rhs", 8 + 4 * 2 + 2)):
        ms, by = ctx.time_pass(which, kk if which != 3 else 0, 20)
        passes[name] = {"us": ms * 1e3, "gbs": gbs(by, ms), "frac": gbs(by, ms) / HBM_PEAK_GBS, "bytes": by}
    b = torch.as_tensor(w.generator(3, 0, "b").standard_normal(n), device="cuda")
    sh = torch.as_tensor(w.generator(3, 0, "shadow").standard_normal(n), device="cuda")
    spmv_b = 12 * nnz + 4 * (n + 1) + 16 * n
    iters = {}
    for mode, byts in (("bicgstab", 2 * spmv_b + 128 * n), ("rbicgstab", 2 * spmv_b + 144 * n + 32 * n * kk)):
        x = torch.zeros_like(b)
        ctx.solve(b, x, shadow=sh, rtol=1e-30, max_it=20, mode=mode)   # warm-up
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = ctx.solve(b, x, shadow=sh, rtol=1e-30, max_it=100, mode=mode)
        torch.cuda.synchronize()
        us = (time.perf_counter() - t0) * 1e6 / max(st.iters, 1)
        iters[mode] = {"us_per_iter": us, "iters": st.iters, "bytes_per_iter": byts,
                       "frac": byts / (us * 1e-6) / 1e9 / HBM_PEAK_GBS}
    ctx.close()
    return {"grid": N, "n": n, "nnz": nnz, "k": kk, "passes": passes, "iteration": iters,
            "note": "recycle space: the k lowest closed-form eigenpairs of the sigma = 0 operator; "
                    "iterations timed end to end on the host around one solve call"}


if __name__ == "__main__":
    main()
