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
    U[-1,1]^3, sigma log-spaced in [1e-2, 1e1]), k = 16.  Round 1 (untimed) builds
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

    def run_batch(mode):
        for x in xs:
            x.zero_()
        sts = batch.solve(bs, xs, shs, rtol=args.rtol, max_it=20000, mode=mode)
        if any(s.status != 0 or s.rel_res_true > args.rtol for s in sts):
            print(f"batched {mode}: not every system converged", file=sys.stderr)
            sys.exit(1)
        return sts

    def run_single(mode):
        out = []
        for ctx, b, sh, x in zip(ctxs, bs, shs, xs):
            x.zero_()
            out.append(ctx.solve(b, x, shadow=sh, rtol=args.rtol, max_it=20000, mode=mode)[1])
        return out

    timed = {}
    for key, fn, mode in (("rbicgstab_batched", run_batch, "rbicgstab"),
                          ("bicgstab_batched", run_batch, "bicgstab"),
                          ("rbicgstab_single", run_single, "rbicgstab"),
                          ("bicgstab_single", run_single, "bicgstab")):
        for _ in range(args.warmup):
            fn(mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            sts = fn(mode)
        torch.cuda.synchronize()
        timed[key] = ((time.perf_counter() - t0) / args.steps, [s.iters for s in sts])
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
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the FP32-storage / FP64-refinement runs (reported beside the FP64 line)")
    ap.add_argument("--secant-max", type=float, default=0.0,
                    help="oblique-projector cap of the recycle setup (0: library default)")
    ap.add_argument("--workload", choices=("sequence", "adjoint", "batched", "large"), default="sequence",
                    help="sequence: the shifted 64^3 sequence (default); adjoint: gradients of "
                         "c^T x on the 128^3 problem through the transposed recycled solve; "
                         "batched: 32 shifted systems of uneven size solved together; large: the "
                         "27-point 160^3 sequence with FP32 storage under FP64 refinement")
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

    import torch
    import workloads as w
    from paper_1406_2831_amd.sequence import GpuSequence

    seq = w.seq_3d(N=args.grid, k=args.k)
    gs = GpuSequence(seq, s_max=512, secant_max=args.secant_max)
    nsys = seq.num_systems

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
    timed, results, passes = {}, {}, {}
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
            # error of each FP32-storage result against the FP64 pipeline's
            res.err_vs_fp64 = [float(torch.linalg.norm(x - xr) / torch.linalg.norm(xr))
                               for x, xr in zip(res.x, x64)]

    # live per-kernel timing of the fused passes (outside the timed steps) with the
    # space the first matrix's RBiCG solve generates: the multi-RHS passes for that
    # matrix's other right-hand sides, the single-system passes (FP64 and FP32
    # storage) and a plain product.  (The space at the end of the sequence depends
    # on rounding through five Ritz steps; the first one does not.)
    gs.run(mode="rbicgstab", rtol=args.rtol, systems=1)
    k_last = int(gs.ctx.blocks()[1])
    nr = seq.nrhs - 1
    for name, which, kk in (("mspmv1_project", 8 + 4 * (nr - 1) + 1, k_last),
                            ("mupdate", 8 + 4 * (nr - 1), k_last),
                            ("mspmv2_project", 8 + 4 * (nr - 1) + 2, k_last),
                            ("spmv1_project", 1, k_last), ("update", 0, k_last),
                            ("spmv2_project", 2, k_last), ("spmv", 3, 0),
                            ("spmv1_project_fp32", 5, k_last), ("update_fp32", 4, k_last),
                            ("spmv2_project_fp32", 6, k_last), ("spmv_fp32", 7, 0)):
        passes[name] = gs.ctx.time_pass(which, kk, args.time_reps)
    rres = results["rbicgstab"]
    gbs = lambda b, ms: b / (ms * 1e-3) / 1e9
    ms_dom, bytes_dom = passes["mspmv1_project"]
    ms_spmv, bytes_spmv = passes["spmv"]
    achieved = gbs(bytes_dom, ms_dom)
    kb = k_bucket(k_last)
    dom_kernel = f"k_mspmv1<{kb}>"
    traffic = counter_traffic(dom_kernel)

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
        "config": {"workload": f"3d 7-point convection-diffusion {args.grid}^3 (n={seq.n}), "
                               f"5 shifts x 4 rhs = {nsys} systems, k={args.k}, rtol={args.rtol}; "
                               f"per shift RBiCG on rhs 1, RBiCGSTAB on rhs 2-4 solved together",
                   "n": seq.n, "nnz": int(seq.K.nnz), "systems": nsys, "k": args.k},
        "rbicgstab": dict(summary("rbicgstab"), solver=rres.solver, k_used=rres.k_used),
        "bicgstab": summary("bicgstab"),
        "rbicgstab_over_bicgstab_time": timed["rbicgstab"] / timed["bicgstab"],
        "single_rhs": {"rbicgstab": summary("rbicgstab_single"), "bicgstab": summary("bicgstab_single")},
        "spmv_gbs": gbs(bytes_spmv, ms_spmv),
        "passes": dict({name: {"us": ms * 1e3, "gbs": gbs(by, ms)} for name, (ms, by) in passes.items()},
                       k=k_last, multi_nrhs=seq.nrhs - 1),
        "roofline": {"bound": "hbm", "kernel": dom_kernel,
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": bytes_dom, "us_per_launch": ms_dom * 1e3},
    }
    # a plain device-to-device copy of known size (outside the timed region):
    # the reference the HBM counters of a profiled run are calibrated with
    if not args.no_fp32:
        r32, b32 = results["rbicgstab_fp32_ir"], results["bicgstab_fp32_ir"]
        out["fp32_ir"] = {
            "rbicgstab_systems_per_s": nsys / timed["rbicgstab_fp32_ir"],
            "rbicgstab_ms_per_step": timed["rbicgstab_fp32_ir"] * 1e3,
            "bicgstab_systems_per_s": nsys / timed["bicgstab_fp32_ir"],
            "bicgstab_ms_per_step": timed["bicgstab_fp32_ir"] * 1e3,
            "rbicgstab_inner_iters": r32.iters, "bicgstab_inner_iters": b32.iters,
            "rbicgstab_matvecs": r32.total_matvecs, "bicgstab_matvecs": b32.total_matvecs,
            "max_rel_res_true_fp64": max(max(r32.rel_res_true), max(b32.rel_res_true)),
            "rbicgstab_err_vs_fp64": r32.err_vs_fp64, "bicgstab_err_vs_fp64": b32.err_vs_fp64}
    if args.calib_copy_mib > 0:
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


if __name__ == "__main__":
    main()
