"""Benchmark: AlgMortar-PCG solves per second on one MI355X.

    python bench.py [--steps K] [--warmup W] [--config c4] [--prec fp64]

Workload (default): the 128^3 TPFA system with K = exp(GRF, sigma 1, ell 8),
4096 subdomains of 8^3 cells, one right-hand side, PCG to relative residual
1e-8 with x0 = 0 (FP64 everywhere).  A step is one full PCG solve (every
iteration: SpMV, dots, axpys and the AlgMortar apply -- local tile sweeps,
interface right-hand side, interface solve, reconstruction).  The set-up
(partition, local factors, basis functions, interface matrix and its
inverse) runs once before the timed region, as the factors are reused
across solves; its time is reported as setup_ms.  Inputs are device
resident when timing starts.

With FP64 local factors (the default) the same workload is also solved with
FP32 and BF16 local factors (the precision form: interface solve, dots and
residuals stay FP64), reported under "precision_forms" with their solve
rates, iteration counts and speedups over FP64.

Prints one JSON line with the metric, the roofline of the dominant kernel
(the local tile sweeps + reconstruction) and the CPU oracle baseline.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "c2": "64^3 layered log10 K in [-3,3] + GRF, contrast 1e6, TPFA 7-point, "
          "512 subdomains of 8^3, 1 RHS, PCG tol 1e-8",
    "c4": "128^3 K = exp(GRF sigma 1, ell 8), TPFA 7-point, 4096 subdomains of 8^3, "
          "1 RHS, PCG tol 1e-8",
    "c1": "64x64 K = exp(GRF), TPFA 5-point, 16 subdomains of 16^2, 1 RHS, PCG tol 1e-10",
    "c5": "96^3 ln K GRF sigma 2, TPFA 7-point, 1728 subdomains of 8^3, 1 RHS, PCG tol 1e-10",
    "c6": "64^3 periodic cross pattern, kappa 1e6 on 2-cell channels through every 8^3 tile, "
          "p fixed on the y faces, TPFA 7-point, 512 subdomains of 8^3, 1 RHS, PCG tol 1e-8",
    "c3": "128x128x64 distorted hexahedra, ln K GRF sigma 2, recursive bisection into "
          "200-800-cell subdomains, 16 RHS (well pairs) solved together, PCG tol 1e-8",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def traffic_record(prec, config, tile_choice):
    """HBM bytes per launch of the local kernel from committed rocprofv3
    counter runs, valid only while the kernel source is unchanged and for the
    wave layout the counters were taken with (the runs pin it with
    ALGMORTAR_TILE; the record keeps one entry per layout measured, under
    "per_tile_choice")."""
    path = os.path.join(ROOT, "profiles", f"k_local_{config}_{prec}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_2607_22905_amd", "csrc", "local_kernels.h"), "rb").read()
    if rec.get("local_kernels_sha256") != hashlib.sha256(src).hexdigest():
        return None
    ent = rec.get("per_tile_choice", {}).get(str(tile_choice))
    return None if ent is None else ent.get("hbm_bytes_per_launch")


def gradient_timing(P, part, m, steps):
    """Gradient evaluations of J = sum over observed cells of (p - p_obs)^2
    with respect to ln K through the differentiation form: device TPFA
    assembly, AlgMortar set-up, forward PCG, adjoint PCG on the same handle
    and the face gradient, each evaluation timed whole (one warm-up first).
    Observed cells and p_obs are those of the workload when it has them,
    else 1000 seeded cells and p_obs = 0."""
    import numpy as np
    import torch

    import paper_2607_22905_amd as am
    dev = torch.device("cuda:0")
    obs = P.extra.get("obs")
    if obs is None:
        obs = np.random.default_rng(7).choice(P.n, size=min(1000, P.n), replace=False)
    obs_t = torch.as_tensor(np.asarray(obs, dtype=np.int64), device=dev)
    pobs = torch.zeros(len(obs), dtype=torch.float64, device=dev)
    atol = P.extra.get("adjoint_tol", 1e-12)
    logK0 = torch.as_tensor(np.ascontiguousarray(P.logK), dtype=torch.float64, device=dev)
    out = {}
    for reuse in (True, False):
        model = am.DarcyModel(P.faces, P.n, part, m, tol=P.tol, adjoint_tol=atol,
                              reuse_handle=reuse)
        times = []
        for i in range(steps + 1):
            # a new permeability each time (the handle's values must change)
            logK = (logK0 * (1.0 + 0.01 * i)).requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p = am.AlgMortarSolve.apply(logK, model)
            J = ((p[obs_t] - pobs) ** 2).sum()
            J.backward()
            torch.cuda.synchronize()
            if i > 0:
                times.append((time.perf_counter() - t0) * 1e3)
        fi, ai = model.last_info, getattr(model, "last_adjoint_info", {})
        model.close()
        out["ms_per_gradient" if reuse else "ms_per_gradient_new_handle"] = float(np.median(times))
    out.update({"evaluations": steps,
                "forward_iterations": fi["iterations"] if fi else None,
                "adjoint_iterations": ai.get("iterations") if ai else None,
                "forward_tol": P.tol, "adjoint_tol": atol, "observed_cells": int(len(obs)),
                "includes": "assembly, set-up (numeric part on one reused handle; the whole "
                            "set-up with a new handle per evaluation), forward solve, adjoint "
                            "solve, face gradient"})
    return out


# The oracle cannot finish the large workloads within the benchmark's time
# limit (at 128^3: about two minutes of set-up and 4 s per PCG iteration on
# eight cores), so it runs on a bounded sample: the same workload recipe at a
# reduced grid (same field model, boundary conditions, sources and subdomain
# shape), solved completely, and its time per PCG iteration is scaled to the
# benchmarked grid by the ratio of cells.
CPU_SAMPLE = {
    "c4": dict(nx=64, ny=64, nz=64),
    "c5": dict(nx=48, ny=48, nz=48),
    "c3": dict(nx=64, ny=64, nz=32),
}


def _oracle_leg(S, part, threads, smooth):
    """One timed oracle run (set-up, then PCG on the first right-hand side)
    with the BLAS pool limited to `threads`."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import AlgMortarCPU, pcg
    from oracle.smoothing import SmoothedAlgMortarCPU
    with threadpool_limits(limits=threads):
        blas = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        t0 = time.perf_counter()
        pre = AlgMortarCPU(S.A, part)
        if smooth is not None:
            pre = SmoothedAlgMortarCPU(pre, smooth[0], smooth[1])
        t_setup = time.perf_counter() - t0
        As = S.A.to_scipy()
        b0 = S.b if S.b.ndim == 1 else S.b[:, 0]
        t0 = time.perf_counter()
        res = pcg(lambda v: As @ v, b0, pre.apply, S.tol)
        t_solve = time.perf_counter() - t0
    return dict(threads=int(blas), setup_s=t_setup, solve_s=t_solve, iterations=res.iterations,
                ms_per_iteration=t_solve / max(res.iterations, 1) * 1e3,
                true_rel_res=res.true_rel_res)


def cpu_baseline(config, P, its_to_converge, smooth=None, theta=None):
    """The FP64 oracle on the host cores, in two legs (one thread, all
    cores): set-up, a complete PCG solve and its iterations on the bounded
    sample of CPU_SAMPLE (the workload itself where it is small), and the
    solve rate scaled to the benchmarked workload (time per iteration times
    the cell ratio, times the GPU's iteration count)."""
    import numpy as np
    from oracle import partition_blocks, partition_bisect
    from workloads import make_config
    kw = dict(CPU_SAMPLE.get(config, {}))
    if theta is not None:
        kw["theta"] = theta
    if smooth is not None or not kw or config in ("c1",):
        S, kw_used = P, {}
    else:
        S, kw_used = make_config(config, **kw), kw
    if S.partition[0] == "blocks":
        part, _ = partition_blocks(S.dims, S.partition[1])
    else:
        _, lo, hi, seed = S.partition
        part, _ = partition_bisect(S.A.row_ptr, S.A.col, S.A.val, S.n, lo, hi, seed)
    ncpu = os.cpu_count()
    # the GPU machine allots 16 host threads per GPU (OMP_NUM_THREADS)
    allc = int(os.environ.get("OMP_NUM_THREADS", ncpu) or ncpu)
    allc = max(1, min(allc, ncpu))
    sm = None
    if smooth is not None:
        sm = smooth
    legs = [_oracle_leg(S, part, t, sm) for t in (1, allc)]
    scale = P.n / S.n
    for leg in legs:
        leg["solves_per_s_scaled"] = 1.0 / (leg["ms_per_iteration"] * 1e-3 * scale * its_to_converge)
    best = legs[-1]
    sample = (f"the oracle on the {config} recipe at {S.dims[0]}x{S.dims[1]}x{S.dims[2]} "
              f"({S.n} cells, 1/{scale:.0f} of the workload), set-up and one complete PCG "
              f"solve ({best['iterations']} iterations) per leg; solves/s scaled by the cell "
              f"ratio and the GPU's {its_to_converge} iterations"
              if kw_used else
              f"the oracle on the workload itself, set-up and one complete PCG solve per leg")
    return dict(value=best["solves_per_s_scaled"], unit="solves/s", cores=best["threads"],
                kind="oracle", sample=sample, os_cpu_count=ncpu, blas_threads_all_cores=best["threads"],
                legs=legs)


def precision_forms(P, part, m, b, x64, args, v64, its64):
    """The precision form on the same workload: FP32 and BF16 local factors
    (BF16: bf16 storage, fp32 arithmetic), FP64 interface solve, dots and
    residuals; with 16 right-hand sides also BF16 x BF16 products on the
    matrix cores (block vectors rounded to BF16, FP32 accumulation); each
    timed like the FP64 run.  Reports solves/s, the speedup over FP64,
    iterations (and their change) and the relative L2 distance of the
    solution from the FP64 one (both at the workload's tolerance)."""
    import numpy as np
    import torch

    import paper_2607_22905_amd as am
    res = {}
    nrhs = P.nrhs
    forms = [("fp32", "fp32", {}), ("bf16", "bf16", {})]
    if nrhs in (1, 16):
        # BF16 x BF16 products on the matrix cores (with one right-hand side:
        # column 0 of each tile); the flag needs the interface solve as its
        # own launches
        forms.append(("bf16_products", "bf16", {"bf16_products": True, "separate_iface": True}))
    for name, prec, kw in forms:
        h = am.AlgMortar(P.A, part, m, prec=prec, graph=not args.no_graph, max_nrhs=nrhs, **kw)
        x = torch.empty_like(b)
        for _ in range(args.warmup):
            h.pcg(b, P.tol, out=x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, info, _ = h.pcg(b, P.tol, out=x)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        its = max(i["iterations"] for i in info)
        v = args.steps * nrhs / el
        err = float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))
        res[name] = {"value": v, "unit": "solves/s", "speedup_vs_fp64": v / v64,
                     "ms_per_step": el / args.steps * 1e3, "iterations": its,
                     "iteration_change_vs_fp64": its - its64,
                     "true_rel_res": max(i["true_rel_res"] for i in info),
                     "rel_l2_vs_fp64_solution": err,
                     "local_tile_autotune": h.tile_choice(nrhs)[0]}
        log(f"bench: {name} local factors: {v:.1f} solves/s ({v / v64:.2f}x FP64), {its} iterations")
        h.close()
    return res


def interface_forms(P, part, m, b, x64, args, v64, its64, separate):
    """The interface solve in its other forms on the same workload, FP64,
    each timed like the main run: the inexact solve (block-Jacobi PCG on S to
    rtol 1e-2, at most 50 inner iterations, flexible outer PCG; Sec. 6, Sec. 7)
    and, where the solve is its own launches, the dense explicit S^-1 product
    in place of the nested-dissection blocks.  Solve rates, speedups over the
    main run, iterations and the solution's relative L2 distance from it."""
    import torch

    import paper_2607_22905_amd as am
    forms = {"inexact_rtol_1e-2": dict(inexact_iface=True)}
    if separate:
        forms["dense_explicit_inverse"] = dict(dense_iface=True)
    res = {}
    nrhs = P.nrhs
    for name, kw in forms.items():
        h = am.AlgMortar(P.A, part, m, graph=not args.no_graph, max_nrhs=nrhs, **kw)
        x = torch.empty_like(b)
        for _ in range(args.warmup):
            h.pcg(b, P.tol, out=x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, info, _ = h.pcg(b, P.tol, out=x)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        its = max(i["iterations"] for i in info)
        v = args.steps * nrhs / el
        res[name] = {"value": v, "unit": "solves/s", "speedup_vs_main": v / v64,
                     "ms_per_step": el / args.steps * 1e3, "iterations": its,
                     "iteration_change_vs_main": its - its64,
                     "true_rel_res": max(i["true_rel_res"] for i in info),
                     "rel_l2_vs_main_solution": float(torch.linalg.norm(x - x64) /
                                                      torch.linalg.norm(x64))}
        if separate or name.startswith("inexact"):
            ms_, by_ = h.time_kernel("gemv", nrhs=nrhs, reps=5)
            res[name]["interface_solve_replayed_us"] = ms_ * 1e3
        log(f"bench: interface form {name}: {v:.1f} solves/s ({v / v64:.2f}x), {its} iterations")
        h.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c4")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-forms", action="store_true",
                    help="skip the FP32 / BF16 local-factor solves and the other interface-solve "
                         "forms of the FP64 run")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--theta", type=float, default=None,
                    help="contrast sweep K -> K^theta (c2, c6)")
    ap.add_argument("--smooth-steps", type=int, default=0,
                    help="block-Jacobi steps before and after the AlgMortar correction (Sec. 5.4)")
    ap.add_argument("--smooth-blocks", default="8,8,16",
                    help="block sizes bx,by,bz of the smoothing partition (Cartesian workloads)")
    ap.add_argument("--grad", type=int, default=0, metavar="K",
                    help="also time K gradient evaluations of a least-squares loss on observed "
                         "cells through the differentiation form (device assembly, set-up, "
                         "forward solve, adjoint solve, face gradient); reported as 'gradient'")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); "
              "the solver has no multi-GPU sharding.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2607_22905_amd as am
    from workloads import make_config

    if args.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    log(f"bench: building workload {args.config}")
    P = make_config(args.config) if args.theta is None else make_config(args.config, theta=args.theta)
    if P.partition[0] == "blocks":
        part, m = am.partition_blocks(P.dims, P.partition[1])
    else:
        _, lo, hi, seed = P.partition
        part, m = am.partition_bisect(P.A, lo, hi, seed)
    dev = torch.device("cuda:0")
    torch.cuda.synchronize()
    log("bench: set-up")
    t0 = time.perf_counter()
    nrhs = P.nrhs
    h = am.AlgMortar(P.A, part, m, prec=args.prec, graph=not args.no_graph, max_nrhs=nrhs)
    smooth = None
    if args.smooth_steps > 0:
        if P.partition[0] != "blocks":
            sys.exit("bench.py: --smooth-steps needs a Cartesian (block-partitioned) workload")
        sb = tuple(int(v) for v in args.smooth_blocks.split(","))
        blocks, nb = am.partition_blocks(P.dims, sb)
        h.set_smoother(blocks, nb, args.smooth_steps)
        smooth = (blocks, args.smooth_steps)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    # right-hand sides as rows of a (k, n) block (column c of the C-ABI's n x k block)
    bh = P.b if P.b.ndim == 1 else np.ascontiguousarray(P.b.T)
    b = torch.as_tensor(bh, dtype=torch.float64, device=dev)
    x = torch.empty_like(b)
    for _ in range(args.warmup):
        h.pcg(b, P.tol, out=x)
    torch.cuda.synchronize()
    log(f"bench: timing {args.steps} solves")
    t0 = time.perf_counter()
    infos = []
    marks = []  # each solve returns after its info is on the host
    for _ in range(args.steps):
        _, info, _ = h.pcg(b, P.tol, out=x)
        infos.append(info)
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    per_step = np.diff(np.array([t0] + marks)) * 1e3
    its = max(i["iterations"] for i in infos[-1])
    # Kernel durations inside a solve: one more solve of the same system with
    # plain launches instead of the graph (same kernels, order, data and cache
    # state), the first and last launch of each operation carrying HIP events
    # on the library's stream (the dispatches' own start and end).
    if smooth is None:
        _, pinfo, prof = h.pcg_profile(b, P.tol, out=x)
        k_ms_total, k_launches = prof["local"]
        k_ms = k_ms_total / max(k_launches, 1)
        _, k_bytes = h.time_kernel("local", nrhs=nrhs, reps=1)
    else:
        # the smoothed solve has no event-timed form: the dominant kernel (the
        # block solves, 2 nu launches per iteration) is timed replayed alone
        prof = {"local": (0.0, 0), "gemv": (0.0, 0), "spmv": (0.0, 0), "update": (0.0, 0)}
        k_ms, k_bytes = h.time_kernel("smooth_block", nrhs=nrhs, reps=20)
        k_launches = 2 * args.smooth_steps * its
    # the same kernels replayed alone (back to back, same input): context only
    iso = {}
    for name in ("local", "gemv", "spmv", "update", "bpart"):
        if name == "gemv" and prof["gemv"][1] == 0:
            continue  # interface solve fused into the local kernel on this handle
        ms_, by_ = h.time_kernel(name, nrhs=nrhs, reps=50 if nrhs == 1 else 10)
        iso[name] = ms_
    others = {}
    for name in ("spmv", "update", "gemv"):
        tot, cnt = prof[name]
        if cnt == 0:
            continue
        ms_ = tot / cnt
        _, by_ = h.time_kernel(name, nrhs=nrhs, reps=1)
        others[name] = {"avg_launch_us": ms_ * 1e3, "launches": cnt, "bytes_per_launch": by_,
                        "achieved_GBs": by_ / (ms_ * 1e-3) / 1e9,
                        "isolated_avg_launch_us": iso[name] * 1e3}
    achieved = k_bytes / (k_ms * 1e-3) / 1e9
    log(f"bench: in-solve launch averages: local {k_ms * 1e3:.1f} us ("
        + ", ".join(f"{k} {v['avg_launch_us']:.1f} us" for k, v in others.items())
        + f"); replayed alone: " + ", ".join(f"{k} {v * 1e3:.1f} us" for k, v in iso.items()))
    tile_choice, tile_us = h.tile_choice(nrhs)
    traffic = traffic_record(args.prec, args.config, tile_choice) if smooth is None else None
    x64 = x.clone()
    out = {
        "metric": "PCG solves/s to 1e-8 rel. residual; precond-apply HBM GB/s vs peak",
        "value": args.steps * nrhs / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "median_ms_per_step": float(np.median(per_step)),
        "nrhs_per_step": nrhs,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else f"f64+{args.prec}-local",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS.get(args.config, args.config)}",
                   "n": P.n, "subdomains": m, "interfaces": h.n_iface, "tol": P.tol,
                   "local_prec": args.prec, "parallelism": "single GPU",
                   **({"theta": args.theta} if args.theta is not None else {}),
                   **({"smooth_steps": args.smooth_steps, "smooth_blocks": args.smooth_blocks}
                      if smooth is not None else {})},
        "iterations": its,
        "true_rel_res": max(i["true_rel_res"] for i in infos[-1]),
        "setup_ms": setup_ms,
        "end_to_end_solves_per_s": nrhs / (setup_ms * 1e-3 + elapsed / args.steps),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": (("k_localt_mf + k_localt_mf2 (16 RHS on the matrix cores: tile sweeps, "
                                 "reconstruction; one launch per window bucket)" if nrhs == 16 else
                                 "k_localt (tile sweeps, fused interface solve, reconstruction)")
                                if smooth is None else
                                "k_localt on the smoothing blocks (block-Jacobi solves)"),
                     "avg_launch_us": k_ms * 1e3, "launches": k_launches,
                     "bytes_per_launch": k_bytes,
                     "timing": ("HIP events attached to the launches of a profiled solve (plain launches, "
                                "hipExtLaunchKernelGGL); with two window buckets, events on the library's stream "
                                "before the fork and after the join of the pair running side by side"
                                if smooth is None else "replayed alone (20 back-to-back launches)"),
                     "isolated_avg_launch_us": iso["local"] * 1e3},
        "other_kernels": others,
        "local_tile_autotune": {"choice": tile_choice, "candidate_us": tile_us},
    }
    h.close()
    if args.prec == "fp64" and smooth is None and not args.no_precision_forms:
        out["precision_forms"] = precision_forms(P, part, m, b, x64, args, out["value"], its)
        out["interface_forms"] = interface_forms(P, part, m, b, x64, args, out["value"], its,
                                                 separate=prof["gemv"][1] > 0)
    if args.grad > 0:
        out["gradient"] = gradient_timing(P, part, m, args.grad)
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(args.config, P, its, smooth, args.theta)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
