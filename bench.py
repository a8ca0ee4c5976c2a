"""Benchmark: AlgMortar-PCG solves per second on one MI355X.

    python bench.py [--steps K] [--warmup W] [--config c2] [--prec fp64]

Workload (default): the 64^3 layered high-contrast TPFA system (contrast
1e6), 512 subdomains of 8^3 cells, one right-hand side, PCG to relative
residual 1e-8 with x0 = 0.  A step is one full PCG solve (every iteration:
SpMV, dots, axpys and the AlgMortar apply -- local band sweeps, interface
right-hand side, interface solve, reconstruction).  The set-up (partition,
local factors, basis functions, interface matrix and its inverse) runs once
before the timed region, as the factors are reused across solves; its time
is reported as setup_ms.  Inputs are device resident when timing starts.

Prints one JSON line with the metric, the roofline of the dominant kernel
(the local band sweeps + reconstruction) and the CPU oracle baseline.
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


def traffic_record(prec, config):
    """HBM bytes per launch of the local kernel from committed rocprofv3
    counter runs, valid only while the kernel source is unchanged."""
    path = os.path.join(ROOT, "profiles", f"k_local_{config}_{prec}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(ROOT, "paper_2607_22905_amd", "csrc", "local_kernels.h"), "rb").read()
    if rec.get("local_kernels_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return rec.get("hbm_bytes_per_launch")


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


def cpu_baseline(P, part, iters, its_to_converge, smooth=None):
    """The FP64 oracle on the host cores: set-up (untimed for the metric),
    then a bounded sample of PCG iterations, extrapolated to a whole solve.
    smooth: (blocks, steps) for the block-Jacobi-smoothed preconditioner."""
    import numpy as np
    from oracle import AlgMortarCPU, pcg
    from oracle.smoothing import SmoothedAlgMortarCPU
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count()
    t0 = time.perf_counter()
    pre = AlgMortarCPU(P.A, part)
    if smooth is not None:
        pre = SmoothedAlgMortarCPU(pre, smooth[0], smooth[1])
    t_setup = time.perf_counter() - t0
    As = P.A.to_scipy()
    t0 = time.perf_counter()
    b0 = P.b if P.b.ndim == 1 else P.b[:, 0]  # the oracle solves one right-hand side at a time
    res = pcg(lambda v: As @ v, b0, pre.apply, 1e-30, maxit=iters)
    t_it = (time.perf_counter() - t0) / max(res.iterations, 1)
    sps = 1.0 / (t_it * its_to_converge)
    return dict(value=sps, unit="solves/s", cores=int(threads), kind="oracle",
                sample=f"oracle set-up ({t_setup:.1f} s, not in the metric) then {res.iterations} "
                       f"PCG iterations ({t_it * 1e3:.1f} ms each) extrapolated to "
                       f"{its_to_converge} iterations per solve",
                setup_s=t_setup)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=12)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--theta", type=float, default=None,
                    help="contrast sweep K -> K^theta (c2, c6)")
    ap.add_argument("--smooth-steps", type=int, default=0,
                    help="block-Jacobi steps before and after the AlgMortar correction (Sec. 5.4)")
    ap.add_argument("--smooth-blocks", default="8,8,32",
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
    traffic = traffic_record(args.prec, args.config) if smooth is None else None
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
                     "kernel": ("k_localt (tile sweeps, fused interface solve, reconstruction)"
                                if smooth is None else
                                "k_localt on the smoothing blocks (block-Jacobi solves)"),
                     "avg_launch_us": k_ms * 1e3, "launches": k_launches,
                     "bytes_per_launch": k_bytes,
                     "timing": ("HIP events attached to the launches of a profiled solve (plain launches, hipExtLaunchKernelGGL)"
                                if smooth is None else "replayed alone (20 back-to-back launches)"),
                     "isolated_avg_launch_us": iso["local"] * 1e3},
        "other_kernels": others,
        "local_tile_autotune": {"choice": tile_choice, "candidate_us": tile_us},
    }
    h.close()
    if args.grad > 0:
        out["gradient"] = gradient_timing(P, part, m, args.grad)
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(P, part, args.cpu_iters, its, smooth)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
