"""Benchmark: PCG solve to 1e-6 relative residual with the multiscale spectral
multigrid preconditioner on one MI355X.

A step is one pass of the whole hot path on the workload: set-up (local
spectral problems on every level, Galerkin operators, smoother and coarsest
factorizations) followed by the preconditioned CG solve.  `value` is the
solve throughput, degrees of freedom per second of solve time, with the
inputs already resident in HBM.  The default workload is the 512^3
random-inclusions field (contrast 1e6, 4 levels) in float64.

Prints one JSON line (rank 0, single GPU).  Progress goes to stderr.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from synth.fields import WORKLOADS, make_field, make_source  # noqa: E402

HBM_PEAK_GBS = 8000.0
COPY_BYTES = 256 << 20
# profiling classes that are one kernel each (the coarse part is a group)
SINGLE_KERNEL = {"cg_spmv": "k_spmv_pcg", "pre_smooth": "k_pre_smooth", "resid_restrict": "k_resid_restrict",
                 "prolong": "k_prolong", "post_smooth": "k_post_fused", "p_update": "k_p_update",
                 "coarsest": "k_coarsest_sym / k_coarsest"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="inclusions512", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=[None, "fp64", "fp32_vcycle", "fp32_basis", "fp32_store"])
    ap.add_argument("--solver", default="pcg", choices=["pcg", "gmres"],
                    help="outer Krylov solver (GMRES: restarted, flexible, right-preconditioned)")
    ap.add_argument("--restart", type=int, default=30, help="GMRES restart length")
    ap.add_argument("--levels", type=int, default=None, help="override the workload's number of levels")
    ap.add_argument("--contrast", type=float, default=None,
                    help="channel / inclusion permeability over the background 1 (channels and inclusions fields)")
    ap.add_argument("--eigs", type=int, default=None, help="override L_c, eigenvectors per level-2 element")
    ap.add_argument("--eigs-coarse", type=int, default=None, help="override L_cc at levels >= 3")
    ap.add_argument("--nu", type=int, default=1, help="block-Jacobi sweeps on the fine level")
    ap.add_argument("--nu-c", type=int, default=0, help="sweeps on the coarse levels (0: same as --nu)")
    ap.add_argument("--eig-threshold-coarse", type=float, default=0.0,
                    help="B_cc > 0: keep the coarse-coarse eigenvalues below it (strategy 2), at most L_cc")
    ap.add_argument("--eig-threshold", type=float, default=0.0,
                    help="B_c > 0: keep the level-2 eigenvalues below it (strategy 2), at most L_c")
    ap.add_argument("--forms", default="fp32_vcycle,fp32_store,learned,learned+fp32_vcycle",
                    help="comma-separated extra forms timed once each after the bench steps and reported "
                         "under 'forms': fp32_vcycle, fp32_basis, fp32_store, learned (CNN warm start), "
                         "learned+<precision>; empty for none")
    ap.add_argument("--ws-tol", type=float, default=1e-4,
                    help="relative residual the learned warm start's local eigensolves accept")
    ap.add_argument("--allow-unconverged", action="store_true",
                    help="report a value even when local eigensolves hit their cycle cap")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=64, help="edge of the field crop timed on the CPU oracle")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run three plain device copies of COPY_BYTES each (counter calibration)")
    return ap.parse_args()


def cpu_baseline(perm, wl, edge, levels):
    """The FP64 oracle on a bounded sample: an edge^3 corner crop of the same
    field with the workload's levels, eigenvector counts, aggregation and
    source kind (a smaller problem than the GPU's), full set-up and PCG."""
    from threadpoolctl import threadpool_limits
    from oracle import Grid, build_hierarchy, Preconditioner, pcg
    crop = np.ascontiguousarray(perm[:edge, :edge, :edge])
    g = Grid.unit_cube(edge)
    cores = min(os.cpu_count() or 1, 16)
    agg = wl.agg
    lv = levels
    while lv > 2 and edge % (8 * agg ** (lv - 2)):
        lv -= 1
    t0 = time.perf_counter()
    hier = build_hierarchy(crop, g, lv, wl.eigs, sub=8, agg=agg, workers=cores,
                           target_cc=wl.eigs_coarse or None)
    pre = Preconditioner(hier)
    t1 = time.perf_counter()
    b = make_source(wl.source, crop.shape).reshape(-1)
    with threadpool_limits(limits=cores):
        ts = time.perf_counter()
        res = pcg(hier.A, b, pre.apply, tol=1e-6)
        t2 = time.perf_counter()
    return {
        "value": g.n / (t2 - ts),
        "unit": "DoF/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{edge}^3 corner crop of the {wl.name} field ({g.n} DoF, {lv} levels, {wl.eigs} / "
                   f"{wl.eigs_coarse or wl.eigs} eigenvectors, agg {agg}, {wl.source} source): a smaller "
                   f"problem than the GPU's; PCG {t2 - ts:.2f} s for {res.iters} iterations with numpy/scipy "
                   f"allowed {cores} threads; set-up {t1 - t0:.2f} s on {cores} worker processes (not timed)"),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not code).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2403_19342_amd.specmg import SpecMG, FP64, FP32_VCYCLE, FP32_BASIS, FP32_STORE, EEIG

    wl = WORKLOADS[args.config]
    if args.contrast is not None and wl.kind not in ("channels", "inclusions"):
        raise SystemExit("--contrast applies to the channels and inclusions fields")
    if args.eigs is not None or args.eigs_coarse is not None:
        wl = dataclasses.replace(wl, eigs=args.eigs or wl.eigs,
                                 eigs_coarse=wl.eigs_coarse if args.eigs_coarse is None else args.eigs_coarse)
    levels = args.levels or wl.levels
    prec = args.precision or wl.precision
    n = wl.n
    log(f"bench: generating the {wl.name} field ({n}^3)")
    perm_h = make_field(wl.kind, n, wl.seed, **({} if args.contrast is None else {"value": args.contrast}))
    b_h = make_source(wl.source, perm_h.shape)
    dev = torch.device("cuda:0")
    perm = torch.as_tensor(perm_h, device=dev)
    b = torch.as_tensor(b_h.reshape(-1), device=dev)
    x = torch.zeros(n ** 3, dtype=torch.float64, device=dev)
    agg = wl.agg
    PREC = {"fp64": FP64, "fp32_vcycle": FP32_VCYCLE, "fp32_basis": FP32_BASIS, "fp32_store": FP32_STORE}
    precision = PREC[prec]

    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def make_ctx(precision_, cnn=None):
        ctx = SpecMG(perm, levels=levels, eigs_per_subdomain=wl.eigs, agg=agg, precision=precision_,
                     eigs_coarse=wl.eigs_coarse, eig_threshold_coarse=args.eig_threshold_coarse,
                     eig_threshold=args.eig_threshold, nu=args.nu, nu_c=args.nu_c, allow_unconverged=True,
                     cnn_weights=cnn, ws_resid_tol=args.ws_tol)
        unconv = ctx.info()["setup"]["eig_unconverged"]
        if unconv and not args.allow_unconverged:
            ctx.close()
            raise SystemExit(f"bench: {unconv} local eigensolves hit their cycle cap (specmg error {EEIG}); "
                             "no value reported")
        return ctx

    def step(profile, precision_=precision, xout=x, cnn=None):
        ctx = make_ctx(precision_, cnn)
        if args.solver == "gmres":
            # the per-kernel timing covers the CG solve only
            rc, info = ctx.gmres_solve(b, xout, restart=args.restart, tol=1e-6, max_iter=1000)
            ctx.close()
            return info, None
        if profile:
            ctx.set_profiling(True)
        rc, info = ctx.pcg_solve(b, xout, tol=1e-6, max_iter=1000)
        prof = ctx.profile() if profile else None
        ctx.close()
        return info, prof

    for i in range(args.warmup):
        info, _ = step(False)
        log(f"bench: warm-up {i}: {info.iters} iterations, solve {info.solve_ms:.1f} ms, "
            f"set-up {info.setup_ms:.0f} ms")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # Only the last timed step records HIP events around every kernel (the
    # per-kernel durations of the roofline); with two or more steps the solve
    # time comes from the steps without them, whose solve the events do not
    # slow down.
    infos, profs = [], []
    for i in range(args.steps):
        info, prof = step(i == args.steps - 1)
        infos.append(info)
        if prof is not None:
            profs.append(prof)
        log(f"bench: step {i}: {info.iters} iterations, solve {info.solve_ms:.1f} ms, "
            f"set-up {info.setup_ms:.0f} ms")
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    plain = infos[:-1] if (len(infos) > 1 and profs) else infos
    solve_s = float(np.mean([i.solve_ms for i in plain])) / 1e3
    setup_s = float(np.mean([i.setup_ms for i in infos])) / 1e3
    iters = [i.iters for i in infos]
    dof = n ** 3
    tot = {}
    for p in profs:
        for k, (ms, cnt, by) in p.items():
            a = tot.setdefault(k, [0.0, 0, by])
            a[0] += ms
            a[1] += cnt
    # the coarse part minus the coarsest product: the coarse levels' own kernels
    if "coarse_part" in tot and tot["coarse_part"][1]:
        cp, cs = tot["coarse_part"], tot.get("coarsest", [0.0, 0, 0.0])
        tot["coarse_levels"] = [cp[0] - cs[0], cp[1], cp[2] - cs[2]]
    kernels = {k: {"avg_us": 1e3 * v[0] / max(v[1], 1), "launches": v[1], "bytes_per_launch": v[2],
                   "GBps": (v[2] / (v[0] / max(v[1], 1) * 1e-3) / 1e9) if v[2] and v[0] > 0 else None}
               for k, v in tot.items() if v[1]}
    roofline, iteration = None, None
    cands = [k for k in kernels if k in SINGLE_KERNEL or k == "coarse_levels"]
    if cands:
        # the kernel (or the coarse levels' kernel group) with the largest share of solve time
        dom = max(cands, key=lambda k: tot[k][0])
        ms, cnt, by = tot[dom]
        avg_ms = ms / max(cnt, 1)
        achieved = by / (avg_ms * 1e-3) / 1e9
        from paper_2403_19342_amd.profile_summary import read_traffic
        measured = read_traffic(os.path.join(ROOT, "profiles", f"hbm_traffic_{wl.name}.md"))
        roofline = {"bound": "hbm", "kernel": SINGLE_KERNEL.get(dom, "coarse levels (kernel group)"),
                    "class": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": measured.get(dom),
                    "bytes_per_launch": by, "avg_launch_us": avg_ms * 1e3}
        # whole CG iteration: every class's algorithmic bytes over the event-timed
        # kernel time, and over the wall time of the plain solves
        whole = [k for k in tot if k not in ("coarsest", "coarse_levels")]
        it_bytes = sum(tot[k][2] * tot[k][1] for k in whole) / max(infos[-1].iters, 1)
        it_kernel_ms = sum(tot[k][0] for k in whole) / max(infos[-1].iters, 1)
        it_wall_ms = solve_s * 1e3 / max(np.mean([i.iters for i in plain]), 1)
        iteration = {"bytes": it_bytes, "kernel_ms": it_kernel_ms, "wall_ms": it_wall_ms,
                     "GBps_kernel": it_bytes / (it_kernel_ms * 1e-3) / 1e9,
                     "GBps_wall": it_bytes / (it_wall_ms * 1e-3) / 1e9,
                     "frac_wall": it_bytes / (it_wall_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    dtype = {FP64: "f64", FP32_BASIS: "f64, f32 level-2 basis",
             FP32_STORE: "f64 arithmetic, f32 storage of V-cycle coefficients"}.get(
        precision, "f32 V-cycle / f64 " + ("CG" if args.solver == "pcg" else "GMRES"))
    out = {
        "metric": ("PCG" if args.solver == "pcg" else "GMRES") +
                  " solve to 1e-6 relative residual, DoF per second of solve time",
        "value": dof / solve_s,
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": (t1 - t0) * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": f"{n}^3", "dof": dof, "levels": levels, "solver": args.solver,
                   "eigs_per_subdomain": wl.eigs, "eigs_coarse": wl.eigs_coarse or wl.eigs, "agg": agg,
                   "field": wl.kind, "source": wl.source,
                   **({} if args.contrast is None else {"contrast": args.contrast}),
                   **({"eig_threshold_coarse": args.eig_threshold_coarse} if args.eig_threshold_coarse > 0 else {}),
                   **({"eig_threshold": args.eig_threshold} if args.eig_threshold > 0 else {}),
                   **({"nu": args.nu, "nu_c": args.nu_c or args.nu} if (args.nu, args.nu_c) != (1, 0) else {}),
                   "tol": 1e-6, "precision": prec},
        "solve_ms": solve_s * 1e3,
        "solve_ms_profiled_step": infos[-1].solve_ms,
        "setup_ms": setup_s * 1e3,
        "iters": iters,
        "rel_resid_true": [i.rel_resid_true for i in infos],
        "eig_unconverged": [i.eig_unconverged for i in infos],
        "dims": list(infos[-1].dims)[: levels],
        "kernels": kernels,
        "iteration": iteration,
        "roofline": roofline,
    }
    forms = [f for f in args.forms.split(",") if f]
    if forms:
        ref = x.clone()
        nref = float(torch.linalg.norm(ref))
        out["forms"] = {}
        for f in forms:
            xf = torch.zeros_like(x)
            cnn = None
            pf = precision
            if f.startswith("learned") and not os.path.exists(
                    os.path.join(ROOT, "paper_2403_19342_amd", "weights", f"cnn_k{wl.eigs}_bf16.npy")):
                log(f"bench: form {f} skipped (no trained network for {wl.eigs} eigenvectors)")
                continue
            if f == "learned":
                wpath = os.path.join(ROOT, "paper_2403_19342_amd", "weights", f"cnn_k{wl.eigs}_bf16.npy")
                cnn = torch.as_tensor(np.load(wpath).astype(np.int16), device=dev)
            elif f.startswith("learned+"):
                wpath = os.path.join(ROOT, "paper_2403_19342_amd", "weights", f"cnn_k{wl.eigs}_bf16.npy")
                cnn = torch.as_tensor(np.load(wpath).astype(np.int16), device=dev)
                pf = PREC[f.split("+", 1)[1]]
            else:
                pf = PREC[f]
            info, _ = step(False, pf, xf, cnn)
            err = float(torch.linalg.norm(xf - ref)) / nref
            out["forms"][f] = {"iters": info.iters, "solve_ms": info.solve_ms, "setup_ms": info.setup_ms,
                               "setup_plus_solve_ms": info.setup_ms + info.solve_ms,
                               "rel_resid_true": info.rel_resid_true, "rel_err_vs_bench_form": err,
                               "ws_fallbacks": info.ws_fallbacks, "replacements": info.replacements,
                               "value": dof / (info.solve_ms * 1e-3)}
            log(f"bench: form {f}: {info.iters} iterations, solve {info.solve_ms:.1f} ms, "
                f"set-up {info.setup_ms:.0f} ms, error vs {prec} {err:.2e}")
    if not args.no_cpu_baseline:
        log(f"bench: timing the CPU oracle on a {args.cpu_sample}^3 crop")
        out["cpu_baseline"] = cpu_baseline(perm_h, wl, args.cpu_sample, levels)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
