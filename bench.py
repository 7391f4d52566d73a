"""Benchmark: PCG solve to 1e-6 relative residual with the multiscale spectral
multigrid preconditioner on one MI355X.

A step is one pass of the whole hot path on the workload: set-up (local
spectral problems on every level, Galerkin operators, smoother and coarsest
factorizations) followed by the preconditioned CG solve.  `value` is the
solve throughput, degrees of freedom per second of solve time, with the
inputs already resident in HBM.

Prints one JSON line (rank 0, single GPU).
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="gauss128", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=[None, "fp64", "fp32_vcycle", "fp32_basis"])
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
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=64, help="edge of the field crop timed on the CPU oracle")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run three plain device copies of COPY_BYTES each (counter calibration)")
    return ap.parse_args()


def cpu_baseline(perm, wl, edge):
    """The FP64 oracle on a bounded sample: an edge^3 corner crop of the same
    field, same levels / eigenvector count / source kind, full set-up and PCG."""
    from threadpoolctl import threadpool_limits
    from oracle import Grid, build_hierarchy, Preconditioner, pcg
    crop = np.ascontiguousarray(perm[:edge, :edge, :edge])
    g = Grid.unit_cube(edge)
    workers = min(os.cpu_count() or 1, 16)
    agg = 4 if edge % (8 * 4 ** max(0, wl.levels - 2)) == 0 else 2
    t0 = time.perf_counter()
    hier = build_hierarchy(crop, g, wl.levels, wl.eigs, sub=8, agg=agg, workers=workers)
    pre = Preconditioner(hier)
    t1 = time.perf_counter()
    b = make_source(wl.source, crop.shape).reshape(-1)
    ts = time.perf_counter()
    with threadpool_limits(limits=1):
        res = pcg(hier.A, b, pre.apply, tol=1e-6)
    t2 = time.perf_counter()
    return {
        "value": g.n / (t2 - ts),
        "unit": "DoF/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{edge}^3 corner crop of the {wl.name} field, {wl.levels} levels, {wl.eigs} eigs, "
                   f"agg {agg}; solve {t2 - ts:.2f} s ({res.iters} iters, numpy/scipy limited to one thread); "
                   f"set-up {t1 - t0:.2f} s on {workers} worker processes"),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not code).", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2403_19342_amd.specmg import SpecMG, FP64, FP32_VCYCLE, FP32_BASIS

    wl = WORKLOADS[args.config]
    if args.contrast is not None and wl.kind not in ("channels", "inclusions"):
        raise SystemExit("--contrast applies to the channels and inclusions fields")
    if args.eigs is not None or args.eigs_coarse is not None:
        wl = dataclasses.replace(wl, eigs=args.eigs or wl.eigs,
                                 eigs_coarse=wl.eigs_coarse if args.eigs_coarse is None else args.eigs_coarse)
    levels = args.levels or wl.levels
    prec = args.precision or wl.precision
    n = wl.n
    perm_h = make_field(wl.kind, n, wl.seed, **({} if args.contrast is None else {"value": args.contrast}))
    b_h = make_source(wl.source, perm_h.shape)
    dev = torch.device("cuda:0")
    perm = torch.as_tensor(perm_h, device=dev)
    b = torch.as_tensor(b_h.reshape(-1), device=dev)
    x = torch.zeros(n ** 3, dtype=torch.float64, device=dev)
    agg = wl.agg
    precision = {"fp32_vcycle": FP32_VCYCLE, "fp32_basis": FP32_BASIS}.get(prec, FP64)

    if args.copy_calibration:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step(profile):
        ctx = SpecMG(perm, levels=levels, eigs_per_subdomain=wl.eigs, agg=agg, precision=precision,
                     eigs_coarse=wl.eigs_coarse, eig_threshold_coarse=args.eig_threshold_coarse,
                     nu=args.nu, nu_c=args.nu_c, allow_unconverged=True)
        if args.solver == "gmres":
            # the per-kernel timing covers the CG solve only
            rc, info = ctx.gmres_solve(b, x, restart=args.restart, tol=1e-6, max_iter=1000)
            ctx.close()
            return info, None
        if profile:
            ctx.set_profiling(True)
        rc, info = ctx.pcg_solve(b, x, tol=1e-6, max_iter=1000)
        prof = ctx.profile() if profile else None
        ctx.close()
        return info, prof

    for _ in range(args.warmup):
        step(False)
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
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    plain = infos[:-1] if (len(infos) > 1 and profs) else infos
    solve_s = float(np.mean([i.solve_ms for i in plain])) / 1e3
    setup_s = float(np.mean([i.setup_ms for i in infos])) / 1e3
    iters = [i.iters for i in infos]
    dof = n ** 3
    # roofline of the kernel class with the largest share of solve time
    tot = {}
    for p in profs:
        for k, (ms, cnt, by) in p.items():
            a = tot.setdefault(k, [0.0, 0, by])
            a[0] += ms
            a[1] += cnt
    fine = [k for k in tot if k in ("cg_spmv", "pre_smooth", "resid_restrict", "prolong", "post_smooth",
                                    "post_residual")]
    roofline = None
    if fine:
        dom = max(fine, key=lambda k: tot[k][0])
        ms, cnt, by = tot[dom]
        from paper_2403_19342_amd.profile_summary import read_traffic
        measured = read_traffic(os.path.join(ROOT, "profiles", f"hbm_traffic_{wl.name}.md"))
        avg_ms = ms / max(cnt, 1)
        achieved = by / (avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": measured.get(dom),
                    "bytes_per_launch": by, "avg_launch_us": avg_ms * 1e3}
    kernels = {k: {"avg_us": 1e3 * v[0] / max(v[1], 1), "launches": v[1],
                   "GBps": (v[2] / (v[0] / max(v[1], 1) * 1e-3) / 1e9) if v[2] and v[0] else None}
               for k, v in tot.items() if v[1]}
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
        "dtype": {FP64: "f64", FP32_BASIS: "f64, f32 level-2 basis"}.get(
            precision, "f32 V-cycle / f64 " + ("CG" if args.solver == "pcg" else "GMRES")),
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": f"{n}^3", "dof": dof, "levels": levels, "solver": args.solver,
                   "eigs_per_subdomain": wl.eigs, "eigs_coarse": wl.eigs_coarse or wl.eigs, "agg": agg,
                   "field": wl.kind, "source": wl.source,
                   **({} if args.contrast is None else {"contrast": args.contrast}),
                   **({"eig_threshold_coarse": args.eig_threshold_coarse} if args.eig_threshold_coarse > 0 else {}),
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
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(perm_h, wl, args.cpu_sample)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
