"""Train the warm-start network on eigenpairs the library's own set-up produces.

    python -m paper_2403_19342_amd.train_cnn --out DIR [--n 128] [--fields 16]
        [--k 6] [--steps 3000] [--batch 512] [--lr 2e-3] [--eval 4]
    python -m paper_2403_19342_amd.train_cnn --out DIR --weights FILE --eval 32

Training fields are Gaussian log-permeability fields with sigma ~ U[2,4] and
correlation length ~ U[0.05,0.2] (seeds 10000, 10001, ...); each field's
level-2 eigenvectors come from a set-up of this library (3 levels, the
coarse levels are not used).  The network, its loss and Adam run in the
library's kernels.  DIR receives theta_f32.npy (float32 master parameters)
and theta_bf16.npy (int16 bf16 bits, the set-up's cnn_weights).  With --eval
E, set-ups with and without the warm start are compared on E test fields
(seeds 1000, 1001, ...) and reported as one JSON line per field.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from synth.fields import learned_field  # noqa: E402


def init_params(k: int, seed: int) -> np.ndarray:
    """He-normal weights, small normal biases, in the library's parameter order;
    the output layer starts near zero, so training starts from the cold modes."""
    from paper_2403_19342_amd.specmg import load_library
    rng = np.random.default_rng(seed)
    shapes = [(32, 1 + k), (32,), (32, 32), (32,), (k, 32), (k,)]
    parts = []
    for i, shp in enumerate(shapes):
        scale = 0.01 if i >= 4 else 1.0
        if len(shp) == 2:
            parts.append(rng.standard_normal(shp[0] * shp[1] * 27) * np.sqrt(2.0 / (shp[1] * 27)) * scale)
        else:
            parts.append(rng.standard_normal(shp[0]) * 0.05 * scale)
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == load_library().specmg_cnn_param_count(k)
    return theta


def dataset(n: int, seeds, k: int, levels: int = 3):
    """Device tensors: patches [N,1000] f32, weights [N,512] f64, targets [N,k,512] f64."""
    import torch
    from paper_2403_19342_amd.specmg import CNN, SpecMG
    Ps, Ss, Fs = [], [], []
    for sd in seeds:
        perm = torch.as_tensor(learned_field(n, sd), device="cuda")
        m = (n // 8) ** 3
        P = torch.empty(m * 1000, dtype=torch.float32, device="cuda")
        S = torch.empty(m * 512, dtype=torch.float64, device="cuda")
        CNN.patches(perm, 0, m, P, S)
        ctx = SpecMG(perm, levels=levels, eigs_per_subdomain=k)
        basis = ctx.level_arrays(2).basis
        ctx.close()
        Ps.append(P.view(m, 1000))
        Ss.append(S.view(m, 512))
        Fs.append(torch.as_tensor(np.ascontiguousarray(basis[:, :k, :]), device="cuda"))
        print(f"field {sd}: {m} elements", flush=True)
    return torch.cat(Ps).contiguous(), torch.cat(Ss).contiguous(), torch.cat(Fs).contiguous()


def train(P, S, F, k: int, steps: int, batch: int, lr: float, seed: int = 0, log_every: int = 100):
    import torch
    from paper_2403_19342_amd.specmg import CNN
    N = P.shape[0]
    batch = min(batch, N)
    net = CNN(k, batch)
    theta = torch.as_tensor(init_params(k, seed), device="cuda")
    theta16 = torch.empty(theta.numel(), dtype=torch.int16, device="cuda")
    m1 = torch.zeros_like(theta)
    m2 = torch.zeros_like(theta)
    grad = torch.empty_like(theta)
    X = torch.empty(batch * net.kp * 512, dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cpu").manual_seed(seed)
    history = []
    t0 = time.perf_counter()
    for it in range(1, steps + 1):
        idx = torch.randperm(N, generator=gen)[:batch].to("cuda")
        Pb, Sb, Fb = P[idx].contiguous(), S[idx].contiguous(), F[idx].contiguous()
        net.load(theta)
        net.forward(Pb, batch, X)
        loss = net.loss_backward(Pb, X, Fb, k, Sb, batch, grad)
        # cosine decay to a tenth of the initial rate
        rate = lr * (0.1 + 0.9 * 0.5 * (1.0 + np.cos(np.pi * (it - 1) / steps)))
        net.adam(theta, grad, m1, m2, rate, it, theta16)
        history.append(loss)
        if it % log_every == 0 or it == steps:
            print(f"step {it}: loss {np.mean(history[-log_every:]):.5f} ({time.perf_counter() - t0:.1f} s)",
                  flush=True)
    torch.cuda.synchronize()
    net.close()
    return theta, theta16, history, time.perf_counter() - t0


def modes_only(k: int):
    """bf16 parameters with a zero output layer: the network returns the cold
    start's cosine modes (the learned set-up without a trained network)."""
    import torch
    th = init_params(k, 0)
    th[-(k * 32 * 27 + k):] = 0.0
    bits = (th.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)   # exact: no rounding needed for 0
    th16 = torch.as_tensor(bits.copy(), device="cuda")
    return th16


def evaluate(theta16, n: int, seeds, k: int, levels: int = 3, ws_resid_tol: float = 1e-3):
    """Set-up and solve per test field for five forms: the plain FP64 method
    (exact local eigensolves), the FP32 V-cycle alone, the FP32 V-cycle with
    the learned set-up started from the cosine modes (no network) and from
    the trained network, and the FP32-basis mode with the trained network.
    Solutions are compared with the plain one."""
    import torch
    from paper_2403_19342_amd.specmg import SpecMG, FP64, FP32_VCYCLE, FP32_BASIS
    from synth.fields import make_source
    out = []
    variants = (("fp64_exact", None, FP64), ("fp32_exact", None, FP32_VCYCLE),
                ("fp32_modes", modes_only(k), FP32_VCYCLE), ("fp32_trained", theta16, FP32_VCYCLE),
                ("fp32basis_trained", theta16, FP32_BASIS))
    for sd in seeds:
        perm = torch.as_tensor(learned_field(n, sd), device="cuda")
        b = torch.as_tensor(make_source("quarter_five_spot", (n, n, n)).reshape(-1), device="cuda")
        row = {"seed": sd}
        x_ref = None
        for name, w, prec in variants:
            ctx = SpecMG(perm, levels=levels, eigs_per_subdomain=k, cnn_weights=w, ws_resid_tol=ws_resid_tol,
                         precision=prec)
            inf = ctx.info()["setup"]
            cyc = ctx.level_arrays(2).status
            x = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
            _, si = ctx.pcg_solve(b, x, tol=1e-6)
            if x_ref is None:
                x_ref = x
            diff = float(torch.linalg.norm(x - x_ref) / torch.linalg.norm(x_ref))
            row[name] = {"setup_ms": inf["setup_ms"], "solve_ms": si.solve_ms,
                         "total_ms": inf["setup_ms"] + si.solve_ms, "iters": si.iters,
                         "rel_resid_true": si.rel_resid_true, "rel_diff_vs_fp64": diff,
                         "fallbacks": inf["ws_fallbacks"], "mean_cycles": float(cyc.mean()),
                         "max_cycles": int(cyc.max())}
            ctx.close()
        out.append(row)
        print(json.dumps(row), flush=True)
    return out


def summarize(rows):
    """Means over test fields of each form's set-up, solve and iterations."""
    names = [k for k in rows[0] if k != "seed"]
    summ = {}
    for nm in names:
        summ[nm] = {f: float(np.mean([r[nm][f] for r in rows]))
                    for f in ("setup_ms", "solve_ms", "total_ms", "iters", "mean_cycles", "fallbacks",
                              "rel_diff_vs_fp64")}
        summ[nm]["max_iter_ratio"] = float(max(r[nm]["iters"] / r[names[0]]["iters"] for r in rows))
    return summ


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--fields", type=int, default=16)
    ap.add_argument("--k", type=int, default=6)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval", type=int, default=4)
    ap.add_argument("--ws-resid-tol", type=float, default=1e-3)
    ap.add_argument("--weights", default=None,
                    help="evaluate these bf16 parameters (int16 .npy) instead of training")
    a = ap.parse_args(argv)
    if a.weights:
        import torch
        theta16 = torch.as_tensor(np.load(a.weights), device="cuda")
        rows = evaluate(theta16, a.n, range(1000, 1000 + a.eval), a.k, ws_resid_tol=a.ws_resid_tol)
        print(json.dumps({"summary": summarize(rows), "fields": len(rows), "weights": a.weights}), flush=True)
        return
    P, S, F = dataset(a.n, range(10000, 10000 + a.fields), a.k)
    theta, theta16, hist, secs = train(P, S, F, a.k, a.steps, a.batch, a.lr)
    os.makedirs(a.out, exist_ok=True)
    np.save(os.path.join(a.out, "theta_f32.npy"), theta.cpu().numpy())
    np.save(os.path.join(a.out, "theta_bf16.npy"), theta16.cpu().numpy())
    print(json.dumps({"train_elements": int(P.shape[0]), "steps": a.steps, "batch": a.batch,
                      "seconds": secs, "loss_first": float(np.mean(hist[:20])),
                      "loss_last": float(np.mean(hist[-20:]))}), flush=True)
    if a.eval:
        rows = evaluate(theta16, a.n, range(1000, 1000 + a.eval), a.k, ws_resid_tol=a.ws_resid_tol)
        print(json.dumps({"summary": summarize(rows), "fields": len(rows)}), flush=True)


if __name__ == "__main__":
    main()
