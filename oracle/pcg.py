"""Preconditioned conjugate gradients around the V-cycle.

The paper runs PETSc GMRES to a relative tolerance of 1e-6 (Section 5); this
solve path uses PCG, which the symmetric preconditioner admits.  Stopping
test: ||r||_2 <= tol ||b||_2 on the recursively updated residual, confirmed on
the true residual b - A x; if the confirmation fails the true residual
replaces the recursive one and the iteration continues.  The result is
shifted to zero mean, the uniqueness condition of Section 2.1.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    converged: bool
    breakdown: bool
    rel_resid_true: float
    history: list


def pcg(A, b, precond, tol: float = 1e-6, max_iter: int = 1000, x0=None) -> PCGResult:
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b))
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A @ x if x0 is not None else b.copy()
    hist = [float(np.linalg.norm(r)) / nb if nb > 0 else 0.0]
    if nb == 0.0:
        return PCGResult(x, 0, True, False, 0.0, hist)
    if hist[0] <= tol:
        rt = float(np.linalg.norm(b - A @ x)) / nb
        return PCGResult(x - x.mean(), 0, True, False, rt, hist)
    z = precond(r)
    p = z.copy()
    rz = float(r @ z)
    it = 0
    converged = False
    breakdown = False
    while it < max_iter:
        q = A @ p
        pq = float(p @ q)
        if not np.isfinite(pq) or pq <= 0.0:
            breakdown = True
            break
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        it += 1
        rn = float(np.linalg.norm(r))
        hist.append(rn / nb)
        if rn <= tol * nb:
            rt = b - A @ x
            if float(np.linalg.norm(rt)) <= tol * nb:
                converged = True
                break
            r = rt
        z = precond(r)
        rz_new = float(r @ z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    x = x - x.mean()
    rel = float(np.linalg.norm(b - A @ x)) / nb
    return PCGResult(x, it, converged, breakdown, rel, hist)
