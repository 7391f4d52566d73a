"""Oracle: restarted flexible GMRES (right preconditioning), FP64.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline of the benchmark, never by the product path.

The paper's experiments use GMRES with its library's default parameters
(restart length 30) as the outer Krylov solver around the multilevel
preconditioner and stop at a relative residual of 1e-6 (Section 5, set-up
of the numerical experiments).  The algorithm is the textbook
flexible GMRES (Saad, "Iterative Methods for Sparse Linear Systems", 2nd
ed., Algorithm 9.6): z_j = M^{-1} v_j is stored, so a preconditioner that
changes between applications (the FP32 V-cycle) is allowed, and the update
is x = x0 + Z_k y_k.  Orthogonalisation is modified Gram-Schmidt, the small
least-squares problem is reduced by Givens rotations.

Stopping (the reading used by the GPU solver too): inside a cycle the
Arnoldi residual |g_{j+1}| is the true residual norm of the current iterate
in exact arithmetic; when it falls to tol * ||b|| (or the cycle is full)
the iterate is formed, the true residual b - A x is computed, and the solve
ends if ||b - A x|| <= tol ||b||, else GMRES restarts from that residual.
The returned solution has zero mean (the operator's null space is the
constants).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class GMRESResult:
    x: np.ndarray
    iters: int                 # Arnoldi steps (one operator and one preconditioner apply each)
    converged: bool
    rel_resid_true: float
    restarts: int
    hist: list = field(default_factory=list)   # |g_{j+1}| / ||b|| after every step


def fgmres(A, b, precond, tol: float = 1e-6, restart: int = 30, max_iter: int = 1000, x0=None) -> GMRESResult:
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    nb = float(np.linalg.norm(b))
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    if nb == 0.0:
        return GMRESResult(np.zeros(n), 0, True, 0.0, 0, [0.0])
    r = b - A @ x
    beta = float(np.linalg.norm(r))
    hist = [beta / nb]
    it = 0
    restarts = 0
    converged = beta <= tol * nb
    while not converged and it < max_iter:
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        V[0] = r / beta
        g[0] = beta
        k = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = A @ Z[j]
            for i in range(j + 1):               # modified Gram-Schmidt
                H[i, j] = float(V[i] @ w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = float(np.linalg.norm(w))
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):                   # previous rotations on column j
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = float(np.hypot(H[j, j], H[j + 1, j]))
            cs[j] = H[j, j] / d
            sn[j] = H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) <= tol * nb or it >= max_iter:
                break
        # y = H_k^{-1} g_k (upper triangular), x += Z_k y
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y
        r = b - A @ x
        beta = float(np.linalg.norm(r))
        converged = beta <= tol * nb
        if not converged:
            restarts += 1
    x = x - x.mean()
    rt = float(np.linalg.norm(b - A @ x)) / nb
    return GMRESResult(x, it, converged, rt, restarts, hist)
