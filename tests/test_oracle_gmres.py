"""Pins of the oracle's flexible GMRES against what the mathematics fixes:
finite termination on a small system (a dense solve), the minimal-residual
property over the Krylov space (a brute-force least-squares problem),
restarted convergence on a positive definite system, a preconditioner that
changes between applications, and agreement with the independent PCG
oracle on the pressure system with the V-cycle."""
import numpy as np
import pytest

from oracle import Grid, Preconditioner, build_hierarchy, fgmres, pcg
from synth.fields import make_field, make_source


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((n, n))
    return Q @ Q.T + n * np.eye(n), rng.standard_normal(n)


def test_finite_termination_matches_dense_solve():
    A, b = _spd(12, 0)
    res = fgmres(A, b, lambda v: v, tol=1e-13, restart=12)
    x = np.linalg.solve(A, b)
    assert res.converged and res.iters <= 12
    assert np.linalg.norm(res.x - (x - x.mean())) <= 1e-12 * np.linalg.norm(x)


@pytest.mark.parametrize("k", [1, 3, 6])
def test_arnoldi_residual_is_the_krylov_minimum(k):
    # with a fixed preconditioner M, x_k = M V_k y minimises ||b - A M v|| over
    # v in K_k(A M, b); brute force: orthonormal basis of the power sequence
    n = 10
    A, b = _spd(n, 1)
    rng = np.random.default_rng(2)
    M = np.diag(rng.uniform(0.5, 2.0, n)) + 0.1 * rng.standard_normal((n, n))   # not symmetric
    res = fgmres(A, b, lambda v: M @ v, tol=1e-300, restart=n, max_iter=k)
    K = np.empty((n, k))
    v = b.copy()
    for j in range(k):
        K[:, j] = v
        v = A @ (M @ v)
    Qk, _ = np.linalg.qr(K)
    AMQ = A @ (M @ Qk)
    y, *_ = np.linalg.lstsq(AMQ, b, rcond=None)
    rmin = np.linalg.norm(b - AMQ @ y)
    assert res.iters == k
    assert abs(res.hist[-1] * np.linalg.norm(b) - rmin) <= 1e-10 * np.linalg.norm(b)


def test_restarted_converges_monotonically():
    A, b = _spd(12, 3)
    res = fgmres(A, b, lambda v: v, tol=1e-10, restart=3, max_iter=500)
    assert res.converged and res.restarts > 0
    h = np.asarray(res.hist)
    assert np.all(np.diff(h) <= 1e-12)


def test_changing_preconditioner_is_allowed():
    A, b = _spd(12, 4)
    rng = np.random.default_rng(5)
    D = [np.diag(rng.uniform(0.2, 5.0, 12)) for _ in range(2)]
    calls = [0]

    def prec(v):
        calls[0] += 1
        return D[calls[0] % 2] @ v

    res = fgmres(A, b, prec, tol=1e-10, restart=12)
    x = np.linalg.solve(A, b)
    assert res.converged
    assert np.linalg.norm(res.x - (x - x.mean())) <= 1e-8 * np.linalg.norm(x)


def test_agrees_with_pcg_on_the_pressure_system():
    perm = make_field("gauss", 16, 7)
    g = Grid.unit_cube(16)
    hier = build_hierarchy(perm, g, 2, 4, sub=8, agg=2, workers=1)
    b = make_source("corner", perm.shape).reshape(-1)
    pre = Preconditioner(hier)
    rg = fgmres(hier.A, b, pre.apply, tol=1e-10, restart=30)
    rc = pcg(hier.A, b, pre.apply, tol=1e-10)
    assert rg.converged and rc.converged
    assert abs(np.mean(rg.x)) <= 1e-14 * np.linalg.norm(rg.x)
    assert np.linalg.norm(rg.x - rc.x) <= 1e-8 * np.linalg.norm(rc.x)
