"""Pins of the smoothing-step counts (nu on the fine level, nu_c on the
coarse levels, Section 5) against dense linear algebra on a tiny grid.

- Two block-Jacobi sweeps from zero, u1 = M^-1 f, u2 = u1 + M^-1 (f - A u1),
  equal (2 M^-1 - M^-1 A M^-1) f, with M^-1 assembled column by column from
  the smoother and the product formed densely.
- The three-level preconditioner with (nu, nu_c) = (2, 2), (2, 1), (1, 2)
  is symmetric (the post-sweeps are the adjoints of the pre-sweeps because
  each block factor is symmetric) and positive on zero-mean vectors, and two
  sweeps give a spectrally better preconditioner than one (fewer CG
  iterations on the same system).
"""
import numpy as np
import pytest

from oracle import Grid, Preconditioner, build_hierarchy, pcg
from synth.fields import make_field, make_source, random_zero_mean


@pytest.fixture(scope="module")
def tiny():
    g = Grid(16, 16, 16, 1 / 16, 1 / 16, 1 / 16)
    perm = make_field("gauss", 16, 2, sigma=2.0)
    return g, build_hierarchy(perm, g, 3, 4, sub=8, agg=2, workers=1)


def _dense(fn, n):
    return np.column_stack([fn(np.eye(n)[:, i]) for i in range(n)])


def test_two_sweeps_closed_form(tiny):
    # fine level on a 16 x 8 x 8 grid (two 8^3 blocks), dense in 1024 columns
    gs = Grid(16, 8, 8, 1 / 16, 1 / 16, 1 / 16)
    hs = build_hierarchy(make_field("gauss", 16, 5, sigma=2.0, shape=gs.shape), gs, 2, 4, sub=8, agg=2, workers=1)
    Ps = Preconditioner(hs, nu=2)
    A = hs.A.toarray()
    f = np.random.default_rng(1).standard_normal(gs.n)
    Minv = _dense(Ps.fine.apply, gs.n)
    want = 2.0 * Minv @ f - Minv @ (A @ (Minv @ f))
    got = Ps._smooth(1, hs.A, f)
    assert np.linalg.norm(got - want) <= 1e-12 * np.linalg.norm(want)
    # coarse level 2 of the three-level hierarchy
    g, hier = tiny
    P = Preconditioner(hier, nu=2, nu_c=2)
    A2 = hier.level(2).A.toarray()
    n2 = A2.shape[0]
    f2 = np.random.default_rng(2).standard_normal(n2)
    M2 = _dense(P.coarse[2].apply, n2)
    want2 = 2.0 * M2 @ f2 - M2 @ (A2 @ (M2 @ f2))
    got2 = P._smooth(2, hier.level(2).A, f2)
    assert np.linalg.norm(got2 - want2) <= 1e-12 * np.linalg.norm(want2)


@pytest.mark.parametrize("nu,nu_c", [(2, 2), (2, 1), (1, 2)])
def test_symmetric_positive_and_better(tiny, nu, nu_c):
    g, hier = tiny
    P = Preconditioner(hier, nu=nu, nu_c=nu_c)
    u = random_zero_mean(g.shape, 3).reshape(-1)
    v = random_zero_mean(g.shape, 4).reshape(-1)
    pu, pv = P.apply(u), P.apply(v)
    assert abs(u @ pv - v @ pu) <= 1e-10 * np.linalg.norm(u) * np.linalg.norm(pv)
    assert u @ pu > 0 and v @ pv > 0
    b = make_source("five_spot", g.shape).reshape(-1)
    one = pcg(hier.A, b, Preconditioner(hier).apply, tol=1e-8)
    two = pcg(hier.A, b, P.apply, tol=1e-8)
    print(f"(nu, nu_c) = ({nu}, {nu_c}): {two.iters} iterations against {one.iters} with (1, 1)")
    assert two.converged and two.iters <= one.iters
