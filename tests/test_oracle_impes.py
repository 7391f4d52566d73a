"""Pins of the two-phase oracle (Section 6) against values fixed by hand,
the Buckley-Leverett solution, conservation and symmetry.

- Relative permeabilities, total mobility and fractional flow at saturations
  where they are simple fractions, worked out by hand from the Corey law and
  viscosities of Section 6, and their clamping outside [0.2, 0.8].
- The saturation scheme (upstream weighting, divergence, adaptive sub-steps)
  against the Buckley-Leverett solution of 1D water flooding: the front
  saturation from the Welge tangent, the rarefaction behind it from the
  characteristic speeds.  First-order upwinding smears the front, so the
  pin is an L1 bound plus convergence under refinement.
- Water volume: interior face fluxes cancel, so each sub-step changes
  sum(phi S) h^3 by exactly dt sum(q_w) h^3.
- Symmetry: a homogeneous grid with the five-spot wells is symmetric under
  x <-> y and both mirror images; the saturation must stay so.
- The pressure solve meets A p = q and has zero mean.
"""
import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import Grid, assemble, recover_flux
from oracle import impes as im
from synth.fields import five_spot, make_field, porosity_field


def test_closed_form_values():
    # S = 0.2: S* = 0, k_w = 0, k_o = 1 -> lambda = 1/3, f_w = 0
    # S = 0.8: S* = 1 -> lambda = 1/0.3 = 10/3, f_w = 1
    # S = 0.5: S* = 1/2, k_w = k_o = 1/4 -> lambda = 5/6 + 1/12 = 11/12, f_w = 10/11
    # S = 0.35: S* = 1/4, k_w = 1/16, k_o = 9/16 -> lambda = 5/24 + 3/16 = 19/48, f_w = 10/19
    s = np.array([0.2, 0.8, 0.5, 0.35])
    lam = np.array([1 / 3, 10 / 3, 11 / 12, 19 / 48])
    fw = np.array([0.0, 1.0, 10 / 11, 10 / 19])
    assert np.allclose(im.total_mobility(s), lam, rtol=1e-14, atol=0)
    assert np.allclose(im.frac_flow(s), fw, rtol=1e-14, atol=1e-16)
    kw, ko = im.rel_perms(s)
    assert np.allclose(kw, [0, 1, 0.25, 1 / 16], rtol=1e-14, atol=1e-16)
    assert np.allclose(ko, [1, 0, 0.25, 9 / 16], rtol=1e-14, atol=1e-16)
    # outside [0.2, 0.8] the law is flat
    assert im.total_mobility(0.05) == im.total_mobility(0.2)
    assert im.frac_flow(0.95) == im.frac_flow(0.8) == 1.0
    # sources: water injected where q > 0, the cell's mixture produced where q < 0
    q = np.array([2.0, -2.0, -2.0])
    assert np.allclose(im.water_source(q, np.array([0.2, 0.5, 0.2])), [2.0, -20 / 11, 0.0], rtol=1e-14)


def _bl_profile(x, t, u, phi):
    """Buckley-Leverett saturation at positions x and time t (initial S = 0.2,
    pure water injected at x = 0), written from the fractional flow in S*."""
    def f(sn):
        a = 10.0 * sn * sn
        return a / (a + (1.0 - sn) ** 2)

    def df(sn):                       # d f / d S* of the expression above
        d = 10.0 * sn * sn + (1.0 - sn) ** 2
        return (20.0 * sn * d - 10.0 * sn * sn * (20.0 * sn - 2.0 * (1.0 - sn))) / (d * d)

    # Welge tangent from (S* = 0, f = 0): sn f'(sn) = f(sn); dS/dS* = 0.6
    snf = brentq(lambda sn: sn * df(sn) - f(sn), 0.05, 0.95)
    speed = lambda sn: u * df(sn) / (0.6 * phi)        # characteristic speed dx/dt
    out = np.full(x.shape, 0.2)
    xf = speed(snf) * t
    for i, xi in enumerate(x):
        if xi < xf:
            # rarefaction: the S* > snf with speed(S*) t = xi (speed decreases there)
            if speed(1.0 - 1e-12) * t >= xi:
                sn = 1.0
            else:
                sn = brentq(lambda s: speed(s) * t - xi, snf, 1.0 - 1e-12)
            out[i] = 0.2 + 0.6 * sn
    return out, 0.2 + 0.6 * snf, xf


def _flood_1d(n, t_end, phi=0.2, u=1.0, ds_max=0.01, axis=2, other=1.0):
    """Water flood along one axis (2: x, 0: z) of a column of n cells; the
    two other spacings are `other`, which must not enter the result."""
    h = 1.0 / n
    shape = [1, 1, 1]
    shape[axis] = n
    shape = tuple(shape)
    hs = [other, other, other]
    hs[2 - axis] = h                   # (hx, hy, hz) with the flow axis at spacing h
    q = np.zeros(n)
    q[0] = u / h
    q[-1] = -u / h
    v = np.zeros(n)
    v[:-1] = u                         # uniform total velocity through every interior face
    zero = np.zeros(shape)
    vel = [zero, zero, zero]
    vel[2 - axis] = v.reshape(shape)
    ph = np.full(shape, phi)
    s = np.full(shape, 0.2)
    t = 0.0
    while t < t_end:
        s, dt = im.transport(ph, q.reshape(shape), vel[0], vel[1], vel[2], s, tuple(hs), 1, ds_max)
        t += dt
    x = (np.arange(n) + 0.5) * h
    return x, s.reshape(-1), t


@pytest.mark.parametrize("axis,other", [(2, 1.0), (0, 7.0)])
def test_buckley_leverett_front(axis, other):
    # along x with unit cross spacings, and along z with cross spacings of 7
    errs = []
    for n in (200, 400):
        x, s, t = _flood_1d(n, 0.02, axis=axis, other=other)
        exact, sf, xf = _bl_profile(x, t, 1.0, 0.2)
        err = np.mean(np.abs(s - exact))
        errs.append(err)
        # the front: where S first drops below the midpoint of S_f and S_wc
        mid = 0.5 * (sf + 0.2)
        xnum = x[np.argmax(s < mid)]
        print(f"n {n}: t {t:.4f}, S_f {sf:.4f}, front {xnum:.4f} vs {xf:.4f}, L1 {err:.4f}")
        assert abs(xnum - xf) <= 0.025
        assert err <= 0.01
        # water volume: injected u t equals the stored phi (S - 0.2) integrated
        assert abs(np.sum(0.2 * (s - 0.2)) / n - 1.0 * t) <= 1e-12 * t + 1e-15
    assert errs[1] <= 0.8 * errs[0]


def test_water_volume_per_substep():
    n = 12
    g = Grid.unit_cube(n)
    perm = make_field("gauss", n, 3, sigma=2.0)
    phi = porosity_field(perm, 3)
    q = five_spot(g.shape)
    rng = np.random.default_rng(4)
    s = rng.uniform(0.2, 0.8, g.shape)
    keff = perm * im.total_mobility(s)
    p = im.pressure_solve(keff, g, q)
    vx, vy, vz = recover_flux(keff, g, p)
    vol = g.hx ** 3
    for _ in range(5):
        expect = np.sum(im.water_source(q, s)) * vol
        s1, dt = im.transport(phi, q, vx, vy, vz, s, g.hx, 1, 1e-3)
        got = np.sum(phi * (s1 - s)) * vol
        assert dt > 0
        assert abs(got - dt * expect) <= 1e-13 * np.sum(np.abs(phi * s)) * vol
        s = s1


def test_five_spot_symmetry_and_bounds():
    g = Grid(15, 15, 3, 1 / 15, 1 / 15, 1 / 15)
    perm = np.ones(g.shape)
    phi = np.full(g.shape, 0.2)
    q = five_spot(g.shape)
    s0 = np.full(g.shape, 0.2)
    s, p, times = im.impes(perm, phi, q, s0, g, steps=3, substeps=20, ds_max=0.01)
    assert all(t > 0 for t in times)
    assert np.max(np.abs(s - s.transpose(0, 2, 1))) <= 1e-12
    assert np.max(np.abs(s - s[:, :, ::-1])) <= 1e-12
    assert np.max(np.abs(s - s[:, ::-1, :])) <= 1e-12
    assert s.min() >= 0.2 - 1e-12 and s.max() <= 0.8 + 1e-12
    # water has entered at the injector and not yet reached the producers
    assert s[1, 7, 7] > 0.3 and s[1, 0, 0] == pytest.approx(0.2, abs=1e-9)


def test_pressure_solve_definition():
    n = 8
    g = Grid.unit_cube(n)
    perm = make_field("gauss", n, 5, sigma=2.0)
    q = five_spot(g.shape).reshape(-1)
    p = im.pressure_solve(perm, g, q)
    A = assemble(perm, g)
    assert np.linalg.norm(A @ p - q) <= 1e-10 * np.linalg.norm(q)
    assert abs(p.mean()) <= 1e-14 * np.max(np.abs(p))
