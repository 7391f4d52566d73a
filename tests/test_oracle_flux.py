"""Pins of the oracle's velocity recovery and mass balance (Section 2.2,
eq. (velocity) and the cell conservation relation): the discrete divergence
of the recovered flux is the assembled operator applied to p (two codes
written from different passages must agree), a linear pressure on a
homogeneous medium gives the constant Darcy flux, a two-cell case by hand,
zero flux through the no-flow boundary, and a balanced solve."""
import numpy as np

from oracle import Grid, Preconditioner, assemble, build_hierarchy, mass_balance, pcg, recover_flux
from synth.fields import make_field, make_source


def test_divergence_of_the_flux_is_A_p():
    g = Grid.unit_cube(6, 5, 4)
    rng = np.random.default_rng(0)
    perm = np.exp(rng.normal(0.0, 2.0, g.shape))
    p = rng.standard_normal(g.n)
    vx, vy, vz = recover_flux(perm, g, p)
    Ap = assemble(perm, g) @ p
    res = mass_balance(g, vx, vy, vz, np.zeros(g.n))
    assert np.max(np.abs(res - Ap)) <= 1e-12 * np.max(np.abs(Ap))


def test_linear_pressure_gives_the_darcy_flux():
    g = Grid.unit_cube(5)
    kappa = 2.5
    perm = np.full(g.shape, kappa)
    x = (np.arange(g.nx) + 0.5) * g.hx
    p = np.broadcast_to(x, g.shape).reshape(-1)
    vx, vy, vz = recover_flux(perm, g, p)
    assert np.allclose(vx[:, :, :-1], -kappa, rtol=1e-14, atol=0)   # v = -kappa dp/dx
    assert np.all(vx[:, :, -1] == 0.0)
    assert np.all(vy == 0.0) and np.all(vz == 0.0)


def test_two_cells_by_hand():
    g = Grid(2, 1, 1, 0.5, 1.0, 1.0)
    perm = np.array([1.0, 3.0]).reshape(g.shape)
    vx, vy, vz = recover_flux(perm, g, np.array([0.0, 1.0]))
    # face kappa 2 / (1/1 + 1/3) = 1.5, v = -1.5 * (1 - 0) / 0.5 = -3
    assert vx.reshape(-1).tolist() == [-3.0, 0.0]
    # cell 0 loses 3 through its +x face of area 1 over volume 0.5: div = -6
    res = mass_balance(g, vx, vy, vz, np.zeros(2))
    assert np.allclose(res, [-6.0, 6.0], rtol=1e-15, atol=0)


def test_no_flow_boundary_and_balanced_solve():
    perm = make_field("gauss", 16, 5)
    g = Grid.unit_cube(16)
    b = make_source("corner", perm.shape).reshape(-1)
    hier = build_hierarchy(perm, g, 2, 4, sub=8, agg=2, workers=1)
    res = pcg(hier.A, b, Preconditioner(hier).apply, tol=1e-10)
    vx, vy, vz = recover_flux(perm, g, res.x)
    assert np.all(vx[:, :, -1] == 0.0) and np.all(vy[:, -1, :] == 0.0) and np.all(vz[-1, :, :] == 0.0)
    mb = mass_balance(g, vx, vy, vz, b)
    assert np.linalg.norm(mb) <= 1e-9 * np.linalg.norm(b)


def test_orthotropic_divergence_of_the_flux_is_A_p():
    # K = diag(kappa_x, kappa_y, kappa_z) per cell, unequal spacings: the
    # discrete divergence of the recovered flux is the assembled operator
    g = Grid(6, 5, 4, 0.3, 0.2, 0.7)
    rng = np.random.default_rng(1)
    perm = np.exp(rng.normal(0.0, 2.0, (3,) + g.shape))
    p = rng.standard_normal(g.n)
    vx, vy, vz = recover_flux(perm, g, p)
    Ap = assemble(perm, g) @ p
    res = mass_balance(g, vx, vy, vz, np.zeros(g.n))
    assert np.max(np.abs(res - Ap)) <= 1e-12 * np.max(np.abs(Ap))


def test_orthotropic_linear_pressures_give_each_axis_its_own_kappa():
    # a constant tensor diag(2, 3, 5): a pressure linear along axis d drives
    # the flux -kappa_d along d and nothing across
    g = Grid.unit_cube(5)
    perm = np.stack([np.full(g.shape, k) for k in (2.0, 3.0, 5.0)])
    c = (np.arange(5) + 0.5) / 5
    for axis, kappa in ((2, 2.0), (1, 3.0), (0, 5.0)):
        shape = [1, 1, 1]
        shape[axis] = 5
        p = np.broadcast_to(c.reshape(shape), g.shape).reshape(-1)
        v = recover_flux(perm, g, p)
        main = v[2 - axis]
        sl = [slice(None)] * 3
        sl[axis] = slice(0, -1)
        assert np.allclose(main[tuple(sl)], -kappa, rtol=1e-14, atol=0)
        for other in range(3):
            if other != 2 - axis:
                assert np.all(v[other] == 0.0)
