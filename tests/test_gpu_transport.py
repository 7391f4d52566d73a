"""Two-phase flow on the GPU against the oracle (Section 6).

- specmg_total_mobility: lambda(S) kappa per cell, S drawn over [0, 1] so
  the clamping of S* is exercised; same operations on both sides, so the bar
  is 1 ulp-level (1e-15 relative).
- specmg_transport: M sub-steps from the same synthetic S, porosity, sources
  (mixed signs) and face velocities (random, with exact zeros) on a cube, a
  ragged grid, a 1D column and a single cell; S within 1e-12 absolute and the
  summed sub-step length within 1e-12 relative.  The sub-step length depends
  on the largest rate, whose rounding may differ in the last bit between the
  two sides, hence not bit-exact.  Edge cases: zero sub-steps, no flow (all
  rates zero: dt = 0), and the argument checks.
- The improved IMPES driver (set-up on lambda(S) kappa, warm-started CG,
  flux recovery, sub-steps) for three pressure steps against the oracle's
  IMPES with a direct pressure solve, on a cube, on a grid whose three
  extents differ, with the FP32 V-cycle, and with the 20 : 10 : 2 cell
  spacings of the two-phase grid of Section 6: S within 1e-7, p within 1e-7
  relative, step lengths within 1e-7 relative (CG stops at 1e-10, and S
  depends on the velocity linearly through M sub-steps).
"""
import numpy as np
import pytest

from oracle import Grid
from oracle import impes as im
from synth.fields import five_spot, make_field, porosity_field, random_saturation
from tests.gpu_util import to_dev, to_host


def _work_size(n):
    return 2 * n + 2048          # the header's workspace rule

pytestmark = pytest.mark.gpu


def _random_inputs(shape, seed):
    rng = np.random.default_rng(seed)
    s = random_saturation(shape, seed)
    phi = rng.uniform(0.05, 0.35, shape)
    q = rng.standard_normal(shape) * (rng.random(shape) < 0.1)
    v = [rng.standard_normal(shape) * (rng.random(shape) < 0.9) for _ in range(3)]
    return s, phi, q, v


def test_total_mobility_matches_oracle():
    import torch
    from paper_2403_19342_amd.specmg import total_mobility
    shape = (9, 10, 11)
    perm = make_field("gauss", 11, 2, shape=shape)
    s = np.random.default_rng(3).uniform(0.0, 1.0, shape)
    out = torch.empty(shape, dtype=torch.float64, device="cuda")
    total_mobility(to_dev(perm), to_dev(s), out)
    ref = perm * im.total_mobility(s)
    err = np.max(np.abs(to_host(out) - ref) / ref)
    print(f"lambda(S) kappa: max rel err {err:.2e}")
    assert err <= 1e-15


@pytest.mark.parametrize("shape,substeps,ds_max,seed,hs", [
    ((32, 32, 32), 25, 1e-3, 1, None),
    ((7, 13, 19), 40, 1e-2, 2, None),
    ((7, 13, 19), 40, 1e-2, 5, (0.1, 0.05, 0.01)),
    ((1, 1, 257), 60, 5e-3, 3, None),
    ((1, 1, 1), 3, 1e-3, 4, None),
])
def test_transport_matches_oracle(shape, substeps, ds_max, seed, hs):
    import torch
    from paper_2403_19342_amd.specmg import transport
    s0, phi, q, (vx, vy, vz) = _random_inputs(shape, seed)
    if s0.size == 1:
        q[...] = 1.0                  # a lone injector cell: S rises by ds_max per sub-step
    h = 1.0 / shape[2] if hs is None else hs
    ref, tref = im.transport(phi, q, vx, vy, vz, s0, h, substeps, ds_max)
    s = to_dev(s0)
    work = torch.empty(_work_size(s0.size), dtype=torch.float64, device="cuda")
    t = torch.empty(1, dtype=torch.float64, device="cuda")
    transport(to_dev(phi), to_dev(q), to_dev(vx), to_dev(vy), to_dev(vz), s, h, substeps, ds_max, work, t)
    torch.cuda.synchronize()
    err = np.max(np.abs(to_host(s) - ref))
    terr = abs(t.item() - tref) / tref
    print(f"{shape} M={substeps}: max |dS| {err:.2e}, t {t.item():.6e} vs {tref:.6e} (rel {terr:.1e})")
    assert err <= 1e-12 and terr <= 1e-12
    assert tref > 0 and np.max(np.abs(to_host(s) - s0)) > 0    # the sub-steps did move S


def test_transport_edge_cases():
    import torch
    from paper_2403_19342_amd.specmg import SpecMGError, transport
    shape = (8, 8, 8)
    s0, phi, q, v = _random_inputs(shape, 5)
    work = torch.empty(_work_size(s0.size), dtype=torch.float64, device="cuda")
    t = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    # zero sub-steps: S unchanged, elapsed time 0
    s = to_dev(s0)
    transport(to_dev(phi), to_dev(q), *[to_dev(x) for x in v], s, 0.125, 0, 1e-3, work, t)
    assert np.array_equal(to_host(s), s0) and t.item() == 0.0
    # no flow and no sources: every rate is zero, dt = 0, S unchanged
    z = np.zeros(shape)
    t.fill_(7.0)
    transport(to_dev(phi), to_dev(z), to_dev(z), to_dev(z), to_dev(z), s, 0.125, 5, 1e-3, work, t)
    assert np.array_equal(to_host(s), s0) and t.item() == 0.0
    # argument checks
    for kw in ({"substeps": -1, "ds_max": 1e-3}, {"substeps": 2, "ds_max": 0.0}, {"substeps": 2, "ds_max": 2.0}):
        with pytest.raises(SpecMGError):
            transport(to_dev(phi), to_dev(q), *[to_dev(x) for x in v], s, 0.125, kw["substeps"], kw["ds_max"],
                      work, t)
    with pytest.raises(ValueError):
        transport(to_dev(phi), to_dev(q), *[to_dev(x) for x in v], s, 0.125, 1, 1e-3, work[:10], t)


@pytest.mark.parametrize("nx,ny,nz,precision,ratios", [(32, 32, 32, 0, None), (48, 32, 16, 0, None),
                                                       (32, 32, 32, 1, None), (32, 32, 32, 0, (20, 10, 2))])
def test_impes_driver_matches_oracle(nx, ny, nz, precision, ratios):
    # ratios: hx : hy : hz of the two-phase grid of Section 6
    import torch
    from paper_2403_19342_amd.impes import Impes
    h = 1.0 / nx if ratios is None else tuple(r / (20.0 * nx) for r in ratios)
    g = Grid(nx, ny, nz, *((h,) * 3 if ratios is None else h))
    perm = make_field("gauss", nx, 6, sigma=2.0, shape=g.shape)
    phi = porosity_field(perm, 6)
    q = five_spot(g.shape)
    s0 = np.full(g.shape, 0.2)
    steps, substeps, ds_max = 3, 20, 1e-2
    sref, pref, tref = im.impes(perm, phi, q, s0, g, steps, substeps, ds_max)
    run = Impes(to_dev(perm), to_dev(phi), to_dev(q), to_dev(s0), levels=3, eigs=4, agg=2, h=h, tol=1e-10,
                substeps=substeps, ds_max=ds_max, precision=precision)
    infos = [run.step() for _ in range(steps)]
    torch.cuda.synchronize()
    s, p = to_host(run.s), to_host(run.p)
    es = np.max(np.abs(s - sref))
    ep = np.linalg.norm(p - pref) / np.linalg.norm(pref)
    et = max(abs(i.dt_total - t) / t for i, t in zip(infos, tref))
    print(f"IMPES {nx}x{ny}x{nz} precision {precision} spacing ratios {ratios}, 3 steps: iterations {[i.iters for i in infos]}, "
          f"max |dS| {es:.2e}, p rel {ep:.2e}, t rel {et:.2e}, S range [{s.min():.4f}, {s.max():.4f}]")
    assert all(i.rel_resid <= 1e-10 for i in infos)
    assert es <= 1e-7 and ep <= 1e-7 and et <= 1e-7
    assert s.max() > 0.3                                   # water has entered
    # warm start: the later pressure steps start from the previous pressure
    assert infos[2].iters < infos[0].iters
