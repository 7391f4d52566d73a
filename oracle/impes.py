"""Oracle: the two-phase flow application of Section 6, FP64.

TEST INFRASTRUCTURE ONLY: imported by tests/ only, never by the product path.

Incompressible, immiscible water/oil flow without gravity or capillary
pressure, with p the pressure and S the water saturation (eqs. v, div_v,
trans_S):

    v = -lambda(S) K grad p,   div v = q,   phi dS/dt + div(f_w(S) v) = q_w,

with the relative permeabilities and viscosities of Section 6:

    S* = (S - 0.2) / 0.6,  k_w = S*^2,  k_o = (1 - S*)^2,
    mu_w = 0.3, mu_o = 3.0,
    lambda = k_w/mu_w + k_o/mu_o,  f_w = (k_w/mu_w) / lambda.

The improved IMPES scheme (eqs. IMP and ES): for each pressure step, solve
the pressure system with the permeability lambda(S^n) kappa, recover the
face velocity v^{n+1}, then take M explicit Euler sub-steps of the
saturation equation in which the water flux through a face uses f_w of the
upstream cell and the sub-step length makes the largest change of S equal
to DS_max.

Readings (where the paper leaves a choice):
  - S* is clamped to [0, 1], so k_w, k_o and f_w are flat outside
    S in [0.2, 0.8].
  - Wells are rate controlled: q is given per cell.  A cell with q > 0
    injects water (q_w = q); a cell with q < 0 produces the mixture it holds
    (q_w = f_w(S) q).  The paper's producers are bottom-hole-pressure wells
    whose well-index term enters the pressure operator; those are not
    modelled here.
  - The sub-step length is dt = DS_max / max_cells |dS/dt|, the rate being
    (q_w - div(f_w v)) / phi at the start of the sub-step; dt = 0 when every
    rate is zero.
  - K is isotropic (one kappa per cell); the spacings may differ per axis
    (the cells of Section 6 measure 20 x 10 x 2 ft): the surface integral of
    eq. ES over a cell is then sum_d (F_+ - F_-) / h_d.

Arrays are (nz, ny, nx) in C order; each face array holds the velocity
through the + face of every cell, zero on the no-flow boundary.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .assembly import Grid, assemble
from .flux import recover_flux

S_WC = 0.2          # connate water saturation: S* = 0 below it
S_SPAN = 0.6        # 1 - S_wc - S_or with S_or = 0.2
MU_W = 0.3
MU_O = 3.0


def rel_perms(s):
    """(k_w, k_o) of the Corey-type law of Section 6."""
    sn = np.clip((np.asarray(s, dtype=np.float64) - S_WC) / S_SPAN, 0.0, 1.0)
    return sn * sn, (1.0 - sn) * (1.0 - sn)


def total_mobility(s):
    kw, ko = rel_perms(s)
    return kw / MU_W + ko / MU_O


def frac_flow(s):
    kw, ko = rel_perms(s)
    lw = kw / MU_W
    return lw / (lw + ko / MU_O)


def water_source(q, s):
    """q_w per cell: injected water where q > 0, the cell's mixture where q < 0."""
    q = np.asarray(q, dtype=np.float64)
    return np.where(q > 0.0, q, frac_flow(s) * q)


def _spacings(h):
    """(hx, hy, hz) from one spacing or a triple."""
    return (float(h),) * 3 if np.ndim(h) == 0 else tuple(float(v) for v in h)


def saturation_rate(phi, q, vx, vy, vz, s, h):
    """dS/dt of eq. ES per cell: (q_w - sum_d (F_+ - F_-) / h_d) / phi, with
    F = f_w(S_upstream) v on the faces of axis d; h one spacing or (hx, hy, hz)."""
    s = np.asarray(s, dtype=np.float64)
    hx, hy, hz = _spacings(h)
    fw = frac_flow(s)
    div = np.zeros(s.shape)
    for axis, v, hd in ((2, vx, hx), (1, vy, hy), (0, vz, hz)):
        v = np.asarray(v, dtype=np.float64).reshape(s.shape)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, -1)
        hi[axis] = slice(1, None)
        lo, hi = tuple(lo), tuple(hi)
        # water flux through the + face of each cell: upstream f_w times v
        up = np.where(v[lo] >= 0.0, fw[lo], fw[hi])
        fplus = np.zeros(s.shape)
        fplus[lo] = up * v[lo]
        fminus = np.zeros(s.shape)                # the - face is the + face of the lower cell
        fminus[hi] = fplus[lo]
        div += (fplus - fminus) / hd
    return (water_source(q, s) - div) / np.asarray(phi, dtype=np.float64)


def transport(phi, q, vx, vy, vz, s0, h, substeps, ds_max):
    """M explicit sub-steps of eq. ES; returns (S after them, total time)."""
    s = np.array(s0, dtype=np.float64, copy=True)
    t = 0.0
    for _ in range(substeps):
        r = saturation_rate(phi, q, vx, vy, vz, s, h)
        rmax = float(np.max(np.abs(r)))
        dt = ds_max / rmax if rmax > 0.0 else 0.0
        s = s + dt * r
        t += dt
    return s, t


def pressure_solve(perm_eff, grid: Grid, q):
    """Zero-mean solution of A p = q for the TPFA matrix of perm_eff (eq. IMP).

    A is singular with the constants as its null space (no-flow boundary,
    connected grid); fixing p_0 = 0 leaves a nonsingular system, and the
    mean is removed afterwards.
    """
    A = assemble(perm_eff, grid).tocsc()
    q = np.asarray(q, dtype=np.float64).reshape(-1)
    p = np.zeros(grid.n)
    p[1:] = spla.spsolve(A[1:, 1:], q[1:])
    return p - p.mean()


def impes(perm, phi, q, s0, grid: Grid, steps, substeps, ds_max):
    """Improved IMPES (eqs. IMP, ES): returns (S, p, per-step total times)."""
    s = np.array(s0, dtype=np.float64, copy=True).reshape(grid.shape)
    perm = np.asarray(perm, dtype=np.float64).reshape(grid.shape)
    p = None
    times = []
    for _ in range(steps):
        keff = perm * total_mobility(s)
        p = pressure_solve(keff, grid, q)
        vx, vy, vz = recover_flux(keff, grid, p)
        s, t = transport(phi, np.asarray(q).reshape(grid.shape), vx, vy, vz, s, (grid.hx, grid.hy, grid.hz),
                         substeps, ds_max)
        times.append(t)
    return s, p, times
