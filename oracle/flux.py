"""Oracle: velocity recovery and the cell mass balance, FP64.

TEST INFRASTRUCTURE ONLY: imported by tests/ only, never by the product path.

Section 2.2: once the pressure system A p = f is solved, the velocity is
recovered as v = M_t^{-1} B^T p.  With the trapezoidal quadrature M_t is
diagonal and the recovered velocity is the two-point flux of eq. (velocity):
on the face between cells i and i+1 of one axis,

    v_{i+1/2} = -kappa_{i+1/2} (p_{i+1} - p_i) / h,
    kappa_{i+1/2} = 2 / (1/kappa_i + 1/kappa_{i+1})   (harmonic mean),

and zero on the no-flow boundary.  Mass conservation on a cell (the 3D
form of the relation printed after eq. (discrete varia)): the face areas
times the jumps of v across the cell equal the cell volume times f,

    h^2 sum_axes (v_{i+1/2} - v_{i-1/2}) = h^3 f_i.

Arrays are (nz, ny, nx) in C order, as in the assembly module; each face
array holds the flux through the +x (+y, +z) face of every cell.
"""
from __future__ import annotations

import numpy as np

from .assembly import Grid


def recover_flux(perm: np.ndarray, grid: Grid, p) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(vx, vy, vz), each (nz, ny, nx): the flux through each cell's + face.

    `perm` is isotropic (nz, ny, nx) or orthotropic (3, nz, ny, nx) holding
    kappa^x, kappa^y, kappa^z (Section 2.1): the faces of one axis take the
    harmonic mean of that axis's component, K being diagonal."""
    perm = np.asarray(perm, dtype=np.float64)
    comps = perm.reshape((3,) + grid.shape) if perm.size == 3 * grid.n else None
    p = np.asarray(p, dtype=np.float64).reshape(grid.shape)
    out = []
    for comp, (axis, h) in enumerate(((2, grid.hx), (1, grid.hy), (0, grid.hz))):
        kappa = comps[comp] if comps is not None else perm.reshape(grid.shape)
        v = np.zeros(grid.shape)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, -1)
        hi[axis] = slice(1, None)
        lo, hi = tuple(lo), tuple(hi)
        kf = 2.0 / (1.0 / kappa[lo] + 1.0 / kappa[hi])
        v[lo] = -kf * (p[hi] - p[lo]) / h
        out.append(v)
    return out[0], out[1], out[2]


def mass_balance(grid: Grid, vx, vy, vz, f) -> np.ndarray:
    """Per cell: (sum over faces of area x outward flux) / volume - f."""
    f = np.asarray(f, dtype=np.float64).reshape(grid.shape)
    net = np.zeros(grid.shape)
    for axis, v, area in ((2, vx, grid.hy * grid.hz), (1, vy, grid.hx * grid.hz), (0, vz, grid.hx * grid.hy)):
        v = np.asarray(v).reshape(grid.shape)
        vm = np.zeros(grid.shape)               # flux through the - face: the + face of the lower cell
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, -1)
        hi[axis] = slice(1, None)
        vm[tuple(hi)] = v[tuple(lo)]
        net += area * (v - vm)
    return (net / (grid.hx * grid.hy * grid.hz) - f).reshape(-1)
