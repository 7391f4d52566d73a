"""Fine-scale discretisation (paper Section 2.2).

Velocity elimination with the trapezoidal rule turns the lowest-order
Raviart-Thomas system into A p = f with A = B M_t^{-1} B^T (eq. p).  On a
Cartesian grid its variational form is eq. (discrete varia): a sum over the
interior faces e of kappa~_e [p]_e [q]_e, where kappa~ = kappa / h^2 per
direction (the normalisation right after eq. velocity) and the face value is
the harmonic average 2 / (1/kappa~_left + 1/kappa~_right) of the two cells'
values for that direction (fig. kappa edge).  No-flow boundaries contribute
nothing.  The paper writes this in 2D; in 3D the z-faces enter the same way.

The weight of the local spectral problems (eq. spepb) is the trace of the
normalised permeability, one value per cell: S = kappa~x + kappa~y + kappa~z.
The cell volume cancels on both sides, as noted under eq. discrete varia.

Arrays are (nz, ny, nx) in C order: flat index i + nx*(j + ny*k).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    nz: int
    hx: float
    hy: float
    hz: float

    @staticmethod
    def unit_cube(nx: int, ny: int | None = None, nz: int | None = None) -> "Grid":
        """(0,1)^3 meshed uniformly (Section 5): h = 1/N per axis."""
        ny = nx if ny is None else ny
        nz = nx if nz is None else nz
        return Grid(nx, ny, nz, 1.0 / nx, 1.0 / ny, 1.0 / nz)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


def normalized_perm(perm: np.ndarray, grid: Grid) -> np.ndarray:
    """kappa~_d = kappa_d / h_d^2 for d = x, y, z; returns shape (3, nz, ny, nx).

    `perm` is either isotropic (nz, ny, nx) or orthotropic (3, nz, ny, nx)
    holding kappa^x, kappa^y, kappa^z (Section 2.1).
    """
    perm = np.asarray(perm, dtype=np.float64)
    if perm.shape == grid.shape:
        perm = np.broadcast_to(perm, (3,) + grid.shape)
    if perm.shape != (3,) + grid.shape:
        raise ValueError(f"perm shape {perm.shape} does not match grid {grid.shape}")
    h2 = np.array([grid.hx ** 2, grid.hy ** 2, grid.hz ** 2]).reshape(3, 1, 1, 1)
    return perm / h2


def transmissibilities(perm: np.ndarray, grid: Grid):
    """Face coefficients kappa~_{i+1/2} as harmonic averages (fig. kappa edge).

    Returns (tx, ty, tz) with shapes (nz,ny,nx-1), (nz,ny-1,nx), (nz-1,ny,nx):
    tx[k,j,i] couples cells (i,j,k) and (i+1,j,k), etc.  Boundary faces carry
    no coefficient (no-flow condition, eq. ell2).
    """
    kt = normalized_perm(perm, grid)
    kx, ky, kz = kt[0], kt[1], kt[2]
    tx = 2.0 / (1.0 / kx[:, :, :-1] + 1.0 / kx[:, :, 1:])
    ty = 2.0 / (1.0 / ky[:, :-1, :] + 1.0 / ky[:, 1:, :])
    tz = 2.0 / (1.0 / kz[:-1, :, :] + 1.0 / kz[1:, :, :])
    return tx, ty, tz


def weight_diag(perm: np.ndarray, grid: Grid) -> np.ndarray:
    """Diagonal of the right-hand form of eq. spepb: tr(kappa~) per cell (flat)."""
    kt = normalized_perm(perm, grid)
    return (kt[0] + kt[1] + kt[2]).reshape(-1)


def _faces(grid: Grid, tx, ty, tz, elem=None):
    """Flat (left, right, coefficient) triples of the kept interior faces.

    With `elem` = (ex, ey, ez) only faces whose two cells lie in the same
    element of that size are kept (the edge set E_h^0(K) of eq. spepb).
    """
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    idx = np.arange(grid.n).reshape(grid.shape)
    out = []
    for axis, t in ((2, tx), (1, ty), (0, tz)):
        sl_l = [slice(None)] * 3
        sl_r = [slice(None)] * 3
        sl_l[axis] = slice(0, -1)
        sl_r[axis] = slice(1, None)
        left = idx[tuple(sl_l)]
        right = idx[tuple(sl_r)]
        coef = t
        if elem is not None:
            e = {2: elem[0], 1: elem[1], 0: elem[2]}[axis]
            m = {2: nx, 1: ny, 0: nz}[axis]
            keep1d = ((np.arange(m - 1) + 1) % e) != 0
            shape = [1, 1, 1]
            shape[axis] = m - 1
            keep = np.broadcast_to(keep1d.reshape(shape), left.shape)
            left, right, coef = left[keep], right[keep], coef[keep]
        out.append((left.reshape(-1), right.reshape(-1), np.asarray(coef).reshape(-1)))
    left = np.concatenate([o[0] for o in out])
    right = np.concatenate([o[1] for o in out])
    coef = np.concatenate([o[2] for o in out])
    return left, right, coef


def _from_faces(n, left, right, coef) -> sp.csr_matrix:
    """sum over faces of coef * (e_l - e_r)(e_l - e_r)^T as a CSR matrix."""
    rows = np.concatenate([left, right, left, right])
    cols = np.concatenate([left, right, right, left])
    vals = np.concatenate([coef, coef, -coef, -coef])
    a = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    a.sum_duplicates()
    return a


def assemble(perm: np.ndarray, grid: Grid) -> sp.csr_matrix:
    """The symmetric positive semidefinite TPFA matrix A of eq. p."""
    tx, ty, tz = transmissibilities(perm, grid)
    return _from_faces(grid.n, *_faces(grid, tx, ty, tz))


def neumann_local(perm: np.ndarray, grid: Grid, elem) -> sp.csr_matrix:
    """Left-hand operator of eq. spepb on every element of size `elem` at once.

    Only faces interior to an element are summed, so the result is block
    diagonal over the elements, each block being that element's A_i.
    """
    tx, ty, tz = transmissibilities(perm, grid)
    return _from_faces(grid.n, *_faces(grid, tx, ty, tz, elem=elem))


def element_cells(grid: Grid, elem) -> np.ndarray:
    """Flat fine-cell indices of every element, shape (m, ex*ey*ez).

    Elements are numbered lexicographically (x fastest) and the cells inside
    an element are listed in local lexicographic order (x fastest).
    """
    ex, ey, ez = elem
    mx, my, mz = grid.nx // ex, grid.ny // ey, grid.nz // ez
    if mx * ex != grid.nx or my * ey != grid.ny or mz * ez != grid.nz:
        raise ValueError("grid not divisible by the element size")
    idx = np.arange(grid.n).reshape(grid.nz, grid.ny, grid.nx)
    blocks = idx.reshape(mz, ez, my, ey, mx, ex).transpose(0, 2, 4, 1, 3, 5)
    return blocks.reshape(mx * my * mz, ex * ey * ez)
