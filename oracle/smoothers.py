"""Block-Jacobi smoothers with incomplete Cholesky blocks (paper Section 5).

The fine smoother M is one block-Jacobi sweep whose blocks are the coarse
elements; the level-l smoother uses the level-(l+1) elements as blocks.  The
paper factors the blocks by incomplete Cholesky rather than full Cholesky.

Fine level: each block is the principal submatrix A_bb of A (its diagonal
keeps the faces leading out of the block).  IC(0) in the block's local
lexicographic order writes A_bb ~ M_b = (D + L) D^{-1} (D + L^T), where L is
the strictly lower part of A_bb and the pivots follow
    d_i = a_ii - sum_{j < i, a_ij != 0} a_ij^2 / d_j.
For a 7-point stencil this is exactly zero-fill incomplete Cholesky: two
grid neighbours never share a third neighbour, so no fill entry ever lands on
the matrix pattern.

Coarse levels: the same construction with dense blocks, one per child
element, on the block 7-point pattern of A_l:
    D_I = A_II - sum_{J < I neighbour} A_IJ D_J^{-1} A_JI.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .assembly import Grid, element_cells


def _lower_upper_neighbours(s: int):
    """Local lexicographic neighbours in an s^3 block: for each local cell a
    list of (neighbour, is_lower) pairs."""
    nb = []
    for k in range(s):
        for j in range(s):
            for i in range(s):
                me = i + s * (j + s * k)
                lst = []
                for (di, dj, dk) in ((-1, 0, 0), (0, -1, 0), (0, 0, -1), (1, 0, 0), (0, 1, 0), (0, 0, 1)):
                    ii, jj, kk = i + di, j + dj, k + dk
                    if 0 <= ii < s and 0 <= jj < s and 0 <= kk < s:
                        o = ii + s * (jj + s * kk)
                        lst.append((o, o < me))
                nb.append(lst)
    return nb


class FineIC:
    """M^{-1} for the fine level: IC(0) on every sub^3 block of A."""

    def __init__(self, A: sp.csr_matrix, grid: Grid, sub: int):
        A = A.tocsr()
        self.cells = element_cells(grid, (sub, sub, sub))      # (m, s^3)
        s3 = sub ** 3
        self.nb = _lower_upper_neighbours(sub)
        m = self.cells.shape[0]
        diag = A.diagonal()
        self.diag = diag[self.cells]                             # (m, s^3)
        # a_ij for every local pair of neighbours, vectorised over blocks
        self.coef = {}
        for i in range(s3):
            for (j, _) in self.nb[i]:
                if (j, i) in self.coef:
                    self.coef[(i, j)] = self.coef[(j, i)]
                else:
                    self.coef[(i, j)] = np.asarray(A[self.cells[:, i], self.cells[:, j]]).reshape(m)
        d = np.zeros((m, s3))
        for i in range(s3):
            acc = self.diag[:, i].copy()
            for (j, low) in self.nb[i]:
                if low:
                    acc -= self.coef[(i, j)] ** 2 / d[:, j]
            d[:, i] = acc
        if np.any(d <= 0.0):
            raise np.linalg.LinAlgError("IC(0) pivot is not positive")
        self.d = d
        self.s3 = s3

    def apply(self, r: np.ndarray) -> np.ndarray:
        """z = M^{-1} r = (D + L^T)^{-1} D (D + L)^{-1} r, block by block."""
        rb = r[self.cells]
        y = np.zeros_like(rb)
        for i in range(self.s3):
            acc = rb[:, i].copy()
            for (j, low) in self.nb[i]:
                if low:
                    acc -= self.coef[(i, j)] * y[:, j]
            y[:, i] = acc / self.d[:, i]
        z = np.zeros_like(rb)
        for i in range(self.s3 - 1, -1, -1):
            acc = np.zeros(rb.shape[0])
            for (j, low) in self.nb[i]:
                if not low:
                    acc += self.coef[(i, j)] * z[:, j]
            z[:, i] = y[:, i] - acc / self.d[:, i]
        out = np.empty_like(r)
        out[self.cells] = z
        return out

    def dense_blocks(self):
        """M_b for every block as dense matrices (tests on tiny grids)."""
        m = self.cells.shape[0]
        out = []
        for b in range(m):
            dmat = np.diag(self.d[b])
            low = np.zeros((self.s3, self.s3))
            for i in range(self.s3):
                for (j, is_low) in self.nb[i]:
                    if is_low:
                        low[i, j] = self.coef[(i, j)][b]
            out.append((dmat + low) @ np.diag(1.0 / self.d[b]) @ (dmat + low.T))
        return out


class CoarseBlockIC:
    """M_l^{-1} for a coarse level: block IC(0) over each parent element.

    `kids` lists, for every parent (level l+1) element, its children (level-l
    elements) in lexicographic order; `agg` is the number of children per
    axis.  `offsets` gives the first level-l DoF of every level-l element.
    """

    def __init__(self, A: sp.csr_matrix, offsets: np.ndarray, kids: np.ndarray, agg: int):
        A = A.tocsr()
        self.offsets = offsets
        self.kids = kids
        self.agg = agg
        self.dofs = [np.arange(offsets[c], offsets[c + 1]) for c in range(len(offsets) - 1)]
        na = agg ** 3
        self.lower = []
        self.upper = []
        for p in range(na):
            px, py, pz = p % agg, (p // agg) % agg, p // (agg * agg)
            lo, up = [], []
            if px > 0:
                lo.append(p - 1)
            if py > 0:
                lo.append(p - agg)
            if pz > 0:
                lo.append(p - agg * agg)
            if px < agg - 1:
                up.append(p + 1)
            if py < agg - 1:
                up.append(p + agg)
            if pz < agg - 1:
                up.append(p + agg * agg)
            self.lower.append(lo)
            self.upper.append(up)
        self.blk = {}
        self.chol = {}
        for E in range(kids.shape[0]):
            for p in range(na):
                c = kids[E, p]
                dc = self.dofs[c]
                piv = A[dc][:, dc].toarray()
                for q in self.lower[p]:
                    cq = kids[E, q]
                    a_cq = A[dc][:, self.dofs[cq]].toarray()
                    self.blk[(c, cq)] = a_cq
                    self.blk[(cq, c)] = a_cq.T
                    piv = piv - a_cq @ sla.cho_solve(self.chol[cq], a_cq.T)
                self.chol[c] = sla.cho_factor(piv, lower=True)

    def apply(self, r: np.ndarray) -> np.ndarray:
        """Block forward then backward substitution with the block pivots."""
        out = np.zeros_like(r)
        na = self.agg ** 3
        for E in range(self.kids.shape[0]):
            y = {}
            for p in range(na):
                c = self.kids[E, p]
                acc = r[self.dofs[c]].copy()
                for q in self.lower[p]:
                    cq = self.kids[E, q]
                    acc -= self.blk[(c, cq)] @ y[cq]
                y[c] = sla.cho_solve(self.chol[c], acc)
            z = {}
            for p in range(na - 1, -1, -1):
                c = self.kids[E, p]
                acc = np.zeros(len(self.dofs[c]))
                for q in self.upper[p]:
                    cq = self.kids[E, q]
                    acc += self.blk[(c, cq)] @ z[cq]
                z[c] = y[c] - sla.cho_solve(self.chol[c], acc)
                out[self.dofs[c]] = z[c]
        return out
