"""Algorithm 1 of the paper, applied recursively over the levels.

One application of the preconditioner to a residual f (zero initial guess):

  1. pre-smooth        u1 = M^{-1} f
  2. restrict          r_c = R_c (f - A u1)
  3.-7. coarse map     e_c = B_c^{-1} r_c   (the same steps one level down;
                       at the coarsest level e = A_L^+ r, the pseudo-inverse)
  8. prolong           u2 = u1 + R_c^T e_c
  9. post-smooth       u* = u2 + M^{-T} (f - A u2)

With two levels this is the exact two-grid preconditioner P_TG (eq. B_TG);
with three it is Algorithm 1 itself, whose inner map is eq. B_c; deeper
hierarchies nest eq. B_c once per extra level.  The smoothers are symmetric,
so M^{-T} = M^{-1}.  nu > 1 repeats the block-Jacobi sweep u += M^{-1}(f - A u).
"""
from __future__ import annotations

import numpy as np

from .smoothers import FineIC, CoarseBlockIC
from .spectral import Hierarchy, _children


def pseudo_inverse(a: np.ndarray) -> np.ndarray:
    """Moore-Penrose inverse of the symmetric coarsest operator.

    The fine operator's kernel is the constants (no-flow boundary, connected
    grid, positive permeability), and the constants lie in every coarse space
    (the paragraph after eq. spectral cc), so A_L has exactly one zero
    eigenvalue.  The pseudo-inverse inverts every other eigenvalue.
    """
    w, q = np.linalg.eigh(a)
    null = int(np.argmin(np.abs(w)))
    keep = np.ones(w.shape[0], dtype=bool)
    keep[null] = False
    return (q[:, keep] / w[keep]) @ q[:, keep].T


class MinNormSolve:
    """The same map as `pseudo_inverse`, e = A_L^+ r, for coarsest spaces too
    large for a dense eigendecomposition: the minimum-norm solution of
    A_L e = r on the range of A_L.

    The kernel of A_L is spanned by z, the coarse coefficients of the
    constant function (the paragraph after eq. spectral cc).  The right-hand
    side is projected onto z's complement, one unknown i0 (the largest |z_i|)
    is fixed at zero and the remaining equations are solved by sparse LU; the
    dropped equation holds by itself because z^T (A_L e - r) = 0 and
    z_i0 != 0.  Removing the component along z gives the solution orthogonal
    to the kernel, which is A_L^+ r.
    """

    def __init__(self, a, z: np.ndarray):
        import scipy.sparse as sp
        import scipy.sparse.linalg as spla
        self.z = z / np.linalg.norm(z)
        self.i0 = int(np.argmax(np.abs(self.z)))
        keep = np.ones(a.shape[0], dtype=bool)
        keep[self.i0] = False
        self.keep = keep
        self.lu = spla.splu(sp.csc_matrix(a)[keep][:, keep].tocsc())

    def __matmul__(self, r: np.ndarray) -> np.ndarray:
        rp = r - (self.z @ r) * self.z
        e = np.zeros_like(rp)
        e[self.keep] = self.lu.solve(rp[self.keep])
        return e - (self.z @ e) * self.z


class Preconditioner:
    """P^{-1} r for a hierarchy built by `build_hierarchy`.

    `coarsest` selects how the coarsest map A_L^+ is formed: "pinv" (dense
    eigendecomposition, `pseudo_inverse`) or "minnorm" (sparse LU on the
    range, `MinNormSolve`, for coarsest spaces of thousands of unknowns).
    Both give the Moore-Penrose inverse."""

    def __init__(self, hier: Hierarchy, nu: int = 1, nu_c: int | None = None, coarsest: str = "pinv"):
        # nu sweeps on the fine level, nu_c on the coarse levels (Section 5
        # names both; nu_c defaults to nu)
        self.h = hier
        self.nu = nu
        self.nu_c = nu if nu_c is None else nu_c
        self.fine = FineIC(hier.A, hier.grid, hier.sub)
        self.coarse = {}
        for l in range(2, hier.nlevels):
            low, up = hier.level(l), hier.level(l + 1)
            kids = _children(up.egrid, hier.agg, low.egrid)
            self.coarse[l] = CoarseBlockIC(low.A, low.offsets, kids, hier.agg)
        top = hier.level(hier.nlevels)
        if coarsest == "pinv":
            self.pinv = pseudo_inverse(top.A.toarray())
        elif coarsest == "minnorm":
            # coefficients of the constant function in the S-orthonormal basis P_L
            z = top.P.T @ hier.S
            self.pinv = MinNormSolve(top.A, np.asarray(z).ravel())
        else:
            raise ValueError(f"unknown coarsest solve {coarsest!r}")

    def _smooth(self, l, A, f, u=None):
        sm = self.fine if l == 1 else self.coarse[l]
        for it in range(self.nu if l == 1 else self.nu_c):
            if u is None:
                u = sm.apply(f)
            else:
                u = u + sm.apply(f - A @ u)
        return u

    def _op(self, l):
        return self.h.A if l == 1 else self.h.level(l).A

    def level_apply(self, l: int, f: np.ndarray) -> np.ndarray:
        """The map f -> u* of Algorithm 1 at level l (l = 1 is the fine grid)."""
        if l == self.h.nlevels:
            return self.pinv @ f
        A = self._op(l)
        R = self.h.level(l + 1).R
        u1 = self._smooth(l, A, f)
        rc = R @ (f - A @ u1)
        ec = self.level_apply(l + 1, rc)
        u2 = u1 + R.T @ ec
        return self._smooth(l, A, f, u2)

    def apply(self, f: np.ndarray) -> np.ndarray:
        return self.level_apply(1, np.asarray(f, dtype=np.float64))

    def dense(self) -> np.ndarray:
        """P^{-1} column by column (tiny grids only)."""
        n = self.h.A.shape[0]
        out = np.zeros((n, n))
        for j in range(n):
            e = np.zeros(n)
            e[j] = 1.0
            out[:, j] = self.apply(e)
        return out
