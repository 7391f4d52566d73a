"""Nested multiscale spaces W_L in ... in W_1 = W_h (paper Section 3).

Level 1 is the fine grid.  Level 2 elements are `sub`^3 fine cells (the
coarse grid T_c); each coarser level groups `agg`^3 elements of the level
below (T_cc and beyond).

* Level 2 (eq. spepb): on every element K solve the generalized problem
  A_K phi = lambda S_K phi, where A_K sums the face terms of eq. discrete varia
  over the faces interior to K and S_K = diag(tr kappa~).  The eigenvectors of
  the smallest eigenvalues, normalised w.r.t. S_K (LAPACK returns them so),
  are the rows of R_c.
* Level l+1 >= 3 (eq. spectral cc): the same two bilinear forms, restricted
  to W_l on the level-(l+1) element E: with B_E the fine-space basis of W_l
  on E, solve (B_E^T A_E B_E) v = lambda (B_E^T S_E B_E) v.  The right-hand
  Gram is the identity when the lower level is S-normalised (noted below
  eq. spectral cc); the oracle forms it anyway and records its distance to I.
  The eigenvectors are the rows of R_{l+1}; the fine-space basis of W_{l+1}
  is P_{l+1} = P_l R_{l+1}^T.
* Galerkin chain: A_{l+1} = R_{l+1} A_l R_{l+1}^T (text above Algorithm 1).

How many eigenvectors to keep (strategy 1 of Section 5 with a fixed target
count L) is decided by `cluster_cut`, which never splits a cluster of equal
eigenvalues; the paper picks its counts 4, 8, 11, 17 from the same concern
(the Laplace eigenvalue ladder of Section 5.2).  Levels >= 3 may use their
own count L_cc, and strategy 2 of Section 5 (keep the eigenvalues below a
threshold B_cc, out of L_cc candidates) through `threshold_target`.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .assembly import Grid, assemble, neumann_local, weight_diag, element_cells

CLUSTER_RTOL = 1.0e-6
CLUSTER_FLOOR = 1.0e-12
CLUSTER_EXTRA = 3


def cluster_cut(lam, target: int, extra: int = CLUSTER_EXTRA, rtol: float = CLUSTER_RTOL,
                floor: float = CLUSTER_FLOOR) -> int:
    """Number of eigenvectors to keep for a target count `target`.

    `lam` holds ascending eigenvalues lambda_0 <= lambda_1 <= ..., at least up
    to index target+extra when the element has that many.  lambda_k and
    lambda_{k-1} count as equal when lambda_k - lambda_{k-1} <= rtol *
    max(|lambda_k|, floor).  If the cut at `target` falls inside a cluster of
    equal values, the kept set grows to the end of the cluster, up to
    target+extra vectors; when the cluster runs past that cap, the kept set
    shrinks instead to end before the cluster (never below one vector).
    """
    lam = np.asarray(lam, dtype=np.float64)
    n = lam.shape[0]
    if target >= n:
        return n

    def same(k):
        return lam[k] - lam[k - 1] <= rtol * max(abs(lam[k]), floor)

    k = target
    cap = min(target + extra, n)
    while k < cap and same(k):
        k += 1
    if k == cap and k < n and same(k):
        k = target
        while k > 1 and same(k):
            k -= 1
    return k


def threshold_target(lam, target: int, threshold: float) -> int:
    """Target count under strategy 2 of Section 5: the number of eigenvalues
    below the threshold B, at least one (the constant function) and at most
    `target` (the number of candidates kept per element).  A threshold <= 0
    selects strategy 1, the fixed count `target`.  The cluster rule is applied
    to the result afterwards."""
    if threshold <= 0:
        return target
    below = int(np.sum(np.asarray(lam, dtype=np.float64) < threshold))
    return max(1, min(target, below))


# ----------------------------------------------------------------------------
# the many small dense eigenproblems, spread over worker processes


def _dense(x):
    """Dense matrix from a payload: ndarray, 1-D diagonal, or CSR triple."""
    if isinstance(x, tuple):
        data, indices, indptr, shape = x
        return sp.csr_matrix((data, indices, indptr), shape=shape).toarray()
    x = np.asarray(x)
    return np.diag(x) if x.ndim == 1 else x


def _eig_chunk(args):
    """Lowest `top`+1 eigenpairs of every (A, B) pencil of a chunk."""
    from threadpoolctl import threadpool_limits
    lo, items, top = args
    out = []
    with threadpool_limits(1):
        for a, b in items:
            a = _dense(a)
            b = _dense(b)
            t = min(a.shape[0] - 1, top)
            out.append(sla.eigh(a, b, subset_by_index=[0, t]))
    return lo, out


def _payload(m):
    m = sp.csr_matrix(m)
    return (m.data, m.indices, m.indptr, m.shape)


def _solve_all(m: int, get, target: int, extra: int, workers: int):
    """scipy.linalg.eigh on all m pencils (A_e, B_e) = get(e); keeps the
    lowest target+extra+1 eigenpairs of each."""
    top = target + extra
    step = max(1, min(64, m // max(1, 4 * workers)))
    chunks = [(lo, [get(e) for e in range(lo, min(m, lo + step))], top)
              for lo in range(0, m, step)]
    results = [None] * m
    if workers > 1 and len(chunks) > 1 and m >= 128:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(min(workers, len(chunks))) as pool:
            for lo, out in pool.imap_unordered(_eig_chunk, chunks):
                results[lo:lo + len(out)] = out
    else:
        for c in chunks:
            lo, out = _eig_chunk(c)
            results[lo:lo + len(out)] = out
    return results


@dataclass
class Level:
    """One coarse level l >= 2 of the hierarchy."""
    index: int                      # l
    elem: tuple                     # element size in fine cells (ex, ey, ez)
    egrid: tuple                    # number of elements per axis (mx, my, mz)
    nkeep: np.ndarray               # kept eigenvectors per element
    lam: list                       # computed eigenvalues per element (ascending)
    offsets: np.ndarray             # first DoF of each element (len m+1)
    R: sp.csr_matrix                # restriction from level l-1 (level 1 = fine)
    P: sp.csc_matrix                # fine-space basis of W_l (n x n_l)
    A: sp.csr_matrix                # Galerkin operator A_l
    gram_err: float = 0.0           # max |B^T S B - I| seen on this level

    @property
    def m(self) -> int:
        return int(np.prod(self.egrid))

    @property
    def dim(self) -> int:
        return int(self.offsets[-1])


@dataclass
class Hierarchy:
    grid: Grid
    sub: int
    agg: int
    nlevels: int
    target: int
    A: sp.csr_matrix                # fine operator (level 1)
    S: np.ndarray                   # fine weight diag(tr kappa~)
    levels: list = field(default_factory=list)   # levels[0] is level 2

    def level(self, l: int) -> Level:
        return self.levels[l - 2]


def _children(egrid_parent, agg, egrid_child):
    """Child element indices of every parent element, children listed
    lexicographically (x fastest) inside the parent; shape (M, agg^3)."""
    mx, my, mz = egrid_child
    idx = np.arange(mx * my * mz).reshape(mz, my, mx)
    px, py, pz = egrid_parent
    blocks = idx.reshape(pz, agg, py, agg, px, agg).transpose(0, 2, 4, 1, 3, 5)
    return blocks.reshape(px * py * pz, agg ** 3)


def build_hierarchy(perm, grid: Grid, nlevels: int, target: int, sub: int = 8, agg: int = 4,
                    workers: int | None = None, A=None, target_cc: int | None = None,
                    threshold_cc: float = 0.0, threshold_c: float = 0.0) -> Hierarchy:
    """Set-up phase: local spectral problems and the Galerkin chain.

    `target` is the count per level-2 element (L_c of Section 5); levels >= 3
    use `target_cc` (L_cc, default `target`).  Strategy 2 of Section 5: when
    `threshold_c` > 0 the level-2 elements keep only the eigenvalues below it
    (B_c) out of `target` candidates, and when `threshold_cc` > 0 the coarser
    elements those below B_cc out of `target_cc` candidates."""
    if nlevels < 2:
        raise ValueError("need at least two levels")
    if target_cc is None:
        target_cc = target
    if workers is None:
        workers = os.cpu_count() or 1
    if A is None:
        A = assemble(perm, grid)
    S = weight_diag(perm, grid)
    hier = Hierarchy(grid, sub, agg, nlevels, target, A, S)

    # ---- level 2: eq. spepb on every sub^3 element
    elem = (sub, sub, sub)
    cells = element_cells(grid, elem)
    m2 = cells.shape[0]
    aloc = neumann_local(perm, grid, elem).tocsr()

    def get2(e):
        c = cells[e]
        return _payload(aloc[c][:, c]), S[c]

    res = _solve_all(m2, get2, target, CLUSTER_EXTRA, workers)
    nkeep = np.array([cluster_cut(w, threshold_target(w, target, threshold_c)) for (w, _) in res],
                     dtype=np.int64)
    offsets = np.concatenate([[0], np.cumsum(nkeep)])
    rows, cols, vals = [], [], []
    for e, (w, v) in enumerate(res):
        k = nkeep[e]
        c = cells[e]
        for j in range(k):
            rows.append(np.full(c.shape[0], offsets[e] + j))
            cols.append(c)
            vals.append(v[:, j])
    n2 = int(offsets[-1])
    R2 = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                       shape=(n2, grid.n))
    gerr = 0.0
    for e, (w, v) in enumerate(res):
        phi = v[:, :nkeep[e]]
        g = phi.T @ (S[cells[e]][:, None] * phi)
        gerr = max(gerr, float(np.max(np.abs(g - np.eye(g.shape[0])))))
    P2 = R2.T.tocsc()
    A2 = (R2 @ A @ R2.T).tocsr()
    egrid = (grid.nx // sub, grid.ny // sub, grid.nz // sub)
    hier.levels.append(Level(2, elem, egrid, nkeep, [w for (w, _) in res], offsets, R2, P2, A2,
                             gerr))

    # ---- levels 3..L: eq. spectral cc restricted to W_l
    for l in range(2, nlevels):
        low = hier.level(l)
        elem_up = tuple(e * agg for e in low.elem)
        egrid_up = tuple(g // agg for g in low.egrid)
        if any(g * agg != h for g, h in zip(egrid_up, low.egrid)) or min(egrid_up) < 1:
            raise ValueError("element grid not divisible by agg")
        kids = _children(egrid_up, agg, low.egrid)
        an = neumann_local(perm, grid, elem_up)
        h_all = (low.P.T @ an @ low.P).tocsr()
        g_all = (low.P.T @ sp.diags(S) @ low.P).tocsr()
        dofs = [np.concatenate([np.arange(low.offsets[c], low.offsets[c + 1]) for c in kid])
                for kid in kids]

        def getl(e, h_all=h_all, g_all=g_all, dofs=dofs):
            d = dofs[e]
            return _payload(h_all[d][:, d]), _payload(g_all[d][:, d])

        mup = kids.shape[0]
        res = _solve_all(mup, getl, target_cc, CLUSTER_EXTRA, workers)
        gerr = 0.0
        for e in range(mup):
            g = _dense(getl(e)[1])
            gerr = max(gerr, float(np.max(np.abs(g - np.eye(g.shape[0])))))
        nk = np.array([cluster_cut(w, threshold_target(w, target_cc, threshold_cc)) for (w, _) in res],
                      dtype=np.int64)
        offs = np.concatenate([[0], np.cumsum(nk)])
        rows, cols, vals = [], [], []
        for e, (w, v) in enumerate(res):
            for j in range(nk[e]):
                rows.append(np.full(dofs[e].shape[0], offs[e] + j))
                cols.append(dofs[e])
                vals.append(v[:, j])
        nup = int(offs[-1])
        R = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(nup, low.dim))
        P = (low.P @ R.T).tocsc()
        Al = (R @ low.A @ R.T).tocsr()
        hier.levels.append(Level(l + 1, elem_up, egrid_up, nk, [w for (w, _) in res], offs, R, P,
                                 Al, gerr))
    return hier
