"""Pins of the CPU oracle against the paper and the mathematics.

None of these re-types the oracle's own formulas: each checks a closed form,
an invariant the paper states, a textbook special case, or a brute-force
computation by a different algorithm.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import Grid, assemble, build_hierarchy, cluster_cut, threshold_target, Preconditioner, pcg
from oracle.assembly import transmissibilities, normalized_perm, element_cells, neumann_local
from oracle.smoothers import FineIC, CoarseBlockIC
from oracle.spectral import _children
from oracle.vcycle import pseudo_inverse
from synth.fields import make_field, random_zero_mean, corner_source


def _rand_perm(shape, seed, contrast=1e6):
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(-0.5 * math.log(contrast), 0.5 * math.log(contrast), size=shape))


# --------------------------------------------------------------------------
# Section 2.2: the TPFA matrix

def test_constant_kernel_and_symmetry():
    g = Grid.unit_cube(6, 5, 4)
    A = assemble(_rand_perm(g.shape, 1), g)
    one = np.ones(g.n)
    scale = abs(A).sum(axis=1).max()
    assert np.max(np.abs(A @ one)) <= 1e-14 * scale
    assert abs(A - A.T).max() == 0.0
    w = np.linalg.eigvalsh(A.toarray())
    assert w[0] >= -1e-12 * scale
    assert np.sum(w <= 1e-10 * scale) == 1          # connected grid: 1-dim kernel


def test_two_cell_hand_computed():
    # 2 x 1 x 1 cells on (0,1)^3: h_x = 1/2, kappa = (1, 3) -> kappa~ = (4, 12);
    # the face value is 2 / (1/4 + 1/12) = 6, so A = [[6, -6], [-6, 6]].
    g = Grid.unit_cube(2, 1, 1)
    perm = np.array([1.0, 3.0]).reshape(1, 1, 2)
    A = assemble(perm, g).toarray()
    assert np.array_equal(A, np.array([[6.0, -6.0], [-6.0, 6.0]]))


def test_orthotropic_faces_use_their_own_direction():
    # x-faces average kappa^x only, z-faces kappa^z only (fig. kappa edge)
    g = Grid.unit_cube(2, 1, 2)
    kx = np.array([[[1.0, 2.0]], [[1.0, 2.0]]])
    ky = np.full(g.shape, 5.0)
    kz = np.array([[[3.0, 7.0]], [[9.0, 7.0]]])
    tx, ty, tz = transmissibilities(np.stack([kx, ky, kz]), g)
    assert np.allclose(tx[0, 0, 0], 2.0 / (1 / 4.0 + 1 / 8.0))      # h = 1/2
    assert np.allclose(tz[0, 0, 0], 2.0 / (1 / 12.0 + 1 / 36.0))
    assert np.allclose(tz[0, 0, 1], 28.0)


def test_harmonic_mean_bound():
    # Analysis section: every face coefficient is at most twice the smaller
    # cell value, hence at most 2 (kappa~x + kappa~y + ...) of either cell.
    g = Grid.unit_cube(5)
    perm = _rand_perm(g.shape, 3)
    kt = normalized_perm(perm, g)
    tx, ty, tz = transmissibilities(perm, g)
    tr = kt.sum(axis=0)
    assert np.all(tx <= 2 * np.minimum(kt[0][:, :, :-1], kt[0][:, :, 1:]) * (1 + 1e-15))
    assert np.all(tx <= 2 * tr[:, :, :-1])
    assert np.all(tz <= 2 * np.minimum(tr[:-1], tr[1:]) * (1 + 1e-15))


def _manufactured_error(N):
    # p = cos(pi x) cos(pi y) cos(pi z) satisfies the no-flow condition on
    # (0,1)^3 with kappa = 1 and f = 3 pi^2 p (the cell volume cancels, so f is
    # the source density at the cell centres).
    g = Grid.unit_cube(N)
    c = (np.arange(N) + 0.5) / N
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    p = np.cos(np.pi * xx) * np.cos(np.pi * yy) * np.cos(np.pi * zz)
    f = 3 * np.pi ** 2 * p
    f = (f - f.mean()).reshape(-1)
    A = assemble(np.ones(g.shape), g)
    dense = A.toarray()
    x = np.linalg.lstsq(dense, f, rcond=None)[0]
    x -= x.mean()
    pe = p.reshape(-1) - p.mean()
    return np.sqrt(np.mean((x - pe) ** 2))


def test_manufactured_second_order():
    e4, e8, e16 = (_manufactured_error(n) for n in (4, 8, 16))
    assert 3.3 < e4 / e8 < 4.7
    assert 3.6 < e8 / e16 < 4.4


# --------------------------------------------------------------------------
# Section 3: local spectral problems

def _dct_ladder(s):
    mu = 2 - 2 * np.cos(np.arange(s) * np.pi / s)
    return np.sort((mu[:, None, None] + mu[None, :, None] + mu[None, None, :]).reshape(-1) / 3)


def test_homogeneous_block_ladder():
    # Discrete Neumann Laplacian on an 8^3 block, weight 3 kappa~: eigenvalues
    # (mu_i + mu_j + mu_k)/3 with mu_m = 2 - 2 cos(m pi / 8); the multiplicities
    # 1, 3, 3, 1, 3, 6 reproduce the ladder {0,1,1,1,2,2,2,3,4,4,4,5x6} of
    # Section 5.2.
    g = Grid.unit_cube(16)
    h = build_hierarchy(np.ones(g.shape), g, 2, 13, sub=8, workers=1)
    ref = _dct_ladder(8)[:17]
    for lam in h.level(2).lam:
        assert np.allclose(lam[:17], ref, rtol=0, atol=1e-13)
    lad = np.round(ref / ref[1], 6)
    assert list(lad[:8]) == [0, 1, 1, 1, 2, 2, 2, 3]
    counts = np.unique(np.round(ref, 10), return_counts=True)[1][:6]
    assert list(counts) == [1, 3, 3, 1, 3, 6]


def test_homogeneous_span_is_lowest_cosines():
    # clean cut at 4: span{1, cos(pi(x+1/2)/8), same in y, same in z}
    g = Grid.unit_cube(8)
    h = build_hierarchy(np.ones(g.shape), g, 2, 4, sub=8, workers=1)
    lev = h.level(2)
    assert list(lev.nkeep) == [4]
    phi = lev.R.toarray().T                        # 512 x 4
    c = np.cos(np.pi * (np.arange(8) + 0.5) / 8)
    one = np.ones(8)
    modes = [np.einsum("k,j,i->kji", a, b, d).reshape(-1)
             for (a, b, d) in ((one, one, one), (one, one, c), (one, c, one), (c, one, one))]
    Q = np.linalg.qr(np.stack(modes, 1))[0]
    P = np.linalg.qr(phi)[0]
    assert np.linalg.norm(P - Q @ (Q.T @ P), 2) < 1e-12


@pytest.mark.parametrize("kind", ["gauss", "inclusions", "channels"])
def test_zero_eigenvalue_constant_vector(kind):
    # Below eq. spectral cc: the smallest eigenvalue is 0 with a constant
    # eigenvector on every element of every level.
    g = Grid.unit_cube(32)
    perm = make_field(kind, 32, 5)
    h = build_hierarchy(perm, g, 3, 6, sub=8, agg=2, workers=1)
    S = h.S
    for l in (2, 3):
        lev = h.level(l)
        for e in range(lev.m):
            assert abs(lev.lam[e][0]) < 1e-12
            assert lev.lam[e][1] > 1e-12
        # the first basis function of each element is the constant there
        P = lev.P.tocsc()
        for e in range(lev.m):
            col = P[:, lev.offsets[e]].toarray().ravel()
            sup = col != 0
            v = col[sup]
            # first-order perturbation: rounding of size ~n eps ||H|| moves the
            # eigenvector by at most that over the gap lambda_1
            bound = max(1e-12, 1e-12 / lev.lam[e][1])
            assert np.max(np.abs(v - v[0])) <= bound * abs(v[0])
            assert abs((v * v * S[sup]).sum() - 1.0) < 1e-12


def test_gram_identity_and_constants_in_every_space():
    # S-orthonormal bases make the right-hand Gram of eq. spectral cc the
    # identity (last paragraph of Section 3); constants lie in W_c and W_cc.
    g = Grid.unit_cube(32)
    perm = make_field("gauss", 32, 9)
    h = build_hierarchy(perm, g, 4, 5, sub=4, agg=2, workers=1)
    for l in (2, 3, 4):
        lev = h.level(l)
        assert lev.gram_err < 1e-12
        P = lev.P
        G = (P.T @ sp.diags(h.S) @ P).toarray()
        assert np.max(np.abs(G - np.eye(G.shape[0]))) < 1e-12
        one = np.ones(g.n)
        proj = P @ (P.T @ (h.S * one))
        assert np.max(np.abs(proj - one)) < 1e-10
        assert np.max(np.abs(lev.A @ (P.T @ (h.S * one)))) < 1e-9 * abs(lev.A).max()


def test_galerkin_chain_matches_direct_triple_product():
    # A_cc = R_cc A_c R_cc^T = (R_cc R_c) A (R_cc R_c)^T (text above Alg. 1)
    g = Grid.unit_cube(16)
    perm = make_field("channels", 16, 4)
    h = build_hierarchy(perm, g, 3, 4, sub=4, agg=2, workers=1)
    P3 = h.level(3).P
    direct = (P3.T @ h.A @ P3).toarray()
    chain = h.level(3).A.toarray()
    assert np.max(np.abs(direct - chain)) < 1e-12 * np.max(np.abs(direct))


def test_level3_problem_equals_fine_neumann_form():
    # eq. spectral cc sums over the fine faces interior to K_cc only: the
    # eigenvalues of the level-3 problem equal those of the fine Neumann form
    # restricted to W_c(K_cc), computed here by an explicit dense basis.
    g = Grid.unit_cube(8)
    perm = make_field("gauss", 8, 2)
    h = build_hierarchy(perm, g, 3, 4, sub=4, agg=2, workers=1)
    B = h.level(2).P.toarray()                             # whole domain = 1 level-3 element
    An = neumann_local(perm, g, (8, 8, 8)).toarray()       # all interior faces
    w = sla.eigh(B.T @ An @ B, B.T @ np.diag(h.S) @ B, eigvals_only=True)
    assert np.allclose(h.level(3).lam[0][:6], w[:6], atol=1e-12)


def test_cluster_rule():
    lad = _dct_ladder(8)
    assert cluster_cut(lad, 4) == 4
    assert cluster_cut(lad, 6) == 7            # grows to the end of the cluster {4,5,6}
    assert cluster_cut(lad, 8) == 8
    assert cluster_cut(lad, 10) == 11
    assert cluster_cut(lad, 12) == 11          # 6-fold cluster 11..16 runs past the cap 15
    assert cluster_cut(lad, 1) == 1
    assert cluster_cut(lad, 2) == 4
    assert cluster_cut(np.array([0.0, 1.0]), 5) == 2


# --------------------------------------------------------------------------
# Section 5: smoothers

def _pattern_ic(a, pattern):
    """Textbook incomplete Cholesky restricted to `pattern` (dense, right-looking)."""
    a = a.copy()
    n = a.shape[0]
    L = np.zeros_like(a)
    for k in range(n):
        L[k, k] = math.sqrt(a[k, k])
        for i in range(k + 1, n):
            if pattern[i, k]:
                L[i, k] = a[i, k] / L[k, k]
        for j in range(k + 1, n):
            if L[j, k] == 0:
                continue
            for i in range(j, n):
                if pattern[i, j] and L[i, k] != 0:
                    a[i, j] -= L[i, k] * L[j, k]
                    a[j, i] = a[i, j]
    return L


@pytest.mark.parametrize("sub,n", [(2, 4), (4, 8)])
def test_fine_ic0_equals_pattern_cholesky(sub, n):
    g = Grid.unit_cube(n)
    perm = _rand_perm(g.shape, 11, contrast=1e4)
    A = assemble(perm, g)
    ic = FineIC(A, g, sub)
    cells = element_cells(g, (sub, sub, sub))
    dense = A.toarray()
    for b, M in enumerate(ic.dense_blocks()):
        c = cells[b]
        abb = dense[np.ix_(c, c)]
        L = _pattern_ic(abb, abb != 0)
        assert np.allclose(L @ L.T, M, rtol=1e-12, atol=1e-12 * np.abs(abb).max())
        # IC(0) keeps the diagonal and the pattern of A_bb
        assert np.allclose(np.diag(M), np.diag(abb), rtol=1e-12)
        off = (abb != 0)
        assert np.allclose(M[off], abb[off], rtol=1e-12, atol=1e-12 * np.abs(abb).max())


def test_fine_ic0_apply_is_inverse_of_factor():
    g = Grid.unit_cube(8)
    A = assemble(_rand_perm(g.shape, 12), g)
    ic = FineIC(A, g, 4)
    cells = element_cells(g, (4, 4, 4))
    r = random_zero_mean(g.shape, 3).reshape(-1)
    z = ic.apply(r)
    for b, M in enumerate(ic.dense_blocks()):
        c = cells[b]
        assert np.allclose(M @ z[c], r[c], rtol=1e-10, atol=1e-12 * np.abs(r).max())


def test_coarse_block_ic_equals_pattern_cholesky():
    # Block IC(0) with dense pivots equals scalar IC(0) on the block pattern.
    g = Grid.unit_cube(16)
    perm = make_field("inclusions", 16, 3)
    h = build_hierarchy(perm, g, 3, 3, sub=4, agg=2, workers=1)
    low, up = h.level(2), h.level(3)
    kids = _children(up.egrid, 2, low.egrid)
    bic = CoarseBlockIC(low.A, low.offsets, kids, 2)
    A2 = low.A.toarray()
    for E in range(kids.shape[0]):
        dofs = np.concatenate([np.arange(low.offsets[c], low.offsets[c + 1]) for c in kids[E]])
        owner = np.concatenate([np.full(low.offsets[c + 1] - low.offsets[c], p)
                                for p, c in enumerate(kids[E])])
        sub = A2[np.ix_(dofs, dofs)]
        pos = np.array([[p % 2, (p // 2) % 2, p // 4] for p in range(8)])
        d = np.abs(pos[owner][:, None, :] - pos[owner][None, :, :]).sum(-1)
        pattern = d <= 1
        L = _pattern_ic(sub, pattern)
        M = L @ L.T
        # the oracle's M_c^{-1} restricted to this parent
        n = A2.shape[0]
        Minv = np.zeros((len(dofs), len(dofs)))
        for j, dj in enumerate(dofs):
            e = np.zeros(n)
            e[dj] = 1.0
            Minv[:, j] = bic.apply(e)[dofs]
        assert np.allclose(Minv @ M, np.eye(len(dofs)), atol=1e-9)


def test_pseudo_inverse_penrose():
    g = Grid.unit_cube(8)
    A = assemble(_rand_perm(g.shape, 7, contrast=1e3), g).toarray()
    X = pseudo_inverse(A)
    s = np.abs(A).max()
    assert np.allclose(A @ X @ A, A, atol=1e-9 * s)
    assert np.allclose(X @ A @ X, X, atol=1e-9 * np.abs(X).max())
    assert np.allclose(A @ X, (A @ X).T, atol=1e-10)
    assert np.allclose(X, np.linalg.pinv(A, hermitian=True), atol=1e-8 * np.abs(X).max())


@pytest.mark.parametrize("levels,target,agg", [(2, 4, 2), (3, 2, 2)])
def test_min_norm_coarsest_is_the_pseudo_inverse(levels, target, agg):
    """The sparse minimum-norm coarsest solve is the Moore-Penrose map: its
    output is orthogonal to the kernel of A_L, solves A_L e = r on the range,
    matches the dense pseudo-inverse, and the whole preconditioner built on it
    matches the one built on the dense pseudo-inverse."""
    from oracle.vcycle import MinNormSolve
    g = Grid.unit_cube(16)
    perm = _rand_perm(g.shape, 11, contrast=1e4)
    h = build_hierarchy(perm, g, levels, target, sub=4, agg=agg, workers=1)
    top = h.level(levels)
    A = top.A.toarray()
    z = np.asarray(top.P.T @ h.S).ravel()
    ms = MinNormSolve(top.A, z)
    zn = z / np.linalg.norm(z)
    assert np.linalg.norm(A @ zn) < 1e-10 * np.abs(A).max()   # z spans the kernel
    r = np.random.default_rng(3).standard_normal(A.shape[0])
    e = ms @ r
    rp = r - (zn @ r) * zn
    assert abs(zn @ e) < 1e-12 * np.linalg.norm(e)
    assert np.linalg.norm(A @ e - rp) < 1e-10 * np.linalg.norm(rp)
    ref = np.linalg.pinv(A, hermitian=True) @ r
    assert np.linalg.norm(e - ref) < 1e-9 * np.linalg.norm(ref)
    f = random_zero_mean(g.shape, 4).reshape(-1)
    p1 = Preconditioner(h).apply(f)
    p2 = Preconditioner(h, coarsest="minnorm").apply(f)
    assert np.linalg.norm(p1 - p2) < 1e-9 * np.linalg.norm(p1)


# --------------------------------------------------------------------------
# Algorithm 1 / Section 4: the preconditioner

@pytest.mark.parametrize("levels,target", [(2, 1), (2, 4), (3, 4)])
def test_preconditioner_symmetric_spectrum_in_unit_interval(levels, target):
    g = Grid.unit_cube(8)
    perm = make_field("inclusions", 8, 1, cover=0.2)
    h = build_hierarchy(perm, g, levels, target, sub=2 if levels == 3 else 4, agg=2, workers=1)
    P = Preconditioner(h).dense()
    assert np.max(np.abs(P - P.T)) < 1e-10 * np.abs(P).max()
    A = h.A.toarray()
    # eigenvalues of P^{-1} A on range(A): generalized problem on the
    # complement of the constants
    Q = np.linalg.qr(np.concatenate([np.ones((g.n, 1)), np.eye(g.n)[:, :-1]], 1))[0][:, 1:]
    Ar = Q.T @ A @ Q
    Pr = Q.T @ P @ Q
    w = np.sort(np.linalg.eigvals(Pr @ Ar).real)
    assert w[0] > 0
    assert w[-1] <= 1 + 1e-10
    if levels == 2:
        # Xu-Zikatanov: lambda_max(P_TG^{-1} A) = 1 exactly
        assert abs(w[-1] - 1) < 1e-10


def test_full_coarse_space_is_exact_solver():
    # L = cells per element: R_c is square, the exact two-grid map is A^+ on
    # range(A) and PCG converges in one iteration.
    g = Grid.unit_cube(8)
    perm = make_field("gauss", 8, 3)
    h = build_hierarchy(perm, g, 2, 8, sub=2, workers=1)
    assert h.level(2).dim == g.n
    pre = Preconditioner(h)
    b = random_zero_mean(g.shape, 1).reshape(-1)
    res = pcg(h.A, b, pre.apply, tol=1e-10)
    assert res.iters == 1


def test_piecewise_constant_coarse_space():
    # L = 1 gives the classical aggregation coarse space
    g = Grid.unit_cube(8)
    perm = make_field("gauss", 8, 4)
    h = build_hierarchy(perm, g, 2, 1, sub=4, workers=1)
    lev = h.level(2)
    Pc = lev.P.toarray()
    cells = element_cells(g, (4, 4, 4))
    for e in range(lev.m):
        col = Pc[:, e]
        assert np.count_nonzero(col) == 64
        assert np.allclose(col[cells[e]], col[cells[e]][0])


@pytest.mark.parametrize("n,sub,levels,agg", [(4, 2, 2, 2), (8, 2, 3, 2), (8, 4, 2, 2)])
def test_pcg_matches_brute_force_pinv(n, sub, levels, agg):
    g = Grid.unit_cube(n)
    perm = _rand_perm(g.shape, 21, contrast=1e6)
    h = build_hierarchy(perm, g, levels, 2, sub=sub, agg=agg, workers=1)
    A = h.A.toarray()
    b = random_zero_mean(g.shape, 5).reshape(-1)
    exact = np.linalg.pinv(A, hermitian=True) @ b
    exact -= exact.mean()
    tol = 1e-8
    res = pcg(h.A, b, Preconditioner(h).apply, tol=tol)
    assert res.converged and not res.breakdown
    w = np.linalg.eigvalsh(A)
    lam_min = w[1]
    bound = tol * np.linalg.norm(b) / lam_min
    assert np.linalg.norm(res.x - exact) <= bound
    assert abs(res.x.mean()) < 1e-14 * np.abs(res.x).max()


def test_pcg_iteration_counts_bounded_across_contrast():
    # Section 5.2: iterations grow with the contrast but stay bounded, and the
    # preconditioner never breaks down.
    g = Grid.unit_cube(32)
    its = []
    for cr in (1, 3, 6):
        rng = np.random.default_rng(8)
        perm = np.ones(g.shape)
        for _ in range(30):
            e = rng.integers(2, 9, 3)
            o = [rng.integers(0, 32 - e[i] + 1) for i in range(3)]
            perm[o[2]:o[2] + e[2], o[1]:o[1] + e[1], o[0]:o[0] + e[0]] = 10.0 ** cr
        h = build_hierarchy(perm, g, 2, 4, sub=8, workers=1)
        res = pcg(h.A, corner_source(g.shape).reshape(-1), Preconditioner(h).apply, tol=1e-6)
        assert res.converged and not res.breakdown
        its.append(res.iters)
    assert max(its) < 60


def _golden(name):
    out = {}
    path = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden", name)
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split(":", 1)
            out[k.strip()] = [int(t) for t in v.split()]
    return out


def test_paper_ladder_on_homogeneous_element():
    # The oracle's level-2 spectrum of a homogeneous 8^3 element reproduces the
    # ladder printed in Section 5.2: equal labels <=> equal eigenvalues, and the
    # clean cuts it names are exactly where the cluster rule keeps the target.
    gold = _golden("homogeneous_ladder.txt")
    lad, cuts = gold["ladder"], gold["clean_cuts"]
    g = Grid.unit_cube(8)
    h = build_hierarchy(np.ones(g.shape), g, 2, len(lad), sub=8, workers=1)
    lam = h.level(2).lam[0][: len(lad)]
    for i in range(1, len(lad)):
        same = abs(lam[i] - lam[i - 1]) <= 1e-9 * max(lam[i], 1e-12)
        assert same == (lad[i] == lad[i - 1]), (i, lam[i - 1], lam[i])
    clean = [i for i in range(1, len(lad)) if lad[i] != lad[i - 1]]
    for c in cuts:
        assert c in clean
        assert cluster_cut(np.asarray(lam), c) == c


# --------------------------------------------------------------------------
# Section 5: coarse-coarse counts L_cc and strategy 2 (threshold B_cc)

def _full_level2(levels=3, **kw):
    # sub = 4 and 64 vectors per level-2 element: W_c = W_h, so eq. spectral cc
    # on a level-3 element of 8^3 cells is the fine Neumann problem there,
    # whose spectrum is the DCT ladder of an 8^3 block
    g = Grid.unit_cube(8)
    return build_hierarchy(np.ones(g.shape), g, levels, 64, sub=4, agg=2, workers=1, **kw)


def test_coarse_coarse_spectrum_with_full_level2_space():
    h = _full_level2(target_cc=10)
    assert list(h.level(2).nkeep) == [64] * 8
    ref = _dct_ladder(8)
    assert np.allclose(h.level(3).lam[0][:14], ref[:14], rtol=0, atol=1e-12)
    assert list(h.level(3).nkeep) == [11]      # L_cc = 10 cuts the cluster 8..10: grows to 11


@pytest.mark.parametrize("b_between,expect", [((0, 1), 1), ((3, 4), 4), ((7, 8), 8)])
def test_threshold_strategy_counts_ladder(b_between, expect):
    # B_cc placed between two rungs of the ladder keeps every eigenvalue below it
    ref = _dct_ladder(8)
    lo, hi = b_between
    B = 0.5 * (ref[lo] + ref[hi])
    h = _full_level2(target_cc=10, threshold_cc=B)
    assert list(h.level(3).nkeep) == [expect]


def test_threshold_strategy_caps_at_candidates():
    # more eigenvalues below B than candidates: L_cc = 4 of them, a clean cut
    ref = _dct_ladder(8)
    h = _full_level2(target_cc=4, threshold_cc=0.5 * (ref[10] + ref[11]))
    assert list(h.level(3).nkeep) == [4]
    assert threshold_target(ref, 4, 0.0) == 4            # strategy 1
    assert threshold_target(ref, 4, 1e-300) == 1         # never below one vector


@pytest.mark.parametrize("b_between,expect", [((0, 1), 1), ((3, 4), 4), ((6, 7), 7)])
def test_level2_threshold_strategy_counts_ladder(b_between, expect):
    # B_c between two rungs of a homogeneous element's ladder keeps exactly the
    # eigenvalues below it on every level-2 element (at most L_c = 8 candidates)
    g = Grid.unit_cube(16)
    ref = _dct_ladder(8)
    lo, hi = b_between
    h = build_hierarchy(np.ones(g.shape), g, 2, 8, sub=8, workers=1, threshold_c=0.5 * (ref[lo] + ref[hi]))
    assert list(h.level(2).nkeep) == [expect] * 8


def test_level2_threshold_caps_at_candidates():
    # more eigenvalues below B_c than the L_c = 4 candidates: 4 of them (a clean cut)
    g = Grid.unit_cube(16)
    ref = _dct_ladder(8)
    h = build_hierarchy(np.ones(g.shape), g, 2, 4, sub=8, workers=1, threshold_c=0.5 * (ref[10] + ref[11]))
    assert list(h.level(2).nkeep) == [4] * 8
