"""FP32-basis mode (float64 fine level and CG, the level-2 basis stored in
float32 and summed in float64 by the restriction and the prolongation)
against the FP64 oracle.

Restriction and prolongation read the same rounded basis, so the V-cycle
stays a fixed symmetric map and plain CG applies.  Bounds, derived as for
the FP32 V-cycle: P^{-1} r within max(1e-5, 1e-6 / lambda_min+(A_L))
relative (basis rounding 6e-8 in both transfers, amplified by the coarsest
pseudo-inverse, factor 10 of headroom); PCG with true residual <= 1e-6,
iterations at most 10 % (+1) above the FP64 oracle's, and the solution
within the residual-derived bound.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import Grid, build_hierarchy, Preconditioner, pcg
from synth.fields import make_field, make_source, random_zero_mean
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

CASES = [
    ("gauss32_l3", 32, "gauss", 1, 3, 6, 2),
    ("incl32_l3", 32, "inclusions", 3, 3, 6, 4),
    ("chan32_l2", 32, "channels", 2, 2, 6, 4),
]


def _ctx(perm, levels, eigs, agg):
    from paper_2403_19342_amd.specmg import SpecMG, FP32_BASIS
    return SpecMG(to_dev(perm), levels=levels, eigs_per_subdomain=eigs, agg=agg, precision=FP32_BASIS)


@pytest.mark.parametrize("name,n,kind,seed,levels,eigs,agg", CASES)
def test_fp32_basis_apply_and_pcg(name, n, kind, seed, levels, eigs, agg):
    import torch
    perm = make_field(kind, n, seed)
    g = Grid.unit_cube(n)
    hier = build_hierarchy(perm, g, levels, eigs, sub=8, agg=agg, workers=1)
    pre = Preconditioner(hier)
    ctx = _ctx(perm, levels, eigs, agg)
    wL = np.linalg.eigvalsh(hier.level(levels).A.toarray())
    tol = max(1e-5, 1e-6 / wL[1])
    r = random_zero_mean(perm.shape, 400).reshape(-1)
    z = torch.empty(g.n, dtype=torch.float64, device="cuda")
    ctx.apply_precond(to_dev(r), z)
    torch.cuda.synchronize()
    zg, zo = to_host(z), pre.apply(r)
    zg -= zg.mean()
    zo -= zo.mean()
    perr = np.linalg.norm(zg - zo) / np.linalg.norm(zo)
    assert perr < tol
    b = make_source("corner", perm.shape).reshape(-1)
    ref = pcg(hier.A, b, pre.apply, tol=1e-6)
    x = torch.empty(g.n, dtype=torch.float64, device="cuda")
    rc, info = ctx.pcg_solve(to_dev(b), x, tol=1e-6)
    xg = to_host(x)
    w = np.sort(spla.eigsh(hier.A.tocsc(), k=2, sigma=-1.0, which="LM", return_eigenvectors=False))
    nb = np.linalg.norm(b)
    bound = (info.rel_resid_true + ref.rel_resid_true) * nb / w[1] / np.linalg.norm(ref.x)
    err = np.linalg.norm(xg - ref.x) / np.linalg.norm(ref.x)
    print(f"{name}: FP32 basis P^-1 r error {perr:.2e} (bound {tol:.1e}); iters {info.iters} (FP64 oracle "
          f"{ref.iters}), solution error {err:.2e} (bound {bound:.1e})")
    assert rc == 0 and info.converged and info.rel_resid_true <= 1e-6
    assert info.iters <= int(1.1 * ref.iters) + 1
    assert err <= bound
    ctx.close()
