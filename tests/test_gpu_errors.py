"""Failure paths of the solve entry points, through the C-ABI on the GPU.

Every case is a normal return with an error code (no kernel faults): the
host checks the source's compatibility (the zero-sum condition on f that
makes A p = f solvable) and the arguments, set-up checks the permeability
on the device and reports it, and CG stops on a non-positive or non-finite
p^T A p (breakdown) or at the iteration cap with the last iterate.  The
context stays usable after ENOCONV and EBREAKDOWN.
"""
import numpy as np
import pytest

from synth.fields import make_field, make_source
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def _ctx(perm, **kw):
    from paper_2403_19342_amd.specmg import SpecMG
    return SpecMG(to_dev(perm), levels=3, eigs_per_subdomain=4, agg=2, **kw)


def _solve_ok(ctx, b):
    import torch
    x = torch.empty(b.size, dtype=torch.float64, device="cuda")
    rc, info = ctx.pcg_solve(to_dev(b), x, tol=1e-6, raise_on_error=False)
    assert rc == 0 and info.converged and info.rel_resid_true <= 1e-6
    return info


@pytest.mark.parametrize("bad", ["zero", "negative", "nan", "inf"])
def test_setup_rejects_bad_permeability(bad):
    from paper_2403_19342_amd.specmg import SpecMGError, EINVAL_PERM
    perm = make_field("gauss", 32, 1)
    perm[3, 5, 7] = {"zero": 0.0, "negative": -1.0, "nan": np.nan, "inf": np.inf}[bad]
    with pytest.raises(SpecMGError) as ei:
        _ctx(perm)
    assert ei.value.code == EINVAL_PERM
    assert "permeability" in str(ei.value)


def test_pcg_rejects_incompatible_source():
    import torch
    from paper_2403_19342_amd.specmg import ERHS
    perm = make_field("gauss", 32, 1)
    ctx = _ctx(perm)
    b = make_source("corner", perm.shape).reshape(-1)
    bad = b.copy()
    bad[100] += 1e-3            # sum f = 1e-3 > 1e-12 sum |f|
    x = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    rc, info = ctx.pcg_solve(to_dev(bad), x, tol=1e-6, raise_on_error=False)
    assert rc == ERHS
    rc, info = ctx.gmres_solve(to_dev(bad), x, tol=1e-6, raise_on_error=False)
    assert rc == ERHS
    _solve_ok(ctx, b)
    ctx.close()


def test_pcg_iteration_cap_returns_last_iterate():
    import torch
    from paper_2403_19342_amd.specmg import ENOCONV
    perm = make_field("inclusions", 32, 3)
    ctx = _ctx(perm)
    b = make_source("corner", perm.shape).reshape(-1)
    x = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    rc, info = ctx.pcg_solve(to_dev(b), x, tol=1e-6, max_iter=1, raise_on_error=False)
    assert rc == ENOCONV
    assert info.iters == 1 and not info.converged
    xg = to_host(x)
    # one CG step from x0 = 0: x = alpha z, a non-zero zero-mean vector whose
    # residual lies between the solve's tolerance and the source's norm
    assert np.linalg.norm(xg) > 0 and abs(xg.mean()) < 1e-12 * np.abs(xg).max()
    assert 1e-6 < info.rel_resid_true < 1.0
    # the context keeps working
    _solve_ok(ctx, b)
    ctx.close()


def test_pcg_breakdown_on_non_finite_source():
    import torch
    from paper_2403_19342_amd.specmg import EBREAKDOWN
    perm = make_field("gauss", 32, 1)
    ctx = _ctx(perm)
    b = make_source("corner", perm.shape).reshape(-1)
    bad = b.copy()
    bad[5] = np.nan
    x = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    rc, info = ctx.pcg_solve(to_dev(bad), x, tol=1e-6, raise_on_error=False)
    assert rc == EBREAKDOWN
    assert not info.converged
    _solve_ok(ctx, b)
    ctx.close()


def test_pcg_rejects_bad_arguments():
    import torch
    from paper_2403_19342_amd.specmg import EINVAL
    perm = make_field("gauss", 32, 1)
    ctx = _ctx(perm)
    b = make_source("corner", perm.shape).reshape(-1)
    x = torch.zeros(b.size, dtype=torch.float64, device="cuda")
    for tol, it in ((0.0, 10), (-1e-6, 10), (1e-6, 0)):
        rc, info = ctx.pcg_solve(to_dev(b), x, tol=tol, max_iter=it, raise_on_error=False)
        assert rc == EINVAL
    _solve_ok(ctx, b)
    ctx.close()


def test_zero_source_gives_zero_solution():
    import torch
    perm = make_field("gauss", 32, 1)
    ctx = _ctx(perm)
    x = torch.ones(perm.size, dtype=torch.float64, device="cuda")
    rc, info = ctx.pcg_solve(torch.zeros_like(x), x, tol=1e-6, raise_on_error=False)
    assert rc == 0 and info.converged and info.iters == 0
    assert float(torch.abs(x).max()) == 0.0
    ctx.close()
