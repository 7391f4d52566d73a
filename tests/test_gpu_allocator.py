"""Device memory through a caller-supplied allocator (specmg_setup_alloc).

The binding's default hands PyTorch's caching allocator to the library, so
every device byte of a context is PyTorch's: the context's arrays show up in
torch.cuda.memory_allocated() while it lives and are returned when it is
destroyed.  Results are bit for bit those of a context on hipMalloc (same
kernels, same order).  An allocator that returns no memory makes set-up fail
with SPECMG_EDEVICE and leaves nothing behind.
"""
import ctypes

import numpy as np
import pytest

from synth.fields import make_field, make_source
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def _solve(perm, allocator):
    import torch
    from paper_2403_19342_amd.specmg import SpecMG
    ctx = SpecMG(to_dev(perm), levels=3, eigs_per_subdomain=6, agg=2, allocator=allocator)
    b = make_source("corner", perm.shape).reshape(-1)
    x = torch.empty(perm.size, dtype=torch.float64, device="cuda")
    rc, info = ctx.pcg_solve(to_dev(b), x, tol=1e-6)
    xg = to_host(x)
    rc2, info2 = ctx.gmres_solve(to_dev(b), x, restart=10, tol=1e-6)
    ctx.close()
    return rc, info.iters, xg, rc2, info2.iters, to_host(x)


def test_torch_allocator_owns_the_context_and_matches_hipmalloc():
    import torch
    from paper_2403_19342_amd.specmg import SpecMG
    perm = make_field("gauss", 64, 1)
    pd = to_dev(perm)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    ctx = SpecMG(pd, levels=3, eigs_per_subdomain=6, agg=2, allocator="torch")
    held = torch.cuda.memory_allocated() - base
    # at least kappa~, the IC pivots, the level-2 basis (9 x 8 B per cell) and the CG vectors
    assert held > 8 * perm.size * (2 + 9 + 6)
    ctx.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
    a = _solve(perm, "torch")
    h = _solve(perm, "hip")
    print(f"torch allocator: context held {held / 2**20:.1f} MiB; PCG {a[1]} / {h[1]} iterations, "
          f"GMRES {a[4]} / {h[4]} steps")
    assert a[0] == 0 and h[0] == 0 and a[3] == 0 and h[3] == 0
    assert a[1] == h[1] and a[4] == h[4]
    assert np.array_equal(a[2], h[2]) and np.array_equal(a[5], h[5])


def test_allocator_failure_is_reported():
    import torch
    from paper_2403_19342_amd.specmg import (load_library, Grid, Opts, Allocator, _ALLOC_FN, _FREE_FN, _stream,
                                             EDEVICE)
    lib = load_library()
    perm = to_dev(make_field("gauss", 32, 1))
    calls = {"alloc": 0, "free": 0}

    def _alloc(nbytes, stream, user):
        calls["alloc"] += 1
        return None

    def _free(ptr, user):
        calls["free"] += 1

    fa, ff = _ALLOC_FN(_alloc), _FREE_FN(_free)
    al = Allocator(fa, ff, None)
    g = Grid(32, 32, 32, 1 / 32, 1 / 32, 1 / 32, 8, 2)
    o = Opts(3, 6, 1, 0, 0, None, 1e-12, 1e-6, 1e-3, 0, 0.0, 0)
    ctx = ctypes.c_void_p()
    rc = lib.specmg_setup_alloc(ctypes.c_void_p(perm.data_ptr()), 1, ctypes.byref(g), ctypes.byref(o),
                                ctypes.byref(al), _stream(), ctypes.byref(ctx))
    assert rc == EDEVICE
    assert ctx.value is None
    assert calls["alloc"] == 1 and calls["free"] == 0
    assert "allocator" in lib.specmg_last_error().decode()
