"""The C-ABI library loads and exports every entry point include/specmg.h
declares; host-side argument validation returns its error codes without
touching a device (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "specmg.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(specmg_[a-z_0-9]+)\s*\(", txt)))


def _lib():
    from paper_2403_19342_amd.specmg import load_library, LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.skip("libspecmg.so not built (run __graft_entry__.build())")
    return load_library()


def test_exports_every_declared_symbol():
    lib = _lib()
    names = _declared()
    assert "specmg_setup" in names and "specmg_pcg_solve" in names and "specmg_apply_precond" in names
    for nm in names:
        assert hasattr(lib, nm), nm


def test_binding_covers_header():
    from paper_2403_19342_amd.specmg import EXPORTED
    assert sorted(EXPORTED) == _declared()


@pytest.mark.parametrize("field,value,code", [
    ("sub", 4, -1), ("agg", 3, -1), ("nx", 36, -1), ("levels", 1, -1), ("eigs_per_subdomain", 0, -1),
    ("eigs_per_subdomain", 9, -1), ("nu", 3, -1), ("nu", 0, -1), ("nu_c", 3, -1), ("nu_c", -1, -1), ("precision", 7, -1), ("hy", 0.0, -1),
    ("hz", -1.0, -1), ("hx", float("nan"), -1), ("hy", float("inf"), -1),
    ("eigs_coarse", 21, -1), ("eigs_coarse", -1, -1), ("eig_threshold_coarse", -1.0, -1),
    ("eig_threshold_coarse", float("inf"), -1), ("eig_threshold", -1.0, -1), ("eig_threshold", float("nan"), -1),
])
def test_setup_rejects_bad_arguments(field, value, code):
    lib = _lib()
    from paper_2403_19342_amd.specmg import Grid, Opts
    g = Grid(32, 32, 32, 1 / 32, 1 / 32, 1 / 32, 8, 4)
    o = Opts(3, 6, 1, 0, 0, None, 1e-12, 1e-6, 1e-3)
    if hasattr(g, field) and field in [f[0] for f in Grid._fields_]:
        setattr(g, field, value)
    else:
        setattr(o, field, value)
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    rc = lib.specmg_setup(fake, 1, ctypes.byref(g), ctypes.byref(o), None, ctypes.byref(ctx))
    assert rc == code
    assert ctx.value is None
    assert lib.specmg_last_error().decode() != ""


def test_null_arguments():
    lib = _lib()
    assert lib.specmg_apply_precond(None, None, None, None) == -1
    assert lib.specmg_pcg_solve(None, None, None, 0, 1e-6, 10, None, None) == -1
    assert lib.specmg_apply_operator(None, None, None, None) == -1
    # the binding's argument types accept the arrays it passes
    i8 = ctypes.c_int32 * 8
    from paper_2403_19342_amd.specmg import SolveInfo
    assert lib.specmg_get_info(None, ctypes.byref(ctypes.c_int32()), ctypes.byref(i8()), ctypes.byref(i8()),
                               ctypes.byref(i8()), ctypes.byref(SolveInfo())) == -1
    lib.specmg_destroy(None)


def test_cnn_arguments_validated_on_host():
    lib = _lib()
    from paper_2403_19342_amd.specmg import Grid, Opts
    from oracle import cnn
    for k in (2, 4, 6, 8):
        assert lib.specmg_cnn_param_count(k) == cnn.n_params(k)
    for k in (0, 1, 5, 9):
        assert lib.specmg_cnn_param_count(k) == -1
    h = ctypes.c_void_p()
    assert lib.specmg_cnn_create(0, 16, ctypes.byref(h)) == -1 and h.value is None
    assert lib.specmg_cnn_create(9, 16, ctypes.byref(h)) == -1
    assert lib.specmg_cnn_create(5, 16, ctypes.byref(h)) == -1
    assert lib.specmg_cnn_create(6, 0, ctypes.byref(h)) == -1
    fake = ctypes.c_void_p(0x1000)
    bad = Grid(36, 32, 32, 1 / 32, 1 / 32, 1 / 32, 8, 4)
    assert lib.specmg_cnn_patches(fake, ctypes.byref(bad), 0, 1, fake, None, None) == -1
    good = Grid(32, 32, 32, 1 / 32, 1 / 32, 1 / 32, 8, 4)
    assert lib.specmg_cnn_patches(fake, ctypes.byref(good), 60, 5, fake, None, None) == -1   # 64 elements
    assert lib.specmg_cnn_adam(fake, fake, fake, fake, 0, 1e-3, 0.9, 0.999, 1e-8, 1, None, None) == -1
    assert lib.specmg_cnn_forward(None, fake, 1, fake, None) == -1
    # the CNN warm start needs its weights
    o = Opts(3, 6, 1, 0, 1, None, 1e-12, 1e-6, 1e-3)
    ctx = ctypes.c_void_p()
    assert lib.specmg_setup(fake, 1, ctypes.byref(good), ctypes.byref(o), None, ctypes.byref(ctx)) == -1
    o.warm_start = 5
    assert lib.specmg_setup(fake, 1, ctypes.byref(good), ctypes.byref(o), None, ctypes.byref(ctx)) == -1


def test_setup_alloc_rejects_incomplete_allocator():
    lib = _lib()
    from paper_2403_19342_amd.specmg import Grid, Opts, Allocator
    g = Grid(32, 32, 32, 1 / 32, 1 / 32, 1 / 32, 8, 4)
    o = Opts(3, 6, 1, 0, 0, None, 1e-12, 1e-6, 1e-3)
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    rc = lib.specmg_setup_alloc(fake, 1, ctypes.byref(g), ctypes.byref(o), ctypes.byref(Allocator()), None,
                                ctypes.byref(ctx))
    assert rc == -1
    assert ctx.value is None
    assert "allocator" in lib.specmg_last_error().decode()


@pytest.mark.parametrize("components,precision,warm", [(2, 0, 0), (3, 1, 0), (3, 3, 0), (3, 0, 1)])
def test_setup_rejects_unsupported_permeability_forms(components, precision, warm):
    # two components do not exist; orthotropic K runs with a float64 fine
    # level only and without the learned warm start (trained on kappa I)
    lib = _lib()
    from paper_2403_19342_amd.specmg import Grid, Opts
    g = Grid(32, 32, 32, 1 / 32, 1 / 32, 1 / 32, 8, 4)
    o = Opts(3, 6, 1, precision, warm, ctypes.c_void_p(0x2000) if warm else None, 1e-12, 1e-6, 1e-3)
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    rc = lib.specmg_setup(fake, components, ctypes.byref(g), ctypes.byref(o), None, ctypes.byref(ctx))
    assert rc == -1 and ctx.value is None
