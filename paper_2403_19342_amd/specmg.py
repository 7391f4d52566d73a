"""ctypes binding of libspecmg (the C-ABI declared in include/specmg.h).

Argument marshalling only: device buffers are torch tensors on the current
device (float64, contiguous, x fastest), streams are torch streams.  Every
numerical step runs in the library's HIP kernels; loading fails loudly when
the library is missing.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspecmg.so")

OK, EINVAL, EINVAL_PERM, ERHS, ENOCONV, EBREAKDOWN, EEIG, EFACT, EDEVICE = 0, -1, -2, -3, -4, -5, -6, -7, -8
FP64, FP32_VCYCLE, FP32_BASIS, FP32_STORE = 0, 1, 2, 3
WS_NONE, WS_CNN = 0, 1

EXPORTED = ["specmg_setup", "specmg_setup_alloc", "specmg_apply_precond", "specmg_pcg_solve", "specmg_gmres_solve",
            "specmg_recover_flux", "specmg_mass_balance", "specmg_apply_operator",
            "specmg_get_info", "specmg_copy_level", "specmg_set_profiling", "specmg_get_profile",
            "specmg_destroy", "specmg_last_error", "specmg_cnn_param_count", "specmg_cnn_create",
            "specmg_cnn_destroy", "specmg_cnn_load", "specmg_cnn_patches", "specmg_cnn_forward",
            "specmg_cnn_loss_backward", "specmg_cnn_adam", "specmg_total_mobility", "specmg_transport",
            "specmg_transport_noalloc"]
TRANSPORT_NOALLOC_MAX_CELLS = 2097152   # SPECMG_TRANSPORT_NOALLOC_MAX_CELLS
PROFILE_CLASSES = ["cg_spmv", "pre_smooth", "resid_restrict", "prolong", "post_smooth", "coarse_part",
                   "coarsest", "p_update"]


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
                ("sub", ctypes.c_int32), ("agg", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("eigs_per_subdomain", ctypes.c_int32),
                ("nu", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("warm_start", ctypes.c_int32), ("cnn_weights", ctypes.c_void_p),
                ("eig_tol", ctypes.c_double), ("cluster_rtol", ctypes.c_double),
                ("ws_resid_tol", ctypes.c_double), ("eigs_coarse", ctypes.c_int32),
                ("eig_threshold_coarse", ctypes.c_double), ("nu_c", ctypes.c_int32),
                ("eig_threshold", ctypes.c_double)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p)]


def torch_allocator():
    """specmg_allocator callbacks over PyTorch's caching allocator (the
    returned object keeps the callbacks alive; hold it as long as the
    context)."""
    import torch
    dev = torch.cuda.current_device()

    def _alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0))
        except Exception:
            return None

    def _free(ptr, user):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:
            pass

    fa, ff = _ALLOC_FN(_alloc), _FREE_FN(_free)
    return Allocator(fa, ff, None), (fa, ff)


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("rel_resid", ctypes.c_double), ("rel_resid_true", ctypes.c_double),
                ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("n_levels", ctypes.c_int32), ("dims", ctypes.c_int32 * 8),
                ("eig_unconverged", ctypes.c_int32), ("ws_fallbacks", ctypes.c_int32),
                ("replacements", ctypes.c_int32)]

    def as_dict(self):
        return {"iters": self.iters, "converged": bool(self.converged), "rel_resid": self.rel_resid,
                "rel_resid_true": self.rel_resid_true, "setup_ms": self.setup_ms,
                "solve_ms": self.solve_ms, "n_levels": self.n_levels,
                "dims": list(self.dims)[: self.n_levels], "eig_unconverged": self.eig_unconverged,
                "ws_fallbacks": self.ws_fallbacks, "replacements": self.replacements}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libspecmg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2403_19342_amd.build`")
    # The device buffers handed to the library come from torch, so the library must bind to
    # the HIP runtime torch loads: import torch first, so that the runtime's soname already
    # resolves to that copy when the library's own dependency is looked up.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.specmg_setup.argtypes = [vp, i32, ctypes.POINTER(Grid), ctypes.POINTER(Opts), vp, ctypes.POINTER(vp)]
    lib.specmg_setup.restype = ctypes.c_int
    lib.specmg_setup_alloc.argtypes = [vp, i32, ctypes.POINTER(Grid), ctypes.POINTER(Opts), ctypes.POINTER(Allocator),
                                       vp, ctypes.POINTER(vp)]
    lib.specmg_setup_alloc.restype = ctypes.c_int
    lib.specmg_apply_precond.argtypes = [vp, vp, vp, vp]
    lib.specmg_apply_precond.restype = ctypes.c_int
    lib.specmg_pcg_solve.argtypes = [vp, vp, vp, i32, dbl, i32, ctypes.POINTER(SolveInfo), vp]
    lib.specmg_pcg_solve.restype = ctypes.c_int
    lib.specmg_gmres_solve.argtypes = [vp, vp, vp, i32, i32, dbl, i32, ctypes.POINTER(SolveInfo), vp]
    lib.specmg_gmres_solve.restype = ctypes.c_int
    lib.specmg_recover_flux.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.specmg_recover_flux.restype = ctypes.c_int
    lib.specmg_mass_balance.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.specmg_mass_balance.restype = ctypes.c_int
    lib.specmg_apply_operator.argtypes = [vp, vp, vp, vp]
    lib.specmg_apply_operator.restype = ctypes.c_int
    lib.specmg_get_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32 * 8), ctypes.POINTER(i32 * 8),
                                    ctypes.POINTER(i32 * 8), ctypes.POINTER(SolveInfo)]
    lib.specmg_get_info.restype = ctypes.c_int
    lib.specmg_copy_level.argtypes = [vp, i32, i32, vp, ctypes.c_size_t]
    lib.specmg_copy_level.restype = ctypes.c_int
    lib.specmg_set_profiling.argtypes = [vp, i32]
    lib.specmg_set_profiling.restype = ctypes.c_int
    lib.specmg_get_profile.argtypes = [vp, ctypes.POINTER(dbl * 8), ctypes.POINTER(i32 * 8), ctypes.POINTER(dbl * 8)]
    lib.specmg_get_profile.restype = ctypes.c_int
    lib.specmg_destroy.argtypes = [vp]
    lib.specmg_destroy.restype = None
    lib.specmg_last_error.argtypes = []
    lib.specmg_last_error.restype = ctypes.c_char_p
    i64 = ctypes.c_int64
    lib.specmg_cnn_param_count.argtypes = [i32]
    lib.specmg_cnn_param_count.restype = i64
    lib.specmg_cnn_create.argtypes = [i32, i32, ctypes.POINTER(vp)]
    lib.specmg_cnn_create.restype = ctypes.c_int
    lib.specmg_cnn_destroy.argtypes = [vp]
    lib.specmg_cnn_destroy.restype = None
    lib.specmg_cnn_load.argtypes = [vp, vp, vp, vp]
    lib.specmg_cnn_load.restype = ctypes.c_int
    lib.specmg_cnn_patches.argtypes = [vp, ctypes.POINTER(Grid), i32, i32, vp, vp, vp]
    lib.specmg_cnn_patches.restype = ctypes.c_int
    lib.specmg_cnn_forward.argtypes = [vp, vp, i32, vp, vp]
    lib.specmg_cnn_forward.restype = ctypes.c_int
    lib.specmg_cnn_loss_backward.argtypes = [vp, vp, vp, vp, i32, vp, i32, ctypes.POINTER(dbl), vp, vp]
    lib.specmg_cnn_loss_backward.restype = ctypes.c_int
    lib.specmg_cnn_adam.argtypes = [vp, vp, vp, vp, i64, dbl, dbl, dbl, dbl, i32, vp, vp]
    lib.specmg_cnn_adam.restype = ctypes.c_int
    lib.specmg_total_mobility.argtypes = [vp, vp, vp, i64, vp]
    lib.specmg_total_mobility.restype = ctypes.c_int
    lib.specmg_transport.argtypes = [ctypes.POINTER(Grid), vp, vp, vp, vp, vp, vp, i32, dbl, vp, vp, vp]
    lib.specmg_transport.restype = ctypes.c_int
    lib.specmg_transport_noalloc.argtypes = [ctypes.POINTER(Grid), vp, vp, vp, vp, vp, vp, i32, dbl, vp, vp]
    lib.specmg_transport_noalloc.restype = ctypes.c_int
    _lib = lib
    return lib


class SpecMGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"specmg error {code}: {msg}")
        self.code = code


def _check(code):
    if code != OK:
        raise SpecMGError(code, _lib.specmg_last_error().decode())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t, dtype=None):
    import torch
    dtype = dtype or torch.float64
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"expected a contiguous {dtype} CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _spacings(h):
    """(hx, hy, hz) from one spacing or a sequence of three."""
    if isinstance(h, (int, float)):
        return float(h), float(h), float(h)
    hs = tuple(float(v) for v in h)
    if len(hs) != 3:
        raise ValueError("h must be one spacing or (hx, hy, hz)")
    return hs


def transport_work_size(n: int) -> int:
    """Doubles of scratch specmg_transport needs for n cells: rates, f_w, per-block maxima."""
    return 2 * n + 2048


def total_mobility(perm, s, perm_eff):
    """perm_eff = perm * lambda(S) on the device (specmg_total_mobility)."""
    lib = load_library()
    if not (perm.numel() == s.numel() == perm_eff.numel()):
        raise ValueError("perm, s and perm_eff must have the same size")
    _check(lib.specmg_total_mobility(_dev_ptr(perm), _dev_ptr(s), _dev_ptr(perm_eff), perm.numel(), _stream()))


def transport(phi, q, vx, vy, vz, s, h, substeps: int, ds_max: float, work, t):
    """Explicit saturation sub-steps with the face velocity fixed (specmg_transport).

    All fields (nz, ny, nx) float64 CUDA tensors; `s` is updated in place,
    `work` holds at least transport_work_size(s.numel()) doubles, `t` (one double) receives
    the summed sub-step lengths.
    """
    lib = load_library()
    if s.dim() != 3:
        raise ValueError("s must have shape (nz, ny, nx)")
    nz, ny, nx = s.shape
    n = s.numel()
    for a in (phi, q, vx, vy, vz):
        if a.numel() != n:
            raise ValueError("every field must have s.numel() entries")
    if work.numel() < transport_work_size(n) or t.numel() < 1:
        raise ValueError(f"work needs {transport_work_size(n)} doubles and t one")
    hx, hy, hz = _spacings(h)
    g = Grid(nx, ny, nz, hx, hy, hz, 8, 2)
    _check(lib.specmg_transport(ctypes.byref(g), _dev_ptr(phi), _dev_ptr(q), _dev_ptr(vx), _dev_ptr(vy),
                                _dev_ptr(vz), _dev_ptr(s), int(substeps), float(ds_max), _dev_ptr(work),
                                _dev_ptr(t), _stream()))


def transport_noalloc(phi, q, vx, vy, vz, s, h, substeps: int, ds_max: float, t):
    """specmg_transport without a workspace argument (specmg_transport_noalloc):
    the library's built-in per-GPU workspace, for grids of at most
    TRANSPORT_NOALLOC_MAX_CELLS cells; calls that overlap on one GPU race."""
    lib = load_library()
    if s.dim() != 3:
        raise ValueError("s must have shape (nz, ny, nx)")
    nz, ny, nx = s.shape
    n = s.numel()
    for a in (phi, q, vx, vy, vz):
        if a.numel() != n:
            raise ValueError("every field must have s.numel() entries")
    if t.numel() < 1:
        raise ValueError("t needs one double")
    hx, hy, hz = _spacings(h)
    g = Grid(nx, ny, nz, hx, hy, hz, 8, 2)
    _check(lib.specmg_transport_noalloc(ctypes.byref(g), _dev_ptr(phi), _dev_ptr(q), _dev_ptr(vx), _dev_ptr(vy),
                                        _dev_ptr(vz), _dev_ptr(s), int(substeps), float(ds_max), _dev_ptr(t),
                                        _stream()))


@dataclass
class LevelArrays:
    nkeep: np.ndarray
    lam: np.ndarray
    basis: np.ndarray
    Ad: np.ndarray
    Aoff: np.ndarray
    status: np.ndarray


class SpecMG:
    """Set-up context of the multiscale spectral multigrid preconditioner."""

    def __init__(self, perm, levels: int, eigs_per_subdomain: int, h=None,
                 agg: int = 4, precision: int = FP64, eig_tol: float = 1e-12, cluster_rtol: float = 1e-6,
                 allow_unconverged: bool = False, cnn_weights=None, ws_resid_tol: float = 1e-3,
                 eigs_coarse: int = 0, eig_threshold_coarse: float = 0.0, nu: int = 1, nu_c: int = 0,
                 allocator: str = "torch", eig_threshold: float = 0.0):
        """allocator: "torch" (the context's device memory comes from PyTorch's
        caching allocator through specmg_setup_alloc) or "hip" (hipMalloc)."""
        lib = load_library()
        import torch
        if perm.dim() == 4 and perm.shape[0] == 3:
            ncomp = 3                      # (kappa_x, kappa_y, kappa_z) per cell
            nz, ny, nx = perm.shape[1:]
        elif perm.dim() == 3:
            ncomp = 1
            nz, ny, nx = perm.shape
        else:
            raise ValueError("perm must have shape (nz, ny, nx) or (3, nz, ny, nx)")
        self.shape = (nz, ny, nx)
        self.n = nx * ny * nz
        if h is None:
            h = 1.0 / nx
        hx, hy, hz = _spacings(h)
        self.grid = Grid(nx, ny, nz, hx, hy, hz, 8, agg)
        ws, wp = WS_NONE, None
        if cnn_weights is not None:
            # bf16 parameter vector, stored as int16 bits in a torch tensor
            if not (cnn_weights.is_cuda and cnn_weights.dtype == torch.int16 and cnn_weights.is_contiguous()):
                raise ValueError("cnn_weights must be a contiguous int16 (bf16 bits) CUDA tensor")
            if cnn_weights.numel() != lib.specmg_cnn_param_count(eigs_per_subdomain):
                raise ValueError("cnn_weights has the wrong length for eigs_per_subdomain")
            ws, wp = WS_CNN, ctypes.c_void_p(cnn_weights.data_ptr())
        self.opts = Opts(levels, eigs_per_subdomain, nu, precision, ws, wp, eig_tol, cluster_rtol, ws_resid_tol,
                         eigs_coarse, eig_threshold_coarse, nu_c, eig_threshold)
        ctx = ctypes.c_void_p()
        perm = perm.contiguous()
        if allocator == "torch":
            self._alloc, self._alloc_keep = torch_allocator()
            rc = lib.specmg_setup_alloc(_dev_ptr(perm), ncomp, ctypes.byref(self.grid), ctypes.byref(self.opts),
                                        ctypes.byref(self._alloc), _stream(), ctypes.byref(ctx))
        elif allocator == "hip":
            rc = lib.specmg_setup(_dev_ptr(perm), ncomp, ctypes.byref(self.grid), ctypes.byref(self.opts),
                                  _stream(), ctypes.byref(ctx))
        else:
            raise ValueError("allocator must be 'torch' or 'hip'")
        if rc == EEIG and allow_unconverged:
            pass
        elif rc != OK:
            _check(rc)
        self._ctx = ctx
        self.levels = levels
        torch.cuda.synchronize()

    def close(self):
        if getattr(self, "_ctx", None):
            _lib.specmg_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply_precond(self, r, z):
        _check(_lib.specmg_apply_precond(self._ctx, _dev_ptr(r), _dev_ptr(z), _stream()))

    def apply_operator(self, x, y):
        _check(_lib.specmg_apply_operator(self._ctx, _dev_ptr(x), _dev_ptr(y), _stream()))

    def pcg_solve(self, rhs, x, tol: float = 1e-6, max_iter: int = 1000, use_x0: bool = False,
                  raise_on_error: bool = True):
        info = SolveInfo()
        rc = _lib.specmg_pcg_solve(self._ctx, _dev_ptr(rhs), _dev_ptr(x), int(use_x0), tol, max_iter,
                                   ctypes.byref(info), _stream())
        if rc != OK and raise_on_error:
            _check(rc)
        return rc, info

    def gmres_solve(self, rhs, x, restart: int = 30, tol: float = 1e-6, max_iter: int = 1000,
                    use_x0: bool = False, raise_on_error: bool = True):
        """Restarted flexible GMRES around the V-cycle (specmg_gmres_solve)."""
        info = SolveInfo()
        rc = _lib.specmg_gmres_solve(self._ctx, _dev_ptr(rhs), _dev_ptr(x), int(use_x0), int(restart), tol,
                                     max_iter, ctypes.byref(info), _stream())
        if rc != OK and raise_on_error:
            _check(rc)
        return rc, info

    def recover_flux(self, p, vx, vy, vz):
        """Face fluxes of the recovered velocity (specmg_recover_flux)."""
        _check(_lib.specmg_recover_flux(self._ctx, _dev_ptr(p), _dev_ptr(vx), _dev_ptr(vy), _dev_ptr(vz),
                                        _stream()))

    def mass_balance(self, vx, vy, vz, f, res):
        """res = discrete divergence of v minus f (specmg_mass_balance)."""
        _check(_lib.specmg_mass_balance(self._ctx, _dev_ptr(vx), _dev_ptr(vy), _dev_ptr(vz), _dev_ptr(f),
                                        _dev_ptr(res), _stream()))

    def set_profiling(self, on: bool = True):
        _check(_lib.specmg_set_profiling(self._ctx, int(on)))

    def profile(self):
        """{class: (total_ms, launches, algorithmic_bytes_per_launch)}"""
        ms = (ctypes.c_double * 8)()
        cnt = (ctypes.c_int32 * 8)()
        by = (ctypes.c_double * 8)()
        _check(_lib.specmg_get_profile(self._ctx, ctypes.byref(ms), ctypes.byref(cnt), ctypes.byref(by)))
        return {PROFILE_CLASSES[i]: (ms[i], cnt[i], by[i]) for i in range(8)}

    def info(self):
        lv = ctypes.c_int32()
        dims = (ctypes.c_int32 * 8)()
        elems = (ctypes.c_int32 * 8)()
        widths = (ctypes.c_int32 * 8)()
        si = SolveInfo()
        _check(_lib.specmg_get_info(self._ctx, ctypes.byref(lv), ctypes.byref(dims), ctypes.byref(elems),
                                    ctypes.byref(widths), ctypes.byref(si)))
        return {"levels": lv.value, "dims": list(dims)[: lv.value], "elems": list(elems)[: lv.value],
                "widths": list(widths)[: lv.value], "setup": si.as_dict()}

    def level_arrays(self, level: int) -> LevelArrays:
        inf = self.info()
        m = inf["elems"][level - 1]
        L = inf["widths"][level - 1]
        if level == 2:
            rows = 512
        else:
            rows = self.grid.agg ** 3 * inf["widths"][level - 2]
        out = {}
        for which, name, dtype, shape in ((0, "nkeep", np.int32, (m,)), (1, "lam", np.float64, (m, L)),
                                          (2, "basis", np.float64, (m, L, rows)),
                                          (3, "Ad", np.float64, (m, L, L)), (4, "Aoff", np.float64, (m, 3, L, L)),
                                          (5, "status", np.int32, (m,))):
            arr = np.empty(shape, dtype=dtype)
            _check(_lib.specmg_copy_level(self._ctx, level, which, arr.ctypes.data_as(ctypes.c_void_p), arr.nbytes))
            out[name] = arr
        return LevelArrays(**out)


class CNN:
    """Workspace of the warm-start network (k outputs, batches of at most
    max_batch level-2 elements).  Parameters are float32 CUDA tensors (the
    master copy) or int16 tensors holding bf16 bits."""

    def __init__(self, k: int, max_batch: int):
        lib = load_library()
        self.k = k
        self.kp = k
        self.max_batch = max_batch
        self.n_params = int(lib.specmg_cnn_param_count(k))
        h = ctypes.c_void_p()
        _check(lib.specmg_cnn_create(k, max_batch, ctypes.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.specmg_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load(self, theta):
        import torch
        if theta.dtype == torch.float32:
            _check(_lib.specmg_cnn_load(self._h, _dev_ptr(theta, torch.float32), None, _stream()))
        else:
            _check(_lib.specmg_cnn_load(self._h, None, _dev_ptr(theta, torch.int16), _stream()))

    @staticmethod
    def patches(perm, e0: int, count: int, patches, s=None):
        import torch
        load_library()
        nz, ny, nx = perm.shape
        g = Grid(nx, ny, nz, 1.0 / nx, 1.0 / nx, 1.0 / nx, 8, 2)
        _check(_lib.specmg_cnn_patches(_dev_ptr(perm), ctypes.byref(g), e0, count,
                                       _dev_ptr(patches, torch.float32),
                                       None if s is None else _dev_ptr(s), _stream()))

    def forward(self, patches, count: int, X):
        import torch
        _check(_lib.specmg_cnn_forward(self._h, _dev_ptr(patches, torch.float32), count,
                                       _dev_ptr(X, torch.float32), _stream()))

    def loss_backward(self, patches, X, phi, ldphi: int, s, count: int, grad) -> float:
        import torch
        loss = ctypes.c_double()
        _check(_lib.specmg_cnn_loss_backward(self._h, _dev_ptr(patches, torch.float32), _dev_ptr(X, torch.float32),
                                             _dev_ptr(phi), ldphi, _dev_ptr(s), count, ctypes.byref(loss),
                                             _dev_ptr(grad, torch.float32), _stream()))
        return loss.value

    @staticmethod
    def adam(theta, grad, m1, m2, lr: float, step: int, theta16=None, beta1=0.9, beta2=0.999, eps=1e-8):
        import torch
        load_library()
        _check(_lib.specmg_cnn_adam(_dev_ptr(theta, torch.float32), _dev_ptr(grad, torch.float32),
                                    _dev_ptr(m1, torch.float32), _dev_ptr(m2, torch.float32), theta.numel(),
                                    lr, beta1, beta2, eps, step,
                                    None if theta16 is None else _dev_ptr(theta16, torch.int16), _stream()))
