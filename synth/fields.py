"""Seeded synthetic inputs: permeability fields and compatible sources.

This module only draws random numbers and lays out arrays.  It holds none of
the solver's arithmetic (no transmissibilities, no operators), so both the CPU
oracle and the GPU path may consume its output byte for byte.

Array convention: a field of shape (nz, ny, nx) in C order, so the flat index
of cell (i, j, k) is i + nx*(j + ny*k) (x fastest).  Values are float64.

The paper's own media (the fractured 256^3 medium of its Section 5.2, the
periodic channel cell of Section 5.1, SPE10 and the Watt field of Section 6)
are not available; these generators stand in for them with the same kind of
structure: high-contrast inclusions, Gaussian log-fields and connected
channels, all with a contrast of up to 1e6.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

LOG_CONTRAST_1E6 = 0.5 * math.log(1.0e6)


def boxes_field(n: int, seed: int, n_boxes: int | None = None, value: float = 1.0e4,
                edge_lo: int = 2, edge_hi: int = 8, cover: float | None = None,
                shape: tuple[int, int, int] | None = None) -> np.ndarray:
    """Background 1 with axis-aligned boxes of `value`.

    Either `n_boxes` boxes are placed, or boxes are placed until the covered
    volume fraction reaches `cover`.  Box edges are uniform integers in
    [edge_lo, edge_hi] per axis; positions are uniform with the box inside the
    domain; overlapping boxes keep `value`.
    """
    nz, ny, nx = shape if shape is not None else (n, n, n)
    rng = np.random.default_rng(seed)
    k = np.ones((nz, ny, nx), dtype=np.float64)
    mask = np.zeros((nz, ny, nx), dtype=bool)
    placed = 0
    total = nx * ny * nz
    covered = 0
    while True:
        if n_boxes is not None and placed >= n_boxes:
            break
        if cover is not None and covered >= cover * total:
            break
        ex, ey, ez = (int(v) for v in rng.integers(edge_lo, edge_hi + 1, size=3))
        ex, ey, ez = min(ex, nx), min(ey, ny), min(ez, nz)
        x0 = int(rng.integers(0, nx - ex + 1))
        y0 = int(rng.integers(0, ny - ey + 1))
        z0 = int(rng.integers(0, nz - ez + 1))
        sub = mask[z0:z0 + ez, y0:y0 + ey, x0:x0 + ex]
        covered += int(sub.size - np.count_nonzero(sub))
        sub[...] = True
        placed += 1
    k[mask] = value
    return k


def gaussian_log_field(n: int, seed: int, sigma: float = 3.0, corr_len: float = 0.1,
                       clip: float = LOG_CONTRAST_1E6,
                       shape: tuple[int, int, int] | None = None) -> np.ndarray:
    """exp of a stationary Gaussian field with exponential covariance.

    Covariance sigma^2 exp(-r / corr_len) with r the distance in the unit cube
    (cell size 1/n).  Sampled exactly by circulant embedding on a periodic box
    twice the domain size per axis, then cropped; the log-field is clipped to
    [-clip, +clip], so the contrast is at most exp(2 clip) (1e6 by default).
    """
    nz, ny, nx = shape if shape is not None else (n, n, n)
    h = 1.0 / n
    rng = np.random.default_rng(seed)
    dims = (2 * nz, 2 * ny, 2 * nx)

    def wrap(m):
        i = np.arange(m)
        return np.minimum(i, m - i) * h

    dz, dy, dx = np.meshgrid(wrap(dims[0]), wrap(dims[1]), wrap(dims[2]), indexing="ij")
    r = np.sqrt(dx * dx + dy * dy + dz * dz)
    cov = (sigma * sigma) * np.exp(-r / corr_len)
    del dx, dy, dz, r
    lam = np.fft.fftn(cov).real
    del cov
    np.maximum(lam, 0.0, out=lam)
    np.sqrt(lam, out=lam)
    white = rng.standard_normal(dims)
    y = np.fft.ifftn(lam * np.fft.fftn(white)).real
    del white, lam
    y = np.ascontiguousarray(y[:nz, :ny, :nx])
    np.clip(y, -clip, clip, out=y)
    return np.exp(y)


def channel_field(n: int, seed: int, n_channels: int = 24, value: float = 1.0e6,
                  shape: tuple[int, int, int] | None = None) -> np.ndarray:
    """Background 1 with sinusoidal channels of `value`.

    Each channel is a horizontal slab of thickness U{2..6} cells whose in-plane
    centreline is c0 + A sin(2 pi s / P + phi) along its axis s (x or y with
    probability 1/2), with A in U[0.02, 0.1] n, P in U[0.25, 1] n and width
    U{3..8} cells.
    """
    nz, ny, nx = shape if shape is not None else (n, n, n)
    rng = np.random.default_rng(seed)
    k = np.ones((nz, ny, nx), dtype=np.float64)
    for _ in range(n_channels):
        thick = int(rng.integers(2, 7))
        width = int(rng.integers(3, 9))
        amp = float(rng.uniform(0.02, 0.1)) * n
        period = float(rng.uniform(0.25, 1.0)) * n
        phase = float(rng.uniform(0.0, 2.0 * math.pi))
        along_x = bool(rng.integers(0, 2))
        z0 = int(rng.integers(0, nz - thick + 1))
        if along_x:
            c0 = float(rng.uniform(0.0, ny))
            s = np.arange(nx) + 0.5
            centre = c0 + amp * np.sin(2.0 * math.pi * s / period + phase)
            t = np.arange(ny)[:, None] + 0.5
            band = np.abs(t - centre[None, :]) <= 0.5 * width      # (ny, nx)
        else:
            c0 = float(rng.uniform(0.0, nx))
            s = np.arange(ny) + 0.5
            centre = c0 + amp * np.sin(2.0 * math.pi * s / period + phase)
            t = np.arange(nx)[None, :] + 0.5
            band = np.abs(t - centre[:, None]) <= 0.5 * width      # (ny, nx)
        k[z0:z0 + thick][:, band] = value
    return k


def corner_source(shape: tuple[int, int, int]) -> np.ndarray:
    """+1 in cell (0,0,0) and -1 in the opposite corner cell."""
    f = np.zeros(shape, dtype=np.float64)
    f[0, 0, 0] = 1.0
    f[-1, -1, -1] = -1.0
    return f


def quarter_five_spot(shape: tuple[int, int, int]) -> np.ndarray:
    """Injector column at (x,y)=(0,0), producer column at the opposite corner.

    Each column holds +-1/nz per cell, so the total is exactly zero in binary
    when nz is a power of two.
    """
    nz, ny, nx = shape
    f = np.zeros(shape, dtype=np.float64)
    f[:, 0, 0] = 1.0 / nz
    f[:, -1, -1] = -1.0 / nz
    return f


def five_spot(shape: tuple[int, int, int]) -> np.ndarray:
    """Four corner columns and one opposite-signed centre column (Section 5).

    The centre column carries +1/nz per cell and each corner column -1/(4 nz)
    per cell.
    """
    nz, ny, nx = shape
    f = np.zeros(shape, dtype=np.float64)
    f[:, ny // 2, nx // 2] = 1.0 / nz
    q = -1.0 / (4.0 * nz)
    for (j, i) in ((0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1)):
        f[:, j, i] += q
    return f


def porosity_field(perm: np.ndarray, seed: int, mean: float = 0.2, spread: float = 0.05,
                   floor: float = 0.05) -> np.ndarray:
    """Porosity loosely following log-permeability, truncated below at `floor`.

    phi = mean + spread * (standardised log kappa + 0.5 N(0,1)), clipped to
    [floor, 0.5]; the floor mirrors the truncation of inactive cells in the
    two-phase model (Section 6).
    """
    rng = np.random.default_rng(seed)
    lk = np.log(np.asarray(perm, dtype=np.float64))
    sd = lk.std()
    z = (lk - lk.mean()) / (sd if sd > 0 else 1.0)
    phi = mean + spread * (z + 0.5 * rng.standard_normal(lk.shape))
    return np.clip(phi, floor, 0.5)


def random_saturation(shape: tuple[int, int, int], seed: int, lo: float = 0.2, hi: float = 0.8) -> np.ndarray:
    """Uniform water saturation in [lo, hi] per cell."""
    return np.random.default_rng(seed).uniform(lo, hi, shape)


def random_zero_mean(shape: tuple[int, int, int], seed: int) -> np.ndarray:
    """Standard normal vector with its mean removed (a compatible source)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(shape)
    v -= v.mean()
    return v


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    levels: int
    eigs: int
    precision: str           # default form: "fp64" (every workload); the mixed forms are options
    seed: int
    kind: str                # field generator
    source: str
    agg: int = 4             # level-l elements per level-(l+1) element along each axis
    eigs_coarse: int = 0     # kept count at levels >= 3 (0: same as eigs)


WORKLOADS = {
    "boxes32": Workload("boxes32", 32, 2, 4, "fp64", 0, "boxes", "corner"),
    "gauss128": Workload("gauss128", 128, 3, 6, "fp64", 1, "gauss", "quarter_five_spot"),
    "channels256": Workload("channels256", 256, 3, 8, "fp64", 2, "channels", "five_spot"),
    # 32^3-cell coarse elements hold up to ~9 inclusions: 2x aggregation and
    # 10 vectors per coarse element keep every inclusion mode in the hierarchy
    "inclusions512": Workload("inclusions512", 512, 4, 6, "fp64", 3, "inclusions", "five_spot", 2, 10),
}


def make_field(kind: str, n: int, seed: int, shape=None, **kw) -> np.ndarray:
    if kind == "boxes":
        return boxes_field(n, seed, n_boxes=kw.get("n_boxes", 20), value=1.0e4,
                           edge_lo=2, edge_hi=8, shape=shape)
    if kind == "inclusions":
        return boxes_field(n, seed, n_boxes=None, value=kw.get("value", 1.0e6), edge_lo=2, edge_hi=16,
                           cover=kw.get("cover", 0.05), shape=shape)
    if kind == "gauss":
        return gaussian_log_field(n, seed, sigma=kw.get("sigma", 3.0),
                                  corr_len=kw.get("corr_len", 0.1), shape=shape)
    if kind == "channels":
        return channel_field(n, seed, n_channels=kw.get("n_channels", 24), value=kw.get("value", 1.0e6), shape=shape)
    if kind == "homogeneous":
        s = shape if shape is not None else (n, n, n)
        return np.ones(s, dtype=np.float64)
    raise ValueError(f"unknown field kind {kind!r}")


def make_source(kind: str, shape) -> np.ndarray:
    if kind == "corner":
        return corner_source(shape)
    if kind == "quarter_five_spot":
        return quarter_five_spot(shape)
    if kind == "five_spot":
        return five_spot(shape)
    raise ValueError(f"unknown source kind {kind!r}")


def learned_field(n: int, seed: int) -> np.ndarray:
    """Gaussian log-field with sigma ~ U[2,4] and correlation length ~ U[0.05,0.2].

    The two hyper-parameters are drawn from a generator seeded with `seed`
    (test fields use seeds 1000..1031, training fields seeds >= 10000).
    """
    rng = np.random.default_rng(seed)
    sigma = float(rng.uniform(2.0, 4.0))
    ell = float(rng.uniform(0.05, 0.2))
    return gaussian_log_field(n, seed + 7919, sigma=sigma, corr_len=ell)
