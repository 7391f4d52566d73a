"""Learned warm start for the level-2 eigenproblems: FP64 reference network.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Not part of the paper: an extension that predicts, for every level-2 element
K, a start block for the local generalized eigenproblem of Section 3
(A_K phi = lambda S_K phi, eq. spepb) from the element's permeability.

Definitions followed here (the GPU kernels implement the same definitions):

* Input patch: log kappa on the 8^3 cells of K plus a one-cell halo (10^3
  values, z slowest, x fastest); outside the domain the nearest boundary
  cell is repeated.  Each patch is standardised by its own mean and standard
  deviation (population, plus 1e-6 under the root).
* Modes: the k lowest cosine modes of the homogeneous element,
  c_j(x, y, z) = cos(pi p_j (x + 1/2) / 8) cos(pi q_j (y + 1/2) / 8)
  cos(pi r_j (z + 1/2) / 8) with (p_j, q_j, r_j) from MODES, evaluated on
  the patch grid (cell coordinates -1 .. 8) and on the element (0 .. 7).
  They are the start block of the cold eigensolve; the network predicts a
  correction to them.
* Network: three 3x3x3 cross-correlations with biases,
    a1 = relu(conv([patch, c_0..c_{k-1}], W1, b1))   1+k -> 32 channels, 10^3 -> 8^3
    a2 = relu(conv(a1, W2, b2))                      32 -> 32 channels, zero padding 1
    X  = c + conv(a2, W3, b3)                        32 -> k channels, zero padding 1
  X (k x 512) holds k cell vectors of K.  Weights are W[o, i, dz, dy, dx].
* Loss of one element, with S the weight diagonal on K normalised to mean 1
  and Phi the k target eigenvectors scaled so that Phi^T S Phi = I:
    C* = (X S X^T)^-1 X S Phi,  loss = || Phi - X^T C* ||_S^2,
  the S-distance of Phi from span(X); it does not change when X is replaced
  by G X (G invertible) or Phi by Phi Q (Q orthogonal).  Because C* minimises
  the inner problem, the gradient is dloss/dX = -2 C* (S (Phi - X^T C*))^T
  (envelope theorem).  The batch loss is the mean over elements.
"""
from __future__ import annotations

import numpy as np

CHANNELS = 32
PATCH = 10
EDGE = 8

# (p, q, r) of the lowest cosine modes of an 8^3 block, by increasing
# p^2 + q^2 + r^2; ties: x before y before z
MODES = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1)]


def mode_grid(j: int, first: int, size: int) -> np.ndarray:
    """Mode j on the cells first .. first+size-1 of each axis, shape (size,)*3 (z, y, x)."""
    p, q, r = MODES[j]
    t = (np.arange(first, first + size) + 0.5) * np.pi / EDGE
    cx, cy, cz = np.cos(p * t), np.cos(q * t), np.cos(r * t)
    return cz[:, None, None] * cy[None, :, None] * cx[None, None, :]


def param_shapes(k: int):
    return [("W1", (CHANNELS, 1 + k, 3, 3, 3)), ("b1", (CHANNELS,)),
            ("W2", (CHANNELS, CHANNELS, 3, 3, 3)), ("b2", (CHANNELS,)),
            ("W3", (k, CHANNELS, 3, 3, 3)), ("b3", (k,))]


def unflatten(theta: np.ndarray, k: int) -> dict:
    """Parameters from the flat vector in the order W1, b1, W2, b2, W3, b3."""
    out, o = {}, 0
    for name, shp in param_shapes(k):
        size = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + size], dtype=np.float64).reshape(shp)
        o += size
    assert o == theta.size
    return out


def flatten(p: dict, k: int) -> np.ndarray:
    return np.concatenate([p[name].reshape(-1) for name, _ in param_shapes(k)])


def n_params(k: int) -> int:
    return sum(int(np.prod(s)) for _, s in param_shapes(k))


def patches(perm: np.ndarray) -> np.ndarray:
    """Standardised log-permeability patches of every 8^3 element,
    shape (m, 10, 10, 10), elements in x-fastest order."""
    nz, ny, nx = perm.shape
    lk = np.log(perm)
    padded = np.pad(lk, 1, mode="edge")
    ez, ey, ex = nz // EDGE, ny // EDGE, nx // EDGE
    out = np.empty((ez * ey * ex, PATCH, PATCH, PATCH))
    e = 0
    for kz in range(ez):
        for ky in range(ey):
            for kx in range(ex):
                p = padded[kz * EDGE:kz * EDGE + PATCH, ky * EDGE:ky * EDGE + PATCH, kx * EDGE:kx * EDGE + PATCH]
                mu = p.mean()
                sd = np.sqrt(((p - mu) ** 2).mean() + 1e-6)
                out[e] = (p - mu) / sd
                e += 1
    return out


def conv(x: np.ndarray, w: np.ndarray, b: np.ndarray, pad: int) -> np.ndarray:
    """3x3x3 cross-correlation: y[o] = b[o] + sum_i sum_d w[o,i,d] x[i, . + d]."""
    if pad:
        x = np.pad(x, ((0, 0), (pad, pad), (pad, pad), (pad, pad)))
    n = x.shape[1] - 2
    y = np.broadcast_to(b[:, None, None, None], (w.shape[0], n, n, n)).copy()
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                y += np.tensordot(w[:, :, dz, dy, dx], x[:, dz:dz + n, dy:dy + n, dx:dx + n], axes=(1, 0))
    return y


def conv_backward(x: np.ndarray, w: np.ndarray, gy: np.ndarray, pad: int):
    """Gradients of conv(x, w, b, pad) given dL/dy: (dL/dx, dL/dw, dL/db)."""
    xp = np.pad(x, ((0, 0), (pad, pad), (pad, pad), (pad, pad))) if pad else x
    n = gy.shape[1]
    gxp = np.zeros_like(xp)
    gw = np.zeros_like(w)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                win = (slice(None), slice(dz, dz + n), slice(dy, dy + n), slice(dx, dx + n))
                gxp[win] += np.tensordot(w[:, :, dz, dy, dx], gy, axes=(0, 0))
                gw[:, :, dz, dy, dx] = np.tensordot(gy, xp[win], axes=([1, 2, 3], [1, 2, 3]))
    gx = gxp[:, pad:-pad, pad:-pad, pad:-pad] if pad else gxp
    return gx, gw, gy.sum(axis=(1, 2, 3))


def network_input(patch: np.ndarray, k: int) -> np.ndarray:
    """The patch and the k mode channels on the patch grid, shape (1+k, 10, 10, 10)."""
    return np.stack([patch] + [mode_grid(j, -1, PATCH) for j in range(k)])


def forward(p: dict, patch: np.ndarray):
    """Network output X (k x 512) and the activations the backward pass needs."""
    k = p["W3"].shape[0]
    x0 = network_input(patch, k)
    z1 = conv(x0, p["W1"], p["b1"], 0)
    a1 = np.maximum(z1, 0.0)
    z2 = conv(a1, p["W2"], p["b2"], 1)
    a2 = np.maximum(z2, 0.0)
    x = conv(a2, p["W3"], p["b3"], 1)
    base = np.stack([mode_grid(j, 0, EDGE) for j in range(k)])
    return (x + base).reshape(k, -1), (x0, z1, a1, z2, a2)


def backward(p: dict, patch: np.ndarray, cache, gX: np.ndarray) -> dict:
    """Parameter gradients from dL/dX (k x 512)."""
    x0, z1, a1, z2, a2 = cache
    k = gX.shape[0]
    g3 = gX.reshape(k, EDGE, EDGE, EDGE)
    ga2, gW3, gb3 = conv_backward(a2, p["W3"], g3, 1)
    gz2 = ga2 * (z2 > 0)
    ga1, gW2, gb2 = conv_backward(a1, p["W2"], gz2, 1)
    gz1 = ga1 * (z1 > 0)
    _, gW1, gb1 = conv_backward(x0, p["W1"], gz1, 0)
    return {"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "W3": gW3, "b3": gb3}


def subspace_loss(X: np.ndarray, phi: np.ndarray, s: np.ndarray):
    """Loss and dloss/dX for one element.

    X: (k, 512) network output; phi: (512, k) target eigenvectors with
    phi^T diag(s) phi = I; s: (512,) weight diagonal of the element.
    """
    m = s.mean()
    sb = s / m
    pb = phi * np.sqrt(m)
    G = (X * sb) @ X.T
    B = (X * sb) @ pb
    C = np.linalg.solve(G, B)
    R = pb - X.T @ C
    loss = float(np.sum(sb[:, None] * R * R))
    gX = -2.0 * C @ (sb[:, None] * R).T
    return loss, gX


def batch_loss_and_grad(theta: np.ndarray, k: int, patch_batch, phi_batch, s_batch):
    """Mean loss over a batch of elements and its gradient w.r.t. theta."""
    p = unflatten(theta, k)
    total = 0.0
    grads = {name: np.zeros(shp) for name, shp in param_shapes(k)}
    m = len(patch_batch)
    for patch, phi, s in zip(patch_batch, phi_batch, s_batch):
        X, cache = forward(p, patch)
        loss, gX = subspace_loss(X, phi, s)
        total += loss / m
        g = backward(p, patch, cache, gX / m)
        for name in grads:
            grads[name] += g[name]
    return total, flatten(grads, k)
