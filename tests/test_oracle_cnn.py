"""Pins of the FP64 reference network and loss of the learned warm start.

The convolution is checked against the convolution sum written as explicit
loops and against the identity kernel; gradients against central finite
differences; the loss against its invariances and its zero set.
"""
import numpy as np
import pytest

from oracle import cnn
from synth.fields import make_field


def _params(k, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(cnn.n_params(k)) * scale


def _brute_conv(x, w, b, pad):
    ci, n = x.shape[0], x.shape[1]
    xp = np.zeros((ci, n + 2 * pad, n + 2 * pad, n + 2 * pad))
    xp[:, pad:pad + n, pad:pad + n, pad:pad + n] = x
    no = n + 2 * pad - 2
    y = np.zeros((w.shape[0], no, no, no))
    for o in range(w.shape[0]):
        for z in range(no):
            for yy in range(no):
                for xx in range(no):
                    acc = b[o]
                    for i in range(ci):
                        for dz in range(3):
                            for dy in range(3):
                                for dx in range(3):
                                    acc += w[o, i, dz, dy, dx] * xp[i, z + dz, yy + dy, xx + dx]
                    y[o, z, yy, xx] = acc
    return y


@pytest.mark.parametrize("pad", [0, 1])
def test_conv_equals_convolution_sum(pad):
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 5, 5))
    w = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    assert np.allclose(cnn.conv(x, w, b, pad), _brute_conv(x, w, b, pad), atol=1e-12)


def test_identity_kernel():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 6, 6, 6))
    w = np.zeros((1, 1, 3, 3, 3))
    w[0, 0, 1, 1, 1] = 1.0
    assert np.array_equal(cnn.conv(x, w, np.zeros(1), 1), x)
    # valid mode keeps the interior
    assert np.array_equal(cnn.conv(x, w, np.zeros(1), 0), x[:, 1:-1, 1:-1, 1:-1])


def test_conv_backward_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 4, 4, 4))
    w = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    gy = rng.standard_normal((3, 4, 4, 4))
    gx, gw, gb = cnn.conv_backward(x, w, gy, 1)
    f = lambda xx, ww, bb: float(np.sum(cnn.conv(xx, ww, bb, 1) * gy))
    eps = 1e-6
    for idx in [(0, 1, 2, 3), (1, 0, 0, 0), (1, 3, 3, 3)]:
        d = np.zeros_like(x)
        d[idx] = eps
        assert abs((f(x + d, w, b) - f(x - d, w, b)) / (2 * eps) - gx[idx]) < 1e-7 * (1 + abs(gx[idx]))
    for idx in [(0, 0, 0, 0, 0), (2, 1, 1, 2, 0), (1, 1, 2, 2, 2)]:
        d = np.zeros_like(w)
        d[idx] = eps
        assert abs((f(x, w + d, b) - f(x, w - d, b)) / (2 * eps) - gw[idx]) < 1e-7 * (1 + abs(gw[idx]))
    assert np.allclose(gb, gy.sum(axis=(1, 2, 3)))


def _element_target(seed, k):
    """A random element: weights s and k S-orthonormal columns."""
    rng = np.random.default_rng(seed)
    s = np.exp(rng.uniform(-3, 3, 512))
    q, _ = np.linalg.qr(rng.standard_normal((512, k)))
    phi = q / np.sqrt(s)[:, None]                 # phi^T S phi = q^T q = I
    return s, phi


def test_loss_invariances_and_zero_set():
    k = 4
    s, phi = _element_target(3, k)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((k, 512))
    l0, _ = cnn.subspace_loss(X, phi, s)
    G = rng.standard_normal((k, k)) + 3 * np.eye(k)
    assert abs(cnn.subspace_loss(G @ X, phi, s)[0] - l0) < 1e-9 * l0
    Q, _ = np.linalg.qr(rng.standard_normal((k, k)))
    assert abs(cnn.subspace_loss(X, phi @ Q, s)[0] - l0) < 1e-9 * l0
    # the S-distance of an orthonormal set from a random span lies in [0, k]
    assert 0.0 < l0 < k
    H = rng.standard_normal((k, k)) + 3 * np.eye(k)
    lz, gz = cnn.subspace_loss(H @ phi.T, phi, s)
    assert lz < 1e-20 and np.abs(gz).max() < 1e-10


def test_loss_gradient_finite_differences():
    k = 3
    s, phi = _element_target(5, k)
    X = np.random.default_rng(6).standard_normal((k, 512))
    _, g = cnn.subspace_loss(X, phi, s)
    eps = 1e-6
    for idx in [(0, 0), (1, 100), (2, 511), (0, 300)]:
        d = np.zeros_like(X)
        d[idx] = eps
        fd = (cnn.subspace_loss(X + d, phi, s)[0] - cnn.subspace_loss(X - d, phi, s)[0]) / (2 * eps)
        assert abs(fd - g[idx]) < 1e-6 * (1 + abs(g[idx]))


def test_network_gradient_finite_differences():
    k = 2
    perm = make_field("gauss", 16, 11, sigma=2.0)
    P = cnn.patches(perm)[:2]
    tg = [_element_target(20 + i, k) for i in range(2)]
    S = [t[0] for t in tg]
    PHI = [t[1] for t in tg]
    theta = _params(k, 7, 0.2)
    loss, g = cnn.batch_loss_and_grad(theta, k, P, PHI, S)
    rng = np.random.default_rng(8)
    sizes = [int(np.prod(s)) for _, s in cnn.param_shapes(k)]
    offs = np.cumsum([0] + sizes)
    picks = [int(offs[i] + rng.integers(0, sizes[i])) for i in range(6)]
    eps = 1e-6
    for i in picks:
        d = np.zeros_like(theta)
        d[i] = eps
        fp = cnn.batch_loss_and_grad(theta + d, k, P, PHI, S)[0]
        fm = cnn.batch_loss_and_grad(theta - d, k, P, PHI, S)[0]
        fd = (fp - fm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3), (i, fd, g[i])


def test_patches_standardised_and_edge_replicated():
    perm = make_field("gauss", 16, 12)
    P = cnn.patches(perm)
    assert P.shape == (8, 10, 10, 10)
    assert np.allclose(P.reshape(8, -1).mean(1), 0, atol=1e-12)
    assert np.allclose(P.reshape(8, -1).std(1), 1, atol=1e-4)
    # element 0 touches x = y = z = 0: its halo repeats the boundary cells
    lk = np.log(perm)
    p = lk[:10, :10, :10].copy()
    raw = np.pad(lk, 1, mode="edge")[:10, :10, :10]
    assert np.array_equal(raw[1:, 1:, 1:], lk[:9, :9, :9])
    assert np.array_equal(raw[0, 1:, 1:], lk[0, :9, :9])
    std = (raw - raw.mean()) / np.sqrt(((raw - raw.mean()) ** 2).mean() + 1e-6)
    assert np.allclose(P[0], std)
    del p


def test_modes_are_the_homogeneous_eigenvectors():
    # the mode channels are eigenvectors of the homogeneous 8^3 element's
    # Neumann matrix (closed form of Section 5.2's ladder): checked against
    # the oracle's own level-2 eigensolve, and the zero network returns them
    from oracle import Grid, build_hierarchy
    g = Grid.unit_cube(8)
    h = build_hierarchy(np.ones(g.shape), g, 2, 8, sub=8, workers=1)
    lam = h.level(2).lam[0]
    A = h.A.toarray()
    for j in range(8):
        c = cnn.mode_grid(j, 0, 8).reshape(-1)
        r = A @ c - (A @ c) @ c / (c @ c) * c
        assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(A @ c) + 1e-14
    k = 4
    p = cnn.unflatten(np.zeros(cnn.n_params(k)), k)
    X, _ = cnn.forward(p, np.zeros((10, 10, 10)))
    for j in range(k):
        assert np.allclose(X[j], cnn.mode_grid(j, 0, 8).reshape(-1))
    # halo values continue the cosines
    assert np.allclose(cnn.mode_grid(1, -1, 10)[0, 0, 1:9], np.cos(np.pi * (np.arange(8) + 0.5) / 8))
    del lam


def test_zero_correction_loss_on_homogeneous_element():
    # with a zero correction the network returns the modes, which span the
    # homogeneous element's lowest eigenvectors at the clean cut 4
    from oracle import Grid, build_hierarchy
    g = Grid.unit_cube(8)
    h = build_hierarchy(np.ones(g.shape), g, 2, 4, sub=8, workers=1)
    phi = h.level(2).R.toarray().T
    s = np.full(512, 3.0 * 64)
    k = 4
    X, _ = cnn.forward(cnn.unflatten(np.zeros(cnn.n_params(k)), k), np.zeros((10, 10, 10)))
    loss, _ = cnn.subspace_loss(X, phi[:, :k], s)
    assert loss < 1e-20
