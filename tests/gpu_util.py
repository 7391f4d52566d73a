"""Helpers shared by the GPU tests: device tensors, oracle set-ups, subspace angles."""
import numpy as np


def cuda():
    import torch
    return torch.device("cuda:0")


def to_dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=cuda())


def to_host(t):
    return t.detach().cpu().numpy()


def subspace_angle(A, B, S=None):
    """sin of the largest principal angle between span(A) and span(B),
    optionally in the S-inner product (S: diagonal weights)."""
    if S is not None:
        w = np.sqrt(S)[:, None]
        A = A * w
        B = B * w
    qa = np.linalg.qr(A)[0]
    qb = np.linalg.qr(B)[0]
    return float(np.linalg.norm(qb - qa @ (qa.T @ qb), 2))
