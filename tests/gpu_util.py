"""Test helpers: conversions between the oracle's 3x3 tensor fields and the
library's 6-plane Mandel layout, and device tensor plumbing."""
import math

import numpy as np

SQ2 = math.sqrt(2.0)
PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))
W = (1.0, 1.0, 1.0, SQ2, SQ2, SQ2)


def t2m(T):
    """(3,3)+shape tensor field -> (6,)+shape Mandel planes."""
    return np.stack([W[a] * T[i, j] for a, (i, j) in enumerate(PAIRS)])


def m2t(v):
    v = np.asarray(v)
    T = np.empty((3, 3) + v.shape[1:])
    for a, (i, j) in enumerate(PAIRS):
        T[i, j] = v[a] / W[a]
        T[j, i] = T[i, j]
    return T


def tensor6(E):
    E = np.asarray(E)
    return [E[0, 0], E[1, 1], E[2, 2], E[1, 2], E[0, 2], E[0, 1]]


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_host(t):
    return t.detach().cpu().double().numpy()


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False
