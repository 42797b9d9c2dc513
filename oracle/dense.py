"""Dense brute force on tiny grids (test infrastructure; FP64 oracle).

Assembles the matrices of Appendix B explicitly -- DFT matrices on the
centred index set, block-diagonal G^ and C in Mandel form -- and solves one
linearised Newton step (Eq. linear_system) exactly on the compatible
subspace E_N = range(G) (Eq. discrete_spaces):

    d_eps = Q y,   (Q^T C Q) y = -Q^T sigma,

where the columns of Q are an orthonormal basis of the eigenvalue-1
eigenspace of the symmetric projection G.  Sizes up to a few hundred nodes.
"""
from __future__ import annotations

import numpy as np

from .projection import dense_G, mandel_block, nodes_to_storage, to_mandel, from_mandel


def field_to_column(T: np.ndarray, K: np.ndarray) -> np.ndarray:
    """(3,3)+shape field -> Mandel column in the node order K."""
    shape = T.shape[2:]
    v = to_mandel(T).reshape(6, -1)
    idx = nodes_to_storage(K, shape)
    return v[:, idx].T.reshape(-1)


def column_to_field(c: np.ndarray, K: np.ndarray, shape) -> np.ndarray:
    idx = nodes_to_storage(K, shape)
    v = np.zeros((6, int(np.prod(shape))))
    v[:, idx] = c.reshape(-1, 6).T
    return from_mandel(v.reshape((6,) + tuple(shape)))


def tangent_blocks(C: np.ndarray, K: np.ndarray) -> np.ndarray:
    """Block-diagonal Mandel tangent (6|N| x 6|N|) from a (3,3,3,3)+shape field."""
    shape = C.shape[4:]
    M = mandel_block(C).reshape(6, 6, -1)
    idx = nodes_to_storage(K, shape)
    n = K.shape[0]
    out = np.zeros((6 * n, 6 * n))
    for r in range(n):
        out[6 * r:6 * r + 6, 6 * r:6 * r + 6] = M[:, :, idx[r]]
    return out


def compatible_basis(Gd: np.ndarray, tol: float = 1e-8) -> np.ndarray:
    w, V = np.linalg.eigh(0.5 * (Gd + Gd.T))
    return V[:, w > 0.5]


def newton_step_exact(sigma: np.ndarray, C: np.ndarray):
    """Exact solution of G C d = -G sigma with d in E_N on a tiny grid."""
    shape = sigma.shape[2:]
    Gd, K = dense_G(shape)
    assert np.max(np.abs(Gd.imag)) < 1e-10
    Gd = Gd.real
    Q = compatible_basis(Gd)
    s = field_to_column(sigma, K)
    Cd = tangent_blocks(C, K)
    y = np.linalg.solve(Q.T @ Cd @ Q, -(Q.T @ s))
    return column_to_field(Q @ y, K, shape)
