"""Projection operator G and its relatives (test infrastructure; FP64 oracle).

Follows the paper's Sec. 2.2-2.3 and Appendices A-B:

* frequencies: integer k on the reduced (centred) index set of an odd grid,
  scaled frequency xi_i = k_i / L_i (Appendix A, below Eq. FT_projection);
  the cell size is L_i = N_i (unit voxels);
* ``ghat`` -- the four-index G^_ijlm(k) of Eq. (FT_projection), with
  G^(0) = 0 (zero-mean property);
* ``apply_G`` -- [G * tau] at the grid nodes = F^-1 G^ F tau
  (Eqs. projection_xk and discrete_projection), using a library FFT for F;
* ``gamma_ref`` -- the reference Green operator of Eq. (Gamma_explicit)
  built from the acoustic tensor A_il = C_ijlm xi_j xi_m;
* ``dense_*`` -- the explicit DFT matrices F, F^-1 of Appendix B on the
  centred index set and the dense projection matrix G = F^-1 G^ F in
  Mandel form (weights sqrt(2) on shear, as Appendix B does in 2-D).

Pins (tests/test_oracle_projection.py): G keeps every compatible field
(symmetric gradient of a periodic displacement) and annihilates every
equilibrated (divergence-free) field and every constant; G^ is idempotent
and symmetric; Gamma^ref(I_s) = G and Gamma^ref(C) C = identity on
compatible fields; the dense matrices built from the DFT definition agree
with the FFT path.
"""
from __future__ import annotations

import functools

import numpy as np

SQ2 = np.sqrt(2.0)

# Mandel ordering used for dense matrices: 11, 22, 33, 23, 13, 12
MANDEL_PAIRS = ((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))
MANDEL_W = np.array([1.0, 1.0, 1.0, SQ2, SQ2, SQ2])


def int_freq(n: int) -> np.ndarray:
    """Integer frequencies of an odd axis in FFT storage order.

    Storage index m corresponds to frequency k = m for m <= (n-1)/2 and
    k = m - n otherwise, i.e. the centred set -(n-1)/2 .. (n-1)/2 of the
    paper's reduced index set (Sec. 2.3) laid out the way an FFT stores it.
    """
    if n % 2 == 0:
        raise ValueError("odd grid sizes only (paper Sec. 2.3)")
    m = np.arange(n)
    return np.where(m <= (n - 1) // 2, m, m - n)


def scaled_freq(shape, L=None):
    """xi_i(k) = k_i / L_i on the full grid, as three arrays (Appendix A)."""
    if L is None:
        L = tuple(float(s) for s in shape)
    ks = [int_freq(n) / float(Li) for n, Li in zip(shape, L)]
    return np.meshgrid(*ks, indexing="ij")


def ghat(shape, L=None) -> np.ndarray:
    """G^_ijlm(k) of Eq. (FT_projection) on every frequency of the grid.

    Returns an array of shape (3, 3, 3, 3) + shape with G^(0) = 0.
    """
    xi = np.stack(scaled_freq(shape, L))            # (3,) + shape
    n2 = np.sum(xi * xi, axis=0)
    zero = n2 == 0.0
    n2s = np.where(zero, 1.0, n2)
    d = np.eye(3)
    G = np.zeros((3, 3, 3, 3) + tuple(shape))
    for i in range(3):
        for j in range(3):
            for l in range(3):
                for m in range(3):
                    t = 0.5 * (xi[i] * d[j, l] * xi[m] + xi[i] * d[j, m] * xi[l]
                               + xi[j] * d[i, l] * xi[m] + xi[j] * d[i, m] * xi[l]) / n2s
                    t = t - xi[i] * xi[j] * xi[l] * xi[m] / (n2s * n2s)
                    G[i, j, l, m] = np.where(zero, 0.0, t)
    return G


@functools.lru_cache(maxsize=4)
def _ghat_cached(shape):
    return ghat(shape)


def _fft(a, axes):
    try:
        import scipy.fft as sf
        return sf.fftn(a, axes=axes, workers=-1)
    except ImportError:  # pragma: no cover
        return np.fft.fftn(a, axes=axes)


def _ifft(a, axes):
    try:
        import scipy.fft as sf
        return sf.ifftn(a, axes=axes, workers=-1)
    except ImportError:  # pragma: no cover
        return np.fft.ifftn(a, axes=axes)


def apply_operator_hat(Ohat: np.ndarray, tau: np.ndarray, check_imag=True) -> np.ndarray:
    """F^-1 [O^(k) : F tau] for a (3,3,3,3)+shape operator and (3,3)+shape field."""
    axes = (2, 3, 4)
    th = _fft(tau, axes)
    out_h = np.einsum("ijlm...,lm...->ij...", Ohat, th)
    out = _ifft(out_h, axes)
    if check_imag:
        scale = max(float(np.max(np.abs(tau))), 1e-300)
        assert float(np.max(np.abs(out.imag))) <= 1e-10 * scale, "non-real projection"
    return out.real.copy()


def apply_G(tau: np.ndarray) -> np.ndarray:
    """[G * tau] at the grid nodes, Eq. (discrete_projection): F^-1 G^ F tau."""
    shape = tuple(tau.shape[2:])
    return apply_operator_hat(_ghat_cached(shape), tau)


def gamma_ref_hat(shape, C_ref: np.ndarray, L=None) -> np.ndarray:
    """Gamma^ref_ijlm(k) of Eq. (Gamma_explicit) for a constant C_ref (3,3,3,3).

    A_il(k) = sum_jm C_ijlm xi_j xi_m, then
    Gamma_ijlm = 1/4 (A^-1_jm xi_i xi_l + A^-1_jl xi_i xi_m
                      + A^-1_im xi_j xi_l + A^-1_il xi_j xi_m),
    and Gamma(0) = 0.
    """
    xi = np.stack(scaled_freq(shape, L))
    n2 = np.sum(xi * xi, axis=0)
    zero = n2 == 0.0
    A = np.einsum("ijlm,j...,m...->il...", C_ref, xi, xi)
    # invert the 3x3 acoustic tensor at every non-zero frequency
    Am = np.moveaxis(A, (0, 1), (-2, -1)).copy()
    Am[zero] = np.eye(3)
    Ainv = np.moveaxis(np.linalg.inv(Am), (-2, -1), (0, 1))
    Gam = 0.25 * (np.einsum("jm...,i...,l...->ijlm...", Ainv, xi, xi)
                  + np.einsum("jl...,i...,m...->ijlm...", Ainv, xi, xi)
                  + np.einsum("im...,j...,l...->ijlm...", Ainv, xi, xi)
                  + np.einsum("il...,j...,m...->ijlm...", Ainv, xi, xi))
    Gam[..., zero] = 0.0
    return Gam


def apply_gamma_ref(tau: np.ndarray, C_ref: np.ndarray) -> np.ndarray:
    shape = tuple(tau.shape[2:])
    return apply_operator_hat(gamma_ref_hat(shape, C_ref), tau)


# ------------------------------------------------------------------ dense
def centred_indices(n: int) -> np.ndarray:
    """The reduced index set -(n-1)/2 .. (n-1)/2 of an odd axis (Sec. 2.3)."""
    h = (n - 1) // 2
    return np.arange(-h, h + 1)


def dense_dft(shape):
    """Scalar DFT matrices on the centred index set, Appendix B.

    Row/column order: nodes k in C order over the centred sets of the three
    axes.  F = 1/|N| [omega^{-km}], F^-1 = [omega^{km}] with
    omega^{km} = exp(2 pi i sum_a k_a m_a / N_a) (Eq. DFT_def).
    Returns (F, Finv, nodes) where nodes is (|N|, 3) integer centred indices.
    """
    axes = [centred_indices(n) for n in shape]
    K = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    phase = np.zeros((K.shape[0], K.shape[0]))
    for a, n in enumerate(shape):
        phase = phase + np.outer(K[:, a], K[:, a]) / float(n)
    W = np.exp(2j * np.pi * phase)
    nN = K.shape[0]
    return np.conj(W) / nN, W, K


def mandel_block(T4: np.ndarray) -> np.ndarray:
    """6x6 Mandel matrix of a fourth-order tensor with minor symmetries."""
    M = np.empty((6, 6) + T4.shape[4:], dtype=T4.dtype)
    for a, (i, j) in enumerate(MANDEL_PAIRS):
        for b, (l, m) in enumerate(MANDEL_PAIRS):
            M[a, b] = MANDEL_W[a] * MANDEL_W[b] * T4[i, j, l, m]
    return M


def to_mandel(T: np.ndarray) -> np.ndarray:
    """(3,3)+shape symmetric field -> (6,)+shape Mandel field."""
    return np.stack([MANDEL_W[a] * T[i, j] for a, (i, j) in enumerate(MANDEL_PAIRS)])


def from_mandel(v: np.ndarray) -> np.ndarray:
    """(6,)+shape Mandel field -> (3,3)+shape symmetric tensor field."""
    T = np.empty((3, 3) + v.shape[1:], dtype=v.dtype)
    for a, (i, j) in enumerate(MANDEL_PAIRS):
        T[i, j] = v[a] / MANDEL_W[a]
        T[j, i] = T[i, j]
    return T


def dense_G(shape, L=None):
    """Dense G = F^-1 G^ F acting on nodal Mandel columns (Appendix B).

    The column stacks, node by node over the centred index set (C order), the
    six Mandel components.  Returns (G, nodes) with G of size 6|N| x 6|N|
    (complex dtype; its imaginary part vanishes for odd grids).
    """
    F, Finv, K = dense_dft(shape)
    nN = K.shape[0]
    if L is None:
        L = tuple(float(s) for s in shape)
    xi = K / np.asarray(L, dtype=float)[None, :]
    d = np.eye(3)
    Gblk = np.zeros((nN, 6, 6))
    for r in range(nN):
        x = xi[r]
        n2 = float(x @ x)
        if n2 == 0.0:
            continue
        T4 = np.zeros((3, 3, 3, 3))
        for i in range(3):
            for j in range(3):
                for l in range(3):
                    for m in range(3):
                        T4[i, j, l, m] = (0.5 * (x[i] * d[j, l] * x[m] + x[i] * d[j, m] * x[l]
                                                 + x[j] * d[i, l] * x[m] + x[j] * d[i, m] * x[l]) / n2
                                          - x[i] * x[j] * x[l] * x[m] / (n2 * n2))
        Gblk[r] = mandel_block(T4)
    # G = (F^-1 (x) I6) blockdiag(Ghat) (F (x) I6)
    Ghat_big = np.zeros((6 * nN, 6 * nN))
    for r in range(nN):
        Ghat_big[6 * r:6 * r + 6, 6 * r:6 * r + 6] = Gblk[r]
    I6 = np.eye(6)
    G = np.kron(Finv, I6) @ Ghat_big @ np.kron(F, I6)
    return G, K


def nodes_to_storage(K: np.ndarray, shape) -> np.ndarray:
    """Flat C-order storage index (index m = k mod N per axis) of each node."""
    idx = [np.mod(K[:, a], n) for a, n in enumerate(shape)]
    return np.ravel_multi_index(idx, shape)
