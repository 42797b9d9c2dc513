"""Pins of the oracle's projection operator against what the mathematics fixes.

None of these checks re-types the G^ formula: compatible fields are built as
symmetric gradients of periodic displacements, equilibrated fields as
divergence-free spectra, and the dense matrices from the DFT definition of
Appendix B.
"""
import numpy as np
import pytest

import synth
from oracle import projection as P

SHAPES = [(5, 5, 5), (3, 5, 7), (7, 3, 5), (9, 9, 9)]


def _fft(a):
    return np.fft.fftn(a, axes=(-3, -2, -1))


def _ifft(a):
    return np.fft.ifftn(a, axes=(-3, -2, -1)).real


def compatible_field(shape, seed):
    """eps = sym grad u for a random periodic trigonometric displacement u."""
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((3,) + shape)
    uh = _fft(u)
    k = np.stack(np.meshgrid(*[np.fft.fftfreq(n) * n for n in shape], indexing="ij"))
    # d/dx_j of exp(2 pi i k.x / N) is 2 pi i k_j / N; keep the physical scaling
    g = 2j * np.pi * k / np.array(shape, dtype=float).reshape(3, 1, 1, 1)
    eh = 0.5 * (g[:, None] * uh[None, :] + g[None, :] * uh[:, None])
    return _ifft(eh)


def equilibrated_field(shape, seed):
    """Zero-mean divergence-free symmetric field: sigma^(k) xi = 0 for k != 0."""
    rng = np.random.default_rng(seed)
    S = synth.random_sym_tensor_field(shape, seed)
    Sh = _fft(S)
    k = np.stack(np.meshgrid(*[np.fft.fftfreq(n) * n for n in shape], indexing="ij"))
    xi = k / np.array(shape, dtype=float).reshape(3, 1, 1, 1)
    n = np.sqrt(np.sum(xi * xi, axis=0))
    q = xi / np.where(n == 0, 1.0, n)
    Pm = np.eye(3).reshape(3, 3, 1, 1, 1) - q[:, None] * q[None, :]
    sh = np.einsum("ij...,jk...,kl...->il...", Pm, Sh, Pm)
    sh[..., 0, 0, 0] = 0.0
    out = _ifft(sh)
    # divergence in Fourier space vanishes by construction; check it here
    div = np.einsum("ij...,j...->i...", _fft(out), xi)
    assert np.max(np.abs(div)) < 1e-10 * max(1.0, np.max(np.abs(sh)))
    del rng
    return out


@pytest.mark.parametrize("shape", SHAPES)
def test_G_keeps_compatible_fields(shape):
    e = compatible_field(shape, 1)
    assert np.max(np.abs(np.mean(e, axis=(2, 3, 4)))) < 1e-13
    g = P.apply_G(e)
    assert np.max(np.abs(g - e)) <= 1e-12 * np.max(np.abs(e))


@pytest.mark.parametrize("shape", SHAPES)
def test_G_annihilates_equilibrated_and_constant_fields(shape):
    s = equilibrated_field(shape, 2)
    T0 = synth.random_sym_tensor_field((1, 1, 1), 3)
    g = P.apply_G(s + T0)
    assert np.max(np.abs(g)) <= 1e-12 * np.max(np.abs(s))


@pytest.mark.parametrize("shape", SHAPES)
def test_G_is_the_orthogonal_projection_onto_compatible_fields(shape):
    e = compatible_field(shape, 4)
    s = equilibrated_field(shape, 5)
    T0 = synth.random_sym_tensor_field((1, 1, 1), 6)
    tau = e + s + T0
    g = P.apply_G(tau)
    assert np.max(np.abs(g - e)) <= 1e-12 * np.max(np.abs(tau))
    # orthogonality of the two parts under the trapezoidal inner product
    assert abs(np.sum(e * s)) <= 1e-12 * np.sqrt(np.sum(e * e) * np.sum(s * s))


@pytest.mark.parametrize("shape", [(5, 5, 5), (3, 5, 7)])
def test_ghat_projection_properties(shape):
    G = P.ghat(shape)
    GG = np.einsum("ijab...,ablm...->ijlm...", G, G)
    assert np.max(np.abs(GG - G)) < 1e-14
    assert np.max(np.abs(G - G.transpose(2, 3, 0, 1, 4, 5, 6))) < 1e-15
    assert np.max(np.abs(G - G.transpose(1, 0, 2, 3, 4, 5, 6))) < 1e-15
    assert np.max(np.abs(G - G.transpose(0, 1, 3, 2, 4, 5, 6))) < 1e-15
    assert np.all(G[..., 0, 0, 0] == 0.0)
    # trace of a projection = its rank: 3 compatible modes out of 6 per k != 0
    M = P.mandel_block(G).reshape(6, 6, -1)
    tr = np.einsum("aa...->...", M)
    assert tr[0] == 0.0
    assert np.max(np.abs(tr[1:] - 3.0)) < 1e-13


@pytest.mark.parametrize("shape", [(5, 5, 5), (3, 5, 7)])
def test_gamma_ref_of_unit_tensor_is_G(shape):
    from oracle.j2 import I4S
    Gam = P.gamma_ref_hat(shape, I4S)
    G = P.ghat(shape)
    assert np.max(np.abs(Gam - G)) < 1e-14


def test_gamma_ref_inverts_reference_stiffness_on_compatible_fields():
    from oracle.j2 import elastic_stiffness
    shape = (5, 7, 3)
    C = elastic_stiffness(0.833, 0.386)
    e = compatible_field(shape, 7)
    out = P.apply_gamma_ref(np.einsum("ijlm,lm...->ij...", C, e), C)
    assert np.max(np.abs(out - e)) <= 1e-12 * np.max(np.abs(e))


@pytest.mark.parametrize("shape", [(3, 3, 3), (5, 5, 5), (3, 5, 7)])
def test_dense_matrix_from_dft_definition_matches_fft_path(shape):
    from oracle.dense import column_to_field, field_to_column
    Gd, K = P.dense_G(shape)
    assert np.max(np.abs(Gd.imag)) < 1e-12
    Gr = Gd.real
    assert np.max(np.abs(Gr - Gr.T)) < 1e-12
    assert np.max(np.abs(Gr @ Gr - Gr)) < 1e-11
    tau = synth.random_sym_tensor_field(shape, 8)
    c = field_to_column(tau, K)
    d = column_to_field(Gr @ c, K, shape)
    assert np.max(np.abs(d - P.apply_G(tau))) <= 1e-12 * np.max(np.abs(tau))
    # F^-1 = |N| F^H (Sec. 2.3, Eq. discrete_projection)
    F, Finv, _ = P.dense_dft(shape)
    n = F.shape[0]
    assert np.max(np.abs(Finv - n * F.conj().T)) < 1e-12
    assert np.max(np.abs(Finv @ F - np.eye(n))) < 1e-12


@pytest.mark.parametrize("shape", [(5, 5, 5), (3, 5, 7)])
def test_curvature_along_compatible_direction_needs_no_projection(shape):
    """p.G(C:p) = (G p).(C:p) = p.(C:p) for compatible p, G being a symmetric
    projection: the CG denominator p.Ap can be taken before the transforms.
    The consistent tangent C is a plastic one of the oracle's return map; a
    direction with an equilibrated part must break the identity."""
    from oracle import j2
    phase = synth.bernoulli(shape, 0.4, 3)
    K, G, sy0, H, _ = j2.material_fields(phase, [synth.SOFT, synth.HARD])
    E = np.diag([0.004, -0.002, -0.002])  # about 60 % of the voxels yield
    eps = E[:, :, None, None, None] + 0.0003 * compatible_field(shape, 10)
    _, C, _, _, plastic = j2.return_map(eps, np.zeros_like(eps), np.zeros(shape), K, G, sy0, H)
    assert plastic.any() and not plastic.all()
    p = compatible_field(shape, 11)
    Cp = j2.ddot42(C, p)
    lhs, rhs = np.sum(p * P.apply_G(Cp)), np.sum(p * Cp)
    assert rhs > 0 and abs(lhs - rhs) <= 1e-12 * rhs
    q = p + equilibrated_field(shape, 12)
    Cq = j2.ddot42(C, q)
    assert abs(np.sum(q * P.apply_G(Cq)) - np.sum(q * Cq)) > 1e-3 * np.sum(q * Cq)


def test_even_grid_rejected():
    with pytest.raises(ValueError):
        P.int_freq(4)
