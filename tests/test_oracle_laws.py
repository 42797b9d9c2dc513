"""Pins of the oracle's non-linear elastic (Sec. 4.1) and visco-plastic
(Sec. 4.3) laws and of the per-voxel law dispatch, by closed forms, scalar
relations solved with an independent root finder, finite differences and,
at the solve level, the two-phase laminate of Sec. 5.1 (uniform sigma_12,
per-layer eps_12 from each layer's own shear response)."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import synth
from oracle import j2, laws, solver as S

G0, K0 = 0.386, 0.833
# Sec. 5.1 table: non-linear elasticity sigma_0/G 0.5, eps_0 0.1, n 10;
# visco-plasticity sigma_0/G 0.1, eps_0 0.1, t_0 0.1, n 0.3
NLE = (K0, G0, 0.5 * G0, 0.0, 10.0, laws.LAW_NONLINEAR_ELASTIC, 0.1, 1.0)
VIS = (K0, G0, 0.1 * G0, 0.0, 0.3, laws.LAW_VISCO, 0.1, 0.1)
ELASTIC = (K0, G0, 1e30, 0.0, 1.0)        # never yields: linear elastic phase 2


def sym(A):
    return 0.5 * (A + A.T)


def pt(law_fn, eps, *args):
    e = np.asarray(eps, dtype=float).reshape(3, 3, 1)
    return law_fn(e, *[np.array([a], dtype=float) if np.isscalar(a) else a for a in args])


def nle_point(eps, mat):
    K, _, s0, _, n, _, e0, _ = mat
    s, C = pt(laws.nonlinear_elastic, eps, K, s0, e0, n)
    return s[..., 0], C[..., 0]


def vis_point(eps, ept, ebt, mat, dt):
    K, G, s0, _, n, _, e0, t0 = mat
    e = np.asarray(eps, dtype=float).reshape(3, 3, 1)
    s, C, ep, eb, fl = laws.visco_return_map(e, np.asarray(ept, dtype=float).reshape(3, 3, 1),
                                             np.array([ebt]), np.array([K]), np.array([G]), np.array([s0]),
                                             np.array([e0]), np.array([t0]), np.array([n]), dt)
    return s[..., 0], C[..., 0], ep[..., 0], float(eb[0])


def fd_tangent(stress, eps, h=1e-8):
    Cfd = np.zeros((3, 3, 3, 3))
    for l in range(3):
        for m in range(3):
            d = np.zeros((3, 3))
            d[l, m] += 0.5 * h
            d[m, l] += 0.5 * h
            Cfd[:, :, l, m] = (stress(eps + d) - stress(eps - d)) / (2.0 * h)
    return Cfd


@pytest.mark.parametrize("n", [10.0, 3.0, 1.0])
@pytest.mark.parametrize("gamma", [0.001, 0.02, 0.05])
def test_nonlinear_elastic_pure_shear_closed_form(n, gamma):
    """eps = gamma (e1 e2 + e2 e1): eps_d = eps, eps_eq = 2 gamma / sqrt(3),
    N_12 = 1/sqrt(3), so sigma_12 = sigma_0 (2 gamma / (sqrt(3) eps_0))^n / sqrt(3)
    and every other stress component vanishes (by hand from Eq. model:nlin:stress)."""
    mat = NLE[:4] + (n,) + NLE[5:]
    eps = np.zeros((3, 3))
    eps[0, 1] = eps[1, 0] = gamma
    s, _ = nle_point(eps, mat)
    tau = mat[2] * (2.0 * gamma / (math.sqrt(3.0) * mat[6])) ** n / math.sqrt(3.0)
    assert abs(s[0, 1] - tau) <= 1e-14 * tau
    off = s.copy()
    off[0, 1] = off[1, 0] = 0.0
    assert np.max(np.abs(off)) <= 1e-16 * tau


def test_nonlinear_elastic_volumetric_and_zero_strain():
    a = 1e-3
    s, C = nle_point(a * np.eye(3), NLE)
    assert np.max(np.abs(s - 3.0 * K0 * a * np.eye(3))) < 1e-18
    # zero strain: tangent K I(x)I (n > 1), plus 2/3 sigma_0/eps_0 I_d for n = 1
    _, C0 = nle_point(np.zeros((3, 3)), NLE)
    assert np.max(np.abs(C0 - K0 * j2.II)) < 1e-15
    lin = NLE[:4] + (1.0,) + NLE[5:]
    _, C1 = nle_point(np.zeros((3, 3)), lin)
    assert np.max(np.abs(C1 - (K0 * j2.II + 2.0 / 3.0 * lin[2] / lin[6] * j2.I4D))) < 1e-15


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("n", [10.0, 1.0, 2.5])
def test_nonlinear_elastic_tangent_matches_finite_differences(seed, n):
    mat = NLE[:4] + (n,) + NLE[5:]
    rng = np.random.default_rng(seed)
    eps = sym(rng.standard_normal((3, 3))) * 0.03
    _, C = nle_point(eps, mat)
    Cfd = fd_tangent(lambda e: nle_point(e, mat)[0], eps)
    assert np.max(np.abs(C - Cfd)) <= 1e-6 * np.max(np.abs(C))
    assert np.max(np.abs(C - C.transpose(2, 3, 0, 1))) < 1e-14 * np.max(np.abs(C))


@pytest.mark.parametrize("gamma", [1e-4, 0.002, 0.01])
@pytest.mark.parametrize("dt", [1e-3, 0.1])
def test_visco_pure_shear_one_step(gamma, dt):
    """From the virgin state in one time step dt: the trial equivalent
    stress is sqrt(3) 2 G gamma, the stress after the step is
    tau = (sigma_eq_tr - 3G dgamma) / sqrt(3) with dgamma from the implicit
    equation of Sec. 4.3, solved here by brentq; the plastic shear strain is
    sqrt(3)/2 dgamma and Norton's rule holds with the final stress."""
    K, G, s0, _, n, _, e0, t0 = VIS
    eps = np.zeros((3, 3))
    eps[0, 1] = eps[1, 0] = gamma
    s, C, ep, eb = vis_point(eps, np.zeros((3, 3)), 0.0, VIS, dt)
    seq_tr = math.sqrt(3.0) * 2.0 * G * gamma
    g0dt = e0 / t0 * dt
    dg = brentq(lambda x: x - g0dt * ((seq_tr - 3.0 * G * x) / s0) ** (1.0 / n), 0.0, seq_tr / (3.0 * G),
                xtol=1e-22, rtol=1e-15)
    tau = (seq_tr - 3.0 * G * dg) / math.sqrt(3.0)
    assert abs(eb - dg) <= 1e-12 * dg
    assert abs(s[0, 1] - tau) <= 1e-12 * tau
    assert abs(ep[0, 1] - 0.5 * math.sqrt(3.0) * dg) <= 1e-12 * dg
    # Norton's rule with the stress at the end of the step (backward Euler)
    assert abs(eb / dt - e0 / t0 * (math.sqrt(3.0) * s[0, 1] / s0) ** (1.0 / n)) <= 1e-9 * eb / dt


@pytest.mark.parametrize("seed", range(5))
def test_visco_equation_residual_and_tangent(seed):
    rng = np.random.default_rng(seed)
    eps = sym(rng.standard_normal((3, 3))) * 0.01
    ept = sym(rng.standard_normal((3, 3))) * 1e-3
    ept -= np.trace(ept) / 3.0 * np.eye(3)
    dt = 1e-3
    s, C, ep, eb = vis_point(eps, ept, 0.01, VIS, dt)
    K, G, s0, _, n, _, e0, t0 = VIS
    dg = eb - 0.01
    sd = s - np.trace(s) / 3.0 * np.eye(3)
    seq = math.sqrt(1.5 * np.sum(sd * sd))
    # the implicit equation at the solution, through the returned stress
    assert abs(dg - e0 / t0 * dt * (seq / s0) ** (1.0 / n)) <= 1e-12 * dg
    assert abs(np.trace(ep - ept)) < 1e-16
    Cfd = fd_tangent(lambda e: vis_point(e, ept, 0.01, VIS, dt)[0], eps)
    assert np.max(np.abs(C - Cfd)) <= 1e-6 * np.max(np.abs(C))
    assert np.max(np.abs(C - C.transpose(2, 3, 0, 1))) < 1e-14 * np.max(np.abs(C))


def test_dispatch_matches_each_law_voxel_by_voxel():
    shape = (5, 3, 3)
    ph = np.arange(np.prod(shape)).reshape(shape) % 4
    mats = [synth.SOFT, NLE, VIS, (K0, G0, 0.003, 0.004, 0.2)]
    eps = synth.random_sym_tensor_field(shape, 1, 0.01)
    ept = synth.random_sym_tensor_field(shape, 2, 1e-3)
    tr = np.einsum("ii...->...", ept)
    for i in range(3):
        ept[i, i] -= tr / 3.0
    ebt = np.random.default_rng(3).uniform(0.0, 2e-3, shape)
    sig, C, ep, eb, _ = laws.constitutive(ph, mats, eps, ept, ebt, dt=1e-3)
    for idx in np.ndindex(shape):
        m = mats[ph[idx]]
        e = eps[(slice(None), slice(None)) + idx]
        if len(m) == 5:
            s_ref, C_ref, ep_ref, eb_ref, _ = j2.point_response(e, ept[(slice(None), slice(None)) + idx], ebt[idx], m)
        elif m[5] == laws.LAW_NONLINEAR_ELASTIC:
            s_ref, C_ref = nle_point(e, m)
            ep_ref, eb_ref = ept[(slice(None), slice(None)) + idx], ebt[idx]
        else:
            s_ref, C_ref, ep_ref, eb_ref = vis_point(e, ept[(slice(None), slice(None)) + idx], ebt[idx], m, 1e-3)
        sl = (slice(None), slice(None)) + idx
        assert np.max(np.abs(sig[sl] - s_ref)) <= 1e-15 * np.max(np.abs(s_ref))
        assert np.max(np.abs(ep[sl] - ep_ref)) <= 1e-17 and abs(eb[idx] - eb_ref) <= 1e-17
        assert np.max(np.abs(C[(slice(None),) * 4 + idx] - C_ref)) <= 1e-15 * np.max(np.abs(C_ref))


# ------------------------------------------------------------- laminate solves
def _laminate(n, mat):
    """n x n x 1 laminate: layers normal to x, phase 1 (the law) where the
    x index is below 4, phase 0 linear elastic."""
    ph = np.zeros((n, n, 1), np.uint8)
    ph[:4] = 1
    return ph, [ELASTIC, mat], 4.0 / n


def test_laminate_nonlinear_elastic_closed_form():
    """Sec. 5.1 with the non-linear elastic phase, one increment to E_12 = 0.05
    with Algorithm 1 as printed: sigma_12 is uniform and eps_12 piecewise
    constant, with f eps_12^nle(tau) + (1 - f) tau / 2G = E_12 and
    eps_12^nle(tau) = sqrt(3)/2 eps_0 (sqrt(3) tau / sigma_0)^(1/n) (inverse of
    the pure-shear closed form)."""
    ph, mats, f = _laminate(11, NLE)
    s = S.Solver(ph, mats, 1e-6, 1e-12, predictor="none")
    st = s.solve_increment(synth.shear_xy(0.05))
    assert st.converged
    _, _, s0, _, n, _, e0, _ = NLE
    e_nle = lambda t: 0.5 * math.sqrt(3.0) * e0 * (math.sqrt(3.0) * t / s0) ** (1.0 / n)
    tau = brentq(lambda t: f * e_nle(t) + (1 - f) * t / (2 * G0) - 0.05, 1e-12, 1.0, xtol=1e-20, rtol=1e-15)
    assert abs(st.Sigma[0, 1] - tau) <= 1e-9 * tau
    eps = s.strain()
    assert np.max(np.abs(eps[0, 1][ph == 1] - e_nle(tau))) <= 1e-9 * 0.05
    assert np.max(np.abs(eps[0, 1][ph == 0] - tau / (2 * G0))) <= 1e-9 * 0.05
    print("nonlinear elastic laminate Newton residuals", st.newton_res)


def test_laminate_power_law_plasticity_closed_form():
    """Sec. 5.1's elasto-plastic column (H/G 0.05, sigma_0/G 0.01, n 0.1), one
    increment to E_12 = 0.05 with Algorithm 1 as printed; per-layer response
    eps_12^pl(tau) = tau/2G + sqrt(3)/2 ((sqrt(3) tau - sigma_0)/H)^(1/n)."""
    mat = (K0, G0, 0.01 * G0, 0.05 * G0, 0.1)
    ph, mats, f = _laminate(11, mat)
    s = S.Solver(ph, mats, 1e-6, 1e-12, predictor="none")
    st = s.solve_increment(synth.shear_xy(0.05))
    assert st.converged
    _, G, s0, H, n = mat
    e_pl = lambda t: t / (2 * G) + (0.5 * math.sqrt(3.0) * ((math.sqrt(3.0) * t - s0) / H) ** (1.0 / n)
                                    if math.sqrt(3.0) * t > s0 else 0.0)
    tau = brentq(lambda t: f * e_pl(t) + (1 - f) * t / (2 * G0) - 0.05, 1e-12, 1.0, xtol=1e-20, rtol=1e-15)
    assert abs(st.Sigma[0, 1] - tau) <= 1e-9 * tau
    eps = s.strain()
    assert np.max(np.abs(eps[0, 1][ph == 1] - e_pl(tau))) <= 1e-9 * 0.05
    print("power-law laminate Newton residuals", st.newton_res)


def test_laminate_visco_plastic_against_scalar_recursion():
    """Sec. 5.1's visco-plastic column, E_12 ramped to 0.05 in equal
    increments of dt = 1e-3 (20 of the paper's 200 steps here).  In the
    laminate sigma_12 = tau is uniform; in the visco-plastic layers backward
    Euler with the stress at the end of the step gives dgamma =
    gamma_0 dt (sqrt(3) tau / sigma_0)^(1/n) and eps_12 = tau/2G + eps_p12 with
    eps_p12 += sqrt(3)/2 dgamma, so every step is a scalar equation in tau,
    solved here by brentq."""
    ph, mats, f = _laminate(11, VIS)
    n_inc, dt = 20, 1e-3
    s = S.Solver(ph, mats, 1e-6, 1e-12, dt=dt)
    _, _, s0, _, n, _, e0, t0 = VIS
    epl = 0.0
    for k in range(1, n_inc + 1):
        E12 = 0.05 * k / 200
        st = s.solve_increment(synth.shear_xy(E12))
        assert st.converged
        dg = lambda t: e0 / t0 * dt * (math.sqrt(3.0) * t / s0) ** (1.0 / n)
        tau = brentq(lambda t: f * (t / (2 * G0) + epl + 0.5 * math.sqrt(3.0) * dg(t)) + (1 - f) * t / (2 * G0)
                     - E12, 0.0, 1.0, xtol=1e-22, rtol=1e-15)
        epl += 0.5 * math.sqrt(3.0) * dg(tau)
        assert abs(st.Sigma[0, 1] - tau) <= 1e-9 * tau
    eps = s.strain()
    assert np.max(np.abs(eps[0, 1][ph == 1] - (tau / (2 * G0) + epl))) <= 1e-9 * E12
    print("visco laminate Newton residuals (last increment)", st.newton_res)
