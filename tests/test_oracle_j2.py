"""Pins of the oracle's J2 return mapping (paper Sec. 4.2) by closed forms,
invariants of the model and finite differences."""
import math

import numpy as np
import pytest

from oracle import j2

SOFT = (0.833, 0.386, 0.003, 0.004, 1.0)
HARD = (0.833, 0.386, 0.006, 0.008, 1.0)


def sym(A):
    return 0.5 * (A + A.T)


def test_elastic_branch_is_hookes_law():
    K, G = SOFT[0], SOFT[1]
    rng = np.random.default_rng(0)
    eps = sym(rng.standard_normal((3, 3))) * 1e-4       # far below yield
    s, C, ep, eb, pl = j2.point_response(eps, np.zeros((3, 3)), 0.0, SOFT)
    assert not pl and eb == 0.0 and np.all(ep == 0.0)
    tr = np.trace(eps)
    ref = K * tr * np.eye(3) + 2.0 * G * (eps - tr / 3.0 * np.eye(3))
    assert np.max(np.abs(s - ref)) < 1e-18
    d = np.eye(3)
    Ce = np.zeros((3, 3, 3, 3))
    for i in range(3):
        for jj in range(3):
            for l in range(3):
                for m in range(3):
                    Ce[i, jj, l, m] = ((K - 2.0 * G / 3.0) * d[i, jj] * d[l, m]
                                       + G * (d[i, l] * d[jj, m] + d[i, m] * d[jj, l]))
    assert np.max(np.abs(C - Ce)) < 1e-15


@pytest.mark.parametrize("mat", [SOFT, HARD])
@pytest.mark.parametrize("gamma", [0.003, 0.006, 0.02, 0.05])
def test_pure_shear_closed_form(mat, gamma):
    """eps = gamma (e1 e2 + e2 e1) from the virgin state.

    By hand from Sec. 4.2 with n = 1: tau = sigma_12, sigma_eq = sqrt(3) tau,
    plastic shear eps_p12 = sqrt(3)/2 dgamma and dgamma = (sqrt(3) tau - s0)/H
    on the yield surface, so gamma = tau/(2G) + (3 tau - sqrt(3) s0)/(2H)
    once sqrt(3) 2 G gamma > s0, else tau = 2 G gamma.
    """
    K, G, s0, H, _ = mat
    eps = np.zeros((3, 3))
    eps[0, 1] = eps[1, 0] = gamma
    s, C, ep, eb, pl = j2.point_response(eps, np.zeros((3, 3)), 0.0, mat)
    if math.sqrt(3.0) * 2.0 * G * gamma <= s0:
        tau = 2.0 * G * gamma
        assert not pl
    else:
        tau = (gamma + math.sqrt(3.0) * s0 / (2.0 * H)) / (1.0 / (2.0 * G) + 3.0 / (2.0 * H))
        assert pl
        assert abs(eb - (math.sqrt(3.0) * tau - s0) / H) < 1e-15
    assert abs(s[0, 1] - tau) < 1e-16
    off = s.copy()
    off[0, 1] = off[1, 0] = 0.0
    assert np.max(np.abs(off)) < 1e-18


def _random_state(seed, scale=4e-3):
    rng = np.random.default_rng(seed)
    eps = sym(rng.standard_normal((3, 3))) * scale
    ept = sym(rng.standard_normal((3, 3))) * 1e-3
    ept -= np.trace(ept) / 3.0 * np.eye(3)
    ebt = float(rng.uniform(0.0, 4e-3))
    return eps, ept, ebt


@pytest.mark.parametrize("seed", range(6))
def test_return_lands_on_yield_surface_with_deviatoric_flow(seed):
    eps, ept, ebt = _random_state(seed, 1e-2)
    s, C, ep, eb, pl = j2.point_response(eps, ept, ebt, SOFT)
    assert pl
    sd = s - np.trace(s) / 3.0 * np.eye(3)
    seq = math.sqrt(1.5 * np.sum(sd * sd))
    assert abs(seq - (SOFT[2] + SOFT[3] * eb)) < 1e-15
    assert abs(np.trace(ep - ept)) < 1e-16
    # plastic strain increment has norm sqrt(3/2) dgamma and is coaxial with s
    dep = ep - ept
    assert abs(math.sqrt(2.0 / 3.0 * np.sum(dep * dep)) - (eb - ebt)) < 1e-15
    assert np.max(np.abs(dep - 1.5 * (eb - ebt) * sd / seq)) < 1e-15


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("mat", [SOFT, HARD])
def test_tangent_matches_finite_differences(seed, mat):
    eps, ept, ebt = _random_state(seed)
    s, C, _, _, pl = j2.point_response(eps, ept, ebt, mat)
    h = 1e-7
    Cfd = np.zeros((3, 3, 3, 3))
    for l in range(3):
        for m in range(3):
            d = np.zeros((3, 3))
            d[l, m] += 0.5 * h
            d[m, l] += 0.5 * h
            sp = j2.point_response(eps + d, ept, ebt, mat)[0]
            sm = j2.point_response(eps - d, ept, ebt, mat)[0]
            Cfd[:, :, l, m] = (sp - sm) / (2.0 * h)
    assert np.max(np.abs(C - Cfd)) <= 1e-6 * np.max(np.abs(C))
    assert np.max(np.abs(C - C.transpose(2, 3, 0, 1))) < 1e-15


def test_plastic_tangent_is_positive_definite():
    """Eigenvalues 3K, 2G', 2GH/(3G+H) on symmetric tensors (Sec. 4.2 tangent)."""
    eps, ept, ebt = _random_state(3, 1e-2)
    K, G, s0, H, _ = SOFT
    s, C, _, _, pl = j2.point_response(eps, ept, ebt, SOFT)
    assert pl
    from oracle.projection import mandel_block
    w = np.linalg.eigvalsh(mandel_block(C))
    assert w.min() > 0.0
    assert abs(w.min() - 2.0 * G * H / (3.0 * G + H)) < 1e-14
    assert abs(w.max() - 3.0 * K) < 1e-14


# power-law hardening: the paper's laminate column (H/G 0.05, sigma_0/G 0.01,
# n 0.1; Sec. 5.1 table) with G = 0.386, and the dual-phase steel's n = 0.2
# (Sec. 5.2) on the soft phase
G0 = 0.386
POW = [(0.833, G0, 0.01 * G0, 0.05 * G0, 0.1), (0.833, G0, 0.003, 0.004, 0.2), (0.833, G0, 0.003, 0.004, 0.5)]


def test_exponent_must_be_positive():
    with pytest.raises(ValueError):
        j2.material_fields(np.zeros((3, 3, 3), np.uint8), [(1.0, 1.0, 1.0, 1.0, 0.0)])


@pytest.mark.parametrize("mat", POW)
@pytest.mark.parametrize("gamma", [0.004, 0.01, 0.05])
def test_power_law_pure_shear_by_root_finding(mat, gamma):
    """eps = gamma (e1 e2 + e2 e1) from the virgin state, one step.  On the
    yield surface sqrt(3) tau = sigma_0 + H eps_p_bar^n, and the plastic shear
    is sqrt(3)/2 eps_p_bar (flow along N = 3/2 s / sigma_eq), so
    gamma = tau / 2G + sqrt(3)/2 ((sqrt(3) tau - sigma_0) / H)^(1/n); its root
    in tau is found here by brentq, independently of the oracle's bisection
    of the return equation."""
    from scipy.optimize import brentq
    K, G, s0, H, n = mat
    eps = np.zeros((3, 3))
    eps[0, 1] = eps[1, 0] = gamma
    s, C, ep, eb, pl = j2.point_response(eps, np.zeros((3, 3)), 0.0, mat)
    assert pl
    f = lambda t: t / (2.0 * G) + 0.5 * math.sqrt(3.0) * ((math.sqrt(3.0) * t - s0) / H) ** (1.0 / n) - gamma
    tau = brentq(f, s0 / math.sqrt(3.0) * (1 + 1e-15), 2.0 * G * gamma, xtol=1e-20, rtol=1e-15)
    assert abs(s[0, 1] - tau) <= 1e-13 * tau
    assert abs(eb - ((math.sqrt(3.0) * tau - s0) / H) ** (1.0 / n)) <= 1e-11 * eb
    assert abs(ep[0, 1] - 0.5 * math.sqrt(3.0) * eb) <= 1e-14 * eb


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("mat", POW)
def test_power_law_return_equation_residual_and_yield_surface(seed, mat):
    K, G, s0, H, n = mat
    for ebt in (0.0, 2e-3):   # first yield (eps_p_bar = 0: infinite slope of the hardening term) and later
        eps, ept, _ = _random_state(seed, 5e-2)
        s, C, ep, eb, pl = j2.point_response(eps, ept, ebt, mat)
        assert pl
        sd = s - np.trace(s) / 3.0 * np.eye(3)
        seq = math.sqrt(1.5 * np.sum(sd * sd))
        assert abs(seq - (s0 + H * eb ** n)) <= 1e-14 * seq
        dep = ep - ept
        assert abs(math.sqrt(2.0 / 3.0 * np.sum(dep * dep)) - (eb - ebt)) <= 1e-14 * (eb - ebt)
        assert abs(np.trace(dep)) < 1e-16


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("mat", POW)
def test_power_law_tangent_matches_finite_differences(seed, mat):
    for ebt in (0.0, 2e-3):
        eps, ept, _ = _random_state(seed, 5e-2)
        s, C, _, _, pl = j2.point_response(eps, ept, ebt, mat)
        assert pl
        h = 1e-8
        Cfd = np.zeros((3, 3, 3, 3))
        for l in range(3):
            for m in range(3):
                d = np.zeros((3, 3))
                d[l, m] += 0.5 * h
                d[m, l] += 0.5 * h
                sp = j2.point_response(eps + d, ept, ebt, mat)[0]
                sm = j2.point_response(eps - d, ept, ebt, mat)[0]
                Cfd[:, :, l, m] = (sp - sm) / (2.0 * h)
        assert np.max(np.abs(C - Cfd)) <= 1e-6 * np.max(np.abs(C))
        assert np.max(np.abs(C - C.transpose(2, 3, 0, 1))) < 1e-15


def test_bisection_reproduces_the_linear_closed_form():
    """With n = 1 the return equation is linear: the bisection used for other
    exponents lands on Phi_tr / (3G + H)."""
    rng = np.random.default_rng(5)
    seq = rng.uniform(0.004, 0.02, 50)
    eb = rng.uniform(0.0, 0.01, 50)
    G, s0, H = np.full(50, 0.386), np.full(50, 0.003), np.full(50, 0.004)
    dg = j2.solve_return_equation(seq, eb, G, s0, H, np.ones(50))
    ref = (seq - s0 - H * eb) / (3.0 * G + H)
    assert np.max(np.abs(dg - ref) / ref) < 1e-15
