"""Pins of the oracle's Newton--CG solve (Algorithm 1) against closed forms,
invariants and dense brute force."""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import synth
from oracle import j2, solver as S
from oracle.dense import newton_step_exact
from oracle.projection import apply_G
from tests.fixtures import load_golden


def test_homogeneous_material_returns_applied_strain():
    """One phase (two identical phases): eps* stays 0 and Sigma is the
    single-point response along the same strain path."""
    ph = synth.bernoulli((7, 5, 9), 0.5, 11)
    mats = [synth.SOFT, synth.SOFT]
    s = S.Solver(ph, mats, 1e-5, 1e-8)
    E_dir = synth.pure_shear_eq(0.02)
    ep, eb = np.zeros((3, 3)), 0.0
    for n in range(1, 6):
        E = n / 5.0 * E_dir
        st = s.solve_increment(E)
        assert st.converged
        assert np.max(np.abs(s.eps_fl)) == 0.0
        sig, _, ep, eb, _ = j2.point_response(E, ep, eb, synth.SOFT)
        assert np.max(np.abs(st.Sigma - sig)) <= 1e-15
        assert st.cg_iters == [0, 0]


def laminate_closed_form(E12, f_soft=7.0 / 11.0, f_hard=4.0 / 11.0):
    """Uniform shear stress tau with piecewise-constant layer strains.

    For layers normal to x under E = E12 (e1 e2 + e2 e1), traction continuity
    makes sigma_12 uniform and compatibility lets eps_12 jump between layers;
    the volume average of eps_12 is E12.  Per phase, from Sec. 4.2 with n = 1
    under monotone proportional shear: eps_12(tau) = tau/(2G) below yield and
    tau/(2G) + (3 tau - sqrt(3) s0)/(2H) beyond (see the J2 closed form).
    """
    def e12(tau, mat):
        K, G, s0, H, _ = mat
        if math.sqrt(3.0) * tau <= s0:
            return tau / (2.0 * G)
        return tau / (2.0 * G) + (3.0 * tau - math.sqrt(3.0) * s0) / (2.0 * H)

    f = lambda t: f_soft * e12(t, synth.SOFT) + f_hard * e12(t, synth.HARD) - E12
    tau = brentq(f, 0.0, 1.0, xtol=1e-18, rtol=1e-15)
    return tau, e12(tau, synth.SOFT), e12(tau, synth.HARD)


def test_laminate_matches_closed_form():
    w = synth.laminate_11()
    s = S.Solver(w.phase, w.materials, w.tol_newton, w.tol_cg)
    soft = w.phase == 0
    for n in range(1, w.n_inc + 1):
        st = s.solve_increment(w.E_at(n))
        assert st.converged
        tau, es, eh = laminate_closed_form(w.E_at(n)[0, 1])
        eps = s.strain()
        assert abs(st.Sigma[0, 1] - tau) <= 1e-10 * tau
        assert np.max(np.abs(eps[0, 1][soft] - es)) <= 1e-10 * es
        assert np.max(np.abs(eps[0, 1][~soft] - eh)) <= 1e-10 * eh
        # every other strain and stress component vanishes
        for (i, k) in [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2)]:
            assert np.max(np.abs(eps[i, k])) < 1e-13
            assert abs(st.Sigma[i, k]) < 1e-15
        # accumulated plastic strain: sqrt(3) (eps12 - tau/2G) ... in the soft layers
        K, G, s0, H, _ = synth.SOFT
        eb_soft = (math.sqrt(3.0) * tau - s0) / H
        assert np.max(np.abs(s.epbar[soft] - eb_soft)) <= 1e-9 * eb_soft
        assert np.all(s.epbar[~soft] == 0.0)


def test_literal_algorithm_on_laminate_with_elastic_phase():
    """The paper's laminate setting (phase 2 linear elastic, Sec. 5.1) with
    Algorithm 1 as printed: one increment reaches the closed-form solution."""
    lam = load_golden("laminate_sec5_1.txt")
    ph = synth.laminate(11, 4)
    G = 0.386
    elastic = (0.833, G, 1e30, 0.0, 1.0)        # never yields
    plastic = (0.833, G, lam["sigma0_over_G"] * G, lam["H_over_G"] * G, 1.0)
    s = S.Solver(ph, [elastic, plastic], lam["eta_newton"], 1e-12, predictor="none")
    E12 = lam["E12"]
    st = s.solve_increment(synth.shear_xy(E12))
    assert st.converged

    def e12(tau, mat):
        K, G, s0, H, _ = mat
        if math.sqrt(3.0) * tau <= s0:
            return tau / (2.0 * G)
        return tau / (2.0 * G) + (3.0 * tau - math.sqrt(3.0) * s0) / (2.0 * H)

    tau = brentq(lambda t: 7.0 / 11.0 * e12(t, elastic) + 4.0 / 11.0 * e12(t, plastic) - E12,
                 0.0, 1.0, xtol=1e-18, rtol=1e-15)
    assert abs(st.Sigma[0, 1] - tau) <= 1e-10 * tau
    eps = s.strain()
    assert np.max(np.abs(eps[0, 1][ph == 1] - e12(tau, plastic))) < 1e-10 * E12


def test_literal_algorithm_stalls_where_the_tangent_predictor_converges():
    """Why the first Newton iteration of an increment is a tangent predictor.
    On the 11^3 two-phase elasto-plastic laminate (both phases plastic), the
    second increment of Algorithm 1 as printed starts from the return map at
    E_new + eps*_old: the whole strain increment lands in every voxel, the
    hard layers yield spuriously, and the Newton corrections grow instead of
    shrinking, then cycle without converging.  The predictor, which solves the
    linearised load step about the last converged state first, converges in
    two iterations, to the laminate's closed form."""
    w = synth.laminate_11()
    lit = S.Solver(w.phase, w.materials, w.tol_newton, w.tol_cg, predictor="none", max_newton=30)
    prd = S.Solver(w.phase, w.materials, w.tol_newton, w.tol_cg, predictor="tangent", max_newton=30)
    assert lit.solve_increment(w.E_at(1)).converged
    assert prd.solve_increment(w.E_at(1)).converged
    st = lit.solve_increment(w.E_at(2))
    assert not st.converged and st.newton_iters == 30
    # the corrections grow at first and never fall below the first one
    assert st.newton_res[1] > st.newton_res[0] > 1.0
    assert min(st.newton_res[1:]) > st.newton_res[0]
    sp = prd.solve_increment(w.E_at(2))
    assert sp.converged and sp.newton_iters == 2
    tau, _, _ = laminate_closed_form(w.E_at(2)[0, 1])
    assert abs(sp.Sigma[0, 1] - tau) <= 1e-10 * tau


@pytest.mark.parametrize("predictor", ["tangent", "none"])
def test_converged_fields_are_compatible_zero_mean_and_equilibrated(predictor):
    w = synth.small_random((9, 7, 5), 0.4, 21, E_eq=0.006, n_inc=3)
    s = S.Solver(w.phase, w.materials, 1e-8, 1e-10, predictor=predictor)
    for n in range(1, w.n_inc + 1):
        st = s.solve_increment(w.E_at(n))
        assert st.converged
    ef = s.eps_fl
    assert np.max(np.abs(ef.mean(axis=(2, 3, 4)))) < 1e-15
    assert np.max(np.abs(apply_G(ef) - ef)) <= 1e-12 * np.max(np.abs(ef))
    sig = s.sigma
    assert np.sqrt(np.sum(apply_G(sig) ** 2)) <= 1e-8 * np.sqrt(np.sum(sig ** 2))
    # Hill--Mandel: <sigma : eps> = Sigma : E when G sigma = 0 and eps* in E_N
    eps = s.strain()
    lhs = np.mean(np.einsum("ij...,ij...->...", sig, eps))
    Sigma = sig.mean(axis=(2, 3, 4))
    rhs = np.sum(Sigma * s.E)
    assert abs(lhs - rhs) <= 1e-9 * abs(rhs)


@pytest.mark.parametrize("shape", [(3, 3, 3), (3, 5, 7)])
def test_newton_step_equals_dense_exact_solve(shape):
    ph = synth.bernoulli(shape, 0.5, 5)
    s = S.Solver(ph, [synth.SOFT, synth.HARD], 1e-12, 1e-14)
    s.solve_increment(synth.pure_shear_eq(0.002))
    s.E = synth.pure_shear_eq(0.0045)          # soft voxels yield, hard do not
    sig, C, _, _, pl = s.constitutive(s.eps_fl)
    assert pl.any() and not pl.all()
    b = -apply_G(sig)
    res = S.cg(lambda p: apply_G(j2.ddot42(C, p)), b, 1e-14, 5000)
    d_exact = newton_step_exact(sig, C)
    assert np.max(np.abs(res.x - d_exact)) <= 1e-10 * np.max(np.abs(d_exact))


def test_lockstep_replay_reproduces_natural_run():
    w = synth.small_random((7, 7, 7), 0.3, 3, E_eq=0.008, n_inc=3)
    s1, st1 = S.run_workload(w)
    counts = [st.cg_iters for st in st1]
    s2, st2 = S.run_workload(w, lockstep=counts)
    assert np.array_equal(s1.eps_fl, s2.eps_fl)
    assert np.array_equal(s1.epbar, s2.epbar)


def test_cg_breakdown_on_indefinite_operator():
    b = np.zeros((3, 3, 3, 3, 3))
    b[0, 1, 1, 0, 0] = b[1, 0, 1, 0, 0] = 1.0
    res = S.cg(lambda p: -p, b, 1e-8)
    assert res.breakdown and res.iters == 0


# ------------------------------------------------------------ basic scheme
def _contrast(r, shape=(7, 7, 7)):
    """Elastic two-phase RVE (never yields) with stiffness contrast r (both
    moduli scaled): the tangent's eigenvalue ratio is r."""
    ph = synth.bernoulli(shape, 0.3, 3)
    soft = (0.833, 0.386, 1e30, 0.0, 1.0)
    hard = (0.833 * r, 0.386 * r, 1e30, 0.0, 1.0)
    return ph, [soft, hard]


def test_gamma_ref_of_scaled_unit_tensor_is_scaled_G():
    """Appendix A, Eq. Gamma_explicit: Gamma_ref is of degree -1 in C_ref, so
    C_ref = c I_s gives G / c -- the reason the basic scheme with that
    reference medium is Richardson's iteration with step 1/c on G C d = -G s."""
    from oracle.j2 import I4S
    from oracle.projection import gamma_ref_hat, ghat
    shape = (5, 3, 7)
    for c in (0.3, 2.5):
        assert np.max(np.abs(gamma_ref_hat(shape, c * I4S) - ghat(shape) / c)) < 1e-14 / c


def test_basic_scheme_reaches_the_galerkin_solution():
    """The collocation system with Gamma_ref = G / c has the same solutions
    as the Galerkin one (Sec. 3.2: the two formulations coincide up to the
    solver), so Newton with the basic scheme lands on the CG result."""
    w = synth.small_random((7, 9, 5), 0.35, 4, E_eq=0.01, n_inc=3)
    a = S.Solver(w.phase, w.materials, 1e-9, 1e-11)
    b = S.Solver(w.phase, w.materials, 1e-9, 1e-11, scheme="basic")
    for n in range(1, 4):
        sa, sb = a.solve_increment(w.E_at(n)), b.solve_increment(w.E_at(n))
        assert sa.converged and sb.converged
    assert np.max(np.abs(a.strain() - b.strain())) <= 1e-9 * 0.01
    assert sum(sum(x) for x in [sb.cg_iters]) > sum(sa.cg_iters)
    # one reference medium per linear solve, between the phases' elastic
    # extremes 2G (deviatoric) and 3K (volumetric)
    assert b.c_ref and all(0.0 < c < 3 * 0.833 for c in b.c_ref)


def test_richardson_grows_with_kappa_and_cg_with_its_root():
    """Sec. 3.2: with the optimal reference medium the basic scheme's
    iteration count grows linearly with the tangent's eigenvalue ratio,
    CG's with its square root.  Elastic contrast r = 2 and 16 (kappa 2, 16):
    Richardson's count rises about 8-fold, CG's about 3-fold."""
    counts = {}
    for r in (2, 16):
        ph, mats = _contrast(r)
        for sch in ("galerkin", "basic"):
            s = S.Solver(ph, mats, 1e-6, 1e-8, predictor="none", scheme=sch)
            counts[(sch, r)] = s.solve_increment(synth.pure_shear_eq(0.01)).cg_iters[0]
    rb = counts[("basic", 16)] / counts[("basic", 2)]
    rc = counts[("galerkin", 16)] / counts[("galerkin", 2)]
    assert 5.0 < rb < 12.0, counts
    assert 2.0 < rc < 4.5, counts
