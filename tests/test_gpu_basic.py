"""GPU parity of the collocation scheme of Sec. 3.2 (the basic scheme):
the operator Gamma_ref of Appendix A (Eq. Gamma_explicit) built on the fly
from the acoustic tensor, and Newton with Richardson solves of
Gamma_ref C d = -Gamma_ref sigma (Eq. linear_system_L-S) with
C_ref = 1/2 (lambda_min + lambda_max) I_s renewed every Newton iteration,
against the FP64 oracle; and the iteration growth that separates it from
conjugate gradients (linear in the tangent's eigenvalue ratio against its
square root)."""
import numpy as np
import pytest

import synth
from oracle import solver as S
from oracle.projection import apply_gamma_ref
from tests.gpu_util import rel_err, t2m, tensor6, to_dev, to_host

pytestmark = pytest.mark.gpu


def _iso(lam0, mu0):
    d = np.eye(3)
    return (lam0 * np.einsum("ij,lm->ijlm", d, d)
            + mu0 * (np.einsum("il,jm->ijlm", d, d) + np.einsum("im,jl->ijlm", d, d)))


@pytest.mark.parametrize("shape", [(5, 7, 9), (15, 15, 15), (31, 9, 5), (61, 9, 5)])
@pytest.mark.parametrize("lam0,mu0", [(0.0, 0.5), (0.7, 0.3), (2.0, 1.3)])
def test_gamma_ref_operator_matches_oracle(shape, lam0, mu0):
    from paper_1601_05970_amd import fftg
    print("Gamma_ref", shape, lam0, mu0, flush=True)
    pl = fftg.Plan(synth.bernoulli(shape, 0.4, 1), [synth.SOFT, synth.HARD])
    tau = synth.random_sym_tensor_field(shape, 9)
    d_out = pl.field()
    pl.apply_Gamma(to_dev(t2m(tau)), d_out, lam0, mu0)
    assert rel_err(to_host(d_out), t2m(apply_gamma_ref(tau, _iso(lam0, mu0)))) < 1e-12


def _opts(w, scheme, predictor=0):
    from paper_1601_05970_amd import fftg
    o = fftg.fftg_options_default()
    o.tol_newton, o.tol_cg, o.scheme, o.predictor = w.tol_newton, w.tol_cg, scheme, predictor
    return o


@pytest.mark.parametrize("shape,seed", [((9, 7, 5), 2), ((15, 15, 15), 3)])
def test_basic_scheme_lockstep_with_oracle(shape, seed):
    """Elasto-plastic two-phase RVE, three increments, Richardson counts
    replayed from the oracle's basic scheme: fields agree to 1e-10."""
    from paper_1601_05970_amd import fftg
    print("basic scheme lockstep", shape, flush=True)
    w = synth.small_random(shape, 0.35, seed, E_eq=0.01, n_inc=3)
    s = S.Solver(w.phase, w.materials, w.tol_newton, w.tol_cg, scheme="basic")
    pl = fftg.Plan(w.phase, w.materials, _opts(w, fftg.FFTG_SCHEME_BASIC))
    h = fftg.History(pl)
    for n in range(1, w.n_inc + 1):
        ref = s.solve_increment(w.E_at(n))
        st = h.solve_increment(tensor6(w.dE(n)), ref.cg_iters)
        assert st["cg_iters"] == ref.cg_iters
        assert rel_err(to_host(h.get_field(fftg.FFTG_FIELD_STRAIN)), t2m(s.strain())) < 1e-10
        assert rel_err(to_host(h.get_field(fftg.FFTG_FIELD_STRESS)), t2m(s.sigma)) < 1e-10
    assert np.max(s.epbar) > 0
    assert rel_err(to_host(h.get_field(fftg.FFTG_FIELD_EPBAR))[0], s.epbar) < 1e-10


def test_richardson_against_cg_iteration_growth():
    """Elastic two-phase RVEs of stiffness contrast r = 2, 8, 32 (tangent
    eigenvalue ratio r), one Newton solve each: the GPU's Richardson and CG
    counts equal the oracle's (within one iteration at the tolerance
    boundary), Richardson's grow about linearly in r and CG's about as its
    square root."""
    from paper_1601_05970_amd import fftg
    print("kappa sweep", flush=True)
    counts = {}
    for r in (2, 8, 32):
        ph = synth.bernoulli((15, 15, 15), 0.3, 3)
        mats = [(0.833, 0.386, 1e30, 0.0, 1.0), (0.833 * r, 0.386 * r, 1e30, 0.0, 1.0)]
        w = synth.Workload("kappa", ph, mats, synth.pure_shear_eq(0.01), 1, 1e-6, 1e-8)
        for name, scheme in (("cg", fftg.FFTG_SCHEME_GALERKIN), ("basic", fftg.FFTG_SCHEME_BASIC)):
            s = S.Solver(ph, mats, 1e-6, 1e-8, predictor="none", scheme="galerkin" if name == "cg" else "basic")
            ref = s.solve_increment(w.E_at(1))
            pl = fftg.Plan(ph, mats, _opts(w, scheme, fftg.FFTG_PREDICTOR_NONE))
            st = fftg.History(pl).solve_increment(tensor6(w.dE(1)))
            assert st["newton_iters"] == ref.newton_iters
            assert all(abs(a - b) <= 1 for a, b in zip(st["cg_iters"], ref.cg_iters)), (st["cg_iters"], ref.cg_iters)
            counts[(name, r)] = st["cg_iters"][0]
    print("  first-solve iterations by contrast:", counts, flush=True)
    for name, lo, hi in (("basic", 10.0, 20.0), ("cg", 2.5, 5.5)):
        ratio = counts[(name, 32)] / counts[(name, 2)]
        assert lo < ratio < hi, (name, ratio, counts)
