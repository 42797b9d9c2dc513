"""GPU parity of the matrix-free product G:(C:p) against the FP64 oracle.

The library is called through its C ABI (ctypes binding); the oracle applies
G with numpy FFTs and the explicit four-index G^ of Appendix A.
"""
import functools

import numpy as np
import pytest

import synth
from oracle import j2
from oracle.projection import apply_G
from tests.gpu_util import m2t, rel_err, t2m, to_dev, to_host

pytestmark = pytest.mark.gpu

SHAPES = [(3, 3, 3), (1, 5, 7), (7, 5, 1), (3, 5, 7), (5, 7, 9), (11, 11, 11), (13, 17, 11),
          (15, 15, 15), (21, 25, 27), (31, 31, 31), (63, 31, 15), (19, 23, 29), (61, 9, 5),
          (47, 5, 59), (3, 53, 43), (127, 3, 5), (3, 255, 3), (5, 3, 127), (31, 9, 5), (9, 5, 31)]


def _plan(shape, phase=None, mats=None, precision=0):
    from paper_1601_05970_amd import fftg
    if phase is None:
        phase = synth.bernoulli(shape, 0.4, 1)
    opt = fftg.fftg_options_default()
    opt.precision = precision
    p = fftg.Plan(phase, mats or [synth.SOFT, synth.HARD], opt)
    return p


@pytest.mark.parametrize("shape", SHAPES)
def test_projection_matches_oracle(shape):
    from paper_1601_05970_amd import fftg
    print("apply IDENTITY", shape, flush=True)
    pl = _plan(shape)
    tau = synth.random_sym_tensor_field(shape, 3)
    d_in = to_dev(t2m(tau))
    d_out = pl.field()
    pl.apply_GK(d_in, d_out, fftg.FFTG_TANGENT_IDENTITY)
    got = to_host(d_out)
    ref = t2m(apply_G(tau))
    assert rel_err(got, ref) < 1e-12


def test_sampled_kernel_timing_counts_every_launch():
    """fftg_profiler_start_every brackets launches 0, every, 2 every, ... of
    one kind; fftg_profiler_seen counts all of them."""
    from paper_1601_05970_amd import fftg
    shape = (15, 15, 15)
    print("profiler sampling", shape, flush=True)
    pl = _plan(shape)
    d_in = to_dev(t2m(synth.random_sym_tensor_field(shape, 4)))
    d_out = pl.field()
    pl.apply_GK(d_in, d_out, fftg.FFTG_TANGENT_IDENTITY)  # autotunes before the profiled window
    fftg.fftg_profiler_start_every(fftg.FFTG_KERNEL_X_PROJ, 3)
    for _ in range(8):
        pl.apply_GK(d_in, d_out, fftg.FFTG_TANGENT_IDENTITY)
    ms, launches, vox = fftg.fftg_profiler_stop()
    assert fftg.fftg_profiler_seen() == 8
    assert launches == 3 and ms > 0.0 and vox == 3 * 15 ** 3


@pytest.mark.parametrize("slab", ["0", "2"])
@pytest.mark.parametrize("shape", [(3, 5, 7), (1, 5, 7), (7, 5, 1), (15, 15, 15), (31, 31, 31), (61, 9, 53),
                                   (5, 63, 63), (13, 17, 11)])
def test_product_schedules_match_oracle(shape, slab, monkeypatch):
    """The five-pass product (FFTG_SLAB=0) and the fused z-y slab passes
    (FFTG_SLAB=2; every shape here fits) against the oracle, FP64 and FP32."""
    import torch
    from paper_1601_05970_amd import fftg
    print("apply schedule", shape, "slab", slab, flush=True)
    monkeypatch.setenv("FFTG_SLAB", slab)
    ph = synth.bernoulli(shape, 0.5, 2)
    mats = [(0.833, 0.386, 0.003, 0.004, 1.0), (2.0, 1.3, 0.006, 0.008, 1.0)]
    p = synth.random_sym_tensor_field(shape, 4)
    K, G, _, _, _ = j2.material_fields(ph, mats)
    ref = t2m(apply_G(j2.ddot42(j2.elastic_stiffness(K, G), p)))
    for prec, tol in ((0, 1e-12), (1, 2e-6)):
        pl = _plan(shape, ph, mats, precision=prec)
        d_out = pl.field(dtype=torch.float32 if prec else torch.float64)
        pl.apply_GK(to_dev(t2m(p)), d_out, fftg.FFTG_TANGENT_ELASTIC)
        assert rel_err(to_host(d_out).astype(np.float64), ref) < tol, prec


@pytest.mark.parametrize("shape", [(19, 23, 29), (31, 31, 31), (61, 9, 53)])
def test_projection_rader_path_matches_oracle(shape, monkeypatch):
    """Prime extents with smooth p-1 taken through Rader's algorithm instead
    of the direct DFT (FFTG_DIRECT_MAX=0 is read at plan creation)."""
    from paper_1601_05970_amd import fftg
    print("apply IDENTITY rader", shape, flush=True)
    monkeypatch.setenv("FFTG_DIRECT_MAX", "0")
    pl = _plan(shape)
    tau = synth.random_sym_tensor_field(shape, 3)
    d_out = pl.field()
    pl.apply_GK(to_dev(t2m(tau)), d_out, fftg.FFTG_TANGENT_IDENTITY)
    assert rel_err(to_host(d_out), t2m(apply_G(tau))) < 1e-12


@pytest.mark.parametrize("shape", [(5, 7, 9), (15, 15, 15), (31, 31, 31)])
def test_elastic_tangent_product_matches_oracle(shape):
    from paper_1601_05970_amd import fftg
    print("apply ELASTIC", shape, flush=True)
    ph = synth.bernoulli(shape, 0.5, 2)
    mats = [(0.833, 0.386, 0.003, 0.004, 1.0), (2.0, 1.3, 0.006, 0.008, 1.0)]
    pl = _plan(shape, ph, mats)
    p = synth.random_sym_tensor_field(shape, 4)
    d_out = pl.field()
    pl.apply_GK(to_dev(t2m(p)), d_out, fftg.FFTG_TANGENT_ELASTIC)
    K, G, _, _, _ = j2.material_fields(ph, mats)
    ref = t2m(apply_G(j2.ddot42(j2.elastic_stiffness(K, G), p)))
    assert rel_err(to_host(d_out), ref) < 1e-12


def _plastic_state(shape, seed):
    rng = np.random.default_rng(seed)
    eps = synth.random_sym_tensor_field(shape, seed, 4e-3)
    ep = synth.random_sym_tensor_field(shape, seed + 1, 1e-3)
    tr = np.einsum("ii...->...", ep)
    for i in range(3):
        ep[i, i] -= tr / 3.0
    eb = rng.uniform(0.0, 3e-3, shape)
    return eps, ep, eb


@pytest.mark.parametrize("shape", [(5, 7, 9), (15, 15, 15), (31, 31, 31)])
def test_consistent_tangent_product_matches_oracle(shape):
    from paper_1601_05970_amd import fftg
    print("apply CURRENT", shape, flush=True)
    ph = synth.bernoulli(shape, 0.4, 5)
    mats = [synth.SOFT, synth.HARD]
    pl = _plan(shape, ph, mats)
    h = fftg.History(pl)
    eps, ep, eb = _plastic_state(shape, 7)
    h.set_field(fftg.FFTG_FIELD_EPS_P, to_dev(t2m(ep)))
    h.set_field(fftg.FFTG_FIELD_EPBAR, to_dev(eb[None]))
    sig = pl.field()
    h.eval_constitutive(to_dev(t2m(eps)), sig)
    K, G, s0, H, _ = j2.material_fields(ph, mats)
    s_ref, C_ref, _, _, plastic = j2.return_map(eps, ep, eb, K, G, s0, H)
    assert 0.05 < plastic.mean() < 0.98
    assert rel_err(to_host(sig), t2m(s_ref)) < 1e-13
    p = synth.random_sym_tensor_field(shape, 8)
    d_out = pl.field()
    pl.apply_GK(to_dev(t2m(p)), d_out, fftg.FFTG_TANGENT_CURRENT, h)
    ref = t2m(apply_G(j2.ddot42(C_ref, p)))
    assert rel_err(to_host(d_out), ref) < 1e-12


@pytest.mark.parametrize("shape", [(15, 15, 15), (31, 31, 31), (63, 63, 63)])
def test_mixed_precision_product_matches_oracle(shape):
    from paper_1601_05970_amd import fftg
    import torch
    print("apply MIXED", shape, flush=True)
    ph = synth.bernoulli(shape, 0.5, 2)
    mats = [synth.SOFT, synth.HARD]
    pl = _plan(shape, ph, mats, precision=fftg.FFTG_MIXED)
    p = synth.random_sym_tensor_field(shape, 4)
    d_out = pl.field(dtype=torch.float32)
    pl.apply_GK(to_dev(t2m(p)), d_out, fftg.FFTG_TANGENT_ELASTIC)
    K, G, _, _, _ = j2.material_fields(ph, mats)
    ref = t2m(apply_G(j2.ddot42(j2.elastic_stiffness(K, G), p)))
    assert rel_err(to_host(d_out), ref) < 2e-6


def _compatible(shape, seed):
    """Symmetric gradient of a random periodic displacement (L_i = n_i)."""
    rng = np.random.default_rng(seed)
    k = [np.fft.fftfreq(n) * n for n in shape]
    out = np.zeros((3, 3) + tuple(shape))
    uh = [np.fft.fftn(rng.standard_normal(shape)) for _ in range(3)]
    for i in range(3):
        for j in range(i, 3):
            gi = (2j * np.pi * k[i] / shape[i]).reshape([-1 if a == i else 1 for a in range(3)])
            gj = (2j * np.pi * k[j] / shape[j]).reshape([-1 if a == j else 1 for a in range(3)])
            e = np.fft.ifftn(0.5 * (gi * uh[j] + gj * uh[i])).real
            out[i, j] = out[j, i] = e
    return out


@functools.lru_cache(maxsize=1)
def _oracle_127_products():
    """The oracle's G and G:(Ce:p) of one random symmetric field at 127^3."""
    shape = (127, 127, 127)
    p = synth.random_sym_tensor_field(shape, 127)
    ph = synth.bernoulli(shape, 0.4, 127)
    K, G, _, _, _ = j2.material_fields(ph, MATS2)
    return p, ph, t2m(apply_G(p)), t2m(apply_G(j2.ddot42(j2.elastic_stiffness(K, G), p)))


MATS2 = [(0.833, 0.386, 0.003, 0.004, 1.0), (2.0, 1.3, 0.006, 0.008, 1.0)]


@pytest.mark.timeout(600)
def test_full_size_127_products_match_oracle():
    """127^3 (Rader's algorithm on every axis, the full-size tile and LDS
    configuration), random incompatible input, element by element against
    the oracle: the projection and the elastic-tangent product, FP64 and the
    FP32 product."""
    import torch
    from paper_1601_05970_amd import fftg
    print("apply 127^3 vs oracle", flush=True)
    p, ph, ref_g, ref_c = _oracle_127_products()
    d_in = to_dev(t2m(p))
    for prec, tol, dt in ((fftg.FFTG_FP64, 1e-12, torch.float64), (fftg.FFTG_MIXED, 3e-6, torch.float32)):
        pl = _plan(p.shape[2:], ph, MATS2, precision=prec)
        for mode, ref in ((fftg.FFTG_TANGENT_IDENTITY, ref_g), (fftg.FFTG_TANGENT_ELASTIC, ref_c)):
            d_out = pl.field(dtype=dt)
            pl.apply_GK(d_in, d_out, mode)
            err = rel_err(to_host(d_out), ref)
            print("  precision", prec, "mode", mode, "rel err %.2e" % err, flush=True)
            assert err < tol
            del d_out
        del pl
        torch.cuda.empty_cache()


def _ghat_at(k):
    """G^(k) for an integer frequency k with |k_i| <= 3, taken from the
    oracle's four-index G^ on a 7^3 grid: G^ depends on the direction of
    xi = k / L only (degree-0 homogeneous), so for cubic cells it is the
    same at that k on any grid."""
    from oracle.projection import ghat
    G = ghat((7, 7, 7))
    return G[(slice(None),) * 4 + tuple(int(c) % 7 for c in k)]


# frequency, seed of the complex symmetric amplitude
MODES = [((0, 0, 0), 1), ((1, 0, 0), 2), ((0, -2, 1), 3), ((3, 1, -2), 4), ((-1, 3, 3), 5), ((2, -3, 1), 6)]


@pytest.mark.timeout(600)
def test_full_size_255_projection_of_fourier_modes():
    """255^3 (Rader's algorithm over 254-point chains, five passes, the
    largest plan): the input is a sum of a few Fourier modes
    Re(T_k exp(2 pi i k.x / 255)), whose projection is Re((G^(k):T_k)
    exp(2 pi i k.x / 255)) in closed form (Appendix A, Eq. FT_projection;
    the constant mode is removed, G^(0) = 0).  Checked element by element,
    FP64 and FP32 product."""
    import torch
    from paper_1601_05970_amd import fftg
    shape = (255, 255, 255)
    print("apply 255^3 Fourier modes", flush=True)
    x = [np.arange(n, dtype=np.float64) for n in shape]
    tau = np.zeros((3, 3) + shape)
    ref = np.zeros((3, 3) + shape)
    for k, seed in MODES:
        rng = np.random.default_rng(seed)
        A = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        T = 0.5 * (A + A.T)
        GT = np.einsum("ijlm,lm->ij", _ghat_at(k), T)
        ph = (2.0 * np.pi * k[0] / shape[0] * x[0])[:, None, None] + \
             (2.0 * np.pi * k[1] / shape[1] * x[1])[None, :, None] + \
             (2.0 * np.pi * k[2] / shape[2] * x[2])[None, None, :]
        c, s = np.cos(ph), np.sin(ph)
        for i in range(3):
            for j in range(3):
                tau[i, j] += T[i, j].real * c - T[i, j].imag * s
                ref[i, j] += GT[i, j].real * c - GT[i, j].imag * s
        del ph, c, s
    d_in = to_dev(t2m(tau))
    del tau
    ref = t2m(ref)
    for prec, tol, dt in ((fftg.FFTG_FP64, 1e-11, torch.float64), (fftg.FFTG_MIXED, 3e-6, torch.float32)):
        pl = _plan(shape, np.zeros(shape, np.uint8), precision=prec)
        d_out = pl.field(dtype=dt)
        pl.apply_GK(d_in, d_out, fftg.FFTG_TANGENT_IDENTITY)
        err = rel_err(to_host(d_out), ref)
        print("  precision", prec, "rel err %.2e" % err, flush=True)
        assert err < tol
        del d_out, pl
        torch.cuda.empty_cache()


@pytest.mark.parametrize("shape", [(127, 127, 127), (255, 255, 255)])
def test_full_size_projection_keeps_compatible_fields(shape):
    """At the large grid sizes the oracle is replaced by a property that
    holds at any size: G leaves a compatible field unchanged, in FP64 and
    in the FP32 apply."""
    from paper_1601_05970_amd import fftg
    import torch
    print("apply compatible", shape, flush=True)
    e = t2m(_compatible(shape, 11))
    for prec, tol, dt in ((fftg.FFTG_FP64, 1e-11, torch.float64), (fftg.FFTG_MIXED, 3e-6, torch.float32)):
        pl = _plan(shape, np.zeros(shape, np.uint8), precision=prec)
        d_out = pl.field(dtype=dt)
        pl.apply_GK(to_dev(e), d_out, fftg.FFTG_TANGENT_IDENTITY)
        assert rel_err(to_host(d_out), e) < tol
        del d_out, pl
        torch.cuda.empty_cache()
