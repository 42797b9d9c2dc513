"""The other two constitutive laws of Sec. 4 and the per-voxel choice of law
(test infrastructure; FP64 oracle).

* ``nonlinear_elastic`` -- Sec. 4.1: sigma = K tr(eps) I
  + sigma_0 (eps_eq / eps_0)^n N with N = 2/3 eps_d / eps_eq and
  eps_eq = sqrt(2/3 eps_d : eps_d) (Eqs. model:nlin:stress, model:nlin:N);
  tangent of Eq. (model:nlin-tangent).  At eps_eq = 0 the deviatoric part of
  the stress vanishes (n > 0) and the tangent is its limit: K I(x)I, plus
  2/3 sigma_0 / eps_0 I_d when n = 1 (for n < 1 the limit is infinite and
  such phases are rejected).
* ``visco_return_map`` -- Sec. 4.3: Norton's rule
  dgamma/dt = eps_0/t_0 (sigma_eq / sigma_0)^(1/n) (Eq. model:visco:gammadot)
  integrated by backward Euler from the trial state of Eq. (model:plas:trial)
  with the real time step dt: the implicit equation
  dgamma = gamma_0 dt ((sigma_eq_tr - 3G dgamma) / sigma_0)^(1/n) of the
  section, whose left minus right side grows monotonically from
  -gamma_0 dt (sigma_eq_tr/sigma_0)^(1/n) at 0 to sigma_eq_tr/3G at
  sigma_eq_tr/3G, is solved by bisection of that bracket; the update is
  Eq. (model:plas:corrector) and the tangent the one printed in the
  section.  The section leaves gamma_0 undefined; it is read as
  gamma_0 = eps_0 / t_0, the factor of Norton's rule.  There is plastic flow
  whenever sigma_eq_tr > 0 (no yield switch).
* ``constitutive`` -- stress, tangent and updated history on a grid whose
  voxels carry different laws.  Material rows: (K, G, sigma_0, H, n) is the
  elasto-plastic law of Sec. 4.2 (``oracle.j2``); longer rows
  (K, G, sigma_0, H, n, law, eps_0, t_0) name the law: 0 elasto-plastic,
  1 non-linear elastic (G unused), 2 visco-plastic (H unused).

Pins (tests/test_oracle_laws.py): central finite differences of both
tangents; the pure-shear response of each law from its closed form (non-
linear elasticity) or from the scalar relation solved by an independent
root finder (visco-plasticity); the implicit equation's residual at the
solution; Norton's rule reproduced by the discrete rate; laminate solves of
each law against their per-layer scalar relations.
"""
from __future__ import annotations

import numpy as np

from . import j2

LAW_J2, LAW_NONLINEAR_ELASTIC, LAW_VISCO = 0, 1, 2

I2 = j2.I2
II = j2.II
I4D = j2.I4D


def _inner(a, b):
    return np.einsum("ij...,ij...->...", a, b)


def nonlinear_elastic(eps, K, s0, eps0, n):
    """(sigma, C) of Sec. 4.1 at strain eps ((3,3)+shape; parameters: shape)."""
    tr = np.einsum("ii...->...", eps)
    ed = j2.deviator(eps)
    eeq = np.sqrt(2.0 / 3.0 * _inner(ed, ed))
    pos = eeq > 0.0
    esafe = np.where(pos, eeq, 1.0)
    N = np.where(pos, 2.0 / 3.0 * ed / esafe, 0.0)
    mag = np.where(pos, s0 * (esafe / eps0) ** n, 0.0)           # sigma_0 (eps_eq/eps_0)^n
    sigma = K * tr * I2.reshape((3, 3) + (1,) * tr.ndim) + mag * N
    # sigma_0 / eps_eq (eps_eq/eps_0)^n, and its limit at eps_eq = 0
    fac = np.where(pos, mag / esafe, np.where(n == 1.0, s0 / eps0, 0.0))
    C = (np.multiply.outer(II, K)
         + fac * ((n - 1.0) * np.einsum("ij...,lm...->ijlm...", N, N)
                  + 2.0 / 3.0 * np.multiply.outer(I4D, np.ones_like(K))))
    return sigma, C


def visco_equation(dgam, seq_tr, G, s0, g0dt, n):
    """Left minus right side of the implicit equation of Sec. 4.3."""
    return dgam - g0dt * ((seq_tr - 3.0 * G * dgam) / s0) ** (1.0 / n)


def solve_visco_equation(seq_tr, G, s0, g0dt, n):
    """Root of visco_equation on [0, sigma_eq_tr / 3G] by bisection until the
    midpoint coincides with an end point (arrays over voxels)."""
    lo = np.zeros_like(seq_tr)
    hi = seq_tr / (3.0 * G)
    for _ in range(2000):
        mid = 0.5 * (lo + hi)
        if np.all((mid <= lo) | (mid >= hi)):
            break
        neg = visco_equation(mid, seq_tr, G, s0, g0dt, n) < 0.0
        lo = np.where(neg, mid, lo)
        hi = np.where(neg, hi, mid)
    return 0.5 * (lo + hi)


def visco_return_map(eps, eps_p_t, epbar_t, K, G, s0, eps0, t0, n, dt):
    """(sigma, C, eps_p, epbar, flowing) of Sec. 4.3 at total strain eps, from
    the history committed at the end of the previous time step."""
    Ce = j2.elastic_stiffness(K, G)
    sig_tr = j2.ddot42(Ce, eps - eps_p_t)
    s_tr = j2.deviator(sig_tr)
    seq_tr = np.sqrt(1.5 * _inner(s_tr, s_tr))
    flow = seq_tr > 0.0
    g0dt = eps0 / t0 * dt
    seq_safe = np.where(flow, seq_tr, 1.0)
    dgam = np.zeros_like(seq_tr)
    if np.any(flow):
        dgam[flow] = solve_visco_equation(seq_tr[flow], G[flow], s0[flow], g0dt[flow], n[flow])
    Ntr = np.where(flow, 1.5 * s_tr / seq_safe, 0.0)
    eps_p = eps_p_t + dgam * Ntr
    epbar = epbar_t + dgam
    sigma = j2.ddot42(Ce, eps - eps_p)
    # (3G + n sigma_0 / (gamma_0 dt) (dgamma / (gamma_0 dt))^(n-1))^-1, as printed
    x = np.where(flow & (dgam > 0.0), dgam / g0dt, 1.0)
    inv = np.where(flow, 1.0 / (3.0 * G + n * s0 / g0dt * x ** (n - 1.0)), 0.0)
    c1 = np.where(flow, 6.0 * G * G * dgam / seq_safe, 0.0)
    c2 = np.where(flow, 4.0 * G * G * (dgam / seq_safe - inv), 0.0)
    C = (Ce - np.multiply.outer(I4D, c1) + c2 * np.einsum("ij...,lm...->ijlm...", Ntr, Ntr))
    return sigma, C, eps_p, epbar, flow


def material_rows(materials):
    """Rows normalised to (K, G, sigma_0, H, n, law, eps_0, t_0)."""
    out = []
    for m in materials:
        m = [float(v) for v in m]
        if len(m) == 5:
            m = m + [LAW_J2, 1.0, 1.0]
        if len(m) != 8:
            raise ValueError("material rows are (K, G, s0, H, n) or (K, G, s0, H, n, law, eps0, t0)")
        if m[5] not in (LAW_J2, LAW_NONLINEAR_ELASTIC, LAW_VISCO):
            raise ValueError("unknown law")
        out.append(m)
    return np.asarray(out)


def constitutive(phase, materials, eps, eps_p_t, epbar_t, dt=1.0):
    """(sigma, C, eps_p, epbar, inelastic) with each voxel's law (inelastic:
    plastic or visco-plastic flow in this step); J2-only grids go through
    oracle.j2 unchanged."""
    rows = material_rows(materials)
    p = np.asarray(phase, dtype=np.intp)
    law = rows[p, 5]
    if np.all(law == LAW_J2):
        K, G, sy0, H, n = j2.material_fields(phase, [r[:5] for r in rows])
        return j2.return_map(eps, eps_p_t, epbar_t, K, G, sy0, H, n)
    sig = np.zeros_like(eps)
    act = np.zeros(eps.shape[2:], dtype=bool)
    C = np.zeros((3, 3) + eps.shape)
    ep = eps_p_t.copy()
    eb = epbar_t.copy()
    par = [rows[p, c] for c in range(8)]
    for lw in (LAW_J2, LAW_NONLINEAR_ELASTIC, LAW_VISCO):
        sel = law == lw
        if not np.any(sel):
            continue
        K, G, s0, H, n, _, e0, t0 = [a[sel] for a in par]
        e = eps[:, :, sel]
        if lw == LAW_J2:
            s_, C_, ep_, eb_, a_ = j2.return_map(e, eps_p_t[:, :, sel], epbar_t[sel], K, G, s0, H, n)
        elif lw == LAW_NONLINEAR_ELASTIC:
            s_, C_ = nonlinear_elastic(e, K, s0, e0, n)
            ep_, eb_, a_ = eps_p_t[:, :, sel], epbar_t[sel], False
        else:
            s_, C_, ep_, eb_, a_ = visco_return_map(e, eps_p_t[:, :, sel], epbar_t[sel], K, G, s0, e0, t0, n, dt)
        sig[:, :, sel] = s_
        C[:, :, :, :, sel] = C_
        ep[:, :, sel] = ep_
        eb[sel] = eb_
        act[sel] = a_
    return sig, C, ep, eb, act


def elastic_tangent(phase, materials):
    """Tangent of the virgin state (zero strain, zero history): the
    consistent tangent the first predictor uses."""
    shape = np.shape(phase)
    z = np.zeros((3, 3) + shape)
    return constitutive(phase, materials, z, z, np.zeros(shape))[1]
