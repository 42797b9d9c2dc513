"""J2 elasto-plasticity, return mapping and consistent tangent (test
infrastructure; FP64 oracle).

Restates Sec. 4.2 of the paper as full tensors, voxel by voxel (vectorised
over the grid only):

* elastic law sigma = Ce : (eps - eps_p), Ce = K I(x)I + 2G I_d
  (Eq. model:plas:stress), I_d = I_s - 1/3 I(x)I;
* yield function Phi = sigma_eq - (sigma_0 + H eps_p_bar^n)
  (Eq. model:plas:yield), sigma_eq = sqrt(3/2 s:s) (Eq. model:eq-stress);
* backward Euler: trial state from the committed history of the previous
  increment (Eq. model:plas:trial); elastic when Phi_tr <= 0
  (Eq. model:plas:elas); otherwise the scalar return equation
  sigma_eq_tr - 3G dgamma - sigma_0 - H (eps_p_bar + dgamma)^n = 0, closed
  form for n = 1; for any other n its left side falls monotonically from
  Phi_tr > 0 at dgamma = 0 to at most 0 at dgamma = Phi_tr / 3G, and the
  root is found by bisection of that bracket down to adjacent floating-point
  numbers; then the update of Eq. (model:plas:corrector) along the trial
  normal N = 3/2 s_tr / sigma_eq_tr (Eq. model:plas:flow);
* consistent tangent
  C = Ce - 6 G^2 dgamma / sigma_eq_tr I_d
        + 4 G^2 (dgamma / sigma_eq_tr - 1 / (3G + n H (eps_p_bar + dgamma)^(n-1))) N (x) N.

Pins (tests/test_oracle_j2.py): elastic branch equals K tr(eps) I + 2G dev(eps);
pure-shear closed form eps_12(tau) = tau/(2G) + (3 tau - sqrt(3) sigma_0)/(2H)
derived from the model by hand (n = 1), and for n != 1 the pure-shear
relation eps_12 = tau/(2G) + sqrt(3)/2 ((sqrt(3) tau - sigma_0)/H)^(1/n)
solved by an independent root finder; the returned state lies on the yield
surface (residual of the return equation at rounding level) and its plastic
strain is deviatoric; the tangent matches central finite differences of the
stress update and has major symmetry.
"""
from __future__ import annotations

import numpy as np

I2 = np.eye(3)
II = np.einsum("ij,lm->ijlm", I2, I2)
I4S = 0.5 * (np.einsum("il,jm->ijlm", I2, I2) + np.einsum("im,jl->ijlm", I2, I2))
I4D = I4S - II / 3.0


def elastic_stiffness(K, G):
    """Ce = K I(x)I + 2G I_d (Eq. model:plas:stress), shape (3,3,3,3)+K.shape."""
    K = np.asarray(K, dtype=float)
    G = np.asarray(G, dtype=float)
    return (np.multiply.outer(II, K) + 2.0 * np.multiply.outer(I4D, G))


def ddot42(A, b):
    """A_ijlm b_lm over trailing grid axes."""
    return np.einsum("ijlm...,lm...->ij...", A, b)


def deviator(t):
    """Deviatoric part t - tr(t)/3 I of a (3,3)+shape field."""
    tr = np.einsum("ii...->...", t)
    return t - (tr / 3.0)[None, None] * I2.reshape((3, 3) + (1,) * (t.ndim - 2))


def material_fields(phase: np.ndarray, materials):
    """Per-voxel parameter arrays (K, G, sigma_0, H, n) from a phase map
    (rows (K, G, sigma_y0, H, n); longer rows, which name other laws, are
    cut to their first five entries)."""
    mats = np.asarray([list(m)[:5] for m in materials], dtype=float)
    if mats.ndim != 2 or mats.shape[1] != 5:
        raise ValueError("materials must be rows (K, G, sigma_y0, H, n)")
    if np.any(mats[:, 4] <= 0.0):
        raise ValueError("the hardening exponent n must be positive")
    p = np.asarray(phase, dtype=np.intp)
    if p.min() < 0 or p.max() >= mats.shape[0]:
        raise ValueError("phase id out of range")
    return tuple(mats[p, c] for c in range(5))


def return_equation(dgam, seq_tr, epbar_t, G, sy0, H, n):
    """Left side of the scalar return equation of Sec. 4.2:
    sigma_eq_tr - 3G dgamma - sigma_0 - H (eps_p_bar + dgamma)^n."""
    return seq_tr - 3.0 * G * dgam - sy0 - H * (epbar_t + dgam) ** n


def solve_return_equation(seq_tr, epbar_t, G, sy0, H, n):
    """dgamma > 0 with return_equation(dgamma) = 0 where Phi_tr > 0 (arrays
    over the plastic voxels).  The left side decreases monotonically in
    dgamma; it is Phi_tr > 0 at 0 and at most 0 at Phi_tr / 3G.  Bisection
    of that bracket until the midpoint coincides with an end point."""
    phi_tr = seq_tr - (sy0 + H * epbar_t ** n)
    lo = np.zeros_like(seq_tr)
    hi = phi_tr / (3.0 * G)
    for _ in range(2000):
        mid = 0.5 * (lo + hi)
        if np.all((mid <= lo) | (mid >= hi)):
            break
        pos = return_equation(mid, seq_tr, epbar_t, G, sy0, H, n) > 0.0
        lo = np.where(pos, mid, lo)
        hi = np.where(pos, hi, mid)
    return 0.5 * (lo + hi)


def return_map(eps, eps_p_t, epbar_t, K, G, sy0, H, n=None):
    """Stress, consistent tangent and updated history at total strain eps.

    eps, eps_p_t: (3,3)+shape; epbar_t, K, G, sy0, H (and n, default 1):
    shape.  The trial state always starts from the committed history
    (eps_p_t, epbar_t) of the previous increment (backward Euler).
    Returns (sigma, C, eps_p_new, epbar_new, plastic_mask).
    """
    if n is None:
        n = np.ones_like(np.asarray(G, dtype=float))
    n = np.broadcast_to(np.asarray(n, dtype=float), np.shape(G))
    lin = n == 1.0
    Ce = elastic_stiffness(K, G)
    sig_tr = ddot42(Ce, eps - eps_p_t)
    s_tr = deviator(sig_tr)
    seq_tr = np.sqrt(1.5 * np.einsum("ij...,ij...->...", s_tr, s_tr))
    hard_t = np.where(lin, H * epbar_t, H * epbar_t ** n)
    phi_tr = seq_tr - (sy0 + hard_t)
    plastic = phi_tr > 0.0

    seq_safe = np.where(plastic, seq_tr, 1.0)
    dgam = np.where(plastic, phi_tr / (3.0 * G + H), 0.0)     # n = 1 closed form
    nl = plastic & ~lin
    if np.any(nl):
        dgam = dgam.copy()
        dgam[nl] = solve_return_equation(seq_tr[nl], epbar_t[nl], G[nl], sy0[nl], H[nl], n[nl])
    Ntr = 1.5 * s_tr / seq_safe
    Ntr = np.where(plastic, Ntr, 0.0)

    eps_p = eps_p_t + dgam * Ntr
    epbar = epbar_t + dgam
    sigma = ddot42(Ce, eps - eps_p)

    # dR/d(dgamma) of the return equation: 3G + n H (eps_p_bar + dgamma)^(n-1)
    slope = np.where(lin, 3.0 * G + H, 3.0 * G + n * H * np.where(nl, epbar, 1.0) ** (n - 1.0))
    c1 = np.where(plastic, 6.0 * G * G * dgam / seq_safe, 0.0)
    c2 = np.where(plastic, 4.0 * G * G * (dgam / seq_safe - 1.0 / slope), 0.0)
    C = (Ce - np.multiply.outer(I4D, c1)
         + c2 * np.einsum("ij...,lm...->ijlm...", Ntr, Ntr))
    return sigma, C, eps_p, epbar, plastic


def point_response(eps, eps_p_t, epbar_t, mat):
    """Single material point version (eps: 3x3) for closed-form checks."""
    K, G, sy0, H, n = mat[:5]
    e = np.asarray(eps, dtype=float).reshape(3, 3, 1)
    ep = np.asarray(eps_p_t, dtype=float).reshape(3, 3, 1)
    sig, C, epn, ebn, pl = return_map(e, ep, np.array([epbar_t], dtype=float),
                                      np.array([K]), np.array([G]),
                                      np.array([sy0]), np.array([H]), np.array([float(n)]))
    return sig[..., 0], C[..., 0], epn[..., 0], float(ebn[0]), bool(pl[0])
