"""Newton--CG solver of Algorithm 1 (test infrastructure; FP64 oracle).

* ``cg`` -- conventional (Hestenes--Stiefel) conjugate gradients for the
  linearised nodal equilibrium G C d_eps = -G sigma (Eq. linear_system),
  started from zero so every iterate stays compatible (Sec. 2.6).  Inner
  products are plain sums of tau:theta over the nodes: the trapezoidal rule
  (Eq. trapz) with equal weights, whose common factor cancels.  The stopping
  test is the relative residual of Algorithm 1's CG loop, evaluated with the
  CG recurrence residual (equal to the true residual in exact arithmetic).
* ``richardson`` -- the fixed-point iteration of the basic scheme (Sec. 3.2),
  used with Gamma_ref of C_ref = 1/2 (lambda_min + lambda_max) I_s, the extreme
  eigenvalues of the tangent's Mandel blocks over the grid, renewed every
  Newton iteration (scheme="basic").
* ``Solver`` -- the incremental-iterative Newton loop of Algorithm 1:
  increments of the mean strain E; Newton iterations until
  ||d_eps|| / ||E|| <= eta_NW, with ||E|| taken as the norm of the nodal
  column of E (E repeated at every node); the constitutive response of every
  Newton iteration is evaluated from the history committed at the end of the
  previous increment; the history is committed after the Newton loop, and the
  converged fluctuation is the initial guess of the next increment.

Readings of points the paper leaves open (shared with the GPU library):
* CG target max(eta_CG ||G s||, 1e-14 ||s||) with s = sigma (or C_last:dE
  for the predictor): a right-hand side under it gives d_eps = 0 with no
  CG iteration (homogeneous and fully elastic states);
* first iteration of an increment: tangent predictor about the last
  converged state (see Solver.solve_increment) -- Algorithm 1 as printed
  (predictor="none") cycles on two-phase elasto-plastic RVEs because its
  first iterate pushes the whole strain increment into every voxel;
* a lockstep option replays given per-Newton CG counts.

Pins (tests/test_oracle_solver.py): homogeneous material returns exactly the
applied mean strain; the laminate reproduces the closed-form per-phase
shear strains; converged fields are compatible, zero-mean and satisfy the
Hill--Mandel identity; on tiny grids one Newton step equals the exact solve
of the projected system assembled from the dense matrices of Appendix B.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import List, Optional

import numpy as np

from . import j2, laws
from .projection import apply_G


def fdot(a: np.ndarray, b: np.ndarray) -> float:
    """sum over nodes of a:b (trapezoidal rule up to the constant weight)."""
    return float(np.sum(a * b))


@dataclasses.dataclass
class CGResult:
    x: np.ndarray
    iters: int
    rel_res: float
    breakdown: bool = False


def cg(apply_A, b: np.ndarray, tol: float, max_iter: int = 2000,
       force_iters: Optional[int] = None, atol: float = 0.0) -> CGResult:
    """Conjugate gradients from x0 = 0 for A x = b.

    Stops as soon as ||r_k|| <= max(tol ||b||, atol) -- checked before the
    first iteration too, so a right-hand side already below the target
    gives x = 0 with no iteration -- or after exactly force_iters iterations
    when given.  Returns the iterate and the number of A applications.
    """
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = fdot(r, r)
    bnorm = math.sqrt(rr)
    target = max(tol * bnorm, atol)
    if force_iters is None and bnorm <= target:
        return CGResult(x, 0, 0.0 if bnorm == 0.0 else 1.0)
    k = 0
    limit = force_iters if force_iters is not None else max_iter
    while k < limit:
        Ap = apply_A(p)
        pAp = fdot(p, Ap)
        if not (pAp > 0.0):
            return CGResult(x, k, math.sqrt(rr) / bnorm, breakdown=True)
        alpha = rr / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = fdot(r, r)
        k += 1
        if force_iters is None and math.sqrt(rr_new) <= target:
            rr = rr_new
            break
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
    return CGResult(x, k, math.sqrt(rr) / bnorm if bnorm > 0 else 0.0)


def richardson(apply_A, b: np.ndarray, tol: float, max_iter: int = 2000,
               force_iters: Optional[int] = None, atol: float = 0.0) -> CGResult:
    """Richardson (fixed-point) iteration x <- x + (b - A x) from x0 = 0 with
    unit step, the basic scheme's solver of Sec. 3.2 (the reference medium
    inside A sets the step).  Residual recurrence r <- r - A r; stopping as
    in cg."""
    x = np.zeros_like(b)
    r = b.copy()
    rr = fdot(r, r)
    bnorm = math.sqrt(rr)
    target = max(tol * bnorm, atol)
    if force_iters is None and bnorm <= target:
        return CGResult(x, 0, 0.0 if bnorm == 0.0 else 1.0)
    k = 0
    limit = force_iters if force_iters is not None else max_iter
    while k < limit:
        x = x + r
        r = r - apply_A(r)
        rr = fdot(r, r)
        k += 1
        if force_iters is None and math.sqrt(rr) <= target:
            break
    return CGResult(x, k, math.sqrt(rr) / bnorm if bnorm > 0 else 0.0)


def tangent_eigen_bounds(C: np.ndarray):
    """Smallest and largest eigenvalue of the 6x6 Mandel blocks of a
    fourth-order tangent field over all voxels (Sec. 3.2, the extreme
    eigenvalues of D over the grid)."""
    from .projection import mandel_block
    M = mandel_block(C)
    Mv = np.moveaxis(M.reshape(6, 6, -1), -1, 0)
    w = np.linalg.eigvalsh(Mv)
    return float(w.min()), float(w.max())


@dataclasses.dataclass
class IncrementStats:
    newton_iters: int
    cg_iters: List[int]
    newton_res: List[float]
    Sigma: np.ndarray
    converged: bool
    seconds: float


class Solver:
    """Algorithm 1 on one RVE, full 3x3 tensor fields in float64."""

    def __init__(self, phase, materials, tol_newton=1e-5, tol_cg=1e-8,
                 max_newton=50, max_cg=2000, zero_rhs_rel=1e-14,
                 predictor: str = "tangent", dt: float = 1.0, scheme: str = "galerkin"):
        self.phase = np.asarray(phase)
        self.shape = tuple(self.phase.shape)
        for n in self.shape:
            if n % 2 == 0 or n < 1:
                raise ValueError("grid extents must be odd and positive")
        self.materials = [tuple(m) for m in materials]
        self.dt = dt  # real time step of every increment (rate-dependent laws, Sec. 4.3)
        self.K, self.G, self.sy0, self.H, _n = j2.material_fields(self.phase, self.materials)
        self.j2_only = bool(np.all(laws.material_rows(self.materials)[:, 5] == laws.LAW_J2))
        self.tol_newton = tol_newton
        self.tol_cg = tol_cg
        self.max_newton = max_newton
        self.max_cg = max_cg
        self.zero_rhs_rel = zero_rhs_rel
        if predictor not in ("tangent", "none"):
            raise ValueError("predictor must be 'tangent' or 'none'")
        self.predictor = predictor
        if scheme not in ("galerkin", "basic"):
            raise ValueError("scheme must be 'galerkin' or 'basic'")
        # galerkin: G C d = -G sigma by CG (Eq. linear_system); basic: the
        # collocation system Gamma_ref C d = -Gamma_ref sigma (Eq.
        # linear_system_L-S) with C_ref = 1/2 (lmin + lmax) I_s of the tangent
        # of each Newton iteration, by Richardson (Sec. 3.2)
        self.scheme = scheme
        self.c_ref: List[float] = []       # reference stiffness of each linear solve (basic scheme)
        z = (3, 3) + self.shape
        self.eps_fl = np.zeros(z)          # fluctuation eps*
        self.eps_p = np.zeros(z)           # committed plastic strain
        self.epbar = np.zeros(self.shape)  # committed accumulated plastic strain
        self.E = np.zeros((3, 3))
        self.increment = 0
        self.sigma = np.zeros(z)
        # consistent tangent at the last converged state (elastic initially)
        self.C_last = (j2.elastic_stiffness(self.K, self.G) if self.j2_only
                       else laws.elastic_tangent(self.phase, self.materials))

    @property
    def nvox(self) -> int:
        return int(np.prod(self.shape))

    def constitutive(self, eps_fl):
        eps = eps_fl + self.E[:, :, None, None, None]
        return laws.constitutive(self.phase, self.materials, eps, self.eps_p, self.epbar, self.dt)

    def _operator(self, C):
        """The operator of the linear system about tangent C: G, or for the
        basic scheme Gamma_ref of C_ref = 1/2 (lmin + lmax) I_s (Appendix A,
        Eq. Gamma_explicit)."""
        if self.scheme == "galerkin":
            return apply_G
        from .projection import apply_operator_hat, gamma_ref_hat
        lo, hi = tangent_eigen_bounds(C)
        c = 0.5 * (lo + hi)
        self.c_ref.append(c)
        Gh = gamma_ref_hat(self.shape, c * j2.I4S)
        return lambda tau: apply_operator_hat(Gh, tau)

    def _linear_step(self, C, b, force, op=apply_G):
        """CG (or, basic scheme, Richardson) solve of op C d = b.

        The residual target is max(eta_CG ||b||, 1e-14 ||s||), where s is
        the field whose projection gave b (sigma, or C_last : dE for the
        predictor): G s cannot be evaluated more accurately than rounding
        of s, so a target below that floor is unreachable.  A right-hand
        side already under the target gives d = 0 without iterating.
        """
        solve = cg if self.scheme == "galerkin" else richardson
        res = solve(lambda p: op(j2.ddot42(C, p)), b, self.tol_cg,
                    self.max_cg, force_iters=force,
                    atol=self.zero_rhs_rel * self._rhs_scale)
        if res.breakdown:
            raise FloatingPointError("CG breakdown: indefinite tangent")
        return res.x, res.iters

    def solve_increment(self, E_new, lockstep: Optional[List[int]] = None) -> IncrementStats:
        """Advance the mean strain to E_new and solve (Algorithm 1 body).

        With predictor == "tangent" the first iteration of the increment is
        the linearised load step G C_last d = -G C_last dE about the last
        converged state (C_last = its consistent tangent); every further
        iteration evaluates the return map at E_new + eps* (Algorithm 1,
        constitutive response and consistent tangent) and at least one such
        iteration always follows the predictor.  With predictor == "none"
        every iteration is of the second kind (Algorithm 1 as printed).

        lockstep, when given, lists the CG iteration count of every Newton
        iteration (predictor included) and fixes the Newton count to its
        length.
        """
        t0 = time.perf_counter()
        E_old = self.E
        self.E = np.array(E_new, dtype=float)
        dE = self.E - E_old
        Enorm = math.sqrt(float(np.sum(self.E * self.E))) * math.sqrt(self.nvox)
        if Enorm == 0.0:
            Enorm = 1.0
        cg_counts: List[int] = []
        res_hist: List[float] = []
        converged = False
        i = 0
        if self.predictor == "tangent":
            dE_field = np.broadcast_to(dE[:, :, None, None, None], (3, 3) + self.shape)
            t = j2.ddot42(self.C_last, dE_field)
            op = self._operator(self.C_last)
            b = -op(t)
            self._rhs_scale = math.sqrt(fdot(t, t))
            force = None if lockstep is None else lockstep[0]
            d, its = self._linear_step(self.C_last, b, force, op)
            self.eps_fl = self.eps_fl + d
            cg_counts.append(its)
            res_hist.append(math.sqrt(fdot(d, d)) / Enorm)
            i = 1
        first_full = i
        while True:
            if lockstep is not None and i >= len(lockstep):
                converged = True
                break
            if lockstep is None and i >= self.max_newton:
                break
            sigma, C, _, _, _ = self.constitutive(self.eps_fl)
            op = self._operator(C)
            b = -op(sigma)
            self._rhs_scale = math.sqrt(fdot(sigma, sigma))
            force = None if lockstep is None else lockstep[i]
            d, its = self._linear_step(C, b, force, op)
            self.eps_fl = self.eps_fl + d
            r = math.sqrt(fdot(d, d)) / Enorm
            cg_counts.append(its)
            res_hist.append(r)
            i += 1
            if lockstep is None and r <= self.tol_newton and i > first_full:
                converged = True
                break
        # commit the history at the converged strain (Algorithm 1, end of increment)
        sigma, C, ep, eb, _ = self.constitutive(self.eps_fl)
        self.eps_p, self.epbar, self.sigma = ep, eb, sigma
        self.C_last = C
        self.increment += 1
        Sigma = sigma.reshape(3, 3, -1).mean(axis=2)
        return IncrementStats(i, cg_counts, res_hist, Sigma, converged,
                              time.perf_counter() - t0)

    def strain(self) -> np.ndarray:
        return self.eps_fl + self.E[:, :, None, None, None]


def run_workload(w, lockstep=None, n_inc=None, predictor="tangent", dt=1.0, scheme="galerkin"):
    """Run the load path of a synth.Workload; returns (solver, [stats])."""
    s = Solver(w.phase, w.materials, w.tol_newton, w.tol_cg, predictor=predictor, dt=dt, scheme=scheme)
    out = []
    for n in range(1, (n_inc or w.n_inc) + 1):
        ls = None if lockstep is None else lockstep[n - 1]
        out.append(s.solve_increment(w.E_at(n), ls))
    return s, out
