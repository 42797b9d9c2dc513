"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds input definitions only: phase maps, per-phase material
parameters, mean-strain load paths and solver tolerances.  It contains none
of the solver's arithmetic (no transforms, no projection, no constitutive
law), so that the FP64 oracle and the HIP library can both consume it while
sharing no code with each other.

Conventions
-----------
* Grids are ``(n0, n1, n2)`` with axis 0 = x (slowest) and axis 2 = z
  (fastest), C order.  Every extent is odd (paper, Sec. 2.3: odd grids keep
  the trigonometric approximation conforming).
* Mean strains are full symmetric 3x3 tensors (tensor components, no Mandel
  weights).
* Materials are tuples ``(K, G, sigma_y0, H, n)`` of the isotropic J2 model
  with power-law hardening (paper, Sec. 4.2); the workloads here use n = 1.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

# Elastic constants shared by every workload: K = 0.833, G = 0.386, i.e.
# E ~ 1.0 and nu ~ 0.3, the Poisson ratio of the dual-phase steel example
# (paper, Sec. 5.2).
K_BULK = 0.833
G_SHEAR = 0.386

SOFT = (K_BULK, G_SHEAR, 0.003, 0.004, 1.0)
HARD = (K_BULK, G_SHEAR, 0.006, 0.008, 1.0)


@dataclasses.dataclass
class Workload:
    """One RVE solve: grid, phase map, materials, load path and tolerances."""

    name: str
    phase: np.ndarray                      # uint8, shape (n0, n1, n2)
    materials: List[Tuple[float, float, float, float, float]]
    E_final: np.ndarray                    # 3x3 symmetric, tensor components
    n_inc: int
    tol_newton: float = 1e-5
    tol_cg: float = 1e-8
    precision: str = "fp64"                # "fp64" or "mixed"

    @property
    def shape(self) -> Tuple[int, int, int]:
        return tuple(int(s) for s in self.phase.shape)

    @property
    def nvox(self) -> int:
        return int(np.prod(self.phase.shape))

    def E_at(self, n: int) -> np.ndarray:
        """Mean strain after increment n (1-based): equal-sized increments."""
        return (float(n) / float(self.n_inc)) * self.E_final

    def dE(self, n: int) -> np.ndarray:
        return self.E_at(n) - self.E_at(n - 1)


# ---------------------------------------------------------------- load paths
def shear_xy(magnitude: float) -> np.ndarray:
    """E = E_xy (e1 (x) e2 + e2 (x) e1) (paper, Sec. 5.1 laminate load)."""
    E = np.zeros((3, 3))
    E[0, 1] = E[1, 0] = magnitude
    return E


def pure_shear_eq(E_eq: float) -> np.ndarray:
    """E = sqrt(3)/2 E_eq (e2 (x) e2 - e1 (x) e1) (paper, Sec. 5.2 load)."""
    E = np.zeros((3, 3))
    E[1, 1] = 0.5 * math.sqrt(3.0) * E_eq
    E[0, 0] = -0.5 * math.sqrt(3.0) * E_eq
    return E


def random_deviatoric_direction(rng: np.random.Generator, E_eq: float) -> np.ndarray:
    """Random traceless symmetric direction with von Mises equivalent strain E_eq.

    Five Gaussian coefficients in an orthonormal basis of deviatoric
    symmetric tensors, scaled so that sqrt(2/3 E:E) = E_eq.
    """
    s2, s6 = 1.0 / math.sqrt(2.0), 1.0 / math.sqrt(6.0)
    basis = [
        np.diag([s2, -s2, 0.0]),
        np.diag([-s6, -s6, 2.0 * s6]),
    ]
    for (i, j) in ((1, 2), (0, 2), (0, 1)):
        B = np.zeros((3, 3))
        B[i, j] = B[j, i] = s2
        basis.append(B)
    c = rng.standard_normal(5)
    D = sum(ci * Bi for ci, Bi in zip(c, basis))
    eq = math.sqrt(2.0 / 3.0 * float(np.sum(D * D)))
    return D * (E_eq / eq)


# ------------------------------------------------------------ microstructures
def laminate(n: int = 11, hard_layers: int = 4) -> np.ndarray:
    """Two-phase laminate: phase 1 where the x-index is below hard_layers."""
    ph = np.zeros((n, n, n), dtype=np.uint8)
    ph[:hard_layers] = 1
    return ph


def bernoulli(shape: Sequence[int], p_hard: float, seed) -> np.ndarray:
    """Each voxel hard (1) with probability p_hard, from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return (rng.random(tuple(shape)) < p_hard).astype(np.uint8)


def voronoi_labels(n: int, seeds: np.ndarray) -> np.ndarray:
    """Periodic Voronoi tessellation of the unit cube sampled at voxel centres.

    Each voxel centre (i + 1/2)/n is assigned the nearest seed under the
    periodic minimum-image distance; ties go to the lowest seed index.
    """
    from scipy.spatial import cKDTree

    c = (np.arange(n) + 0.5) / n
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    tree = cKDTree(np.mod(seeds, 1.0), boxsize=1.0)
    # query the two nearest seeds so that exact ties resolve to the lower id
    d, idx = tree.query(pts, k=2)
    lab = idx[:, 0].copy()
    tie = np.isclose(d[:, 0], d[:, 1], rtol=0.0, atol=1e-15)
    lab[tie] = np.minimum(idx[tie, 0], idx[tie, 1])
    return lab.reshape(n, n, n)


def voronoi_two_phase(n: int, n_grains: int, hard_fraction: float,
                      rng: np.random.Generator) -> np.ndarray:
    """Voronoi grains, round(hard_fraction * n_grains) of them hard."""
    seeds = rng.random((n_grains, 3))
    lab = voronoi_labels(n, seeds)
    n_hard = int(round(hard_fraction * n_grains))
    hard = rng.permutation(n_grains)[:n_hard]
    is_hard = np.zeros(n_grains, dtype=np.uint8)
    is_hard[hard] = 1
    return is_hard[lab]


# --------------------------------------------------------------- workloads
def laminate_11() -> Workload:
    """11^3 two-phase laminate in shear, E_xy ramped to 0.02 in 5 steps."""
    return Workload("laminate_11", laminate(11, 4), [SOFT, HARD],
                    shear_xy(0.02), 5)


def random_31(n: int = 31) -> Workload:
    """31^3 Bernoulli(0.3) two-phase RVE (seed 1), pure shear 0.02 in 10."""
    return Workload(f"random_{n}", bernoulli((n, n, n), 0.3, 1), [SOFT, HARD],
                    pure_shear_eq(0.02), 10)


def voronoi_127(n: int = 127, n_inc: int = 20, precision: str = "mixed") -> Workload:
    """Periodic Voronoi, 200 grains (seed 2), 20 % hard, pure shear 0.02."""
    rng = np.random.default_rng(2)
    seeds = rng.random((200, 3))
    lab = voronoi_labels(n, seeds)
    hard = rng.permutation(200)[:40]
    is_hard = np.zeros(200, dtype=np.uint8)
    is_hard[hard] = 1
    return Workload(f"voronoi_{n}", is_hard[lab], [SOFT, HARD],
                    pure_shear_eq(0.02), n_inc, precision=precision)


def batch_rve(r: int, n_inc: int = 10, precision: str = "fp64") -> Workload:
    """RVE r of the 64-RVE batch: N in {15,31,63}, hard fraction and yield
    contrast drawn from default_rng([3, r])."""
    rng = np.random.default_rng([3, r])
    n = int(rng.choice([15, 31, 63]))
    h = float(rng.uniform(0.1, 0.5))
    c = float(rng.uniform(1.5, 4.0))
    ph = (rng.random((n, n, n)) < h).astype(np.uint8)
    hard = (K_BULK, G_SHEAR, c * 0.003, c * 0.004, 1.0)
    return Workload(f"batch_{r}", ph, [SOFT, hard], pure_shear_eq(0.02),
                    n_inc, precision=precision)


def batch_64(n_inc: int = 10, precision: str = "fp64", count: int = 64) -> List[Workload]:
    return [batch_rve(r, n_inc, precision) for r in range(count)]


@dataclasses.dataclass
class Request:
    """One request of the served stream."""

    rid: int
    arrival: float            # seconds after stream start
    workload: Workload


def serving_stream(n_requests: int = 200, rate: float = 1.0, seed: int = 4,
                   sizes=(31, 63, 127, 255), weights=(0.4, 0.3, 0.2, 0.1)) -> List[Request]:
    """Poisson arrivals of Voronoi RVE solves of mixed size and precision."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        n = int(rng.choice(list(sizes), p=list(weights)))
        grains = int(rng.integers(50, 401))
        h = float(rng.uniform(0.1, 0.4))
        E = random_deviatoric_direction(rng, 0.02)
        n_inc = int(rng.integers(5, 21))
        prec = "fp64" if rng.random() < 0.5 else "mixed"
        sub = np.random.default_rng([4, rid])
        ph = voronoi_two_phase(n, grains, h, sub)
        w = Workload(f"req_{rid}", ph, [SOFT, HARD], E, n_inc, precision=prec)
        out.append(Request(rid, t, w))
    return out


def small_random(shape, p_hard=0.4, seed=0, E_eq=0.02, n_inc=3) -> Workload:
    """Small Bernoulli RVE of arbitrary odd shape for tests."""
    ph = bernoulli(shape, p_hard, seed)
    return Workload(f"small_{'x'.join(map(str, shape))}_{seed}", ph,
                    [SOFT, HARD], pure_shear_eq(E_eq), n_inc)


def random_field(shape, ncomp, seed, scale=1.0) -> np.ndarray:
    """Seeded standard-normal field of shape (ncomp,) + shape, float64."""
    rng = np.random.default_rng(seed)
    return scale * rng.standard_normal((ncomp,) + tuple(shape))


def random_sym_tensor_field(shape, seed, scale=1.0) -> np.ndarray:
    """Seeded symmetric 3x3 tensor field, shape (3, 3) + shape."""
    rng = np.random.default_rng(seed)
    A = scale * rng.standard_normal((3, 3) + tuple(shape))
    return 0.5 * (A + A.transpose(1, 0, *range(2, A.ndim)))
