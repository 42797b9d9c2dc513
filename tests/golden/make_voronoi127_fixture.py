"""Writes the oracle fixture of the 127^3 Voronoi RVE (mixed-precision
workload): the FP64 oracle's solve of its first increments, stored compactly
for the GPU parity test of that workload (too large for the oracle to run
inside a test).

Calls only the oracle (oracle/) and the seeded input generators (synth/).
Stored per increment n = 1..N_INC (arrays indexed [n-1]):
  cg_counts     CG iterations of every Newton iteration (flat, with offsets),
                so the GPU can replay the oracle's path in lockstep;
  newton_res    ||d eps*|| / ||E|| of every Newton iteration (flat, same offsets);
  Sigma         volume average of sigma (3x3);
  strain_s      total strain at the sample voxels (3x3 x n_samples);
  epbar_s       accumulated plastic strain at the sample voxels;
  rel_eq        ||G sigma|| / ||sigma|| at the committed state
                (Eq. nodal_equilibrium_equations);
and once: sample (the sampled voxel indices, seeded) and the tolerances.

Usage: python tests/golden/make_voronoi127_fixture.py [--tight] [--n-inc N]
  default: the workload's own tolerances (eta_NW 1e-5, eta_CG 1e-8)
  --tight: eta_NW 1e-10, eta_CG 1e-13 (the discrete solution itself)
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import solver as S  # noqa: E402
from oracle.projection import apply_G  # noqa: E402

N_SAMPLES = 4096


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--tight", action="store_true")
    ap.add_argument("--n-inc", type=int, default=3)
    args = ap.parse_args()
    w = synth.voronoi_127(precision="fp64")
    tol_nw, tol_cg = (1e-10, 1e-13) if args.tight else (w.tol_newton, w.tol_cg)
    s = S.Solver(w.phase, w.materials, tol_nw, tol_cg)
    rng = np.random.default_rng(127127)
    sample = np.stack([rng.integers(0, n, N_SAMPLES) for n in w.shape])
    idx = tuple(sample)
    out = {"sample": sample, "tol_newton": tol_nw, "tol_cg": tol_cg, "n_inc_total": w.n_inc}
    cg, res, offs, Sig, strain_s, epbar_s, rel_eq = [], [], [0], [], [], [], []
    for n in range(1, args.n_inc + 1):
        t0 = time.perf_counter()
        st = s.solve_increment(w.E_at(n))
        assert st.converged, f"increment {n} did not converge"
        cg += st.cg_iters
        res += st.newton_res
        offs.append(len(cg))
        Sig.append(st.Sigma)
        strain_s.append(s.strain()[(slice(None), slice(None)) + idx])
        epbar_s.append(s.epbar[idx])
        g = apply_G(s.sigma)
        rel_eq.append(float(np.sqrt(np.sum(g * g) / np.sum(s.sigma * s.sigma))))
        print(f"increment {n}: newton {st.newton_iters} cg {st.cg_iters} rel_eq {rel_eq[-1]:.3e} "
              f"({time.perf_counter() - t0:.0f} s)", flush=True)
    out.update(cg_counts=np.array(cg, dtype=np.int64), newton_res=np.array(res), offsets=np.array(offs),
               Sigma=np.array(Sig), strain_s=np.array(strain_s), epbar_s=np.array(epbar_s),
               rel_eq=np.array(rel_eq))
    name = "voronoi127_oracle_tight.npz" if args.tight else "voronoi127_oracle.npz"
    np.savez_compressed(os.path.join(HERE, name), **out)
    print("wrote", name)


if __name__ == "__main__":
    main()
