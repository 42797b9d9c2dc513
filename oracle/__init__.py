"""FP64 CPU oracle for the Galerkin-FFT Newton--CG solver (test infrastructure).

This package is test infrastructure, not part of the product.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it; the
HIP library never calls it and it never calls the HIP library.

It is a plain, slow, deliberately unoptimised restatement of the method of
Zeman, de Geus, Vondrejc, Peerlings and Geers, "A finite element perspective
on non-linear FFT-based micromechanical simulations" (arXiv:1601.05970):

* ``projection`` -- the projection operator G of Eq. (conv_def) applied as
  F^-1 G^ F (Eq. discrete_projection) with the explicit four-index G^(k) of
  Appendix A (Eq. FT_projection); the reference Green operator Gamma^ref of
  Appendix A (Eq. Gamma_explicit); dense DFT and projection matrices of
  Appendix B for brute-force checks on tiny grids.
* ``j2`` -- the elasto-plastic J2 model of Sec. 4.2 (power-law hardening):
  backward-Euler elastic predictor / plastic corrector and the consistent
  tangent, as full fourth-order tensors.
* ``laws`` -- the non-linear elastic (Sec. 4.1) and visco-plastic (Sec. 4.3)
  models, and the choice of law per voxel.
* ``solver`` -- conjugate gradients on the linearised system
  (Eq. linear_system) and the incremental-iterative Newton loop of
  Algorithm 1.

Everything works on full 3x3 tensor fields of shape (3, 3, n0, n1, n2) in
float64 (the paper's derivation is 2-D; its 3-D extension is the obvious one,
and the paper states the extension is direct).  The GPU library stores
6-component Mandel vectors instead; the two share no code.

Parity status per function is stated in each module header.
"""
