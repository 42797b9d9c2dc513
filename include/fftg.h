/* fftg.h -- C ABI of the Galerkin-FFT Newton--CG solver for periodic
 * small-strain micromechanics on AMD Instinct MI355X (gfx950).
 *
 * Method: Zeman, de Geus, Vondrejc, Peerlings, Geers, "A finite element
 * perspective on non-linear FFT-based micromechanical simulations"
 * (arXiv:1601.05970).  Given a periodic cell sampled on an odd regular grid
 * (Sec. 2.3), a phase map, phases of the three constitutive laws of Sec. 4
 * (elasto-plasticity with power-law hardening, non-linear elasticity,
 * visco-plasticity) and a mean-strain path E(t), the library finds the
 * fluctuating strain eps* with G sigma(E + eps*) = 0 (Eq.
 * nodal_equilibrium_equations) by the
 * incremental Newton--conjugate-gradient iteration of Algorithm 1, applying
 * the projection G = F^-1 G^ F (Eq. discrete_projection) matrix-free with
 * FFTs and G^(k) of Appendix A (Eq. FT_projection) evaluated on the fly.
 *
 * Conventions for every entry point
 * ---------------------------------
 * Grid: extents n0, n1, n2 >= 1, all odd (even grids are not conforming,
 *   Sec. 2.3).  Axis 0 = x is slowest, axis 2 = z fastest (C order).
 *   Supported extents: products of 3, 5, 7, 11, 13, 17, primes p whose
 *   p - 1 is a product of 2, 3, 4, 5, 7, 9, 11, 13, 17 (e.g. 11, 15, 31, 63,
 *   127, 255), and any odd extent up to 64 (direct DFT); others give
 *   FFTG_E_UNSUPPORTED.  Cell size L_i = n_i.
 * Tensor fields on the device: 6 contiguous planes of n0*n1*n2 values each,
 *   Mandel order [11, 22, 33, sqrt2*e23, sqrt2*e13, sqrt2*e12] (Appendix B,
 *   extended to 3-D).  Host 6-vectors in this API (dE, E, Sigma) are plain
 *   tensor components [11, 22, 33, 23, 13, 12] without Mandel weights.
 * Ownership: host arrays passed to a call are copied before it returns.
 *   Device pointers passed in (d_*) stay owned by the caller, must be
 *   device memory of the plan's device, sized as stated, and must not alias.
 * Errors: every call returns an fftg_status; on failure fftg_last_error()
 *   gives a message (thread-local).  No C++ exception crosses the ABI.
 * Streams: all device work of a plan is ordered on the stream given at plan
 *   creation (NULL = default stream).  Calls that return host results
 *   synchronise that stream; fftg_apply_GK is asynchronous.
 * Threads: a plan, its histories and batches are not thread-safe; distinct
 *   plans may be used from distinct threads.
 */
#ifndef FFTG_H
#define FFTG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FFTG_OK = 0,
  FFTG_E_INVALID = -1,        /* bad argument (null, even extent, phase id, parameter) */
  FFTG_E_NOMEM = -2,          /* device or pinned host allocation failed */
  FFTG_E_HIP = -3,            /* a HIP runtime call failed */
  FFTG_E_NOT_CONVERGED = -4,  /* Newton or CG iteration cap reached; stats filled */
  FFTG_E_BREAKDOWN = -5,      /* CG met p.Ap <= 0 or not finite (indefinite tangent); stats filled */
  FFTG_E_UNSUPPORTED = -6,    /* grid extent or material law not implemented */
  FFTG_E_NONFINITE = -7       /* the stress or the Newton update became NaN or infinite
                                 (e.g. a non-finite strain handed in); stats filled */
} fftg_status;

typedef enum { FFTG_FP64 = 0, FFTG_MIXED = 1 } fftg_precision;

/* Constitutive operator used inside the product G:(C:p). */
typedef enum {
  FFTG_TANGENT_CURRENT = 0,  /* consistent tangent held by the history */
  FFTG_TANGENT_IDENTITY = 1, /* C = identity: plain projection G p */
  FFTG_TANGENT_ELASTIC = 2   /* elastic stiffness Ce of each voxel's phase */
} fftg_tangent_mode;

/* First Newton iteration of an increment.
 * TANGENT: linearised load step G C_last d = -G C_last dE about the last
 *   converged state (C_last = its consistent tangent), then full Newton
 *   iterations (at least one).  NONE: Algorithm 1 exactly as printed, every
 *   iteration starting from the return map at E_new + eps*. */
typedef enum { FFTG_PREDICTOR_TANGENT = 0, FFTG_PREDICTOR_NONE = 1 } fftg_predictor;

/* How each linearised system is set up and solved.
 * GALERKIN: G C d = -G sigma (Eq. linear_system) by conjugate gradients
 *   (Algorithm 1).
 * BASIC: the collocation scheme of Sec. 3.2, Gamma_ref C d = -Gamma_ref sigma
 *   (Eqs. L-S_discrete, linear_system_L-S) with Gamma_ref of Appendix A
 *   (Eq. Gamma_explicit) for C_ref = 1/2 (lambda_min + lambda_max) I_s, the
 *   extreme eigenvalues of the tangent over all voxels, renewed every Newton
 *   iteration, solved by the Richardson iteration d <- d - Gamma_ref (C d +
 *   sigma) (the basic scheme); iteration counts grow with lambda_max /
 *   lambda_min instead of its square root.  FP64 plans only. */
typedef enum { FFTG_SCHEME_GALERKIN = 0, FFTG_SCHEME_BASIC = 1 } fftg_scheme;

/* Constitutive law of a phase (Sec. 4). */
typedef enum {
  FFTG_LAW_J2 = 0,                /* elasto-plasticity, Sec. 4.2 */
  FFTG_LAW_NONLINEAR_ELASTIC = 1, /* non-linear elasticity, Sec. 4.1 */
  FFTG_LAW_VISCO = 2              /* visco-plasticity, Sec. 4.3 */
} fftg_law;

/* One phase.  Fields by law:
 * J2 (Eqs. model:plas:stress, model:plas:yield): bulk modulus K > 0, shear
 *   modulus G > 0, initial yield stress sigma_y0 > 0, hardening modulus
 *   H >= 0, hardening exponent 0 < n <= 1 (n = 1: closed-form return; else
 *   the scalar return equation is solved per voxel); eps0, t0 unused.
 * NONLINEAR_ELASTIC (Eq. model:nlin:stress): K > 0, reference stress
 *   sigma_y0 = sigma_0 > 0, reference strain eps0 > 0, exponent n >= 1; G > 0
 *   only sets the ELASTIC product (fftg_apply_GK) of the phase; H unused.
 *   Its tangent at zero strain has no deviatoric stiffness for n > 1, so
 *   solves of such phases take FFTG_PREDICTOR_NONE.
 * VISCO (Eq. model:visco:gammadot): K > 0, G > 0, sigma_y0 = sigma_0 > 0,
 *   rate-sensitivity exponent 0 < n <= 1, eps0 > 0, t0 > 0 (gamma_0 =
 *   eps0 / t0); the time step is fftg_options.dt; H unused.
 * Other exponents give FFTG_E_UNSUPPORTED (the compact consistent tangent
 * stores the rank-one term with one sign per phase). */
typedef struct {
  double K, G, sigma_y0, H, n;
  int law;            /* fftg_law */
  double eps0, t0;
} fftg_material;

typedef struct {
  int precision;          /* fftg_precision */
  double tol_newton;      /* eta_NW: stop when ||d eps*|| / ||E|| <= tol (E as nodal column) */
  double tol_cg;          /* eta_CG: stop when ||r|| <= tol ||G s|| */
  int max_newton;         /* Newton iterations per increment (<= FFTG_MAX_NEWTON) */
  int max_cg;             /* CG iterations per Newton iteration */
  int predictor;          /* fftg_predictor */
  double rhs_floor;       /* CG also stops at ||r|| <= rhs_floor ||s|| (default 1e-14) */
  double mixed_cg_floor;  /* MIXED only: effective eta_CG >= this, and the floor of the
                             FP32-evaluated predictor right-hand side (default 1e-5) */
  int cg_chunk;           /* CG iterations enqueued between host checks (default 16) */
  double dt;              /* real time step of every increment, for VISCO phases (default 1) */
  int scheme;             /* fftg_scheme (default GALERKIN) */
} fftg_options;

#define FFTG_MAX_NEWTON 64

typedef struct {
  int newton_iters;
  int cg_iters[FFTG_MAX_NEWTON];
  double newton_res[FFTG_MAX_NEWTON]; /* ||d eps*|| / ||E|| per Newton iteration */
  double Sigma[6];                    /* volume average of sigma after the increment */
  int converged;                      /* 1 when the Newton test was met (or lockstep done) */
  int total_cg;                       /* sum of cg_iters */
  double seconds;                     /* wall time of the call */
  double rel_equilibrium;             /* ||G sigma|| / ||sigma|| at the committed state: how far
                                         the result is from nodal equilibrium (Eq.
                                         nodal_equilibrium_equations); 0 when sigma = 0 */
} fftg_stats;

typedef struct fftg_plan_s* fftg_plan;
typedef struct fftg_history_s* fftg_history;
typedef struct fftg_batch_s* fftg_batch;

/* Fills *opt with defaults: FP64, tol_newton 1e-5, tol_cg 1e-8,
 * max_newton 50, max_cg 2000, TANGENT predictor, rhs_floor 1e-14,
 * mixed_cg_floor 1e-5, cg_chunk 16, dt 1, GALERKIN scheme. */
void fftg_options_default(fftg_options* opt);

/* Creates a plan for one RVE (Sec. 2.3 grid, Sec. 4 phases).
 * phase: host, n0*n1*n2 bytes, C order, values < n_phases.
 * mats: host, n_phases entries (n_phases <= 16).  opt: NULL = defaults.
 * hip_stream: a hipStream_t or NULL.  Allocates the device work buffers. */
fftg_status fftg_plan_create(fftg_plan* out, int n0, int n1, int n2, const uint8_t* phase, int n_phases,
                             const fftg_material* mats, const fftg_options* opt, void* hip_stream);
void fftg_plan_destroy(fftg_plan plan);

/* Device state of one load path on a plan: eps* = 0, eps_p = 0,
 * eps_p_bar = 0, E = 0, tangent = elastic (Algorithm 1, initial conditions). */
fftg_status fftg_history_create(fftg_plan plan, fftg_history* out);
void fftg_history_destroy(fftg_history hist);

/* One increment of Algorithm 1: E <- E + dE, Newton--CG to convergence,
 * then the history commit (eps_p, eps_p_bar, tangent, Sigma).
 * dE: host, 6 tensor components.  lockstep: NULL for natural stopping, or
 * n_lockstep CG counts that fix the number of Newton iterations and the CG
 * iterations of each (used to replay another implementation's path).
 * stats: may be NULL.  Returns FFTG_E_NOT_CONVERGED / FFTG_E_BREAKDOWN /
 * FFTG_E_NONFINITE with stats filled (Sigma: average stress at the last
 * iterate) and the history not committed: E and eps* stay at the last
 * iterate, eps_p and eps_p_bar keep the values committed at the end of the
 * previous increment (a caller may restore a checkpoint and retry with a
 * smaller dE). */
fftg_status fftg_solve_increment(fftg_plan plan, fftg_history hist, const double dE[6], const int* lockstep,
                                 int n_lockstep, fftg_stats* stats);

/* d_out = G:(C:d_in) (Eq. linear_system operator; Eq. discrete_projection
 * for G).  d_in: device double, 6 planes.  d_out: device, 6 planes of double
 * (FP64 plan) or float (MIXED plan).  hist supplies the CURRENT tangent and
 * may be NULL for IDENTITY / ELASTIC.  Asynchronous on the plan's stream. */
fftg_status fftg_apply_GK(fftg_plan plan, fftg_history hist, const double* d_in, void* d_out,
                          fftg_tangent_mode mode);

/* d_out = Gamma_ref : d_in, the Green operator of the collocation scheme
 * (Sec. 3.2, Eq. L-S_discrete) for the isotropic reference medium
 * C_ref = lam0 I(x)I + 2 mu0 I_s (mu0 > 0, lam0 + 2 mu0 > 0), built per
 * frequency from the acoustic tensor (Appendix A, Eq. Gamma_explicit); with
 * lam0 = 0, mu0 = 1/2 (C_ref = I_s) it is G.  d_in, d_out: device double,
 * 6 planes.  FP64 plans only.  Asynchronous on the plan's stream. */
fftg_status fftg_apply_Gamma(fftg_plan plan, const double* d_in, double* d_out, double lam0, double mu0);

/* Return map (Sec. 4.2) at the total strain d_eps (device double, 6 planes)
 * from the history's committed eps_p, eps_p_bar, without committing.
 * Writes sigma to d_sigma (device double, 6 planes) and sets the history's
 * CURRENT tangent. */
fftg_status fftg_eval_constitutive(fftg_plan plan, fftg_history hist, const double* d_eps, double* d_sigma);

typedef enum {
  FFTG_FIELD_FLUCT = 0,   /* eps*, 6 planes */
  FFTG_FIELD_STRAIN = 1,  /* E + eps*, 6 planes */
  FFTG_FIELD_STRESS = 2,  /* sigma of the last return map, 6 planes */
  FFTG_FIELD_EPS_P = 3,   /* committed plastic strain, 6 planes */
  FFTG_FIELD_EPBAR = 4,   /* committed accumulated plastic strain, 1 plane */
  FFTG_FIELD_TANGENT = 5  /* compact tangent {2G', m}, 7 planes, plan's apply precision */
} fftg_field;

/* Copies a field to d_out (device, sized as listed; double unless noted).
 * Synchronises the plan's stream. */
fftg_status fftg_get_field(fftg_plan plan, fftg_history hist, int which, void* d_out);
/* Overwrites FLUCT, EPS_P or EPBAR from d_in (device double). */
fftg_status fftg_set_field(fftg_plan plan, fftg_history hist, int which, const void* d_in);
/* Mean strain E (6 tensor components) and completed increment count. */
fftg_status fftg_history_get_E(fftg_history hist, double E[6], int* increments);

/* Checkpoint of a history (end of an increment): eps*, eps_p, eps_p_bar,
 * tangent, E and the increment count, to / from a host buffer.
 * fftg_history_save with host_buf NULL sets *bytes to the size needed. */
fftg_status fftg_history_save(fftg_plan plan, fftg_history hist, void* host_buf, size_t* bytes);
fftg_status fftg_history_restore(fftg_plan plan, fftg_history hist, const void* host_buf, size_t bytes);

/* Device bytes one plan plus one history of this grid and precision take
 * (admission control). */
size_t fftg_footprint_bytes(int n0, int n1, int n2, int precision);

/* Many (plan, history) pairs advanced together: every launch covers the
 * tiles of all members, so RVEs of different size share each kernel.
 * Plans must share one precision and the stream of plans[0] is used. */
fftg_status fftg_batch_create(fftg_batch* out, int count, const fftg_plan* plans, const fftg_history* hists);
void fftg_batch_destroy(fftg_batch batch);
/* One increment for every member: dE is host count*6; lockstep NULL;
 * stats: host array of count (may be NULL).  A member that fails to
 * converge is reported in its stats; the call returns the first error. */
fftg_status fftg_batch_solve_increment(fftg_batch batch, const double* dE, fftg_stats* stats);

/* Event timing of one kernel kind, for benchmarks and tracing.  While the
 * profiler runs, every launch of that kernel (any plan or batch) is
 * bracketed by two HIP events on the stream it is launched on.  stop
 * synchronises the recorded events and returns the summed kernel time in
 * milliseconds, the number of launches and the voxels those launches
 * covered (sum over the RVEs each launch processed); any output may be
 * NULL.  Safe to call while other threads solve on distinct plans. */
typedef enum {
  FFTG_KERNEL_ZFWD = 0,        /* p update + p.(C:p), tangent contraction, real-to-complex DFT along z */
  FFTG_KERNEL_Y_FWD = 1,       /* DFT along y */
  FFTG_KERNEL_X_PROJ = 2,      /* DFT along x, G^(k) projection, inverse DFT along x */
  FFTG_KERNEL_Y_INV = 3,       /* inverse DFT along y */
  FFTG_KERNEL_ZINV = 4,        /* complex-to-real inverse DFT along z + CG x, r update and r.r */
  FFTG_KERNEL_FINALIZE = 5,    /* per-RVE totals of tile partial sums, CG scalar steps */
  FFTG_KERNEL_CONSTITUTIVE = 6,/* J2 return map + consistent tangent */
  FFTG_KERNEL_NEWTON = 7,      /* eps* += d eps, ||d eps|| */
  FFTG_KERNEL_COUNT = 8
} fftg_kernel_id;
fftg_status fftg_profiler_start(int kernel_id);
/* As fftg_profiler_start, but brackets only launches 0, every, 2 every, ...
 * of that kind (every >= 1; FFTG_E_INVALID otherwise): each pair of events
 * adds a few microseconds of queue processing between kernels, which
 * sampling keeps out of most of a timed run.  stop then reports the
 * bracketed launches only; fftg_profiler_seen gives all of them. */
fftg_status fftg_profiler_start_every(int kernel_id, int every);
fftg_status fftg_profiler_stop(double* total_ms, long long* launches, double* voxels);
/* As fftg_profiler_start_every for every kind whose bit (1 << kernel_id) is
 * set in kernel_mask (nonzero, below 1 << FFTG_KERNEL_COUNT), sampled per
 * kind; stop and seen then report the sums over those kinds. */
fftg_status fftg_profiler_start_set(unsigned kernel_mask, int every);
/* Totals of one kind from the last run, valid after fftg_profiler_stop:
 * summed time of its bracketed launches (ms), their count, the voxels they
 * covered, and all its launches (bracketed or not); any output may be NULL. */
fftg_status fftg_profiler_kind(int kernel_id, double* ms, long long* launches, double* voxels, long long* seen);
/* Launches of the profiled kind since the last start, bracketed or not
 * (kept after stop until the next start). */
long long fftg_profiler_seen(void);

const char* fftg_last_error(void);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * product of fftg_apply_GK in its IDENTITY or ELASTIC form, FP64, without a
 * plan and without any allocation.  d_out = G:(C:d_in) on an n0 x n1 x n2
 * grid, C = identity or the elastic stiffness Ce of each voxel's phase.
 * d_in, d_out: device double, 6 planes each (layout as everywhere above),
 * caller-owned, non-aliasing, on the current device.  ELASTIC: d_phase is
 * the device phase map (n0*n1*n2 bytes, ids < n_phases: not checked, the map
 * stays on the device), mats a host array of n_phases <= 16 entries (K, G
 * used); IDENTITY ignores both (may be NULL).  hip_stream: a stream of the
 * current device or NULL.  Asynchronous.
 * Work memory: one static device array of 16 MiB per device (held until the
 * process ends), holding the descriptor, the FFT root tables and the half
 * spectrum; grids whose half spectrum (6 n0 n1 (n2+1)/2 complex doubles)
 * exceeds 16 MiB - 64 KiB (63^3 fits, 75^3 does not) give FFTG_E_INVALID,
 * extents that need Rader's algorithm (primes above 53 and other extents
 * above 64 without a 3/5/7/11/13/17 factorisation) FFTG_E_UNSUPPORTED.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (several streams or threads) race and must be serialised by
 * the caller.  Each call rewrites everything it reads from the array. */
fftg_status fftg_apply_GK_noalloc(int n0, int n1, int n2, const double* d_in, double* d_out, fftg_tangent_mode mode,
                                  const uint8_t* d_phase, int n_phases, const fftg_material* mats,
                                  void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* FFTG_H */
