// Internal device/host structures of the Galerkin-FFT library.
//
// Data layout in HBM (one RVE, grid n0 x n1 x n2, all odd, C order, axis 2
// fastest):
//   * real symmetric tensor fields: 6 SoA planes of nvox values each, Mandel
//     order [11, 22, 33, sqrt2*23, sqrt2*13, sqrt2*12];
//   * spectrum: 6 SoA planes of n0 * n1 * H complex values, H = (n2+1)/2
//     (half spectrum along axis 2; odd n2 has no Nyquist bin);
//   * compact consistent tangent: 7 SoA planes {2G', m_0..m_5} with
//     C:p = (K - 2G'/3) tr(p) I + 2G' p - (m.p) m, K from the phase table.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fftg {

constexpr int kMaxStages = 8;
constexpr int kMaxPhases = 16;
constexpr int kMaxAxisLen = 1024;

// Aligned to its size, so that the compiler may always move a complex
// value with one 16-byte (FP64) or 8-byte (FP32) access: every complex
// array here (device allocations, LDS carve-ups, host vectors) starts on
// such a boundary and is indexed by whole elements.
template <class T>
struct alignas(2 * sizeof(T)) cx {
  T re, im;
};

// One transform length: either a Stockham chain of direct radices, or Rader's
// algorithm for a prime p with its length-(p-1) cyclic convolution done by a
// Stockham chain.
// How an axis is transformed: a Stockham chain over N, Rader's algorithm
// over prime N (chains over N-1), or the O(N^2) direct DFT from a root table.
enum AxisKind { AX_CHAIN = 0, AX_RADER = 1, AX_DIRECT = 2 };

struct AxisDev {
  int N;
  int rader;            // AX_CHAIN, AX_RADER or AX_DIRECT
  int M;                // chain length (N, or N-1 for Rader; N for the direct DFT)
  int nst;              // stages of the chain
  int radix[kMaxStages];
  // tables (device pointers); roots are exp(-2 pi i m / M), m < M
  const cx<double>* tw64;
  const cx<float>* tw32;
  // Rader only
  const int* perm_in;        // g^q mod N, q < M
  const int* perm_out;       // g^-m mod N, m < M
  const cx<double>* bf64;    // DFT_M(b)/M, b_q = exp(-2 pi i g^-q / N)
  const cx<double>* bi64;    // same with exp(+...)
  const cx<float>* bf32;
  const cx<float>* bi32;
};

// A phase on the device.  The elasto-plastic and visco-plastic laws share
// one return equation, seq_tr - 3G dg - sy - Hh (a0 + dg)^n = 0, with
// (sy, Hh, a0) = (sigma_y0, H, eps_p_bar) for J2 and (0, sigma_0 /
// (gamma_0 dt)^n, 0) for Norton's rule integrated by backward Euler; the
// non-linear elastic law uses sy = sigma_0 and e0 = eps_0.  csign is the sign
// of the rank-one term of the compact tangent (-1 except non-linear
// elasticity with n > 1).
enum LawDev { LAW_J2 = 0, LAW_NLE = 1, LAW_VISCO = 2 };
struct MatDev {
  double K, G, sy, Hh, n, csign, e0;
  int law, pad_;
};

// Per-RVE scalar state of the CG solve and the reductions.
struct CgState {
  double rr, rr_new, pAp, alpha, beta;
  double rr_prev;                      // r.r of the previous iteration (folded steps)
  double bnorm2, target2, snorm2, dnorm2;
  double eta2, floor2;
  double Sigma[6];
  // reference medium of the collocation scheme, C_ref = lam0 I(x)I + 2 mu0 I_s,
  // and the extreme eigenvalues of the tangent it was chosen from
  double lam0, mu0, lmin, lmax;
  int iters, done, force, max_iter, status;
  int rich;                            // 1: Richardson iteration (beta = 0, unit step) instead of CG
};

// Scalar steps of k_finalize (which partial sums it totals, and what for).
enum FinStep { FIN_SNORM = 0, FIN_RESID, FIN_PAP, FIN_RR, FIN_DNORM, FIN_SIGMA, FIN_LAMBDA };

enum CgStatus { CG_RUNNING = 0, CG_CONVERGED = 1, CG_MAXITER = 2, CG_BREAKDOWN = 3, CG_FORCED = 4 };

// Buffer roles referenced by kernels through the descriptor.
enum Role {
  R_EPS_FL = 0, R_EPS_P, R_EPBAR, R_SIG, R_X, R_R, R_P, R_P2, R_USER_IN, R_USER_OUT, R_NROLES
};

enum Pass { P_ZF = 0, P_Y, P_X, P_ZI, P_VEC, P_NPASS };

// Flag in the member-count argument of the tiled kernels: blocks are mapped
// to tiles XCD-contiguously.
constexpr int kLaunchRemap = 1 << 30;

struct RveDev {
  int n0, n1, n2, H;
  long long nvox, nspec;
  AxisDev ax[3];             // transforms of axes x, y, z (by value: one load less per kernel)
  void* buf[R_NROLES];       // double* except R_USER_OUT in mixed mode
  void* tang;                // 7 planes, double (FP64) or float (mixed)
  void* spec;                // 6 complex planes, sized for double
  const uint8_t* phase;
  int n_phases;
  int mixed;                 // apply precision: 0 double, 1 float
  CgState* cg;
  double* partial;           // per-block partial sums, >= tiles of any pass (p.(C:p) in CG)
  double* partial_rr;        // per-block partial sums of r.r in CG (disjoint from partial)
  double E[6];               // mean strain, Mandel
  double dE[6];              // load increment, Mandel
  int tiles[P_NPASS];        // tiles of each pass for this RVE
  int skip;                  // 1: RVE masked out of batched launches
  int fold;                  // 1: CG scalar steps folded into the consumer kernels
  // last: the kernels' scalar loads of the fields above stay within the
  // first kilobyte (with the table in the middle, the CG pointer sat past
  // 1.5 KB and the y and x passes of the 64-RVE batch ran 20 % slower)
  MatDev mats[kMaxPhases];
};

// Apply modes (kernel flags)
enum ApplyIn { IN_ROLE = 0, IN_CONST_DE = 1 };
enum Tangent { TAN_CURRENT = 0, TAN_IDENTITY = 1, TAN_ELASTIC = 2 };
// p update of the forward pass (kernel flag update_p)
enum PUpdate {
  PU_NONE = 0,   // product of the input role
  PU_CG = 1,     // p <- r + beta p (stopping test and beta folded in), partials of p.(C:p)
  PU_TIMING = 2  // as PU_CG with beta = 0, reading and writing no CG state (timing outside a solve)
};
enum ApplyOut {
  OUT_CG = 0,        // x += alpha p, r -= alpha G:(C:p) (alpha folded in), partials of r.r
  OUT_RESIDUAL = 1,  // write R and P, zero X, partials of r.r -> rr, bnorm2, target2
  OUT_PLAIN = 2,     // write the out role only
  OUT_CG_TIMING = 3  // as OUT_CG with alpha = 0, reading and writing no CG state (timing outside a solve)
};

struct LaunchCfg {
  int rows_per_tile;   // z passes
  int lines_y;         // y pass: h-block width
  int lines_x;         // x pass: h-block width (x 6 components)
  int vec_per_tile;    // elementwise kernels (voxels per tile)
  int threads_z, threads_y, threads_x, threads_v;
  int slab;            // 1: z and y transforms fused per y-z plane (k_slab_fwd / k_slab_inv)
  int threads_s;       // slab passes
  int big_radix;       // 1 when some axis needs the radix-11/13/17 codelets
  int direct31;        // bit a (0 x, 1 y, 2 z): every member takes axis a by the 31-point direct DFT
  int lext[3];         // per axis (0 x, 1 y, 2 z): LDS line-buffer extent, points per line (0: 2 x extent)
  int lext32x;         // the same for the FP32 x pass (its lines are not padded)
  int rtab[3];         // per axis: 1 when some member takes it by Rader's algorithm (full LDS tables)
  int xcd_remap;       // 1: blocks mapped to tiles XCD-contiguously
  int n0max, n1max, n2max;  // largest extents of the launch (LDS table sizing)
};

// Axes whose transform runs in place (the compile-time chains of 15, 63 and
// 255 points, and Rader's algorithm for 127 points over its compile-time
// 126-point chain): their lines need one buffer in LDS instead of two.
// Host (tile sizing) and device (buffer carving) agree through this test.
__host__ __device__ constexpr bool inplace_axis(int rader, int M) {
  return (rader == AX_CHAIN && (M == 15 || M == 63 || M == 255)) || (rader == AX_RADER && M == 126);
}
// LDS stride (points) of the x pass's lines of an n-point axis.  FP64
// 63-point lines are padded to 73 points: at stride 63 (-1 mod 16 in 16-byte
// units) the neighbouring lines of an in-place stage and the h-neighbours of
// the gather hit the same LDS banks, at 73 (9 mod 16) far fewer do (x pass
// 114 -> 110 us on the FP64 64-RVE batch).  FP32 lines, and the y and z
// passes' lines, keep stride n: padded, they ran slower.
__host__ __device__ constexpr int xline_stride(int rader, int M, int n, int fp32) {
  return (!fp32 && rader == AX_CHAIN && M == 63) ? 73 : n;
}
// LDS points per line that a member's transform of an n-point axis needs
// (xpass64: the FP64 x pass's stride): one stride in place, two for a
// ping-pong pair.  A launch sizes its tiles for the largest value over its
// members, so in-place members of a mixed launch still save space (a
// 63-point line in place takes about what a 31-point pair does).
__host__ __device__ constexpr int line_ext(int rader, int M, int n, int xpass64 = 0) {
  return (inplace_axis(rader, M) ? 1 : 2) * (xpass64 ? xline_stride(rader, M, n, 0) : n);
}

// Sizes of the RVEs a launch covers, from which the launch configuration is
// chosen (host).
struct GridSum {
  int n0 = 1, n1 = 1, n2 = 1;      // maxima over members
  long long rows = 0;               // sum of n0*n1
  long long yl = 0;                 // sum of 6*n0 (y-line groups per h)
  long long xl = 0;                 // sum of n1
  long long hmax = 1;
  long long vox = 0;
  int big = 0;
  int direct31 = 7;                 // bit a: every member's axis a is the 31-point direct DFT
  int lext[3] = {0, 0, 0};          // per axis: largest line_ext over members (0: 2 x extent)
  int lext32x = 0;                  // the FP32 x pass's (unpadded lines)
  int rtab[3] = {0, 0, 0};          // per axis: some member takes it by Rader's algorithm
};

// Host side (runtime.cpp): the heuristic launch configuration and the tile
// counts of every pass of one RVE under it.
LaunchCfg choose_cfg(const GridSum& gs);
void compute_tiles(const LaunchCfg& c, int n0, int n1, int n2, long long nvox, int tiles[P_NPASS]);

// Host side (kernels.hip): LDS bytes of the pass kernels and their launchers.
// (n is the largest extent of the launch, which sizes the tables; ext the
// largest line_ext, 0 for 2n; rtab 1 when some member takes the axis by
// Rader's algorithm, whose tables are larger.)
size_t lds_z(int mixed, int rows, int n2, int ext = 0, int rtab = 1);
size_t lds_y(int mixed, int lines, int n1, int ext = 0, int rtab = 1);
size_t lds_x(int mixed, int lines, int n0, int ext = 0, int rtab = 1);
size_t lds_slab(int mixed, int n1, int n2);
hipError_t launch_zfwd(int mixed, const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg, size_t lds,
                       int in_mode, int in_role, int tan_mode, int want_norm, int check_done, int update_p,
                       hipStream_t s);
hipError_t launch_ypass(int mixed, int dir, const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg,
                        size_t lds, int check_done, hipStream_t s);
hipError_t launch_xpass(int mixed, const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg, size_t lds,
                        double scale, int check_done, hipStream_t s, int gamma = 0);
hipError_t launch_tangent_bounds(const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg, hipStream_t s);
hipError_t launch_set_cref(const RveDev* rv, int nrve, double lam0, double mu0, hipStream_t s);
hipError_t launch_zinv(int mixed, const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg, size_t lds,
                       int out_mode, int out_role, int check_done, int p_role, hipStream_t s);
hipError_t launch_slab_fwd(int mixed, const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg, size_t lds,
                           int in_mode, int in_role, int tan_mode, int want_norm, int check_done, int update_p,
                           int p_in, int p_out, hipStream_t s);
hipError_t launch_slab_inv(int mixed, const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg, size_t lds,
                           int out_mode, int out_role, int check_done, int p_role, hipStream_t s);
hipError_t launch_newton_update(const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg, hipStream_t s);
hipError_t launch_finalize(const RveDev* rv, int nrve, int step, hipStream_t s);
hipError_t launch_constitutive(int mixed, const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg,
                               int eps_role, int commit, hipStream_t s);
hipError_t launch_cg_setup(const RveDev* rv, int nrve, double eta2, double floor2, int max_iter, int force,
                           hipStream_t s, int rich = 0);

}  // namespace fftg
