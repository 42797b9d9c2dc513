// HIP kernels of the Galerkin-FFT Newton--CG hot path (gfx950).
//
// One application of G:(C:p) (paper Eq. linear_system, with G = F^-1 G^ F of
// Eq. discrete_projection) is five launches over a half spectrum:
//   zf : tau = C(x):p(x) per voxel, then real-to-complex DFT along axis 2
//        (two real rows packed into one complex line);
//   y  : complex DFT along axis 1, per component;
//   x  : complex DFT along axis 0 for all six components, the projection
//        G^(k):tau^(k) evaluated on the fly from k (Appendix A,
//        Eq. FT_projection, with G^(0) = 0), inverse DFT along axis 0;
//   y  : inverse DFT along axis 1;
//   zi : complex-to-real inverse DFT along axis 2;
// or, where a y-z plane fits in LDS, three (the slab passes fuse zf with y
// and y with zi).  Inside CG (Algorithm 1) the first pass also forms
// p <- r + beta p and the partial sums of p.(C:p), and the last one applies
// x += alpha p, r -= alpha G:(C:p) and sums r.r, so an iteration is the five
// (or three) product launches and nothing else.  The per-voxel J2 return map
// and consistent tangent (Sec. 4.2) and the Newton update are elementwise
// kernels.
//
// Every kernel walks a list of tiles that may span several RVEs (batched
// launches); a single solve is a batch of one.  Reductions are deterministic
// and free of atomics: per-tile partial sums, totalled in a fixed order by
// the consuming kernel (k_finalize, or every tile of the next kernel).
#include <hip/hip_runtime.h>

#include "fft_lds.h"
#include "fftg_internal.h"

namespace fftg {

constexpr double kSqrt2 = 1.41421356237309504880;

// ------------------------------------------------------------------ helpers
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  The bijection below hands XCD x a contiguous range of tiles, so
// neighbouring tiles that share cache lines are served by one L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int q = n >> 3, r = n & 7;
  const int x = b & 7, i = b >> 3;
  return x * q + min(x, r) + i;
}

// A kernel's nrve argument is the member count, with kLaunchRemap set when
// tiles are spread XCD-contiguously (an argument, so that it arrives with
// the first load of the kernel).  The descriptor array of a launch is
// followed by a prefix table of tile offsets, starts[pass][r] for
// r = 0..nrve; a block finds its RVE by binary search over that table.
// Members skipped from a launch own no tiles, so no block reaches them.
__device__ __forceinline__ bool launch_single(int nrve_arg) { return (nrve_arg & ~kLaunchRemap) == 1; }
__device__ __forceinline__ int find_rve(const RveDev* __restrict__ rv, int nrve_arg, int pass, int& tile) {
  const int nrve = nrve_arg & ~kLaunchRemap;
  const int br = xcd_tile(blockIdx.x, gridDim.x);  // formed unconditionally: no branch before the loads
  const int b = (nrve_arg & kLaunchRemap) ? br : (int)blockIdx.x;
  if (nrve == 1) {  // the grid is exactly the one RVE's tiles
    tile = b;
    return 0;
  }
  const int* __restrict__ st = reinterpret_cast<const int*>(rv + nrve) + pass * (nrve + 1);
  if (b >= st[nrve]) {
    tile = -1;
    return -1;
  }
  int lo = 0, hi = nrve;  // invariant: st[lo] <= b < st[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (st[mid] <= b) lo = mid;
    else hi = mid;
  }
  tile = b - st[lo];
  return lo;
}

// One DPP move of a double (two 32-bit halves); lanes whose source is out of
// the row, or whose row is masked off, read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, true);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 64 lanes of a full wave, returned to every lane: an inclusive
// scan within each row of 16 lanes (row shifts by 1, 2, 4, 8), then row 0's
// and row 2's totals into rows 1 and 3, and rows 0-1's total into rows 2 and
// 3 (row broadcasts of lanes 15 and 31), so that lane 63 holds the total; in
// registers, with no trip through the LDS crossbar.  Fixed order, so every
// wave of every tile adds the same values the same way.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0x111, 0xf>(v);  // row_shr:1
  v += dpp_f64<0x112, 0xf>(v);  // row_shr:2
  v += dpp_f64<0x114, 0xf>(v);  // row_shr:4
  v += dpp_f64<0x118, 0xf>(v);  // row_shr:8
  v += dpp_f64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the workgroup; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
  }
  __syncthreads();
  return r;
}

// The same total, formed identically by every thread after a single barrier
// (per-wave sums in sh[w], added in the same order as block_sum).
// Thread 0's flag travels in sh[8] and is returned to every thread: the
// one value that another tile of the launch may change while this one runs.
// The caller must not write sh[0..8] again before another barrier.
__device__ __forceinline__ double block_total(double v, int flag0, double* sh, int& flag) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  if (threadIdx.x == 0) sh[8] = flag0 ? 1.0 : 0.0;
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
  double r = 0.0;
  for (int i = 0; i < nw; ++i) r += sh[i];
  flag = sh[8] != 0.0;
  return r;
}

// block_sum for the last reduction of a kernel: valid in thread 0, one
// barrier (no later use of sh to protect).
__device__ __forceinline__ double block_sum_last(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) r += sh[i];
  }
  return r;
}

// Stores a tile's partial sums (nv values held by thread 0) at
// partial[i * ntiles + tile].  The per-RVE totals are formed by k_finalize,
// launched after the producer on the same stream: the kernel boundary makes
// the partials visible, so no fence or atomic is needed inside the producer
// (a device-scope fence costs an L2 write-back and invalidate per tile).
__device__ __forceinline__ void put_partials(const double* vals, int nv, double* partial, int ntiles, int tile) {
  if (threadIdx.x == 0)
    for (int i = 0; i < nv; ++i) partial[i * ntiles + tile] = vals[i];
}

// Sum of p[0..n) over the workgroup in a fixed order (two accumulators per
// thread, then the block tree); valid in thread 0.  Split in two so that a
// kernel can issue the loads of its own share early and reduce later:
// thread_partials is the per-thread part, block_sum the rest.  Each round
// issues sixteen loads before any add (indices past the end load element
// n - 1 and add zero), so up to 16 x blockDim partials cost one memory round
// trip.
__device__ __forceinline__ double thread_partials(const double* __restrict__ pp, int n) {
  const FFTG_GLOBAL double* p = gmem(pp);
  const int st = blockDim.x;
  constexpr int U = 16;
  double a0 = 0.0, a1 = 0.0;
  for (int t = threadIdx.x; t < n; t += U * st) {
    double v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) v[k] = p[min(t + k * st, n - 1)];
#pragma unroll
    for (int k = 0; k < U; k += 2) {
      a0 += (t + k * st < n) ? v[k] : 0.0;
      a1 += (t + (k + 1) * st < n) ? v[k + 1] : 0.0;
    }
  }
  return a0 + a1;
}
__device__ double sum_partials(const double* __restrict__ p, int n, double* sh) {
  return block_sum(thread_partials(p, n), sh);
}

// Thread 0's copy of the CG stop flag, shared through LDS with the whole
// workgroup (its barrier also publishes the caller's LDS writes): in the
// kernels that apply a folded scalar step, tile 0 may set the flag while
// other tiles of the same launch start, and all threads of a tile must agree.
__device__ __forceinline__ int done_publish(int v) {
  __shared__ int s_done2;
  if (threadIdx.x == 0) s_done2 = v;
  __syncthreads();
  return s_done2;
}

// Compact consistent tangent applied to a Mandel vector:
// tau = (K - g2/3) tr(p) [1,1,1,0,0,0] + g2 p + csign (m.p) m.
template <class T>
__device__ __forceinline__ void tangent_apply(const T p[6], T K, T g2, const T m[6], T csign, T tau[6]) {
  const T tr = p[0] + p[1] + p[2];
  const T mp = csign * (m[0] * p[0] + m[1] * p[1] + m[2] * p[2] + m[3] * p[3] + m[4] * p[4] + m[5] * p[5]);
  const T lam = (K - g2 * T(1.0 / 3.0)) * tr;
#pragma unroll
  for (int c = 0; c < 6; ++c) tau[c] = g2 * p[c] + mp * m[c] + (c < 3 ? lam : T(0));
}

// G^(k) : T for a complex Mandel vector t, q = xi/|xi| (Appendix A):
// (G^ : T)_ij = q_i v_j + q_j v_i - (q.v) q_i q_j, v = T q.  Called with
// q = xi itself (not normalised), as = 1/|xi|^2 and scale carrying another
// 1/|xi|^2, it gives the same G^ : T without a square root: q_i v_j is then
// |xi|^2 times its normalised value and (q.v) q_i q_j is |xi|^4 times it,
// so the (q.v) term takes the extra factor as and the whole the factor in
// scale.
template <class T>
__device__ __forceinline__ void ghat_apply(cx<T> t[6], T q0, T q1, T q2, T scale, T as = T(1)) {
  const T r2 = T(1.0 / kSqrt2);
  cx<T> T11 = t[0], T22 = t[1], T33 = t[2];
  cx<T> T23 = {t[3].re * r2, t[3].im * r2};
  cx<T> T13 = {t[4].re * r2, t[4].im * r2};
  cx<T> T12 = {t[5].re * r2, t[5].im * r2};
  cx<T> v0 = {T11.re * q0 + T12.re * q1 + T13.re * q2, T11.im * q0 + T12.im * q1 + T13.im * q2};
  cx<T> v1 = {T12.re * q0 + T22.re * q1 + T23.re * q2, T12.im * q0 + T22.im * q1 + T23.im * q2};
  cx<T> v2 = {T13.re * q0 + T23.re * q1 + T33.re * q2, T13.im * q0 + T23.im * q1 + T33.im * q2};
  cx<T> a = {as * (q0 * v0.re + q1 * v1.re + q2 * v2.re), as * (q0 * v0.im + q1 * v1.im + q2 * v2.im)};
  const T s2 = T(kSqrt2) * scale;
  t[0] = {scale * (T(2) * q0 * v0.re - a.re * q0 * q0), scale * (T(2) * q0 * v0.im - a.im * q0 * q0)};
  t[1] = {scale * (T(2) * q1 * v1.re - a.re * q1 * q1), scale * (T(2) * q1 * v1.im - a.im * q1 * q1)};
  t[2] = {scale * (T(2) * q2 * v2.re - a.re * q2 * q2), scale * (T(2) * q2 * v2.im - a.im * q2 * q2)};
  t[3] = {s2 * (q1 * v2.re + q2 * v1.re - a.re * q1 * q2), s2 * (q1 * v2.im + q2 * v1.im - a.im * q1 * q2)};
  t[4] = {s2 * (q0 * v2.re + q2 * v0.re - a.re * q0 * q2), s2 * (q0 * v2.im + q2 * v0.im - a.im * q0 * q2)};
  t[5] = {s2 * (q0 * v1.re + q1 * v0.re - a.re * q0 * q1), s2 * (q0 * v1.im + q1 * v0.im - a.im * q0 * q1)};
}

// Gamma^ref(k) : T of the collocation scheme (Appendix A, Eq.
// Gamma_explicit) for an isotropic reference medium
// C_ref = lam0 I(x)I + 2 mu0 I_s: with the acoustic tensor
// A_il = C_ijlm q_j q_m = mu0 (q.q) delta_il + (lam0 + mu0) q_i q_l (q = xi/|xi|,
// Gamma^ref is of degree 0 in xi), w = A^-1 (T q) and
// (Gamma^ref : T)_ij = (q_i w_j + q_j w_i) / 2, i.e. the four terms of the
// explicit form contracted with a symmetric T.  A is inverted by cofactors.
template <class T>
__device__ __forceinline__ void gamma_apply(cx<T> t[6], T q0, T q1, T q2, T lam0, T mu0, T scale) {
  const T r2 = T(1.0 / kSqrt2);
  const cx<T> T11 = t[0], T22 = t[1], T33 = t[2];
  const cx<T> T23 = {t[3].re * r2, t[3].im * r2};
  const cx<T> T13 = {t[4].re * r2, t[4].im * r2};
  const cx<T> T12 = {t[5].re * r2, t[5].im * r2};
  const T qq = q0 * q0 + q1 * q1 + q2 * q2, a = lam0 + mu0;
  const T A00 = mu0 * qq + a * q0 * q0, A11 = mu0 * qq + a * q1 * q1, A22 = mu0 * qq + a * q2 * q2;
  const T A01 = a * q0 * q1, A02 = a * q0 * q2, A12 = a * q1 * q2;
  const T c00 = A11 * A22 - A12 * A12, c01 = A02 * A12 - A01 * A22, c02 = A01 * A12 - A02 * A11;
  const T c11 = A00 * A22 - A02 * A02, c12 = A01 * A02 - A00 * A12, c22 = A00 * A11 - A01 * A01;
  const T id = T(1) / (A00 * c00 + A01 * c01 + A02 * c02);
  const cx<T> v0 = {T11.re * q0 + T12.re * q1 + T13.re * q2, T11.im * q0 + T12.im * q1 + T13.im * q2};
  const cx<T> v1 = {T12.re * q0 + T22.re * q1 + T23.re * q2, T12.im * q0 + T22.im * q1 + T23.im * q2};
  const cx<T> v2 = {T13.re * q0 + T23.re * q1 + T33.re * q2, T13.im * q0 + T23.im * q1 + T33.im * q2};
  const cx<T> w0 = {id * (c00 * v0.re + c01 * v1.re + c02 * v2.re), id * (c00 * v0.im + c01 * v1.im + c02 * v2.im)};
  const cx<T> w1 = {id * (c01 * v0.re + c11 * v1.re + c12 * v2.re), id * (c01 * v0.im + c11 * v1.im + c12 * v2.im)};
  const cx<T> w2 = {id * (c02 * v0.re + c12 * v1.re + c22 * v2.re), id * (c02 * v0.im + c12 * v1.im + c22 * v2.im)};
  const T hs = T(0.5 * kSqrt2) * scale;
  t[0] = {scale * q0 * w0.re, scale * q0 * w0.im};
  t[1] = {scale * q1 * w1.re, scale * q1 * w1.im};
  t[2] = {scale * q2 * w2.re, scale * q2 * w2.im};
  t[3] = {hs * (q1 * w2.re + q2 * w1.re), hs * (q1 * w2.im + q2 * w1.im)};
  t[4] = {hs * (q0 * w2.re + q2 * w0.re), hs * (q0 * w2.im + q2 * w0.im)};
  t[5] = {hs * (q0 * w1.re + q1 * w0.re), hs * (q0 * w1.im + q1 * w0.im)};
}

__device__ __forceinline__ int sfreq(int m, int n) { return (2 * m < n) ? m : m - n; }

template <class T>
constexpr int kFp32 = std::is_same<T, float>::value ? 1 : 0;

// LDS carve-up for a tile: axis tables, Rader slots and the reduction
// scratch, then nl lines of stride ld and the ping-pong scratch.  An axis
// transformed in place never touches scratch, and the host sized the tile
// for the largest line_ext of the launch, so scratch may lie past the end
// of the allocation for such an axis: everything else sits before line, at
// offsets that do not depend on the transform.
template <class T>
struct TileLds {
  AxisLds<T> ax;
  cx<T>* line;
  cx<T>* scratch;
  cx<T>* dc;
  double* red;
  // The tables are only carved out: the kernel copies them with
  // axis_lds_fetch / axis_lds_store around its own loads.
  // Every offset is a multiple of 16 bytes that the compiler can see
  // (rounded up explicitly), so it keeps 16-byte LDS accesses on the lines.
  __device__ TileLds(char* base, int nl, int ld, const AxisDev& P, int ldmax) {
    axis_lds_setup<T>(P, base, ax);
    const size_t tb = axis_lds_bytes<T>(ldmax, P.rader == AX_RADER);
    const size_t db = ((size_t)(nl + 1) * sizeof(cx<T>) + 15) / 16 * 16;
    dc = reinterpret_cast<cx<T>*>(base + tb);
    red = reinterpret_cast<double*>(base + tb + db);
    line = reinterpret_cast<cx<T>*>(base + tb + db + 16 * sizeof(double));
    scratch = line + (size_t)nl * ld;
  }
};

// CG scalars read at the start of an iteration, loaded by every thread with
// the kernel's other loads and used after the step's barrier, when the loads
// have landed.  The address passes through a vector register (an empty
// asm): values loaded from a uniform address are otherwise moved to scalar
// registers, and so waited for, right where they are loaded.
struct CgPeekB {
  int done, iters, status, force, max_iter, rich;
  double rr_prev, target2, beta;
};
__device__ __forceinline__ const FFTG_GLOBAL CgState* cg_vaddr(CgState* cg) {
  __asm__ volatile("" : "+v"(cg));
  return gmem(cg);
}
__device__ __forceinline__ CgPeekB cg_peek_b(CgState* cg) {
  const FFTG_GLOBAL CgState* g = cg_vaddr(cg);
  return CgPeekB{g->done, g->iters, g->status, g->force, g->max_iter, g->rich, g->rr_prev, g->target2, g->beta};
}


// Start of a CG iteration in the kernel that forms p <- r + beta p.  With
// the scalar steps folded (rv.fold), every tile totals the r.r partials of
// the last vector update (same order in each tile, so the same value),
// applies the stopping test and forms beta; tile 0 publishes the state.
// Other tiles of the launch read only rr_prev, iters and status: tile 0
// writes no rr_prev or iters, and it writes CG_BREAKDOWN, the one status
// value tested, only where status already holds it (a breakdown is found by
// the vector update, which must not write the stop flag that its own tiles
// read; the solve stops here).  The stop flag itself may change under the
// launch, so only thread 0's copy counts (shared with the total through
// LDS); every thread then takes the same decision.  Returns false when the
// solve has stopped (the tile exits).  red needs 9 doubles; called by the
// whole workgroup.  PU_TIMING does the same loads and sums with beta = 0 and
// no state.
// (dn: the stop flag of this launch's test, as thread 0 holds it; pk: the
// scalars above; pa: this thread's share of the r.r partials, loaded by the
// caller with its data when folded.)
__device__ bool cg_begin_iter(const RveDev& rv, int tile, int dn, const CgPeekB& pk, double pa, int mode,
                              double* red, double& beta) {
  CgState* cg = rv.cg;
  const bool timing = mode == PU_TIMING;
  // One barrier: every thread forms the same r.r total and takes the same
  // decision from it and from the CG scalars (none of which this launch
  // changes in a way the tests below can see), except the stop flag, which
  // is thread 0's copy.  The branches come after the loads have landed.
  int stopped;
  const double rr = block_total(rv.fold ? pa : 0.0, dn, red, stopped);
  beta = 0.0;
  if (stopped) return false;  // stopped before this launch: no state change
  if (timing || pk.iters == 0) return true;  // iteration 0: the residual pass has set p = r
  if (!rv.fold) {
    beta = pk.beta;  // k_finalize took the step
    return true;
  }
  const int it = pk.iters;
  int st = CG_RUNNING;
  if (pk.status == CG_BREAKDOWN) {
    st = CG_BREAKDOWN;
  } else if (pk.force >= 0) {
    if (it >= pk.force) st = CG_FORCED;
  } else if (rr <= pk.target2) {
    st = CG_CONVERGED;
  } else if (it >= pk.max_iter) {
    st = CG_MAXITER;
  }
  const double b = pk.rich ? 0.0 : rr / pk.rr_prev;   // Richardson: p = r
  if (tile == 0 && threadIdx.x == 0) {
    cg->rr = rr;
    cg->rr_new = rr;
    cg->status = st;
    if (st != CG_RUNNING) {
      __hip_atomic_store(&cg->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      cg->beta = b;
    }
  }
  if (st != CG_RUNNING) return false;
  beta = b;
  return true;
}

// Inputs of the forward pass at one voxel: the input (or r and the old p),
// the phase and the consistent tangent.  voxel_load only loads, so that a
// kernel can issue them before it waits on anything else.
template <class T>
struct VoxIn {
  double a[6], b[6];
  T g2, m[6];
  int ph;
};
template <class T>
__device__ __forceinline__ void voxel_load(long long v, long long nvox, int in_mode, const double* in, int update_p,
                                           const double* rres, const double* p_old, int tan_mode, const void* tang,
                                           const uint8_t* phase, VoxIn<T>& vi) {
  if (in_mode != IN_CONST_DE) {
    const FFTG_GLOBAL double* a = gmem(update_p ? rres : in);
#pragma unroll
    for (int c = 0; c < 6; ++c) vi.a[c] = a[c * nvox + v];
    if (update_p) {
      const FFTG_GLOBAL double* b = gmem(p_old);
#pragma unroll
      for (int c = 0; c < 6; ++c) vi.b[c] = b[c * nvox + v];
    }
  }
  if (tan_mode != TAN_IDENTITY) vi.ph = gmem(phase)[v];
  if (tan_mode == TAN_CURRENT) {
    const FFTG_GLOBAL T* tg = gmem((const T*)tang);
    vi.g2 = tg[v];
#pragma unroll
    for (int c = 0; c < 6; ++c) vi.m[c] = tg[(c + 1) * nvox + v];
  }
}

// tau = C(x):p(x) at voxel v from its loaded inputs.  With update_p,
// p = r + beta p_old is formed here, its components [own_lo, own_hi) are
// stored to p_new (p_new may equal p_old when the caller owns all six
// components of the voxel), and the return value is their share of p.tau
// (else 0).
template <class T>
__device__ __forceinline__ double voxel_compute(const VoxIn<T>& vi, long long v, long long nvox, int in_mode,
                                                const double* dE, int update_p, double beta, double* p_new,
                                                int own_lo, int own_hi, int tan_mode,
                                                const MatDev* __restrict__ mats, T tau[6]) {
  T p[6];
  double pd[6];
  if (in_mode == IN_CONST_DE) {
#pragma unroll
    for (int c = 0; c < 6; ++c) p[c] = T(dE[c]);
  } else if (update_p) {
    FFTG_GLOBAL double* pw = gmem(p_new);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double pn = vi.a[c] + beta * vi.b[c];
      if (c >= own_lo && c < own_hi) pw[c * nvox + v] = pn;
      pd[c] = pn;
      p[c] = T(pn);
    }
  } else {
#pragma unroll
    for (int c = 0; c < 6; ++c) p[c] = T(vi.a[c]);
  }
  if (tan_mode == TAN_IDENTITY) {
#pragma unroll
    for (int c = 0; c < 6; ++c) tau[c] = p[c];
  } else {
    const MatDev& mt = mats[vi.ph];
    T g2, m[6];
    if (tan_mode == TAN_ELASTIC) {
      g2 = T(2.0 * mt.G);
#pragma unroll
      for (int c = 0; c < 6; ++c) m[c] = T(0);
    } else {
      g2 = vi.g2;
#pragma unroll
      for (int c = 0; c < 6; ++c) m[c] = vi.m[c];
    }
    tangent_apply<T>(p, T(mt.K), g2, m, T(mt.csign), tau);
  }
  double d = 0.0;
  if (update_p) {
#pragma unroll
    for (int c = 0; c < 6; ++c)
      if (c >= own_lo && c < own_hi) d += pd[c] * double(tau[c]);
  }
  return d;
}

// Material table of a launch member into LDS, in two halves like the axis
// tables (threads past n fetch and store entry n - 1 again, so that no load
// sits behind a branch).
__device__ __forceinline__ MatDev mats_fetch(const MatDev* mats, int n) {
  const int i = min((int)threadIdx.x, n - 1);
  const FFTG_GLOBAL double* m = gmem(&mats[i].K);
  const FFTG_GLOBAL int* l = gmem(&mats[i].law);
  return MatDev{m[0], m[1], m[2], m[3], m[4], m[5], m[6], l[0], 0};
}
__device__ __forceinline__ void mats_store(const MatDev& m, int n, MatDev* s_mats) {
  s_mats[min((int)threadIdx.x, n - 1)] = m;
}

// ------------------------------------------------------------- z forward
// tau = C(x):p(x) (or p, or Ce:p, or C(x):dE) for a tile of rows, R2C along z.
template <class T, int BIG, int NF>
__global__ void __launch_bounds__(256) k_zfwd(const RveDev* __restrict__ rvs, int nrve, int rows_per_tile, int ldmax,
                                              int in_mode, int in_role, int tan_mode, int want_norm,
                                              int check_done, int update_p) {
  extern __shared__ __align__(16) char smem[];
  int tile;
  const int ri = find_rve(rvs, nrve, P_ZF, tile);
  if (ri < 0) return;
  const RveDev& rv = rvs[ri];
  // descriptor fields, all loaded in one batch (the empty asm keeps the
  // compiler from deferring any of them past the first use of another)
  int n0 = rv.n0, n1 = rv.n1, n2 = rv.n2, H = rv.H, nph = rv.n_phases, fold = rv.fold, nti = rv.tiles[P_ZI];
  long long nvox = rv.nvox;
  const long long nspec = rv.nspec;
  CgState* cg = rv.cg;
  const double* in = (const double*)rv.buf[in_role];
  const double* rres = (const double*)rv.buf[R_R];
  double* pw = (double*)rv.buf[R_P];
  const void* tang = rv.tang;
  const uint8_t* phase = rv.phase;
  const double* prr = rv.partial_rr;
  const MatDev* mats = rv.mats;
  TileLds<T> L(smem, 3 * rows_per_tile, n2, rv.ax[2], ldmax);
  __asm__ volatile(""
                   : "+s"(n0), "+s"(n1), "+s"(n2), "+s"(H), "+s"(nph), "+s"(fold), "+s"(nti), "+s"(nvox), "+s"(cg),
                     "+s"(in), "+s"(rres), "+s"(pw), "+s"(tang), "+s"(phase), "+s"(prr), "+s"(L.ax.M),
                     "+s"(L.ax.g_tw)
                   :
                   : "memory");
  // A launch over several RVEs tests the stop flag before any load, so that
  // members that stopped in an earlier launch move no data (a single RVE
  // loads it with its data).  Tile 0 may set the flag during this launch; a
  // tile that already sees it takes the decision every tile takes.
  if (check_done && !launch_single(nrve) && *gmem(&cg->done)) return;
  const int nrows_tot = n0 * n1;
  const int row0 = tile * rows_per_tile;
  const int nrows = min(rows_per_tile, nrows_tot - row0);
  const int ld = n2;
  const int nvt = nrows * n2;
  const int bd = blockDim.x;
  const FastDiv fn2(n2), fH(H), f3(3);
  __shared__ MatDev s_mats[kMaxPhases];  // per-voxel material lookups from LDS
  // Loads in program order before anything that waits: tables, this
  // thread's first voxel, the material table, the CG scalars, then the r.r
  // partials (a loop that waits as it sums); the LDS stores come after.
  // CG search direction update fused here: p <- r + beta p (in place: this
  // tile owns every component of its voxels).
  const AxisFetch<T> tf = axis_lds_fetch<T>(L.ax);
  auto vox_of = [&](int t) {
    const int r = fn2.div(t);
    return (long long)(row0 + r) * n2 + (t - r * n2);
  };
  VoxIn<T> vi0;
  voxel_load<T>(vox_of(min((int)threadIdx.x, nvt - 1)), nvox, in_mode, in, update_p, rres, pw, tan_mode, tang, phase,
                vi0);
  const MatDev mt = mats_fetch(mats, nph);
  const CgPeekB pk = cg_peek_b(cg);
  const double pa = (update_p && fold) ? thread_partials(prr, nti) : 0.0;
  axis_lds_store<T>(L.ax, tf);
  mats_store(mt, nph, s_mats);
  // Either branch ends in a barrier that also publishes the tables and
  // materials.  The stop flag is thread 0's copy, shared through LDS: in
  // the CG form tile 0 may set it while other tiles of the launch start.
  const int dn = check_done ? pk.done : 0;
  double beta = 0.0;
  if (update_p) {
    if (!cg_begin_iter(rv, tile, dn, pk, pa, update_p, L.red, beta)) return;
  } else if (done_publish(dn)) {
    return;
  }
  double nrm = 0.0;  // ||tau||^2 (want_norm) or p.tau (update_p)
  auto process = [&](const VoxIn<T>& vi, int t) {
    const int r = fn2.div(t);
    const int z = t - r * n2;
    const long long v = (long long)(row0 + r) * n2 + z;
    T tau[6];
    nrm += voxel_compute<T>(vi, v, nvox, in_mode, rv.dE, update_p, beta, pw, 0, 6, tan_mode, s_mats, tau);
    if (want_norm) {
#pragma unroll
      for (int c = 0; c < 6; ++c) nrm += double(tau[c]) * double(tau[c]);
    }
#pragma unroll
    for (int pr = 0; pr < 3; ++pr) L.line[(3 * r + pr) * ld + z] = cx<T>{tau[2 * pr], tau[2 * pr + 1]};
  };
  if ((int)threadIdx.x < nvt) process(vi0, threadIdx.x);
  for (int t = threadIdx.x + bd; t < nvt; t += bd) {
    VoxIn<T> vi;
    voxel_load<T>(vox_of(t), nvox, in_mode, in, update_p, rres, pw, tan_mode, tang, phase, vi);
    process(vi, t);
  }
  __syncthreads();
  cx<T>* res = line_fft<-1, T, BIG, NF>(L.line, L.scratch, ld, 3 * nrows, L.ax, L.dc);
  // untangle two real transforms: A_k = (Z_k + conj Z_-k)/2, B_k = (Z_k - conj Z_-k)/(2i)
  FFTG_GLOBAL cx<T>* spec = gmem((cx<T>*)rv.spec);
  for (int t = threadIdx.x; t < nrows * 3 * H; t += blockDim.x) {
    const int rp = fH.div(t);
    const int k = t - rp * H;
    const int r = f3.div(rp), pr = rp - 3 * r;
    const cx<T> zk = res[rp * ld + k];
    const cx<T> zm = res[rp * ld + (k == 0 ? 0 : n2 - k)];
    const cx<T> A = {T(0.5) * (zk.re + zm.re), T(0.5) * (zk.im - zm.im)};
    const cx<T> B = {T(0.5) * (zk.im + zm.im), T(-0.5) * (zk.re - zm.re)};
    const long long o = (long long)(row0 + r) * H + k;
    gstore(spec + (2 * pr) * nspec + o, A);
    gstore(spec + (2 * pr + 1) * nspec + o, B);
  }
  if (want_norm || update_p) {
    const double s = block_sum_last(nrm, L.red);
    put_partials(&s, 1, rv.partial, rv.tiles[P_ZF], tile);
  }
}

// --------------------------------------------------------------- y pass
template <class T, int DIR, int BIG, int NF>
__global__ void __launch_bounds__(256) k_ypass(const RveDev* __restrict__ rvs, int nrve, int lines_per_tile,
                                               int ldmax, int check_done) {
  extern __shared__ __align__(16) char smem[];
  int tile;
  const int ri = find_rve(rvs, nrve, P_Y, tile);
  if (ri < 0) return;
  const RveDev& rv = rvs[ri];
  // descriptor fields, all loaded in one batch (the empty asm keeps the
  // compiler from deferring any of them past the first use of another)
  int n0 = rv.n0, n1 = rv.n1, H = rv.H;
  const long long nspec = rv.nspec;
  cx<T>* const spec = (cx<T>*)rv.spec;
  CgState* const cg = rv.cg;
  TileLds<T> L(smem, lines_per_tile, n1, rv.ax[1], ldmax);
  __asm__ volatile("" : "+s"(n0), "+s"(n1), "+s"(H) : : "memory");
  const int ld = n1;
  const int nhb = (H + lines_per_tile - 1) / lines_per_tile;
  const int c = tile / (n0 * nhb);
  const int rem = tile - c * n0 * nhb;
  const int i0 = rem / nhb;
  const int h0 = (rem - i0 * nhb) * lines_per_tile;
  const int nh = min(lines_per_tile, H - h0);
  // Stop flag (no writer during the launch): a launch over several RVEs
  // tests it before the loads, so that members that have stopped move no
  // data.  A launch over one RVE loads it with the data (as a per-thread
  // value, so that nothing waits for it alone) and skips the transform and
  // the stores once the data have arrived.
  const bool single = launch_single(nrve);
  if (check_done && !single && *gmem(&cg->done)) return;
  const AxisFetch<T> tf = axis_lds_fetch<T>(L.ax);
  const int dn1 = cg_vaddr(cg)->done;  // unconditional: a guarded load would be waited for at its guard
  FFTG_GLOBAL cx<T>* base = gmem(spec) + c * nspec + (long long)i0 * n1 * H + h0;
  const FastDiv fnh(nh);
  lds_gather<4>(
      L.line, base, n1 * nh,
      [=](int t) {
        const int y = fnh.div(t);
        return (long long)y * H + (t - y * nh);
      },
      [=](int t) {
        const int y = fnh.div(t);
        return (t - y * nh) * ld + y;
      });
  axis_lds_store<T>(L.ax, tf);
  if (check_done && single && dn1) return;
  __syncthreads();
  cx<T>* res = line_fft<DIR, T, BIG, NF>(L.line, L.scratch, ld, nh, L.ax, L.dc);
  for (int t = threadIdx.x; t < n1 * nh; t += blockDim.x) {
    const int y = fnh.div(t);
    const int hh = t - y * nh;
    gstore(base + (long long)y * H + hh, res[hh * ld + y]);
  }
}

// --------------------------------------------------- x pass with G^(k)
// (GAMMA = 1: the collocation scheme's Gamma^ref(k) of the reference medium
// held in the CG state instead of G^(k).)
template <class T, int BIG, int NF, int GAMMA = 0>
__global__ void __launch_bounds__(256) k_xpass(const RveDev* __restrict__ rvs, int nrve, int lines_per_tile,
                                               int ldmax, double scale_in, int check_done) {
  extern __shared__ __align__(16) char smem[];
  int tile;
  const int ri = find_rve(rvs, nrve, P_X, tile);
  if (ri < 0) return;
  const RveDev& rv = rvs[ri];
  // descriptor fields, all loaded in one batch (the empty asm keeps the
  // compiler from deferring any of them past the first use of another)
  int n0 = rv.n0, n1 = rv.n1, n2 = rv.n2, H = rv.H;
  const long long nspec = rv.nspec, nvox = rv.nvox;
  FFTG_GLOBAL cx<T>* const spec = gmem((cx<T>*)rv.spec);
  CgState* const cg = rv.cg;
  TileLds<T> L(smem, 6 * lines_per_tile, xline_stride(rv.ax[0].rader, rv.ax[0].M, n0, kFp32<T>), rv.ax[0],
               ldmax);
  __asm__ volatile("" : "+s"(n0), "+s"(n1), "+s"(n2), "+s"(H) : : "memory");
  const int nhb = (H + lines_per_tile - 1) / lines_per_tile;
  const int i1 = tile / nhb;
  const int h0 = (tile - i1 * nhb) * lines_per_tile;
  const int nh = min(lines_per_tile, H - h0);
  const int ld = xline_stride(L.ax.rader, L.ax.M, n0, kFp32<T>);
  const int nl = 6 * nh;
  // stop flag: as in the y pass (tested first only over several RVEs)
  const bool single = launch_single(nrve);
  if (check_done && !single && *gmem(&cg->done)) return;
  const AxisFetch<T> tf = axis_lds_fetch<T>(L.ax);
  const int dn1 = cg_vaddr(cg)->done;  // unconditional: a guarded load would be waited for at its guard
  const long long rs = (long long)n1 * H;
  const long long off = (long long)i1 * H + h0;
  const FastDiv fnh(nh);
  // The tile's R = n0 nh pairs (x, hh), six components each.  For the
  // gather and the scatter the threads form G groups (G the largest divisor
  // of 6 with G R <= blockDim, else 1), group g owning components g, g + G,
  // ...: a thread splits its pair index once and its component addresses
  // differ by constants.  Line c nh + hh of LDS holds component c at kz
  // index hh: element (c, x, hh) sits at c lcs + hh ld + x.
  const int R = n0 * nh;
  const int bd = blockDim.x;
  const int G = (6 * R <= bd) ? 6 : (3 * R <= bd) ? 3 : (2 * R <= bd) ? 2 : 1;
  const FastDiv fR(R);
  const int grp = (G > 1) ? fR.div(threadIdx.x) : 0;
  const int r0 = (int)threadIdx.x - grp * R;
  const int rstep = (G > 1) ? R : bd;   // G > 1: one pair per thread
  const int lcs = nh * ld;
  const long long gstr = (long long)G * nspec;
  auto xmove = [&](auto nu_c, auto&& op) {
    constexpr int NU = decltype(nu_c)::value;
    if (grp >= G) return;
    for (int r = r0; r < R; r += rstep) {
      const int x = fnh.div(r);
      const int hh = r - x * nh;
      op(IntC<NU>{}, spec + (long long)x * rs + off + hh + grp * nspec, hh * ld + x + grp * lcs);
    }
  };
  auto xmove_any = [&](auto&& op) {
    switch (G) {
      case 6: xmove(IntC<1>{}, op); break;
      case 3: xmove(IntC<2>{}, op); break;
      case 2: xmove(IntC<3>{}, op); break;
      default: xmove(IntC<6>{}, op); break;
    }
  };
  xmove_any([&](auto nu_c, const FFTG_GLOBAL cx<T>* g, int l) {
    constexpr int NU = decltype(nu_c)::value;
    cx<T> v[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) v[u] = gload(g + u * gstr);
#pragma unroll
    for (int u = 0; u < NU; ++u) L.line[l + u * G * lcs] = v[u];
  });
  axis_lds_store<T>(L.ax, tf);
  if (check_done && single && dn1) return;
  __syncthreads();
  cx<T>* res = line_fft<-1, T, BIG, NF>(L.line, L.scratch, ld, nl, L.ax, L.dc);
  cx<T>* oth = (res == L.line) ? L.scratch : L.line;
  // projection on every frequency (k0, k1, k2) of the tile; xi_i = k_i / L_i, L_i = n_i
  const T scale = T(scale_in / double(nvox));   // inverse DFT normalisation 1/|N|
  const double inv_n0 = 1.0 / double(n0), inv_n2 = 1.0 / double(n2);
  const double k1 = double(sfreq(i1, n1)) / double(n1);
  T lam0 = T(0), mu0 = T(0);
  if constexpr (GAMMA) {
    const FFTG_GLOBAL CgState* g = cg_vaddr(cg);
    lam0 = T(g->lam0);
    mu0 = T(g->mu0);
  }
  for (int t = threadIdx.x; t < R; t += bd) {
    const int x = fnh.div(t);
    const int hh = t - x * nh;
    const double k0 = double(sfreq(x, n0)) * inv_n0;
    const double k2 = double(h0 + hh) * inv_n2;
    const double nn = k0 * k0 + k1 * k1 + k2 * k2;
    cx<T>* const e = res + hh * ld + x;
    cx<T> v[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = e[c * lcs];
    if (nn == 0.0) {
#pragma unroll
      for (int c = 0; c < 6; ++c) v[c] = cx<T>{T(0), T(0)};
    } else if constexpr (GAMMA) {
      const double inv = 1.0 / sqrt(nn);
      gamma_apply<T>(v, T(k0 * inv), T(k1 * inv), T(k2 * inv), lam0, mu0, scale);
    } else {
      const double i2 = 1.0 / nn;
      ghat_apply<T>(v, T(k0), T(k1), T(k2), T(double(scale) * i2), T(i2));
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) e[c * lcs] = v[c];
  }
  __syncthreads();
  if constexpr (NF > 0) {
    // inverse x transform of line c * nh + hh; the thread that forms outputs
    // x = k and n0 - k stores them to the spectrum at once (no pass of its
    // own; the runs are nh frequencies long, as in the general store)
    direct_dft_io<1, T, NF>(
        nl, L.ax, [&](int l) { return res[l * ld]; },
        [&](int l, int j, cx<T>& a, cx<T>& b) {
          a = res[l * ld + j];
          b = res[l * ld + NF - j];
        },
        [&](int l, int k, cx<T> xk, cx<T> xm) {
          const int c = fnh.div(l), hh = l - c * nh;
          FFTG_GLOBAL cx<T>* o = spec + c * nspec + off + hh;
          gstore(o + k * rs, xk);
          if (k > 0) gstore(o + (NF - k) * rs, xm);
        });
  } else {
    cx<T>* res2 = line_fft<1, T, BIG, NF>(res, oth, ld, nl, L.ax, L.dc);
    xmove_any([&](auto nu_c, FFTG_GLOBAL cx<T>* g, int l) {
      constexpr int NU = decltype(nu_c)::value;
#pragma unroll
      for (int u = 0; u < NU; ++u) gstore(g + u * gstr, res2[l + u * G * lcs]);
    });
  }
}

// CG scalars read by the vector update, loaded by every thread with the
// kernel's other loads (none is written during the launch but the stop
// flag, of which thread 0's copy counts) and used after the step's barrier,
// when the loads have landed.
struct CgPeek {
  int done, rich;
  double rr, alpha;
};
__device__ __forceinline__ CgPeek cg_peek(CgState* cg) {
  const FFTG_GLOBAL CgState* g = cg_vaddr(cg);
  return CgPeek{g->done, g->rich, g->rr, g->alpha};
}

// alpha = r.r / p.(C:p) for the CG vector update of the inverse z pass.  p is
// compatible (a combination of outputs of G) and G is an orthogonal
// projection, so p.(C:p) = (G p).(C:p) = p.G:(C:p) = p.Ap: the forward pass
// sums it while p and C:p are in registers, and alpha is known before the
// inverse transform ends.  Folded (rv.fold): every tile totals the forward
// pass's partials (pa: this thread's share, loaded early by the caller; same
// order in each tile, so the same value) and tile 0 publishes the state;
// the other tiles read only rr, which no tile of this launch writes.  A
// breakdown (p.(C:p) <= 0 or not finite) makes every tile exit unchanged and
// is recorded in status only, for the next forward pass to stop the solve:
// the stop flag is read by these tiles without a barrier between tiles.
// Not folded: k_finalize formed alpha (and the stop flag, before this
// launch).  With check_done the stop flag counts, as thread 0 loaded it.
// Returns false when the tile must exit (the same answer in every thread).
// Called by the whole workgroup (its barrier also publishes the caller's
// LDS writes).  With timing, the same loads and sums give alpha = 0 and
// touch no state.
__device__ bool cg_alpha(const RveDev& rv, int tile, const CgPeek& pk, bool check_done, double pa, bool timing,
                         double* red, double& alpha) {
  CgState* cg = rv.cg;
  // one barrier, every thread takes the same decision (as cg_begin_iter)
  int stopped;
  const double pap = block_total(rv.fold ? pa : 0.0, check_done ? pk.done : 0, red, stopped);
  alpha = 0.0;
  if (stopped) return false;  // stopped before this launch: no state change
  if (!rv.fold) {
    if (!timing) alpha = pk.alpha;
    return true;
  }
  if (timing) return true;
  const double rr = pk.rr;
  // Richardson: unit step, no curvature test (its operator need not be SPD)
  const bool brk = !pk.rich && (!(pap > 0.0) || !(pap < INFINITY));
  const double a = pk.rich ? 1.0 : rr / pap;
  if (tile == 0 && threadIdx.x == 0) {
    cg->pAp = pap;
    if (brk) {
      cg->status = CG_BREAKDOWN;
    } else {
      cg->alpha = a;
      cg->rr_prev = rr;
      cg->iters += 1;
    }
  }
  if (brk) return false;
  alpha = a;
  return true;
}

// ------------------------------------------------------------- z inverse
template <class T, int BIG, int NF>
__global__ void __launch_bounds__(256) k_zinv(const RveDev* __restrict__ rvs, int nrve, int rows_per_tile, int ldmax,
                                              int out_mode, int out_role, int check_done, int p_role) {
  extern __shared__ __align__(16) char smem[];
  int tile;
  const int ri = find_rve(rvs, nrve, P_ZI, tile);
  if (ri < 0) return;
  const RveDev& rv = rvs[ri];
  // descriptor fields, all loaded in one batch (the empty asm keeps the
  // compiler from deferring any of them past the first use of another)
  int n0 = rv.n0, n1 = rv.n1, n2 = rv.n2, H = rv.H;
  long long nspec = rv.nspec;
  const long long nvox = rv.nvox;
  const cx<T>* specp = (const cx<T>*)rv.spec;
  CgState* cg = rv.cg;
  int fold = rv.fold, ntz = rv.tiles[P_ZF];
  const double* part = rv.partial;
  TileLds<T> L(smem, 3 * rows_per_tile, n2, rv.ax[2], ldmax);
  __asm__ volatile(""
                   : "+s"(n0), "+s"(n1), "+s"(n2), "+s"(H), "+s"(nspec), "+s"(specp), "+s"(cg), "+s"(fold),
                     "+s"(ntz), "+s"(part), "+s"(L.ax.M), "+s"(L.ax.g_tw)
                   :
                   : "memory");
  const FFTG_GLOBAL cx<T>* const spec = gmem(specp);
  const int nrows_tot = n0 * n1;
  const int row0 = tile * rows_per_tile;
  const int nrows = min(rows_per_tile, nrows_tot - row0);
  const int ld = n2;
  const bool cg_out = out_mode == OUT_CG || out_mode == OUT_CG_TIMING;
  // Stop flag (no writer during the launch).  The CG form over one RVE
  // loads it in thread 0 with the data and decides at the alpha barrier;
  // otherwise it is tested before any load, so that members of a batch that
  // have stopped move no data.
  const bool late = cg_out && launch_single(nrve);
  if (check_done && !late && *gmem(&cg->done)) return;
  const AxisFetch<T> tf = axis_lds_fetch<T>(L.ax);
  // Z_k = A_k + i B_k, Z_{n-k} = conj(A_k) + i conj(B_k): each pair (A_k,
  // B_k) of the half spectrum is loaded once and fills both z = k and
  // z = n - k of its packed line.  Loads are issued in program order before
  // anything that waits: this thread's first two pairs, then the partials (a
  // loop that waits as it sums), then the stop flag; the LDS stores come
  // after.
  const FastDiv fn2(n2), fH(H), f3(3);
  const int ne = nrows * 3 * H;
  const int bd = blockDim.x;
  cx<T> A[2], B[2];
  int ti[2];
  auto load2 = [&](int t0) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      ti[u] = min(t0 + u * bd, ne - 1);  // past the end: the last pair again, same values to the same places
      const int rp = fH.div(ti[u]);
      const int k = ti[u] - rp * H;
      const int r = f3.div(rp), pr = rp - 3 * r;
      const long long o = (long long)(row0 + r) * H + k;
      A[u] = gload(spec + (2 * pr) * nspec + o);
      B[u] = gload(spec + (2 * pr + 1) * nspec + o);
    }
  };
  auto store2 = [&]() {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int rp = fH.div(ti[u]);
      const int k = ti[u] - rp * H;
      cx<T>* const ln = L.line + rp * ld;
      ln[k] = cx<T>{A[u].re - B[u].im, A[u].im + B[u].re};
      if (k > 0) ln[n2 - k] = cx<T>{A[u].re + B[u].im, -A[u].im + B[u].re};
    }
  };
  load2(threadIdx.x);
  const CgPeek pk = cg_peek(cg);
  // this thread's share of the p.(C:p) partials
  const double pa = (cg_out && fold) ? thread_partials(part, ntz) : 0.0;
  // the vector update's inputs at this thread's first voxel (v = row0 n2 + t)
  const int nvt = nrows * n2;
  double xv0[6], rv0[6], pv0[6];
  if (cg_out) {
    const long long v = (long long)row0 * n2 + min((int)threadIdx.x, nvt - 1);
    const FFTG_GLOBAL double* gx = gmem((const double*)rv.buf[R_X]);
    const FFTG_GLOBAL double* gr = gmem((const double*)rv.buf[R_R]);
    const FFTG_GLOBAL double* gp = gmem((const double*)rv.buf[p_role]);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      xv0[c] = gx[c * nvox + v];
      rv0[c] = gr[c * nvox + v];
      pv0[c] = gp[c * nvox + v];
    }
  }
  store2();
  for (int t0 = threadIdx.x + 2 * bd; t0 < ne; t0 += 2 * bd) {
    load2(t0);
    store2();
  }
  axis_lds_store<T>(L.ax, tf);
  double alpha = 0.0;
  if (cg_out) {
    if (!cg_alpha(rv, tile, pk, check_done && late, pa, out_mode == OUT_CG_TIMING, L.red, alpha)) return;
  } else {
    __syncthreads();
  }
  cx<T>* res = line_fft<1, T, BIG, NF>(L.line, L.scratch, ld, 3 * nrows, L.ax, L.dc);
  double dot = 0.0;
  if (cg_out) {
    // x += alpha p, r -= alpha G:(C:p), partials of the new r.r
    FFTG_GLOBAL double* __restrict__ xx = gmem((double*)rv.buf[R_X]);
    FFTG_GLOBAL double* __restrict__ rr = gmem((double*)rv.buf[R_R]);
    const FFTG_GLOBAL double* __restrict__ p = gmem((const double*)rv.buf[p_role]);
    auto update = [&](int t, const double* xv, const double* rv6, const double* pv) {
      const int r = fn2.div(t);
      const int z = t - r * n2;
      const long long v = (long long)(row0 + r) * n2 + z;
#pragma unroll
      for (int pr = 0; pr < 3; ++pr) {
        const cx<T> w = res[(3 * r + pr) * ld + z];
        const int c0 = 2 * pr, c1 = 2 * pr + 1;
        const double r0 = rv6[c0] - alpha * double(w.re), r1 = rv6[c1] - alpha * double(w.im);
        xx[c0 * nvox + v] = xv[c0] + alpha * pv[c0];
        xx[c1 * nvox + v] = xv[c1] + alpha * pv[c1];
        rr[c0 * nvox + v] = r0;
        rr[c1 * nvox + v] = r1;
        dot += r0 * r0 + r1 * r1;
      }
    };
    if ((int)threadIdx.x < nvt) update(threadIdx.x, xv0, rv0, pv0);
    for (int t = threadIdx.x + blockDim.x; t < nvt; t += blockDim.x) {
      const long long v = (long long)row0 * n2 + t;
      double xv[6], rv6[6], pv[6];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        xv[c] = xx[c * nvox + v];
        rv6[c] = rr[c * nvox + v];
        pv[c] = p[c * nvox + v];
      }
      update(t, xv, rv6, pv);
    }
    const double s = block_sum_last(dot, L.red);
    put_partials(&s, 1, rv.partial_rr, rv.tiles[P_ZI], tile);
    return;
  } else if (out_mode == OUT_RESIDUAL) {
    FFTG_GLOBAL double* rr = gmem((double*)rv.buf[R_R]);
    FFTG_GLOBAL double* pp = gmem((double*)rv.buf[R_P]);
    FFTG_GLOBAL double* xx = gmem((double*)rv.buf[R_X]);
    for (int t = threadIdx.x; t < nrows * n2; t += blockDim.x) {
      const int r = fn2.div(t);
      const int z = t - r * n2;
      const long long v = (long long)(row0 + r) * n2 + z;
#pragma unroll
      for (int pr = 0; pr < 3; ++pr) {
        const cx<T> w = res[(3 * r + pr) * ld + z];
        const double a0 = double(w.re), a1 = double(w.im);
        rr[(2 * pr) * nvox + v] = a0;
        rr[(2 * pr + 1) * nvox + v] = a1;
        pp[(2 * pr) * nvox + v] = a0;
        pp[(2 * pr + 1) * nvox + v] = a1;
        xx[(2 * pr) * nvox + v] = 0.0;
        xx[(2 * pr + 1) * nvox + v] = 0.0;
        dot += a0 * a0 + a1 * a1;
      }
    }
  } else {
    FFTG_GLOBAL T* out = gmem((T*)rv.buf[out_role]);
    for (int t = threadIdx.x; t < nrows * n2; t += blockDim.x) {
      const int r = fn2.div(t);
      const int z = t - r * n2;
      const long long v = (long long)(row0 + r) * n2 + z;
#pragma unroll
      for (int pr = 0; pr < 3; ++pr) {
        const cx<T> w = res[(3 * r + pr) * ld + z];
        out[(2 * pr) * nvox + v] = w.re;
        out[(2 * pr + 1) * nvox + v] = w.im;
      }
    }
    return;
  }
  const double s = block_sum_last(dot, L.red);
  put_partials(&s, 1, rv.partial, rv.tiles[P_ZI], tile);
}

// ------------------------------------------------------- slab passes
// For grids whose y-z plane fits in LDS the z and y transforms of a plane
// run in one kernel: tile (x, pr) owns Mandel components 2pr and 2pr+1 of
// plane x, packed as the real and imaginary parts of one complex z-line per
// y (two real transforms in one complex transform, as in the z passes).
// LDS: tables of the z and y axes, two buffers of n1 (n2 + 1) points, Rader
// slots and the reduction scratch.
template <class T>
struct SlabLds {
  AxisLds<T> az, ay;
  cx<T>* b0;
  cx<T>* b1;
  cx<T>* dc;
  double* red;
  // The tables are only carved out: the kernels copy them with
  // axis_lds_fetch / axis_lds_store around their own loads.
  __device__ SlabLds(char* base, int n1max, int n2max, const AxisDev& Pz, const AxisDev& Py) {
    axis_lds_setup<T>(Pz, base, az);
    char* q = base + axis_lds_bytes<T>(n2max);
    axis_lds_setup<T>(Py, q, ay);
    q += axis_lds_bytes<T>(n1max);
    const size_t S = (size_t)n1max * (n2max + 1);
    b0 = reinterpret_cast<cx<T>*>(q);
    b1 = b0 + S;
    dc = b1 + S;
    const int nd = max(n1max, n2max + 1);
    red = reinterpret_cast<double*>(dc + nd + (nd & 1));
  }
};

template <class T, int BIG, int NF>
__global__ void __launch_bounds__(512) k_slab_fwd(const RveDev* __restrict__ rvs, int nrve, int n1max, int n2max,
                                                  int in_mode, int in_role, int tan_mode, int want_norm,
                                                  int check_done, int update_p, int p_in, int p_out) {
  extern __shared__ __align__(16) char smem[];
  int tile;
  const int ri = find_rve(rvs, nrve, P_ZF, tile);
  if (ri < 0) return;
  const RveDev& rv = rvs[ri];
  // descriptor fields, all loaded in one batch (the empty asm keeps the
  // compiler from deferring any of them past the first use of another)
  int n1 = rv.n1, n2 = rv.n2, H = rv.H, nph = rv.n_phases, fold = rv.fold, nti = rv.tiles[P_ZI];
  long long nvox = rv.nvox;
  const long long nspec = rv.nspec;
  CgState* cg = rv.cg;
  const double* in = (const double*)rv.buf[in_role];
  const double* rres = (const double*)rv.buf[R_R];
  const double* pin = (const double*)rv.buf[p_in];
  double* pout = (double*)rv.buf[p_out];
  const void* tang = rv.tang;
  const uint8_t* phase = rv.phase;
  const double* prr = rv.partial_rr;
  const MatDev* mats = rv.mats;
  SlabLds<T> L(smem, n1max, n2max, rv.ax[2], rv.ax[1]);
  __asm__ volatile(""
                   : "+s"(n1), "+s"(n2), "+s"(H), "+s"(nph), "+s"(nvox), "+s"(cg), "+s"(in), "+s"(rres), "+s"(pin),
                     "+s"(tang), "+s"(phase), "+s"(prr), "+s"(L.az.g_tw), "+s"(L.ay.g_tw)
                   :
                   : "memory");
  // stop flag of a batched launch before any load (as in the z pass)
  if (check_done && !launch_single(nrve) && *gmem(&cg->done)) return;
  const int x = tile / 3, pr = tile - 3 * (tile / 3);
  const long long v0 = (long long)x * n1 * n2;
  const int npl = n1 * n2;
  __shared__ MatDev s_mats[kMaxPhases];  // per-voxel material lookups from LDS
  // Loads in program order before anything that waits (as in the z pass):
  // tables, this thread's first two voxels (a plane has up to twice as many
  // voxels as a tile has threads at 31^2), materials, CG scalars, partials.
  const AxisFetch<T> tfz = axis_lds_fetch<T>(L.az);
  const AxisFetch<T> tfy = axis_lds_fetch<T>(L.ay);
  const int t1 = (int)threadIdx.x + (int)blockDim.x;
  VoxIn<T> vi0, vi1;
  voxel_load<T>(v0 + min((int)threadIdx.x, npl - 1), nvox, in_mode, in, update_p, rres, pin, tan_mode, tang, phase,
                vi0);
  voxel_load<T>(v0 + min(t1, npl - 1), nvox, in_mode, in, update_p, rres, pin, tan_mode, tang, phase, vi1);
  const MatDev mt = mats_fetch(mats, nph);
  const CgPeekB pk = cg_peek_b(cg);
  const double pa = (update_p && fold) ? thread_partials(prr, nti) : 0.0;
  axis_lds_store<T>(L.az, tfz);
  axis_lds_store<T>(L.ay, tfy);
  mats_store(mt, nph, s_mats);
  // either branch ends in a barrier that also publishes tables and materials
  const int dn = check_done ? pk.done : 0;
  double beta = 0.0;
  if (update_p) {
    if (!cg_begin_iter(rv, tile, dn, pk, pa, update_p, L.red, beta)) return;
  } else if (done_publish(dn)) {
    return;
  }
  double nrm = 0.0;  // ||tau||^2 (want_norm) or p.tau over the tile's components (update_p)
  auto process = [&](const VoxIn<T>& vi, int t) {
    T tau[6];
    nrm += voxel_compute<T>(vi, v0 + t, nvox, in_mode, rv.dE, update_p, beta, pout, 2 * pr, 2 * pr + 2, tan_mode,
                            s_mats, tau);
    // selects, not an indexed read: a runtime index into tau would put it in scratch
    const T a = pr == 0 ? tau[0] : (pr == 1 ? tau[2] : tau[4]);
    const T b = pr == 0 ? tau[1] : (pr == 1 ? tau[3] : tau[5]);
    if (want_norm) nrm += double(a) * double(a) + double(b) * double(b);
    L.b0[t] = cx<T>{a, b};  // z-line y at y * n2
  };
  if ((int)threadIdx.x < npl) process(vi0, threadIdx.x);
  if (t1 < npl) process(vi1, t1);
  for (int t = t1 + blockDim.x; t < npl; t += blockDim.x) {
    VoxIn<T> vi;
    voxel_load<T>(v0 + t, nvox, in_mode, in, update_p, rres, pin, tan_mode, tang, phase, vi);
    process(vi, t);
  }
  // the tile's partial (p.tau or ||tau||^2) is complete here: its per-wave
  // sums go to LDS ahead of the barrier the transforms need anyway (slots 16
  // on, clear of the CG step's, which other waves may still be reading), and
  // thread 0 adds them at the end
  const bool part_out = want_norm || update_p;
  if (part_out) {
    nrm = wave_sum(nrm);
    if ((threadIdx.x & 63) == 0) L.red[16 + (threadIdx.x >> 6)] = nrm;
  }
  __syncthreads();
  // z transform of the packed lines, untangled into y-lines: component
  // 2pr + c2, frequency k -> line c2 * H + k
  const FastDiv fH(H), fn1(n1);
  cx<T>* yl;
  if constexpr (NF > 0) {
    // the thread that forms X_k and X_(n2-k) of packed line y holds both
    // components' frequency k: untangled as they are stored (no pass of
    // its own)
    direct_dft_io<-1, T, NF>(
        n1, L.az, [&](int y) { return L.b0[y * n2]; },
        [&](int y, int j, cx<T>& a, cx<T>& b) {
          a = L.b0[y * n2 + j];
          b = L.b0[y * n2 + NF - j];
        },
        [&](int y, int k, cx<T> zk, cx<T> zm) {
          L.b1[k * n1 + y] = cx<T>{T(0.5) * (zk.re + zm.re), T(0.5) * (zk.im - zm.im)};
          L.b1[(H + k) * n1 + y] = cx<T>{T(0.5) * (zk.im + zm.im), T(-0.5) * (zk.re - zm.re)};
        });
    yl = L.b1;
  } else {
    cx<T>* res = line_fft<-1, T, BIG, NF>(L.b0, L.b1, n2, n1, L.az, L.dc);
    yl = (res == L.b0) ? L.b1 : L.b0;
    for (int t = threadIdx.x; t < n1 * H; t += blockDim.x) {
      const int y = fH.div(t);
      const int k = t - y * H;
      const cx<T> zk = res[y * n2 + k];
      const cx<T> zm = res[y * n2 + (k == 0 ? 0 : n2 - k)];
      yl[k * n1 + y] = cx<T>{T(0.5) * (zk.re + zm.re), T(0.5) * (zk.im - zm.im)};
      yl[(H + k) * n1 + y] = cx<T>{T(0.5) * (zk.im + zm.im), T(-0.5) * (zk.re - zm.re)};
    }
  }
  __syncthreads();
  FFTG_GLOBAL cx<T>* spec = gmem((cx<T>*)rv.spec);
  if constexpr (NF > 0) {
    // y transform of y-line c2 * H + kz; the thread that forms outputs
    // ky = k and n1 - k stores them to the spectrum at once (no pass of its
    // own: lanes of a wave cover four kz at sixteen ky, runs of 64 bytes)
    direct_dft_io<-1, T, NF>(
        2 * H, L.ay, [&](int l) { return yl[l * n1]; },
        [&](int l, int j, cx<T>& a, cx<T>& b) {
          a = yl[l * n1 + j];
          b = yl[l * n1 + NF - j];
        },
        [&](int l, int k, cx<T> xk, cx<T> xm) {
          const int c2 = l >= H ? 1 : 0, kz = l - c2 * H;
          FFTG_GLOBAL cx<T>* o = spec + (2 * pr + c2) * nspec + (long long)x * n1 * H + kz;
          gstore(o + (long long)k * H, xk);
          if (k > 0) gstore(o + (long long)(NF - k) * H, xm);
        });
  } else {
    cx<T>* res2 = line_fft<-1, T, BIG, NF>(yl, yl == L.b0 ? L.b1 : L.b0, n1, 2 * H, L.ay, L.dc);
    for (int t = threadIdx.x; t < 2 * n1 * H; t += blockDim.x) {
      const int cy = fH.div(t);
      const int k = t - cy * H;
      const int c2 = fn1.div(cy), y = cy - c2 * n1;
      gstore(spec + (2 * pr + c2) * nspec + ((long long)x * n1 + y) * H + k, res2[(c2 * H + k) * n1 + y]);
    }
  }
  if (part_out && threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    double sp = 0.0;
    for (int i = 0; i < nw; ++i) sp += L.red[16 + i];
    put_partials(&sp, 1, rv.partial, rv.tiles[P_ZF], tile);
  }
}

template <class T, int BIG, int NF>
__global__ void __launch_bounds__(512) k_slab_inv(const RveDev* __restrict__ rvs, int nrve, int n1max, int n2max,
                                                  int out_mode, int out_role, int check_done, int p_role) {
  extern __shared__ __align__(16) char smem[];
  int tile;
  const int ri = find_rve(rvs, nrve, P_ZI, tile);
  if (ri < 0) return;
  const RveDev& rv = rvs[ri];
  // descriptor fields, all loaded in one batch (the empty asm keeps the
  // compiler from deferring any of them past the first use of another)
  int n1 = rv.n1, n2 = rv.n2, H = rv.H, fold = rv.fold, ntz = rv.tiles[P_ZF];
  long long nspec = rv.nspec;
  const long long nvox = rv.nvox;
  const cx<T>* specp = (const cx<T>*)rv.spec;
  CgState* cg = rv.cg;
  const double* part = rv.partial;
  SlabLds<T> L(smem, n1max, n2max, rv.ax[2], rv.ax[1]);
  __asm__ volatile(""
                   : "+s"(n1), "+s"(n2), "+s"(H), "+s"(fold), "+s"(ntz), "+s"(nspec), "+s"(specp), "+s"(cg),
                     "+s"(part), "+s"(L.az.M), "+s"(L.az.g_tw), "+s"(L.ay.M), "+s"(L.ay.g_tw)
                   :
                   : "memory");
  const FFTG_GLOBAL cx<T>* const spec = gmem(specp);
  const int x = tile / 3, pr = tile - 3 * (tile / 3);
  const long long v0 = (long long)x * n1 * n2;
  const int npl = n1 * n2;
  const int c0 = 2 * pr, c1 = 2 * pr + 1;
  const bool cg_out = out_mode == OUT_CG || out_mode == OUT_CG_TIMING;
  // Stop flag as in the z pass: the CG form over one RVE decides at the
  // alpha barrier, otherwise it is tested before any load.
  const bool late = cg_out && launch_single(nrve);
  if (check_done && !late && *gmem(&cg->done)) return;
  // Loads in program order before anything that waits: tables, the
  // spectrum, the CG scalars, the partials, this thread's first two voxels.
  const AxisFetch<T> tfz = axis_lds_fetch<T>(L.az);
  const AxisFetch<T> tfy = axis_lds_fetch<T>(L.ay);
  const FastDiv fH(H), fn1(n1), fn2(n2);
  lds_gather<4>(
      L.b0, spec, 2 * n1 * H,
      [=](int t) {
        const int cy = fH.div(t);
        const int k = t - cy * H;
        const int c2 = fn1.div(cy), y = cy - c2 * n1;
        return (2 * pr + c2) * nspec + ((long long)x * n1 + y) * H + k;
      },
      [=](int t) {
        const int cy = fH.div(t);
        const int k = t - cy * H;
        const int c2 = fn1.div(cy), y = cy - c2 * n1;
        return (c2 * H + k) * n1 + y;
      });
  const CgPeek pk = cg_peek(cg);
  const double pa = (cg_out && fold) ? thread_partials(part, ntz) : 0.0;
  // the two voxels whose CG update this thread takes first: in the 31-point
  // builds those of its first z-transform task (z-line y, pair k and n2 - k),
  // else voxels t and t + blockDim of the plane
  const int t1 = (int)threadIdx.x + (int)blockDim.x;
  constexpr int Hq = (NF + 1) / 2;  // z-transform tasks per line (31-point builds)
  long long va, vb;
  if constexpr (NF > 0) {
    const int tq = min((int)threadIdx.x, n1 * Hq - 1);
    const int yq = tq / Hq, kq = tq - yq * Hq;
    va = v0 + (long long)yq * n2 + kq;
    vb = v0 + (long long)yq * n2 + (kq == 0 ? 0 : n2 - kq);
  } else {
    va = v0 + min((int)threadIdx.x, npl - 1);
    vb = v0 + min(t1, npl - 1);
  }
  double xv0[2], rv0[2], pv0[2], xv1[2], rv1[2], pv1[2];
  if (cg_out) {
    const long long v = va;
    const long long w = vb;
    const FFTG_GLOBAL double* gx = gmem((const double*)rv.buf[R_X]);
    const FFTG_GLOBAL double* gr = gmem((const double*)rv.buf[R_R]);
    const FFTG_GLOBAL double* gp = gmem((const double*)rv.buf[p_role]);
    xv0[0] = gx[c0 * nvox + v];
    xv0[1] = gx[c1 * nvox + v];
    rv0[0] = gr[c0 * nvox + v];
    rv0[1] = gr[c1 * nvox + v];
    pv0[0] = gp[c0 * nvox + v];
    pv0[1] = gp[c1 * nvox + v];
    xv1[0] = gx[c0 * nvox + w];
    xv1[1] = gx[c1 * nvox + w];
    rv1[0] = gr[c0 * nvox + w];
    rv1[1] = gr[c1 * nvox + w];
    pv1[0] = gp[c0 * nvox + w];
    pv1[1] = gp[c1 * nvox + w];
  }
  axis_lds_store<T>(L.az, tfz);
  axis_lds_store<T>(L.ay, tfy);
  double alpha = 0.0;
  if (cg_out) {
    if (!cg_alpha(rv, tile, pk, check_done && late, pa, out_mode == OUT_CG_TIMING, L.red, alpha)) return;
  } else {
    __syncthreads();
  }
  cx<T>* res = line_fft<1, T, BIG, NF>(L.b0, L.b1, n1, 2 * H, L.ay, L.dc);
  cx<T>* oth = (res == L.b0) ? L.b1 : L.b0;
  // x += alpha p, r -= alpha G:(C:p) at voxel v on the tile's two
  // components, and the r.r partial (CG form)
  double dot = 0.0;
  FFTG_GLOBAL double* __restrict__ xx = gmem((double*)rv.buf[R_X]);
  FFTG_GLOBAL double* __restrict__ rr = gmem((double*)rv.buf[R_R]);
  const FFTG_GLOBAL double* __restrict__ pg = gmem((const double*)rv.buf[p_role]);
  auto update = [&](long long v, cx<T> w, const double* xv, const double* rv2, const double* pv) {
    const double r0 = rv2[0] - alpha * double(w.re), r1 = rv2[1] - alpha * double(w.im);
    xx[c0 * nvox + v] = xv[0] + alpha * pv[0];
    xx[c1 * nvox + v] = xv[1] + alpha * pv[1];
    rr[c0 * nvox + v] = r0;
    rr[c1 * nvox + v] = r1;
    dot += r0 * r0 + r1 * r1;
  };
  auto update_load = [&](long long v, cx<T> w) {
    const double xv[2] = {xx[c0 * nvox + v], xx[c1 * nvox + v]};
    const double rv2[2] = {rr[c0 * nvox + v], rr[c1 * nvox + v]};
    const double pv[2] = {pg[c0 * nvox + v], pg[c1 * nvox + v]};
    update(v, w, xv, rv2, pv);
  };
  // z-line y (at y * n2): Z_z = A_z + i B_z, Z_{n2-k} = conj(A_k) + i conj(B_k)
  cx<T>* res2 = oth;
  bool updated = false;  // the CG update already done inside the z transform
  if constexpr (NF > 0) {
    // the pair Z_j, Z_(n2-j) that the z transform takes together needs only
    // A_j and B_j: the packing is folded into the transform's loads; and the
    // thread that forms the outputs z = k and n2 - k of line y applies the
    // CG update to those two voxels at once (no pass of its own for either)
    direct_dft_io<1, T, NF>(
        n1, L.az,
        [&](int y) {
          const cx<T> A = res[y], B = res[H * n1 + y];
          return cx<T>{A.re - B.im, A.im + B.re};
        },
        [&](int y, int j, cx<T>& a, cx<T>& b) {
          const cx<T> A = res[j * n1 + y], B = res[(H + j) * n1 + y];
          a = cx<T>{A.re - B.im, A.im + B.re};
          b = cx<T>{A.re + B.im, -A.im + B.re};
        },
        [&](int y, int k, cx<T> xk, cx<T> xm) {
          if (cg_out) {
            const long long v_a = v0 + (long long)y * n2 + k, v_b = v0 + (long long)y * n2 + (NF - k);
            if (y * Hq + k == (int)threadIdx.x) {  // this thread's first task: inputs prefetched
              update(v_a, xk, xv0, rv0, pv0);
              if (k > 0) update(v_b, xm, xv1, rv1, pv1);
            } else {
              update_load(v_a, xk);
              if (k > 0) update_load(v_b, xm);
            }
          } else {
            oth[y * n2 + k] = xk;
            if (k > 0) oth[y * n2 + NF - k] = xm;
          }
        });
    updated = cg_out;
    if (!cg_out) __syncthreads();
  } else {
    for (int t = threadIdx.x; t < n1 * n2; t += blockDim.x) {
      const int y = fn2.div(t);
      const int z = t - y * n2;
      cx<T> Zv;
      if (z < H) {
        const cx<T> A = res[z * n1 + y], B = res[(H + z) * n1 + y];
        Zv = cx<T>{A.re - B.im, A.im + B.re};
      } else {
        const int k = n2 - z;
        const cx<T> A = res[k * n1 + y], B = res[(H + k) * n1 + y];
        Zv = cx<T>{A.re + B.im, -A.im + B.re};
      }
      oth[t] = Zv;
    }
    __syncthreads();
    res2 = line_fft<1, T, BIG, NF>(oth, res, n2, n1, L.az, L.dc);
  }
  if (cg_out) {
    if (!updated) {
      if ((int)threadIdx.x < npl) update(va, res2[threadIdx.x], xv0, rv0, pv0);
      if (t1 < npl) update(vb, res2[t1], xv1, rv1, pv1);
      for (int t = t1 + blockDim.x; t < npl; t += blockDim.x) update_load(v0 + t, res2[t]);
    }
    const double s = block_sum_last(dot, L.red);
    put_partials(&s, 1, rv.partial_rr, rv.tiles[P_ZI], tile);
    return;
  } else if (out_mode == OUT_RESIDUAL) {
    FFTG_GLOBAL double* rr = gmem((double*)rv.buf[R_R]);
    FFTG_GLOBAL double* pp = gmem((double*)rv.buf[R_P]);
    FFTG_GLOBAL double* xx = gmem((double*)rv.buf[R_X]);
    for (int t = threadIdx.x; t < n1 * n2; t += blockDim.x) {
      const long long v = v0 + t;
      const cx<T> w = res2[t];
      const double a0 = double(w.re), a1 = double(w.im);
      rr[c0 * nvox + v] = a0;
      rr[c1 * nvox + v] = a1;
      pp[c0 * nvox + v] = a0;
      pp[c1 * nvox + v] = a1;
      xx[c0 * nvox + v] = 0.0;
      xx[c1 * nvox + v] = 0.0;
      dot += a0 * a0 + a1 * a1;
    }
  } else {
    FFTG_GLOBAL T* out = gmem((T*)rv.buf[out_role]);
    for (int t = threadIdx.x; t < n1 * n2; t += blockDim.x) {
      const long long v = v0 + t;
      const cx<T> w = res2[t];
      out[c0 * nvox + v] = w.re;
      out[c1 * nvox + v] = w.im;
    }
    return;
  }
  const double s = block_sum_last(dot, L.red);
  put_partials(&s, 1, rv.partial, rv.tiles[P_ZI], tile);
}

// ------------------------------------------------------- Newton update
// eps* += x (Algorithm 1, iterative update) and ||x||^2.
__global__ void __launch_bounds__(256) k_newton_update(const RveDev* __restrict__ rvs, int nrve, int vox_per_tile) {
  __shared__ double red[16];
  int tile;
  const int ri = find_rve(rvs, nrve, P_VEC, tile);
  if (ri < 0) return;
  const RveDev& rv = rvs[ri];
  const long long nvox = rv.nvox;
  double* __restrict__ e = (double*)rv.buf[R_EPS_FL];
  const double* __restrict__ x = (const double*)rv.buf[R_X];
  const long long v0 = (long long)tile * vox_per_tile;
  const int nv = (int)min((long long)vox_per_tile, nvox - v0);
  double acc = 0.0;
  for (int t = threadIdx.x; t < nv; t += blockDim.x) {
    const long long v = v0 + t;
    double dv[6], ev[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      dv[c] = x[c * nvox + v];
      ev[c] = e[c * nvox + v];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      e[c * nvox + v] = ev[c] + dv[c];
      acc += dv[c] * dv[c];
    }
  }
  const double s = block_sum(acc, red);
  put_partials(&s, 1, rv.partial, rv.tiles[P_VEC], tile);
}

// ------------------------------------------------ return maps (Sec. 4)
// Root of f(dg) = seq - 3G dg - sy - Hh (a0 + dg)^n, n != 1, given
// f(0) = phi > 0: f falls monotonically and f(phi / 3G) <= 0, so Newton's
// method is kept inside the bracket [lo, hi] that every evaluation narrows
// (a step that would leave it bisects instead), started from the right end
// (where the derivative is finite even at a0 = 0).  Stops when the step is
// below a few ulps of dg; slope returns 3G + n Hh (a0 + dg)^(n-1).
__device__ double return_root(double seq, double a0, double G, double sy, double Hh, double n, double phi,
                              double& slope) {
  double lo = 0.0, hi = phi / (3.0 * G), x = hi;
  for (int it = 0; it < 200; ++it) {
    const double ax = a0 + x;
    const double pw = pow(ax, n);
    const double f = seq - 3.0 * G * x - sy - Hh * pw;
    if (f > 0.0) lo = x;
    else hi = x;
    const double df = -3.0 * G - n * Hh * pw / ax;
    double xn = x - f / df;
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    const bool done = fabs(xn - x) <= 4e-16 * x || !(hi - lo > 4e-16 * hi);
    x = xn;
    if (done) break;
  }
  slope = 3.0 * G + n * Hh * pow(a0 + x, n - 1.0);
  return x;
}

// Per voxel, by the phase's law: trial state from the committed history;
// elasto-plastic (Sec. 4.2): elastic when Phi_tr <= 0, else the return
// equation (closed form dg = Phi_tr / (3G + H) for n = 1) along
// N = 3/2 s_tr / seq_tr; visco-plastic (Sec. 4.3): the same equation with
// sy = 0, Hh = sigma_0 / (gamma_0 dt)^n, a0 = 0, flowing whenever seq_tr > 0;
// non-linear elastic (Sec. 4.1): sigma = K tr(eps) I + sigma_0 (eps_eq /
// eps_0)^n N, N = 2/3 eps_d / eps_eq, no history.  Writes sigma (Mandel),
// the compact tangent {2G', m} with C = K I(x)I + 2G' I_d + csign m (x) m:
// inelastic 2G' = 2G (1 - 3G dg/seq_tr), m = sqrt(-c) N,
// c = 4G^2 (dg/seq_tr - 1/slope); non-linear elastic 2G' = 2/3 s/eps_eq,
// m = sqrt(|c|) N, c = (n - 1) s/eps_eq with s = sigma_0 (eps_eq/eps_0)^n.
// commit: 0 evaluates only (Newton iterations); 1 also writes the new
// history and per-tile sums of sigma (the end of an increment); 2 writes
// the sums of sigma but leaves the history (an increment that failed).
template <class TT>
__global__ void __launch_bounds__(256) k_constitutive(const RveDev* __restrict__ rvs, int nrve, int vox_per_tile,
                                                      int eps_role, int commit) {
  __shared__ double red[16];
  int tile;
  const int ri = find_rve(rvs, nrve, P_VEC, tile);
  if (ri < 0) return;
  const RveDev& rv = rvs[ri];
  const long long nvox = rv.nvox;
  const double* ein = (const double*)rv.buf[eps_role];
  const bool add_E = (eps_role == R_EPS_FL);
  double* ep = (double*)rv.buf[R_EPS_P];
  double* eb = (double*)rv.buf[R_EPBAR];
  double* sg = (double*)rv.buf[R_SIG];
  TT* tg = (TT*)rv.tang;
  const long long v0 = (long long)tile * vox_per_tile;
  const int nv = (int)min((long long)vox_per_tile, nvox - v0);
  double ssum[6] = {0, 0, 0, 0, 0, 0};
  for (int t = threadIdx.x; t < nv; t += blockDim.x) {
    const long long v = v0 + t;
    const MatDev mt = rv.mats[rv.phase[v]];
    double e[6], epv[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      e[c] = ein[c * nvox + v] + (add_E ? rv.E[c] : 0.0);
      epv[c] = ep[c * nvox + v];
    }
    const double ebv = eb[v];
    double d[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) d[c] = e[c] - epv[c];
    const double tr = d[0] + d[1] + d[2];
#pragma unroll
    for (int c = 0; c < 3; ++c) d[c] -= tr * (1.0 / 3.0);
    double dd = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) dd += d[c] * d[c];
    const double G = mt.G, K = mt.K, n = mt.n;
    double sig[6], g2, m[6];
    if (mt.law == LAW_NLE) {
      // no plastic strain: d is the strain deviator, tr its trace
      const double eeq = sqrt((2.0 / 3.0) * dd);
      if (eeq > 0.0) {
        const double s = mt.sy * pow(eeq / mt.e0, n);
        const double f = s / eeq;
        const double sm = sqrt(fabs((n - 1.0) * f));
        g2 = (2.0 / 3.0) * f;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const double Nc = (2.0 / 3.0) * d[c] / eeq;
          sig[c] = s * Nc + (c < 3 ? K * tr : 0.0);
          m[c] = sm * Nc;
        }
      } else {
        g2 = n == 1.0 ? (2.0 / 3.0) * mt.sy / mt.e0 : 0.0;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          sig[c] = c < 3 ? K * tr : 0.0;
          m[c] = 0.0;
        }
      }
    } else {
      const double seq = 2.0 * G * sqrt(1.5 * dd);
      const double a0 = mt.law == LAW_VISCO ? 0.0 : ebv;
      const double hard = n == 1.0 ? mt.Hh * a0 : (a0 > 0.0 ? mt.Hh * pow(a0, n) : 0.0);
      const double phi = seq - (mt.sy + hard);
      if (phi > 0.0) {
        double dg, slope;
        if (n == 1.0) {
          dg = phi / (3.0 * G + mt.Hh);
          slope = 3.0 * G + mt.Hh;
        } else {
          dg = return_root(seq, a0, G, mt.sy, mt.Hh, n, phi, slope);
        }
        const double ns = 1.5 * 2.0 * G / seq;   // N = ns * d
        double Nv[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) Nv[c] = ns * d[c];
        const double cc = 4.0 * G * G * (dg / seq - 1.0 / slope);
        const double sm = sqrt(-cc);
        g2 = 2.0 * G * (1.0 - 3.0 * G * dg / seq);
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          sig[c] = 2.0 * G * (d[c] - dg * Nv[c]) + (c < 3 ? K * tr : 0.0);
          m[c] = sm * Nv[c];
        }
        if (commit == 1) {
#pragma unroll
          for (int c = 0; c < 6; ++c) ep[c * nvox + v] = epv[c] + dg * Nv[c];
          eb[v] = ebv + dg;
        }
      } else {
        g2 = 2.0 * G;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          sig[c] = 2.0 * G * d[c] + (c < 3 ? K * tr : 0.0);
          m[c] = 0.0;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      sg[c * nvox + v] = sig[c];
      ssum[c] += sig[c];
    }
    tg[v] = TT(g2);
#pragma unroll
    for (int c = 0; c < 6; ++c) tg[(c + 1) * nvox + v] = TT(m[c]);
  }
  if (commit) {
    double s[6];
    for (int c = 0; c < 6; ++c) s[c] = block_sum(ssum[c], red);
    put_partials(s, 6, rv.partial, rv.tiles[P_VEC], tile);
  }
}

// ------------------------------------------------------------- finalize
// One workgroup per RVE: sums the tile partials of the preceding producer
// kernel in a fixed order and applies the scalar step that uses the total.
//   FIN_SNORM  ||C:dE||^2 of the right-hand side floor
//   FIN_RESID  b.b of the CG right-hand side: target, start or skip of CG
//   FIN_PAP    p.(C:p) = p.Ap of the forward pass: alpha = r.r / p.Ap
//              (breakdown when p.Ap <= 0 or not finite)
//   FIN_RR     r.r after the vector update: iteration count, stopping test, beta
//   FIN_DNORM  ||d eps||^2 of the Newton update
//   FIN_SIGMA  volume average of sigma (six sums)
__global__ void __launch_bounds__(256) k_finalize(const RveDev* __restrict__ rvs, int nrve, int step) {
  __shared__ double red[16];
  const int ri = blockIdx.x;
  if (ri >= nrve) return;
  const RveDev& rv = rvs[ri];
  if (rv.skip) return;
  CgState* cg = rv.cg;
  if ((step == FIN_PAP || step == FIN_RR) && (rv.fold || cg->done)) return;
  const int pass = (step == FIN_SNORM || step == FIN_PAP) ? P_ZF
                   : ((step == FIN_RESID || step == FIN_RR) ? P_ZI : P_VEC);
  const int nt = rv.tiles[pass];
  if (step == FIN_LAMBDA) {
    // smallest and largest tangent eigenvalue over the tiles; the collocation
    // scheme's reference medium C_ref = 1/2 (lmin + lmax) I_s = 2 mu0 I_s
    double lo = INFINITY, hi = 0.0;
    for (int t = threadIdx.x; t < nt; t += blockDim.x) {
      lo = fmin(lo, rv.partial[t]);
      hi = fmax(hi, rv.partial[nt + t]);
    }
    __shared__ double slo[256], shi[256];
    slo[threadIdx.x] = lo;
    shi[threadIdx.x] = hi;
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int i = 1; i < (int)blockDim.x; ++i) {
      lo = fmin(lo, slo[i]);
      hi = fmax(hi, shi[i]);
    }
    cg->lmin = lo;
    cg->lmax = hi;
    cg->lam0 = 0.0;
    cg->mu0 = 0.25 * (lo + hi);
    return;
  }
  const int nv = step == FIN_SIGMA ? 6 : 1;
  const double* part = step == FIN_RR ? rv.partial_rr : rv.partial;
  double tot[6];
  for (int i = 0; i < nv; ++i) tot[i] = sum_partials(part + (size_t)i * nt, nt, red);
  if (threadIdx.x != 0) return;
  const double t = tot[0];
  switch (step) {
    case FIN_SNORM:
      cg->snorm2 = t;
      break;
    case FIN_RESID: {
      cg->rr = t;
      cg->bnorm2 = t;
      cg->beta = 0.0;
      const double t1 = cg->eta2 * t, t2 = cg->floor2 * cg->snorm2;
      cg->target2 = t1 > t2 ? t1 : t2;
      cg->iters = 0;
      if (cg->force >= 0) {
        cg->done = (cg->force == 0);
        cg->status = cg->done ? CG_FORCED : CG_RUNNING;
      } else {
        cg->done = (t <= cg->target2);
        cg->status = cg->done ? CG_CONVERGED : CG_RUNNING;
      }
      break;
    }
    case FIN_PAP:
      cg->pAp = t;
      if (cg->rich) {
        cg->alpha = 1.0;
      } else if (!(t > 0.0) || !(t < INFINITY)) {
        cg->done = 1;
        cg->status = CG_BREAKDOWN;
      } else {
        cg->alpha = cg->rr / t;
      }
      break;
    case FIN_RR: {
      cg->iters += 1;
      cg->rr_new = t;
      int done = 0, st = CG_RUNNING;
      if (cg->force >= 0) {
        if (cg->iters >= cg->force) {
          done = 1;
          st = CG_FORCED;
        }
      } else if (t <= cg->target2) {
        done = 1;
        st = CG_CONVERGED;
      } else if (cg->iters >= cg->max_iter) {
        done = 1;
        st = CG_MAXITER;
      }
      cg->beta = cg->rich ? 0.0 : t / cg->rr;
      cg->rr = t;
      cg->status = st;
      cg->done = done;
      break;
    }
    case FIN_DNORM:
      cg->dnorm2 = t;
      break;
    case FIN_SIGMA:
      for (int c = 0; c < 6; ++c) cg->Sigma[c] = tot[c] / double(rv.nvox);
      break;
    default:
      break;
  }
}

// CG configuration of every RVE of a launch before a linear solve.
__global__ void k_cg_setup(RveDev* __restrict__ rvs, int nrve, double eta2, double floor2, int max_iter,
                           int force, int rich) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrve) return;
  CgState* cg = rvs[r].cg;
  cg->rich = rich;
  cg->eta2 = eta2;
  cg->floor2 = floor2;
  cg->max_iter = max_iter;
  cg->force = force;
  cg->iters = 0;
  cg->done = 0;
  cg->status = CG_RUNNING;
}

// Extreme eigenvalues of each voxel's consistent tangent, per tile (min in
// partial[tile], max in partial[tiles + tile]).  For the compact tangent
// C = K I(x)I + 2G' I_d + csign m (x) m with a deviatoric m they are 3K
// (volumetric), 2G' (four deviatoric directions normal to m) and
// 2G' + csign |m|^2 (along m).
__global__ void __launch_bounds__(256) k_tangent_bounds(const RveDev* __restrict__ rvs, int nrve, int vox_per_tile) {
  __shared__ double slo[256], shi[256];
  int tile;
  const int ri = find_rve(rvs, nrve, P_VEC, tile);
  if (ri < 0) return;
  const RveDev& rv = rvs[ri];
  const long long nvox = rv.nvox;
  const double* tg = (const double*)rv.tang;
  const long long v0 = (long long)tile * vox_per_tile;
  const int nv = (int)min((long long)vox_per_tile, nvox - v0);
  double lo = INFINITY, hi = 0.0;
  for (int t = threadIdx.x; t < nv; t += blockDim.x) {
    const long long v = v0 + t;
    const MatDev& mt = rv.mats[rv.phase[v]];
    const double g2 = tg[v];
    double mm = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) mm += tg[(c + 1) * nvox + v] * tg[(c + 1) * nvox + v];
    const double a = 3.0 * mt.K, b = g2, c = g2 + mt.csign * mm;
    lo = fmin(lo, fmin(a, fmin(b, c)));
    hi = fmax(hi, fmax(a, fmax(b, c)));
  }
  slo[threadIdx.x] = lo;
  shi[threadIdx.x] = hi;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)blockDim.x; ++i) {
      lo = fmin(lo, slo[i]);
      hi = fmax(hi, shi[i]);
    }
    const int nt = rv.tiles[P_VEC];
    rv.partial[tile] = lo;
    rv.partial[nt + tile] = hi;
  }
}

// Reference medium C_ref = lam0 I(x)I + 2 mu0 I_s of every member (the
// operator Gamma_ref of fftg_apply_Gamma).
__global__ void k_set_cref(RveDev* __restrict__ rvs, int nrve, double lam0, double mu0) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrve) return;
  rvs[r].cg->lam0 = lam0;
  rvs[r].cg->mu0 = mu0;
}

__global__ void k_add_const(double* __restrict__ f, long long nvox, double e0, double e1, double e2, double e3,
                            double e4, double e5) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 6 * nvox) return;
  const int c = (int)(i / nvox);
  const double e[6] = {e0, e1, e2, e3, e4, e5};
  f[i] += e[c];
}

// ------------------------------------------------------------ launchers
// the Rader slots, the reduction scratch and nl lines of ext points each
// (line and, unless in place, scratch)
template <class T>
static size_t tile_lds(int nl, int ext) {
  return (size_t)nl * ext * sizeof(cx<T>) + (size_t)(nl + 2) * sizeof(cx<T>) + 16 * sizeof(double) + 64;
}

size_t lds_z(int mixed, int rows, int n2, int ext, int rtab) {
  if (ext <= 0) ext = 2 * n2;
  return mixed ? tile_lds<float>(3 * rows, ext) + axis_lds_bytes<float>(n2, rtab)
               : tile_lds<double>(3 * rows, ext) + axis_lds_bytes<double>(n2, rtab);
}
size_t lds_y(int mixed, int lines, int n1, int ext, int rtab) {
  if (ext <= 0) ext = 2 * n1;
  return mixed ? tile_lds<float>(lines, ext) + axis_lds_bytes<float>(n1, rtab)
               : tile_lds<double>(lines, ext) + axis_lds_bytes<double>(n1, rtab);
}
template <class T>
static size_t slab_lds(int n1, int n2) {
  const int nd = n1 > n2 + 1 ? n1 : n2 + 1;
  return axis_lds_bytes<T>(n2) + axis_lds_bytes<T>(n1) + (size_t)2 * n1 * (n2 + 1) * sizeof(cx<T>) +
         (size_t)(nd + 2) * sizeof(cx<T>) + 32 * sizeof(double) + 64;
}
size_t lds_slab(int mixed, int n1, int n2) { return mixed ? slab_lds<float>(n1, n2) : slab_lds<double>(n1, n2); }
size_t lds_x(int mixed, int lines, int n0, int ext, int rtab) {
  if (ext <= 0) ext = 2 * n0;
  return mixed ? tile_lds<float>(6 * lines, ext) + axis_lds_bytes<float>(n0, rtab)
               : tile_lds<double>(6 * lines, ext) + axis_lds_bytes<double>(n0, rtab);
}

template <class T, int BIG, int NF>
static void zfwd_go(dim3 G, dim3 B, size_t lds, hipStream_t s, const RveDev* rv, int nrve, int rows, int ldmax,
                    int in_mode, int in_role, int tan_mode, int want_norm, int check_done, int update_p) {
  hipLaunchKernelGGL((k_zfwd<T, BIG, NF>), G, B, lds, s, rv, nrve, rows, ldmax, in_mode, in_role, tan_mode, want_norm,
                     check_done, update_p);
}
template <int DIR>
struct ypass_go {
  template <class T, int BIG, int NF>
  static void go(dim3 G, dim3 B, size_t lds, hipStream_t s, const RveDev* rv, int nrve, int lines, int ldmax,
                 int check_done) {
    hipLaunchKernelGGL((k_ypass<T, DIR, BIG, NF>), G, B, lds, s, rv, nrve, lines, ldmax, check_done);
  }
};
template <class T, int BIG, int NF>
static void xpass_go(dim3 G, dim3 B, size_t lds, hipStream_t s, const RveDev* rv, int nrve, int lines, int ldmax,
                     double scale, int check_done) {
  hipLaunchKernelGGL((k_xpass<T, BIG, NF>), G, B, lds, s, rv, nrve, lines, ldmax, scale, check_done);
}
template <int BIG>
static void xpass_gamma_go(dim3 G, dim3 B, size_t lds, hipStream_t s, const RveDev* rv, int nrve, int lines,
                           int ldmax, double scale, int check_done) {
  hipLaunchKernelGGL((k_xpass<double, BIG, 0, 1>), G, B, lds, s, rv, nrve, lines, ldmax, scale, check_done);
}
template <class T, int BIG, int NF>
static void zinv_go(dim3 G, dim3 B, size_t lds, hipStream_t s, const RveDev* rv, int nrve, int rows, int ldmax,
                    int out_mode, int out_role, int check_done, int p_role) {
  hipLaunchKernelGGL((k_zinv<T, BIG, NF>), G, B, lds, s, rv, nrve, rows, ldmax, out_mode, out_role, check_done, p_role);
}
template <class T, int BIG, int NF>
static void slab_fwd_go(dim3 G, dim3 B, size_t lds, hipStream_t s, const RveDev* rv, int nrve, int n1max, int n2max,
                        int in_mode, int in_role, int tan_mode, int want_norm, int check_done, int update_p, int p_in,
                        int p_out) {
  hipLaunchKernelGGL((k_slab_fwd<T, BIG, NF>), G, B, lds, s, rv, nrve, n1max, n2max, in_mode, in_role, tan_mode,
                     want_norm, check_done, update_p, p_in, p_out);
}
template <class T, int BIG, int NF>
static void slab_inv_go(dim3 G, dim3 B, size_t lds, hipStream_t s, const RveDev* rv, int nrve, int n1max, int n2max,
                        int out_mode, int out_role, int check_done, int p_role) {
  hipLaunchKernelGGL((k_slab_inv<T, BIG, NF>), G, B, lds, s, rv, nrve, n1max, n2max, out_mode, out_role, check_done,
                     p_role);
}

// Member count with the tile-mapping flag for the tiled kernels.
static int nrve_arg(int nrve, const LaunchCfg& cfg) { return nrve | (cfg.xcd_remap ? kLaunchRemap : 0); }

// Launches fn<T, BIG, NF> for the launch's precision and codelet set, with
// the kernels built for 31-point lines (NF = 31) when every member takes
// each axis the kernel transforms (the bits of axes in cfg.direct31) by the
// 31-point direct DFT.
#define DISPATCH_TBF(fn, axes, ...)                                    \
  do {                                                                 \
    const bool f31 = !cfg.big_radix && (cfg.direct31 & (axes)) == (axes); \
    if (mixed) {                                                    \
      if (cfg.big_radix) fn<float, 1, 0>(__VA_ARGS__);              \
      else if (f31) fn<float, 0, 31>(__VA_ARGS__);                  \
      else fn<float, 0, 0>(__VA_ARGS__);                            \
    } else {                                                        \
      if (cfg.big_radix) fn<double, 1, 0>(__VA_ARGS__);             \
      else if (f31) fn<double, 0, 31>(__VA_ARGS__);                 \
      else fn<double, 0, 0>(__VA_ARGS__);                           \
    }                                                               \
  } while (0)

hipError_t launch_zfwd(int mixed, const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg, size_t lds,
                       int in_mode, int in_role, int tan_mode, int want_norm, int check_done, int update_p,
                       hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  const int nr = nrve_arg(nrve, cfg);
  DISPATCH_TBF(zfwd_go, 4, dim3(tiles), dim3(cfg.threads_z), lds, s, rv, nr, cfg.rows_per_tile, cfg.n2max, in_mode,
              in_role, tan_mode, want_norm, check_done, update_p);
  return hipGetLastError();
}

hipError_t launch_ypass(int mixed, int dir, const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg,
                        size_t lds, int check_done, hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  const int nr = nrve_arg(nrve, cfg);
  const dim3 G(tiles), B(cfg.threads_y);
  if (dir < 0)
    DISPATCH_TBF(ypass_go<-1>::go, 2, G, B, lds, s, rv, nr, cfg.lines_y, cfg.n1max, check_done);
  else
    DISPATCH_TBF(ypass_go<1>::go, 2, G, B, lds, s, rv, nr, cfg.lines_y, cfg.n1max, check_done);
  return hipGetLastError();
}

hipError_t launch_xpass(int mixed, const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg, size_t lds,
                        double scale, int check_done, hipStream_t s, int gamma) {
  if (tiles <= 0) return hipSuccess;
  const int nr = nrve_arg(nrve, cfg);
  if (gamma) {
    // the collocation operator runs in FP64 with the general transforms
    if (mixed) return hipErrorInvalidValue;
    if (cfg.big_radix)
      xpass_gamma_go<1>(dim3(tiles), dim3(cfg.threads_x), lds, s, rv, nr, cfg.lines_x, cfg.n0max, scale, check_done);
    else
      xpass_gamma_go<0>(dim3(tiles), dim3(cfg.threads_x), lds, s, rv, nr, cfg.lines_x, cfg.n0max, scale, check_done);
    return hipGetLastError();
  }
  DISPATCH_TBF(xpass_go, 1, dim3(tiles), dim3(cfg.threads_x), lds, s, rv, nr, cfg.lines_x, cfg.n0max, scale,
              check_done);
  return hipGetLastError();
}

hipError_t launch_zinv(int mixed, const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg, size_t lds,
                       int out_mode, int out_role, int check_done, int p_role, hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  const int nr = nrve_arg(nrve, cfg);
  DISPATCH_TBF(zinv_go, 4, dim3(tiles), dim3(cfg.threads_z), lds, s, rv, nr, cfg.rows_per_tile, cfg.n2max, out_mode,
              out_role, check_done, p_role);
  return hipGetLastError();
}

hipError_t launch_slab_fwd(int mixed, const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg, size_t lds,
                           int in_mode, int in_role, int tan_mode, int want_norm, int check_done, int update_p,
                           int p_in, int p_out, hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  const int nr = nrve_arg(nrve, cfg);
  DISPATCH_TBF(slab_fwd_go, 6, dim3(tiles), dim3(cfg.threads_s), lds, s, rv, nr, cfg.n1max, cfg.n2max, in_mode,
              in_role, tan_mode, want_norm, check_done, update_p, p_in, p_out);
  return hipGetLastError();
}

hipError_t launch_slab_inv(int mixed, const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg, size_t lds,
                           int out_mode, int out_role, int check_done, int p_role, hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  const int nr = nrve_arg(nrve, cfg);
  DISPATCH_TBF(slab_inv_go, 6, dim3(tiles), dim3(cfg.threads_s), lds, s, rv, nr, cfg.n1max, cfg.n2max, out_mode,
              out_role, check_done, p_role);
  return hipGetLastError();
}

hipError_t launch_newton_update(const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg, hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  const int nr = nrve_arg(nrve, cfg);
  hipLaunchKernelGGL(k_newton_update, dim3(tiles), dim3(cfg.threads_v), 0, s, rv, nr, cfg.vec_per_tile);
  return hipGetLastError();
}

hipError_t launch_constitutive(int mixed, const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg,
                               int eps_role, int commit, hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  const int nr = nrve_arg(nrve, cfg);
  if (mixed)
    hipLaunchKernelGGL(k_constitutive<float>, dim3(tiles), dim3(cfg.threads_v), 0, s, rv, nr, cfg.vec_per_tile,
                       eps_role, commit);
  else
    hipLaunchKernelGGL(k_constitutive<double>, dim3(tiles), dim3(cfg.threads_v), 0, s, rv, nr,
                       cfg.vec_per_tile, eps_role, commit);
  return hipGetLastError();
}

hipError_t launch_finalize(const RveDev* rv, int nrve, int step, hipStream_t s) {
  if (nrve <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(nrve), dim3(256), 0, s, rv, nrve, step);
  return hipGetLastError();
}

hipError_t launch_cg_setup(const RveDev* rv, int nrve, double eta2, double floor2, int max_iter, int force,
                           hipStream_t s, int rich) {
  hipLaunchKernelGGL(k_cg_setup, dim3((nrve + 63) / 64), dim3(64), 0, s, (RveDev*)rv, nrve, eta2, floor2,
                     max_iter, force, rich);
  return hipGetLastError();
}

hipError_t launch_tangent_bounds(const RveDev* rv, int nrve, int tiles, const LaunchCfg& cfg, hipStream_t s) {
  if (tiles <= 0) return hipSuccess;
  const int nr = nrve_arg(nrve, cfg);
  hipLaunchKernelGGL(k_tangent_bounds, dim3(tiles), dim3(256), 0, s, rv, nr, cfg.vec_per_tile);
  return hipGetLastError();
}

hipError_t launch_set_cref(const RveDev* rv, int nrve, double lam0, double mu0, hipStream_t s) {
  hipLaunchKernelGGL(k_set_cref, dim3((nrve + 63) / 64), dim3(64), 0, s, (RveDev*)rv, nrve, lam0, mu0);
  return hipGetLastError();
}

}  // namespace fftg

hipError_t fftg_add_const(double* f, long long nvox, const double* E, hipStream_t s) {
  const long long n = 6 * nvox;
  hipLaunchKernelGGL(fftg::k_add_const, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, f, nvox, E[0], E[1],
                     E[2], E[3], E[4], E[5]);
  return hipGetLastError();
}
