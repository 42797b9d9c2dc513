// fftg_apply_GK_noalloc: the product G:(C:p) of fftg_apply_GK without a
// plan and without any device allocation, for callers that cannot allocate.
//
// Everything the five product passes need besides the caller's input and
// output -- the launch descriptor, the CG state the passes read, the FFT
// root tables and the half spectrum -- lives in one file-scope device array,
// `scratch`, of kScratchBytes.  The array exists once per device (the code
// object's loader places it); its address on a device is looked up with
// hipGetSymbolAddress the first time the entry point runs with that device
// current, and host code uses only that address (the array's own name is a
// host-side stand-in, not a device address).  A setup kernel rewrites the
// descriptor, clears the CG state and recomputes the root tables on every
// call, so a call never depends on what an earlier one left; calls that
// overlap on one device share the array and race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/fftg.h"
#include "fft_lds.h"
#include "fftg_internal.h"

// Message slot shared with the rest of the library (runtime.cpp).
void fftg_set_last_error(const char* msg);

namespace fftg {
namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;   // per device
constexpr size_t kDescOff = 0;                       // RveDev
constexpr size_t kCgOff = 4096;                      // CgState
constexpr size_t kPartOff = 4608;                    // (valid, never written by these passes)
constexpr size_t kTabOff = 8192;                     // root tables, 3 x kMaxAxisLen complex double
constexpr size_t kSpecOff = 65536;                   // half spectrum
static_assert(sizeof(RveDev) <= kCgOff - kDescOff, "descriptor slot");
static_assert(sizeof(CgState) <= kPartOff - kCgOff, "CG state slot");
static_assert(kTabOff + 3 * kMaxAxisLen * sizeof(cx<double>) <= kSpecOff, "table slots");

constexpr int kMaxDevices = 64;

}  // namespace
}  // namespace fftg

static __device__ __align__(256) char scratch[fftg::kScratchBytes];

namespace fftg {
namespace {

std::mutex g_mutex;
char* g_base[kMaxDevices];  // scratch address per device (null until looked up)

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
hipError_t scratch_base(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mutex);
  if (!g_base[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_base[dev] = static_cast<char*>(ptr);
  }
  *out = g_base[dev];
  return hipSuccess;
}

// What a plan would build for one axis, without Rader's algorithm (whose
// tables are computed on the host): a Stockham chain of odd radices, or the
// direct DFT for primes up to 53 and for extents up to 64 without a chain.
// Returns false where only Rader's algorithm applies.
bool axis_kind(int N, AxisDev& d) {
  d = AxisDev{};
  d.N = N;
  d.M = N;
  if (N == 1) {
    d.rader = AX_CHAIN;
    return true;
  }
  bool prime = N >= 2;
  for (int q = 2; q * q <= N; ++q)
    if (N % q == 0) prime = false;
  int rad[kMaxStages], ns = 0, m = N;
  const int odd[] = {9, 7, 5, 3, 11, 13, 17};
  for (int r : odd)
    while (m % r == 0 && ns < kMaxStages) {
      rad[ns++] = r;
      m /= r;
    }
  if (m == 1) {
    d.rader = AX_CHAIN;
    d.nst = ns;
    for (int i = 0; i < ns; ++i) d.radix[i] = rad[i];
    return true;
  }
  if ((prime && N <= 53) || N <= 64) {
    d.rader = AX_DIRECT;
    return true;
  }
  return false;
}

// Writes the descriptor (a kernel argument, so nothing is staged in host
// memory), clears the CG state and fills the root tables of the three axes
// (table a at tab + a kMaxAxisLen: exp(-2 pi i m / M), m < M).
__global__ void __launch_bounds__(256) k_noalloc_setup(RveDev d, char* base, int M0, int M1, int M2) {
  const int t = threadIdx.x;
  const int* src = reinterpret_cast<const int*>(&d);
  int* dst = reinterpret_cast<int*>(base + kDescOff);
  for (int i = t; i < (int)(sizeof(RveDev) / sizeof(int)); i += blockDim.x) dst[i] = src[i];
  int* cg = reinterpret_cast<int*>(base + kCgOff);
  for (int i = t; i < (int)(sizeof(CgState) / sizeof(int)); i += blockDim.x) cg[i] = 0;
  cx<double>* tab = reinterpret_cast<cx<double>*>(base + kTabOff);
  const int Ms[3] = {M0, M1, M2};
  for (int a = 0; a < 3; ++a) {
    const int M = Ms[a];
    for (int m = t; m < M; m += blockDim.x) {
      double s, c;
      sincospi(2.0 * (double)m / (double)M, &s, &c);
      tab[a * kMaxAxisLen + m] = cx<double>{c, -s};
    }
  }
}

fftg_status fail_msg(fftg_status st, const char* msg) {
  fftg_set_last_error(msg);
  return st;
}

}  // namespace
}  // namespace fftg

using namespace fftg;

extern "C" fftg_status fftg_apply_GK_noalloc(int n0, int n1, int n2, const double* d_in, double* d_out,
                                             fftg_tangent_mode mode, const uint8_t* d_phase, int n_phases,
                                             const fftg_material* mats, void* hip_stream) {
  const int ns[3] = {n0, n1, n2};
  for (int i = 0; i < 3; ++i)
    if (ns[i] < 1 || ns[i] % 2 == 0 || ns[i] > kMaxAxisLen)
      return fail_msg(FFTG_E_INVALID, "grid extents must be odd, >= 1 and <= 1024");
  if (!d_in || !d_out) return fail_msg(FFTG_E_INVALID, "NULL field pointer");
  if (mode != FFTG_TANGENT_IDENTITY && mode != FFTG_TANGENT_ELASTIC)
    return fail_msg(FFTG_E_INVALID, "noalloc product: mode must be IDENTITY or ELASTIC");
  if (mode == FFTG_TANGENT_ELASTIC) {
    if (!d_phase || !mats) return fail_msg(FFTG_E_INVALID, "ELASTIC needs a phase map and materials");
    if (n_phases < 1 || n_phases > kMaxPhases) return fail_msg(FFTG_E_INVALID, "n_phases must be in 1..16");
    for (int i = 0; i < n_phases; ++i)
      if (!(mats[i].K > 0) || !(mats[i].G > 0)) return fail_msg(FFTG_E_INVALID, "material needs K > 0, G > 0");
  }
  RveDev d{};
  d.n0 = n0;
  d.n1 = n1;
  d.n2 = n2;
  d.H = (n2 + 1) / 2;
  d.nvox = (long long)n0 * n1 * n2;
  d.nspec = (long long)n0 * n1 * d.H;
  const size_t spec_bytes = (size_t)6 * d.nspec * sizeof(cx<double>);
  if (spec_bytes > kScratchBytes - kSpecOff)
    return fail_msg(FFTG_E_INVALID,
                    "noalloc product: grid too large for the static scratch (6 n0 n1 (n2+1)/2 complex doubles "
                    "must fit 16 MiB - 64 KiB, e.g. 63^3)");
  GridSum gs;
  gs.n0 = n0;
  gs.n1 = n1;
  gs.n2 = n2;
  gs.rows = (long long)n0 * n1;
  gs.yl = 6LL * n0;
  gs.xl = n1;
  gs.hmax = d.H;
  gs.vox = d.nvox;
  for (int a = 0; a < 3; ++a) {
    if (!axis_kind(ns[a], d.ax[a]))
      return fail_msg(FFTG_E_UNSUPPORTED,
                      "noalloc product: extent needs Rader's algorithm (prime > 53 beyond 64 points); use a plan");
    for (int s = 0; s < d.ax[a].nst; ++s)
      if (d.ax[a].radix[s] > 9) gs.big = 1;
    if (!(d.ax[a].rader == AX_DIRECT && d.ax[a].M == 31)) gs.direct31 &= ~(1 << a);
  }
  char* base = nullptr;
  hipError_t e = scratch_base(&base);
  if (e != hipSuccess) return fail_msg(FFTG_E_HIP, hipGetErrorString(e));
  for (int a = 0; a < 3; ++a) d.ax[a].tw64 = reinterpret_cast<cx<double>*>(base + kTabOff) + a * kMaxAxisLen;
  d.buf[R_USER_IN] = const_cast<double*>(d_in);
  d.buf[R_USER_OUT] = d_out;
  d.spec = base + kSpecOff;
  d.phase = d_phase;
  if (mode == FFTG_TANGENT_ELASTIC) {
    d.n_phases = n_phases;
    for (int i = 0; i < n_phases; ++i) d.mats[i] = MatDev{mats[i].K, mats[i].G, 0.0, 0.0, 1.0, -1.0, 1.0, LAW_J2, 0};
  } else {
    d.n_phases = 1;  // the passes load the table even where the identity needs none
    d.mats[0] = MatDev{1.0, 0.5, 0.0, 0.0, 1.0, -1.0, 1.0, LAW_J2, 0};
  }
  d.mixed = 0;
  d.cg = reinterpret_cast<CgState*>(base + kCgOff);
  d.partial = reinterpret_cast<double*>(base + kPartOff);
  d.partial_rr = d.partial + 4;
  LaunchCfg cfg = choose_cfg(gs);
  cfg.slab = 0;  // the five passes (the slab form needs a second search-direction buffer)
  compute_tiles(cfg, n0, n1, n2, d.nvox, d.tiles);
  d.fold = 0;
  d.skip = 0;
  hipStream_t s = (hipStream_t)hip_stream;
  const RveDev* dv = reinterpret_cast<const RveDev*>(base + kDescOff);
  hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(256), 0, s, d, base, d.ax[0].M, d.ax[1].M, d.ax[2].M);
  e = hipGetLastError();
  const int tan = mode == FFTG_TANGENT_ELASTIC ? TAN_ELASTIC : TAN_IDENTITY;
  if (e == hipSuccess)
    e = launch_zfwd(0, dv, 1, d.tiles[P_ZF], cfg, lds_z(0, cfg.rows_per_tile, n2), IN_ROLE, R_USER_IN, tan, 0, 0,
                    PU_NONE, s);
  if (e == hipSuccess) e = launch_ypass(0, -1, dv, 1, d.tiles[P_Y], cfg, lds_y(0, cfg.lines_y, n1), 0, s);
  if (e == hipSuccess) e = launch_xpass(0, dv, 1, d.tiles[P_X], cfg, lds_x(0, cfg.lines_x, n0), 1.0, 0, s);
  if (e == hipSuccess) e = launch_ypass(0, 1, dv, 1, d.tiles[P_Y], cfg, lds_y(0, cfg.lines_y, n1), 0, s);
  if (e == hipSuccess)
    e = launch_zinv(0, dv, 1, d.tiles[P_ZI], cfg, lds_z(0, cfg.rows_per_tile, n2), OUT_PLAIN, R_USER_OUT, 0, R_P, s);
  if (e != hipSuccess) return fail_msg(FFTG_E_HIP, hipGetErrorString(e));
  return FFTG_OK;
}
