// Batched 1-D complex FFTs of odd length held in LDS.
//
// A workgroup transforms nl lines at once; line l lives at buf + l * ld.
// Lengths N whose prime factors are direct radices (3, 5, 7, 9, 11, 13, 17)
// run a Stockham autosort chain (one radix per stage, ping-pong between two
// LDS buffers).  A prime N beyond those runs Rader's algorithm: with g a
// primitive root mod N, X[g^-m] = x_0 + (a (*) b)_m, a_q = x[g^q],
// b_j = w^(g^-j), a cyclic convolution of length N-1 done as
// DFT_{N-1}^-1 (DFT_{N-1}(a) * DFT_{N-1}(b)/(N-1)), and X_0 = x_0 + sum a_q.
// The length-(N-1) chains use radix 2 or 4 for the even part.
//
// These are the fast transforms F and F^-1 of the paper's Eq.
// (DFT_forward_inverse); normalisation is left to the caller.
#pragma once

#include <type_traits>

#include "fftg_internal.h"

namespace fftg {

template <int R>
struct RadixConst;
#include "radix_consts.h"

// Global-memory view of a device pointer.  Pointers read from a launch
// descriptor are generic, and loads through them compile to flat loads: the
// compiler must then assume that they may alias LDS (so each is waited for
// before the next LDS store) and they count against the LDS wait counter
// too.  Through this view they are global loads, which can be issued in
// batches ahead of the stores that consume them.
#define FFTG_GLOBAL __attribute__((address_space(1)))
template <class V>
__device__ __forceinline__ FFTG_GLOBAL V* gmem(V* p) {
  return (FFTG_GLOBAL V*)p;
}
// Element loads and stores through such views (complex values component by
// component: the compiler merges them into one wide access).
template <class V>
__device__ __forceinline__ V gload(const FFTG_GLOBAL V* p) {
  return *p;
}
template <class T>
__device__ __forceinline__ cx<T> gload(const FFTG_GLOBAL cx<T>* p) {
  const FFTG_GLOBAL T* q = (const FFTG_GLOBAL T*)p;
  return cx<T>{q[0], q[1]};
}
template <class T>
__device__ __forceinline__ void gstore(FFTG_GLOBAL cx<T>* p, cx<T> v) {
  FFTG_GLOBAL T* q = (FFTG_GLOBAL T*)p;
  q[0] = v.re;
  q[1] = v.im;
}

// lds[dst(t)] = g[src(t)] for t < n (n >= 1) over the workgroup; each
// thread issues the loads of up to U elements before it stores any of them.
// Indices past the end repeat element n - 1 (the same value to the same
// place), so that no load or store sits behind a branch: the compiler would
// otherwise sink each load next to its guarded store and wait for them one
// at a time.
template <int U, class V, class Src, class Dst>
__device__ __forceinline__ void lds_gather(V* lds, const FFTG_GLOBAL V* g, int n, Src src, Dst dst) {
  const int bd = blockDim.x;
  for (int t0 = threadIdx.x; t0 < n; t0 += U * bd) {
    V v[U];
    int ti[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ti[u] = min(t0 + u * bd, n - 1);
      v[u] = gload(g + src(ti[u]));
    }
#pragma unroll
    for (int u = 0; u < U; ++u) lds[dst(ti[u])] = v[u];
  }
}

// A compile-time integer passed by value (for generic lambdas).
template <int V>
struct IntC {
  static constexpr int value = V;
};

template <class T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// a * (s * i) for s = +1 / -1
template <int S, class T>
__device__ __forceinline__ cx<T> mul_si(cx<T> a) {
  return S > 0 ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}

// Integer division by a workgroup-uniform divisor through the FP32
// reciprocal, exact for 0 <= t < 2^22: the reciprocal instruction is within
// one unit in the last place, so the float quotient t * inv is off by less
// than one and a single remainder test corrects it.
struct FastDiv {
  float inv;
  int d;
  __device__ __forceinline__ explicit FastDiv(int d_) : inv(__builtin_amdgcn_rcpf((float)d_)), d(d_) {}
  __device__ __forceinline__ int div(int t) const {
    int q = (int)((float)t * inv);
    const int r = t - q * d;
    q += (r >= d) ? 1 : 0;
    q -= (r < 0) ? 1 : 0;
    return q;
  }
};

// Direct DFT of R points in registers: X_k = sum_n v_n exp(DIR 2 pi i n k / R).
// run_store hands each output to st(k, X_k) as soon as it is formed, so the
// codelet never holds inputs and outputs at the same time.
template <int R, int DIR, class T>
struct Dft {
  // odd R: with s_j = v_j + v_{R-j}, d_j = v_j - v_{R-j} (formed in place),
  // X_k = A_k + DIR i B_k and X_{R-k} = A_k - DIR i B_k, where
  // A_k = v_0 + sum_j s_j cos(2 pi jk/R), B_k = sum_j d_j sin(2 pi jk/R).
  template <class S>
  __device__ __forceinline__ static void run_store(cx<T>* v, S&& st) {
    constexpr int m = (R - 1) / 2;
#pragma unroll
    for (int j = 1; j <= m; ++j) {
      const cx<T> a = v[j], b = v[R - j];
      v[j] = cadd(a, b);
      v[R - j] = csub(a, b);
    }
    cx<T> x0 = v[0];
#pragma unroll
    for (int j = 1; j <= m; ++j) x0 = cadd(x0, v[j]);
    st(0, x0);
    if constexpr (R <= 9) {
#pragma unroll
      for (int k = 1; k <= m; ++k) one_pair(v, k, k, st);
    } else {
      // large radices: the k loop stays rolled (constants by uniform index)
      // so that the unrolled body, and the register footprint, stay small
#pragma unroll 1
      for (int k = 1; k <= m; ++k) one_pair(v, k, k, st);
    }
  }

  template <class S>
  __device__ __forceinline__ static void one_pair(const cx<T>* v, int k, int, S&& st) {
    constexpr int m = (R - 1) / 2;
    cx<T> A = v[0];
    cx<T> B = {T(0), T(0)};
    int jk = 0;
#pragma unroll
    for (int j = 1; j <= m; ++j) {
      jk += k;
      if (jk >= R) jk -= R;   // (j k) mod R
      const T c = T(RadixConst<R>::c[jk]);
      const T sn = T(RadixConst<R>::s[jk]);
      A.re += v[j].re * c;
      A.im += v[j].im * c;
      B.re += v[R - j].re * sn;
      B.im += v[R - j].im * sn;
    }
    const cx<T> iB = mul_si<DIR>(B);
    st(k, cadd(A, iB));
    st(R - k, csub(A, iB));
  }
};

template <int DIR, class T>
struct Dft<2, DIR, T> {
  template <class S>
  __device__ __forceinline__ static void run_store(cx<T>* v, S&& st) {
    const cx<T> a = v[0], b = v[1];
    st(0, cadd(a, b));
    st(1, csub(a, b));
  }
};

template <int DIR, class T>
struct Dft<4, DIR, T> {
  template <class S>
  __device__ __forceinline__ static void run_store(cx<T>* v, S&& st) {
    const cx<T> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const cx<T> s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
    const cx<T> t = mul_si<DIR>(d13);
    st(0, cadd(s02, s13));
    st(2, csub(s02, s13));
    st(1, cadd(d02, t));
    st(3, csub(d02, t));
  }
};

// N1 N2 points (coprime factors) by the prime-factor (Good-Thomas) split,
// which needs no twiddles: with input index n = (N2 n1 + N1 n2) mod N and
// output index k = (c1 k1 + c2 k2) mod N, c1 = N2 (N2^-1 mod N1) and
// c2 = N1 (N1^-1 mod N2) (so k1 = k mod N1, k2 = k mod N2), the kernel
// w_N^(n k) factors into w_N1^(n1 k1) w_N2^(n2 k2).  N2 N1-point DFTs over
// n1, then N1 N2-point DFTs over n2, all indices fixed at compile time.
__host__ __device__ constexpr int inv_mod(int a, int m) {
  int r = 1;
  while ((a * r) % m != 1) ++r;
  return r;
}
template <int N1, int N2, int DIR, class T>
struct PfaDft {
  static constexpr int N = N1 * N2;
  static constexpr int c1 = N2 * inv_mod(N2 % N1, N1);
  static constexpr int c2 = N1 * inv_mod(N1 % N2, N2);
  template <class S>
  __device__ __forceinline__ static void run_store(cx<T>* v, S&& st) {
    cx<T> b[N1][N2];
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) {
      cx<T> a[N1];
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) a[n1] = v[(N2 * n1 + N1 * n2) % N];
      Dft<N1, DIR, T>::run_store(a, [&](int k1, cx<T> x) { b[k1][n2] = x; });
    }
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1)
      Dft<N2, DIR, T>::run_store(b[k1], [&](int k2, cx<T> x) { st((c1 * k1 + c2 * k2) % N, x); });
  }
};
template <int DIR, class T>
struct Dft<15, DIR, T> : PfaDft<3, 5, DIR, T> {};

// One Stockham stage of radix R over nl lines of an M-point chain.
// Butterfly j of a line reads src[j + q M/R], twiddles by w_M^(q k M/(Ns R))
// with k = j mod Ns, and writes dst[(j - k) R + k + q Ns].
template <int R, int DIR, class T>
__device__ __forceinline__ void stockham_stage(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst,
                                               int ld, int nl, int M, int Ns,
                                               const cx<T>* __restrict__ tw) {
  const int nb = M / R;
  const int total = nb * nl;
  const int tstep = M / (Ns * R);
  const FastDiv fnb(nb), fns(Ns);
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int line = fnb.div(t);
    const int j = t - line * nb;
    const int k = j - fns.div(j) * Ns;
    const cx<T>* s = src + line * ld + j;
    cx<T> v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = s[q * nb];
    if (Ns > 1) {
#pragma unroll
      for (int q = 1; q < R; ++q) {
        cx<T> w = tw[q * k * tstep];
        if (DIR > 0) w.im = -w.im;
        v[q] = cmul(v[q], w);
      }
    }
    cx<T>* d = dst + line * ld + (j - k) * R + k;
    Dft<R, DIR, T>::run_store(v, [&](int q, cx<T> x) { d[q * Ns] = x; });
  }
}

template <class T>
__device__ __forceinline__ const cx<T>* axis_tw(const AxisDev& P);
template <>
__device__ __forceinline__ const cx<double>* axis_tw<double>(const AxisDev& P) { return P.tw64; }
template <>
__device__ __forceinline__ const cx<float>* axis_tw<float>(const AxisDev& P) { return P.tw32; }

template <class T>
__device__ __forceinline__ const cx<T>* rader_bhat(const AxisDev& P, int dir);
template <>
__device__ __forceinline__ const cx<double>* rader_bhat<double>(const AxisDev& P, int dir) {
  return dir < 0 ? P.bf64 : P.bi64;
}
template <>
__device__ __forceinline__ const cx<float>* rader_bhat<float>(const AxisDev& P, int dir) {
  return dir < 0 ? P.bf32 : P.bi32;
}

// LDS copy of one axis' tables, loaded once per workgroup so that the
// barrier-separated stages never wait on global memory.
template <class T>
struct AxisLds {
  const AxisDev* dev;  // sizes and radices (uniform loads)
  int M, nst, rader;
  cx<T>* tw;     // M roots exp(-2 pi i m / M)
  int* pin;      // Rader permutations (M each)
  int* pout;
  cx<T>* bf;     // Rader DFT_M(b)/M, forward and inverse
  cx<T>* bi;
  const cx<T>* g_tw;  // root table in global memory
};

// LDS bytes of the tables of an axis of length <= N: the roots, and for
// Rader's algorithm (rader != 0) its two kernel transforms and its two
// permutations.  A multiple of 16 either way.
template <class T>
__host__ __device__ constexpr size_t axis_lds_bytes(int N, int rader = 1) {
  return rader ? (((size_t)N * (3 * sizeof(cx<T>) + 2 * sizeof(int))) + 15) / 16 * 16
               : ((size_t)N * sizeof(cx<T>) + 15) / 16 * 16;
}

// Carves the tables out of base and reads the axis fields (no table loads).
template <class T>
__device__ __forceinline__ void axis_lds_setup(const AxisDev& P, char* base, AxisLds<T>& A) {
  A.dev = &P;
  A.M = P.M;
  A.nst = P.nst;
  A.rader = P.rader;
  const int N = P.N;
  A.tw = reinterpret_cast<cx<T>*>(base);
  A.bf = A.tw + N;
  A.bi = A.bf + N;
  A.pin = reinterpret_cast<int*>(A.bi + N);
  A.pout = A.pin + N;
  A.g_tw = axis_tw<T>(P);
}

// The table copy in two halves: fetch loads this thread's first roots into
// registers, store writes them and copies the rest (and the Rader tables).
// A kernel issues its own data loads in between, so that both wait for one
// memory round trip instead of two; the caller's next __syncthreads
// publishes the tables.
template <class T>
struct AxisFetch {
  cx<T> v[2];
  int t[2];
};
template <class T>
__device__ __forceinline__ AxisFetch<T> axis_lds_fetch(const AxisLds<T>& A) {
  AxisFetch<T> f;
  const FFTG_GLOBAL cx<T>* g = gmem(A.g_tw);
  const int bd = blockDim.x;
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    f.t[u] = min((int)threadIdx.x + u * bd, A.M - 1);
    f.v[u] = gload(g + f.t[u]);
  }
  return f;
}
template <class T>
__device__ __forceinline__ void axis_lds_store(const AxisLds<T>& A, const AxisFetch<T>& f) {
  const int bd = blockDim.x;
#pragma unroll
  for (int u = 0; u < 2; ++u) A.tw[f.t[u]] = f.v[u];
  const int M = A.M;
  if (M > 2 * bd) {
    const FFTG_GLOBAL cx<T>* g = gmem(A.g_tw);
    for (int t = threadIdx.x + 2 * bd; t < M; t += bd) A.tw[t] = gload(g + t);
  }
  if (A.rader == AX_RADER) {
    const AxisDev& P = *A.dev;
    const FFTG_GLOBAL cx<T>* bf = gmem(rader_bhat<T>(P, -1));
    const FFTG_GLOBAL cx<T>* bi = gmem(rader_bhat<T>(P, 1));
    const FFTG_GLOBAL int* qi = gmem(P.perm_in);
    const FFTG_GLOBAL int* qo = gmem(P.perm_out);
    for (int t = threadIdx.x; t < M; t += bd) {
      const cx<T> b = gload(bf + t), c = gload(bi + t);
      const int d = qi[t], e = qo[t];
      A.bf[t] = b;
      A.bi[t] = c;
      A.pin[t] = d;
      A.pout[t] = e;
    }
  }
}

// Runs the Stockham chain of P on a (result ends in a; buffers are swapped).
// BIG = 0 compiles only the radix 2, 3, 4, 5, 7, 9 codelets (lower register
// use); BIG = 1 adds 11, 13, 17.
template <int DIR, class T, int BIG>
__device__ void run_chain(cx<T>*& a, cx<T>*& b, int ld, int nl, const AxisLds<T>& P) {
  const cx<T>* tw = P.tw;
  int Ns = 1;
  for (int s = 0; s < P.nst; ++s) {
    const int R = P.dev->radix[s];
    switch (R) {
      case 2: stockham_stage<2, DIR, T>(a, b, ld, nl, P.M, Ns, tw); break;
      case 3: stockham_stage<3, DIR, T>(a, b, ld, nl, P.M, Ns, tw); break;
      case 4: stockham_stage<4, DIR, T>(a, b, ld, nl, P.M, Ns, tw); break;
      case 5: stockham_stage<5, DIR, T>(a, b, ld, nl, P.M, Ns, tw); break;
      case 7: stockham_stage<7, DIR, T>(a, b, ld, nl, P.M, Ns, tw); break;
      case 9: stockham_stage<9, DIR, T>(a, b, ld, nl, P.M, Ns, tw); break;
      case 11: if (BIG) stockham_stage<11, DIR, T>(a, b, ld, nl, P.M, Ns, tw); break;
      case 13: if (BIG) stockham_stage<13, DIR, T>(a, b, ld, nl, P.M, Ns, tw); break;
      case 17: if (BIG) stockham_stage<17, DIR, T>(a, b, ld, nl, P.M, Ns, tw); break;
      default: break;  // rejected at plan creation
    }
    __syncthreads();
    cx<T>* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
}

// Chains of compile-time length, each line owned by TL consecutive lanes of
// one wavefront.  For the extents met most often (15, 63, 255) the radices,
// butterfly counts and twiddle strides are constants, so a lane forms its
// butterfly indices with a few integer operations, and the stages of a line
// exchange data through LDS ordered by the wavefront alone: the LDS performs
// one wavefront's operations in issue order, so a stage reads what the
// previous one wrote without a workgroup barrier.  Same Stockham stages as
// stockham_stage (butterfly j reads src[j + q M/R], twiddles by
// w_M^(q k M/(Ns R)), k = j mod Ns, writes dst[(j - k) R + k + q Ns]).
template <int TL_, int... Rs>
struct CtSpec {
  static constexpr int TL = TL_;                    // lanes per line
  static constexpr int NST = (int)sizeof...(Rs);    // stages
};
template <int N>
struct CtPlan {
  static constexpr bool ok = false;
};
template <>
struct CtPlan<15> {
  static constexpr bool ok = true;
  using spec = CtSpec<5, 3, 5>;     // 5 and 3 butterflies per stage
};
template <>
struct CtPlan<63> {
  static constexpr bool ok = true;
  using spec = CtSpec<9, 9, 7>;     // 7 and 9 butterflies per stage
};
template <>
struct CtPlan<255> {
  static constexpr bool ok = true;
  using spec = CtSpec<17, 15, 17>;  // 17 and 15 butterflies per stage (radix 15 by the prime-factor split)
};

// Orders this wavefront's LDS accesses for the compiler (the hardware keeps
// them in order); no instruction is emitted.
__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __asm__ volatile("" ::: "memory");
}

// One stage in place: every lane loads the inputs of all its butterflies,
// the wavefront's reads are ordered before its writes, and the outputs go
// back to the same line.  A stage reads and writes every point
// of the line exactly once and the line belongs to one wavefront, so no
// write can land before a read of the old value.  The inputs of all the
// lane's butterflies are live at once (IT x R points).
// (The loads and stores go through ldf(i) and stf(i, x) for chain position
// i, so that a caller can fold a permutation or a pointwise step into a
// stage: the reads of the stage still cover every position once before any
// write.)
template <int R, int DIR, class T, int M, int NS, int TL, class Ld, class St>
__device__ __forceinline__ void ct_stage_io(Ld&& ldf, St&& stf, const cx<T>* __restrict__ tw, int g) {
  constexpr int NB = M / R;
  constexpr int TSTEP = M / (NS * R);
  constexpr int IT = (NB + TL - 1) / TL;
  cx<T> v[IT][R];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int j = g + it * TL;
    if (NB % TL == 0 || it < IT - 1 || j < NB) {
#pragma unroll
      for (int q = 0; q < R; ++q) v[it][q] = ldf(j + q * NB);
    }
  }
  wave_lds_order();
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int j = g + it * TL;
    if (NB % TL == 0 || it < IT - 1 || j < NB) {
      const int k = NS > 1 ? j % NS : 0;
      if constexpr (NS > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          cx<T> w = tw[q * k * TSTEP];
          if (DIR > 0) w.im = -w.im;
          v[it][q] = cmul(v[it][q], w);
        }
      }
      const int d = (j - k) * R + k;
      Dft<R, DIR, T>::run_store(v[it], [&](int q, cx<T> x) { stf(d + q * NS, x); });
    }
  }
}

// The stages of a chain in place, the first reading through ldf and the
// last writing through stf (the others read and write a).
template <int... Rs>
struct Radices {};
template <int DIR, class T, int M, int NS, int TL, class Ld, class St, int R, int... Rest>
__device__ __forceinline__ void ct_run_io(cx<T>* a, Ld&& ldf, St&& stf, const cx<T>* tw, int g,
                                          Radices<R, Rest...>) {
  if constexpr (sizeof...(Rest) == 0) {
    ct_stage_io<R, DIR, T, M, NS, TL>(ldf, stf, tw, g);
  } else {
    ct_stage_io<R, DIR, T, M, NS, TL>(ldf, [&](int i, cx<T> x) { a[i] = x; }, tw, g);
    wave_lds_order();
    ct_run_io<DIR, T, M, NS * R, TL>(a, [&](int i) { return a[i]; }, stf, tw, g, Radices<Rest...>{});
  }
}
template <int DIR, class T, int M, int TL, class Ld, class St, int... Rs>
__device__ __forceinline__ void ct_chain_io(cx<T>* a, Ld&& ldf, St&& stf, const cx<T>* tw, int g, CtSpec<TL, Rs...>) {
  ct_run_io<DIR, T, M, 1, TL>(a, ldf, stf, tw, g, Radices<Rs...>{});
}

// nl lines of N points (stride ld) transformed in place in line (every
// stage loads a single butterfly per lane, so holding its inputs costs no
// more registers than the butterfly itself; no second buffer).  Called by
// the whole workgroup (blockDim a multiple of 64); ends with a workgroup
// barrier.
template <int DIR, class T, int N>
__device__ __forceinline__ cx<T>* ct_fft(cx<T>* line, int ld, int nl, const cx<T>* tw) {
  using S = typename CtPlan<N>::spec;
  static_assert(inplace_axis(AX_CHAIN, N), "the host sizes these lines for one buffer");
  constexpr int TL = S::TL;
  constexpr int G = 64 / TL;  // lines per wavefront
  const int lane = (int)threadIdx.x & 63;
  const int grp = lane / TL;
  const int g = lane - grp * TL;
  const int ngr = ((int)blockDim.x >> 6) * G;
  if (grp < G) {
    for (int l = ((int)threadIdx.x >> 6) * G + grp; l < nl; l += ngr) {
      cx<T>* const a = line + l * ld;
      ct_chain_io<DIR, T, N>(a, [&](int i) { return a[i]; }, [&](int i, cx<T> x) { a[i] = x; }, tw, g, S{});
    }
  }
  __syncthreads();
  return line;
}

// Rader's algorithm for a prime N whose convolution length M = N - 1 has a
// compile-time chain, each line owned by TL lanes of one
// wavefront (as ct_fft), all in place in the line.  x_0 stays in line[0];
// the first forward stage reads a_q = x_(g^q) straight from its permuted
// place, the last forward stage multiplies its outputs by DFT_M(b)/M
// (keeping a's DFT at 0, the sum of x_1..x_(N-1), in dc), and the last
// inverse stage writes X_(g^-m) = x_0 + (a (*) b)_m to its permuted place;
// X_0 = x_0 + that sum.  Every stage reads all M points before it writes
// (the gather and the scatter are permutations of line[1..M]), and every
// step is line-local, so the steps are ordered by the wavefront alone.
template <int N>
struct CtRader {
  static constexpr bool ok = false;
};
template <>
struct CtRader<127> {
  static constexpr bool ok = true;
  using spec = CtSpec<18, 7, 2, 9>;   // 126 = 7 2 9: 18, 63 and 14 butterflies per stage
};

template <int DIR, class T, int N>
__device__ __forceinline__ cx<T>* ct_rader(cx<T>* line, int ld, int nl, const AxisLds<T>& P, cx<T>* dc) {
  using S = typename CtRader<N>::spec;
  constexpr int M = N - 1;
  constexpr int TL = S::TL;
  constexpr int G = 64 / TL;
  const int lane = (int)threadIdx.x & 63;
  const int grp = lane / TL;
  const int g = lane - grp * TL;
  const int ngr = ((int)blockDim.x >> 6) * G;
  const cx<T>* bh = DIR < 0 ? P.bf : P.bi;
  if (grp < G) {
    for (int l = ((int)threadIdx.x >> 6) * G + grp; l < nl; l += ngr) {
      cx<T>* const ln = line + l * ld;
      cx<T>* const a = ln + 1;
      const cx<T> x0 = ln[0];
      ct_chain_io<-1, T, M>(
          a, [&](int i) { return ln[P.pin[i]]; },
          [&](int i, cx<T> x) {
            if (i == 0) dc[l] = x;
            a[i] = cmul(x, bh[i]);
          },
          P.tw, g, S{});
      wave_lds_order();
      ct_chain_io<1, T, M>(
          a, [&](int i) { return a[i]; }, [&](int i, cx<T> x) { ln[P.pout[i]] = cadd(x0, x); }, P.tw, g, S{});
      wave_lds_order();
      if (g == 0) ln[0] = cadd(x0, dc[l]);
      wave_lds_order();
    }
  }
  __syncthreads();
  return line;
}

// Direct DFT of nl odd-length lines: X_k = sum_j x_j w^(jk),
// w = exp(-+ 2 pi i / N).  With s_j = x_j + x_(N-j) and d_j = x_j - x_(N-j)
// (j = 1 .. (N-1)/2) and theta = 2 pi j k / N,
//   X_k = A + DIR i B,  X_(N-k) = A - DIR i B,
//   A = x_0 + sum_j s_j cos theta,  B = sum_j d_j sin theta,
// so one thread forms the pair X_k, X_(N-k) (k = 1 .. (N-1)/2; slot 0 forms
// X_0) with four multiply-adds per j.  The root table holds
// exp(-i theta) = (cos theta, -sin theta).  FP64 forms the roots w^(jk) by
// recurrence in registers from w^k (one table read; the error after (N-1)/2
// steps stays near 1e-15), FP32 reads them from the table.  NF > 0 fixes N at
// compile time (all steps unrolled); NF == 0 takes N from the plan.
// The input comes from in0(l) -> x_0 and in(l, j, x_j&, x_(N-j)&), the
// output goes to out(l, k, X_k, X_(N-k)) (k = 0: X_0 twice), so that a
// caller can fold a pre- or post-processing step into the transform.  No
// barrier.
template <int DIR, class T, int NF, class In0, class In, class Out>
__device__ __forceinline__ void direct_dft_io(int nl, const AxisLds<T>& P, In0&& in0, In&& in, Out&& out) {
  const int N = NF > 0 ? NF : P.M;
  const int Hn = (N + 1) / 2;
  const FastDiv fh(Hn);
  for (int t = threadIdx.x; t < nl * Hn; t += blockDim.x) {
    const int l = NF > 0 ? t / Hn : fh.div(t);
    const int k = t - l * Hn;
    const cx<T> x0 = in0(l);
    T ar = x0.re, ai = x0.im, cr = T(0), ci = T(0);  // A and C = -B = sum_j d_j (-sin theta)
    auto step = [&](cx<T> a, cx<T> b, cx<T> w) {
      ar += (a.re + b.re) * w.re;
      ai += (a.im + b.im) * w.re;
      cr += (a.re - b.re) * w.im;
      ci += (a.im - b.im) * w.im;
    };
    if constexpr (NF > 0) {
      // every LDS read of the line (and, in FP32, of the roots) is issued
      // before the first multiply-add, so the thread waits once
      constexpr int H = (NF - 1) / 2;
      [[maybe_unused]] const cx<T> wk = P.tw[k];  // FP64 only (root recurrence)
      cx<T> va[H], vb[H];
#pragma unroll
      for (int j = 0; j < H; ++j) in(l, j + 1, va[j], vb[j]);
      if constexpr (std::is_same<T, double>::value) {
        __builtin_amdgcn_sched_barrier(0);
        cx<T> w = wk;
#pragma unroll
        for (int j = 0; j < H; ++j) {
          step(va[j], vb[j], w);
          w = cmul(w, wk);
        }
      } else {
        cx<T> wt[H];
        int idx = 0;
#pragma unroll
        for (int j = 0; j < H; ++j) {
          idx += k;
          idx -= (idx >= N) ? N : 0;
          wt[j] = P.tw[idx];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < H; ++j) step(va[j], vb[j], wt[j]);
      }
    } else if (std::is_same<T, double>::value) {
      const cx<T> wk = P.tw[k];
      cx<T> w = wk;
#pragma unroll 4
      for (int j = 1; j < Hn; ++j) {
        cx<T> a, b;
        in(l, j, a, b);
        step(a, b, w);
        w = cmul(w, wk);
      }
    } else {
      int idx = 0;
#pragma unroll 4
      for (int j = 1; j < Hn; ++j) {
        idx += k;
        idx -= (idx >= N) ? N : 0;
        cx<T> a, b;
        in(l, j, a, b);
        step(a, b, P.tw[idx]);
      }
    }
    // i B = -i C = (C.im, -C.re)
    const T pr = DIR > 0 ? ar + ci : ar - ci;
    const T pi = DIR > 0 ? ai - cr : ai + cr;
    const T mr = DIR > 0 ? ar - ci : ar + ci;
    const T mi = DIR > 0 ? ai + cr : ai - cr;
    out(l, k, cx<T>{pr, pi}, cx<T>{mr, mi});
  }
}

// The direct DFT of nl lines from line into scratch (same stride ld).
template <int DIR, class T, int NF>
__device__ __forceinline__ void direct_dft(const cx<T>* line, cx<T>* scratch, int ld, int nl, const AxisLds<T>& P) {
  const int N = NF > 0 ? NF : P.M;
  direct_dft_io<DIR, T, NF>(
      nl, P, [&](int l) { return line[l * ld]; },
      [&](int l, int j, cx<T>& a, cx<T>& b) {
        a = line[l * ld + j];
        b = line[l * ld + N - j];
      },
      [&](int l, int k, cx<T> xk, cx<T> xm) {
        cx<T>* o = scratch + l * ld;
        o[k] = xk;
        if (k > 0) o[N - k] = xm;
      });
}

// In-LDS FFT of nl lines of length P.N, DIR = -1 forward, +1 inverse
// (unnormalised); NF > 0 compiles only the unrolled direct DFT of NF-point
// lines.  line and scratch each hold nl lines of stride ld >= N (scratch
// may alias line where inplace_axis holds); dc holds nl scratch slots
// (Rader only).  Returns the buffer holding the result (line or scratch).
// Must be called by the whole workgroup.
template <int DIR, class T, int BIG, int NF = 0>
__device__ __forceinline__ cx<T>* line_fft(cx<T>* line, cx<T>* scratch, int ld, int nl, const AxisLds<T>& P, cx<T>* dc) {
  if constexpr (NF > 0) {
    // kernels built for one line length run only where every line of the
    // launch takes the NF-point direct DFT (the host checks the plan's
    // axes): that length with every step unrolled, so that each thread
    // issues all its LDS reads before its first wait (more registers, hence
    // a separate build), and no other transform compiled in
    direct_dft<DIR, T, NF>(line, scratch, ld, nl, P);
    __syncthreads();
    return scratch;
  }
  if (P.rader == AX_CHAIN) {
    if (P.M == 63) return ct_fft<DIR, T, 63>(line, ld, nl, P.tw);
    if (P.M == 15) return ct_fft<DIR, T, 15>(line, ld, nl, P.tw);
    if constexpr (BIG) {
      if (P.M == 255) return ct_fft<DIR, T, 255>(line, ld, nl, P.tw);
    }
    cx<T>* a = line;
    cx<T>* b = scratch;
    run_chain<DIR, T, BIG>(a, b, ld, nl, P);
    return a;
  }
  if (P.rader == AX_DIRECT) {
    direct_dft<DIR, T, 0>(line, scratch, ld, nl, P);
    __syncthreads();
    return scratch;
  }
  if constexpr (BIG) {
    // 127 points: built only into the big-radix kernels (plans with such an
    // axis take them), whose register budget the in-place stages fit
    if (P.M == 126) return ct_rader<DIR, T, 127>(line, ld, nl, P, dc);
  }
  const int M = P.M;
  const int total = nl * M;
  const FastDiv fm(M);
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int l = fm.div(t);
    const int q = t - l * M;
    scratch[l * ld + q] = line[l * ld + P.pin[q]];
  }
  __syncthreads();
  cx<T>* a = scratch;
  cx<T>* b = line + 1;
  run_chain<-1, T, BIG>(a, b, ld, nl, P);
  const cx<T>* bh = DIR < 0 ? P.bf : P.bi;
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int l = fm.div(t);
    const int q = t - l * M;
    const cx<T> v = a[l * ld + q];
    if (q == 0) dc[l] = v;
    a[l * ld + q] = cmul(v, bh[q]);
  }
  __syncthreads();
  run_chain<1, T, BIG>(a, b, ld, nl, P);
  // a == scratch here (2 * nst swaps); scatter back, x_0 still in line[0]
  for (int t = threadIdx.x; t < total; t += blockDim.x) {
    const int l = fm.div(t);
    const int m = t - l * M;
    line[l * ld + P.pout[m]] = cadd(line[l * ld], a[l * ld + m]);
  }
  __syncthreads();
  for (int l = threadIdx.x; l < nl; l += blockDim.x) line[l * ld] = cadd(line[l * ld], dc[l]);
  __syncthreads();
  return line;
}

}  // namespace fftg
