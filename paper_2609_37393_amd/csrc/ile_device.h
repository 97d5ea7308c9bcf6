// Device side of the factored extrinsic likelihood for gfx950.
//
// One lane evaluates one extrinsic sample.  Per sample (Eq. (def:lnL:Decomposed)):
//   sky frame and arrival times in FP64 (the delay feeds a sub-sample read),
//   antenna factors F_k = F+ + i Fx from the shared polarisation tensors,
//   -2Y_lm(incl, phiref) from per-mode Fourier coefficients in incl,
//   the data term x Re sum conj(F_k Y) Q_k(t_k) with a four-point Lagrange read
//   of the time-major table Q[k][t][mode] (taps outside the window read 0),
//   the model-norm term x^2/4 sum_k [|F_k|^2 a_k + Re(F_k^2 b_k)].
//
// Model-norm term.  a_k = Y^H U_k Y and b_k = Y^T V_k Y depend on the sample
// only through (incl, phiref), and both are finite trigonometric polynomials:
// d^l_{m,2}(incl) has degree l in incl (even/odd in incl for even/odd m), and
// the phiref dependence of a pair of modes is e^{i(m'-m) phi} (a_k) or
// e^{i(m+m') phi} (b_k).  So with L = max l,
//   g_c(incl, phi) in { a_k/4, Re b_k/4, -Im b_k/4 }
//   = sum_b C[b][c] beta_b(incl, phi),
//   beta_b in { cos(n incl) [1 | cos(q phi) | sin(q phi)], q even,
//               sin(n incl) [cos(q phi) | sin(q phi)],     q odd },
// n <= 2L, q <= 2L, and the per-sample work is one contraction of the basis
// values with the uniform coefficient table C (scalar loads).  C is exact up
// to rounding: a setup kernel samples g_c on a grid finer than twice the
// degree and projects (discrete orthogonality).  The finite angular harmonic
// content this relies on is the paper's Eq. (ap:angleharm) argument applied to
// (incl, phiref).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace rift {

constexpr int KMAX = 8;    // detectors
constexpr int MMAX = 25;   // modes
constexpr int LMAXC = 8;   // largest l
constexpr int QPAD = 4;    // zero rows on each side of every Q series
// Q tables hold W consecutive (internal) modes per time row, W = 2 for FP64
// and 4 for FP32: a row is 32 bytes in both, and a four-row stencil of one
// mode group is 128 bytes.
constexpr int QW64 = 2;
constexpr int QW32 = 4;
__host__ __device__ constexpr int q_groups(int M, int W) { return (M + W - 1) / W; }
// LDS staging of the data term: one unit is the 128-byte stencil block of a
// (mode group, detector) pair for each of the 64 lanes of a wavefront; every
// wavefront owns two unit buffers.
constexpr int STAGE_UNIT = 64 * 128;
constexpr int STAGE_WAVE = 2 * STAGE_UNIT;

template <class R>
struct alignas(2 * sizeof(R)) C2 {
  R x, y;
};

// Per-point description, resident in device memory (uniform per block).
struct PointDesc {
  int32_t K;        // real detectors
  int32_t M;        // modes
  int32_t n_t;      // table samples per detector and mode
  int32_t L;        // mode class: max l rounded to 2, 3, 4 or 8
  int32_t B;        // basis functions of the class
  int32_t KT;       // detector class (padded K)
  int32_t m_min;    // smallest m (modes are stored sorted by m)
  int32_t pad0;
  int64_t n;        // samples of this point in a batch
  int64_t s0;       // first sample column of this point in a batch
  double t0, inv_dt, gmst, d_ref;
  double T;         // mixed path: refinement margin (nats)
  double lnN;       // ln(n)
  double dten[KMAX][6];   // D00, D11, D22, 2 D01, 2 D02, 2 D12
  double rpos[KMAX][3];   // light-seconds
  int32_t m[MMAX];        // m of internal mode i (sorted ascending)
  int32_t odd[MMAX];      // m odd
  double ycoef[MMAX][LMAXC + 1];  // d^l_{m,2}(incl) sqrt((2l+1)/4pi) = sum_n ycoef cos|sin(n incl)
  float ycoef32[MMAX][LMAXC + 1];
  float dten32[KMAX][6];
  // mixed path, a-priori bound on |lnL_FP32 - lnL_FP64| of one sample:
  //   x bnd_d + x^2 sum_k [ (|F_k| + eF[k])^2 bnd_q[k]
  //                         + (2 (|F_k| + eF[k]) eF[k] + eF[k]^2) l1q[k] ]
  // (written on the device by k_bound; see there for the derivation)
  double bnd_d;
  double bnd_q[KMAX];
  double l1q[KMAX];  // sum of |C| over detector k's three coefficient columns
  double eF[KMAX];   // bound on |F_FP32 - F| of detector k
  // arrival-time binning (sorted evaluation): a Morton key of bin_bits
  // bits per detector over the first bin_dims detectors; its top bin_cb
  // bits are the coarse bucket.  The point's sort tiles are bin_st0 ..
  // bin_st0 + bin_nst - 1; its [coarse bucket][sort tile] count matrix
  // starts at bin_mbase.
  int32_t bin_dims;
  int32_t bin_bits;
  int32_t bin_cb;
  int32_t bin_nst;
  int32_t bin_st0;
  int32_t bin_pad;
  int64_t bin_mbase;
  // Q of each detector in groups of W internal modes, QPAD zero rows at both
  // ends of every series: [KT][ceil(M / W)][n_t + 2 QPAD][W] complex, the
  // slots past M zero.  A stencil starting at row j-1 in [-QPAD, n_t] reads
  // padded rows j-1+QPAD .. j+2+QPAD.
  const double* Q64;
  const float* Q32;
  const double* C64;      // [B][3 KT]
  const float* C32;       // [B][3 KT]
};

// Work unit: samples [s, s + cnt) (global columns) of point p.
struct Tile {
  int32_t p;
  int32_t cnt;
  int64_t s;
};

template <int L>
struct Cls {
  static constexpr int NI = 2 * L;                        // incl degree of g_c
  static constexpr int NQ = 2 * L;                        // phi degree of g_c
  static constexpr int MAXM = (L == 2) ? 5 : (L == 3) ? 12 : (L == 4) ? 21 : 25;
  static constexpr int NY = L + 1;                        // Fourier terms of d_lm
  static constexpr int B = (NI + 1) + (NQ / 2) * 2 * (NI + 1) + ((NQ + 1) / 2) * 2 * NI;
};

__device__ __forceinline__ void sincos_(double a, double* s, double* c) { sincos(a, s, c); }
__device__ __forceinline__ void sincos_(float a, float* s, float* c) { sincosf(a, s, c); }

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Address spaces: the point description and the coefficient tables are read
// with uniform addresses through the constant space (scalar loads into
// SGPRs); per-lane data (samples, the Q table, outputs) through the global
// space (vector loads).
#define RIFT_CONST __attribute__((address_space(4)))
#define RIFT_GLOBAL __attribute__((address_space(1)))
#define RIFT_LDS __attribute__((address_space(3)))

struct PointDesc;
typedef const RIFT_CONST PointDesc* PDesc;

template <class T>
__device__ __forceinline__ const RIFT_CONST T* as_const(const T* p) {
  return (const RIFT_CONST T*)p;
}
template <class T>
__device__ __forceinline__ const RIFT_GLOBAL T* as_global(const T* p) {
  return (const RIFT_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ RIFT_GLOBAL T* as_global_w(T* p) {
  return (RIFT_GLOBAL T*)p;
}

// Identity the optimiser cannot see through.  Applied to the (uniform) point
// pointer at the top of every sample iteration so that the ~10^3 uniform
// coefficient loads of a sample stay scalar loads inside the loop instead of
// being hoisted out of it.
template <class T>
__device__ __forceinline__ const RIFT_CONST T* opaque(const T* p) {
  uint64_t v = (uint64_t)p;
  asm volatile("" : "+s"(v));
  return (const RIFT_CONST T*)v;
}
template <class T>
__device__ __forceinline__ const RIFT_CONST T* opaque(const RIFT_CONST T* p) {
  uint64_t v = (uint64_t)p;
  asm volatile("" : "+s"(v));
  return (const RIFT_CONST T*)v;
}
// Empty register use: the value must be computed before this point.
template <class R>
__device__ __forceinline__ void pin(R& v) {
  asm volatile("" : "+v"(v));
}
// Empty scalar use: the (uniform) value must be in SGPRs at this point.
template <class R>
__device__ __forceinline__ void pin_s(R v) {
  asm volatile("" ::"s"(v));
}
// Pin a (uniform) global pointer to SGPRs, so that per-lane accesses at a
// 32-bit offset from it use the scalar-base addressing form.
__device__ __forceinline__ const RIFT_GLOBAL char* uniform_ptr(const RIFT_GLOBAL char* p) {
  uint64_t v = (uint64_t)p;
  asm volatile("" : "+s"(v));
  return (const RIFT_GLOBAL char*)v;
}
template <class R>
__device__ __forceinline__ C2<R> ldq(const RIFT_GLOBAL R* q, int64_t idx) {
  C2<R> v;
  v.x = q[2 * idx];
  v.y = q[2 * idx + 1];
  return v;
}

template <class R>
struct Tab;
template <>
struct Tab<double> {
  static constexpr int W = QW64;
  static __device__ __forceinline__ const RIFT_GLOBAL double* Q(PDesc P) { return as_global(P->Q64); }
  static __device__ __forceinline__ const RIFT_CONST double* C(PDesc P) { return as_const(P->C64); }
  static __device__ __forceinline__ double y(PDesc P, int i, int n) { return P->ycoef[i][n]; }
  static __device__ __forceinline__ double d(PDesc P, int k, int a) { return P->dten[k][a]; }
};
template <>
struct Tab<float> {
  static constexpr int W = QW32;
  static __device__ __forceinline__ const RIFT_GLOBAL float* Q(PDesc P) { return as_global(P->Q32); }
  static __device__ __forceinline__ const RIFT_CONST float* C(PDesc P) { return as_const(P->C32); }
  static __device__ __forceinline__ float y(PDesc P, int i, int n) { return P->ycoef32[i][n]; }
  static __device__ __forceinline__ float d(PDesc P, int k, int a) { return P->dten32[k][a]; }
};

// Row b of the harmonic basis of class L (the order of the coefficient
// table): kind 0 = cos(n incl); 1, 2 = cos(n incl) {cos, sin}(q phi) for even
// q >= 2; 3, 4 = sin(n incl) {cos, sin}(q phi) for odd q.  Packed as
// kind | n << 4 | q << 12.
template <int L>
__host__ __device__ constexpr int basis_row(int b) {
  constexpr int NI = 2 * L;
  int bb = b;
  for (int q = 0; q <= NI; ++q) {
    if (q == 0) {
      if (bb <= NI) return 0 | (bb << 4);
      bb -= NI + 1;
    } else if ((q & 1) == 0) {
      if (bb < 2 * (NI + 1)) return (1 + (bb & 1)) | ((bb >> 1) << 4) | (q << 12);
      bb -= 2 * (NI + 1);
    } else {
      if (bb < 2 * NI) return (3 + (bb & 1)) | ((1 + (bb >> 1)) << 4) | (q << 12);
      bb -= 2 * NI;
    }
  }
  return -1;
}

// Model-norm contraction acc[c] = sum_b C[b][c] beta_b(incl, phi), fully
// unrolled over the B x 3 KT coefficients (classes L <= 4): every index is a
// template constant, so the tables below stay in registers.  The uniform
// coefficients stream through SGPRs in chunks of 128 bytes, each chunk
// prefetched while the previous one is used.  Scalar loads complete out of
// order, so the wait for a chunk (pin_s) comes before the next chunk is
// issued (a wait never covers the prefetch), and the accumulators are pinned
// after each chunk's FMAs so that those FMAs stay ahead of the next wait.
template <class R, int KT, int L>
struct Contract {
  static constexpr int NI = 2 * L;
  static constexpr int W = 3 * KT;
  static constexpr int NC = Cls<L>::B * W;
  static constexpr int CH = 128 / (int)sizeof(R);
  static constexpr int NCH = (NC + CH - 1) / CH;
  struct Tabs {
    R ct[NI + 1], st[NI + 1];  // cos(n incl), sin(n incl)
    R ex[NI + 1], ey[NI + 1];  // e^{i q phi}
  };

  template <int J>
  static __device__ __forceinline__ void coef(R c, R* acc, const Tabs& T) {
    if constexpr (J < NC) {
      constexpr int rb = basis_row<L>(J / W);
      constexpr int kind = rb & 15, n = (rb >> 4) & 255, q = rb >> 12;
      R beta;
      if constexpr (kind == 0) beta = T.ct[n];
      else if constexpr (kind == 1) beta = T.ct[n] * T.ex[q];
      else if constexpr (kind == 2) beta = T.ct[n] * T.ey[q];
      else if constexpr (kind == 3) beta = T.st[n] * T.ex[q];
      else beta = T.st[n] * T.ey[q];
      acc[J % W] = fma(c, beta, acc[J % W]);
    }
  }
  template <int C, int... I>
  static __device__ __forceinline__ void fm(const R (&buf)[CH], R* acc, const Tabs& T,
                                            std::integer_sequence<int, I...>) {
    (coef<C * CH + I>(buf[I], acc, T), ...);
  }
  template <int C>
  static __device__ __forceinline__ void ld(R (&buf)[CH], const RIFT_CONST R* Cc) {
    const RIFT_CONST R* p = opaque(Cc) + C * CH;
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (C * CH + i < NC) buf[i] = p[i];
  }
  template <int C>
  static __device__ __forceinline__ void wait(const R (&buf)[CH]) {
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (C * CH + i < NC) pin_s(buf[i]);
  }
  template <int C>
  static __device__ __forceinline__ void step(const RIFT_CONST R* Cc, R (&cur)[CH], R (&nxt)[CH],
                                              R* acc, const Tabs& T) {
    if constexpr (C < NCH) {
      wait<C>(cur);
      if constexpr (C + 1 < NCH) ld<C + 1>(nxt, Cc);
      fm<C>(cur, acc, T, std::make_integer_sequence<int, CH>{});
#pragma unroll
      for (int c = 0; c < W; ++c) pin(acc[c]);
      step<C + 1>(Cc, nxt, cur, acc, T);
    }
  }
  static __device__ __forceinline__ void run(PDesc P, R ci, R si, R cf, R sf, R* acc) {
    Tabs T;
    T.ct[0] = 1;
    T.st[0] = 0;
    T.ct[1] = ci;
    T.st[1] = si;
#pragma unroll
    for (int n = 2; n <= NI; ++n) {
      T.ct[n] = 2 * ci * T.ct[n - 1] - T.ct[n - 2];
      T.st[n] = 2 * ci * T.st[n - 1] - T.st[n - 2];
    }
    T.ex[0] = 1;
    T.ey[0] = 0;
    T.ex[1] = cf;
    T.ey[1] = sf;
#pragma unroll
    for (int q = 2; q <= NI; ++q) {
      T.ex[q] = T.ex[q - 1] * cf - T.ey[q - 1] * sf;
      T.ey[q] = T.ex[q - 1] * sf + T.ey[q - 1] * cf;
    }
    const RIFT_CONST R* Cc = Tab<R>::C(P);
    R bA[CH], bB[CH];
    ld<0>(bA, Cc);
    step<0>(Cc, bA, bB, acc, T);
  }
};

// Per-mode arithmetic of the data term, every multiply-add written as an
// explicit fma (with multiply-adds otherwise fused only within one source
// expression, an expression gives the same bits in every kernel that inlines
// it).
//   phase_up: ph <- ph e^{i phi};  phase_down: ph <- ph e^{-i phi}
template <class R>
__device__ __forceinline__ void phase_up(C2<R>& ph, R cf, R sf) {
  const R a = fma(ph.x, cf, -ph.y * sf), b = fma(ph.y, cf, ph.x * sf);
  ph.x = a;
  ph.y = b;
}
template <class R>
__device__ __forceinline__ void phase_down(C2<R>& ph, R cf, R sf) {
  const R a = fma(ph.x, cf, ph.y * sf), b = fma(ph.y, cf, -ph.x * sf);
  ph.x = a;
  ph.y = b;
}
// d_i(incl) from its Fourier coefficients (sin series for odd m).
template <class R, int NY>
__device__ __forceinline__ R mode_d(PDesc P, int i, const R* cn, const R* sn) {
  R d = 0;
  if (P->odd[i]) {
#pragma unroll
    for (int n = 1; n < NY; ++n) d = fma(Tab<R>::y(P, i, n), sn[n], d);
  } else {
#pragma unroll
    for (int n = 0; n < NY; ++n) d = fma(Tab<R>::y(P, i, n), cn[n], d);
  }
  return d;
}
// Z += conj(Y) Qhat with Qhat the Lagrange combination of four taps.
template <class R>
__device__ __forceinline__ void mode_acc(C2<R>& Z, const R* w, C2<R> q0, C2<R> q1, C2<R> q2, C2<R> q3,
                                         R yx, R yy) {
  const R qx = fma(w[3], q3.x, fma(w[2], q2.x, fma(w[1], q1.x, w[0] * q0.x)));
  const R qy = fma(w[3], q3.y, fma(w[2], q2.y, fma(w[1], q1.y, w[0] * q0.y)));
  Z.x = fma(yx, qx, Z.x);
  Z.x = fma(yy, qy, Z.x);
  Z.y = fma(yx, qy, Z.y);
  Z.y = fma(-yy, qx, Z.y);
}
// The four Lagrange weights on nodes -1, 0, 1, 2 at fraction s.
template <class R>
__device__ __forceinline__ void lagrange4(R s, R* w) {
  w[0] = -s * (s - 1) * (s - 2) * (R)(1.0 / 6.0);
  w[1] = (s + 1) * (s - 1) * (s - 2) * (R)0.5;
  w[2] = -(s + 1) * s * (s - 2) * (R)0.5;
  w[3] = (s + 1) * s * (s - 1) * (R)(1.0 / 6.0);
}

// Row coordinate of a stencil: u = (t_k - t0) / dt.  A non-finite u poisons
// the sample; a finite u far outside the stored window is moved to just
// outside it (every tap then reads a zero pad row, the zero extension of the
// window), which also keeps the integer row in range.
__device__ __forceinline__ bool stencil_u(double& u, int n_t) {
  if (!(fabs(u) <= 1.0e300)) {  // NaN or infinite
    u = 0.0;
    return false;
  }
  u = fmin(fmax(u, -2.0 * QPAD), (double)n_t + 2.0 * QPAD);
  return true;
}

// a - 2 pi rint(a / 2 pi) in FP64 (2 pi split into two doubles): the angle
// in [-pi, pi] that the FP32 arithmetic starts from, so that its rounding to
// FP32 is at most pi 2^-25 rad whatever the size of the input angle.
__device__ __forceinline__ double reduce_2pi(double a) {
  const double k = rint(a * 0.15915494309189533577);
  double r = fma(-k, 6.283185307179586232, a);
  return fma(-k, 2.4492935982947064e-16, r);
}

// Detector groups of the data term (KT >= 2): at most three detectors share
// a pass over the modes; a remainder of one is split as 2 + 2, so every group
// has two or three detectors.
__host__ __device__ constexpr int det_group_size(int KT, int j) {
  int n3 = KT / 3, r = KT % 3;
  if (r == 1) {
    n3 -= 1;
    r = 4;
  }
  if (j < n3) return 3;
  const int jj = j - n3;
  if (r == 2) return jj == 0 ? 2 : 0;
  if (r == 4) return jj < 2 ? 2 : 0;
  return 0;
}
__host__ __device__ constexpr int det_group_start(int KT, int j) {
  int s = 0;
  for (int t = 0; t < j; ++t) s += det_group_size(KT, t);
  return s;
}

// Data term of detectors K0 .. K0+G-1 (2 <= G <= 3):
//   sum_k Re[conj(F_k) sum_i conj(Y_i) Qhat_{k,i}]
//   = sum_k Fre_k Re(Z_k) + Fim_k Im(Z_k),  Z_k = sum_i conj(Y_i) Qhat_{k,i},
// with Y_i = d_i(incl) e^{i m_i phi} (modes sorted by m, so the phase walks
// upward from e^{i m_min phi}) and Qhat the four-point Lagrange read at
// fraction sfr_k of the cell that starts at byte offset boff_k.
//
// The table holds W modes per time row, so the four stencil rows of a mode
// group are one contiguous 128-byte block per lane, at a 32-bit offset from
// the uniform start of series (k, group).  The blocks are read cooperatively:
// eight lanes fetch the eight 16-byte chunks of one lane's block, so a read
// instruction touches about 8 blocks' cache lines instead of 64 (the vector
// memory path costs about one cycle per distinct line per instruction).  The
// reads go straight to LDS (global_load_lds): lane l = 8 q + c' of read t
// fetches chunk c = c' ^ key(j) of the block of lane j = 8 t + q, which lands
// at j * 128 + c' * 16 = j * 128 + (c ^ key(j)) * 16.  With key(j) =
// (j >> 1) & 7 the eight lanes of equal j * 128 mod 256 within any sixteen
// consecutive lanes read eight different 16-byte columns, so lane j's own
// reads of its chunks are free of bank conflicts.
//
// Units (group p, detector g) are streamed with g fastest through the
// wavefront's two LDS buffers: unit u+1 is in flight while unit u is
// combined.  Requires the whole wavefront to be active.
//
// With CPLX, the imaginary part Im sum_k conj(F_k) Z_k is added to *acc_im as
// well (the complex data term whose real part is returned).
template <class R, int NY, int K0, int G, bool CPLX = false>
__device__ __forceinline__ double data_group(PDesc P, const RIFT_GLOBAL char* Qb, uint64_t gstride,
                                             uint64_t kstride, int M, int NGR, const uint32_t* boff,
                                             RIFT_LDS unsigned char* stage, const R* sfr, const R* Fre,
                                             const R* Fim, const R* cn, const R* sn, R cf, R sf,
                                             double* acc_im = nullptr) {
  static_assert(G >= 2 && G <= 3, "detector groups of two or three");
  constexpr int W = Tab<R>::W;
  static_assert(4 * W * sizeof(C2<R>) == 128, "128-byte stencil blocks");
  typedef R R2 __attribute__((ext_vector_type(2)));
  typedef float F4 __attribute__((ext_vector_type(4)));
  R w[G][4];
#pragma unroll
  for (int g = 0; g < G; ++g) lagrange4(sfr[K0 + g], w[g]);
  C2<R> Z[G];
#pragma unroll
  for (int g = 0; g < G; ++g) Z[g].x = Z[g].y = 0;
  C2<R> ph;
  ph.x = 1;
  ph.y = 0;
  const int mmin = P->m_min;
  for (int t = 0; t < -mmin; ++t) phase_down(ph, cf, sf);
  int mc = mmin < 0 ? mmin : 0;
  // Y of the W modes of group p; the slots past M repeat mode M-1 (their
  // taps are zero, so they add exact zeros)
  R yx[W], yy[W];
  auto ycomp = [&](int p) {
#pragma unroll
    for (int s = 0; s < W; ++s) {
      const int i = p * W + s;
      const int ic = i < M ? i : M - 1;
      const int mi = P->m[ic];
      while (mc < mi) {
        phase_up(ph, cf, sf);
        ++mc;
      }
      const R d = mode_d<R, NY>(P, ic, cn, sn);
      yx[s] = d * ph.x;
      yy[s] = d * ph.y;
    }
  };
  const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
  const int q = lane >> 3;
  // key(8 t + q) = ((t & 1) << 2) | (q >> 1): the chunk offsets of even and odd reads
  const uint32_t cx0 = (uint32_t)((lane & 7) ^ (q >> 1)) << 4;
  const uint32_t cx1 = (uint32_t)((lane & 7) ^ (4 | (q >> 1))) << 4;
  // read t of detector g: this lane's source offset
  uint32_t offt[G][8];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int t = 0; t < 8; ++t) offt[g][t] = (uint32_t)__shfl((int)boff[K0 + g], 8 * t + q) + ((t & 1) ? cx1 : cx0);
  // chunk c of this lane's block: rbase ^ (c << 4)
  const uint32_t rbase = (uint32_t)lane * 128u + ((uint32_t)((lane >> 1) & 7) << 4);
  auto issue = [&](int p, int g, int b) {
    const RIFT_GLOBAL char* ser = uniform_ptr(Qb + (uint64_t)(K0 + g) * kstride + (uint64_t)p * gstride);
    RIFT_LDS unsigned char* dst = stage + b * STAGE_UNIT;
#pragma unroll
    for (int t = 0; t < 8; ++t)
      __builtin_amdgcn_global_load_lds((const RIFT_GLOBAL void*)(ser + offt[g][t]), (RIFT_LDS void*)(dst + t * 1024),
                                       16, 0, 0);
  };
  auto consume = [&](int b, int g) {
    const RIFT_LDS unsigned char* src = stage + b * STAGE_UNIT;
    C2<R> u[4][W];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const uint32_t a = rbase ^ ((uint32_t)c << 4);
      if constexpr (sizeof(R) == 8) {
        const R2 v = *(const RIFT_LDS R2*)(src + a);
        u[c >> 1][c & 1].x = v.x;
        u[c >> 1][c & 1].y = v.y;
      } else {
        const F4 v = *(const RIFT_LDS F4*)(src + a);
        u[c >> 1][2 * (c & 1)].x = v.x;
        u[c >> 1][2 * (c & 1)].y = v.y;
        u[c >> 1][2 * (c & 1) + 1].x = v.z;
        u[c >> 1][2 * (c & 1) + 1].y = v.w;
      }
    }
#pragma unroll
    for (int s = 0; s < W; ++s) mode_acc(Z[g], w[g], u[0][s], u[1][s], u[2][s], u[3][s], yx[s], yy[s]);
    // the unit is combined here, before the next refill is issued (instead
    // of its FMAs sinking past later units, keeping their reads live)
    pin(Z[g].x);
    pin(Z[g].y);
  };
  // Unit u = p G + g uses buffer u & 1; an iteration covers an even number of
  // units, so every buffer index is a constant.  Each buffer is refilled only
  // after the LDS reads of its previous unit have completed, and a unit is
  // read only after its own global reads have (the newer unit's eight reads
  // may still be in flight).
  constexpr int UPI = (G % 2 == 0) ? G : 2 * G;
  const int total = NGR * G;
  issue(0, 0, 0);
#pragma unroll 1
  for (int p0 = 0; p0 < NGR; p0 += UPI / G) {
#pragma unroll
    for (int v = 0; v < UPI; ++v) {
      const int p = p0 + v / G;
      const int g = v % G;
      if (g == 0 && p >= NGR) break;
      if (p * G + g + 1 < total) {
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        issue(g + 1 == G ? p + 1 : p, (g + 1) % G, (v + 1) & 1);
        if (g == 0) ycomp(p);
        asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
      } else {
        if (g == 0) ycomp(p);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      }
      consume(v & 1, g);
    }
  }
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  double acc = 0.0;
#pragma unroll
  for (int g = 0; g < G; ++g)
    acc += (double)(Fre[K0 + g] * Z[g].x) + (double)(Fim[K0 + g] * Z[g].y);
  if constexpr (CPLX) {
    double ai = 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) ai += (double)(Fre[K0 + g] * Z[g].y) - (double)(Fim[K0 + g] * Z[g].x);
    *acc_im += ai;
  }
  return acc;
}

// Result of one sample evaluation.
struct Eval {
  double lnL;
  float bound;  // a-priori |lnL - lnL_FP64| bound (FP32 arithmetic only)
};

// Data term of one sample with its taps read straight from the table.
template <class R, int KT, int L, bool CPLX = false>
__device__ __forceinline__ double data_direct(PDesc P, RIFT_LDS unsigned char* stage, const int32_t* row,
                                              const R* sfr, const R* Fre, const R* Fim, const R* cn,
                                              const R* sn, R cf, R sf, double* im = nullptr) {
  static_assert(KT >= 2, "detector counts are padded to at least two");
  constexpr int NY = Cls<L>::NY;
  constexpr int W = Tab<R>::W;
  const int M = P->M;
  const int NGR = q_groups(M, W);
  uint32_t boff[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) boff[k] = (uint32_t)row[k] * (uint32_t)(W * sizeof(C2<R>));
  const RIFT_GLOBAL char* Qb = (const RIFT_GLOBAL char*)Tab<R>::Q(P);
  const uint64_t gstride = (uint64_t)(P->n_t + 2 * QPAD) * (W * sizeof(C2<R>));
  const uint64_t kstride = (uint64_t)NGR * gstride;
  constexpr int G0 = det_group_size(KT, 0), G1 = det_group_size(KT, 1), G2 = det_group_size(KT, 2);
  double data = data_group<R, NY, 0, G0, CPLX>(P, Qb, gstride, kstride, M, NGR, boff, stage, sfr, Fre, Fim, cn,
                                               sn, cf, sf, im);
  if constexpr (G1 > 0)
    data += data_group<R, NY, det_group_start(KT, 1), G1, CPLX>(P, Qb, gstride, kstride, M, NGR, boff, stage, sfr,
                                                                Fre, Fim, cn, sn, cf, sf, im);
  if constexpr (G2 > 0)
    data += data_group<R, NY, det_group_start(KT, 2), G2, CPLX>(P, Qb, gstride, kstride, M, NGR, boff, stage, sfr,
                                                                Fre, Fim, cn, sn, cf, sf, im);
  return data;
}

// Antenna factors of one sample and, for the data term, its stencils: the sky
// frame (FP64), the polarisation tensors and F_k = F+ + i Fx (R), and per
// detector the arrival time t_k and stencil row / fraction (FP64 phase).
template <class R, int KT>
struct Sky {
  R Fre[KT], Fim[KT];
  R sfr[KT];        // fractional position inside the stencil cell
  int32_t row[KT];  // padded index of the first stencil row, in [0, n_t + QPAD]
  bool bad;         // a non-finite arrival time
  double N[3];      // direction to the source
};
// The stencils of every detector for geocentric time t (the sky frame in S).
template <class R, int KT>
__device__ __forceinline__ void sky_stencils(PDesc P, double t, Sky<R, KT>& S) {
  const int n_t = P->n_t;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const RIFT_CONST double* r = P->rpos[k];
    const double tk = t - (r[0] * S.N[0] + r[1] * S.N[1] + r[2] * S.N[2]);
    double u = (tk - P->t0) * P->inv_dt;
    if (!stencil_u(u, n_t)) S.bad = true;
    const double jf = floor(u);
    const R s = (R)(u - jf);
    int j0 = (int)jf - 1;  // stencil rows j0 .. j0+3
    // wholly outside the stored window: read four zero pad rows
    j0 = j0 < -QPAD ? -QPAD : (j0 > n_t ? n_t : j0);
    S.row[k] = j0 + QPAD;
    S.sfr[k] = s;
  }
}
template <class R, int KT, bool STENCIL>
__device__ __forceinline__ void sky_eval(PDesc P, double ra, double dec, double psi, double tref, Sky<R, KT>& S) {
  double sg, cg, sd, cd;
  sincos_(P->gmst - ra, &sg, &cg);
  sincos_(dec, &sd, &cd);
  const double N0 = cd * cg, N1 = -cd * sg, N2 = sd;
  S.N[0] = N0;
  S.N[1] = N1;
  S.N[2] = N2;
  R sp, cp;
  sincos_((R)psi, &sp, &cp);
  const R ea0 = (R)sg, ea1 = (R)cg;
  const R ed0 = (R)(-sd * cg), ed1 = (R)(sd * sg), ed2 = (R)cd;
  const R X0 = -cp * ea0 + sp * ed0, X1 = -cp * ea1 + sp * ed1, X2 = sp * ed2;
  const R Y0 = sp * ea0 + cp * ed0, Y1 = sp * ea1 + cp * ed1, Y2 = cp * ed2;
  const R ep[6] = {X0 * X0 - Y0 * Y0, X1 * X1 - Y1 * Y1, X2 * X2 - Y2 * Y2,
                   X0 * X1 - Y0 * Y1, X0 * X2 - Y0 * Y2, X1 * X2 - Y1 * Y2};
  const R ex[6] = {2 * X0 * Y0, 2 * X1 * Y1, 2 * X2 * Y2,
                   X0 * Y1 + Y0 * X1, X0 * Y2 + Y0 * X2, X1 * Y2 + Y1 * X2};
  S.bad = false;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    R fp = 0, fx = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      fp += Tab<R>::d(P, k, a) * ep[a];
      fx += Tab<R>::d(P, k, a) * ex[a];
    }
    S.Fre[k] = fp;
    S.Fim[k] = fx;
  }
  if constexpr (STENCIL) sky_stencils<R, KT>(P, tref, S);
}

// The angles that the FP32 arithmetic takes, reduced in FP64 first.
template <class R>
__device__ __forceinline__ void reduce_angles(double& psi, double& incl, double& phi) {
  if constexpr (sizeof(R) == 4) {
    psi = reduce_2pi(psi);
    incl = reduce_2pi(incl);
    phi = reduce_2pi(phi);
  }
}

// Model-norm term sum_k |F_k|^2 a_k/4 + Re(F_k^2 b_k)/4 from the basis
// contraction at (incl, phiref); with BOUND, also the model-norm part of the
// FP32 error bound (see PointDesc).  `trig` is this lane's column of a
// block-shared scratch array (stride `ts` elements) that receives
// cos(n incl), n = 0..NI, then sin(n incl), for the runtime contraction loop
// of the l <= 8 class.
template <class R, int KT, int L>
__device__ __forceinline__ void norm_contract(PDesc P, R* __restrict__ trig, int ts, R ci, R si, R cf, R sf,
                                              R* acc) {
  typedef Cls<L> CL;
  constexpr int NI = CL::NI;
#pragma unroll
  for (int c = 0; c < 3 * KT; ++c) acc[c] = 0;
  if constexpr (L <= 4) {
    Contract<R, KT, L>::run(P, ci, si, cf, sf, acc);
  } else {
    {
      R c0 = 1, c1 = ci, s0 = 0, s1 = si;
#pragma unroll
      for (int n = 0; n <= NI; ++n) {
        trig[n * ts] = (n == 0) ? c0 : c1;
        trig[(NI + 1 + n) * ts] = (n == 0) ? s0 : s1;
        if (n > 0) {
          const R c2 = 2 * ci * c1 - c0, s2 = 2 * ci * s1 - s0;
          c0 = c1;
          c1 = c2;
          s0 = s1;
          s1 = s2;
        }
      }
    }
    // runtime loop over basis rows (reads cos/sin(n incl) from this lane's
    // column of the block-shared scratch array)
    const RIFT_CONST R* Cc = Tab<R>::C(P);
    {
      // q = 0: rows n = 0..NI, basis cos(n incl)
      R cur[3 * KT];
#pragma unroll
      for (int c = 0; c < 3 * KT; ++c) cur[c] = Cc[c];
      R tcur = trig[0];
#pragma unroll 1
      for (int n = 0; n <= NI; ++n) {
        const int nn = (n < NI) ? n + 1 : n;
        R nxt[3 * KT];
#pragma unroll
        for (int c = 0; c < 3 * KT; ++c) nxt[c] = Cc[nn * 3 * KT + c];
        const R tnxt = trig[nn * ts];
#pragma unroll
        for (int c = 0; c < 3 * KT; ++c) acc[c] = fma(cur[c], tcur, acc[c]);
#pragma unroll
        for (int c = 0; c < 3 * KT; ++c) cur[c] = nxt[c];
        tcur = tnxt;
      }
    }
    {
      // q >= 1: pairs of rows (T_n cos(q phi), T_n sin(q phi)); even q pairs
      // with cos(n incl) for n = 0..NI, odd q with sin(n incl) for n = 1..NI
      const int B = CL::B;
      int b = NI + 1;
      C2<R> eq;
      eq.x = cf;
      eq.y = sf;
      R cur[6 * KT];
#pragma unroll
      for (int c = 0; c < 6 * KT; ++c) cur[c] = Cc[b * 3 * KT + c];
#pragma unroll 1
      for (int q = 1; q <= NI; ++q) {
        const int odd = q & 1;
        const int base = odd ? (NI + 1) : 0;
        R tcur = trig[(base + odd) * ts];
#pragma unroll 1
        for (int n = odd; n <= NI; ++n, b += 2) {
          // next pair of rows (the last iteration re-reads its own rows)
          const int bn = (b + 2 < B) ? b + 2 : b;
          R nxt[6 * KT];
#pragma unroll
          for (int c = 0; c < 6 * KT; ++c) nxt[c] = Cc[bn * 3 * KT + c];
          const int tn = (n < NI) ? base + n + 1 : base + n;
          const R tnxt = trig[tn * ts];
          const R b1 = tcur * eq.x, b2 = tcur * eq.y;
#pragma unroll
          for (int c = 0; c < 3 * KT; ++c) {
            acc[c] = fma(cur[c], b1, acc[c]);
            acc[c] = fma(cur[3 * KT + c], b2, acc[c]);
          }
#pragma unroll
          for (int c = 0; c < 6 * KT; ++c) cur[c] = nxt[c];
          tcur = tnxt;
        }
        const R ex_ = eq.x * cf - eq.y * sf, ey_ = eq.x * sf + eq.y * cf;
        eq.x = ex_;
        eq.y = ey_;
      }
    }
  }
}

template <class R, int KT, int L, bool BOUND>
__device__ __forceinline__ double quad_term(PDesc P, R* __restrict__ trig, int ts, R ci, R si, R cf, R sf,
                                            const R* Fre, const R* Fim, double* wq_out) {
  R acc[3 * KT];
  norm_contract<R, KT, L>(P, trig, ts, ci, si, cf, sf, acc);
  double quad = 0.0;
  double wq = 0.0;  // model-norm part of the error bound (see PointDesc)
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const R f2 = Fre[k] * Fre[k] + Fim[k] * Fim[k];
    const R g2r = Fre[k] * Fre[k] - Fim[k] * Fim[k];
    const R g2i = 2 * Fre[k] * Fim[k];
    quad += (double)(f2 * acc[3 * k]) + (double)(g2r * acc[3 * k + 1]) +
            (double)(g2i * acc[3 * k + 2]);
    if (BOUND) {
      const double e = P->eF[k];
      const double fe = sqrt((double)f2) + e;  // >= |F_k| of the exact arithmetic
      wq += fe * fe * P->bnd_q[k] + (2.0 * fe + e) * e * P->l1q[k];
    }
  }
  if (BOUND) *wq_out = wq;
  return quad;
}

// cos(n incl), sin(n incl) for n < NY by the Chebyshev recurrences.
template <class R, int NY>
__device__ __forceinline__ void incl_harmonics(R ci, R si, R* cn, R* sn) {
  R c0 = 1, c1 = ci, s0 = 0, s1 = si;
#pragma unroll
  for (int n = 0; n < NY; ++n) {
    cn[n] = (n == 0) ? c0 : c1;
    sn[n] = (n == 0) ? s0 : s1;
    if (n > 0) {
      const R c2 = 2 * ci * c1 - c0, s2 = 2 * ci * s1 - s0;
      c0 = c1;
      c1 = c2;
      s0 = s1;
      s1 = s2;
    }
  }
}

// lnL = x data - x^2 quad with x = D_ref / D (FP64), NaN for a poisoned
// sample, and the a-priori FP32 bound |x| bnd_d + x^2 wq, rounded up on the
// way to FP32 (the factor covers the conversion).
template <bool BOUND>
__device__ __forceinline__ Eval combine(PDesc P, double dist, double data, double quad, double wq, bool bad) {
  const double x = P->d_ref / dist;
  Eval e;
  e.lnL = x * data - x * x * quad;
  if (bad) e.lnL = __builtin_nan("");
  e.bound = 0.0f;
  if (BOUND) e.bound = (float)((fabs(x) * P->bnd_d + x * x * wq) * (1.0 + 1.0e-6));
  return e;
}

// The distance-free terms of one sample: lnL(x) = x data - x^2 quad with
// x = D_ref / D; wq is the model-norm part of the FP32 bound (BOUND only).
struct Terms {
  double data, quad, wq;
  bool bad;
};

// Gauss-Hermite rule of the distance marginal (weight e^{-xi^2/2}; up to
// DM_MAX nodes) and the prior p(D) proportional to D^2 on [d_min, d_max].
constexpr int DM_MAX = 64;
struct DistRule {
  int32_t n;
  int32_t pad;
  double d_min, d_max;
  double ln_norm;  // ln(3 / (d_max^3 - d_min^3))
  double xi[DM_MAX], w[DM_MAX];
};

// ln of the likelihood marginalised over distance, Eq. (ap:dgh), from the
// terms: with lnL(x) = K x - R x^2 / 2 (K = data, R = 2 quad), the peak
// x* = K / R and width sigma = R^-1/2 of Eq. (ap:dpeak) centre and scale the
// nodes, and the rule's weights times e^{lnL(x* + xi sigma)} are
// sigma W_i e^{K^2 / 2R}, so
//   ln L_d = K^2 / 2R + ln sigma + ln sum_i W_i p_x(x* + xi_i sigma),
//   p_x(x) = d_ref^3 x^-4 3 / (d_max^3 - d_min^3) on [d_ref/d_max, d_ref/d_min].
// No node inside the prior gives -inf; a poisoned sample gives NaN.  R >= 0
// holds exactly, so R <= 0 comes only from rounding where the model has no
// power (F_k Y = 0, hence K = 0 too): lnL = 0 at every distance and the
// marginal is the prior's mass, ln L_d = 0.
__device__ __forceinline__ double dist_marginal(const DistRule& G, double d_ref, const Terms& t) {
  const double Kd = t.data, Rd = 2.0 * t.quad;
  if (t.bad || !(fabs(Kd) <= 1.0e300) || !(fabs(Rd) <= 1.0e300)) return __builtin_nan("");
  if (!(Rd > 0.0)) return 0.0;
  const double xs = Kd / Rd;
  const double sig = 1.0 / sqrt(Rd);
  const double xlo = d_ref / G.d_max, xhi = d_ref / G.d_min;
  double s = 0.0;
  for (int i = 0; i < G.n; ++i) {
    const double x = fma(G.xi[i], sig, xs);
    if (x >= xlo && x <= xhi) {
      const double r = d_ref / x;  // D at the node: p_x = D^4 / d_ref (normalised below)
      const double r2 = r * r;
      s = fma(G.w[i], r2 * r2, s);
    }
  }
  if (!(s > 0.0)) return -__builtin_inf();
  // p_x(x) = d_ref^3 x^-4 exp(ln_norm) = (d_ref / x)^4 exp(ln_norm) / d_ref
  return 0.5 * Kd * xs + log(sig) + G.ln_norm - log(d_ref) + log(s);
}

// The fixed-spacing rule over geocentric time (Eq. (ap:tfixed)): n (odd)
// times t0 + k h, composite Simpson weights, prior uniform over the window.
struct TimeRule {
  int32_t n;
  int32_t pad;
  double t0, h;
  double ln_scale;                // ln(h / T) = -ln(n - 1), T = (n - 1) h
  double lw_end, lw_odd, lw_even;  // ln(1/3), ln(4/3), ln(2/3)
};

// ln of the likelihood marginalised over geocentric time, per sample:
//   ln L_t = ln[(h / T) sum_k w_k e^{lnL(t0 + k h)}].
// The model-norm term does not depend on time, so it is evaluated once; the
// data term once per time (new stencils, the same F and Y).  The log-sum
// runs online with one exp per time.  A poisoned sample gives NaN.  The
// whole wavefront calls this together (the data term reads cooperatively).
template <class R, int KT, int L, class DataFn>
__device__ __forceinline__ double eval_tmarg_with(PDesc P, R* __restrict__ trig, int ts, double ra, double dec,
                                                  double psi, double incl, double phi, double dist,
                                                  const TimeRule& T, DataFn&& data_fn) {
  constexpr int NY = Cls<L>::NY;
  reduce_angles<R>(psi, incl, phi);
  Sky<R, KT> S;
  sky_eval<R, KT, false>(P, ra, dec, psi, 0.0, S);
  R si, ci;
  sincos_((R)incl, &si, &ci);
  R cn[NY], sn[NY];
  incl_harmonics<R, NY>(ci, si, cn, sn);
  R sf, cf;
  sincos_((R)phi, &sf, &cf);
  double wq = 0.0;
  const double quad = quad_term<R, KT, L, false>(P, trig, ts, ci, si, cf, sf, S.Fre, S.Fim, &wq);
  const double x = P->d_ref / dist;
  const double base = -x * x * quad;
  double m = -__builtin_inf(), sum = 0.0;
  bool bad = !(fabs(x) <= 1.0e300) || !(fabs(base) <= 1.0e300);
  for (int k = 0; k < T.n; ++k) {
    S.bad = false;
    sky_stencils<R, KT>(P, fma((double)k, T.h, T.t0), S);
    bad = bad || S.bad;
    __builtin_amdgcn_s_setprio(1);
    const double data = data_fn(S.row, S.sfr, S.Fre, S.Fim, cn, sn, cf, sf);
    __builtin_amdgcn_s_setprio(0);
    const double lw = (k == 0 || k == T.n - 1) ? T.lw_end : ((k & 1) ? T.lw_odd : T.lw_even);
    const double l = fma(x, data, base) + lw;
    if (l > m) {
      sum = (sum == 0.0) ? 1.0 : fma(sum, exp(m - l), 1.0);
      m = l;
    } else {
      sum += exp(l - m);
    }
  }
  if (bad || !(m == m)) return __builtin_nan("");
  return m + log(sum) + T.ln_scale;
}

// The data pass of the band-limited full-window rule (Eq. (ap:tband)): at
// fixed other parameters the exponent is x kappa(t) - x^2 quad with kappa the
// band-limited data term; this pass takes x kappa at the T.n nodes
// t0 + k h (new stencils, the same F and Y) into kap[k N + i] (when `live`)
// and returns the time-independent -x^2 quad (NaN for a poisoned sample).
// The reconstruction between the nodes and the exponential sum run in a
// separate kernel over these values.  The whole wavefront calls this
// together (the data term reads cooperatively).
template <class R, int KT, int L, class DataFn>
__device__ __forceinline__ double eval_tkappa_with(PDesc P, R* __restrict__ trig, int ts, double ra, double dec,
                                                   double psi, double incl, double phi, double dist,
                                                   const TimeRule& T, RIFT_GLOBAL double* kap, int64_t N, int64_t i,
                                                   bool live, DataFn&& data_fn) {
  constexpr int NY = Cls<L>::NY;
  reduce_angles<R>(psi, incl, phi);
  Sky<R, KT> S;
  sky_eval<R, KT, false>(P, ra, dec, psi, 0.0, S);
  R si, ci;
  sincos_((R)incl, &si, &ci);
  R cn[NY], sn[NY];
  incl_harmonics<R, NY>(ci, si, cn, sn);
  R sf, cf;
  sincos_((R)phi, &sf, &cf);
  double wq = 0.0;
  const double quad = quad_term<R, KT, L, false>(P, trig, ts, ci, si, cf, sf, S.Fre, S.Fim, &wq);
  const double x = P->d_ref / dist;
  const double base = -x * x * quad;
  bool bad = !(fabs(x) <= 1.0e300) || !(fabs(base) <= 1.0e300);
  for (int k = 0; k < T.n; ++k) {
    S.bad = false;
    sky_stencils<R, KT>(P, fma((double)k, T.h, T.t0), S);
    bad = bad || S.bad;
    __builtin_amdgcn_s_setprio(1);
    const double data = data_fn(S.row, S.sfr, S.Fre, S.Fim, cn, sn, cf, sf);
    __builtin_amdgcn_s_setprio(0);
    if (live) kap[(int64_t)k * N + i] = x * data;
  }
  return bad ? __builtin_nan("") : base;
}

// The rule over polarisation (Sec. "Angles: finite harmonic content"): at
// fixed other parameters lnL is q(u) = a + Re(c1 e^{iu}) + Re(c2 e^{2iu}) in
// u = 2 (psi' - psi) (Eq. (ap:psiexp)); with psi uniform on [0, pi),
// L_psi = (1 / 2 pi) int_0^{2 pi} e^{q(u)} du by
//   method 0: the periodic trapezoid rule on n points (the product grid),
//   method 1: Laplace's method at the dominant maximum u* (Eq. (ap:psilaplace)),
//             L_psi = e^{q(u*)} sqrt(2 pi / A) / (2 pi), A = -q''(u*), where
//             A >= 100 (relative error O(1/A) below ~1e-3); a q without
//             such a maximum (weak signal, or two peaks merging) is
//             integrated by the periodic trapezoid rule on 256 points.
constexpr double PSI_LAPLACE_MIN_A = 100.0;
constexpr int PSI_FALLBACK_POINTS = 256;
struct PsiRule {
  int32_t method;
  int32_t n;
  double ln_n;
};

// q(u) and its first two derivatives.
__device__ __forceinline__ void psi_q(double a, double c1r, double c1i, double c2r, double c2i, double su, double cu,
                                      double* q, double* d1, double* d2) {
  const double s2 = 2.0 * su * cu, c2 = cu * cu - su * su;
  const double r1 = c1r * cu - c1i * su, i1 = c1r * su + c1i * cu;  // c1 e^{iu}
  const double r2 = c2r * c2 - c2i * s2, i2 = c2r * s2 + c2i * c2;  // c2 e^{2iu}
  *q = a + r1 + r2;
  *d1 = -i1 - 2.0 * i2;
  *d2 = -r1 - 4.0 * r2;
}

// The periodic trapezoid rule for q on n points: ln[(1/n) sum_j e^{q(2 pi j/n)}].
__device__ __forceinline__ double psi_trapezoid(int n, double ln_n, double a, double c1r, double c1i, double c2r,
                                                double c2i) {
  double q, d1, d2;
  double m = -__builtin_inf(), sum = 0.0;
  for (int j = 0; j < n; ++j) {
    double su, cu;
    sincospi(2.0 * (double)j / (double)n, &su, &cu);
    psi_q(a, c1r, c1i, c2r, c2i, su, cu, &q, &d1, &d2);
    if (q > m) {
      sum = (sum == 0.0) ? 1.0 : fma(sum, exp(m - q), 1.0);
      m = q;
    } else {
      sum += exp(q - m);
    }
  }
  return m + log(sum) - ln_n;
}

// The cell partition of Eq. (ap:psicells).  With z = e^{iu}, 2 i z^2 q'(u) = 0
// is the quartic 2 c2 z^4 + c1 z^3 - conj(c1) z - 2 conj(c2) = 0 (exact leading
// zeros stripped); its roots, by the Aberth-Ehrlich iteration, that lie within
// 1e-3 of the unit circle are polished by Newton's method on q'(u) and kept
// if they settle on a zero of q'.  The sorted stationary angles cut the
// circle into cells on which q is monotone; each cell is integrated by
// 8-point Gauss-Legendre on sub-intervals of 2 sigma out to 8 sigma from its
// higher end, then of doubling length to its far end, sigma =
// min(A^{-1/2}, width / 8) from the curvature A = -q'' at that end.
struct Cx {
  double x, y;
};
__device__ __forceinline__ Cx cx_mul(Cx a, Cx b) { return Cx{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ Cx cx_add(Cx a, Cx b) { return Cx{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ Cx cx_sub(Cx a, Cx b) { return Cx{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ Cx cx_div(Cx a, Cx b) {
  const double d = b.x * b.x + b.y * b.y;
  return Cx{(a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d};
}

constexpr double PSI_GL8_X[8] = {-0.96028985649753623168, -0.79666647741362673959, -0.52553240991632898582,
                                 -0.18343464249564980494, 0.18343464249564980494,  0.52553240991632898582,
                                 0.79666647741362673959,  0.96028985649753623168};
// ln of the 8-point Gauss-Legendre weights
constexpr double PSI_GL8_LNW[8] = {-2.29037458272350180621, -1.50336299698040232187, -1.15929697855282975993,
                                   -1.01422394453275765969, -1.01422394453275765969, -1.15929697855282975993,
                                   -1.50336299698040232187, -2.29037458272350180621};

__device__ __forceinline__ int psi_stationary(double c1r, double c1i, double c2r, double c2i, double* st) {
  // coefficients, highest degree first: 2 c2, c1, 0, -conj(c1), -2 conj(c2)
  Cx co[5] = {Cx{2.0 * c2r, 2.0 * c2i}, Cx{c1r, c1i}, Cx{0.0, 0.0}, Cx{-c1r, c1i}, Cx{-2.0 * c2r, 2.0 * c2i}};
  int lead = 0;
  while (lead < 4 && co[lead].x == 0.0 && co[lead].y == 0.0) ++lead;
  const int D = 4 - lead;  // degree after stripping exact leading zeros
  if (D < 1) return 0;
  Cx z[4];
  for (int k = 0; k < D; ++k) {
    double sk, ck;
    sincos(1.5707963267948966 * k + 0.4, &sk, &ck);
    z[k] = Cx{ck, sk};
  }
  for (int it = 0; it < 60; ++it) {
    double moved = 0.0;
    for (int k = 0; k < D; ++k) {
      Cx p = co[lead], dp = Cx{0.0, 0.0};
      for (int j = lead + 1; j <= 4; ++j) {
        dp = cx_add(cx_mul(dp, z[k]), p);
        p = cx_add(cx_mul(p, z[k]), co[j]);
      }
      if (p.x == 0.0 && p.y == 0.0) continue;
      const Cx ratio = cx_div(p, dp);
      Cx sum{0.0, 0.0};
      for (int j = 0; j < D; ++j)
        if (j != k) sum = cx_add(sum, cx_div(Cx{1.0, 0.0}, cx_sub(z[k], z[j])));
      const Cx w = cx_div(ratio, cx_sub(Cx{1.0, 0.0}, cx_mul(ratio, sum)));
      z[k] = cx_sub(z[k], w);
      moved = fmax(moved, fabs(w.x) + fabs(w.y));
    }
    if (!(moved > 1e-16)) break;
  }
  const double scale = sqrt(c1r * c1r + c1i * c1i) + 2.0 * sqrt(c2r * c2r + c2i * c2i);
  int n = 0;
  for (int k = 0; k < D; ++k) {
    const double r = sqrt(z[k].x * z[k].x + z[k].y * z[k].y);
    if (!(fabs(r - 1.0) <= 1e-3)) continue;
    double u = atan2(z[k].y, z[k].x);
    double q, d1, d2;
    for (int it = 0; it < 30; ++it) {
      double su, cu;
      sincos(u, &su, &cu);
      psi_q(0.0, c1r, c1i, c2r, c2i, su, cu, &q, &d1, &d2);
      if (d2 == 0.0) break;
      const double step = d1 / d2;
      u -= step;
      if (fabs(step) < 1e-15) break;
    }
    double su, cu;
    sincos(u, &su, &cu);
    psi_q(0.0, c1r, c1i, c2r, c2i, su, cu, &q, &d1, &d2);
    if (!(fabs(d1) <= 1e-9 * fmax(scale, 1e-300))) continue;
    u = fmod(u, 6.283185307179586477);
    if (u < 0.0) u += 6.283185307179586477;
    st[n++] = u;
  }
  // sort, and drop repeats (two roots settling on one point)
  for (int a = 1; a < n; ++a)
    for (int b = a; b > 0 && st[b] < st[b - 1]; --b) {
      const double t = st[b];
      st[b] = st[b - 1];
      st[b - 1] = t;
    }
  int m = 0;
  for (int a = 0; a < n; ++a)
    if (m == 0 || st[a] - st[m - 1] > 1e-12) st[m++] = st[a];
  return m;
}

__device__ __forceinline__ double psi_cells(double a, double c1r, double c1i, double c2r, double c2i) {
  double st[4];
  const int ns = psi_stationary(c1r, c1i, c2r, c2i, st);
  const int nc = ns < 2 ? 1 : ns;
  double m = -__builtin_inf(), sum = 0.0;
  for (int c = 0; c < nc; ++c) {
    const double lo = ns < 2 ? 0.0 : st[c];
    const double hi = ns < 2 ? 6.283185307179586477 : (c + 1 < ns ? st[c + 1] : st[0] + 6.283185307179586477);
    const double width = hi - lo;
    double ql, qh, d1, d2l, d2h, s, cc;
    sincos(lo, &s, &cc);
    psi_q(a, c1r, c1i, c2r, c2i, s, cc, &ql, &d1, &d2l);
    sincos(hi, &s, &cc);
    psi_q(a, c1r, c1i, c2r, c2i, s, cc, &qh, &d1, &d2h);
    const bool top_lo = ql >= qh;
    const double A = -(top_lo ? d2l : d2h);
    const double sigma = A > 0.0 ? fmin(1.0 / sqrt(A), width / 8.0) : width / 8.0;
    double d0 = 0.0;
    for (int j = 1; d0 < width; ++j) {
      const double d1e = fmin(width, j <= 4 ? 2.0 * sigma * j : 2.0 * d0);
      const double h = d1e - d0;
      const double lnh = log(0.5 * h);
      for (int g = 0; g < 8; ++g) {
        const double dist = d0 + 0.5 * h + 0.5 * h * PSI_GL8_X[g];
        const double u = top_lo ? lo + dist : hi - dist;
        double su, cu, q, dd1, dd2;
        sincos(u, &su, &cu);
        psi_q(a, c1r, c1i, c2r, c2i, su, cu, &q, &dd1, &dd2);
        const double l = q + lnh + PSI_GL8_LNW[g];
        const double dl = l - m;
        const double e = exp(-fabs(dl));
        const bool up = dl > 0.0;
        sum = up ? fma(sum, e, 1.0) : sum + e;
        m = up ? l : m;
      }
      d0 = d1e;
    }
  }
  return m + log(sum) - 1.8378770664093454836;  // ln(2 pi)
}

// ln L_psi from the coefficients of q (see PsiRule).  Laplace: the best of 32
// equally spaced points, then Newton steps on q' = 0 (the maximum is then the
// dominant one unless another lies within the grid's resolution of it).
__device__ __forceinline__ double psi_marginal(const PsiRule& G, double a, double c1r, double c1i, double c2r,
                                               double c2i) {
  double q, d1, d2;
  if (G.method == 0) return psi_trapezoid(G.n, G.ln_n, a, c1r, c1i, c2r, c2i);
  if (G.method == 2) return psi_cells(a, c1r, c1i, c2r, c2i);
  double best = -__builtin_inf(), ub = 0.0;
  for (int j = 0; j < 32; ++j) {
    double su, cu;
    sincospi((double)j / 16.0, &su, &cu);
    psi_q(a, c1r, c1i, c2r, c2i, su, cu, &q, &d1, &d2);
    if (q > best) {
      best = q;
      ub = 3.14159265358979323846 * (double)j / 16.0;
    }
  }
  double u = ub;
  for (int it = 0; it < 8; ++it) {
    double su, cu;
    sincos(u, &su, &cu);
    psi_q(a, c1r, c1i, c2r, c2i, su, cu, &q, &d1, &d2);
    if (!(d2 < 0.0)) break;
    u -= d1 / d2;
  }
  double su, cu;
  sincos(u, &su, &cu);
  psi_q(a, c1r, c1i, c2r, c2i, su, cu, &q, &d1, &d2);
  const double A = -d2;
  if (!(A >= PSI_LAPLACE_MIN_A))
    return psi_trapezoid(PSI_FALLBACK_POINTS, 5.5451774444795623, a, c1r, c1i, c2r, c2i);  // ln 256
  return q - 0.5 * log(2.0 * 3.14159265358979323846 * A);
}

// ln of the likelihood marginalised over polarisation, per sample: the data
// term as the complex W = sum_k conj(F_k) Z_k (one gather), the model-norm
// term as A0 = sum_k |F_k|^2 a_k / 4 and B = sum_k F_k^2 b_k / 4 (one
// contraction), then, with F_k(psi + u/2) = e^{-iu} F_k(psi),
//   q(u) = x Re(e^{iu} W) - x^2 [A0 + Re(e^{-2iu} B)]:
//   a = -x^2 A0, c1 = x W, c2 = -x^2 conj(B).
template <class R, int KT, int L, class DataFn>
__device__ __forceinline__ double eval_pmarg_with(PDesc P, R* __restrict__ trig, int ts, double ra, double dec,
                                                  double psi, double incl, double phi, double tref, double dist,
                                                  const PsiRule& G, DataFn&& data_fn) {
  constexpr int NY = Cls<L>::NY;
  reduce_angles<R>(psi, incl, phi);
  Sky<R, KT> S;
  sky_eval<R, KT, true>(P, ra, dec, psi, tref, S);
  R si, ci;
  sincos_((R)incl, &si, &ci);
  R cn[NY], sn[NY];
  incl_harmonics<R, NY>(ci, si, cn, sn);
  R sf, cf;
  sincos_((R)phi, &sf, &cf);
  double wim = 0.0;
  __builtin_amdgcn_s_setprio(1);
  const double wre = data_fn(S.row, S.sfr, S.Fre, S.Fim, cn, sn, cf, sf, &wim);
  __builtin_amdgcn_s_setprio(0);
  R acc[3 * KT];
  norm_contract<R, KT, L>(P, trig, ts, ci, si, cf, sf, acc);
  double A0 = 0.0, Bre = 0.0, Bim = 0.0;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const R f2 = S.Fre[k] * S.Fre[k] + S.Fim[k] * S.Fim[k];
    const R g2r = S.Fre[k] * S.Fre[k] - S.Fim[k] * S.Fim[k];
    const R g2i = 2 * S.Fre[k] * S.Fim[k];
    A0 += (double)(f2 * acc[3 * k]);
    Bre += (double)(g2r * acc[3 * k + 1]) + (double)(g2i * acc[3 * k + 2]);
    Bim += (double)(g2i * acc[3 * k + 1]) - (double)(g2r * acc[3 * k + 2]);
  }
  const double x = P->d_ref / dist;
  if (S.bad || !(fabs(x) <= 1.0e300) || !(fabs(wre) <= 1.0e300) || !(fabs(wim) <= 1.0e300) ||
      !(fabs(A0) <= 1.0e300) || !(fabs(Bre) + fabs(Bim) <= 1.0e300))
    return __builtin_nan("");
  const double x2 = x * x;
  return psi_marginal(G, -x2 * A0, x * wre, x * wim, -x2 * Bre, x2 * Bim);
}

// The data pass of the joint phiref / psi marginal by exact reconstruction
// (ERAI, Eqs. (ap:angleharm), (ap:nyquist)).  At fixed sky, inclination,
// time and distance, lnL in the offsets (alpha, u = 2 (psi' - psi)) is
//   q(alpha, u) = a(alpha) + Re(c1(alpha) e^{iu}) + Re(c2(alpha) e^{2iu}),
// c1 = x W (the complex data term, degree m_max in alpha), a = -x^2 A0 and
// c2 = -x^2 conj(B) (the model norm, degree 2 m_max), as in the polarisation
// marginal.  This pass samples c1 at the G.nd = 2 m_max + 1 angles
// phi + 2 pi j / nd (one gather each, the same stencils) and (a, c2) at the
// G.nq = 4 m_max + 1 angles phi + 2 pi j / nq (one contraction each), which
// determine them exactly, into out rows [2 j], [2 j + 1] (c1) and
// [2 nd + 3 j + 0 .. 2] (a, c2) of stride N (when `live`).  Returns whether
// the sample is poisoned.  The whole wavefront calls this together.
struct AngleRule {
  int32_t nd, nq;
  double dd, dq;  // 2 pi / nd, 2 pi / nq
};

template <class R, int KT, int L, class DataFn>
__device__ __forceinline__ bool eval_erai_with(PDesc P, R* __restrict__ trig, int ts, double ra, double dec,
                                               double psi, double incl, double phi, double tref, double dist,
                                               const AngleRule& G, RIFT_GLOBAL double* out, int64_t N, int64_t i,
                                               bool live, DataFn&& data_fn) {
  constexpr int NY = Cls<L>::NY;
  reduce_angles<R>(psi, incl, phi);
  Sky<R, KT> S;
  sky_eval<R, KT, true>(P, ra, dec, psi, tref, S);
  R si, ci;
  sincos_((R)incl, &si, &ci);
  R cn[NY], sn[NY];
  incl_harmonics<R, NY>(ci, si, cn, sn);
  const double x = P->d_ref / dist;
  const double x2 = x * x;
  bool bad = S.bad || !(fabs(x) <= 1.0e300);
  for (int j = 0; j < G.nd; ++j) {
    R sf, cf;
    sincos_((R)fma((double)j, G.dd, phi), &sf, &cf);
    double wim = 0.0;
    __builtin_amdgcn_s_setprio(1);
    const double wre = data_fn(S.row, S.sfr, S.Fre, S.Fim, cn, sn, cf, sf, &wim);
    __builtin_amdgcn_s_setprio(0);
    bad = bad || !(fabs(wre) <= 1.0e300) || !(fabs(wim) <= 1.0e300);
    if (live) {
      out[(int64_t)(2 * j) * N + i] = x * wre;
      out[(int64_t)(2 * j + 1) * N + i] = x * wim;
    }
  }
  const int r0 = 2 * G.nd;
  for (int j = 0; j < G.nq; ++j) {
    R sf, cf;
    sincos_((R)fma((double)j, G.dq, phi), &sf, &cf);
    R acc[3 * KT];
    norm_contract<R, KT, L>(P, trig, ts, ci, si, cf, sf, acc);
    double A0 = 0.0, Bre = 0.0, Bim = 0.0;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      const R f2 = S.Fre[k] * S.Fre[k] + S.Fim[k] * S.Fim[k];
      const R g2r = S.Fre[k] * S.Fre[k] - S.Fim[k] * S.Fim[k];
      const R g2i = 2 * S.Fre[k] * S.Fim[k];
      A0 += (double)(f2 * acc[3 * k]);
      Bre += (double)(g2r * acc[3 * k + 1]) + (double)(g2i * acc[3 * k + 2]);
      Bim += (double)(g2i * acc[3 * k + 1]) - (double)(g2r * acc[3 * k + 2]);
    }
    bad = bad || !(fabs(A0) <= 1.0e300) || !(fabs(Bre) + fabs(Bim) <= 1.0e300);
    if (live) {
      out[(int64_t)(r0 + 3 * j) * N + i] = -x2 * A0;
      out[(int64_t)(r0 + 3 * j + 1) * N + i] = -x2 * Bre;
      out[(int64_t)(r0 + 3 * j + 2) * N + i] = x2 * Bim;
    }
  }
  return bad;
}

// Everything per sample up to the distance: the terms.  R is the arithmetic
// type of the bulk (FP64 or FP32); the sky frame, delays and the final
// combination are always FP64.  The data term comes from
// data_fn(row, sfr, Fre, Fim, cn, sn, cf, sf).
template <class R, int KT, int L, bool BOUND, class DataFn>
__device__ __forceinline__ Terms eval_terms_with(PDesc P, R* __restrict__ trig, int ts, double ra, double dec,
                                                 double psi, double incl, double phi, double tref,
                                                 DataFn&& data_fn) {
  constexpr int NY = Cls<L>::NY;
  reduce_angles<R>(psi, incl, phi);
  Sky<R, KT> S;
  sky_eval<R, KT, true>(P, ra, dec, psi, tref, S);
  R si, ci;
  sincos_((R)incl, &si, &ci);
  R cn[NY], sn[NY];
  incl_harmonics<R, NY>(ci, si, cn, sn);
  R sf, cf;
  sincos_((R)phi, &sf, &cf);
  __builtin_amdgcn_s_setprio(1);
  const double data = data_fn(S.row, S.sfr, S.Fre, S.Fim, cn, sn, cf, sf);
  __builtin_amdgcn_s_setprio(0);
  Terms t;
  t.wq = 0.0;
  t.data = data;
  t.quad = quad_term<R, KT, L, BOUND>(P, trig, ts, ci, si, cf, sf, S.Fre, S.Fim, &t.wq);
  t.bad = S.bad;
  return t;
}

template <class R, int KT, int L, bool BOUND, class DataFn>
__device__ __forceinline__ Eval eval_sample_with(PDesc P, R* __restrict__ trig, int ts, double ra,
                                                 double dec, double psi, double incl, double phi,
                                                 double tref, double dist, DataFn&& data_fn) {
  const Terms t = eval_terms_with<R, KT, L, BOUND>(P, trig, ts, ra, dec, psi, incl, phi, tref, data_fn);
  return combine<BOUND>(P, dist, t.data, t.quad, t.wq, t.bad);
}

// `stage` is this wavefront's STAGE_WAVE bytes of LDS; the whole wavefront
// must call these together.
template <class R, int KT, int L>
__device__ __forceinline__ Terms eval_terms(PDesc P, R* __restrict__ trig, int ts, RIFT_LDS unsigned char* stage,
                                           double ra, double dec, double psi, double incl, double phi,
                                           double tref) {
  return eval_terms_with<R, KT, L, false>(
      P, trig, ts, ra, dec, psi, incl, phi, tref,
      [&](const int32_t* row, const R* sfr, const R* Fre, const R* Fim, const R* cn, const R* sn, R cf,
          R sf) { return data_direct<R, KT, L>(P, stage, row, sfr, Fre, Fim, cn, sn, cf, sf); });
}
template <class R, int KT, int L>
__device__ __forceinline__ double eval_pmarg(PDesc P, R* __restrict__ trig, int ts, RIFT_LDS unsigned char* stage,
                                            double ra, double dec, double psi, double incl, double phi, double tref,
                                            double dist, const PsiRule& G) {
  return eval_pmarg_with<R, KT, L>(
      P, trig, ts, ra, dec, psi, incl, phi, tref, dist, G,
      [&](const int32_t* row, const R* sfr, const R* Fre, const R* Fim, const R* cn, const R* sn, R cf, R sf,
          double* im) { return data_direct<R, KT, L, true>(P, stage, row, sfr, Fre, Fim, cn, sn, cf, sf, im); });
}
template <class R, int KT, int L>
__device__ __forceinline__ double eval_tmarg(PDesc P, R* __restrict__ trig, int ts, RIFT_LDS unsigned char* stage,
                                            double ra, double dec, double psi, double incl, double phi, double dist,
                                            const TimeRule& T) {
  return eval_tmarg_with<R, KT, L>(
      P, trig, ts, ra, dec, psi, incl, phi, dist, T,
      [&](const int32_t* row, const R* sfr, const R* Fre, const R* Fim, const R* cn, const R* sn, R cf,
          R sf) { return data_direct<R, KT, L>(P, stage, row, sfr, Fre, Fim, cn, sn, cf, sf); });
}
template <class R, int KT, int L>
__device__ __forceinline__ bool eval_erai(PDesc P, R* __restrict__ trig, int ts, RIFT_LDS unsigned char* stage,
                                         double ra, double dec, double psi, double incl, double phi, double tref,
                                         double dist, const AngleRule& G, RIFT_GLOBAL double* out, int64_t N,
                                         int64_t i, bool live) {
  return eval_erai_with<R, KT, L>(
      P, trig, ts, ra, dec, psi, incl, phi, tref, dist, G, out, N, i, live,
      [&](const int32_t* row, const R* sfr, const R* Fre, const R* Fim, const R* cn, const R* sn, R cf, R sf,
          double* im) { return data_direct<R, KT, L, true>(P, stage, row, sfr, Fre, Fim, cn, sn, cf, sf, im); });
}
template <class R, int KT, int L>
__device__ __forceinline__ double eval_tkappa(PDesc P, R* __restrict__ trig, int ts, RIFT_LDS unsigned char* stage,
                                             double ra, double dec, double psi, double incl, double phi, double dist,
                                             const TimeRule& T, RIFT_GLOBAL double* kap, int64_t N, int64_t i,
                                             bool live) {
  return eval_tkappa_with<R, KT, L>(
      P, trig, ts, ra, dec, psi, incl, phi, dist, T, kap, N, i, live,
      [&](const int32_t* row, const R* sfr, const R* Fre, const R* Fim, const R* cn, const R* sn, R cf,
          R sf) { return data_direct<R, KT, L>(P, stage, row, sfr, Fre, Fim, cn, sn, cf, sf); });
}
template <class R, int KT, int L, bool BOUND>
__device__ __forceinline__ Eval eval_sample(PDesc P, R* __restrict__ trig, int ts,
                                            RIFT_LDS unsigned char* stage, double ra, double dec, double psi,
                                            double incl, double phi, double tref, double dist) {
  return eval_sample_with<R, KT, L, BOUND>(
      P, trig, ts, ra, dec, psi, incl, phi, tref, dist,
      [&](const int32_t* row, const R* sfr, const R* Fre, const R* Fim, const R* cn, const R* sn, R cf,
          R sf) { return data_direct<R, KT, L>(P, stage, row, sfr, Fre, Fim, cn, sn, cf, sf); });
}

// ---------------------------------------------------------------------------
// log-sum-exp pairs (max, sum exp(l - max)); NaN propagates through the sum.
// ---------------------------------------------------------------------------
struct MS {
  double m, s;
};
__device__ __forceinline__ MS ms_of(double l) {
  MS r;
  if (l != l) {
    r.m = -__builtin_inf();
    r.s = __builtin_nan("");
  } else if (l == -__builtin_inf()) {
    r.m = l;
    r.s = 0.0;
  } else {
    r.m = l;
    r.s = 1.0;
  }
  return r;
}
// Add one sample's l to (max, sum): one exp instead of two.
__device__ __forceinline__ MS ms_push(MS a, double l) {
  if (l != l) {  // NaN poisons the sum
    a.s = __builtin_nan("");
    return a;
  }
  if (l == -__builtin_inf()) return a;
  if (l > a.m) {
    a.s = (a.s == 0.0) ? 1.0 : a.s * exp(a.m - l) + 1.0;
    a.m = l;
  } else {
    a.s += exp(l - a.m);
  }
  return a;
}
__device__ __forceinline__ MS ms_combine(MS a, MS b) {
  MS r;
  r.m = fmax(a.m, b.m);
  const double ta = (a.s == 0.0) ? 0.0 : a.s * exp(a.m - r.m);
  const double tb = (b.s == 0.0) ? 0.0 : b.s * exp(b.m - r.m);
  r.s = ta + tb;
  return r;
}
__device__ __forceinline__ MS ms_wave(MS v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    MS o;
    o.m = __shfl_xor(v.m, off);
    o.s = __shfl_xor(v.s, off);
    v = ms_combine(v, o);
  }
  return v;
}
// Block-wide reduction in a fixed order (deterministic).  `sh` holds one MS
// per wave.
__device__ __forceinline__ MS ms_block(MS v, MS* sh) {
  v = ms_wave(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  MS r = sh[0];
  for (int w = 1; w < nw; ++w) r = ms_combine(r, sh[w]);
  return r;
}

__device__ __forceinline__ double dmax_wave(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ double dsum_wave(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

}  // namespace rift
