// The composite-index likelihood of the generalised detector response
// (Sec. "A generalized detector response"): the mode index widens to
// A = (a, lm) and the static antenna factor F_k to a coefficient C~^k_a per
// composite term a, Eq. (slowrot:lnL:Decomposed):
//
//   lnL = x Re sum_k sum_a sum_lm conj(C~^k_a Y_lm) Q_{k,a lm}(t_k)
//       - x^2/4 sum_k [ c_k^H U_k c_k + Re(c_k^T V_k c_k) ],   c_{k,(a,lm)} = C~^k_a Y_lm.
//
// Two responses:
//   rotation (Path A): a <-> sidereal harmonic n = a - 2, n = -2..2.  F_k over
//     the Greenwich hour angle g is a degree-2 trigonometric polynomial,
//     F_k(g) = sum_n A_n e^{i n g} (Eq. (slowrot:Fharm)); A_n is the exact
//     five-point transform of F_k at g_j = 2 pi j / 5 for the sample's dec and
//     psi.  C~_n = A_n e^{i n g(t_ref)} e^{i n W (t_k - t_ref)} (the post-phase
//     of Eq. (slowrot:postphase), the bank's modulation referenced to the
//     template's own time), g(t) = gmst + W t - ra; the delay is held at the
//     arrival time t_k of the sky frame at t_ref.
//   arms (Path D): a <-> order p of the arm-projection expansion,
//     b_p = 1/2 [ (x.N)^p e:xx - (y.N)^p e:yy ] (Eq. (fsize:bp)) with
//     e:aa = (X.a + i Y.a)^2 for the complex polarisation tensor e = e+ + i ex;
//     static sky frame.
//
// One lane evaluates one sample, in FP64.  Per detector the lane's C~ goes to
// LDS; the mode harmonics Y stay in registers (modes sorted by m, the phase
// walked upward; the kernel is compiled for mode capacities 5, 12 and 25 so
// that short mode sets keep few registers).  The quadratic term runs over
// pairs a <= a' of composite terms, G_aa' = Y^H U_aa' Y and H_aa' = Y^T V_aa' Y,
// and uses the symmetries G_a'a = conj(G_aa') (U Hermitian) and H_a'a = H_aa'
// (V symmetric).  A set-up kernel packs U and V per call into the order the
// contraction walks, [k][pair][i][j] (Re U, Im U, Re V, Im V) with internal
// mode indices and row stride equal to the capacity, so that the uniform
// entries reach the lanes through the scalar path at constant offsets.
//
// For the longer mode sets (l <= 3 with 10 or more modes, l <= 4 with 13 or
// more) the pair forms take the harmonic form of the static path instead:
// each of Re G, Im G, Re H, Im H of a block is a trigonometric polynomial in
// (incl, phiref) of degree 2L in each, with the parity that d_i d_j has in
// incl (that of m_i - m_j, equal to that of m_i + m_j), so it lies in the
// static path's real basis of class L (145 functions at L = 4).  A set-up
// kernel projects every block onto that basis per call; a lane then sums
// 4 B uniform coefficients against basis values built from cos(n incl),
// sin(n incl), cos(q phiref), sin(q phiref), instead of 4 M^2 entries
// (580 against 1764 at 21 modes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/rift_ile.h"
#include "ile_device.h"
#include "ile_host.h"

namespace rift {
namespace {

constexpr int WIDE_ARMS_MAX_TERMS = 8;
constexpr int WIDE_BLOCK = 256;     // lanes per block up to 12 terms
constexpr int WIDE_BLOCK_21 = 128;  // up to 21 terms: the coefficient columns in 43 KB of LDS
constexpr int WIDE_BASIS_BLOCK = 512;  // threads of the harmonic set-up: one per grid point

struct WideDesc {
  int32_t K, M, n_t, n_a, response, npairs;
  int32_t hb, hb_pad;         // class L of the harmonic form of the pair forms, 0: the entries
  double t0, inv_dt, gmst, omega, d_ref;
  double dten[KMAX][6];      // D00, D11, D22, 2 D01, 2 D02, 2 D12
  double rpos[KMAX][3];      // light-seconds
  double arms[KMAX][2][3];   // arm unit vectors
  int32_t perm[MMAX];        // caller's index of internal mode i (modes sorted by m)
  int32_t m[MMAX];
  int32_t odd[MMAX];
  double ycoef[MMAX][LMAXC + 1];
  const double* Q;           // caller's [K][n_a][M][n_t] complex
  const double* UV;          // packed [K][pair][MC][MC][4], or [K][pair][B][4] coefficients (hb > 0)
};
static_assert(sizeof(WideDesc) <= 3584, "the description travels as a kernel argument");

// Complex response D : (e+ + i ex) of the six-value tensor d at axes X, Y.
__device__ __forceinline__ C2<double> response6(const double* d, const double* X, const double* Y) {
  const double ep[6] = {X[0] * X[0] - Y[0] * Y[0], X[1] * X[1] - Y[1] * Y[1], X[2] * X[2] - Y[2] * Y[2],
                        X[0] * X[1] - Y[0] * Y[1], X[0] * X[2] - Y[0] * Y[2], X[1] * X[2] - Y[1] * Y[2]};
  const double ex[6] = {2 * X[0] * Y[0], 2 * X[1] * Y[1], 2 * X[2] * Y[2],
                        X[0] * Y[1] + Y[0] * X[1], X[0] * Y[2] + Y[0] * X[2], X[1] * Y[2] + Y[1] * X[2]};
  C2<double> f;
  f.x = f.y = 0.0;
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    f.x += d[a] * ep[a];
    f.y += d[a] * ex[a];
  }
  return f;
}

// Polarisation axes X, Y at hour angle g for dec, psi (the static sky frame).
__device__ __forceinline__ void axes(double sg, double cg, double sd, double cd, double sp, double cp, double* X,
                                     double* Y, double* N) {
  const double ea[3] = {sg, cg, 0.0};
  const double ed[3] = {-sd * cg, sd * sg, cd};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    X[i] = -cp * ea[i] + sp * ed[i];
    Y[i] = sp * ea[i] + cp * ed[i];
  }
  N[0] = cd * cg;
  N[1] = -cd * sg;
  N[2] = sd;
}

// Packs U and V of every detector into [k][pair][i][j][4] = (Re U, Im U,
// Re V, Im V) of block (a, b), pair = the index of a <= b in row order, with
// internal mode indices i, j < MC (entries past M are zero).
template <int MC>
__global__ void k_wide_pack(WideDesc D, const double* __restrict__ U, const double* __restrict__ V,
                            double* __restrict__ out) {
  const int64_t per_det = (int64_t)D.npairs * MC * MC;
  const int64_t total = (int64_t)D.K * per_det;
  const int A = D.n_a * D.M;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / per_det);
    int r = (int)(e - (int64_t)k * per_det);
    const int pr = r / (MC * MC);
    r -= pr * MC * MC;
    const int i = r / MC, j = r - (r / MC) * MC;
    int a = 0, rem = pr;
    while (rem >= D.n_a - a) {
      rem -= D.n_a - a;
      ++a;
    }
    const int b = a + rem;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < D.M && j < D.M) {
      const int64_t o = 2 * (((int64_t)k * A + a * D.M + D.perm[i]) * A + b * D.M + D.perm[j]);
      v[0] = U[o];
      v[1] = U[o + 1];
      v[2] = V[o];
      v[3] = V[o + 1];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) out[4 * e + c] = v[c];
  }
}

// G_ab = Y^H U_ab Y and H_ab = Y^T V_ab Y of one packed block, accumulated
// into g[4] = (Re G, Im G, Re H, Im H): the rows II in turn (a template
// recursion, so that every mode index and table offset is a compile-time
// constant and Y stays in registers), each row's columns in an unrolled loop.
template <int II, int MC>
struct PairForms {
  static __device__ __forceinline__ void run(const RIFT_CONST double* blk, int M, const double* yr,
                                             const double* yi, double* g) {
    if constexpr (II < MC) {
      if (II < M) {
        double tr = 0.0, ti = 0.0, vr = 0.0, vi = 0.0;  // (U Y)_II, (V Y)_II
#pragma unroll
        for (int jj = 0; jj < MC; ++jj) {
          if (jj < M) {
            const RIFT_CONST double* e = blk + 4 * (II * MC + jj);
            const double ur = e[0], ui = e[1], wr = e[2], wi = e[3];
            tr += ur * yr[jj] - ui * yi[jj];
            ti += ur * yi[jj] + ui * yr[jj];
            vr += wr * yr[jj] - wi * yi[jj];
            vi += wr * yi[jj] + wi * yr[jj];
          }
        }
        // conj(Y_II) (U Y)_II and Y_II (V Y)_II
        g[0] += yr[II] * tr + yi[II] * ti;
        g[1] += yr[II] * ti - yi[II] * tr;
        g[2] += yr[II] * vr - yi[II] * vi;
        g[3] += yr[II] * vi + yi[II] * vr;
        PairForms<II + 1, MC>::run(blk, M, yr, yi, g);
      }
    }
  }
};

// The entry form for the 5-mode capacity with the coefficients streamed
// through double-buffered 128-byte scalar chunks (four entries each; the
// static path's prefetch): the whole MC x MC block is read, the entries past
// M being zero in the pack and Y zero there, so every index is a template
// constant.  Row i's (U Y)_i and (V Y)_i accumulate across chunk boundaries.
template <int MC>
struct PairFormsP {
  static constexpr int NC = 4 * MC * MC;
  static constexpr int CH = 16;
  static constexpr int NCH = (NC + CH - 1) / CH;
  struct Row {
    double tr, ti, vr, vi;
  };
  template <int E>
  static __device__ __forceinline__ void entry(const double* e, const double* yr, const double* yi, double* g,
                                               Row& R) {
    if constexpr (E < MC * MC) {
      constexpr int i = E / MC, j = E % MC;
      if constexpr (j == 0) R.tr = R.ti = R.vr = R.vi = 0.0;
      R.tr += e[0] * yr[j] - e[1] * yi[j];
      R.ti += e[0] * yi[j] + e[1] * yr[j];
      R.vr += e[2] * yr[j] - e[3] * yi[j];
      R.vi += e[2] * yi[j] + e[3] * yr[j];
      if constexpr (j == MC - 1) {
        g[0] += yr[i] * R.tr + yi[i] * R.ti;
        g[1] += yr[i] * R.ti - yi[i] * R.tr;
        g[2] += yr[i] * R.vr - yi[i] * R.vi;
        g[3] += yr[i] * R.vi + yi[i] * R.vr;
      }
    }
  }
  template <int C>
  static __device__ __forceinline__ void ld(double (&buf)[CH], const RIFT_CONST double* c) {
    const RIFT_CONST double* p = c + C * CH;
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (C * CH + i < NC) buf[i] = p[i];
  }
  template <int C>
  static __device__ __forceinline__ void wait(const double (&buf)[CH]) {
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (C * CH + i < NC) pin_s(buf[i]);
  }
  template <int C>
  static __device__ __forceinline__ void step(const RIFT_CONST double* c, double (&cur)[CH], double (&nxt)[CH],
                                              const double* yr, const double* yi, double* g, Row& R) {
    if constexpr (C < NCH) {
      wait<C>(cur);
      if constexpr (C + 1 < NCH) ld<C + 1>(nxt, c);
      entry<4 * C>(cur, yr, yi, g, R);
      entry<4 * C + 1>(cur + 4, yr, yi, g, R);
      entry<4 * C + 2>(cur + 8, yr, yi, g, R);
      entry<4 * C + 3>(cur + 12, yr, yi, g, R);
#pragma unroll
      for (int k = 0; k < 4; ++k) pin(g[k]);
      pin(R.tr);
      pin(R.ti);
      pin(R.vr);
      pin(R.vi);
      step<C + 1>(c, nxt, cur, yr, yi, g, R);
    }
  }
  static __device__ __forceinline__ void run(const RIFT_CONST double* c, const double* yr, const double* yi,
                                             double* g) {
    Row R;
    R.tr = R.ti = R.vr = R.vi = 0.0;
    double bA[CH], bB[CH];
    ld<0>(bA, c);
    step<0>(c, bA, bB, yr, yi, g, R);
  }
};

// The same four forms of one block in the harmonic basis of class L, summed
// per harmonic q in phi: the rows of one q are consecutive and q increases
// along them (basis_row), so
// g[c] += cos(q phi) sum_n C[(n, cos)][c] T_n(incl)
//       + sin(q phi) sum_n C[(n, sin)][c] T_n(incl),
// T_n = cos(n incl) for even q and sin(n incl) for odd q (q = 0: the first
// sum alone), with e^{i q phi} advanced by one factor e^{i phi} per q.
// Every row's kind and degrees are template constants; no product of basis
// values is formed, so only the cos(n incl), sin(n incl) tables stay live
// across the pairs.
template <int L>
struct HarmForms {
  static constexpr int B = Cls<L>::B;
  static constexpr int NC = 4 * B;              // coefficients of one block
  static constexpr int CH = 16;                 // one 128-byte chunk: four rows
  static constexpr int NCH = (NC + CH - 1) / CH;
  struct Run {
    double pc[4], ps[4];  // the two sums of the current q
    double er, ei;        // e^{i q phi}
  };
  template <int J>
  static __device__ __forceinline__ void term(const double* e, const double* cn, const double* sn, double cf,
                                              double sf, double* g, Run& R) {
    if constexpr (J < B) {
      constexpr int rb = basis_row<L>(J);
      constexpr int kind = rb & 15, nn = (rb >> 4) & 255, q = rb >> 12;
      constexpr bool last = (J + 1 == B) || ((basis_row<L>(J + 1) >> 12) != q);
      const double tn = (kind == 3 || kind == 4) ? sn[nn] : cn[nn];
      if constexpr (kind == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) g[k] = fma(e[k], tn, g[k]);
      } else {
        double* acc = (kind == 1 || kind == 3) ? R.pc : R.ps;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = fma(e[k], tn, acc[k]);
        if constexpr (last) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            g[k] = fma(R.pc[k], R.er, fma(R.ps[k], R.ei, g[k]));
            R.pc[k] = 0.0;
            R.ps[k] = 0.0;
          }
          const double nr = R.er * cf - R.ei * sf, ni = R.er * sf + R.ei * cf;
          R.er = nr;
          R.ei = ni;
        }
      }
    }
  }
  // The uniform coefficients stream through SGPRs in 128-byte chunks, each
  // chunk prefetched while the previous one is used (the static path's
  // scheme): the wait for a chunk comes before the next chunk is issued, and
  // the accumulators are pinned after each chunk's FMAs so that those FMAs
  // stay ahead of the next wait.
  template <int C>
  static __device__ __forceinline__ void ld(double (&buf)[CH], const RIFT_CONST double* c) {
    const RIFT_CONST double* p = c + C * CH;
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (C * CH + i < NC) buf[i] = p[i];
  }
  template <int C>
  static __device__ __forceinline__ void wait(const double (&buf)[CH]) {
#pragma unroll
    for (int i = 0; i < CH; ++i)
      if (C * CH + i < NC) pin_s(buf[i]);
  }
  template <int C>
  static __device__ __forceinline__ void step(const RIFT_CONST double* c, double (&cur)[CH], double (&nxt)[CH],
                                              const double* cn, const double* sn, double cf, double sf, double* g,
                                              Run& R) {
    if constexpr (C < NCH) {
      wait<C>(cur);
      if constexpr (C + 1 < NCH) ld<C + 1>(nxt, c);
      term<4 * C>(cur, cn, sn, cf, sf, g, R);
      term<4 * C + 1>(cur + 4, cn, sn, cf, sf, g, R);
      term<4 * C + 2>(cur + 8, cn, sn, cf, sf, g, R);
      term<4 * C + 3>(cur + 12, cn, sn, cf, sf, g, R);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        pin(g[k]);
        pin(R.pc[k]);
        pin(R.ps[k]);
      }
      step<C + 1>(c, nxt, cur, cn, sn, cf, sf, g, R);
    }
  }
  static __device__ __forceinline__ void run(const RIFT_CONST double* c, const double* cn, const double* sn,
                                             double cf, double sf, double* g) {
    Run R;
#pragma unroll
    for (int k = 0; k < 4; ++k) R.pc[k] = R.ps[k] = 0.0;
    R.er = cf;  // the first group after q = 0 is q = 1
    R.ei = sf;
    double bA[CH], bB[CH];
    ld<0>(bA, c);
    step<0>(c, bA, bB, cn, sn, cf, sf, g, R);
  }
};

// Harmonic-basis coefficients of the pair forms, one block per (detector,
// pair a <= b): Re G, Im G, Re H, Im H of the block sampled on an NG x NG
// grid of (incl, phi) over [0, 2 pi)^2, NG = 4L + 4 (more than twice the
// degree 2L in each), then projected on the basis rows (discrete
// orthogonality on that grid).  Every angle on the grid is a multiple of
// 2 pi / NG, so cos and sin come from one table of NG entries each; the
// block's U and V entries are staged in LDS; a thread per grid point, then
// each basis row's projection split over WIDE_BASIS_BLOCK / B threads.  U, V in the caller's order
// [K][A][A] complex; out [K][pair][B][4].
template <int L>
__global__ void k_wide_basis(WideDesc D, const double* __restrict__ U, const double* __restrict__ V,
                             double* __restrict__ out) {
  constexpr int NG = 4 * L + 4, B = Cls<L>::B, MX = Cls<L>::MAXM;
  constexpr int PS = WIDE_BASIS_BLOCK / B;  // threads per basis row in the projection
  __shared__ double g[4][NG * NG];
  __shared__ double part[PS][B][4];
  __shared__ double ct[NG], st[NG];
  __shared__ double uv[MX * MX][4];
  const int k = blockIdx.x / D.npairs, pr = blockIdx.x - k * D.npairs;
  int a = 0, rem = pr;
  while (rem >= D.n_a - a) {
    rem -= D.n_a - a;
    ++a;
  }
  const int b = a + rem;
  const int M = D.M, A = D.n_a * D.M;
  for (int j = threadIdx.x; j < NG; j += blockDim.x) {
    double sj, cj;
    sincospi(2.0 * j / NG, &sj, &cj);
    ct[j] = cj;
    st[j] = sj;
  }
  for (int e = threadIdx.x; e < M * M; e += blockDim.x) {
    const int i = e / M, j = e - (e / M) * M;
    const int64_t o = 2 * (((int64_t)k * A + a * M + D.perm[i]) * A + b * M + D.perm[j]);
    uv[e][0] = U[o];
    uv[e][1] = U[o + 1];
    uv[e][2] = V[o];
    uv[e][3] = V[o + 1];
  }
  __syncthreads();
  // index of the angle n * (2 pi c / NG) in the tables
  auto ix = [](int n, int c) { return ((n * c) % NG + NG) % NG; };
  for (int gp = threadIdx.x; gp < NG * NG; gp += blockDim.x) {
    const int pi_ = gp / NG, pf = gp - (gp / NG) * NG;
    double yr[MX], yi[MX];
#pragma unroll
    for (int i = 0; i < MX; ++i) {
      yr[i] = yi[i] = 0.0;
      if (i < M) {
        double d = 0.0;
        for (int q = 0; q <= L; ++q) d += D.ycoef[i][q] * (D.odd[i] ? st[ix(q, pi_)] : ct[ix(q, pi_)]);
        const int r = ix(D.m[i], pf);
        yr[i] = d * ct[r];
        yi[i] = d * st[r];
      }
    }
    double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < MX; ++i) {
      if (i < M) {
        double tr = 0.0, ti = 0.0, wr = 0.0, wi = 0.0;
#pragma unroll
        for (int j = 0; j < MX; ++j) {
          if (j < M) {
            const double* e = uv[i * M + j];
            tr += e[0] * yr[j] - e[1] * yi[j];
            ti += e[0] * yi[j] + e[1] * yr[j];
            wr += e[2] * yr[j] - e[3] * yi[j];
            wi += e[2] * yi[j] + e[3] * yr[j];
          }
        }
        v[0] += yr[i] * tr + yi[i] * ti;
        v[1] += yr[i] * ti - yi[i] * tr;
        v[2] += yr[i] * wr - yi[i] * wi;
        v[3] += yr[i] * wi + yi[i] * wr;
      }
    }
    for (int c = 0; c < 4; ++c) g[c][gp] = v[c];
  }
  __syncthreads();
  // each row's sum over the grid split over PS threads, then reduced
  for (int w = threadIdx.x; w < PS * B; w += blockDim.x) {
    const int r = w % B, sp = w / B;
    const int rb = basis_row<L>(r);
    const int kind = rb & 15, nn = (rb >> 4) & 255, q = rb >> 12;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int gp = sp; gp < NG * NG; gp += PS) {
      const int pi_ = gp / NG, pf = gp - (gp / NG) * NG;
      const double ti = (kind >= 3) ? st[ix(nn, pi_)] : ct[ix(nn, pi_)];
      const double tf = (kind == 0) ? 1.0 : (kind == 1 || kind == 3) ? ct[ix(q, pf)] : st[ix(q, pf)];
      const double t = ti * tf;
      for (int c = 0; c < 4; ++c) acc[c] += g[c][gp] * t;
    }
    for (int c = 0; c < 4; ++c) part[sp][r][c] = acc[c];
  }
  __syncthreads();
  for (int r = threadIdx.x; r < B; r += blockDim.x) {
    const int rb = basis_row<L>(r);
    const int nn = (rb >> 4) & 255, q = rb >> 12;
    const double norm = 1.0 / ((double)NG * NG * (nn == 0 ? 1.0 : 0.5) * (q == 0 ? 1.0 : 0.5));
    double* o = out + ((int64_t)blockIdx.x * B + r) * 4;
    for (int c = 0; c < 4; ++c) {
      double v = 0.0;
      for (int sp = 0; sp < PS; ++sp) v += part[sp][r][c];
      o[c] = v * norm;
    }
  }
}

// cos(2 pi j / 5), sin(2 pi j / 5), j = 0..4: the five hour angles of the
// rotation harmonics and the factors of their transform (e^{-2 pi i n j / 5}
// is entry (n j) mod 5, conjugated).
__constant__ double kC5[5] = {1.0, 0.30901699437494745, -0.80901699437494745, -0.80901699437494745,
                              0.30901699437494745};
__constant__ double kS5[5] = {0.0, 0.95105651629515353, 0.58778525229247314, -0.58778525229247314,
                              -0.95105651629515353};

// sin and cos of |x| <= 1 by their Taylor series through x^19 / 19! and
// x^18 / 18! (truncation below 1e-17): the rotation over the light-travel
// time, Omega (t_k - t_ref), which the validation keeps within one radian.
__device__ __forceinline__ void sincos_small(double x, double* s, double* c) {
  const double x2 = x * x;
  double ps = -1.0 / 121645100408832000.0;  // -1/19!
  ps = fma(ps, x2, 1.0 / 355687428096000.0);
  ps = fma(ps, x2, -1.0 / 1307674368000.0);
  ps = fma(ps, x2, 1.0 / 6227020800.0);
  ps = fma(ps, x2, -1.0 / 39916800.0);
  ps = fma(ps, x2, 1.0 / 362880.0);
  ps = fma(ps, x2, -1.0 / 5040.0);
  ps = fma(ps, x2, 1.0 / 120.0);
  ps = fma(ps, x2, -1.0 / 6.0);
  *s = fma(ps * x2, x, x);
  double pc = 1.0 / 6402373705728000.0;  // 1/18!
  pc = fma(pc, x2, -1.0 / 20922789888000.0);
  pc = fma(pc, x2, 1.0 / 87178291200.0);
  pc = fma(pc, x2, -1.0 / 479001600.0);
  pc = fma(pc, x2, 1.0 / 3628800.0);
  pc = fma(pc, x2, -1.0 / 40320.0);
  pc = fma(pc, x2, 1.0 / 720.0);
  pc = fma(pc, x2, -1.0 / 24.0);
  pc = fma(pc, x2, 0.5);
  *c = fma(-pc, x2, 1.0);
}

// Occupancy: three wavefronts per SIMD (<= 168 VGPRs) for up to 5 modes, two
// otherwise (the 25-mode capacity's Y alone holds 100 VGPRs).  NT is the
// capacity of the coefficient columns in LDS (NT x BLK complex values).
template <int MC, int NT, int BLK, int HL = 0>
__global__ void __launch_bounds__(BLK, MC <= 5 && NT <= 12 ? 3 : 2) k_wide(WideDesc D, const double* __restrict__ theta, int64_t n,
                                                              const double* __restrict__ lnw,
                                                              double* __restrict__ lnL, double* __restrict__ part) {
  __shared__ double cre[NT][BLK], cim[NT][BLK];
  __shared__ MS sh[BLK / 64];
  const int t = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * BLK + t;
  const bool live = i0 < n;
  const int64_t i = live ? i0 : n - 1;
  const RIFT_GLOBAL double* th = as_global(theta) + i;
  const double ra = th[0], dec = th[n], psi = th[2 * n], incl = th[3 * n], phi = th[4 * n];
  const double tref = th[5 * n], dist = th[6 * n];
  const int K = D.K, M = D.M, n_t = D.n_t, n_a = D.n_a;
  const bool rot = D.response == RIFT_RESP_ROTATION || D.response == RIFT_RESP_ROTATION_DELAY;
  const bool drift = D.response == RIFT_RESP_ROTATION_DELAY && n_a > 5;

  // sky frame at t_ref (the rotation response advances the sidereal angle)
  const double gm = rot ? D.gmst + D.omega * tref : D.gmst;
  const double gref = gm - ra;
  double sg, cg, sd, cd, sp, cp;
  sincos(gref, &sg, &cg);
  sincos(dec, &sd, &cd);
  sincos(psi, &sp, &cp);
  double X[3], Y3[3], N[3];
  axes(sg, cg, sd, cd, sp, cp, X, Y3, N);

  // harmonics Y_i = d_i(incl) e^{i m_i phi}, internal (m-sorted) modes
  double ci, si, cf, sf;
  sincos(incl, &si, &ci);
  sincos(phi, &sf, &cf);
  double cn[LMAXC + 1], sn[LMAXC + 1];
  {
    double c0 = 1.0, c1 = ci, s0 = 0.0, s1 = si;
#pragma unroll
    for (int q = 0; q <= LMAXC; ++q) {
      cn[q] = (q == 0) ? c0 : c1;
      sn[q] = (q == 0) ? s0 : s1;
      if (q > 0) {
        const double c2 = 2.0 * ci * c1 - c0, s2 = 2.0 * ci * s1 - s0;
        c0 = c1;
        c1 = c2;
        s0 = s1;
        s1 = s2;
      }
    }
  }
  double yr[MC], yi[MC];
  {
    C2<double> ph;
    ph.x = 1.0;
    ph.y = 0.0;
    const int mmin = D.m[0];
    for (int q = 0; q < -mmin; ++q) phase_down(ph, cf, sf);
    int mc = mmin < 0 ? mmin : 0;
#pragma unroll
    for (int j = 0; j < MC; ++j) {
      yr[j] = yi[j] = 0.0;
      if (j < M) {
        const int mj = D.m[j];
        while (mc < mj) {
          phase_up(ph, cf, sf);
          ++mc;
        }
        double d = 0.0;
        if (D.odd[j]) {
#pragma unroll
          for (int q = 1; q <= LMAXC; ++q) d += D.ycoef[j][q] * sn[q];
        } else {
#pragma unroll
          for (int q = 0; q <= LMAXC; ++q) d += D.ycoef[j][q] * cn[q];
        }
        yr[j] = d * ph.x;
        yi[j] = d * ph.y;
      }
    }
  }

  double data = 0.0, quad = 0.0;
  bool bad = false;
  for (int k = 0; k < K; ++k) {
    const double tk = tref - (D.rpos[k][0] * N[0] + D.rpos[k][1] * N[1] + D.rpos[k][2] * N[2]);
    // composite coefficients of this detector -> this lane's LDS column
    if (rot) {
      // F_k at the five hour angles g_j = 2 pi j / 5, then A_n by the exact
      // five-point transform, then the phases e^{i n theta_k}
      // (the frames at the five hour angles do not depend on k; they are
      // rebuilt per detector rather than kept live across the loop, which
      // would hold 120 registers)
      double sdk = sd, cdk = cd, spk = sp, cpk = cp;
      asm volatile("" : "+v"(sdk), "+v"(cdk), "+v"(spk), "+v"(cpk));
      C2<double> Fg[5];
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        double Xj[3], Yj[3], Nj[3];
        axes(kS5[j], kC5[j], sdk, cdk, spk, cpk, Xj, Yj, Nj);
        Fg[j] = response6(D.dten[k], Xj, Yj);
      }
      // e^{i theta_k} = e^{i g(t_ref)} e^{i Omega (t_k - t_ref)}
      double sdl, cdl;
      sincos_small(D.omega * (tk - tref), &sdl, &cdl);
      const double e1c = cg * cdl - sg * sdl, e1s = sg * cdl + cg * sdl;
      const double e2c = e1c * e1c - e1s * e1s, e2s = 2.0 * e1c * e1s;
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        const int nn = a - 2;
        double ar = 0.0, ai = 0.0;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          const int r = ((nn * j) % 5 + 5) % 5;
          const double c = kC5[r], s = -kS5[r];  // e^{-i n g_j}
          ar += Fg[j].x * c - Fg[j].y * s;
          ai += Fg[j].x * s + Fg[j].y * c;
        }
        ar *= 0.2;
        ai *= 0.2;
        // e^{i n theta_k}
        const double er = (nn == 0) ? 1.0 : (nn == 1 || nn == -1) ? e1c : e2c;
        const double ei = (nn == 0) ? 0.0 : (nn == 1) ? e1s : (nn == -1) ? -e1s : (nn == 2) ? e2s : -e2s;
        cre[a][t] = ar * er - ai * ei;
        cim[a][t] = ar * ei + ai * er;
      }
      if (drift) {
        // first order in the delay drift (Path B, p = 1).  The drift's
        // harmonics in the modulation phase, -dt: m = -1, 0, +1 from
        // rho e^{i g(t_ref)}, rho = r_x + i r_y.  With the post-phases
        // folded in, C~_(1, n) = sum_m C~_(0, n - m) D_m e^{i m Omega (t_k - t_ref)}
        // for n = -3 .. 3, the order-0 terms read back from this lane's column
        const double rer = D.rpos[k][0] * cg - D.rpos[k][1] * sg, rei = D.rpos[k][0] * sg + D.rpos[k][1] * cg;
        // D_m e^{i m Omega (t_k - t_ref)}, m = -1, 0, +1
        const double hr = 0.5 * cd * rer, hi = 0.5 * cd * rei;
        const double dmr[3] = {hr * cdl - hi * sdl, -cd * rer, hr * cdl - hi * sdl};
        const double dmi[3] = {hr * (-sdl) - hi * cdl, 0.0, hr * sdl + hi * cdl};
#pragma unroll
        for (int b = 0; b < 7; ++b) {
          const int nn = b - 3;
          double cr = 0.0, ci = 0.0;
#pragma unroll
          for (int m = -1; m <= 1; ++m) {
            const int q = nn - m;
            if (q < -2 || q > 2) continue;
            const double xr = cre[q + 2][t], xi = cim[q + 2][t];
            cr += xr * dmr[m + 1] - xi * dmi[m + 1];
            ci += xr * dmi[m + 1] + xi * dmr[m + 1];
          }
          cre[5 + b][t] = cr;
          cim[5 + b][t] = ci;
        }
        if (NT >= 21 && n_a >= 21) {
          // order 2: the drift's square, (D~ * D~)_m for m = -2..2, and
          // C~_(2, n) = 1/2 sum_m C~_(0, n - m) (D~ * D~)_m for n = -4..4
          double d2r[5], d2i[5];
#pragma unroll
          for (int m = 0; m < 5; ++m) {
            d2r[m] = 0.0;
            d2i[m] = 0.0;
          }
#pragma unroll
          for (int m1 = 0; m1 < 3; ++m1)
#pragma unroll
            for (int m2 = 0; m2 < 3; ++m2) {
              d2r[m1 + m2] += dmr[m1] * dmr[m2] - dmi[m1] * dmi[m2];
              d2i[m1 + m2] += dmr[m1] * dmi[m2] + dmi[m1] * dmr[m2];
            }
#pragma unroll
          for (int b = 0; b < 9; ++b) {
            const int nn = b - 4;
            double cr = 0.0, ci = 0.0;
#pragma unroll
            for (int m = -2; m <= 2; ++m) {
              const int q = nn - m;
              if (q < -2 || q > 2) continue;
              const double xr = cre[q + 2][t], xi = cim[q + 2][t];
              cr += xr * d2r[m + 2] - xi * d2i[m + 2];
              ci += xr * d2i[m + 2] + xi * d2r[m + 2];
            }
            cre[12 + b][t] = 0.5 * cr;
            cim[12 + b][t] = 0.5 * ci;
          }
        }
      }
    } else {
      const double* ax = D.arms[k][0];
      const double* ay = D.arms[k][1];
      const double xX = X[0] * ax[0] + X[1] * ax[1] + X[2] * ax[2];
      const double xY = Y3[0] * ax[0] + Y3[1] * ax[1] + Y3[2] * ax[2];
      const double yX = X[0] * ay[0] + X[1] * ay[1] + X[2] * ay[2];
      const double yY = Y3[0] * ay[0] + Y3[1] * ay[1] + Y3[2] * ay[2];
      const double exr = xX * xX - xY * xY, exi = 2.0 * xX * xY;
      const double eyr = yX * yX - yY * yY, eyi = 2.0 * yX * yY;
      const double ux = N[0] * ax[0] + N[1] * ax[1] + N[2] * ax[2];
      const double uy = N[0] * ay[0] + N[1] * ay[1] + N[2] * ay[2];
      double px = 1.0, py = 1.0;
      for (int a = 0; a < n_a; ++a) {
        cre[a][t] = 0.5 * (px * exr - py * eyr);
        cim[a][t] = 0.5 * (px * exi - py * eyi);
        px *= ux;
        py *= uy;
      }
    }
    // four-point Lagrange stencil at t_k (taps outside the window read zero)
    double u = (tk - D.t0) * D.inv_dt;
    if (!(fabs(u) <= 1.0e300)) {
      bad = true;
      u = 0.0;
    }
    u = fmin(fmax(u, -8.0), (double)n_t + 8.0);
    const double jf = floor(u);
    const double s = u - jf;
    const int j0 = (int)jf - 1;
    double w[4];
    lagrange4(s, w);
#pragma unroll
    for (int tap = 0; tap < 4; ++tap)
      if (j0 + tap < 0 || j0 + tap >= n_t) w[tap] = 0.0;
    // the four rows read are jc .. jc+3, inside the window; row jc + r carries
    // tap r + jc - j0 (weight 0 when that is not a tap or lies outside)
    const int jc = j0 < 0 ? 0 : (j0 > n_t - 4 ? n_t - 4 : j0);
    double wr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int tp = r + jc - j0;
      double v = 0.0;
#pragma unroll
      for (int tap = 0; tap < 4; ++tap) v = (tp == tap) ? w[tap] : v;
      wr[r] = v;
    }
    // data term: Re sum_a conj(C~_a) sum_i conj(Y_i) Qhat_{a,i}
    for (int a = 0; a < n_a; ++a) {
      double zr = 0.0, zi = 0.0;
#pragma unroll
      for (int j = 0; j < MC; ++j) {
        if (j < M) {
          const RIFT_GLOBAL double* q =
              as_global(D.Q) + 2 * ((((int64_t)k * n_a + a) * M + D.perm[j]) * (int64_t)n_t + jc);
          double qr = 0.0, qi = 0.0;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            qr += wr[r] * q[2 * r];
            qi += wr[r] * q[2 * r + 1];
          }
          // conj(Y) Qhat
          zr += yr[j] * qr + yi[j] * qi;
          zi += yr[j] * qi - yi[j] * qr;
        }
      }
      // Re[conj(C~_a) z]
      data += cre[a][t] * zr + cim[a][t] * zi;
    }
    // model-norm term over pairs a <= a'
    constexpr int BS = HL > 0 ? 4 * Cls<(HL > 0 ? HL : 2)>::B : MC * MC * 4;
    const RIFT_CONST double* blk = as_const(D.UV) + (int64_t)k * D.npairs * BS;
    for (int a = 0; a < n_a; ++a) {
      for (int b = a; b < n_a; ++b, blk += BS) {
        double g[4] = {0.0, 0.0, 0.0, 0.0};  // Re G, Im G, Re H, Im H
        if constexpr (HL > 0) {
          // the phase sequence is rebuilt per pair, not hoisted out of the
          // loops (it would hold 4 HL values in registers throughout)
          double cfo = cf, sfo = sf;
          asm volatile("" : "+v"(cfo), "+v"(sfo));
          HarmForms<HL>::run(opaque(blk), cn, sn, cfo, sfo, g);
        }
        else if constexpr (MC == 5)
          PairFormsP<5>::run(opaque(blk), yr, yi, g);
        else
          PairForms<0, MC>::run(opaque(blk), M, yr, yi, g);
        const double gr = g[0], gi = g[1], hr = g[2], hi = g[3];
        const double car = cre[a][t], cai = cim[a][t], cbr = cre[b][t], cbi = cim[b][t];
        // conj(C_a) C_b G_ab and C_a C_b H_ab, counted twice off the diagonal
        const double pr = car * cbr + cai * cbi, pim = car * cbi - cai * cbr;
        const double qr = car * cbr - cai * cbi, qim = car * cbi + cai * cbr;
        const double f = (a == b) ? 1.0 : 2.0;
        quad += f * ((pr * gr - pim * gi) + (qr * hr - qim * hi));
      }
    }
  }
  const double x = D.d_ref / dist;
  double l = x * data - 0.25 * x * x * quad;
  if (bad) l = __builtin_nan("");
  if (live && lnL) as_global_w(lnL)[i] = l;
  if (part) {
    MS acc;
    acc.m = -__builtin_inf();
    acc.s = 0.0;
    if (live) acc = ms_push(acc, l + (lnw ? as_global(lnw)[i] : 0.0));
    const MS r = ms_block(acc, sh);
    if (t == 0) {
      part[2 * blockIdx.x] = r.m;
      part[2 * blockIdx.x + 1] = r.s;
    }
  }
}

// ln Z and n_eff from the blocks' (max, sum) pairs, one block, fixed order.
__global__ void k_wide_merge(double lnN, const double* __restrict__ part, int nb, double* __restrict__ lnZ,
                             double* __restrict__ neff) {
  __shared__ MS sh[WIDE_BLOCK / 64];
  MS acc;
  acc.m = -__builtin_inf();
  acc.s = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    MS o;
    o.m = part[2 * b];
    o.s = part[2 * b + 1];
    if (o.s != o.s) acc.s = o.s;
    else if (o.s != 0.0) acc = ms_combine(acc, o);
  }
  const MS r = ms_block(acc, sh);
  if (threadIdx.x == 0) {
    double z;
    if (r.s != r.s) z = __builtin_nan("");
    else if (r.m == -__builtin_inf()) z = -__builtin_inf();
    else z = r.m + log(r.s) - lnN;
    lnZ[0] = z;
    if (neff) neff[0] = (r.m == -__builtin_inf() && r.s == r.s) ? 0.0 : r.s;
  }
}

int validate_wide(const rift_ile_point_wide* pt) {
  if (!pt) return RIFT_EINVAL;
  if (pt->n_det < 1 || pt->n_det > RIFT_ILE_MAX_DET) return RIFT_EINVAL;
  if (pt->n_modes < 1 || pt->n_modes > RIFT_ILE_MAX_MODES) return RIFT_EINVAL;
  if (pt->n_t < 4 || pt->n_t > RIFT_ILE_MAX_NT) return RIFT_EINVAL;
  if (pt->response == RIFT_RESP_ROTATION) {
    if (pt->n_terms != 5) return RIFT_EINVAL;
    if (!std::isfinite(pt->omega)) return RIFT_EINVAL;
  } else if (pt->response == RIFT_RESP_ROTATION_DELAY) {
    if (pt->n_terms != 5 && pt->n_terms != 12 && pt->n_terms != 21) return RIFT_EINVAL;
    if (!std::isfinite(pt->omega)) return RIFT_EINVAL;
  } else if (pt->response == RIFT_RESP_ARMS) {
    if (pt->n_terms < 1 || pt->n_terms > WIDE_ARMS_MAX_TERMS || !pt->det_arms) return RIFT_EINVAL;
    for (int a = 0; a < 6 * pt->n_det; ++a)
      if (!std::isfinite(pt->det_arms[a])) return RIFT_EINVAL;
  } else {
    return RIFT_EINVAL;
  }
  if (!pt->lm || !pt->Q || !pt->U || !pt->V || !pt->det_tensor || !pt->det_pos) return RIFT_EINVAL;
  if ((((uintptr_t)pt->Q) | ((uintptr_t)pt->U) | ((uintptr_t)pt->V)) & 7u) return RIFT_EINVAL;
  if (!std::isfinite(pt->t0) || !std::isfinite(pt->dt) || !(pt->dt > 0.0)) return RIFT_EINVAL;
  if (!std::isfinite(pt->gmst_rad) || !std::isfinite(pt->d_ref) || !(pt->d_ref > 0.0)) return RIFT_EINVAL;
  for (int i = 0; i < pt->n_modes; ++i) {
    const int l = pt->lm[2 * i], m = pt->lm[2 * i + 1];
    if (l < 2 || l > RIFT_ILE_MAX_L || m < -l || m > l) return RIFT_EINVAL;
    for (int j = 0; j < i; ++j)
      if (pt->lm[2 * j] == l && pt->lm[2 * j + 1] == m) return RIFT_EINVAL;
  }
  for (int a = 0; a < 9 * pt->n_det; ++a)
    if (!std::isfinite(pt->det_tensor[a])) return RIFT_EINVAL;
  for (int a = 0; a < 3 * pt->n_det; ++a)
    if (!std::isfinite(pt->det_pos[a])) return RIFT_EINVAL;
  // rotation: the turn over the light-travel time, Omega |r_k|, stays within
  // one radian (the post-phase is evaluated by a series on that range)
  if (pt->response == RIFT_RESP_ROTATION || pt->response == RIFT_RESP_ROTATION_DELAY)
    for (int k = 0; k < pt->n_det; ++k) {
      const double* r = pt->det_pos + 3 * k;
      if (!(fabs(pt->omega) * sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) <= 1.0)) return RIFT_EINVAL;
    }
  return RIFT_OK;
}

// One call: description to the device, the sample kernel, optionally the merge.
int wide_run(const rift_ile_point_wide* pt, int64_t n, const double* theta, const double* lnw, double* lnL,
             double* lnZ, double* neff, void* stream) {
  int rc = validate_wide(pt);
  if (rc) return rc;
  if (n < 0) return RIFT_EINVAL;
  if (n == 0) return lnZ ? RIFT_EINVAL : RIFT_OK;
  auto bad_ptr = [](const void* p) { return !p || (((uintptr_t)p) & 7u); };
  if (bad_ptr(theta) || (lnL && bad_ptr(lnL)) || (lnw && bad_ptr(lnw)) || (lnZ && bad_ptr(lnZ)) ||
      (neff && bad_ptr(neff)))
    return RIFT_EINVAL;
  if (!lnL && !lnZ) return RIFT_EINVAL;
  const int blk = pt->n_terms <= 12 ? WIDE_BLOCK : WIDE_BLOCK_21;
  const int64_t nb = (n + blk - 1) / blk;
  if (nb > 0x7fffffff) return RIFT_EUNSUPPORTED;
  WideDesc D;
  memset(&D, 0, sizeof(D));
  D.K = pt->n_det;
  D.M = pt->n_modes;
  D.n_t = pt->n_t;
  D.n_a = pt->n_terms;
  D.npairs = pt->n_terms * (pt->n_terms + 1) / 2;
  D.response = pt->response;
  D.t0 = pt->t0;
  D.inv_dt = 1.0 / pt->dt;
  D.gmst = pt->gmst_rad;
  D.omega = (pt->response == RIFT_RESP_ROTATION || pt->response == RIFT_RESP_ROTATION_DELAY) ? pt->omega : 0.0;
  D.d_ref = pt->d_ref;
  for (int k = 0; k < pt->n_det; ++k) {
    const double* d = pt->det_tensor + 9 * k;
    const double six[6] = {d[0], d[4], d[8], d[1] + d[3], d[2] + d[6], d[5] + d[7]};
    for (int a = 0; a < 6; ++a) D.dten[k][a] = six[a];
    for (int a = 0; a < 3; ++a) D.rpos[k][a] = pt->det_pos[3 * k + a];
    if (pt->response == RIFT_RESP_ARMS)
      for (int e = 0; e < 2; ++e)
        for (int a = 0; a < 3; ++a) D.arms[k][e][a] = pt->det_arms[6 * k + 3 * e + a];
  }
  std::vector<int> perm(pt->n_modes);
  for (int i = 0; i < pt->n_modes; ++i) perm[i] = i;
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return pt->lm[2 * a + 1] < pt->lm[2 * b + 1]; });
  for (int i = 0; i < pt->n_modes; ++i) {
    const int l = pt->lm[2 * perm[i]], m = pt->lm[2 * perm[i] + 1];
    D.perm[i] = perm[i];
    D.m[i] = m;
    D.odd[i] = (m & 1) ? 1 : 0;
    ylm_fourier(l, m, D.ycoef[i]);
  }
  D.Q = pt->Q;
  const int MC = pt->n_modes <= 5 ? 5 : (pt->n_modes <= 12 ? 12 : 25);
  // the harmonic form where its basis is shorter than a block's entries
  int lmax = 0;
  for (int i = 0; i < pt->n_modes; ++i) lmax = std::max(lmax, (int)pt->lm[2 * i]);
  const int M2 = pt->n_modes * pt->n_modes;
  D.hb = (MC == 12 && lmax == 3 && Cls<3>::B < M2) ? 3 : (MC == 25 && lmax == 4 && Cls<4>::B < M2) ? 4 : 0;
  const int blk_vals = D.hb == 3 ? 4 * Cls<3>::B : D.hb == 4 ? 4 * Cls<4>::B : 4 * MC * MC;
  // stream-ordered scratch: the packed U/V blocks (or their coefficients),
  // then the blocks' (max, sum) pairs
  const size_t uv_bytes = sizeof(double) * (size_t)D.K * D.npairs * blk_vals;
  const size_t part_bytes = lnZ ? sizeof(double) * 2 * (size_t)nb : 0;
  hipStream_t st = (hipStream_t)stream;
  void* scratch = nullptr;
  if (hipMallocAsync(&scratch, uv_bytes + part_bytes, st) != hipSuccess) return RIFT_ENOMEM;
  D.UV = (const double*)scratch;
  double* d_part = lnZ ? (double*)((char*)scratch + uv_bytes) : nullptr;
  const int64_t pe = (int64_t)D.K * D.npairs * MC * MC;
  const unsigned pgrid = (unsigned)std::min<int64_t>((pe + 255) / 256, 1024);
  const bool wide21 = blk == WIDE_BLOCK_21;
  const dim3 grid((unsigned)nb), block(blk);
  switch (MC) {
    case 5:
      hipLaunchKernelGGL(k_wide_pack<5>, dim3(pgrid), dim3(256), 0, st, D, pt->U, pt->V, (double*)scratch);
      if (wide21)
        hipLaunchKernelGGL((k_wide<5, 21, WIDE_BLOCK_21>), grid, block, 0, st, D, theta, n, lnw, lnL, d_part);
      else
        hipLaunchKernelGGL((k_wide<5, 12, WIDE_BLOCK>), grid, block, 0, st, D, theta, n, lnw, lnL, d_part);
      break;
    case 12:
      if (D.hb == 3) {
        hipLaunchKernelGGL(k_wide_basis<3>, dim3((unsigned)(D.K * D.npairs)), dim3(WIDE_BASIS_BLOCK), 0, st, D,
                           pt->U, pt->V, (double*)scratch);
        if (wide21)
          hipLaunchKernelGGL((k_wide<12, 21, WIDE_BLOCK_21, 3>), grid, block, 0, st, D, theta, n, lnw, lnL, d_part);
        else
          hipLaunchKernelGGL((k_wide<12, 12, WIDE_BLOCK, 3>), grid, block, 0, st, D, theta, n, lnw, lnL, d_part);
        break;
      }
      hipLaunchKernelGGL(k_wide_pack<12>, dim3(pgrid), dim3(256), 0, st, D, pt->U, pt->V, (double*)scratch);
      if (wide21)
        hipLaunchKernelGGL((k_wide<12, 21, WIDE_BLOCK_21>), grid, block, 0, st, D, theta, n, lnw, lnL, d_part);
      else
        hipLaunchKernelGGL((k_wide<12, 12, WIDE_BLOCK>), grid, block, 0, st, D, theta, n, lnw, lnL, d_part);
      break;
    default:
      if (D.hb == 4) {
        hipLaunchKernelGGL(k_wide_basis<4>, dim3((unsigned)(D.K * D.npairs)), dim3(WIDE_BASIS_BLOCK), 0, st, D,
                           pt->U, pt->V, (double*)scratch);
        if (wide21)
          hipLaunchKernelGGL((k_wide<21, 21, WIDE_BLOCK_21, 4>), grid, block, 0, st, D, theta, n, lnw, lnL, d_part);
        else
          hipLaunchKernelGGL((k_wide<21, 12, WIDE_BLOCK, 4>), grid, block, 0, st, D, theta, n, lnw, lnL, d_part);
        break;
      }
      hipLaunchKernelGGL(k_wide_pack<25>, dim3(pgrid), dim3(256), 0, st, D, pt->U, pt->V, (double*)scratch);
      if (wide21)
        hipLaunchKernelGGL((k_wide<25, 21, WIDE_BLOCK_21>), grid, block, 0, st, D, theta, n, lnw, lnL, d_part);
      else
        hipLaunchKernelGGL((k_wide<25, 12, WIDE_BLOCK>), grid, block, 0, st, D, theta, n, lnw, lnL, d_part);
  }
  if (lnZ)
    hipLaunchKernelGGL(k_wide_merge, dim3(1), dim3(WIDE_BLOCK), 0, st, log((double)n), (const double*)d_part, (int)nb,
                       lnZ, neff);
  rc = hipGetLastError() == hipSuccess ? RIFT_OK : RIFT_EDEVICE;
  // released in stream order, after the kernels above
  if (hipFreeAsync(scratch, st) != hipSuccess && !rc) rc = RIFT_EDEVICE;
  return rc;
}

}  // namespace
}  // namespace rift

extern "C" int rift_ile_wide_lnL(const rift_ile_point_wide* pt, int64_t n, const double* theta, double* lnL,
                                 void* stream) {
  if (!lnL && n > 0) return RIFT_EINVAL;
  return rift::wide_run(pt, n, theta, nullptr, lnL, nullptr, nullptr, stream);
}

extern "C" int rift_ile_wide_lnZ(const rift_ile_point_wide* pt, int64_t n, const double* theta, const double* lnw,
                                 double* lnZ, double* neff, double* lnL, void* stream) {
  if (!lnZ || n < 1) return RIFT_EINVAL;
  return rift::wide_run(pt, n, theta, lnw, lnL, lnZ, neff, stream);
}
