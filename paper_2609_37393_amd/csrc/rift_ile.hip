// Host side, setup kernels and entry points of the MI355X factored extrinsic
// likelihood (C ABI declared in include/rift_ile.h).
//
// Flow of one batch (Eqs. (def:lnL:Decomposed), (lnL:MonteCarlo), (neff)):
//   plan creation (once per set of points):
//     k_repack   Q[K][M][n_t] (paper order) -> Q[KT][ceil(M/W)][n_t + 2 QPAD][W], W modes
//                per row (FP64, FP32)
//     k_qmax     max |Q_k| per detector (error bound of the mixed path)
//     k_basis    harmonic-basis coefficients of the model-norm term
//   evaluation (no allocation, no host synchronisation -> graph-capturable):
//     FP64 : k_tiles<double>  one persistent launch over (point, sample-block)
//            tiles, per-tile (max, sum exp) partials -> k_merge -> ln Z, n_eff
//     MIXED: k_tiles<float> (value + a-priori bound) -> k_select (M_low, and
//            the samples whose bound reaches within T of the best) -> k_refine
//            (FP64 recompute of those) -> k_final (LSE + omitted-error sum)
//            -> k_merge
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/rift_ile.h"
#include "ile_host.h"
#include "ile_kernels.h"

using namespace rift;

namespace {

// ---------------------------------------------------------------------------
// Setup kernels
// ---------------------------------------------------------------------------

// Q[k][i][t] (caller order, complex) -> Qt[k][i_internal / W][QPAD + t][i_internal % W]:
// W internal modes per padded time row, QPAD zero rows at both ends of every
// series, zero slots past M and zero padded detectors.
template <class T>
__global__ void k_repack(const double* __restrict__ Q, T* __restrict__ Qt,
                         const int32_t* __restrict__ perm, int K, int KT, int M, int n_t, int W) {
  const int ntp = n_t + 2 * QPAD;
  const int ngr = q_groups(M, W);
  const int64_t total = (int64_t)KT * ngr * ntp * W;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int sl = (int)(e % W);
    const int64_t rest = e / W;
    const int tp = (int)(rest % ntp);
    const int64_t kg = rest / ntp;
    const int g = (int)(kg % ngr);
    const int k = (int)(kg / ngr);
    const int i = g * W + sl;
    const int t = tp - QPAD;
    double re = 0.0, im = 0.0;
    if (k < K && i < M && t >= 0 && t < n_t) {
      const int64_t src = ((int64_t)k * M + perm[i]) * n_t + t;
      re = Q[2 * src];
      im = Q[2 * src + 1];
    }
    Qt[2 * e] = (T)re;
    Qt[2 * e + 1] = (T)im;
  }
}

// out[k] = max |Q64| over detector k's n complex entries, one block per detector.
__global__ void k_qmax(const double* __restrict__ Q64, double* __restrict__ out, int64_t n) {
  const int k = blockIdx.x;
  const double* q = Q64 + 2 * (int64_t)k * n;
  double m = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) m = fmax(m, hypot(q[2 * e], q[2 * e + 1]));
  m = dmax_wave(m);
  __shared__ double sh[16];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, sh[w]);
    out[k] = r;
  }
}

// Basis function b of class L: kind 0 = cos(n i), 1 = cos(n i) cos(q f),
// 2 = cos(n i) sin(q f), 3 = sin(n i) cos(q f), 4 = sin(n i) sin(q f).
// The order matches the contraction loop of eval_sample.
__host__ __device__ inline void basis_index(int L, int b, int* kind, int* n, int* q) {
  const int NI = 2 * L;
  int bb = b;
  for (int qq = 0; qq <= NI; ++qq) {
    if (qq == 0) {
      if (bb <= NI) { *kind = 0; *n = bb; *q = 0; return; }
      bb -= NI + 1;
    } else if ((qq & 1) == 0) {
      if (bb < 2 * (NI + 1)) { *kind = 1 + (bb & 1); *n = bb >> 1; *q = qq; return; }
      bb -= 2 * (NI + 1);
    } else {
      if (bb < 2 * NI) { *kind = 3 + (bb & 1); *n = 1 + (bb >> 1); *q = qq; return; }
      bb -= 2 * NI;
    }
  }
  *kind = -1; *n = 0; *q = 0;
}

inline int basis_count(int L) {
  const int NI = 2 * L, NQ = 2 * L;
  return (NI + 1) + (NQ / 2) * 2 * (NI + 1) + ((NQ + 1) / 2) * 2 * NI;
}

// Harmonic-basis coefficients of g_c = (a_k/4, Re b_k/4, -Im b_k/4) for one
// detector per block: sample g_c on an NG x NG grid of (incl, phi) over
// [0, 2 pi)^2 (NG = 4L + 4, more than twice the degree 2L) and project
// (discrete orthogonality of the basis on that grid).  U, V in caller order,
// modes mapped through perm.  Writes column 3k..3k+2 of C64/C32 [B][3 KT].
__global__ void k_basis(const PointDesc* __restrict__ P, const double* __restrict__ U,
                        const double* __restrict__ V, const int32_t* __restrict__ perm,
                        double* __restrict__ C64, float* __restrict__ C32) {
  extern __shared__ double g[];  // [3][NG][NG]
  const int k = blockIdx.x;
  const int M = P->M, L = P->L, KT = P->KT, B = P->B;
  const int NG = 4 * L + 4;
  const double two_pi = 6.283185307179586476925286766559;
  for (int gp = threadIdx.x; gp < NG * NG; gp += blockDim.x) {
    const int pi_ = gp / NG, pf = gp % NG;
    const double inc = two_pi * pi_ / NG, ph = two_pi * pf / NG;
    double yr[MMAX], yi[MMAX];
    for (int i = 0; i < M; ++i) {
      double d = 0.0;
      for (int n = 0; n <= L; ++n) {
        const double c = P->ycoef[i][n];
        d += P->odd[i] ? c * sin(n * inc) : c * cos(n * inc);
      }
      double s, cc;
      sincos(P->m[i] * ph, &s, &cc);
      yr[i] = d * cc;
      yi[i] = d * s;
    }
    double ar = 0.0, br = 0.0, bi = 0.0;
    if (k < P->K) {
      for (int i = 0; i < M; ++i) {
        const int ci = perm[i];
        for (int j = 0; j < M; ++j) {
          const int cj = perm[j];
          const int64_t o = 2 * (((int64_t)k * M + ci) * M + cj);
          const double ur = U[o], ui = U[o + 1], vr = V[o], vi = V[o + 1];
          // Re[conj(Y_i) U_ij Y_j] and Y_i V_ij Y_j
          const double wr = yr[i] * yr[j] + yi[i] * yi[j];
          const double wi = yr[i] * yi[j] - yi[i] * yr[j];
          ar += ur * wr - ui * wi;
          const double sr = yr[i] * yr[j] - yi[i] * yi[j];
          const double si = yr[i] * yi[j] + yi[i] * yr[j];
          br += vr * sr - vi * si;
          bi += vr * si + vi * sr;
        }
      }
    }
    g[0 * NG * NG + gp] = 0.25 * ar;
    g[1 * NG * NG + gp] = 0.25 * br;
    g[2 * NG * NG + gp] = -0.25 * bi;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    int kind, n, q;
    basis_index(L, b, &kind, &n, &q);
    double acc[3] = {0.0, 0.0, 0.0};
    for (int gp = 0; gp < NG * NG; ++gp) {
      const int pi_ = gp / NG, pf = gp % NG;
      const double inc = two_pi * pi_ / NG, ph = two_pi * pf / NG;
      double t;
      if (kind == 0) t = cos(n * inc);
      else if (kind == 1) t = cos(n * inc) * cos(q * ph);
      else if (kind == 2) t = cos(n * inc) * sin(q * ph);
      else if (kind == 3) t = sin(n * inc) * cos(q * ph);
      else t = sin(n * inc) * sin(q * ph);
      for (int c = 0; c < 3; ++c) acc[c] += g[c * NG * NG + gp] * t;
    }
    const double nu_i = (n == 0) ? 1.0 : 0.5;
    const double nu_f = (q == 0) ? 1.0 : 0.5;
    const double norm = 1.0 / ((double)NG * NG * nu_i * nu_f);
    for (int c = 0; c < 3; ++c) {
      const double v = acc[c] * norm;
      C64[b * 3 * KT + 3 * k + c] = v;
      if (C32) C32[b * 3 * KT + 3 * k + c] = (float)v;
    }
  }
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int n, int32_t v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// out[i] = the a-priori bound of sample i's returned lnL: 0 where the value
// was recomputed in FP64 (its bound entry marked negative) or is FP64.
__global__ void k_bound_out(const float* __restrict__ bnd, double* __restrict__ out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = bnd ? fmax(0.0, (double)bnd[i]) : 0.0;
}

// Constants of the mixed path's a-priori error bound of one point (one
// thread; written into the point's device description).  With u = 2^-24 the
// FP32 unit roundoff, the FP32 pass starts from angles reduced to [-pi, pi]
// (rounding <= pi u / 2) and:
//  * antenna: F = D : (e+ + i ex), six products of polarisation-tensor
//    entries that carry a few u each (sincos, the FP64 -> FP32 cast of the sky
//    frame, two products and a difference), plus 2 |F| pi u / 2 from the
//    rounded psi: |F_FP32 - F| <= eF = 40 u sum|D| (D in its six-value form
//    with doubled off-diagonals, so that |F+|, |Fx| <= sum|D|, |F| <= 1.5 sum|D|);
//  * data term: every product F conj(Y) Qhat carries the table's rounding, the
//    Lagrange weights', Y's (Fourier series in incl of <= 9 terms, phase walk
//    of <= 16 steps), F's, and the (M K)-term accumulation: a bound of
//    2 (60 + M K) u |F| |Y| |Qhat| per term, with |Qhat| <= 1.25 max|Q|
//    (1.25 = largest sum of |Lagrange weights| on a cell) and |Y_i| <= the sum
//    of |Fourier coefficients| of mode i:
//      bnd_d = 2 * 1.25 (60 + M K) u  sum_k 1.5 sum|D_k| max|Q_k|  sum_i,n |ycoef_in|;
//  * model-norm term: quad_k = |F|^2 A + Re F^2 Br + Im F^2 Bi with
//    |A|, |Br|, |Bi| bounded by the sum of the basis coefficients' |C|
//    (|basis function| <= 1), whose FP32 contraction is off by at most
//    bnd_q = 2 (60 + B) u l1q (coefficient and basis-function rounding, the
//    Chebyshev and phase recurrences, the B-term sum); the FP32 weights |F|^2,
//    F^2 differ from the exact ones by <= (2 |F| + eF) eF.
__global__ void k_bound(PointDesc* __restrict__ P, const double* __restrict__ qmax) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double u = 5.9604644775390625e-08;  // 2^-24
  const int M = P->M, K = P->K, KT = P->KT, B = P->B;
  double ysum = 0.0;
  for (int i = 0; i < M; ++i)
    for (int n = 0; n <= LMAXC; ++n) ysum += fabs(P->ycoef[i][n]);
  double fq = 0.0;
  for (int k = 0; k < KT; ++k) {
    double dsum = 0.0;
    for (int a = 0; a < 6; ++a) dsum += fabs(P->dten[k][a]);
    if (k < K) fq += 1.5 * dsum * qmax[k];
    P->eF[k] = 40.0 * u * dsum;
    double l1 = 0.0;
    for (int b = 0; b < B; ++b)
      for (int c = 0; c < 3; ++c) l1 += fabs(P->C64[(size_t)b * 3 * KT + 3 * k + c]);
    P->l1q[k] = l1;
    P->bnd_q[k] = 2.0 * (60.0 + (double)B) * u * l1;
  }
  P->bnd_d = 2.0 * 1.25 * (60.0 + (double)M * K) * u * fq * ysum;
}

// Samples that may lie within T of the best go to the point's refine list;
// their bound is set to -1 to mark them.  Each block first reduces its
// point's M_low = max over the point's tiles of max(lnL32 + lnw - bound)
// (fixed order).
//
// A sample whose bound is at most `tau` is never listed: its FP32 value is
// already that close to the FP64 one (its share of the ln Z error is counted
// by k_final).  `T_over` >= 0 replaces the point's margin T.
__global__ void k_select(const PointDesc* __restrict__ descs, const Tile* __restrict__ tiles,
                         int n_tiles, const int32_t* __restrict__ trange, const double* __restrict__ tmax,
                         const double* __restrict__ lnL, const double* __restrict__ lnw,
                         float* __restrict__ bnd, int32_t* __restrict__ cnt,
                         int32_t* __restrict__ list, float tau, double T_over) {
  __shared__ double sh[8];
  const int tidx = blockIdx.x;
  if (tidx >= n_tiles) return;
  const Tile t = tiles[tidx];
  const PointDesc* P = descs + t.p;
  double m = -__builtin_inf();
  for (int u = trange[2 * t.p] + threadIdx.x; u < trange[2 * t.p + 1]; u += blockDim.x) m = fmax(m, tmax[u]);
  m = dmax_wave(m);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  m = sh[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, sh[w]);
  const double thr = m - (T_over >= 0.0 ? T_over : P->T);
  for (int o = threadIdx.x; o < t.cnt; o += blockDim.x) {
    const int64_t i = t.s + o;
    const float b = bnd[i];
    const double v = lnL[i] + (lnw ? lnw[i] : 0.0) + (double)b;
    // (a sample at -inf adds nothing, also when the whole point is at -inf)
    if (b > tau && v >= thr && v != -__builtin_inf()) {
      const int slot = atomicAdd(cnt + t.p, 1);
      list[P->s0 + slot] = (int32_t)(i - P->s0);
      bnd[i] = -1.0f;
    }
  }
}

// Mixed path: per tile, the maximum m_t of the final values, their sum
// relative to it, and the bound on what the unrefined samples can still be
// off by, also relative to m_t:
//   err_t = sum_{unrefined} exp(lnL32 + lnw - m_t) (e^{bound} - 1).
// With the maximum taken first, one exp per sample serves both sums.
__global__ void k_final(const Tile* __restrict__ tiles, const double* __restrict__ lnL,
                        const double* __restrict__ lnw, const float* __restrict__ bnd,
                        double* __restrict__ part, double* __restrict__ terr) {
  __shared__ double shm[8], shs[8], she[8];
  const int tidx = blockIdx.x;
  const Tile t = tiles[tidx];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double m = -__builtin_inf();  // fmax passes over NaN
  for (int o = threadIdx.x; o < t.cnt; o += blockDim.x) {
    const int64_t i = t.s + o;
    m = fmax(m, lnL[i] + (lnw ? lnw[i] : 0.0));
  }
  m = dmax_wave(m);
  if (lane == 0) shm[wave] = m;
  __syncthreads();
  m = shm[0];
  for (int w = 1; w < nw; ++w) m = fmax(m, shm[w]);
  double sum = 0.0, err = 0.0;
  if (m != __builtin_inf()) {
    for (int o = threadIdx.x; o < t.cnt; o += blockDim.x) {
      const int64_t i = t.s + o;
      const double l = lnL[i] + (lnw ? lnw[i] : 0.0);
      if (l != l) {
        sum += l;  // NaN poisons the sum
      } else if (l != -__builtin_inf()) {
        const double x = exp(l - m);
        sum += x;
        // e^{l - m} (e^b - 1), bounded by e^{l - m + b} where e^b alone
        // would overflow (a far-off sample with a wide bound: its term is tiny)
        const double b = (double)bnd[i];
        if (b > 0.0) err += (b < 30.0) ? x * expm1(b) : exp(l - m + b);
      }
    }
  } else {
    sum = __builtin_nan("");  // a value of +inf: ln Z is NaN, as on the FP64 path
  }
  sum = dsum_wave(sum);
  err = dsum_wave(err);
  if (lane == 0) {
    shs[wave] = sum;
    she[wave] = err;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sv = shs[0], e = she[0];
    for (int w = 1; w < nw; ++w) {
      sv += shs[w];
      e += she[w];
    }
    part[2 * tidx] = m;
    part[2 * tidx + 1] = sv;
    terr[tidx] = e;
  }
}

// Per point: combine tile partials in a fixed order -> ln Z, n_eff, and (with
// per-tile error terms relative to each tile's maximum) the error bound.
// The largest tile maximum M comes first; then every tile's sum and error
// term are scaled by exp(m_t - M), the exponentials independent of each other.
// Launched with 512 threads (at most 8 wavefronts: the per-wave slots below).
__global__ void k_merge(const PointDesc* __restrict__ descs, const int32_t* __restrict__ trange,
                        const double* __restrict__ part, const double* __restrict__ terr,
                        double* __restrict__ lnZ, double* __restrict__ neff, double* __restrict__ lnZ_err) {
  __shared__ double shm[8], shs[8], she[8];
  const int p = blockIdx.x;
  const int t0 = trange[2 * p], t1 = trange[2 * p + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double m = -__builtin_inf();
  for (int t = t0 + (int)threadIdx.x; t < t1; t += blockDim.x) m = fmax(m, part[2 * t]);
  m = dmax_wave(m);
  if (lane == 0) shm[wave] = m;
  __syncthreads();
  m = shm[0];
  for (int w = 1; w < nw; ++w) m = fmax(m, shm[w]);
  double sum = 0.0, err = 0.0;
  for (int t = t0 + (int)threadIdx.x; t < t1; t += blockDim.x) {
    const double st = part[2 * t + 1];
    const double et = terr ? terr[t] : 0.0;
    if (m == -__builtin_inf()) {
      sum += (st != st) ? st : 0.0;
    } else if (st != 0.0 || et != 0.0) {
      const double f = exp(part[2 * t] - m);
      sum += st * f;
      err += et * f;
    }
  }
  sum = dsum_wave(sum);
  err = dsum_wave(err);
  if (lane == 0) {
    shs[wave] = sum;
    she[wave] = err;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    MS r;
    r.m = m;
    r.s = shs[0];
    double e = she[0];
    for (int w = 1; w < nw; ++w) {
      r.s += shs[w];
      e += she[w];
    }
    const PointDesc* P = descs + p;
    double z;
    if (r.s != r.s) z = __builtin_nan("");
    else if (r.m == -__builtin_inf()) z = -__builtin_inf();
    else z = r.m + log(r.s) - P->lnN;
    lnZ[p] = z;
    if (neff) neff[p] = (r.m == -__builtin_inf() && r.s == r.s) ? 0.0 : r.s;
    if (lnZ_err) {
      double bound = 0.0;
      if (terr && r.s > 0.0) bound = log1p(e / r.s);
      lnZ_err[p] = bound;
    }
  }
}

// Exclusive scan of n int32 (three kernels): block sums, scan of the sums,
// per-block scan plus offset.  Each block covers SCAN_CHUNK elements.
constexpr int SCAN_T = 256, SCAN_PER = 16, SCAN_CHUNK = SCAN_T * SCAN_PER;

// sh: one slot per wavefront plus one (the total)
__device__ __forceinline__ int32_t block_excl_scan(int32_t v, int32_t* sh, int32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int32_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t acc = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      const int32_t t = sh[w];
      sh[w] = acc;
      acc += t;
    }
    sh[blockDim.x >> 6] = acc;
  }
  __syncthreads();
  const int32_t r = x - v + sh[wave];
  *total = sh[blockDim.x >> 6];
  __syncthreads();
  return r;
}

__global__ void k_scan_sums(const int32_t* __restrict__ a, int64_t n, int32_t* __restrict__ sums) {
  __shared__ int32_t sh[9];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER;
  int32_t v = 0;
  for (int j = 0; j < SCAN_PER; ++j)
    if (base + j < n) v += a[base + j];
  int32_t tot;
  block_excl_scan(v, sh, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void k_scan_top(int32_t* __restrict__ sums, int nb) {
  // one block: exclusive scan of nb block sums, in chunks of the block size
  __shared__ int32_t sh[9];
  int32_t carry = 0;
  for (int b0 = 0; b0 < nb; b0 += blockDim.x) {
    const int j = b0 + threadIdx.x;
    const int32_t v = (j < nb) ? sums[j] : 0;
    int32_t tot;
    const int32_t e = block_excl_scan(v, sh, &tot);
    if (j < nb) sums[j] = carry + e;
    carry += tot;
  }
}

// (may run in place: out == a)
__global__ void k_scan_apply(const int32_t* a, int64_t n, const int32_t* __restrict__ sums, int32_t* out,
                             int32_t* __restrict__ out2) {
  __shared__ int32_t sh[9];
  const int64_t base = (int64_t)blockIdx.x * SCAN_CHUNK + (int64_t)threadIdx.x * SCAN_PER;
  int32_t loc[SCAN_PER];
  int32_t v = 0;
  for (int j = 0; j < SCAN_PER; ++j) {
    loc[j] = (base + j < n) ? a[base + j] : 0;
    v += loc[j];
  }
  int32_t tot;
  int32_t e = block_excl_scan(v, sh, &tot) + sums[blockIdx.x];
  for (int j = 0; j < SCAN_PER; ++j) {
    if (base + j < n) {
      out[base + j] = e;
      if (out2) out2[base + j] = e;
    }
    e += loc[j];
  }
}

// ---------------------------------------------------------------------------
// Arrival-time binning: the samples of each point are sorted by a Morton key
// of their stencil rows at (up to) three detectors, so that the 64 lanes of a
// wavefront read nearby rows of every Q series.  The binned batch is a copy
// of theta as 64-byte records (ra, dec, psi, incl, phiref, tref, dist, and
// sample index << 16 in the last slot), which the evaluation kernel reads in
// order.
//
// No device-scope atomics (they serialise across the XCDs) and no random
// gathers (a scattered 8-byte read costs a whole cache line):
//   k_bin_range   per sort tile: stencil coordinates (FP32; they only decide
//                 the order) and their range;
//   k_bin_hist    per sort tile: the point's range, the key of every sample,
//                 and the tile's coarse-bucket histogram -> column of the
//                 point's [coarse bucket][sort tile] count matrix;
//   k_scan_*      exclusive scan of the count matrix (positions);
//   k_bin_coarse  per sort tile: every record to the next slot of its coarse
//                 bucket (LDS cursors; theta read in input order);
//   k_bin_chunk   per chunk of 2048 coarse-ordered records: counting sort by
//                 the key in LDS, records moved to their final positions.
// The order inside a cell is not fixed; lnL values do not depend on it and
// every reduction runs in input order.
// ---------------------------------------------------------------------------
constexpr int BIN_TILE = 4096;   // samples per sort tile
constexpr int BIN_T = 1024;      // threads of the sort kernels
constexpr int BIN_CB_MAX = 10;   // coarse buckets per point <= 1024

// Stencil row coordinate u_k = (t_k - t0)/dt of the first bin_dims detectors
// per sample (FP32), and its range per sort tile.
__global__ void __launch_bounds__(BIN_T) k_bin_range(const PointDesc* __restrict__ descs,
                                                     const Tile* __restrict__ stiles,
                                                     const double* __restrict__ theta, int64_t N,
                                                     float* __restrict__ ucoord,
                                                     float* __restrict__ rpart) {
  const Tile t = stiles[blockIdx.x];
  const PointDesc* P = descs + t.p;
  const int D = P->bin_dims;
  const float gmst = (float)P->gmst, t0 = (float)P->t0, idt = (float)P->inv_dt;
  float rp[3][3];
  for (int k = 0; k < 3; ++k)
    for (int c = 0; c < 3; ++c) rp[k][c] = (k < D) ? (float)P->rpos[k][c] : 0.0f;
  float lo[3] = {__builtin_inff(), __builtin_inff(), __builtin_inff()};
  float hi[3] = {-__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
  for (int o = threadIdx.x; o < t.cnt; o += blockDim.x) {
    const int64_t i = t.s + o;
    float sg, cg, sd, cd;
    __sincosf(gmst - (float)theta[i], &sg, &cg);
    __sincosf((float)theta[N + i], &sd, &cd);
    const float N0 = cd * cg, N1 = -cd * sg, N2 = sd;
    const float tr = (float)theta[5 * N + i];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (k >= D) break;
      const float tk = tr - (rp[k][0] * N0 + rp[k][1] * N1 + rp[k][2] * N2);
      const float u = (tk - t0) * idt;
      ucoord[3 * i + k] = u;
      if (u == u && fabsf(u) < 1e9f) {
        lo[k] = fminf(lo[k], u);
        hi[k] = fmaxf(hi[k], u);
      }
    }
  }
  __shared__ float sh[2][3][BIN_T / 64];
  for (int k = 0; k < 3; ++k) {
    float a = lo[k], b = hi[k];
    for (int off = 32; off >= 1; off >>= 1) {
      a = fminf(a, __shfl_xor(a, off));
      b = fmaxf(b, __shfl_xor(b, off));
    }
    if ((threadIdx.x & 63) == 0) {
      sh[0][k][threadIdx.x >> 6] = a;
      sh[1][k][threadIdx.x >> 6] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int k = threadIdx.x;
    float a = sh[0][k][0], b = sh[1][k][0];
    for (int w = 1; w < BIN_T / 64; ++w) {
      a = fminf(a, sh[0][k][w]);
      b = fmaxf(b, sh[1][k][w]);
    }
    rpart[6 * blockIdx.x + 2 * k] = a;
    rpart[6 * blockIdx.x + 2 * k + 1] = b;
  }
}

// Keys and the coarse histogram of every sort tile, written to column
// (tile - bin_st0) of the point's [coarse bucket][sort tile] matrix.  Each
// block first reduces the point's range from the tile partials (fixed order).
__global__ void __launch_bounds__(BIN_T) k_bin_hist(const PointDesc* __restrict__ descs,
                                                    const Tile* __restrict__ stiles,
                                                    const float* __restrict__ ucoord,
                                                    const float* __restrict__ rpart,
                                                    uint16_t* __restrict__ key,
                                                    int32_t* __restrict__ mat) {
  __shared__ int32_t h[1 << BIN_CB_MAX];
  __shared__ float rng[6][BIN_T / 64];
  const Tile t = stiles[blockIdx.x];
  const PointDesc* P = descs + t.p;
  const int D = P->bin_dims, bits = P->bin_bits;
  const int tb = D * bits, cb = P->bin_cb;
  const int nc = 1 << cb;
  for (int c = threadIdx.x; c < nc; c += blockDim.x) h[c] = 0;
  {
    const int t0 = P->bin_st0, nt = P->bin_nst;
    for (int c = 0; c < 6; ++c) {
      const bool mx = c & 1;
      float v = mx ? -__builtin_inff() : __builtin_inff();
      for (int j = threadIdx.x; j < nt; j += blockDim.x)
        v = mx ? fmaxf(v, rpart[6 * (t0 + j) + c]) : fminf(v, rpart[6 * (t0 + j) + c]);
      for (int off = 32; off >= 1; off >>= 1) {
        const float o = __shfl_xor(v, off);
        v = mx ? fmaxf(v, o) : fminf(v, o);
      }
      if ((threadIdx.x & 63) == 0) rng[c][threadIdx.x >> 6] = v;
    }
  }
  __syncthreads();
  float lo[3], scl[3];
  const int ncell = 1 << bits;
  for (int k = 0; k < 3; ++k) {
    float a = rng[2 * k][0], b = rng[2 * k + 1][0];
    for (int w = 1; w < BIN_T / 64; ++w) {
      a = fminf(a, rng[2 * k][w]);
      b = fmaxf(b, rng[2 * k + 1][w]);
    }
    lo[k] = (a <= b) ? a : 0.0f;
    scl[k] = (a <= b) ? (float)ncell / (b - a + 1e-3f) : 0.0f;
  }
  for (int o = threadIdx.x; o < t.cnt; o += blockDim.x) {
    const int64_t i = t.s + o;
    uint32_t k = 0;
    for (int d = 0; d < D; ++d) {
      const float f = (ucoord[3 * i + d] - lo[d]) * scl[d];
      const int c = (f >= 0.0f) ? (f < (float)(ncell - 1) ? (int)f : ncell - 1) : 0;  // NaN -> 0
      // Morton interleave: detector d at bit positions d, d + D, d + 2D, ...
      for (int bb = 0; bb < bits; ++bb) k |= (((uint32_t)c >> bb) & 1u) << (D * bb + d);
    }
    key[i] = (uint16_t)k;
    atomicAdd(&h[k >> (tb - cb)], 1);
  }
  __syncthreads();
  const int64_t col = blockIdx.x - P->bin_st0;
  for (int c = threadIdx.x; c < nc; c += blockDim.x) mat[P->bin_mbase + (int64_t)c * P->bin_nst + col] = h[c];
}

// Coarse scatter: every sample of a sort tile takes the next slot of its
// coarse bucket in this tile's range (LDS cursors) and its record goes there,
// with (sample index << 16 | key) in the last slot.  Slots are global sample
// positions (the scanned matrix starts each point at its first column).
__global__ void __launch_bounds__(BIN_T) k_bin_coarse(const PointDesc* __restrict__ descs,
                                                      const Tile* __restrict__ stiles,
                                                      const uint16_t* __restrict__ key,
                                                      const int32_t* __restrict__ mat,
                                                      const double* __restrict__ theta, int64_t N,
                                                      double* __restrict__ trec) {
  __shared__ int32_t cur[1 << BIN_CB_MAX];
  const Tile t = stiles[blockIdx.x];
  const PointDesc* P = descs + t.p;
  const int tb = P->bin_dims * P->bin_bits, cb = P->bin_cb;
  const int nc = 1 << cb;
  const int64_t col = blockIdx.x - P->bin_st0;
  for (int c = threadIdx.x; c < nc; c += blockDim.x) cur[c] = mat[P->bin_mbase + (int64_t)c * P->bin_nst + col];
  __syncthreads();
  for (int o = threadIdx.x; o < t.cnt; o += blockDim.x) {
    const int64_t i = t.s + o;
    const uint32_t k = key[i];
    const int64_t slot = atomicAdd(&cur[k >> (tb - cb)], 1);
    const long long tag = ((long long)i << 16) | (long long)k;
    double2* dst = reinterpret_cast<double2*>(trec + 8 * slot);
    dst[0] = make_double2(theta[i], theta[N + i]);
    dst[1] = make_double2(theta[2 * N + i], theta[3 * N + i]);
    dst[2] = make_double2(theta[4 * N + i], theta[5 * N + i]);
    dst[3] = make_double2(theta[6 * N + i], __longlong_as_double(tag));
  }
}

// Fine order: the coarse-ordered records of each point are cut into chunks
// of BIN_CHUNK; each block counting-sorts one chunk by its key offset from
// the chunk's smallest key (LDS histogram) and moves the records to their
// places.  Every block does the same work whatever the key distribution.  A
// chunk whose keys span more than BIN_SPAN values (several sparse coarse
// cells, each already small) keeps its coarse order.
constexpr int BIN_CT = 256;
constexpr int BIN_CPER = 8;
constexpr int BIN_CHUNK = BIN_CT * BIN_CPER;
constexpr int BIN_SPAN = 4096;
__global__ void __launch_bounds__(BIN_CT) k_bin_chunk(const Tile* __restrict__ chunks,
                                                      const double* __restrict__ trec,
                                                      double* __restrict__ aos) {
  __shared__ int32_t h[BIN_SPAN];
  __shared__ int32_t ws[BIN_CT / 64 + 1];
  __shared__ uint32_t mm[2][BIN_CT / 64];
  const Tile t = chunks[blockIdx.x];
  uint32_t kk[BIN_CPER];
  uint32_t lo = 0xffffffffu, hi = 0u;
#pragma unroll
  for (int j = 0; j < BIN_CPER; ++j) {
    const int q = j * BIN_CT + threadIdx.x;
    kk[j] = 0;
    if (q < t.cnt) {
      kk[j] = (uint32_t)(__double_as_longlong(trec[8 * (t.s + q) + 7]) & 0xffff);
      lo = min(lo, kk[j]);
      hi = max(hi, kk[j]);
    }
  }
  for (int off = 32; off >= 1; off >>= 1) {
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, off));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, off));
  }
  if ((threadIdx.x & 63) == 0) {
    mm[0][threadIdx.x >> 6] = lo;
    mm[1][threadIdx.x >> 6] = hi;
  }
  for (int b = threadIdx.x; b < BIN_SPAN; b += BIN_CT) h[b] = 0;
  __syncthreads();
  lo = mm[0][0];
  hi = mm[1][0];
  for (int w = 1; w < BIN_CT / 64; ++w) {
    lo = min(lo, mm[0][w]);
    hi = max(hi, mm[1][w]);
  }
  const bool sort = hi >= lo && hi - lo < (uint32_t)BIN_SPAN;
  int32_t dst[BIN_CPER];
  if (sort) {
#pragma unroll
    for (int j = 0; j < BIN_CPER; ++j)
      if (j * BIN_CT + (int)threadIdx.x < t.cnt) atomicAdd(&h[kk[j] - lo], 1);
    __syncthreads();
    // exclusive scan of the BIN_SPAN bins (each thread a contiguous run)
    constexpr int per = BIN_SPAN / BIN_CT;
    const int b0 = threadIdx.x * per;
    int32_t run = 0;
#pragma unroll
    for (int b = 0; b < per; ++b) run += h[b0 + b];
    int32_t tot;
    int32_t off = block_excl_scan(run, ws, &tot);
#pragma unroll
    for (int b = 0; b < per; ++b) {
      const int32_t v = h[b0 + b];
      h[b0 + b] = off;
      off += v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < BIN_CPER; ++j)
      dst[j] = (j * BIN_CT + (int)threadIdx.x < t.cnt) ? atomicAdd(&h[kk[j] - lo], 1) : 0;
  } else {
#pragma unroll
    for (int j = 0; j < BIN_CPER; ++j) dst[j] = j * BIN_CT + threadIdx.x;
  }
#pragma unroll
  for (int j = 0; j < BIN_CPER; ++j) {
    const int q = j * BIN_CT + threadIdx.x;
    if (q < t.cnt) {
      const double2* from = reinterpret_cast<const double2*>(trec + 8 * (t.s + q));
      double2* to = reinterpret_cast<double2*>(aos + 8 * (t.s + dst[j]));
#pragma unroll
      for (int c = 0; c < 4; ++c) to[c] = from[c];
    }
  }
}

// Per-tile (max, sum) over lnL + lnw in input order (deterministic).
__global__ void k_lse_tiles(const Tile* __restrict__ tiles, const double* __restrict__ lnL,
                            const double* __restrict__ lnw, double* __restrict__ part) {
  __shared__ MS sh[8];
  const Tile t = tiles[blockIdx.x];
  MS acc;
  acc.m = -__builtin_inf();
  acc.s = 0.0;
  for (int o = threadIdx.x; o < t.cnt; o += blockDim.x) {
    const int64_t i = t.s + o;
    acc = ms_push(acc, lnL[i] + (lnw ? lnw[i] : 0.0));
  }
  const MS r = ms_block(acc, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r.m;
    part[2 * blockIdx.x + 1] = r.s;
  }
}

// The band-limited full-window rule over geocentric time (Eq. (ap:tband)),
// after the data pass: x kappa at the n nodes t0 + j h of every sample is
// reconstructed at the fine points t0 + (k / M) h, k = 0 .. (n - 1) M, by the
// sinc series sum_j x kappa_j sinc(k / M - j), the time-independent remainder
// is added and the exponentials are summed by the trapezoid rule under a
// prior uniform on the window:
//   ln L_t = ln[(1 / ((n - 1) M)) sum_k w_k e^{l_k}], w = 1, ends 1/2.
// The sinc weights depend on (k mod M, k div M - j) only: a table
// tab[s][d + NB - 1] = sinc(d + s / M), |d| < NB, read with uniform indices.
constexpr int TBAND_MAX_NODES = 64;
constexpr int TBAND_MAX_FINE = 64;

// sin(pi (d + f)) = (-1)^d sin(pi f): exact zeros at the nodes (s = 0).
__global__ void k_sinc_table(int NB, int M, double* __restrict__ tab) {
  const int W = 2 * NB - 1;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < M * W; e += gridDim.x * blockDim.x) {
    const int s = e / W, d = e - s * W - (NB - 1);
    double v;
    if (s == 0) {
      v = d == 0 ? 1.0 : 0.0;
    } else {
      const double f = (double)s / (double)M;
      v = ((d & 1) ? -1.0 : 1.0) * sinpi(f) / (3.14159265358979323846 * ((double)d + f));
    }
    tab[e] = v;
  }
}

// One sample per lane; NB >= n nodes held in registers (zero past n, so the
// unrolled sums need no bounds).  The fine points run by sub-offset s, whose
// table row is staged in LDS, then in blocks of eight consecutive node
// intervals, whose sums share the row's reads T_s[ii + q - j] (the same
// address in every lane: broadcast reads).  The sample loop is uniform per
// block (the staging synchronises).  L holds the remainder on entry and
// ln L_t on return.
constexpr int TBAND_BLK = 8;
template <int NB>
__global__ void __launch_bounds__(256) k_tband(int64_t N, int n, int M, const double* __restrict__ kap,
                                               const double* __restrict__ tab, double ln_scale,
                                               double* __restrict__ L) {
  constexpr int W = 2 * NB - 1;
  __shared__ double row[W + TBAND_BLK];
  for (int64_t ib = blockIdx.x * (int64_t)blockDim.x; ib < N; ib += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = ib + threadIdx.x;
    const bool live = i < N;
    double y[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) y[j] = (live && j < n) ? kap[(int64_t)j * N + i] : 0.0;
    const double base = live ? L[i] : 0.0;
    double m = -__builtin_inf(), sum = 0.0;
    for (int s = 0; s < M; ++s) {
      __syncthreads();
      for (int e = threadIdx.x; e < W + TBAND_BLK; e += blockDim.x) row[e] = e < W ? tab[s * W + e] : 0.0;
      __syncthreads();
      // fine points ii M + s <= (n - 1) M
      const int last = s == 0 ? n - 1 : n - 2;
      for (int ii = 0; ii <= last; ii += TBAND_BLK) {
        const double* T = row + (NB - 1) + ii;  // T[q - j] = sinc(ii + q - j + s / M)
        double v[TBAND_BLK];
#pragma unroll
        for (int q = 0; q < TBAND_BLK; ++q) v[q] = 0.0;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
#pragma unroll
          for (int q = 0; q < TBAND_BLK; ++q) v[q] = fma(y[j], T[q - j], v[q]);
        }
#pragma unroll
        for (int q = 0; q < TBAND_BLK; ++q) {
          if (ii + q > last) break;
          const bool end = s == 0 && (ii + q == 0 || ii + q == n - 1);
          const double l = v[q] + base + (end ? -0.69314718055994530942 : 0.0);
          // one exp and no divergent branch: e = exp(-|l - m|) rescales the
          // sum when l is the new maximum and is the new term otherwise (the
          // first point: m = -inf, e = 0, sum = 1); a NaN l poisons the sum
          const double d = l - m;
          const double e = exp(-fabs(d));
          const bool up = d > 0.0;
          sum = up ? fma(sum, e, 1.0) : sum + e;
          m = up ? l : m;
        }
      }
    }
    if (live) L[i] = (m == m && sum == sum) ? m + log(sum) + ln_scale : __builtin_nan("");
  }
}

// The joint phiref / psi marginal by exact reconstruction (ERAI), after the
// data pass: per sample the angular coefficients at their sampling angles
// (c1 at nd = 2 m_max + 1, a and c2 at nq = 4 m_max + 1 angles) determine
//   q(alpha, u) = a(alpha) + Re(c1(alpha) e^{iu}) + Re(c2(alpha) e^{2iu})
// exactly; e^q is averaged over the periodic grid alpha_a = 2 pi a / n_phi,
// u_b = 2 pi b / n_psi (psi offset pi b / n_psi), the trapezoid rule on the
// torus with phiref uniform on [0, 2 pi) and psi on [0, pi).
constexpr int ERAI_MAX_M = 4;

// (a N - j n) / (n N) turns between fine angle a of n and sampling angle j
// of N; the Dirichlet kernel of odd N, sin(pi N d) / (N sin(pi d)), is 1 at
// the coincident angles (tested exactly on integers).
__device__ __forceinline__ double dirichlet_weight(int a, int n, int j, int N) {
  const int64_t num = (int64_t)a * N - (int64_t)j * n;
  if (num % ((int64_t)n * N) == 0) return 1.0;
  return sinpi((double)num / (double)n) / ((double)N * sinpi((double)num / ((double)n * (double)N)));
}

// Uniform tables: interpolation weights wd [n_phi][NDM] and wq [n_phi][NQM]
// (zero past nd, nq), and tu [n_psi][4] = cos u, sin u, cos 2u, sin 2u.
__global__ void k_erai_tables(int n_phi, int n_psi, int nd, int nq, int NDM, int NQM, double* __restrict__ wd,
                              double* __restrict__ wq, double* __restrict__ tu) {
  const int stride = gridDim.x * blockDim.x;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n_phi * NDM; e += stride) {
    const int a = e / NDM, j = e - a * NDM;
    wd[e] = j < nd ? dirichlet_weight(a, n_phi, j, nd) : 0.0;
  }
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n_phi * NQM; e += stride) {
    const int a = e / NQM, j = e - a * NQM;
    wq[e] = j < nq ? dirichlet_weight(a, n_phi, j, nq) : 0.0;
  }
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < n_psi; b += stride) {
    double s1, c1, s2, c2;
    sincospi(2.0 * (double)b / (double)n_psi, &s1, &c1);
    sincospi(4.0 * (double)b / (double)n_psi, &s2, &c2);
    tu[4 * b] = c1;
    tu[4 * b + 1] = s1;
    tu[4 * b + 2] = c2;
    tu[4 * b + 3] = s2;
  }
}

// One sample per lane, its coefficients in registers (zero past nd, nq);
// the grid loops are uniform, the tables read with uniform addresses.  L
// holds NaN (poisoned) or 0 on entry and ln L_{phi psi} on return.
template <int NDM, int NQM>
__global__ void __launch_bounds__(256) k_erai(int64_t N, int nd, int nq, int n_phi, int n_psi,
                                              const double* __restrict__ ang, const double* __restrict__ wd,
                                              const double* __restrict__ wq, const double* __restrict__ tu,
                                              double ln_scale, double* __restrict__ L) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    double c1r[NDM], c1i[NDM], ca[NQM], c2r[NQM], c2i[NQM];
#pragma unroll
    for (int j = 0; j < NDM; ++j) {
      c1r[j] = j < nd ? ang[(int64_t)(2 * j) * N + i] : 0.0;
      c1i[j] = j < nd ? ang[(int64_t)(2 * j + 1) * N + i] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < NQM; ++j) {
      const int64_t r = 2 * nd + 3 * j;
      ca[j] = j < nq ? ang[r * N + i] : 0.0;
      c2r[j] = j < nq ? ang[(r + 1) * N + i] : 0.0;
      c2i[j] = j < nq ? ang[(r + 2) * N + i] : 0.0;
    }
    const double flag = L[i];
    double m = -__builtin_inf(), sum = 0.0;
    for (int p = 0; p < n_phi; ++p) {
      const double* __restrict__ Wd = wd + p * NDM;
      const double* __restrict__ Wq = wq + p * NQM;
      double C1r = 0.0, C1i = 0.0, A = 0.0, C2r = 0.0, C2i = 0.0;
#pragma unroll
      for (int j = 0; j < NDM; ++j) {
        C1r = fma(Wd[j], c1r[j], C1r);
        C1i = fma(Wd[j], c1i[j], C1i);
      }
#pragma unroll
      for (int j = 0; j < NQM; ++j) {
        A = fma(Wq[j], ca[j], A);
        C2r = fma(Wq[j], c2r[j], C2r);
        C2i = fma(Wq[j], c2i[j], C2i);
      }
      for (int b = 0; b < n_psi; ++b) {
        const double* __restrict__ U = tu + 4 * b;
        const double l = A + C1r * U[0] - C1i * U[1] + C2r * U[2] - C2i * U[3];
        // one exp, no divergent branch (as in k_tband)
        const double d = l - m;
        const double e = exp(-fabs(d));
        const bool up = d > 0.0;
        sum = up ? fma(sum, e, 1.0) : sum + e;
        m = up ? l : m;
      }
    }
    L[i] = (flag == flag && m == m && sum == sum) ? m + log(sum) + ln_scale : __builtin_nan("");
  }
}

// Per-tile max(lnL32 + lnw - bound) in input order (mixed path).
__global__ void k_tmax_tiles(const Tile* __restrict__ tiles, const double* __restrict__ lnL,
                             const double* __restrict__ lnw, const float* __restrict__ bnd,
                             double* __restrict__ tmax) {
  __shared__ double shd[8];
  const Tile t = tiles[blockIdx.x];
  double m = -__builtin_inf();
  for (int o = threadIdx.x; o < t.cnt; o += blockDim.x) {
    const int64_t i = t.s + o;
    const double v = lnL[i] + (lnw ? lnw[i] : 0.0) - (double)bnd[i];
    if (v == v) m = fmax(m, v);
  }
  m = dmax_wave(m);
  if ((threadIdx.x & 63) == 0) shd[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = shd[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, shd[w]);
    tmax[blockIdx.x] = r;
  }
}

// ---------------------------------------------------------------------------
// Host helpers
// ---------------------------------------------------------------------------
#define HCHK(x)                                   \
  do {                                            \
    hipError_t e_ = (x);                          \
    if (e_ != hipSuccess) return RIFT_EDEVICE;    \
  } while (0)

inline int kt_class(int K) { return K <= 2 ? 2 : (K <= 3 ? 3 : (K <= 5 ? 5 : 8)); }
inline int l_class(int lmax) { return lmax <= 2 ? 2 : (lmax <= 3 ? 3 : (lmax <= 4 ? 4 : 8)); }
inline int lbit(int L) { return L == 2 ? 1 : (L == 3 ? 2 : (L == 4 ? 4 : 8)); }

struct DeviceInfo {
  int dev = -1;
  int n_cu = 0;
  int max_lds = 0;  // LDS bytes per block
};

int device_info(DeviceInfo* di) {
  HCHK(hipGetDevice(&di->dev));
  HCHK(hipDeviceGetAttribute(&di->n_cu, hipDeviceAttributeMultiprocessorCount, di->dev));
  HCHK(hipDeviceGetAttribute(&di->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, di->dev));
  return RIFT_OK;
}

int validate_point(const rift_ile_point* pt) {
  if (!pt) return RIFT_EINVAL;
  if (pt->n_det < 1 || pt->n_det > RIFT_ILE_MAX_DET) return RIFT_EINVAL;
  if (pt->n_modes < 1 || pt->n_modes > RIFT_ILE_MAX_MODES) return RIFT_EINVAL;
  // stencil offsets inside a series are 32-bit byte offsets of 32-byte rows
  if (pt->n_t < 4 || pt->n_t > RIFT_ILE_MAX_NT) return RIFT_EINVAL;
  if ((int64_t)pt->n_t * pt->n_modes * RIFT_ILE_MAX_DET > ((int64_t)1 << 40)) return RIFT_EINVAL;
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
  for (int k = 0; k < pt->n_det; ++k) {
    for (int a = 0; a < 9; ++a)
      if (!std::isfinite(pt->det_tensor[9 * k + a])) return RIFT_EINVAL;
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(pt->det_pos[3 * k + a])) return RIFT_EINVAL;
  }
  return RIFT_OK;
}

int check_dev_ptr(const void* p) { return (p && (((uintptr_t)p) & 7u) == 0) ? RIFT_OK : RIFT_EINVAL; }

// Mixed path: a sample whose a-priori bound is at most kRefineTau nats keeps
// its FP32 value; rift_ile_lnL recomputes every other sample that can lie
// within kPosteriorMargin nats of the best one (the posterior-relevant set).
constexpr double kRefineTau = 1.0e-4;
constexpr double kPosteriorMargin = 20.0;

// Blocks of 256 threads for an elementwise pass over n entries (grid-stride).
unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096)); }

// Rough relative cost per sample of a point (for tile ordering).
double point_cost(int KT, int L, int M) {
  return 200.0 + 12.0 * M * KT + 3.0 * KT * basis_count(L);
}

}  // namespace

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
struct rift_ile_plan_s {
  int n_points = 0;
  int prec = RIFT_FP64;
  DeviceInfo di;
  int KT = 2;
  int lset = 0;
  int64_t N = 0;
  std::vector<int64_t> n_per;
  std::vector<PointDesc> h_desc;
  PointDesc* d_desc = nullptr;
  std::vector<void*> bufs;  // device allocations owned by the plan
  // allocation-free plans: every buffer is carved from a fixed device region
  char* arena = nullptr;
  size_t arena_cap = 0;
  size_t arena_off = 0;
  // tiles (depend on the config)
  rift_ile_config cfg{256, 4, 0, 0};
  std::vector<Tile> h_tiles;
  Tile* d_tiles = nullptr;
  int n_tiles = 0;
  int32_t* d_trange = nullptr;  // [n_points][2]
  double* d_part = nullptr;     // [n_tiles][2]
  double* d_tmax = nullptr;     // [n_tiles]
  double* d_terr = nullptr;     // [n_tiles]
  int32_t* d_counter = nullptr;
  // mixed scratch
  int32_t* d_cnt = nullptr;   // [n_points]
  int32_t* d_list = nullptr;  // [N]
  float* d_bnd = nullptr;     // [N]
  double* d_L = nullptr;      // [N]
  int refine_blocks = 32;
  // binning (sorted evaluation), see k_bin_*
  bool bin_ready = false;          // buffers below allocated (on first use of sort)
  std::vector<Tile> h_stiles;
  std::vector<Tile> h_chunks;      // BIN_CHUNK-record chunks of every point
  int n_stiles = 0;
  Tile* d_stiles = nullptr;        // sort tiles of BIN_TILE samples
  int64_t n_mat = 0;               // [coarse bucket][sort tile] entries, all points
  float* d_ucoord = nullptr;       // [N][3]
  float* d_rpart = nullptr;        // [n_stiles][6]
  uint16_t* d_key = nullptr;       // [N]
  int32_t* d_mat = nullptr;        // [n_mat]
  int32_t* d_scan = nullptr;       // block sums of the matrix scan
  double* d_trec = nullptr;        // [N][8] records after the coarse scatter
  Tile* d_chunks = nullptr;        // fine-sort chunks
  int n_chunks = 0;
  double* d_aos = nullptr;         // [N][8] records in binned order
  hipStream_t last = nullptr;
  // optional timing of the main evaluation kernel
  bool profiling = false;
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  // distance marginal: the rule of the last rift_ile_plan_lnZ_dmarg call
  DistRule dm{};
  // time marginal: the rule of the last rift_ile_plan_lnZ_tmarg call
  TimeRule tm{};
  // polarisation marginal: the rule of the last rift_ile_plan_lnZ_pmarg call
  PsiRule pm{};
  double* kap = nullptr;  // band-limited time rule: x kappa at the nodes (stream-ordered, per call)
  AngleRule am{};
  double* ang = nullptr;  // ERAI: the angular coefficients (stream-ordered, per call)
};

namespace {

int palloc(rift_ile_plan p, size_t bytes, void** out) {
  if (p->arena) {
    const size_t off = (p->arena_off + 255) & ~(size_t)255;
    const size_t len = bytes < 256 ? 256 : bytes;
    if (off > p->arena_cap || len > p->arena_cap - off) return RIFT_ESCRATCH;
    *out = p->arena + off;
    p->arena_off = off + len;
    return RIFT_OK;
  }
  void* d = nullptr;
  if (hipMalloc(&d, bytes < 256 ? 256 : bytes) != hipSuccess) return RIFT_ENOMEM;
  p->bufs.push_back(d);
  *out = d;
  return RIFT_OK;
}

void plan_free_all(rift_ile_plan p) {
  for (void* b : p->bufs) (void)hipFree(b);
  p->bufs.clear();
}

int build_tiles(rift_ile_plan p) {
  const int S = p->cfg.block * p->cfg.tile_blocks;
  // points in decreasing cost per sample; each point's tiles are contiguous
  std::vector<int> order(p->n_points);
  for (int i = 0; i < p->n_points; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const PointDesc &A = p->h_desc[a], &Bd = p->h_desc[b];
    return point_cost(A.KT, A.L, A.M) > point_cost(Bd.KT, Bd.L, Bd.M);
  });
  std::vector<int32_t> trange(2 * p->n_points);
  p->h_tiles.clear();
  for (int oi = 0; oi < p->n_points; ++oi) {
    const int pi = order[oi];
    const PointDesc& D = p->h_desc[pi];
    trange[2 * pi] = (int32_t)p->h_tiles.size();
    for (int64_t s = 0; s < D.n; s += S) {
      Tile t;
      t.p = pi;
      t.cnt = (int32_t)std::min<int64_t>(S, D.n - s);
      t.s = D.s0 + s;
      p->h_tiles.push_back(t);
    }
    trange[2 * pi + 1] = (int32_t)p->h_tiles.size();
  }
  if (p->h_tiles.size() > (size_t)0x7fffffff) return RIFT_EUNSUPPORTED;
  p->n_tiles = (int)p->h_tiles.size();
  // release the previous tiling's buffers (the caller has synchronised)
  for (void* b : {(void*)p->d_tiles, (void*)p->d_trange, (void*)p->d_part, (void*)p->d_tmax, (void*)p->d_terr}) {
    auto it = std::find(p->bufs.begin(), p->bufs.end(), b);
    if (b && it != p->bufs.end()) {
      (void)hipFree(b);
      p->bufs.erase(it);
    }
  }
  // (re)allocate tile-sized buffers
  void* v;
  int st;
  if ((st = palloc(p, sizeof(Tile) * p->n_tiles, &v))) return st;
  p->d_tiles = (Tile*)v;
  if ((st = palloc(p, sizeof(int32_t) * 2 * p->n_points, &v))) return st;
  p->d_trange = (int32_t*)v;
  if ((st = palloc(p, sizeof(double) * 2 * p->n_tiles, &v))) return st;
  p->d_part = (double*)v;
  if ((st = palloc(p, sizeof(double) * p->n_tiles, &v))) return st;
  p->d_tmax = (double*)v;
  if ((st = palloc(p, sizeof(double) * p->n_tiles, &v))) return st;
  p->d_terr = (double*)v;
  HCHK(hipMemcpy(p->d_tiles, p->h_tiles.data(), sizeof(Tile) * p->n_tiles, hipMemcpyHostToDevice));
  HCHK(hipMemcpy(p->d_trange, trange.data(), sizeof(int32_t) * 2 * p->n_points, hipMemcpyHostToDevice));
  return RIFT_OK;
}

// Kernel tables -------------------------------------------------------------
tile_fn pick_tiles_kt(int mode, int KT, int lset) {
#define RIFT_PICK(K)                                 \
  switch (mode) {                                    \
    case MODE_LSE64: return get_tiles64_kt##K(lset); \
    case MODE_PASS32: return get_tiles32_kt##K(lset); \
    case MODE_DMARG64: return get_tilesdm_kt##K(lset); \
    case MODE_TMARG64: return get_tilestm_kt##K(lset); \
    case MODE_TBAND64: return get_tilestb_kt##K(lset); \
    case MODE_ERAI64: return get_tilesea_kt##K(lset); \
    default: return get_tilespm_kt##K(lset);         \
  }
  switch (KT) {
    case 2: RIFT_PICK(2)
    case 3: RIFT_PICK(3)
    case 5: RIFT_PICK(5)
    default: RIFT_PICK(8)
  }
#undef RIFT_PICK
}
refine_fn pick_refine_kt(int KT, int lset) {
  switch (KT) {
    case 2: return get_refine_kt2(lset);
    case 3: return get_refine_kt3(lset);
    case 5: return get_refine_kt5(lset);
    default: return get_refine_kt8(lset);
  }
}
grad_fn pick_grad_kt(int KT, int L) {
  switch (KT) {
    case 2: return get_grad_kt2(L);
    case 3: return get_grad_kt3(L);
    case 5: return get_grad_kt5(L);
    default: return get_grad_kt8(L);
  }
}
grad_fn pick_gradw_kt(int KT, int L) {
  switch (KT) {
    case 2: return get_gradw_kt2(L);
    case 3: return get_gradw_kt3(L);
    case 5: return get_gradw_kt5(L);
    default: return get_gradw_kt8(L);
  }
}
grad_dm_fn pick_graddm_kt(int KT, int L, bool wide) {
  switch (KT) {
    case 2: return wide ? get_gradwdm_kt2(L) : get_graddm_kt2(L);
    case 3: return wide ? get_gradwdm_kt3(L) : get_graddm_kt3(L);
    case 5: return wide ? get_gradwdm_kt5(L) : get_graddm_kt5(L);
    default: return wide ? get_gradwdm_kt8(L) : get_graddm_kt8(L);
  }
}

int validate_config(const rift_ile_config* c) {
  if (!c) return RIFT_EINVAL;
  if (c->block != 64 && c->block != 128 && c->block != 256 && c->block != 512) return RIFT_EINVAL;
  if (c->tile_blocks < 1 || c->tile_blocks > 64) return RIFT_EINVAL;
  if (c->blocks_per_cu < 0 || c->blocks_per_cu > 32) return RIFT_EINVAL;
  if (c->sort != 0 && c->sort != 1) return RIFT_EINVAL;
  return RIFT_OK;
}

// Dynamic LDS of the likelihood kernels: each wavefront's staging buffers of
// the data term, then (l <= 8 class) a trig column per lane.
size_t eval_lds_bytes(int lset, int block, size_t rsz) {
  const size_t trig = (lset & 8) ? (size_t)trig_rows(lset) * block * rsz : 0;
  return (size_t)(block / 64) * STAGE_WAVE + trig;
}

int launch_tiles(rift_ile_plan p, int mode, const double* theta, const double* lnw, double* lnL,
                 hipStream_t st) {
  TileArgs a;
  a.descs = p->d_desc;
  a.tiles = p->d_tiles;
  a.n_tiles = p->n_tiles;
  a.persistent = p->cfg.blocks_per_cu > 0 ? 1 : 0;
  a.counter = p->d_counter;
  a.theta = theta;
  a.lnw = lnw;
  a.N = p->N;
  a.lnL = lnL;
  a.bnd = p->d_bnd;
  a.part = p->d_part;
  a.tmax = p->d_tmax;
  a.cnt = p->d_cnt;
  a.theta_aos = p->cfg.sort ? p->d_aos : nullptr;
  a.dm = p->dm;
  a.tm = p->tm;
  a.pm = p->pm;
  a.kap = p->kap;
  a.am = p->am;
  a.ang = p->ang;
  const size_t rsz = (mode == MODE_PASS32 ? sizeof(float) : sizeof(double));
  const size_t shm = eval_lds_bytes(p->lset, p->cfg.block, rsz);
  if (shm + 1024 > (size_t)p->di.max_lds) return RIFT_EUNSUPPORTED;
  tile_fn f = pick_tiles_kt(mode, p->KT, p->lset);
  if (!f) return RIFT_EUNSUPPORTED;
  int grid = p->n_tiles;
  if (a.persistent) grid = std::min(p->n_tiles, p->cfg.blocks_per_cu * p->di.n_cu);
  if (grid <= 0) return RIFT_OK;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (p->profiling) {
    HCHK(hipEventCreate(&e0));
    HCHK(hipEventCreate(&e1));
    p->ev.push_back(e0);
    p->ev.push_back(e1);
    HCHK(hipEventRecord(e0, st));
  }
  hipLaunchKernelGGL(f, dim3(grid), dim3(p->cfg.block), shm, st, a);
  HCHK(hipGetLastError());
  if (p->profiling) HCHK(hipEventRecord(e1, st));
  return RIFT_OK;
}

void clear_events(rift_ile_plan p) {
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  p->ev.clear();
}

// Device buffers of the binning, allocated the first time a configuration
// with sort = 1 is used (146 bytes per sample).
int ensure_bin_buffers(rift_ile_plan p) {
  if (p->bin_ready) return RIFT_OK;
  if (p->N > 0x7fffffff) return RIFT_EUNSUPPORTED;
  const int64_t N = p->N;
  void* v;
  int st;
#define BCHK(x) \
  if ((st = (x))) return st
  BCHK(palloc(p, sizeof(Tile) * p->n_stiles, &v));
  p->d_stiles = (Tile*)v;
  HCHK(hipMemcpy(p->d_stiles, p->h_stiles.data(), sizeof(Tile) * p->n_stiles, hipMemcpyHostToDevice));
  BCHK(palloc(p, sizeof(Tile) * p->n_chunks, &v));
  p->d_chunks = (Tile*)v;
  HCHK(hipMemcpy(p->d_chunks, p->h_chunks.data(), sizeof(Tile) * p->n_chunks, hipMemcpyHostToDevice));
  BCHK(palloc(p, sizeof(float) * 3 * N, &v));
  p->d_ucoord = (float*)v;
  BCHK(palloc(p, sizeof(float) * 6 * p->n_stiles, &v));
  p->d_rpart = (float*)v;
  BCHK(palloc(p, sizeof(uint16_t) * N, &v));
  p->d_key = (uint16_t*)v;
  BCHK(palloc(p, sizeof(int32_t) * p->n_mat, &v));
  p->d_mat = (int32_t*)v;
  BCHK(palloc(p, sizeof(int32_t) * ((p->n_mat + SCAN_CHUNK - 1) / SCAN_CHUNK + 1), &v));
  p->d_scan = (int32_t*)v;
  BCHK(palloc(p, sizeof(double) * 8 * N, &v));
  p->d_trec = (double*)v;
  BCHK(palloc(p, sizeof(double) * 8 * N, &v));
  p->d_aos = (double*)v;
  if (!p->d_L) {  // lnL of the binned evaluation when the caller asks for none
    BCHK(palloc(p, sizeof(double) * N, &v));
    p->d_L = (double*)v;
  }
#undef BCHK
  p->bin_ready = true;
  return RIFT_OK;
}

// Arrival-time binning of the batch (see k_bin_*): records in d_aos.
int run_binning(rift_ile_plan p, const double* theta, hipStream_t st) {
  hipLaunchKernelGGL(k_bin_range, dim3(p->n_stiles), dim3(BIN_T), 0, st, p->d_desc, p->d_stiles, theta, p->N,
                     p->d_ucoord, p->d_rpart);
  hipLaunchKernelGGL(k_bin_hist, dim3(p->n_stiles), dim3(BIN_T), 0, st, p->d_desc, p->d_stiles,
                     (const float*)p->d_ucoord, (const float*)p->d_rpart, p->d_key, p->d_mat);
  const int nb = (int)((p->n_mat + SCAN_CHUNK - 1) / SCAN_CHUNK);
  hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(SCAN_T), 0, st, (const int32_t*)p->d_mat, p->n_mat, p->d_scan);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_T), 0, st, p->d_scan, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(SCAN_T), 0, st, (const int32_t*)p->d_mat, p->n_mat,
                     (const int32_t*)p->d_scan, p->d_mat, (int32_t*)nullptr);
  hipLaunchKernelGGL(k_bin_coarse, dim3(p->n_stiles), dim3(BIN_T), 0, st, p->d_desc, p->d_stiles,
                     (const uint16_t*)p->d_key, (const int32_t*)p->d_mat, theta, p->N, p->d_trec);
  hipLaunchKernelGGL(k_bin_chunk, dim3(p->n_chunks), dim3(BIN_CT), 0, st, (const Tile*)p->d_chunks,
                     (const double*)p->d_trec, p->d_aos);
  HCHK(hipGetLastError());
  return RIFT_OK;
}

}  // namespace

extern "C" {

int rift_ile_version(void) { return RIFT_ILE_VERSION; }

const char* rift_ile_strerror(int status) {
  switch (status) {
    case RIFT_OK: return "ok";
    case RIFT_EINVAL: return "invalid argument";
    case RIFT_EDEVICE: return "HIP runtime error";
    case RIFT_ENOMEM: return "out of memory";
    case RIFT_EUNSUPPORTED: return "unsupported request";
    case RIFT_ESCRATCH: return "request exceeds the fixed scratch of the allocation-free entry point";
    default: return "unknown status";
  }
}

int rift_ile_plan_profile(rift_ile_plan plan, int enable) {
  if (!plan) return RIFT_EINVAL;
  if (enable) {
    if (plan->last) HCHK(hipStreamSynchronize(plan->last));
    clear_events(plan);
  }
  plan->profiling = enable != 0;
  return RIFT_OK;
}

int rift_ile_plan_profile_read(rift_ile_plan plan, double* total_ms, int64_t* launches) {
  if (!plan || !total_ms || !launches) return RIFT_EINVAL;
  double tot = 0.0;
  for (size_t i = 0; i + 1 < plan->ev.size(); i += 2) {
    HCHK(hipEventSynchronize(plan->ev[i + 1]));
    float ms = 0.0f;
    HCHK(hipEventElapsedTime(&ms, plan->ev[i], plan->ev[i + 1]));
    tot += ms;
  }
  *total_ms = tot;
  *launches = (int64_t)(plan->ev.size() / 2);
  return RIFT_OK;
}

int rift_ile_plan_destroy(rift_ile_plan plan) {
  if (!plan) return RIFT_EINVAL;
  if (plan->last) (void)hipStreamSynchronize(plan->last);
  clear_events(plan);
  plan_free_all(plan);
  delete plan;
  return RIFT_OK;
}

namespace {
// Plan creation; with `arena` set, every device buffer of the plan is carved
// from [arena, arena + arena_cap) instead of allocated (RIFT_ESCRATCH if it
// does not fit, before anything is enqueued).
int plan_create_impl(const rift_ile_point* pts, int32_t n_points, const int64_t* n_per_point, int precision,
                     void* stream, char* arena, size_t arena_cap, rift_ile_plan* out) {
  if (!out || !pts || !n_per_point || n_points < 1 || n_points > (1 << 20)) return RIFT_EINVAL;
  if (precision != RIFT_FP64 && precision != RIFT_MIXED) return RIFT_EINVAL;
  int64_t N = 0;
  for (int p = 0; p < n_points; ++p) {
    int st = validate_point(pts + p);
    if (st) return st;
    if (n_per_point[p] < 1 || n_per_point[p] > ((int64_t)1 << 31) - 1) return RIFT_EINVAL;
    N += n_per_point[p];
  }
  if (N > ((int64_t)1 << 40)) return RIFT_EINVAL;
  *out = nullptr;
  rift_ile_plan p = new (std::nothrow) rift_ile_plan_s;
  if (!p) return RIFT_ENOMEM;
  p->arena = arena;
  p->arena_cap = arena ? arena_cap : 0;
  hipStream_t st = (hipStream_t)stream;
  int rc = device_info(&p->di);
  if (rc) { delete p; return rc; }
  p->n_points = n_points;
  p->prec = precision;
  p->N = N;
  p->n_per.assign(n_per_point, n_per_point + n_points);
  p->h_desc.resize(n_points);
  const bool mixed = precision == RIFT_MIXED;
  int KT = 2;
  for (int i = 0; i < n_points; ++i) KT = std::max(KT, kt_class(pts[i].n_det));
  p->KT = KT;

#define PCHK(x)                 \
  do {                          \
    int s_ = (x);               \
    if (s_) {                   \
      plan_free_all(p);         \
      delete p;                 \
      return s_;                \
    }                           \
  } while (0)
#define PHIP(x)                    \
  do {                             \
    if ((x) != hipSuccess) {       \
      plan_free_all(p);            \
      delete p;                    \
      return RIFT_EDEVICE;         \
    }                              \
  } while (0)

  void* v = nullptr;
  PCHK(palloc(p, sizeof(PointDesc) * n_points, &v));
  p->d_desc = (PointDesc*)v;
  std::vector<int32_t*> d_perm(n_points);
  std::vector<double*> d_qmax(n_points);
  // host copies staged to the device: they live until the final synchronisation
  std::vector<std::vector<int32_t>> h_perm(n_points);
  int64_t s0 = 0;
  for (int pi = 0; pi < n_points; ++pi) {
    const rift_ile_point& pt = pts[pi];
    PointDesc& D = p->h_desc[pi];
    memset(&D, 0, sizeof(D));
    const int K = pt.n_det, M = pt.n_modes;
    int lmax = 2;
    for (int i = 0; i < M; ++i) lmax = std::max(lmax, (int)pt.lm[2 * i]);
    D.K = K;
    D.M = M;
    D.n_t = pt.n_t;
    D.L = l_class(lmax);
    D.B = basis_count(D.L);
    D.KT = KT;
    D.n = n_per_point[pi];
    D.s0 = s0;
    s0 += D.n;
    D.t0 = pt.t0;
    D.inv_dt = 1.0 / pt.dt;
    D.gmst = pt.gmst_rad;
    D.d_ref = pt.d_ref;
    D.lnN = log((double)D.n);
    // binning: a Morton key of about 32 samples per cell (<= 16 bits), coarse
    // buckets of about 1024 samples (<= 1024 per point)
    D.bin_dims = std::min(K, 3);
    {
      int tb = (int)ceil(log2(std::max(1.0, (double)D.n / 32.0)));
      tb = std::max(0, std::min(16, tb));
      D.bin_bits = tb / D.bin_dims;
      tb = D.bin_bits * D.bin_dims;
      int cb = (int)ceil(log2(std::max(1.0, (double)D.n / 1024.0)));
      cb = std::max(0, std::min(BIN_CB_MAX, cb));
      D.bin_cb = std::min(cb, tb);
    }
    // refinement margin: an unrefined sample weighs < e^{-T} of the best one
    D.T = log((double)D.n) + 12.0;
    p->lset |= lbit(D.L);
    for (int k = 0; k < K; ++k) {
      const double* d = pt.det_tensor + 9 * k;
      const double six[6] = {d[0], d[4], d[8], d[1] + d[3], d[2] + d[6], d[5] + d[7]};
      for (int a = 0; a < 6; ++a) {
        D.dten[k][a] = six[a];
        D.dten32[k][a] = (float)six[a];
      }
      for (int a = 0; a < 3; ++a) D.rpos[k][a] = pt.det_pos[3 * k + a];
    }
    // modes sorted by m (stable) so the phase e^{i m phi} walks upward
    std::vector<int32_t>& perm = h_perm[pi];
    perm.resize(M);
    for (int i = 0; i < M; ++i) perm[i] = i;
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return pt.lm[2 * a + 1] < pt.lm[2 * b + 1]; });
    for (int i = 0; i < M; ++i) {
      const int l = pt.lm[2 * perm[i]], m = pt.lm[2 * perm[i] + 1];
      D.m[i] = m;
      D.odd[i] = (m & 1) ? 1 : 0;
      ylm_fourier(l, m, D.ycoef[i]);
      for (int n = 0; n <= LMAXC; ++n) D.ycoef32[i][n] = (float)D.ycoef[i][n];
    }
    D.m_min = D.m[0];
    // device tables
    const int64_t qrows = (int64_t)KT * (pt.n_t + 2 * QPAD);
    PCHK(palloc(p, sizeof(double) * 2 * qrows * q_groups(M, QW64) * QW64, &v));
    D.Q64 = (const double*)v;
    if (mixed) {
      PCHK(palloc(p, sizeof(float) * 2 * qrows * q_groups(M, QW32) * QW32, &v));
      D.Q32 = (const float*)v;
    }
    PCHK(palloc(p, sizeof(double) * D.B * 3 * KT, &v));
    D.C64 = (const double*)v;
    if (mixed) {
      PCHK(palloc(p, sizeof(float) * D.B * 3 * KT, &v));
      D.C32 = (const float*)v;
    }
    PCHK(palloc(p, sizeof(int32_t) * M, &v));
    d_perm[pi] = (int32_t*)v;
    PCHK(palloc(p, sizeof(double) * KT, &v));
    d_qmax[pi] = (double*)v;
  }
  // kernel instances exist for one class (1, 2, 4, 8) and for any mix of the
  // l <= 4 classes (7); a batch mixing l > 4 with smaller points runs every
  // point in the l <= 8 class (exact for any l <= 8)
  if (!(p->lset & 8) && p->lset != 1 && p->lset != 2 && p->lset != 4) p->lset = 7;
  if ((p->lset & 8) && p->lset != 8) {
    p->lset = 8;
    for (int pi = 0; pi < n_points; ++pi) {
      PointDesc& D = p->h_desc[pi];
      if (D.L != 8) {
        D.L = 8;
        D.B = basis_count(8);
        for (auto* b : {(void*)D.C64, (void*)D.C32}) {
          if (!b) continue;
          auto it = std::find(p->bufs.begin(), p->bufs.end(), b);
          if (it != p->bufs.end()) { (void)hipFree(*it); p->bufs.erase(it); }
        }
        PCHK(palloc(p, sizeof(double) * D.B * 3 * KT, &v));
        D.C64 = (const double*)v;
        D.C32 = nullptr;
        if (mixed) {
          PCHK(palloc(p, sizeof(float) * D.B * 3 * KT, &v));
          D.C32 = (const float*)v;
        }
      }
    }
  }
  // binning layout: sort tiles, count-matrix blocks and coarse buckets per
  // point, all in point order (so the matrix scan starts point p at s0)
  std::vector<Tile>& stiles = p->h_stiles;
  {
    int64_t mbase = 0;
    for (int pi = 0; pi < n_points; ++pi) {
      PointDesc& D = p->h_desc[pi];
      D.bin_st0 = (int32_t)stiles.size();
      for (int64_t s = 0; s < D.n; s += BIN_TILE) {
        Tile t;
        t.p = pi;
        t.cnt = (int32_t)std::min<int64_t>(BIN_TILE, D.n - s);
        t.s = D.s0 + s;
        stiles.push_back(t);
      }
      D.bin_nst = (int32_t)stiles.size() - D.bin_st0;
      D.bin_mbase = mbase;
      mbase += ((int64_t)1 << D.bin_cb) * D.bin_nst;
      for (int64_t s = 0; s < D.n; s += BIN_CHUNK) {
        Tile t;
        t.p = pi;
        t.cnt = (int32_t)std::min<int64_t>(BIN_CHUNK, D.n - s);
        t.s = D.s0 + s;
        p->h_chunks.push_back(t);
      }
    }
    p->n_chunks = (int)p->h_chunks.size();
    if (stiles.size() > (size_t)0x7fffffff || p->h_chunks.size() > (size_t)0x7fffffff) {
      plan_free_all(p);
      delete p;
      return RIFT_EUNSUPPORTED;
    }
    p->n_stiles = (int)stiles.size();
    p->n_mat = mbase;
  }
  // the rest of the plan's device memory, before anything is enqueued (an
  // allocation that fails leaves nothing enqueued)
  PCHK(palloc(p, sizeof(int32_t) * 64, &v));
  p->d_counter = (int32_t*)v;
  if (mixed) {
    PCHK(palloc(p, sizeof(double) * N, &v));
    p->d_L = (double*)v;
    PCHK(palloc(p, sizeof(int32_t) * n_points, &v));
    p->d_cnt = (int32_t*)v;
    PCHK(palloc(p, sizeof(int32_t) * N, &v));
    p->d_list = (int32_t*)v;
    PCHK(palloc(p, sizeof(float) * N, &v));
    p->d_bnd = (float*)v;
  }
  // initial launch shape: a small batch gets one-block tiles of 64..256
  // samples, so that it still spreads over the CUs
  {
    int64_t S = N / (2 * (int64_t)std::max(1, p->di.n_cu));
    if (S < 1024) {
      int b = 64;
      while (b < 256 && 2 * b <= S) b *= 2;
      p->cfg = rift_ile_config{b, 1, 0, 0};
    }
  }
  PCHK(build_tiles(p));
  // set-up on the stream
  PHIP(hipMemcpyAsync(p->d_desc, p->h_desc.data(), sizeof(PointDesc) * n_points, hipMemcpyHostToDevice, st));
  for (int pi = 0; pi < n_points; ++pi) {
    const rift_ile_point& pt = pts[pi];
    PointDesc& D = p->h_desc[pi];
    PHIP(hipMemcpyAsync(d_perm[pi], h_perm[pi].data(), sizeof(int32_t) * pt.n_modes, hipMemcpyHostToDevice, st));
    const int64_t qper = (int64_t)(pt.n_t + 2 * QPAD) * q_groups(pt.n_modes, QW64) * QW64;
    const int gq = (int)std::min<int64_t>((KT * qper + 255) / 256, 65535);
    hipLaunchKernelGGL(k_repack<double>, dim3(gq), dim3(256), 0, st, pt.Q, (double*)D.Q64, d_perm[pi],
                       pt.n_det, KT, pt.n_modes, pt.n_t, QW64);
    if (D.Q32)
      hipLaunchKernelGGL(k_repack<float>, dim3(gq), dim3(256), 0, st, pt.Q, (float*)D.Q32, d_perm[pi],
                         pt.n_det, KT, pt.n_modes, pt.n_t, QW32);
    const int NG = 4 * D.L + 4;
    hipLaunchKernelGGL(k_basis, dim3(KT), dim3(256), sizeof(double) * 3 * NG * NG, st,
                       p->d_desc + pi, pt.U, pt.V, d_perm[pi], (double*)D.C64, (float*)D.C32);
    if (mixed) {
      // error-bound constants of the mixed path, from the table maxima and
      // the basis coefficients
      hipLaunchKernelGGL(k_qmax, dim3(KT), dim3(1024), 0, st, D.Q64, d_qmax[pi], qper);
      hipLaunchKernelGGL(k_bound, dim3(1), dim3(64), 0, st, p->d_desc + pi, (const double*)d_qmax[pi]);
    }
    PHIP(hipGetLastError());
  }
  // the persistent kernel leaves it at 0 after each launch
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, st, p->d_counter, 64, 0);
  PHIP(hipGetLastError());
  // the staged host copies (mode permutations) are released on return
  PHIP(hipStreamSynchronize(st));
#undef PCHK
#undef PHIP
  p->last = st;
  *out = p;
  return RIFT_OK;
}
}  // namespace

int rift_ile_plan_create(const rift_ile_point* pts, int32_t n_points, const int64_t* n_per_point,
                         int precision, void* stream, rift_ile_plan* out) {
  return plan_create_impl(pts, n_points, n_per_point, precision, stream, nullptr, 0, out);
}

int rift_ile_plan_get_config(rift_ile_plan plan, rift_ile_config* cfg) {
  if (!plan || !cfg) return RIFT_EINVAL;
  *cfg = plan->cfg;
  return RIFT_OK;
}

int rift_ile_plan_set_config(rift_ile_plan plan, const rift_ile_config* cfg) {
  if (!plan) return RIFT_EINVAL;
  int st = validate_config(cfg);
  if (st) return st;
  if (plan->last) HCHK(hipStreamSynchronize(plan->last));
  // the likelihood kernels' LDS must fit one block (the FP64 form needs the most)
  if (eval_lds_bytes(plan->lset, cfg->block, sizeof(double)) + 1024 > (size_t)plan->di.max_lds)
    return RIFT_EUNSUPPORTED;
  if (cfg->sort && (st = ensure_bin_buffers(plan))) return st;
  const bool retile = cfg->block * cfg->tile_blocks != plan->cfg.block * plan->cfg.tile_blocks;
  plan->cfg = *cfg;
  if (retile) return build_tiles(plan);
  return RIFT_OK;
}

// Mixed-path tail after the FP32 pass wrote lnL and bound of every sample
// (and each tile's max of lnL + lnw - bound): list the samples that can
// matter (margin T_over, or each point's own T when negative), recompute them
// in FP64 and, if wanted, export every sample's bound.
static int mixed_refine(rift_ile_plan p, const double* theta, const double* lnw, double* L, double T_over,
                 double* lnL_bnd, hipStream_t st) {
  hipLaunchKernelGGL(k_select, dim3(p->n_tiles), dim3(p->cfg.block), 0, st, p->d_desc, p->d_tiles,
                     p->n_tiles, (const int32_t*)p->d_trange, (const double*)p->d_tmax, (const double*)L, lnw,
                     p->d_bnd, p->d_cnt, p->d_list, (float)kRefineTau, T_over);
  refine_fn rf = pick_refine_kt(p->KT, p->lset);
  if (!rf) return RIFT_EUNSUPPORTED;
  hipLaunchKernelGGL(rf, dim3(p->refine_blocks, p->n_points), dim3(256),
                     eval_lds_bytes(p->lset, 256, sizeof(double)), st, p->d_desc, theta, p->N,
                     (const int32_t*)p->d_cnt, (const int32_t*)p->d_list, L);
  if (lnL_bnd)
    hipLaunchKernelGGL(k_bound_out, dim3(grid_for(p->N)), dim3(256), 0, st, (const float*)p->d_bnd, lnL_bnd, p->N);
  HCHK(hipGetLastError());
  return RIFT_OK;
}

int rift_ile_plan_lnZ(rift_ile_plan p, const double* theta, const double* lnw, double* lnZ,
                      double* neff, double* lnL, double* lnL_bnd, double* lnZ_err, void* stream) {
  if (!p || check_dev_ptr(theta) || check_dev_ptr(lnZ)) return RIFT_EINVAL;
  if ((lnw && check_dev_ptr(lnw)) || (neff && check_dev_ptr(neff)) || (lnL && check_dev_ptr(lnL)) ||
      (lnZ_err && check_dev_ptr(lnZ_err)) || (lnL_bnd && check_dev_ptr(lnL_bnd)))
    return RIFT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  p->last = st;
  int rc;
  const bool sorted = p->cfg.sort != 0;
  double* L = lnL ? lnL : p->d_L;
  if (sorted && !p->bin_ready) return RIFT_EUNSUPPORTED;
  if (sorted && (rc = run_binning(p, theta, st))) return rc;
  if (p->prec == RIFT_FP64) {
    if ((rc = launch_tiles(p, MODE_LSE64, theta, lnw, sorted ? L : lnL, st))) return rc;
    if (sorted)
      hipLaunchKernelGGL(k_lse_tiles, dim3(p->n_tiles), dim3(p->cfg.block), 0, st, p->d_tiles, (const double*)L,
                         lnw, p->d_part);
    hipLaunchKernelGGL(k_merge, dim3(p->n_points), dim3(512), 0, st, p->d_desc, p->d_trange, p->d_part,
                       (const double*)nullptr, lnZ, neff, lnZ_err);
    if (lnL_bnd)
      hipLaunchKernelGGL(k_bound_out, dim3(grid_for(p->N)), dim3(256), 0, st, (const float*)nullptr, lnL_bnd, p->N);
    HCHK(hipGetLastError());
    return RIFT_OK;
  }
  if ((rc = launch_tiles(p, MODE_PASS32, theta, lnw, L, st))) return rc;
  if (sorted)
    hipLaunchKernelGGL(k_tmax_tiles, dim3(p->n_tiles), dim3(p->cfg.block), 0, st, p->d_tiles, (const double*)L,
                       lnw, (const float*)p->d_bnd, p->d_tmax);
  if ((rc = mixed_refine(p, theta, lnw, L, -1.0, lnL_bnd, st))) return rc;
  hipLaunchKernelGGL(k_final, dim3(p->n_tiles), dim3(p->cfg.block), 0, st, p->d_tiles, (const double*)L,
                     lnw, (const float*)p->d_bnd, p->d_part, p->d_terr);
  hipLaunchKernelGGL(k_merge, dim3(p->n_points), dim3(512), 0, st, p->d_desc, p->d_trange, p->d_part,
                     (const double*)p->d_terr, lnZ, neff, lnZ_err);
  HCHK(hipGetLastError());
  return RIFT_OK;
}

namespace {

// Orthonormal polynomials of the weight e^{-x^2/2} on the real line (the
// probabilists' Hermite He_k normalised): q_0 = (2 pi)^{-1/4},
// x q_k = sqrt(k + 1) q_{k+1} + sqrt(k) q_{k-1}.  Returns q_n(x); with sum2,
// also sum_{k < n} q_k(x)^2.
double hermite_q(int n, double x, double* sum2) {
  double qm = 0.0, q = 0.63161877774606470129;  // (2 pi)^{-1/4}
  double s = 0.0;
  for (int k = 0; k < n; ++k) {
    s += q * q;
    const double qn = (x * q - sqrt((double)k) * qm) / sqrt((double)(k + 1));
    qm = q;
    q = qn;
  }
  if (sum2) *sum2 = s;
  return q;
}

}  // namespace

// Gauss-Hermite rule of n nodes for the weight e^{-x^2/2}: the nodes are the n
// simple roots of q_n, bracketed by the sign changes of q_n on a grid finer
// than their spacing (the grid never meets x = 0, a root for odd n) and
// bisected to the last bit; the weights are the Christoffel numbers
// 1 / sum_{k<n} q_k(x_i)^2.  Ascending nodes.
extern "C" int rift_ile_gauss_hermite(int n, double* nodes, double* weights) {
  if (n < 1 || n > DM_MAX || !nodes || !weights) return RIFT_EINVAL;
  const double L = 2.0 * sqrt((double)n) + 3.0;  // beyond the largest root
  const int steps = 200000;
  const double h = 2.0 * L / steps;
  int found = 0;
  double xa = -L + 0.5 * h, fa = hermite_q(n, xa, nullptr);
  for (int j = 1; j < steps && found < n; ++j) {
    const double xb = -L + (j + 0.5) * h, fb = hermite_q(n, xb, nullptr);
    if ((fa < 0.0) != (fb < 0.0)) {
      double lo = xa, hi = xb, flo = fa;
      for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        const double fm = hermite_q(n, mid, nullptr);
        if ((fm < 0.0) == (flo < 0.0)) {
          lo = mid;
          flo = fm;
        } else {
          hi = mid;
        }
      }
      const double r = 0.5 * (lo + hi);
      double s2;
      (void)hermite_q(n, r, &s2);
      nodes[found] = r;
      weights[found] = 1.0 / s2;
      ++found;
    }
    xa = xb;
    fa = fb;
  }
  return found == n ? RIFT_OK : RIFT_EDEVICE;
}

}  // extern "C"

namespace {

int plan_grad_rule(rift_ile_plan p, int32_t point, int64_t n, const double* theta, int coords, double* lnL,
                   double* grad, bool marg, void* stream);

// The plan's distance rule for `prior` (nodes cached per node count).
int set_dist_rule(rift_ile_plan p, const rift_ile_dist_prior* prior) {
  const double d0 = prior->d_min, d1 = prior->d_max;
  if (!(d0 > 0.0) || !(d1 > d0) || !(d1 <= 1.0e60)) return RIFT_EINVAL;
  if (prior->n_nodes < 1 || prior->n_nodes > DM_MAX) return RIFT_EINVAL;
  if (p->dm.n != prior->n_nodes) {
    DistRule g{};
    g.n = prior->n_nodes;
    if (rift_ile_gauss_hermite(g.n, g.xi, g.w)) return RIFT_EDEVICE;
    p->dm = g;
  }
  p->dm.d_min = d0;
  p->dm.d_max = d1;
  // 3 / (d_max^3 - d_min^3), in logs (d_max^3 may overflow only past 1e102)
  p->dm.ln_norm = log(3.0) - 3.0 * log(d1) - log1p(-(d0 / d1) * (d0 / d1) * (d0 / d1));
  return RIFT_OK;
}

}  // namespace

extern "C" {

int rift_ile_plan_lnZ_dmarg(rift_ile_plan p, const double* theta, const double* lnw, const rift_ile_dist_prior* prior,
                            double* lnZ, double* neff, double* lnLd, void* stream) {
  if (!p || !prior || check_dev_ptr(theta) || check_dev_ptr(lnZ)) return RIFT_EINVAL;
  if ((lnw && check_dev_ptr(lnw)) || (neff && check_dev_ptr(neff)) || (lnLd && check_dev_ptr(lnLd)))
    return RIFT_EINVAL;
  int rc0 = set_dist_rule(p, prior);
  if (rc0) return rc0;
  hipStream_t st = (hipStream_t)stream;
  p->last = st;
  int rc;
  const bool sorted = p->cfg.sort != 0;
  double* L = lnLd ? lnLd : p->d_L;
  if (sorted && (!p->bin_ready || !L)) return RIFT_EUNSUPPORTED;
  if (sorted && (rc = run_binning(p, theta, st))) return rc;
  if ((rc = launch_tiles(p, MODE_DMARG64, theta, lnw, sorted ? L : lnLd, st))) return rc;
  if (sorted)
    hipLaunchKernelGGL(k_lse_tiles, dim3(p->n_tiles), dim3(p->cfg.block), 0, st, p->d_tiles, (const double*)L, lnw,
                       p->d_part);
  hipLaunchKernelGGL(k_merge, dim3(p->n_points), dim3(512), 0, st, p->d_desc, p->d_trange, p->d_part,
                     (const double*)nullptr, lnZ, neff, (double*)nullptr);
  HCHK(hipGetLastError());
  return RIFT_OK;
}

int rift_ile_plan_grad_dmarg(rift_ile_plan p, int32_t point, int64_t n, const double* theta,
                             const rift_ile_dist_prior* prior, double* lnLd, double* grad, void* stream) {
  if (!p || !prior || point < 0 || point >= p->n_points || n < 0) return RIFT_EINVAL;
  int rc = set_dist_rule(p, prior);
  if (rc) return rc;
  if (n == 0) return RIFT_OK;
  // one adjoint pass: its epilogue takes the distance posterior's moments
  return plan_grad_rule(p, point, n, theta, RIFT_COORD_COS_INCL | RIFT_COORD_LN_DIST, lnLd, grad, true, stream);
}

int rift_ile_plan_lnZ_tmarg(rift_ile_plan p, const double* theta, const double* lnw, const rift_ile_time_rule* rule,
                            double* lnZ, double* neff, double* lnLt, void* stream) {
  if (!p || !rule || check_dev_ptr(theta) || check_dev_ptr(lnZ)) return RIFT_EINVAL;
  if ((lnw && check_dev_ptr(lnw)) || (neff && check_dev_ptr(neff)) || (lnLt && check_dev_ptr(lnLt)))
    return RIFT_EINVAL;
  if (rule->n_t < 3 || rule->n_t > 1000001 || (rule->n_t % 2) == 0) return RIFT_EINVAL;
  if (!std::isfinite(rule->t_start) || !(rule->h > 0.0) || !std::isfinite(rule->h)) return RIFT_EINVAL;
  if (!std::isfinite(rule->t_start + (rule->n_t - 1) * rule->h)) return RIFT_EINVAL;
  TimeRule t{};
  t.n = rule->n_t;
  t.t0 = rule->t_start;
  t.h = rule->h;
  t.ln_scale = -log((double)(rule->n_t - 1));
  t.lw_end = log(1.0 / 3.0);
  t.lw_odd = log(4.0 / 3.0);
  t.lw_even = log(2.0 / 3.0);
  p->tm = t;
  hipStream_t st = (hipStream_t)stream;
  p->last = st;
  int rc;
  const bool sorted = p->cfg.sort != 0;
  double* L = lnLt ? lnLt : p->d_L;
  if (sorted && (!p->bin_ready || !L)) return RIFT_EUNSUPPORTED;
  if (sorted && (rc = run_binning(p, theta, st))) return rc;
  if ((rc = launch_tiles(p, MODE_TMARG64, theta, lnw, sorted ? L : lnLt, st))) return rc;
  if (sorted)
    hipLaunchKernelGGL(k_lse_tiles, dim3(p->n_tiles), dim3(p->cfg.block), 0, st, p->d_tiles, (const double*)L, lnw,
                       p->d_part);
  hipLaunchKernelGGL(k_merge, dim3(p->n_points), dim3(512), 0, st, p->d_desc, p->d_trange, p->d_part,
                     (const double*)nullptr, lnZ, neff, (double*)nullptr);
  HCHK(hipGetLastError());
  return RIFT_OK;
}

int rift_ile_plan_lnZ_tband(rift_ile_plan p, const double* theta, const double* lnw, const rift_ile_band_rule* rule,
                            double* lnZ, double* neff, double* lnLt, void* stream) {
  if (!p || !rule || check_dev_ptr(theta) || check_dev_ptr(lnZ)) return RIFT_EINVAL;
  if ((lnw && check_dev_ptr(lnw)) || (neff && check_dev_ptr(neff)) || (lnLt && check_dev_ptr(lnLt)))
    return RIFT_EINVAL;
  if (rule->n_t < 2 || rule->n_t > TBAND_MAX_NODES || rule->n_fine < 1 || rule->n_fine > TBAND_MAX_FINE)
    return RIFT_EINVAL;
  if (!std::isfinite(rule->t_start) || !(rule->h > 0.0) || !std::isfinite(rule->h)) return RIFT_EINVAL;
  if (!std::isfinite(rule->t_start + (rule->n_t - 1) * rule->h)) return RIFT_EINVAL;
  const int n = rule->n_t, M = rule->n_fine;
  const int NB = n <= 16 ? 16 : (n <= 32 ? 32 : 64);
  TimeRule t{};
  t.n = n;
  t.t0 = rule->t_start;
  t.h = rule->h;
  p->tm = t;
  hipStream_t st = (hipStream_t)stream;
  p->last = st;
  int rc;
  const bool sorted = p->cfg.sort != 0;
  if (sorted && !p->bin_ready) return RIFT_EUNSUPPORTED;
  // stream-ordered scratch: kap [n][N], the sinc table [M][2 NB - 1], and
  // the per-sample values when the caller takes none
  const int64_t N = p->N;
  const size_t tab_n = (size_t)M * (2 * NB - 1);
  const size_t bytes = sizeof(double) * ((size_t)n * N + tab_n + (lnLt ? 0 : (size_t)N));
  double* w = nullptr;
  if (hipMallocAsync((void**)&w, bytes, st) != hipSuccess) return RIFT_ENOMEM;
  double* tab = w + (size_t)n * N;
  double* L = lnLt ? lnLt : tab + tab_n;
  p->kap = w;
  rc = sorted ? run_binning(p, theta, st) : RIFT_OK;
  if (!rc) rc = launch_tiles(p, MODE_TBAND64, theta, lnw, L, st);
  p->kap = nullptr;
  if (!rc) {
    hipLaunchKernelGGL(k_sinc_table, dim3((unsigned)((tab_n + 255) / 256)), dim3(256), 0, st, NB, M, tab);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((N + 255) / 256, (int64_t)p->di.n_cu * 8));
    const double ln_scale = -log((double)(n - 1) * (double)M);
    const double* kc = w;
    if (NB == 16)
      hipLaunchKernelGGL(k_tband<16>, dim3(grid), dim3(256), 0, st, N, n, M, kc, (const double*)tab, ln_scale, L);
    else if (NB == 32)
      hipLaunchKernelGGL(k_tband<32>, dim3(grid), dim3(256), 0, st, N, n, M, kc, (const double*)tab, ln_scale, L);
    else
      hipLaunchKernelGGL(k_tband<64>, dim3(grid), dim3(256), 0, st, N, n, M, kc, (const double*)tab, ln_scale, L);
    if (p->n_tiles > 0)
      hipLaunchKernelGGL(k_lse_tiles, dim3(p->n_tiles), dim3(p->cfg.block), 0, st, p->d_tiles, (const double*)L,
                         lnw, p->d_part);
    hipLaunchKernelGGL(k_merge, dim3(p->n_points), dim3(512), 0, st, p->d_desc, p->d_trange, p->d_part,
                       (const double*)nullptr, lnZ, neff, (double*)nullptr);
    if (hipGetLastError() != hipSuccess) rc = RIFT_EDEVICE;
  }
  if (hipFreeAsync(w, st) != hipSuccess && !rc) rc = RIFT_EDEVICE;
  return rc;
}

int rift_ile_plan_lnZ_erai(rift_ile_plan p, const double* theta, const double* lnw, const rift_ile_angle_rule* rule,
                           double* lnZ, double* neff, double* lnLa, void* stream) {
  if (!p || !rule || check_dev_ptr(theta) || check_dev_ptr(lnZ)) return RIFT_EINVAL;
  if ((lnw && check_dev_ptr(lnw)) || (neff && check_dev_ptr(neff)) || (lnLa && check_dev_ptr(lnLa)))
    return RIFT_EINVAL;
  if (rule->n_phi < 1 || rule->n_phi > 4096 || rule->n_psi < 1 || rule->n_psi > 4096) return RIFT_EINVAL;
  int m_max = 0;
  for (const PointDesc& D : p->h_desc) m_max = std::max(m_max, std::max(std::abs(D.m[0]), std::abs(D.m[D.M - 1])));
  if (m_max > ERAI_MAX_M) return RIFT_EUNSUPPORTED;
  const int nd = 2 * m_max + 1, nq = 4 * m_max + 1;
  const int NDM = m_max <= 2 ? 5 : 9, NQM = m_max <= 2 ? 9 : 17;
  AngleRule g{};
  g.nd = nd;
  g.nq = nq;
  g.dd = 2.0 * 3.14159265358979323846 / nd;
  g.dq = 2.0 * 3.14159265358979323846 / nq;
  p->am = g;
  hipStream_t st = (hipStream_t)stream;
  p->last = st;
  const bool sorted = p->cfg.sort != 0;
  if (sorted && !p->bin_ready) return RIFT_EUNSUPPORTED;
  // stream-ordered scratch: the coefficients [2 nd + 3 nq][N], the tables,
  // and the per-sample values when the caller takes none
  const int64_t N = p->N;
  const size_t rows = (size_t)(2 * nd + 3 * nq);
  const size_t nwd = (size_t)rule->n_phi * NDM, nwq = (size_t)rule->n_phi * NQM, ntu = 4 * (size_t)rule->n_psi;
  const size_t bytes = sizeof(double) * (rows * N + nwd + nwq + ntu + (lnLa ? 0 : (size_t)N));
  double* w = nullptr;
  if (hipMallocAsync((void**)&w, bytes, st) != hipSuccess) return RIFT_ENOMEM;
  double* wd = w + rows * N;
  double* wq = wd + nwd;
  double* tu = wq + nwq;
  double* L = lnLa ? lnLa : tu + ntu;
  p->ang = w;
  int rc = sorted ? run_binning(p, theta, st) : RIFT_OK;
  if (!rc) rc = launch_tiles(p, MODE_ERAI64, theta, lnw, L, st);
  p->ang = nullptr;
  if (!rc) {
    const size_t big = std::max(std::max(nwd, nwq), (size_t)rule->n_psi);
    hipLaunchKernelGGL(k_erai_tables, dim3((unsigned)std::min<size_t>((big + 255) / 256, 1024)), dim3(256), 0, st,
                       rule->n_phi, rule->n_psi, nd, nq, NDM, NQM, wd, wq, tu);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((N + 255) / 256, (int64_t)p->di.n_cu * 8));
    const double ln_scale = -log((double)rule->n_phi * (double)rule->n_psi);
    if (NDM == 5)
      hipLaunchKernelGGL((k_erai<5, 9>), dim3(grid), dim3(256), 0, st, N, nd, nq, rule->n_phi, rule->n_psi,
                         (const double*)w, (const double*)wd, (const double*)wq, (const double*)tu, ln_scale, L);
    else
      hipLaunchKernelGGL((k_erai<9, 17>), dim3(grid), dim3(256), 0, st, N, nd, nq, rule->n_phi, rule->n_psi,
                         (const double*)w, (const double*)wd, (const double*)wq, (const double*)tu, ln_scale, L);
    if (p->n_tiles > 0)
      hipLaunchKernelGGL(k_lse_tiles, dim3(p->n_tiles), dim3(p->cfg.block), 0, st, p->d_tiles, (const double*)L,
                         lnw, p->d_part);
    hipLaunchKernelGGL(k_merge, dim3(p->n_points), dim3(512), 0, st, p->d_desc, p->d_trange, p->d_part,
                       (const double*)nullptr, lnZ, neff, (double*)nullptr);
    if (hipGetLastError() != hipSuccess) rc = RIFT_EDEVICE;
  }
  if (hipFreeAsync(w, st) != hipSuccess && !rc) rc = RIFT_EDEVICE;
  return rc;
}

int rift_ile_plan_lnZ_pmarg(rift_ile_plan p, const double* theta, const double* lnw, const rift_ile_psi_rule* rule,
                            double* lnZ, double* neff, double* lnLp, void* stream) {
  if (!p || !rule || check_dev_ptr(theta) || check_dev_ptr(lnZ)) return RIFT_EINVAL;
  if ((lnw && check_dev_ptr(lnw)) || (neff && check_dev_ptr(neff)) || (lnLp && check_dev_ptr(lnLp)))
    return RIFT_EINVAL;
  if (rule->method != RIFT_PSI_TRAPEZOID && rule->method != RIFT_PSI_LAPLACE && rule->method != RIFT_PSI_CELLS)
    return RIFT_EINVAL;
  if (rule->method == RIFT_PSI_TRAPEZOID && (rule->n_points < 1 || rule->n_points > 65536)) return RIFT_EINVAL;
  PsiRule g{};
  g.method = rule->method == RIFT_PSI_TRAPEZOID ? 0 : (rule->method == RIFT_PSI_LAPLACE ? 1 : 2);
  g.n = rule->method == RIFT_PSI_TRAPEZOID ? rule->n_points : 0;
  g.ln_n = g.n > 0 ? log((double)g.n) : 0.0;
  p->pm = g;
  hipStream_t st = (hipStream_t)stream;
  p->last = st;
  int rc;
  const bool sorted = p->cfg.sort != 0;
  double* L = lnLp ? lnLp : p->d_L;
  if (sorted && (!p->bin_ready || !L)) return RIFT_EUNSUPPORTED;
  if (sorted && (rc = run_binning(p, theta, st))) return rc;
  if ((rc = launch_tiles(p, MODE_PMARG64, theta, lnw, sorted ? L : lnLp, st))) return rc;
  if (sorted)
    hipLaunchKernelGGL(k_lse_tiles, dim3(p->n_tiles), dim3(p->cfg.block), 0, st, p->d_tiles, (const double*)L, lnw,
                       p->d_part);
  hipLaunchKernelGGL(k_merge, dim3(p->n_points), dim3(512), 0, st, p->d_desc, p->d_trange, p->d_part,
                     (const double*)nullptr, lnZ, neff, (double*)nullptr);
  HCHK(hipGetLastError());
  return RIFT_OK;
}

int rift_ile_plan_refined(rift_ile_plan p, int64_t* n_refined) {
  if (!p || !n_refined) return RIFT_EINVAL;
  *n_refined = 0;
  if (p->prec != RIFT_MIXED) return RIFT_OK;
  if (p->last) HCHK(hipStreamSynchronize(p->last));
  std::vector<int32_t> c(p->n_points);
  HCHK(hipMemcpy(c.data(), p->d_cnt, sizeof(int32_t) * p->n_points, hipMemcpyDeviceToHost));
  for (int32_t v : c) *n_refined += v;
  return RIFT_OK;
}

}  // extern "C"

namespace {

// The plan's gradient launch; with `marg`, of the likelihood marginalised over
// distance under the plan's current distance rule.
int plan_grad_rule(rift_ile_plan p, int32_t point, int64_t n, const double* theta, int coords, double* lnL,
                   double* grad, bool marg, void* stream) {
  if (!p || point < 0 || point >= p->n_points || n < 0) return RIFT_EINVAL;
  if (coords < 0 || coords > (RIFT_COORD_COS_INCL | RIFT_COORD_LN_DIST)) return RIFT_EINVAL;
  if (n == 0) return RIFT_OK;
  if (check_dev_ptr(theta) || check_dev_ptr(grad) || (lnL && check_dev_ptr(lnL))) return RIFT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  p->last = st;
  const PointDesc& D = p->h_desc[point];
  // a batch that cannot give every CU 256 samples runs 16 lanes per sample
  const bool wide = n <= (int64_t)256 * p->di.n_cu;
  grad_fn f = wide ? pick_gradw_kt(p->KT, D.L) : pick_grad_kt(p->KT, D.L);
  grad_dm_fn fdm = marg ? pick_graddm_kt(p->KT, D.L, wide) : nullptr;
  if (!f || (marg && !fdm)) return RIFT_EUNSUPPORTED;
  const int64_t blocks = wide ? std::min<int64_t>((n + 15) / 16, (int64_t)p->di.n_cu * 8)
                              : std::min<int64_t>((n + 255) / 256, (int64_t)p->di.n_cu * 16);
  const size_t shm = wide ? 0 : (size_t)trig_rows(lbit(D.L)) * 256 * sizeof(double);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (p->profiling) {
    HCHK(hipEventCreate(&e0));
    HCHK(hipEventCreate(&e1));
    p->ev.push_back(e0);
    p->ev.push_back(e1);
    HCHK(hipEventRecord(e0, st));
  }
  if (marg)
    hipLaunchKernelGGL(fdm, dim3((unsigned)blocks), dim3(256), shm, st, (const PointDesc*)(p->d_desc + point), theta,
                       n, lnL, grad, coords, p->dm);
  else
    hipLaunchKernelGGL(f, dim3((unsigned)blocks), dim3(256), shm, st,
                       (const PointDesc*)(p->d_desc + point),
                       theta, n, lnL, grad, coords);
  HCHK(hipGetLastError());
  if (p->profiling) HCHK(hipEventRecord(e1, st));
  return RIFT_OK;
}

}  // namespace

extern "C" {

int rift_ile_plan_grad(rift_ile_plan p, int32_t point, int64_t n, const double* theta, int coords,
                       double* lnL, double* grad, void* stream) {
  return plan_grad_rule(p, point, n, theta, coords, lnL, grad, false, stream);
}

int rift_ile_plan_tune(rift_ile_plan p, const double* theta, const double* lnw, void* stream) {
  if (!p || check_dev_ptr(theta) || (lnw && check_dev_ptr(lnw))) return RIFT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const bool prof = p->profiling;
  p->profiling = false;
  static const rift_ile_config cands[] = {
      {256, 1, 0, 1}, {256, 4, 0, 1}, {128, 4, 0, 1}, {512, 2, 0, 1}, {256, 1, 4, 1}, {256, 2, 4, 1},
      {256, 4, 4, 1}, {256, 8, 2, 1}, {128, 8, 4, 1}, {512, 1, 2, 1}, {64, 16, 8, 1},
      {256, 4, 0, 0}, {256, 8, 2, 0}, {512, 2, 0, 0}, {64, 1, 0, 0}, {128, 1, 0, 0},
  };
  const int nc = (int)(sizeof(cands) / sizeof(cands[0]));
  double* d_out = nullptr;
  if (hipMalloc(&d_out, sizeof(double) * 2 * p->n_points) != hipSuccess) return RIFT_ENOMEM;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipFree(d_out);
    return RIFT_EDEVICE;
  }
  int best = -1;
  float best_ms = 1e30f;
  int rc = RIFT_OK;
  for (int c = 0; c < nc && rc == RIFT_OK; ++c) {
    rc = rift_ile_plan_set_config(p, &cands[c]);
    if (rc == RIFT_EUNSUPPORTED) {  // e.g. binning of a batch beyond int32 positions
      rc = RIFT_OK;
      continue;
    }
    if (rc) break;
    rc = rift_ile_plan_lnZ(p, theta, lnw, d_out, d_out + p->n_points, nullptr, nullptr, nullptr, st);  // warm-up
    if (rc) break;
    float ms_sum = 0.0f;
    for (int r = 0; r < 3 && rc == RIFT_OK; ++r) {
      (void)hipEventRecord(e0, st);
      rc = rift_ile_plan_lnZ(p, theta, lnw, d_out, d_out + p->n_points, nullptr, nullptr, nullptr, st);
      (void)hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) rc = RIFT_EDEVICE;
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms_sum += ms;
    }
    if (rc == RIFT_OK && ms_sum < best_ms) {
      best_ms = ms_sum;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(d_out);
  p->profiling = prof;
  if (rc) return rc;
  if (best < 0) return RIFT_EUNSUPPORTED;
  rc = rift_ile_plan_set_config(p, &cands[best]);
  return rc ? rc : best;
}

int rift_ile_lnZ(const rift_ile_point* pts, int32_t n_points, const int64_t* n_per_point,
                 const double* theta, const double* lnw, double* lnZ, double* neff, double* lnL,
                 int precision, void* stream) {
  if (check_dev_ptr(theta) || check_dev_ptr(lnZ)) return RIFT_EINVAL;
  if (precision != RIFT_FP64 && precision != RIFT_MIXED) return RIFT_EINVAL;
  rift_ile_plan p = nullptr;
  int rc = rift_ile_plan_create(pts, n_points, n_per_point, precision, stream, &p);
  if (rc) return rc;
  rc = rift_ile_plan_lnZ(p, theta, lnw, lnZ, neff, lnL, nullptr, nullptr, stream);
  int rc2 = rift_ile_plan_destroy(p);
  return rc ? rc : rc2;
}

int rift_ile_lnL(const rift_ile_point* pt, int64_t n, const double* theta, double* lnL, double* lnL_bnd,
                 int precision, void* stream) {
  if (n < 0) return RIFT_EINVAL;
  if (precision != RIFT_FP64 && precision != RIFT_MIXED && precision != RIFT_FP32) return RIFT_EINVAL;
  if (n == 0) return validate_point(pt);
  if (check_dev_ptr(theta) || check_dev_ptr(lnL) || (lnL_bnd && check_dev_ptr(lnL_bnd))) return RIFT_EINVAL;
  rift_ile_plan p = nullptr;
  int rc = rift_ile_plan_create(pt, 1, &n, precision == RIFT_FP64 ? RIFT_FP64 : RIFT_MIXED, stream, &p);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  p->cfg.sort = 0;  // input-order evaluation: no reduction follows
  if (precision == RIFT_FP64) {
    rc = launch_tiles(p, MODE_LSE64, theta, nullptr, lnL, st);
    if (!rc && lnL_bnd) {
      hipLaunchKernelGGL(k_bound_out, dim3(grid_for(n)), dim3(256), 0, st, (const float*)nullptr, lnL_bnd, n);
      if (hipGetLastError() != hipSuccess) rc = RIFT_EDEVICE;
    }
  } else {
    rc = launch_tiles(p, MODE_PASS32, theta, nullptr, lnL, st);
    if (!rc && precision == RIFT_MIXED) {
      // every sample that can lie within kPosteriorMargin of the best one
      rc = mixed_refine(p, theta, nullptr, lnL, kPosteriorMargin, lnL_bnd, st);
    } else if (!rc && lnL_bnd) {
      hipLaunchKernelGGL(k_bound_out, dim3(grid_for(n)), dim3(256), 0, st, (const float*)p->d_bnd, lnL_bnd, n);
      if (hipGetLastError() != hipSuccess) rc = RIFT_EDEVICE;
    }
  }
  int rc2 = rift_ile_plan_destroy(p);
  return rc ? rc : rc2;
}

int rift_ile_grad(const rift_ile_point* pt, int64_t n, const double* theta, int coords, double* lnL,
                  double* grad, int precision, void* stream) {
  if (n < 0) return RIFT_EINVAL;
  if (precision == RIFT_MIXED || precision == RIFT_FP32) return RIFT_EUNSUPPORTED;
  if (precision != RIFT_FP64) return RIFT_EINVAL;
  if (coords < 0 || coords > (RIFT_COORD_COS_INCL | RIFT_COORD_LN_DIST)) return RIFT_EINVAL;
  if (n == 0) return validate_point(pt);
  if (check_dev_ptr(theta) || check_dev_ptr(grad)) return RIFT_EINVAL;
  rift_ile_plan p = nullptr;
  int rc = rift_ile_plan_create(pt, 1, &n, RIFT_FP64, stream, &p);
  if (rc) return rc;
  rc = rift_ile_plan_grad(p, 0, n, theta, coords, lnL, grad, stream);
  int rc2 = rift_ile_plan_destroy(p);
  return rc ? rc : rc2;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free entry point: its plan lives in a fixed device array, one
// copy per GPU, held until the process ends.  Host code never passes the
// array's name to a kernel or a copy: it passes the device address that
// hipGetSymbolAddress returns for the current device (kept per device).
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[RIFT_ILE_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// The current device's scratch address, looked up once per device.
int scratch_of_current_device(char** out) {
  int dev = -1;
  HCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return RIFT_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return RIFT_EDEVICE;
    g_scratch[dev] = (char*)ptr;
  }
  *out = g_scratch[dev];
  return RIFT_OK;
}
}  // namespace

extern "C" int rift_ile_lnZ_noalloc(const rift_ile_point* pts, int32_t n_points, const int64_t* n_per_point,
                                    const double* theta, const double* lnw, double* lnZ, double* neff,
                                    double* lnL, int precision, void* stream) {
  if (check_dev_ptr(theta) || check_dev_ptr(lnZ)) return RIFT_EINVAL;
  if (precision != RIFT_FP64 && precision != RIFT_MIXED) return RIFT_EINVAL;
  char* base = nullptr;
  int rc = scratch_of_current_device(&base);
  if (rc) return rc;
  rift_ile_plan p = nullptr;
  rc = plan_create_impl(pts, n_points, n_per_point, precision, stream, base, RIFT_ILE_NOALLOC_SCRATCH_BYTES, &p);
  if (rc) return rc;
  rc = rift_ile_plan_lnZ(p, theta, lnw, lnZ, neff, lnL, nullptr, nullptr, stream);
  int rc2 = rift_ile_plan_destroy(p);
  return rc ? rc : rc2;
}
