// The importance-sampling normalisation of the gradient samplers (Eq.
// (sampler-menu:is)) with the defensive proposal of Sec. "Mode coverage,
// adaptive clouds, and evidence":
//   q = alpha p + (1 - alpha) sum_m a_m N(mu_m, s C_m),
// p the samples' prior and each Gaussian component fitted to one recovered
// mode by the moments of its chains or cloud (C widened by s > 1).  Two parts:
//   * rift_ile_moments: the weighted mean and covariance of a cloud, a
//     two-pass reduction (log-weights normalised on the fly, then the
//     centred second moments), deterministic (fixed-order block partials);
//   * rift_ile_mixture_is: a set-up kernel factors each s C_m (Cholesky and
//     the inverse factor), then one lane per draw picks the prior or a
//     component from the caller's uniform, draws, and evaluates ln p - ln q
//     with every component's full density.
// Coordinates are the samplers' (ra, dec, psi, cos incl, phiref, tref, ln D).
// ra, psi and phiref are periodic (2 pi, pi, 2 pi): a component is the
// density of its Gaussian draw taken modulo those periods, a sum over the
// lattice of periodic images.  Relative to the image nearest the mean, the
// images within K_j periods are kept, K_j = ceil(9 sigma_j / P_j - 1/2) for the
// component's marginal width sigma_j; the images left out carry a Gaussian
// mass below 2 Phi(-9) per periodic row (about 2e-19).  A component wider
// than half a period in a periodic row is refused (K_j <= 4).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>

#include "../../include/rift_ile.h"

namespace {

constexpr int MOM_BLOCK = 256;
constexpr int MOM_GRID_MAX = 1024;
constexpr int IS_BLOCK = 256;
constexpr double TWO_PI = 6.283185307179586476925;
constexpr double PI = 3.141592653589793238463;
constexpr double HALF_PI = 1.570796326794896619231;
// rows 0 (ra), 2 (psi), 4 (phiref) and their periods
__device__ __constant__ const int PER_ROW[3] = {0, 2, 4};
__device__ __forceinline__ double period(int p) { return p == 1 ? PI : TWO_PI; }

// ---------------------------------------------------------------------------
// Moments
// ---------------------------------------------------------------------------

// Running (max log-weight m, sum of e^{w - m}, sums of e^{w - m} c_j).
struct Mom1 {
  double m, s, c[7];
};

__device__ __forceinline__ void mom_push(Mom1& a, double w, const double* x) {
  if (w == -__builtin_inf()) return;
  const double d = w - a.m;
  const double e = exp(-fabs(d));
  const bool up = d > 0.0;
  a.s = up ? fma(a.s, e, 1.0) : a.s + e;
#pragma unroll
  for (int j = 0; j < 7; ++j) a.c[j] = up ? fma(a.c[j], e, x[j]) : fma(e, x[j], a.c[j]);
  a.m = up ? w : a.m;
}

__device__ __forceinline__ Mom1 mom_merge(const Mom1& a, const Mom1& b) {
  if (b.m == -__builtin_inf() && b.s == 0.0) return a;
  if (a.m == -__builtin_inf() && a.s == 0.0) return b;
  const double m = fmax(a.m, b.m);
  const double ea = exp(a.m - m), eb = exp(b.m - m);
  Mom1 r;
  r.m = (a.m == a.m && b.m == b.m) ? m : __builtin_nan("");
  r.s = a.s * ea + b.s * eb;
#pragma unroll
  for (int j = 0; j < 7; ++j) r.c[j] = a.c[j] * ea + b.c[j] * eb;
  return r;
}

__device__ Mom1 mom_block(Mom1 a, Mom1* sh) {
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int o = MOM_BLOCK / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = mom_merge(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  return sh[0];
}

__global__ void __launch_bounds__(MOM_BLOCK) k_mom_first(int64_t n, const double* __restrict__ c,
                                                        const double* __restrict__ lnw, Mom1* __restrict__ part) {
  __shared__ Mom1 sh[MOM_BLOCK];
  Mom1 a;
  a.m = -__builtin_inf();
  a.s = 0.0;
#pragma unroll
  for (int j = 0; j < 7; ++j) a.c[j] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double w = lnw ? lnw[i] : 0.0;
    if (w == -__builtin_inf()) continue;
    double x[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) x[j] = c[j * n + i];
    mom_push(a, w, x);
  }
  const Mom1 r = mom_block(a, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// The weights' normaliser and the mean: st = (m, s, mean[7]); NaN mean when
// no sample carries weight or a weight is NaN.
__global__ void __launch_bounds__(MOM_BLOCK) k_mom_mean(int nb, const Mom1* __restrict__ part,
                                                       double* __restrict__ st) {
  __shared__ Mom1 sh[MOM_BLOCK];
  Mom1 a;
  a.m = -__builtin_inf();
  a.s = 0.0;
#pragma unroll
  for (int j = 0; j < 7; ++j) a.c[j] = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) a = mom_merge(a, part[b]);
  const Mom1 r = mom_block(a, sh);
  if (threadIdx.x == 0) {
    const bool ok = r.m == r.m && r.s > 0.0 && r.m != -__builtin_inf();
    st[0] = r.m;
    st[1] = ok ? r.s : __builtin_nan("");
#pragma unroll
    for (int j = 0; j < 7; ++j) st[2 + j] = ok ? r.c[j] / r.s : __builtin_nan("");
  }
}

// Sum over a block of 28 values per thread (wave shuffles, then the waves).
__device__ void sum28_block(double* v, double* sh) {
#pragma unroll
  for (int k = 0; k < 28; ++k) {
    double x = v[k];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    v[k] = x;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 28; ++k) sh[wave * 28 + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < MOM_BLOCK / 64; ++w)
#pragma unroll
      for (int k = 0; k < 28; ++k) v[k] += sh[w * 28 + k];
  }
}

// Centred second moments: sum_i W_i d_j d_k (j <= k), W_i = e^{w_i - m} / s.
__global__ void __launch_bounds__(MOM_BLOCK) k_mom_second(int64_t n, const double* __restrict__ c,
                                                         const double* __restrict__ lnw,
                                                         const double* __restrict__ st, double* __restrict__ part) {
  __shared__ double sh[(MOM_BLOCK / 64) * 28];
  const double m = st[0], s = st[1];
  double mu[7];
#pragma unroll
  for (int j = 0; j < 7; ++j) mu[j] = st[2 + j];
  double acc[28];
#pragma unroll
  for (int k = 0; k < 28; ++k) acc[k] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double w = lnw ? lnw[i] : 0.0;
    if (w == -__builtin_inf()) continue;
    const double W = exp(w - m) / s;
    double d[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) d[j] = c[j * n + i] - mu[j];
    int k = 0;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      const double wd = W * d[j];
#pragma unroll
      for (int l = j; l < 7; ++l) acc[k++] += wd * d[l];
    }
  }
  sum28_block(acc, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 28; ++k) part[blockIdx.x * 28 + k] = acc[k];
  }
}

__global__ void __launch_bounds__(MOM_BLOCK) k_mom_final(int nb, const double* __restrict__ part,
                                                        const double* __restrict__ st, double* __restrict__ mean,
                                                        double* __restrict__ cov) {
  __shared__ double sh[(MOM_BLOCK / 64) * 28];
  double acc[28];
#pragma unroll
  for (int k = 0; k < 28; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
    for (int k = 0; k < 28; ++k) acc[k] += part[b * 28 + k];
  sum28_block(acc, sh);
  if (threadIdx.x == 0) {
    const bool ok = st[1] == st[1];
    int k = 0;
    for (int j = 0; j < 7; ++j) {
      mean[j] = st[2 + j];
      for (int l = j; l < 7; ++l) {
        const double v = ok ? acc[k] : __builtin_nan("");
        cov[j * 7 + l] = v;
        cov[l * 7 + j] = v;
        ++k;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Mixture draws and weights
// ---------------------------------------------------------------------------

// One component's table (98 doubles).  L and its inverse Li are lower
// triangular, packed by rows (row r starts at r (r + 1) / 2).
struct IsComp {
  double mu[7];     // the mean as given (the draws)
  double mur[7];    // the mean with ra, psi, phiref reduced into [0, P) (the density)
  double L[28];     // Cholesky factor of s C_m
  double Li[28];    // L^-1
  double g[3][7];   // P_j times column j of L^-1 for the periodic rows (one image step), the row
                    // with the most images last
  double lognorm;   // ln((1 - alpha) a_m) - sum_j ln L_jj - 3.5 ln(2 pi)
  double thr;       // alpha + (1 - alpha) (a_0 + .. + a_m)
  double K[3];      // image half-counts in the order of g
  double gg, egg;   // |g[2]|^2 and e^{-|g[2]|^2}
};

struct IsArgs {
  int32_t n_comp, rows, n_rows;  // rows: bit j set when row j is sampled by the components
  double alpha, scale;
  double a[RIFT_IS_MAX_COMP];
  double t_min, t_max, lnd_min, lnd_max, d3min, d3span;
  double lc[7];  // the constant part of each row's normalised prior log-density
};

__device__ __forceinline__ int tri(int r) { return r * (r + 1) / 2; }

// One thread per component: factor, invert, image counts, normaliser and the
// component's selection threshold.  status[0] = 0, or 1 + the first refused
// component (s C_m not positive definite or not finite, or wider than half a
// period in a periodic row).
__global__ void k_is_setup(IsArgs A, const double* __restrict__ mean, const double* __restrict__ cov,
                           IsComp* __restrict__ tab, int32_t* __restrict__ status, int32_t* __restrict__ user) {
  __shared__ int first_bad;
  if (threadIdx.x == 0) first_bad = INT_MAX;
  __syncthreads();
  const int m = threadIdx.x;
  if (m < A.n_comp) {
    IsComp T;
    bool ok = true;
    // the sampled rows' covariance embedded in 7 x 7 with the identity on the
    // other rows (no cross terms, so their factor rows are unit and unused)
    double S[7][7];
    for (int r = 0; r < 7; ++r)
      for (int q = 0; q <= r; ++q) {
        const bool sr = (A.rows >> r) & 1, sq = (A.rows >> q) & 1;
        S[r][q] = (sr && sq) ? A.scale * cov[(size_t)m * 49 + r * 7 + q] : (r == q ? 1.0 : 0.0);  // lower triangle
      }
    for (int j = 0; j < 7; ++j) T.mu[j] = T.mur[j] = ((A.rows >> j) & 1) ? mean[m * 7 + j] : 0.0;
    // Cholesky by columns of rows
    for (int r = 0; r < 7; ++r) {
      for (int q = 0; q <= r; ++q) {
        double v = S[r][q];
        for (int k = 0; k < q; ++k) v -= T.L[tri(r) + k] * T.L[tri(q) + k];
        if (q == r) {
          ok = ok && v > 0.0 && v < __builtin_inf();
          T.L[tri(r) + r] = sqrt(v);
        } else {
          T.L[tri(r) + q] = v / T.L[tri(q) + q];
        }
      }
    }
    // inverse of the lower factor by forward substitution
    for (int q = 0; q < 7; ++q) {
      for (int r = 0; r < q; ++r) T.Li[tri(q) + r] = 0.0;
      T.Li[tri(q) + q] = 1.0 / T.L[tri(q) + q];
    }
    for (int r = 1; r < 7; ++r)
      for (int q = 0; q < r; ++q) {
        double v = 0.0;
        for (int k = q; k < r; ++k) v += T.L[tri(r) + k] * T.Li[tri(k) + q];
        T.Li[tri(r) + q] = -v / T.L[tri(r) + r];
      }
    double ldet = 0.0;
    for (int r = 0; r < 7; ++r) ldet += log(T.L[tri(r) + r]);
    double K[3];
    for (int p = 0; p < 3; ++p) {
      const int j = PER_ROW[p];
      const double P = period(p);
      T.mur[j] = T.mu[j] - P * floor(T.mu[j] / P);
      const bool sampled = (A.rows >> j) & 1;
      const double sig = sqrt(S[j][j]);
      ok = ok && (!sampled || (sig <= 0.5 * P && T.mu[j] == T.mu[j] && fabs(T.mu[j]) < 1e15));
      K[p] = (ok && sampled) ? fmax(0.0, ceil(9.0 * sig / P - 0.5)) : 0.0;
    }
    // the row with the most images innermost (summed by a recurrence)
    int inner = 2;
    if (K[0] > K[inner]) inner = 0;
    if (K[1] > K[inner]) inner = 1;
    int order[3] = {0, 1, 2};
    order[inner] = 2;
    order[2] = inner;
    for (int q = 0; q < 3; ++q) {
      const int p = order[q], j = PER_ROW[p];
      const double P = period(p);
      T.K[q] = K[p];
      for (int r = 0; r < 7; ++r) T.g[q][r] = r >= j ? P * T.Li[tri(r) + j] : 0.0;
    }
    T.gg = 0.0;
    for (int r = 0; r < 7; ++r) T.gg += T.g[2][r] * T.g[2][r];
    T.egg = exp(-T.gg);
    for (int j = 0; j < 7; ++j) ok = ok && T.mu[j] == T.mu[j] && fabs(T.mu[j]) < __builtin_inf();
    T.lognorm = log((1.0 - A.alpha) * A.a[m]) - ldet - 0.5 * A.n_rows * log(TWO_PI);
    double cum = 0.0;
    for (int k = 0; k <= m; ++k) cum += A.a[k];
    T.thr = A.alpha + (1.0 - A.alpha) * cum;
    tab[m] = T;
    if (!ok) atomicMin(&first_bad, m + 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int s = first_bad == INT_MAX ? 0 : first_bad;
    status[0] = s;
    if (user) user[0] = s;
  }
}

__device__ __forceinline__ void lse_push(double& mx, double& s, double v) {
  if (v == -__builtin_inf()) return;
  const double d = v - mx;
  const double e = exp(-fabs(d));
  const bool up = d > 0.0;
  s = up ? fma(s, e, 1.0) : s + e;
  mx = up ? v : mx;
}

__global__ void __launch_bounds__(IS_BLOCK) k_is_draw(int64_t n, IsArgs A, const IsComp* __restrict__ tab,
                                                     const int32_t* __restrict__ status,
                                                     const double* __restrict__ z, const double* __restrict__ v,
                                                     const double* __restrict__ u, double* __restrict__ theta,
                                                     double* __restrict__ lnw, int32_t* __restrict__ comp) {
  __shared__ IsComp sh[RIFT_IS_MAX_COMP];
  {
    const double* src = (const double*)tab;
    double* dst = (double*)sh;
    const int nd = A.n_comp * (int)(sizeof(IsComp) / sizeof(double));
    for (int k = threadIdx.x; k < nd; k += blockDim.x) dst[k] = src[k];
  }
  __syncthreads();
  const bool refused = status[0] != 0;
  const double ln_alpha = A.alpha > 0.0 ? log(A.alpha) : -__builtin_inf();
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double ui = u[i];
    double c[7];
    int m = -1;
    const bool all_rows = A.rows == 0x7f;
    if (ui < A.alpha || A.n_comp == 0 || !all_rows) {
      // a prior draw (the rows a component does not sample keep it)
      double w[7];
#pragma unroll
      for (int j = 0; j < 7; ++j) w[j] = v[j * n + i];
      c[0] = TWO_PI * w[0];
      c[1] = asin(2.0 * w[1] - 1.0);
      c[2] = PI * w[2];
      c[3] = 2.0 * w[3] - 1.0;
      c[4] = TWO_PI * w[4];
      c[5] = A.t_min + (A.t_max - A.t_min) * w[5];
      c[6] = log(A.d3min + w[6] * A.d3span) / 3.0;
    }
    if (!(ui < A.alpha || A.n_comp == 0)) {
      m = A.n_comp - 1;
      for (int k = 0; k < A.n_comp - 1; ++k)
        if (ui < sh[k].thr) {
          m = k;
          break;
        }
      double zz[7];
#pragma unroll
      for (int j = 0; j < 7; ++j) zz[j] = z[j * n + i];
      const IsComp& T = sh[m];
#pragma unroll
      for (int r = 0; r < 7; ++r) {
        double x = T.mu[r];
#pragma unroll
        for (int k = 0; k <= r; ++k) x += T.L[tri(r) + k] * zz[k];
        if ((A.rows >> r) & 1) c[r] = x;
      }
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        const int j = p == 0 ? 0 : (p == 1 ? 2 : 4);
        const double P = period(p);
        double x = c[j] - P * floor(c[j] / P);
        if (x >= P) x = 0.0;  // a rounding of a tiny negative value up to the period
        c[j] = x;
      }
    }
    // ln p of the sampled rows, normalised, on the box
    const bool in_row[7] = {c[0] >= 0.0 && c[0] < TWO_PI, fabs(c[1]) < HALF_PI, c[2] >= 0.0 && c[2] < PI,
                            fabs(c[3]) <= 1.0, c[4] >= 0.0 && c[4] < TWO_PI, c[5] >= A.t_min && c[5] <= A.t_max,
                            c[6] >= A.lnd_min && c[6] <= A.lnd_max};
    bool inside = true;
    double lp = 0.0;
#pragma unroll
    for (int j = 0; j < 7; ++j)
      if ((A.rows >> j) & 1) {
        inside = inside && in_row[j];
        lp += A.lc[j];
      }
    if (A.rows & 2) lp += log(cos(c[1]));
    if (A.rows & 64) lp += 3.0 * c[6];
    if (!inside) lp = -__builtin_inf();
    double out_w = -__builtin_inf();
    if (inside) {
      // ln q: the prior's share and every component's wrapped density
      double mx = -__builtin_inf(), s = 0.0;
      lse_push(mx, s, ln_alpha + lp);
      for (int k = 0; k < A.n_comp; ++k) {
        const IsComp& T = sh[k];
        if (T.lognorm == -__builtin_inf()) continue;
        double d[7];
#pragma unroll
        for (int j = 0; j < 7; ++j) d[j] = ((A.rows >> j) & 1) ? c[j] - T.mur[j] : 0.0;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
          const int j = p == 0 ? 0 : (p == 1 ? 2 : 4);
          const double P = period(p);
          d[j] -= P * rint(d[j] / P);
        }
        double y0[7];
#pragma unroll
        for (int r = 0; r < 7; ++r) {
          double x = 0.0;
#pragma unroll
          for (int q = 0; q <= r; ++q) x += T.Li[tri(r) + q] * d[q];
          y0[r] = x;
        }
        // the images: outer rows by loops; along the inner row the quadratic
        // form is Q(k) = C + 2 B k + A k^2, summed from its smallest term
        // outwards by the ratio e^{-(Q(k+-1) - Q(k))/2}, itself multiplied by
        // e^{-A} per step (two exponentials and a logarithm per line)
        const int Ka = (int)T.K[0], Kb = (int)T.K[1], Kc = (int)T.K[2];
        const double A = T.gg;
        for (int ka = -Ka; ka <= Ka; ++ka)
          for (int kb = -Kb; kb <= Kb; ++kb) {
            double C = 0.0, B = 0.0;
#pragma unroll
            for (int r = 0; r < 7; ++r) {
              const double b = y0[r] + ka * T.g[0][r] + kb * T.g[1][r];
              C += b * b;
              B += b * T.g[2][r];
            }
            if (Kc == 0) {
              lse_push(mx, s, T.lognorm - 0.5 * C);
              continue;
            }
            const double kc = fmin(fmax(rint(-B / A), (double)-Kc), (double)Kc);
            const double Qc = C + kc * (2.0 * B + A * kc);
            double line = 1.0, t = 1.0;
            double r = exp(-B - A * (kc + 0.5));
            for (int k = (int)kc + 1; k <= Kc; ++k) {
              t *= r;
              line += t;
              r *= T.egg;
            }
            t = 1.0;
            r = exp(B + A * (kc - 0.5));
            for (int k = (int)kc - 1; k >= -Kc; --k) {
              t *= r;
              line += t;
              r *= T.egg;
            }
            lse_push(mx, s, T.lognorm - 0.5 * Qc + log(line));
          }
      }
      const double lq = mx == -__builtin_inf() ? mx : mx + log(s);
      out_w = lp - lq;
    }
    // onto the box for the likelihood
    const double dec = fmin(fmax(c[1], -HALF_PI), HALF_PI);
    const double ci = fmin(fmax(c[3], -1.0), 1.0);
    const double t = fmin(fmax(c[5], A.t_min), A.t_max);
    const double lnd = fmin(fmax(c[6], A.lnd_min), A.lnd_max);
    double th[7] = {c[0], dec, c[2], acos(ci), c[4], t, exp(lnd)};
    if (refused) {
      out_w = __builtin_nan("");
#pragma unroll
      for (int j = 0; j < 7; ++j) th[j] = __builtin_nan("");
    }
#pragma unroll
    for (int j = 0; j < 7; ++j) theta[j * n + i] = th[j];
    lnw[i] = out_w;
    if (comp) comp[i] = m;
  }
}

bool misaligned(const void* q) { return !q || (((uintptr_t)q) & 7u); }

}  // namespace

extern "C" int rift_ile_moments(int64_t n, const double* c, const double* lnw, double* mean, double* cov,
                                void* stream) {
  if (n < 0 || misaligned(mean) || misaligned(cov) || (n > 0 && misaligned(c)) || (lnw && misaligned(lnw)))
    return RIFT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int nb = (int)std::min<int64_t>(std::max<int64_t>((n + MOM_BLOCK - 1) / MOM_BLOCK, 1), MOM_GRID_MAX);
  const size_t bytes = sizeof(Mom1) * (size_t)nb + sizeof(double) * (16 + 28 * (size_t)nb);
  void* w = nullptr;
  if (hipMallocAsync(&w, bytes, st) != hipSuccess) return RIFT_ENOMEM;
  Mom1* part1 = (Mom1*)w;
  double* S = (double*)(part1 + nb);
  double* part2 = S + 16;
  hipLaunchKernelGGL(k_mom_first, dim3(nb), dim3(MOM_BLOCK), 0, st, n, c, lnw, part1);
  hipLaunchKernelGGL(k_mom_mean, dim3(1), dim3(MOM_BLOCK), 0, st, nb, (const Mom1*)part1, S);
  hipLaunchKernelGGL(k_mom_second, dim3(nb), dim3(MOM_BLOCK), 0, st, n, c, lnw, (const double*)S, part2);
  hipLaunchKernelGGL(k_mom_final, dim3(1), dim3(MOM_BLOCK), 0, st, nb, (const double*)part2, (const double*)S, mean,
                     cov);
  int rc = hipGetLastError() != hipSuccess ? RIFT_EDEVICE : RIFT_OK;
  if (hipFreeAsync(w, st) != hipSuccess && !rc) rc = RIFT_EDEVICE;
  return rc;
}

extern "C" int rift_ile_mixture_is(int64_t n, const rift_ile_mixture* mix, const rift_ile_hmc_prior* prior,
                                   const double* z, const double* v, const double* u, double* theta, double* lnw,
                                   int32_t* comp, int32_t* status, void* stream) {
  if (n < 0 || !mix || !prior) return RIFT_EINVAL;
  const int nc = mix->n_comp;
  if (nc < 0 || nc > RIFT_IS_MAX_COMP) return RIFT_EINVAL;
  if (!(mix->alpha >= 0.0 && mix->alpha <= 1.0)) return RIFT_EINVAL;
  if (nc == 0 && mix->alpha != 1.0) return RIFT_EINVAL;
  if (mix->rows < 1 || mix->rows > 0x7f) return RIFT_EINVAL;
  if (!(mix->scale > 0.0 && mix->scale < __builtin_inf())) return RIFT_EINVAL;
  if (!(prior->t_min < prior->t_max) || !std::isfinite(prior->t_min) || !std::isfinite(prior->t_max) ||
      !(prior->d_min > 0.0 && prior->d_min < prior->d_max) || !std::isfinite(prior->d_max))
    return RIFT_EINVAL;
  IsArgs A{};
  A.n_comp = nc;
  A.rows = mix->rows;
  A.n_rows = __builtin_popcount((unsigned)mix->rows);
  A.alpha = mix->alpha;
  A.scale = mix->scale;
  if (nc > 0) {
    if (!mix->a || misaligned(mix->mean) || misaligned(mix->cov)) return RIFT_EINVAL;
    double sum = 0.0;
    for (int m = 0; m < nc; ++m) {
      if (!(mix->a[m] > 0.0 && mix->a[m] < __builtin_inf())) return RIFT_EINVAL;
      A.a[m] = mix->a[m];
      sum += mix->a[m];
    }
    if (!(fabs(sum - 1.0) <= 1e-12)) return RIFT_EINVAL;
  }
  if (n > 0 && (misaligned(z) || misaligned(v) || misaligned(u) || misaligned(theta) || misaligned(lnw) ||
                (comp && (((uintptr_t)comp) & 3u))))
    return RIFT_EINVAL;
  if (status && (((uintptr_t)status) & 3u)) return RIFT_EINVAL;
  A.t_min = prior->t_min;
  A.t_max = prior->t_max;
  A.lnd_min = log(prior->d_min);
  A.lnd_max = log(prior->d_max);
  A.d3min = prior->d_min * prior->d_min * prior->d_min;
  A.d3span = prior->d_max * prior->d_max * prior->d_max - A.d3min;
  const double lc[7] = {-log(TWO_PI), -log(2.0), -log(PI), -log(2.0), -log(TWO_PI),
                        -log(prior->t_max - prior->t_min), log(3.0) - log(A.d3span)};
  for (int j = 0; j < 7; ++j) A.lc[j] = lc[j];
  hipStream_t st = (hipStream_t)stream;
  const size_t bytes = sizeof(IsComp) * (size_t)std::max(nc, 1) + 256;
  void* w = nullptr;
  if (hipMallocAsync(&w, bytes, st) != hipSuccess) return RIFT_ENOMEM;
  IsComp* tab = (IsComp*)w;
  int32_t* stat = (int32_t*)(tab + std::max(nc, 1));
  hipLaunchKernelGGL(k_is_setup, dim3(1), dim3(64), 0, st, A, mix->mean, mix->cov, tab, stat, status);
  if (n > 0) {
    const int nb = (int)std::min<int64_t>((n + IS_BLOCK - 1) / IS_BLOCK, 8192);
    hipLaunchKernelGGL(k_is_draw, dim3(nb), dim3(IS_BLOCK), 0, st, n, A, (const IsComp*)tab, (const int32_t*)stat, z,
                       v, u, theta, lnw, comp);
  }
  int rc = hipGetLastError() != hipSuccess ? RIFT_EDEVICE : RIFT_OK;
  if (hipFreeAsync(w, st) != hipSuccess && !rc) rc = RIFT_EDEVICE;
  return rc;
}
