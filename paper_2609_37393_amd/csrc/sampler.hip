// Building block of gradient-based samplers on the likelihood's gradient
// (Sec. "Sampling the differentiable extrinsic likelihood"): the position
// update (drift) of a leapfrog step in the sampler's coordinates
// (ra, dec, psi, cos incl, phiref, tref, ln dist), theta += step * p, with a
// reflecting boundary on cos incl: a state that leaves [-1, 1] is folded back
// (a triangle wave of period 4) and its momentum in cos incl changes sign
// after an odd number of folds, which keeps the dynamics reversible and
// volume-preserving on the bounded coordinate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "../../include/rift_ile.h"

namespace {

struct Step7 {
  double s[7];
};

// theta_a += step_a p_a for one coordinate; for cos incl (a == 3) a result
// outside [-1, 1] is folded back, c' = 1 - |((c + 1) mod 4) - 2|, and p_a
// changes sign after an odd number of folds.  Non-finite values pass.
__device__ __forceinline__ double drift_one(int a, double c, double& p, double step) {
  double q = c + step * p;
  if (a == 3 && !(fabs(q) <= 1.0) && q == q && fabs(q) < 1.0e300) {
    double r = fmod(q + 1.0, 4.0);
    if (r < 0.0) r += 4.0;
    q = 1.0 - fabs(r - 2.0);
    if (r > 2.0) p = -p;
  }
  return q;
}

__global__ void k_drift(int64_t n, double* __restrict__ theta, double* __restrict__ p, Step7 step) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      double pa = p[a * n + i];
      theta[a * n + i] = drift_one(a, theta[a * n + i], pa, step.s[a]);
      if (a == 3) p[a * n + i] = pa;
    }
  }
}

struct HmcPrior {
  double t_min, t_max, lnd_min, lnd_max;
};

// ln of the prior density in the sampler coordinates, up to a constant: the
// isotropic, uniform-in-volume prior is ln cos dec + 3 ln D on the box (ra,
// psi and phiref periodic, cos incl in [-1, 1]), -inf outside.
__device__ __forceinline__ double hmc_log_prior(const HmcPrior& P, double dec, double ci, double t, double lnd) {
  const bool inside = fabs(dec) < 1.57079632679489661923 && fabs(ci) <= 1.0 && t >= P.t_min && t <= P.t_max &&
                      lnd >= P.lnd_min && lnd <= P.lnd_max;
  return inside ? log(cos(dec)) + 3.0 * lnd : -__builtin_inf();
}

// d ln pi / dc_a = dlnL/dc_a + d ln prior / dc_a; the prior's part is
// -tan(dec) in dec and 3 in ln D.
__device__ __forceinline__ double dlnpi(int a, double g, double dec) {
  if (a == 1) return g - tan(dec);
  if (a == 6) return g + 3.0;
  return g;
}

// The start of a transition, after the gradient at the start state: momenta
// p = z / sigma (mass diag(sigma^-2)), the start state and lnL kept, the start
// energy H0 = -lnL - ln prior + sum sigma^2 p^2 / 2, then the first half kick
// p += h dlnpi/dc and the first drift.
__global__ void k_hmc_first(int64_t n, double* __restrict__ c, const double* __restrict__ z,
                            const double* __restrict__ g, const double* __restrict__ lnL, double h, Step7 sig,
                            Step7 step, HmcPrior P, double* __restrict__ p, double* __restrict__ c0,
                            double* __restrict__ H0, double* __restrict__ lnL0) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double ca[7], pa[7];
    double kin = 0.0;
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      ca[a] = c[a * n + i];
      pa[a] = z[a * n + i] / sig.s[a];
      const double v = sig.s[a] * pa[a];
      kin = fma(v, v, kin);
      c0[a * n + i] = ca[a];
    }
    const double l = lnL[i];
    H0[i] = -(l + hmc_log_prior(P, ca[1], ca[3], ca[5], ca[6])) + 0.5 * kin;
    lnL0[i] = l;
    const double dec = ca[1];
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      pa[a] = fma(h, dlnpi(a, g[a * n + i], dec), pa[a]);
      c[a * n + i] = drift_one(a, ca[a], pa[a], step.s[a]);
      p[a * n + i] = pa[a];
    }
  }
}

// Between two drifts: the half kick that ends one leapfrog step and the one
// that starts the next (both at the current state), then the drift.
__global__ void k_hmc_mid(int64_t n, double* __restrict__ c, double* __restrict__ p, const double* __restrict__ g,
                          double h, Step7 step) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double dec = c[n + i];
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      const double ga = dlnpi(a, g[a * n + i], dec);
      double pa = fma(h, ga, p[a * n + i]);
      pa = fma(h, ga, pa);
      c[a * n + i] = drift_one(a, c[a * n + i], pa, step.s[a]);
      p[a * n + i] = pa;
    }
  }
}

// The last half kick, the final energy, acceptance against ln u and the
// returned state: the proposal if accepted, else the start state and its lnL.
__global__ void k_hmc_end(int64_t n, double* __restrict__ c, const double* __restrict__ p,
                          const double* __restrict__ g, const double* __restrict__ lnL1, double h,
                          const double* __restrict__ c0, const double* __restrict__ lnL0,
                          const double* __restrict__ H0, const double* __restrict__ u, Step7 sig, HmcPrior P,
                          double* __restrict__ lnL_out, int32_t* __restrict__ accepted) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double dec = c[n + i];
    double kin = 0.0;
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      const double pa = fma(h, dlnpi(a, g[a * n + i], dec), p[a * n + i]);
      const double v = sig.s[a] * pa;
      kin = fma(v, v, kin);
    }
    const double H1 = -(lnL1[i] + hmc_log_prior(P, dec, c[3 * n + i], c[5 * n + i], c[6 * n + i])) + 0.5 * kin;
    const double d = H0[i] - H1;
    const bool acc = (fabs(H1) <= 1.0e300) && (log(u[i]) < d);
    if (!acc) {
#pragma unroll
      for (int a = 0; a < 7; ++a) c[a * n + i] = c0[a * n + i];
    }
    if (lnL_out) lnL_out[i] = acc ? lnL1[i] : lnL0[i];
    if (accepted) accepted[i] = acc ? 1 : 0;
  }
}

}  // namespace

extern "C" int rift_ile_leapfrog_drift(int64_t n, double* theta, double* p, const double* step, void* stream) {
  if (n < 0 || !step) return RIFT_EINVAL;
  if (n == 0) return RIFT_OK;
  if (!theta || !p || (((uintptr_t)theta) & 7u) || (((uintptr_t)p) & 7u)) return RIFT_EINVAL;
  Step7 s;
  for (int a = 0; a < 7; ++a) {
    if (!std::isfinite(step[a])) return RIFT_EINVAL;
    s.s[a] = step[a];
  }
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_drift, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, n, theta, p, s);
  return hipGetLastError() == hipSuccess ? RIFT_OK : RIFT_EDEVICE;
}

extern "C" int rift_ile_plan_hmc(rift_ile_plan plan, int32_t point, int64_t n, double* theta, const double* z,
                                 const double* u, const double* sigma, double eps, int32_t n_leapfrog,
                                 const rift_ile_hmc_prior* prior, double* lnL, int32_t* accepted, void* stream) {
  if (!plan || n < 0 || !sigma || !prior) return RIFT_EINVAL;
  if (!(eps > 0.0) || !std::isfinite(eps) || n_leapfrog < 1 || n_leapfrog > 10000) return RIFT_EINVAL;
  if (!std::isfinite(prior->t_min) || !std::isfinite(prior->t_max) || !(prior->t_max > prior->t_min)) return RIFT_EINVAL;
  if (!(prior->d_min > 0.0) || !(prior->d_max > prior->d_min) || !std::isfinite(prior->d_max)) return RIFT_EINVAL;
  Step7 sig, step;
  for (int a = 0; a < 7; ++a) {
    if (!(sigma[a] > 0.0) || !std::isfinite(sigma[a])) return RIFT_EINVAL;
    sig.s[a] = sigma[a];
    step.s[a] = eps * sigma[a] * sigma[a];
  }
  if (n == 0) return RIFT_OK;
  auto bad = [](const void* q) { return !q || (((uintptr_t)q) & 7u); };
  if (bad(theta) || bad(z) || bad(u) || (lnL && bad(lnL)) || (accepted && (((uintptr_t)accepted) & 3u)))
    return RIFT_EINVAL;
  HmcPrior P;
  P.t_min = prior->t_min;
  P.t_max = prior->t_max;
  P.lnd_min = log(prior->d_min);
  P.lnd_max = log(prior->d_max);
  hipStream_t st = (hipStream_t)stream;
  // stream-ordered scratch: p, c0, g [7][n]; lnL, lnL0, H0 [n]
  double* w = nullptr;
  if (hipMallocAsync((void**)&w, sizeof(double) * 24 * (size_t)n, st) != hipSuccess) return RIFT_ENOMEM;
  double *p = w, *c0 = w + 7 * n, *g = w + 14 * n, *l1 = w + 21 * n, *l0 = w + 22 * n, *H0 = w + 23 * n;
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  constexpr int coords = RIFT_COORD_COS_INCL | RIFT_COORD_LN_DIST;
  const double h = 0.5 * eps;
  // L + 1 gradients; between them one fused kernel each (kicks and drift)
  int rc = rift_ile_plan_grad(plan, point, n, theta, coords, l1, g, stream);
  if (!rc)
    hipLaunchKernelGGL(k_hmc_first, dim3(grid), dim3(256), 0, st, n, theta, z, (const double*)g, (const double*)l1, h,
                       sig, step, P, p, c0, H0, l0);
  for (int s = 1; s < n_leapfrog && !rc; ++s) {
    rc = rift_ile_plan_grad(plan, point, n, theta, coords, l1, g, stream);
    if (!rc) hipLaunchKernelGGL(k_hmc_mid, dim3(grid), dim3(256), 0, st, n, theta, p, (const double*)g, h, step);
  }
  if (!rc) rc = rift_ile_plan_grad(plan, point, n, theta, coords, l1, g, stream);
  if (!rc)
    hipLaunchKernelGGL(k_hmc_end, dim3(grid), dim3(256), 0, st, n, theta, (const double*)p, (const double*)g,
                       (const double*)l1, h, (const double*)c0, (const double*)l0, (const double*)H0, u, sig, P,
                       lnL, accepted);
  if (!rc && hipGetLastError() != hipSuccess) rc = RIFT_EDEVICE;
  if (hipFreeAsync(w, st) != hipSuccess && !rc) rc = RIFT_EDEVICE;
  return rc;
}
