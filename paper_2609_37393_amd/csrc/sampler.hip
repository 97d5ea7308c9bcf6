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
#include <vector>

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
  int32_t dmarg;  // the likelihood marginalised over distance: row 6 not part of the target
};

// ln of the prior density in the sampler coordinates, up to a constant: the
// isotropic, uniform-in-volume prior is ln cos dec + 3 ln D on the box (ra,
// psi and phiref periodic, cos incl in [-1, 1]), -inf outside.
// With the distance marginalised, the distance row is not part of the
// target: no ln D term and no distance box.
__device__ __forceinline__ double hmc_log_prior(const HmcPrior& P, double dec, double ci, double t, double lnd) {
  const bool inside = fabs(dec) < 1.57079632679489661923 && fabs(ci) <= 1.0 && t >= P.t_min && t <= P.t_max &&
                      (P.dmarg || (lnd >= P.lnd_min && lnd <= P.lnd_max));
  return inside ? log(cos(dec)) + (P.dmarg ? 0.0 : 3.0 * lnd) : -__builtin_inf();
}

// d ln pi / dc_a = dlnL/dc_a + d ln prior / dc_a; the prior's part is
// -tan(dec) in dec and 3 in ln D.
__device__ __forceinline__ double dlnpi(const HmcPrior& P, int a, double g, double dec) {
  if (a == 1) return g - tan(dec);
  if (a == 6) return P.dmarg ? 0.0 : g + 3.0;
  return g;
}

// The start of a transition, after the gradient at the start state: momenta
// p = z / sigma (mass diag(sigma^-2)), the start state and lnL kept, the start
// energy H0 = -lnL - ln prior + sum sigma^2 p^2 / 2, then the first half kick
// p += h dlnpi/dc and the first drift.
__global__ void k_hmc_first(int64_t n, double* __restrict__ c, const double* __restrict__ z,
                            const double* __restrict__ g, const double* __restrict__ lnL, double h, double beta,
                            Step7 sig, Step7 step, HmcPrior P, double* __restrict__ p, double* __restrict__ c0,
                            double* __restrict__ H0, double* __restrict__ lnL0) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double ca[7], pa[7];
    double kin = 0.0;
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      ca[a] = c[a * n + i];
      pa[a] = (P.dmarg && a == 6) ? 0.0 : z[a * n + i] / sig.s[a];
      const double v = sig.s[a] * pa[a];
      kin = fma(v, v, kin);
      c0[a * n + i] = ca[a];
    }
    const double l = lnL[i];
    H0[i] = -(beta * l + hmc_log_prior(P, ca[1], ca[3], ca[5], ca[6])) + 0.5 * kin;
    lnL0[i] = l;
    const double dec = ca[1];
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      pa[a] = fma(h, dlnpi(P, a, beta * g[a * n + i], dec), pa[a]);
      c[a * n + i] = drift_one(a, ca[a], pa[a], step.s[a]);
      p[a * n + i] = pa[a];
    }
  }
}

// Between two drifts: the half kick that ends one leapfrog step and the one
// that starts the next (both at the current state), then the drift.
__global__ void k_hmc_mid(int64_t n, double* __restrict__ c, double* __restrict__ p, const double* __restrict__ g,
                          double h, double beta, Step7 step, HmcPrior P) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double dec = c[n + i];
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      const double ga = dlnpi(P, a, beta * g[a * n + i], dec);
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
                          const double* __restrict__ g, const double* __restrict__ lnL1, double h, double beta,
                          const double* __restrict__ c0, const double* __restrict__ lnL0,
                          const double* __restrict__ H0, const double* __restrict__ u, Step7 sig, HmcPrior P,
                          double* __restrict__ lnL_out, int32_t* __restrict__ accepted) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double dec = c[n + i];
    double kin = 0.0;
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      const double pa = fma(h, dlnpi(P, a, beta * g[a * n + i], dec), p[a * n + i]);
      const double v = sig.s[a] * pa;
      kin = fma(v, v, kin);
    }
    const double H1 =
        -(beta * lnL1[i] + hmc_log_prior(P, dec, c[3 * n + i], c[5 * n + i], c[6 * n + i])) + 0.5 * kin;
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

// ---------------------------------------------------------------------------
// No-U-Turn transitions (multinomial NUTS with the generalised criterion) of
// a batch of chains in lockstep: every pass takes one leapfrog step of every
// active chain from its own moving edge in its own direction, with one
// gradient launch for the batch between a "pre" kernel (half kick and drift)
// and a "post" kernel (half kick, energy, leaf sampling, U-turn checks,
// merge).  Per-chain state is SoA in a stream-ordered scratch; the random
// numbers are the caller's.
// ---------------------------------------------------------------------------
constexpr int NUTS_MAX_DEPTH = 10;
constexpr double NUTS_MAX_DH = 1000.0;

// Row offsets (in units of n doubles) of the state.
struct NutsLayout {
  int cL, pL, gL, cR, pR, gR, cX, pX, gX, cS, lS, cT, lT, rho, rhoS, ckP, ckS, H0, logW, logWs, lX, cE, lE, gE;
  int rows;
};
__host__ __device__ inline NutsLayout nuts_layout(int D) {
  NutsLayout L;
  int r = 0;
  L.cL = r; r += 7; L.pL = r; r += 7; L.gL = r; r += 7;
  L.cR = r; r += 7; L.pR = r; r += 7; L.gR = r; r += 7;
  L.cX = r; r += 7; L.pX = r; r += 7; L.gX = r; r += 7;
  L.cS = r; r += 7; L.lS = r; r += 1; L.cT = r; r += 7; L.lT = r; r += 1;
  L.rho = r; r += 7; L.rhoS = r; r += 7;
  L.ckP = r; r += 7 * D; L.ckS = r; r += 7 * D;
  L.H0 = r++; L.logW = r++; L.logWs = r++; L.lX = r++;
  L.cE = r; r += 7; L.lE = r; r += 1; L.gE = r; r += 7;
  L.rows = r;
  return L;
}
// int state rows: depth j, leaf k within the subtree, direction, leaves used,
// status (1 active), divergent, leapfrog steps
enum { NI_J = 0, NI_K, NI_DIR, NI_LEAF, NI_ACT, NI_DIV, NI_STEPS, NI_ROWS };

__device__ __forceinline__ double lae(double a, double b) {  // ln(e^a + e^b)
  const double m = fmax(a, b);
  if (m == -__builtin_inf()) return m;
  return m + log(exp(a - m) + exp(b - m));
}

__device__ __forceinline__ double nuts_energy(const HmcPrior& P, double beta, double l, const double* c,
                                              const double* p, Step7 sig) {
  double kin = 0.0;
#pragma unroll
  for (int a = 0; a < 7; ++a) {
    const double v = sig.s[a] * p[a];
    kin = fma(v, v, kin);
  }
  return -(beta * l + hmc_log_prior(P, c[1], c[3], c[5], c[6])) + 0.5 * kin;
}

// After the gradient at the start: momenta, start energy, the one-state
// trajectory.  A start whose energy is not finite is done at once.
__global__ void k_nuts_init(int64_t n, const double* __restrict__ c0, const double* __restrict__ z, Step7 sig,
                            double beta, HmcPrior P, double* __restrict__ W, int32_t* __restrict__ I, NutsLayout Ly) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double c[7], p[7];
    const double l = W[Ly.lE * n + i];
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      c[a] = c0[a * n + i];
      p[a] = (P.dmarg && a == 6) ? 0.0 : z[a * n + i] / sig.s[a];
    }
    const double dec = c[1];
    const double H0 = nuts_energy(P, beta, l, c, p, sig);
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      const double g = dlnpi(P, a, beta * W[(Ly.gE + a) * n + i], dec);
      W[(Ly.cL + a) * n + i] = c[a];
      W[(Ly.pL + a) * n + i] = p[a];
      W[(Ly.gL + a) * n + i] = g;
      W[(Ly.cR + a) * n + i] = c[a];
      W[(Ly.pR + a) * n + i] = p[a];
      W[(Ly.gR + a) * n + i] = g;
      W[(Ly.cS + a) * n + i] = c[a];
      W[(Ly.rho + a) * n + i] = p[a];
    }
    W[Ly.lS * n + i] = l;
    W[Ly.H0 * n + i] = H0;
    W[Ly.logW * n + i] = 0.0;
    I[NI_J * n + i] = 0;
    I[NI_K * n + i] = 0;
    I[NI_DIR * n + i] = 1;
    I[NI_LEAF * n + i] = 0;
    I[NI_ACT * n + i] = (fabs(H0) <= 1.0e300) ? 1 : 0;
    I[NI_DIV * n + i] = 0;
    I[NI_STEPS * n + i] = 0;
  }
}

// Half kick and drift of every active chain from its moving edge (a new
// subtree starts from the trajectory's edge in the drawn direction); the
// point to evaluate goes to cE (inactive chains evaluate their candidate).
__global__ void k_nuts_pre(int64_t n, const double* __restrict__ dirs, double eps, Step7 sig2, double* __restrict__ W,
                           int32_t* __restrict__ I, NutsLayout Ly) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (!I[NI_ACT * n + i]) {
#pragma unroll
      for (int a = 0; a < 7; ++a) W[(Ly.cE + a) * n + i] = W[(Ly.cS + a) * n + i];
      continue;
    }
    const int j = I[NI_J * n + i];
    if (I[NI_K * n + i] == 0) {
      const int d = dirs[(int64_t)j * n + i] < 0.5 ? -1 : 1;
      I[NI_DIR * n + i] = d;
      const int c = d < 0 ? Ly.cL : Ly.cR, pp = d < 0 ? Ly.pL : Ly.pR, g = d < 0 ? Ly.gL : Ly.gR;
#pragma unroll
      for (int a = 0; a < 7; ++a) {
        W[(Ly.cX + a) * n + i] = W[(c + a) * n + i];
        W[(Ly.pX + a) * n + i] = W[(pp + a) * n + i];
        W[(Ly.gX + a) * n + i] = W[(g + a) * n + i];
        W[(Ly.rhoS + a) * n + i] = 0.0;
      }
      W[Ly.logWs * n + i] = -__builtin_inf();
    }
    const double h = 0.5 * eps * (double)I[NI_DIR * n + i];
    const double ds = eps * (double)I[NI_DIR * n + i];
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      double pa = fma(h, W[(Ly.gX + a) * n + i], W[(Ly.pX + a) * n + i]);
      const double ca = drift_one(a, W[(Ly.cX + a) * n + i], pa, ds * sig2.s[a]);
      W[(Ly.cX + a) * n + i] = ca;
      W[(Ly.pX + a) * n + i] = pa;
      W[(Ly.cE + a) * n + i] = ca;
    }
  }
}

__device__ __forceinline__ bool no_uturn(const double* pa, const double* pb, const double* rho, Step7 sig2) {
  double da = 0.0, db = 0.0;
#pragma unroll
  for (int a = 0; a < 7; ++a) {
    da = fma(sig2.s[a] * pa[a], rho[a], da);
    db = fma(sig2.s[a] * pb[a], rho[a], db);
  }
  return da > 0.0 && db > 0.0;
}

// The second half kick and the leaf's bookkeeping (see nuts_chain in the
// reference description: leaf sampling, block checks, merge, trajectory
// check).
__global__ void k_nuts_post(int64_t n, const double* __restrict__ merges, const double* __restrict__ leaves, double eps,
                            double beta, Step7 sig, Step7 sig2, HmcPrior P, int D, double* __restrict__ W,
                            int32_t* __restrict__ I, NutsLayout Ly) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (!I[NI_ACT * n + i]) continue;
    const int j = I[NI_J * n + i], k = I[NI_K * n + i], dir = I[NI_DIR * n + i];
    const double h = 0.5 * eps * (double)dir;
    double c[7], p[7], g[7];
#pragma unroll
    for (int a = 0; a < 7; ++a) c[a] = W[(Ly.cX + a) * n + i];
    const double l = W[Ly.lE * n + i];
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      g[a] = dlnpi(P, a, beta * W[(Ly.gE + a) * n + i], c[1]);
      p[a] = fma(h, g[a], W[(Ly.pX + a) * n + i]);
      W[(Ly.pX + a) * n + i] = p[a];
      W[(Ly.gX + a) * n + i] = g[a];
    }
    W[Ly.lX * n + i] = l;
    const int leaf = I[NI_LEAF * n + i] + 1;
    I[NI_LEAF * n + i] = leaf;
    I[NI_STEPS * n + i] += 1;
    const double H0 = W[Ly.H0 * n + i];
    const double H = nuts_energy(P, beta, l, c, p, sig);
    if (!(H - H0 <= NUTS_MAX_DH)) {
      I[NI_DIV * n + i] = 1;
      I[NI_ACT * n + i] = 0;
      continue;
    }
    const double lw = H0 - H;
    const double lws = lae(W[Ly.logWs * n + i], lw);
    W[Ly.logWs * n + i] = lws;
    if (leaves[(int64_t)(leaf - 1) * n + i] < exp(lw - lws)) {
#pragma unroll
      for (int a = 0; a < 7; ++a) W[(Ly.cT + a) * n + i] = c[a];
      W[Ly.lT * n + i] = l;
    }
    // block checkpoints: the first leaf of every block that starts here
    double rs[7];
#pragma unroll
    for (int a = 0; a < 7; ++a) rs[a] = W[(Ly.rhoS + a) * n + i];
    for (int lv = 1; lv <= j; ++lv) {
      if (k % (1 << lv) != 0) break;
#pragma unroll
      for (int a = 0; a < 7; ++a) {
        W[(Ly.ckP + 7 * (lv - 1) + a) * n + i] = p[a];
        W[(Ly.ckS + 7 * (lv - 1) + a) * n + i] = rs[a];
      }
    }
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      rs[a] += p[a];
      W[(Ly.rhoS + a) * n + i] = rs[a];
    }
    // U-turn checks of the blocks that end here, smallest first
    bool valid = true;
    for (int lv = 1; lv <= j && valid; ++lv) {
      if ((k + 1) % (1 << lv) != 0) break;
      double pa[7], rb[7];
#pragma unroll
      for (int a = 0; a < 7; ++a) {
        pa[a] = W[(Ly.ckP + 7 * (lv - 1) + a) * n + i];
        rb[a] = rs[a] - W[(Ly.ckS + 7 * (lv - 1) + a) * n + i];
      }
      valid = no_uturn(pa, p, rb, sig2);
    }
    if (!valid) {
      I[NI_ACT * n + i] = 0;
      continue;
    }
    if (k + 1 < (1 << j)) {
      I[NI_K * n + i] = k + 1;
      continue;
    }
    // the subtree is complete and valid: merge it
    const double logW = W[Ly.logW * n + i];
    if (merges[(int64_t)j * n + i] < exp(lws - logW)) {
#pragma unroll
      for (int a = 0; a < 7; ++a) W[(Ly.cS + a) * n + i] = W[(Ly.cT + a) * n + i];
      W[Ly.lS * n + i] = W[Ly.lT * n + i];
    }
    W[Ly.logW * n + i] = lae(logW, lws);
    double rho[7], pl[7], pr[7];
    const int ec = dir < 0 ? Ly.cL : Ly.cR, ep = dir < 0 ? Ly.pL : Ly.pR, eg = dir < 0 ? Ly.gL : Ly.gR;
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      rho[a] = W[(Ly.rho + a) * n + i] + rs[a];
      W[(Ly.rho + a) * n + i] = rho[a];
      W[(ec + a) * n + i] = c[a];
      W[(ep + a) * n + i] = p[a];
      W[(eg + a) * n + i] = g[a];
    }
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      pl[a] = W[(Ly.pL + a) * n + i];
      pr[a] = W[(Ly.pR + a) * n + i];
    }
    I[NI_J * n + i] = j + 1;
    I[NI_K * n + i] = 0;
    if (!no_uturn(pl, pr, rho, sig2) || j + 1 >= D) I[NI_ACT * n + i] = 0;
  }
}

__global__ void k_nuts_count(int64_t n, const int32_t* __restrict__ I, int32_t* __restrict__ cnt) {
  __shared__ int32_t sh[256];
  int32_t c = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    c += I[NI_ACT * n + i];
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) cnt[blockIdx.x] = sh[0];
}

__global__ void k_nuts_out(int64_t n, const double* __restrict__ W, const int32_t* __restrict__ I, NutsLayout Ly,
                           double* __restrict__ theta, double* __restrict__ lnL, int32_t* __restrict__ info) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int a = 0; a < 7; ++a) theta[a * n + i] = W[(Ly.cS + a) * n + i];
    if (lnL) lnL[i] = W[Ly.lS * n + i];
    if (info) {
      info[i] = I[NI_J * n + i];
      info[n + i] = I[NI_STEPS * n + i];
      info[2 * n + i] = I[NI_DIV * n + i];
    }
  }
}

// ---------------------------------------------------------------------------
// The SMC ladder's update (Eq. (sampler-menu:smc-update)) on the tempered
// targets L^beta p (Eq. (sampler-menu:tempered-target)).  Log-sums run
// online as (max, sum e^{v - max}, sum e^{v - max} l) triples with one exp
// per term and no divergent branch; L^0 = 1 also where ln L = -inf.
// ---------------------------------------------------------------------------
constexpr int SMC_BLOCK = 256;
constexpr int SMC_GRID_MAX = 1024;
constexpr int SMC_ITERS = 40;

struct Acc3 {
  double m, s, t;
};

__device__ __forceinline__ void acc_push(Acc3& a, double v, double l) {
  if (v == -__builtin_inf()) return;
  const double d = v - a.m;
  const double e = exp(-fabs(d));
  const bool up = d > 0.0;
  a.s = up ? fma(a.s, e, 1.0) : a.s + e;
  a.t = up ? fma(a.t, e, l) : fma(e, l, a.t);
  a.m = up ? v : a.m;
}

__device__ __forceinline__ Acc3 acc_merge(Acc3 a, Acc3 b) {
  if (b.m == -__builtin_inf() && b.s == 0.0) return a;
  if (a.m == -__builtin_inf() && a.s == 0.0) return b;
  const double m = fmax(a.m, b.m);
  const double ea = exp(a.m - m), eb = exp(b.m - m);
  Acc3 r;
  r.m = (a.m == a.m && b.m == b.m) ? m : __builtin_nan("");
  r.s = a.s * ea + b.s * eb;
  r.t = a.t * ea + b.t * eb;
  return r;
}

// Block reduction of one triple (SMC_BLOCK threads); the result in thread 0.
__device__ Acc3 acc_block(Acc3 a, Acc3* sh) {
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int o = SMC_BLOCK / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = acc_merge(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  return sh[0];
}

__device__ __forceinline__ double tempered(double d, double l) { return d == 0.0 ? 0.0 : d * l; }

struct SmcState {
  double lnS;        // ln sum_i W_i of the input weights
  double rest;       // 1 - beta
  double lo, hi, d;  // bracket of the step and the current step
  int32_t done, iter;
};

// Pass over the samples: with which = 0 the triple of lnW alone; with
// which = 1 the triples of lnW + d l and lnW + 2 d l at the state's step
// (skipped once the search is done unless `force`).
__global__ void __launch_bounds__(SMC_BLOCK) k_smc_pass(int64_t n, const double* __restrict__ lnW,
                                                       const double* __restrict__ lnL,
                                                       const SmcState* __restrict__ st, int which, int force,
                                                       Acc3* __restrict__ part) {
  __shared__ Acc3 sh[SMC_BLOCK];
  if (which == 1 && st->done && !force) return;
  const double d = which == 1 ? st->d : 0.0;
  Acc3 a1{-__builtin_inf(), 0.0, 0.0}, a2{-__builtin_inf(), 0.0, 0.0};
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double w = lnW[i];
    if (which == 0) {
      acc_push(a1, w, 0.0);
    } else {
      const double l = lnL[i];
      acc_push(a1, w + tempered(d, l), l);
      acc_push(a2, w + tempered(2.0 * d, l), l);
    }
  }
  const Acc3 r1 = acc_block(a1, sh);
  __syncthreads();
  const Acc3 r2 = acc_block(a2, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r1;
    part[2 * blockIdx.x + 1] = r2;
  }
}

__device__ Acc3 combine_parts(int nb, const Acc3* __restrict__ part, int which, Acc3* sh) {
  Acc3 a{-__builtin_inf(), 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += blockDim.x) a = acc_merge(a, part[2 * b + which]);
  return acc_block(a, sh);
}

// The input weights' normaliser; the search starts at the whole remaining step.
__global__ void __launch_bounds__(SMC_BLOCK) k_smc_init(int nb, const Acc3* __restrict__ part, double rest,
                                                       SmcState* __restrict__ st) {
  __shared__ Acc3 sh[SMC_BLOCK];
  const Acc3 r = combine_parts(nb, part, 0, sh);
  if (threadIdx.x == 0) {
    st->lnS = r.m + log(r.s);
    st->rest = rest;
    st->lo = 0.0;
    st->hi = rest;
    st->d = rest;
    st->done = rest == 0.0 ? 1 : 0;
    st->iter = 0;
  }
}

// One step of the safeguarded Newton search for the largest step d in
// (0, rest] with ln cess(d) = 2 K(d) - K(2 d) >= ln target, K(d) =
// ln sum_i W_i L_i^d: the function is non-increasing in d with derivative
// 2 (mean_d l - mean_2d l), the means under the tilted weights.  A step that
// leaves the bracket bisects it instead.
__global__ void __launch_bounds__(SMC_BLOCK) k_smc_step(int nb, const Acc3* __restrict__ part, double ln_target,
                                                       SmcState* __restrict__ st) {
  __shared__ Acc3 sh[SMC_BLOCK];
  if (st->done) return;
  const Acc3 r1 = combine_parts(nb, part, 0, sh);
  __syncthreads();
  const Acc3 r2 = combine_parts(nb, part, 1, sh);
  if (threadIdx.x != 0) return;
  const double K1 = r1.m + log(r1.s) - st->lnS, K2 = r2.m + log(r2.s) - st->lnS;
  const double f = 2.0 * K1 - K2 - ln_target;
  const double fp = 2.0 * (r1.t / r1.s - r2.t / r2.s);
  double d = st->d, lo = st->lo, hi = st->hi;
  if (!(f == f)) {
    st->d = __builtin_nan("");
    st->done = 1;
    return;
  }
  if (st->iter == 0 && f >= 0.0) {
    st->done = 1;  // the whole remaining step qualifies
    return;
  }
  if (f >= 0.0) lo = d;
  else hi = d;
  double dn = d - f / fp;
  if (!(dn > lo && dn < hi)) dn = 0.5 * (lo + hi);
  const bool conv = fabs(dn - d) <= 4e-16 * d || hi - lo <= 4e-16 * hi;
  st->lo = lo;
  st->hi = hi;
  st->d = dn;
  st->iter += 1;
  st->done = conv ? 1 : 0;
}

// Outputs: beta + d and dlnZ = K(d) (from a pass at the final step).
__global__ void __launch_bounds__(SMC_BLOCK) k_smc_finish(int nb, const Acc3* __restrict__ part, double beta,
                                                         SmcState* __restrict__ st, double* __restrict__ out) {
  __shared__ Acc3 sh[SMC_BLOCK];
  const Acc3 r1 = combine_parts(nb, part, 0, sh);
  if (threadIdx.x == 0) {
    const double K1 = r1.m + log(r1.s) - st->lnS;
    out[0] = beta + st->d;
    out[1] = K1;
    st->lnS += K1;  // the new weights' normaliser, relative to the inputs
  }
}

// ln W_i <- ln W_i + d l_i - (lnS + dlnZ): normalised new weights.
__global__ void k_smc_apply(int64_t n, double* __restrict__ lnW, const double* __restrict__ lnL,
                            const SmcState* __restrict__ st) {
  const double d = st->d, c = st->lnS;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    lnW[i] = lnW[i] + tempered(d, lnL[i]) - c;
}

// Systematic resampling: the normalised cumulative weights by a two-level
// scan (SMC_CHUNK samples per block), then each draw's first index whose
// cumulative weight exceeds (i + u) / n, and the states gathered from it.
constexpr int SMC_CHUNK = 4 * SMC_BLOCK;

__global__ void __launch_bounds__(SMC_BLOCK) k_cdf_local(int64_t n, const double* __restrict__ lnW,
                                                        const SmcState* __restrict__ st, double* __restrict__ C,
                                                        double* __restrict__ bsum) {
  __shared__ double sh[SMC_BLOCK];
  const double lnS = st->lnS;
  const int64_t base = (int64_t)blockIdx.x * SMC_CHUNK + 4 * threadIdx.x;
  double v[4], run = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    v[q] = base + q < n ? exp(lnW[base + q] - lnS) : 0.0;
    run += v[q];
  }
  sh[threadIdx.x] = run;
  __syncthreads();
  // inclusive scan of the thread sums
  for (int o = 1; o < SMC_BLOCK; o <<= 1) {
    const double x = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0.0;
    __syncthreads();
    sh[threadIdx.x] += x;
    __syncthreads();
  }
  double acc = threadIdx.x > 0 ? sh[threadIdx.x - 1] : 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    acc += v[q];
    if (base + q < n) C[base + q] = acc;
  }
  if (threadIdx.x == SMC_BLOCK - 1) bsum[blockIdx.x] = sh[SMC_BLOCK - 1];
}

// Exclusive scan of the block sums (one block, sequential per thread chunk).
__global__ void __launch_bounds__(SMC_BLOCK) k_cdf_blocks(int nb, double* __restrict__ bsum) {
  __shared__ double sh[SMC_BLOCK];
  const int per = (nb + SMC_BLOCK - 1) / SMC_BLOCK;
  const int b0 = threadIdx.x * per;
  double run = 0.0;
  for (int b = b0; b < b0 + per && b < nb; ++b) run += bsum[b];
  sh[threadIdx.x] = run;
  __syncthreads();
  for (int o = 1; o < SMC_BLOCK; o <<= 1) {
    const double x = (int)threadIdx.x >= o ? sh[threadIdx.x - o] : 0.0;
    __syncthreads();
    sh[threadIdx.x] += x;
    __syncthreads();
  }
  double acc = threadIdx.x > 0 ? sh[threadIdx.x - 1] : 0.0;
  for (int b = b0; b < b0 + per && b < nb; ++b) {
    const double x = bsum[b];
    bsum[b] = acc;
    acc += x;
  }
}

__global__ void k_cdf_offset(int64_t n, double* __restrict__ C, const double* __restrict__ boff) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    C[i] += boff[i / SMC_CHUNK];
}

__global__ void k_resample_pick(int64_t n, const double* __restrict__ C, double u,
                                const double* __restrict__ th_in, double* __restrict__ th_out,
                                int64_t* __restrict__ anc) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double U = ((double)i + u) / (double)n;
    int64_t lo = 0, hi = n;  // first k with C[k] > U, in [0, n]
    while (lo < hi) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if (C[mid] > U) hi = mid;
      else lo = mid + 1;
    }
    const int64_t a = lo < n ? lo : n - 1;
    if (anc) anc[i] = a;
    if (th_out) {
#pragma unroll
      for (int r = 0; r < 7; ++r) th_out[r * n + i] = th_in[r * n + a];
    }
  }
}

// ---------------------------------------------------------------------------
// The cloud's random-walk Metropolis move (after resampling, with a proposal
// covariance estimated from the cloud): c' = c + L z, L L^T = scale C.

// One thread: the Cholesky factor of scale C (lower, packed by rows) into L;
// status 0, or 1 when scale C is not positive definite or not finite.
__global__ void k_rwm_setup(const double* __restrict__ cov, double scale, double* __restrict__ L,
                            int32_t* __restrict__ status, int32_t* __restrict__ user) {
  if (threadIdx.x != 0) return;
  bool ok = true;
  double F[28];
  for (int r = 0; r < 7; ++r)
    for (int q = 0; q <= r; ++q) {
      double v = scale * cov[r * 7 + q];
      for (int k = 0; k < q; ++k) v -= F[r * (r + 1) / 2 + k] * F[q * (q + 1) / 2 + k];
      if (q == r) {
        ok = ok && v > 0.0 && v < __builtin_inf();
        F[r * (r + 1) / 2 + r] = sqrt(v);
      } else {
        F[r * (r + 1) / 2 + q] = v / F[q * (q + 1) / 2 + q];
      }
    }
  for (int k = 0; k < 28; ++k) L[k] = ok ? F[k] : 0.0;
  status[0] = ok ? 0 : 1;
  if (user) user[0] = status[0];
}

__global__ void k_rwm_propose(int64_t n, const double* __restrict__ c, const double* __restrict__ z,
                              const double* __restrict__ L, double* __restrict__ c1) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double zz[7];
#pragma unroll
    for (int a = 0; a < 7; ++a) zz[a] = z[a * n + i];
#pragma unroll
    for (int r = 0; r < 7; ++r) {
      double x = c[r * n + i];
#pragma unroll
      for (int k = 0; k <= r; ++k) x += L[r * (r + 1) / 2 + k] * zz[k];
      c1[r * n + i] = x;
    }
  }
}

// Accepted when ln u < beta (lnL' - lnL) + ln p(c') - ln p(c) (L^0 = 1); a
// proposal outside the prior's box, a NaN, or a refused factor rejects.
__global__ void k_rwm_accept(int64_t n, double* __restrict__ c, const double* __restrict__ c1,
                             const double* __restrict__ l1, double* __restrict__ lnL, const double* __restrict__ u,
                             double beta, HmcPrior P, const int32_t* __restrict__ status,
                             int32_t* __restrict__ accepted) {
  const bool refused = status[0] != 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double lp0 = hmc_log_prior(P, c[n + i], c[3 * n + i], c[5 * n + i], c[6 * n + i]);
    const double lp1 = hmc_log_prior(P, c1[n + i], c1[3 * n + i], c1[5 * n + i], c1[6 * n + i]);
    const double l0 = lnL[i], ln1 = l1[i];
    const double d = (beta == 0.0 ? 0.0 : beta * (ln1 - l0)) + lp1 - lp0;
    const bool acc = !refused && lp1 != -__builtin_inf() && log(u[i]) < d;
    if (acc) {
#pragma unroll
      for (int a = 0; a < 7; ++a) c[a * n + i] = c1[a * n + i];
      lnL[i] = ln1;
    }
    if (accepted) accepted[i] = acc ? 1 : 0;
  }
}

// lnL and its gradient in the samplers' coordinates: of the likelihood, or,
// with a distance prior, of the likelihood marginalised over distance.
int sampler_grad(rift_ile_plan plan, int32_t point, int64_t n, const double* c, const rift_ile_dist_prior* dm,
                 double* l, double* g, void* stream) {
  constexpr int coords = RIFT_COORD_COS_INCL | RIFT_COORD_LN_DIST;
  return dm ? rift_ile_plan_grad_dmarg(plan, point, n, c, dm, l, g, stream)
            : rift_ile_plan_grad(plan, point, n, c, coords, l, g, stream);
}

bool bad_dist_prior(const rift_ile_dist_prior* dm) {
  return dm && (!(dm->d_min > 0.0) || !(dm->d_max > dm->d_min) || !(dm->d_max <= 1.0e60) || dm->n_nodes < 1 ||
                dm->n_nodes > 64);
}

}  // namespace

extern "C" int rift_ile_plan_rwm(rift_ile_plan plan, int32_t point, int64_t n, double* theta, const double* z,
                                 const double* u, const double* cov, double scale, const rift_ile_hmc_prior* prior,
                                 double beta, double* lnL, int32_t* accepted, int32_t* status, void* stream) {
  if (!plan || n < 0 || !prior) return RIFT_EINVAL;
  if (!(beta >= 0.0 && beta <= 1.0)) return RIFT_EINVAL;
  if (!(scale > 0.0) || !std::isfinite(scale)) return RIFT_EINVAL;
  if (!std::isfinite(prior->t_min) || !std::isfinite(prior->t_max) || !(prior->t_max > prior->t_min)) return RIFT_EINVAL;
  if (!(prior->d_min > 0.0) || !(prior->d_max > prior->d_min) || !std::isfinite(prior->d_max)) return RIFT_EINVAL;
  auto bad = [](const void* q) { return !q || (((uintptr_t)q) & 7u); };
  if (bad(cov) || (status && (((uintptr_t)status) & 3u))) return RIFT_EINVAL;
  if (n > 0 && (bad(theta) || bad(z) || bad(u) || bad(lnL) || (accepted && (((uintptr_t)accepted) & 3u))))
    return RIFT_EINVAL;
  HmcPrior P{};
  P.t_min = prior->t_min;
  P.t_max = prior->t_max;
  P.lnd_min = log(prior->d_min);
  P.lnd_max = log(prior->d_max);
  hipStream_t st = (hipStream_t)stream;
  // stream-ordered scratch: the factor and status, then c', g [7][n] and lnL' [n]
  double* w = nullptr;
  if (hipMallocAsync((void**)&w, sizeof(double) * (32 + 15 * (size_t)n), st) != hipSuccess) return RIFT_ENOMEM;
  double* L = w;
  int32_t* stat = (int32_t*)(w + 28);
  double *c1 = w + 32, *g = c1 + 7 * n, *l1 = g + 7 * n;
  hipLaunchKernelGGL(k_rwm_setup, dim3(1), dim3(64), 0, st, cov, scale, L, stat, status);
  int rc = RIFT_OK;
  if (n > 0) {
    const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
    constexpr int coords = RIFT_COORD_COS_INCL | RIFT_COORD_LN_DIST;
    hipLaunchKernelGGL(k_rwm_propose, dim3(grid), dim3(256), 0, st, n, (const double*)theta, z, (const double*)L,
                       c1);
    rc = rift_ile_plan_grad(plan, point, n, c1, coords, l1, g, stream);
    if (!rc)
      hipLaunchKernelGGL(k_rwm_accept, dim3(grid), dim3(256), 0, st, n, theta, (const double*)c1,
                         (const double*)l1, lnL, u, beta, P, (const int32_t*)stat, accepted);
  }
  if (!rc && hipGetLastError() != hipSuccess) rc = RIFT_EDEVICE;
  if (hipFreeAsync(w, st) != hipSuccess && !rc) rc = RIFT_EDEVICE;
  return rc;
}

static int nuts_impl(rift_ile_plan plan, int32_t point, int64_t n, double* theta, const double* z,
                     const double* dirs, const double* merges, const double* leaves, const double* sigma, double eps,
                     int32_t max_depth, const rift_ile_hmc_prior* prior, const rift_ile_dist_prior* dm, double beta,
                     double* lnL, int32_t* info, void* stream) {
  if (!plan || n < 0 || !sigma || !prior || bad_dist_prior(dm)) return RIFT_EINVAL;
  if (!(eps > 0.0) || !std::isfinite(eps) || max_depth < 1 || max_depth > NUTS_MAX_DEPTH) return RIFT_EINVAL;
  if (!(beta >= 0.0 && beta <= 1.0)) return RIFT_EINVAL;
  if (!std::isfinite(prior->t_min) || !std::isfinite(prior->t_max) || !(prior->t_max > prior->t_min)) return RIFT_EINVAL;
  if (!(prior->d_min > 0.0) || !(prior->d_max > prior->d_min) || !std::isfinite(prior->d_max)) return RIFT_EINVAL;
  Step7 sig, sig2;
  for (int a = 0; a < 7; ++a) {
    if (!(sigma[a] > 0.0) || !std::isfinite(sigma[a])) return RIFT_EINVAL;
    sig.s[a] = sigma[a];
    sig2.s[a] = sigma[a] * sigma[a];
  }
  if (n == 0) return RIFT_OK;
  auto bad = [](const void* q) { return !q || (((uintptr_t)q) & 7u); };
  if (bad(theta) || bad(z) || bad(dirs) || bad(merges) || bad(leaves) || (lnL && bad(lnL)) ||
      (info && (((uintptr_t)info) & 3u)))
    return RIFT_EINVAL;
  HmcPrior P{};
  P.t_min = prior->t_min;
  P.t_max = prior->t_max;
  P.lnd_min = log(prior->d_min);
  P.lnd_max = log(prior->d_max);
  hipStream_t st = (hipStream_t)stream;
  const NutsLayout Ly = nuts_layout(max_depth);
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  const unsigned cgrid = (unsigned)std::min<int64_t>((n + 255) / 256, 256);
  const size_t bytes = sizeof(double) * (size_t)Ly.rows * (size_t)n + sizeof(int32_t) * ((size_t)NI_ROWS * n + cgrid);
  void* w = nullptr;
  if (hipMallocAsync(&w, bytes, st) != hipSuccess) return RIFT_ENOMEM;
  double* Wd = (double*)w;
  int32_t* I = (int32_t*)(Wd + (size_t)Ly.rows * n);
  int32_t* cnt = I + (size_t)NI_ROWS * n;
  std::vector<int32_t> hc(cgrid);
  P.dmarg = dm ? 1 : 0;
  int rc = sampler_grad(plan, point, n, theta, dm, Wd + (size_t)Ly.lE * n, Wd + (size_t)Ly.gE * n, stream);
  if (!rc)
    hipLaunchKernelGGL(k_nuts_init, dim3(grid), dim3(256), 0, st, n, (const double*)theta, z, sig, beta, P, Wd, I, Ly);
  const int iters = (1 << max_depth) - 1;
  for (int it = 0; it < iters && !rc; ++it) {
    hipLaunchKernelGGL(k_nuts_pre, dim3(grid), dim3(256), 0, st, n, dirs, eps, sig2, Wd, I, Ly);
    rc = sampler_grad(plan, point, n, Wd + (size_t)Ly.cE * n, dm, Wd + (size_t)Ly.lE * n, Wd + (size_t)Ly.gE * n,
                      stream);
    if (rc) break;
    hipLaunchKernelGGL(k_nuts_post, dim3(grid), dim3(256), 0, st, n, merges, leaves, eps, beta, sig, sig2, P,
                       (int)max_depth, Wd, I, Ly);
    // every fourth pass, stop once no chain is active (synchronises)
    if ((it & 3) == 3 && it + 1 < iters) {
      hipLaunchKernelGGL(k_nuts_count, dim3(cgrid), dim3(256), 0, st, n, (const int32_t*)I, cnt);
      if (hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * cgrid, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        rc = RIFT_EDEVICE;
        break;
      }
      int64_t act = 0;
      for (int32_t v : hc) act += v;
      if (act == 0) break;
    }
  }
  if (!rc)
    hipLaunchKernelGGL(k_nuts_out, dim3(grid), dim3(256), 0, st, n, (const double*)Wd, (const int32_t*)I, Ly, theta, lnL,
                       info);
  if (!rc && hipGetLastError() != hipSuccess) rc = RIFT_EDEVICE;
  if (hipFreeAsync(w, st) != hipSuccess && !rc) rc = RIFT_EDEVICE;
  return rc;
}

extern "C" int rift_ile_plan_nuts(rift_ile_plan plan, int32_t point, int64_t n, double* theta, const double* z,
                                  const double* dirs, const double* merges, const double* leaves, const double* sigma,
                                  double eps, int32_t max_depth, const rift_ile_hmc_prior* prior, double beta,
                                  double* lnL, int32_t* info, void* stream) {
  return nuts_impl(plan, point, n, theta, z, dirs, merges, leaves, sigma, eps, max_depth, prior, nullptr, beta, lnL,
                   info, stream);
}

extern "C" int rift_ile_plan_nuts_dmarg(rift_ile_plan plan, int32_t point, int64_t n, double* theta, const double* z,
                                        const double* dirs, const double* merges, const double* leaves,
                                        const double* sigma, double eps, int32_t max_depth,
                                        const rift_ile_hmc_prior* prior, const rift_ile_dist_prior* dprior,
                                        double beta, double* lnLd, int32_t* info, void* stream) {
  if (!dprior) return RIFT_EINVAL;
  return nuts_impl(plan, point, n, theta, z, dirs, merges, leaves, sigma, eps, max_depth, prior, dprior, beta, lnLd,
                   info, stream);
}

extern "C" int rift_ile_smc_reweight(int64_t n, const double* lnL, double* lnW, double beta, double target,
                                     double* out, void* stream) {
  if (n < 1 || !(beta >= 0.0 && beta <= 1.0) || !(target > 0.0 && target <= 1.0)) return RIFT_EINVAL;
  auto bad = [](const void* q) { return !q || (((uintptr_t)q) & 7u); };
  if (bad(lnL) || bad(lnW) || bad(out)) return RIFT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int nb = (int)std::min<int64_t>((n + SMC_BLOCK - 1) / SMC_BLOCK, SMC_GRID_MAX);
  void* w = nullptr;
  const size_t bytes = sizeof(Acc3) * 2 * (size_t)nb + sizeof(SmcState);
  if (hipMallocAsync(&w, bytes, st) != hipSuccess) return RIFT_ENOMEM;
  Acc3* part = (Acc3*)w;
  SmcState* S = (SmcState*)(part + 2 * nb);
  const double ln_target = log(target);
  hipLaunchKernelGGL(k_smc_pass, dim3(nb), dim3(SMC_BLOCK), 0, st, n, (const double*)lnW, lnL,
                     (const SmcState*)S, 0, 1, part);
  hipLaunchKernelGGL(k_smc_init, dim3(1), dim3(SMC_BLOCK), 0, st, nb, (const Acc3*)part, 1.0 - beta, S);
  for (int it = 0; it < SMC_ITERS; ++it) {
    hipLaunchKernelGGL(k_smc_pass, dim3(nb), dim3(SMC_BLOCK), 0, st, n, (const double*)lnW, lnL,
                       (const SmcState*)S, 1, 0, part);
    hipLaunchKernelGGL(k_smc_step, dim3(1), dim3(SMC_BLOCK), 0, st, nb, (const Acc3*)part, ln_target, S);
  }
  hipLaunchKernelGGL(k_smc_pass, dim3(nb), dim3(SMC_BLOCK), 0, st, n, (const double*)lnW, lnL, (const SmcState*)S,
                     1, 1, part);
  hipLaunchKernelGGL(k_smc_finish, dim3(1), dim3(SMC_BLOCK), 0, st, nb, (const Acc3*)part, beta, S, out);
  hipLaunchKernelGGL(k_smc_apply, dim3(nb), dim3(SMC_BLOCK), 0, st, n, lnW, lnL, (const SmcState*)S);
  int rc = hipGetLastError() != hipSuccess ? RIFT_EDEVICE : RIFT_OK;
  if (hipFreeAsync(w, st) != hipSuccess && !rc) rc = RIFT_EDEVICE;
  return rc;
}

extern "C" int rift_ile_smc_resample(int64_t n, const double* lnW, double u, const double* theta_in,
                                     double* theta_out, int64_t* ancestors, void* stream) {
  if (n < 1 || !(u >= 0.0 && u < 1.0)) return RIFT_EINVAL;
  auto bad = [](const void* q) { return !q || (((uintptr_t)q) & 7u); };
  if (bad(lnW) || (ancestors && bad(ancestors))) return RIFT_EINVAL;
  if ((theta_out != nullptr) != (theta_in != nullptr)) return RIFT_EINVAL;
  if (theta_out && (bad(theta_in) || bad(theta_out) || theta_in == theta_out)) return RIFT_EINVAL;
  if (!theta_out && !ancestors) return RIFT_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  const int nb = (int)std::min<int64_t>((n + SMC_BLOCK - 1) / SMC_BLOCK, SMC_GRID_MAX);
  const int64_t nc = (n + SMC_CHUNK - 1) / SMC_CHUNK;
  const size_t bytes = sizeof(Acc3) * 2 * (size_t)nb + sizeof(SmcState) + sizeof(double) * ((size_t)n + (size_t)nc);
  void* w = nullptr;
  if (hipMallocAsync(&w, bytes, st) != hipSuccess) return RIFT_ENOMEM;
  Acc3* part = (Acc3*)w;
  SmcState* S = (SmcState*)(part + 2 * nb);
  double* C = (double*)(S + 1);
  double* bsum = C + n;
  hipLaunchKernelGGL(k_smc_pass, dim3(nb), dim3(SMC_BLOCK), 0, st, n, lnW, (const double*)nullptr,
                     (const SmcState*)S, 0, 1, part);
  hipLaunchKernelGGL(k_smc_init, dim3(1), dim3(SMC_BLOCK), 0, st, nb, (const Acc3*)part, 0.0, S);
  hipLaunchKernelGGL(k_cdf_local, dim3((unsigned)nc), dim3(SMC_BLOCK), 0, st, n, lnW, (const SmcState*)S, C, bsum);
  hipLaunchKernelGGL(k_cdf_blocks, dim3(1), dim3(SMC_BLOCK), 0, st, (int)nc, bsum);
  hipLaunchKernelGGL(k_cdf_offset, dim3(nb), dim3(SMC_BLOCK), 0, st, n, C, (const double*)bsum);
  hipLaunchKernelGGL(k_resample_pick, dim3(nb), dim3(SMC_BLOCK), 0, st, n, (const double*)C, u, theta_in, theta_out,
                     ancestors);
  int rc = hipGetLastError() != hipSuccess ? RIFT_EDEVICE : RIFT_OK;
  if (hipFreeAsync(w, st) != hipSuccess && !rc) rc = RIFT_EDEVICE;
  return rc;
}

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
  return rift_ile_plan_hmc_tempered(plan, point, n, theta, z, u, sigma, eps, n_leapfrog, prior, 1.0, lnL, accepted,
                                    stream);
}

static int hmc_impl(rift_ile_plan plan, int32_t point, int64_t n, double* theta, const double* z, const double* u,
                    const double* sigma, double eps, int32_t n_leapfrog, const rift_ile_hmc_prior* prior,
                    const rift_ile_dist_prior* dm, double beta, double* lnL, int32_t* accepted, void* stream) {
  if (!plan || n < 0 || !sigma || !prior || bad_dist_prior(dm)) return RIFT_EINVAL;
  if (!(beta >= 0.0 && beta <= 1.0)) return RIFT_EINVAL;
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
  HmcPrior P{};
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
  const double h = 0.5 * eps;
  P.dmarg = dm ? 1 : 0;
  // L + 1 gradients; between them one fused kernel each (kicks and drift)
  int rc = sampler_grad(plan, point, n, theta, dm, l1, g, stream);
  if (!rc)
    hipLaunchKernelGGL(k_hmc_first, dim3(grid), dim3(256), 0, st, n, theta, z, (const double*)g, (const double*)l1, h,
                       beta, sig, step, P, p, c0, H0, l0);
  for (int s = 1; s < n_leapfrog && !rc; ++s) {
    rc = sampler_grad(plan, point, n, theta, dm, l1, g, stream);
    if (!rc)
      hipLaunchKernelGGL(k_hmc_mid, dim3(grid), dim3(256), 0, st, n, theta, p, (const double*)g, h, beta, step, P);
  }
  if (!rc) rc = sampler_grad(plan, point, n, theta, dm, l1, g, stream);
  if (!rc)
    hipLaunchKernelGGL(k_hmc_end, dim3(grid), dim3(256), 0, st, n, theta, (const double*)p, (const double*)g,
                       (const double*)l1, h, beta, (const double*)c0, (const double*)l0, (const double*)H0, u, sig,
                       P, lnL, accepted);
  if (!rc && hipGetLastError() != hipSuccess) rc = RIFT_EDEVICE;
  if (hipFreeAsync(w, st) != hipSuccess && !rc) rc = RIFT_EDEVICE;
  return rc;
}

extern "C" int rift_ile_plan_hmc_tempered(rift_ile_plan plan, int32_t point, int64_t n, double* theta,
                                          const double* z, const double* u, const double* sigma, double eps,
                                          int32_t n_leapfrog, const rift_ile_hmc_prior* prior, double beta,
                                          double* lnL, int32_t* accepted, void* stream) {
  return hmc_impl(plan, point, n, theta, z, u, sigma, eps, n_leapfrog, prior, nullptr, beta, lnL, accepted, stream);
}

extern "C" int rift_ile_plan_hmc_dmarg(rift_ile_plan plan, int32_t point, int64_t n, double* theta, const double* z,
                                       const double* u, const double* sigma, double eps, int32_t n_leapfrog,
                                       const rift_ile_hmc_prior* prior, const rift_ile_dist_prior* dprior, double beta,
                                       double* lnLd, int32_t* accepted, void* stream) {
  if (!dprior) return RIFT_EINVAL;
  return hmc_impl(plan, point, n, theta, z, u, sigma, eps, n_leapfrog, prior, dprior, beta, lnLd, accepted, stream);
}
