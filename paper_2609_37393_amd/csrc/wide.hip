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
// walked upward).  The quadratic term runs over pairs a <= a' of composite
// terms, G_aa' = Y^H U_aa' Y and H_aa' = Y^T V_aa' Y with U, V read through
// the scalar path (uniform across the lanes), and uses the symmetries
// G_a'a = conj(G_aa') (U Hermitian) and H_a'a = H_aa' (V symmetric).
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

constexpr int WIDE_MAX_TERMS = 8;  // composite terms per detector
constexpr int WIDE_MAX_MODES = 25;
constexpr int WIDE_BLOCK = 256;

struct WideDesc {
  int32_t K, M, n_t, n_a, response, pad;
  double t0, inv_dt, gmst, omega, d_ref, lnN;
  double dten[KMAX][6];      // D00, D11, D22, 2 D01, 2 D02, 2 D12
  double rpos[KMAX][3];      // light-seconds
  double arms[KMAX][2][3];   // arm unit vectors
  int32_t perm[MMAX];        // caller's index of internal mode i (modes sorted by m)
  int32_t m[MMAX];
  int32_t odd[MMAX];
  double ycoef[MMAX][LMAXC + 1];
  const double* Q;           // caller's [K][n_a][M][n_t] complex
  const double* U;           // caller's [K][n_a M][n_a M] complex
  const double* V;
};
typedef const RIFT_CONST WideDesc* WDesc;

// Complex response D : (e+ + i ex) of the six-value tensor d at axes X, Y.
__device__ __forceinline__ C2<double> response6(const RIFT_CONST double* d, const double* X, const double* Y) {
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

// G_ab = Y^H U_ab Y and H_ab = Y^T V_ab Y, accumulated into g[4] = (Re G,
// Im G, Re H, Im H): the rows II of both blocks in turn (a template recursion,
// so that every mode index is a compile-time constant and Y stays in
// registers), each row's columns in an unrolled loop.
template <int II>
struct PairForms {
  static __device__ __forceinline__ void run(WDesc P, const RIFT_CONST double* Uk, const RIFT_CONST double* Vk, int A,
                                             int a, int b, int M, const double* yr, const double* yi, double* g) {
    if constexpr (II < WIDE_MAX_MODES) {
      if (II < M) {
        const int64_t row = (int64_t)(a * M + P->perm[II]) * A + b * M;
        double tr = 0.0, ti = 0.0, vr = 0.0, vi = 0.0;  // (U Y)_II, (V Y)_II
#pragma unroll
        for (int jj = 0; jj < WIDE_MAX_MODES; ++jj) {
          if (jj < M) {
            const int64_t o = 2 * (row + P->perm[jj]);
            const double ur = Uk[o], ui = Uk[o + 1], wr = Vk[o], wi = Vk[o + 1];
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
        PairForms<II + 1>::run(P, Uk, Vk, A, a, b, M, yr, yi, g);
      }
    }
  }
};

__global__ void __launch_bounds__(WIDE_BLOCK) k_wide(const WideDesc* __restrict__ desc,
                                                     const double* __restrict__ theta, int64_t n,
                                                     const double* __restrict__ lnw, double* __restrict__ lnL,
                                                     double* __restrict__ part) {
  __shared__ double cre[WIDE_MAX_TERMS][WIDE_BLOCK], cim[WIDE_MAX_TERMS][WIDE_BLOCK];
  __shared__ MS sh[WIDE_BLOCK / 64];
  WDesc P = opaque(desc);
  const int t = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * WIDE_BLOCK + t;
  const bool live = i0 < n;
  const int64_t i = live ? i0 : n - 1;
  const RIFT_GLOBAL double* th = as_global(theta) + i;
  const double ra = th[0], dec = th[n], psi = th[2 * n], incl = th[3 * n], phi = th[4 * n];
  const double tref = th[5 * n], dist = th[6 * n];
  const int K = P->K, M = P->M, n_t = P->n_t, n_a = P->n_a;
  const bool rot = P->response == RIFT_RESP_ROTATION;

  // sky frame at t_ref (the rotation response advances the sidereal angle)
  const double gm = rot ? P->gmst + P->omega * tref : P->gmst;
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
  double yr[WIDE_MAX_MODES], yi[WIDE_MAX_MODES];
  {
    C2<double> ph;
    ph.x = 1.0;
    ph.y = 0.0;
    const int mmin = P->m[0];
    for (int q = 0; q < -mmin; ++q) phase_down(ph, cf, sf);
    int mc = mmin < 0 ? mmin : 0;
#pragma unroll
    for (int j = 0; j < WIDE_MAX_MODES; ++j) {
      yr[j] = yi[j] = 0.0;
      if (j < M) {
        const int mj = P->m[j];
        while (mc < mj) {
          phase_up(ph, cf, sf);
          ++mc;
        }
        double d = 0.0;
        if (P->odd[j]) {
#pragma unroll
          for (int q = 1; q <= LMAXC; ++q) d += P->ycoef[j][q] * sn[q];
        } else {
#pragma unroll
          for (int q = 0; q <= LMAXC; ++q) d += P->ycoef[j][q] * cn[q];
        }
        yr[j] = d * ph.x;
        yi[j] = d * ph.y;
      }
    }
  }

  double data = 0.0, quad = 0.0;
  bool bad = false;
  const int A = n_a * M;
  for (int k = 0; k < K; ++k) {
    const RIFT_CONST double* r = P->rpos[k];
    const double tk = tref - (r[0] * N[0] + r[1] * N[1] + r[2] * N[2]);
    // composite coefficients of this detector -> this lane's LDS column
    if (rot) {
      // F_k at the five hour angles g_j = 2 pi j / 5, then A_n by the exact
      // five-point transform, then the phases e^{i n theta_k}
      C2<double> Fg[5];
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        double sgj, cgj;
        sincospi(0.4 * j, &sgj, &cgj);
        double Xj[3], Yj[3], Nj[3];
        axes(sgj, cgj, sd, cd, sp, cp, Xj, Yj, Nj);
        Fg[j] = response6(P->dten[k], Xj, Yj);
      }
      const double thk = gref + P->omega * (tk - tref);
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        const int nn = a - 2;
        double ar = 0.0, ai = 0.0;
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          double s, c;
          sincospi(-0.4 * nn * j, &s, &c);  // e^{-i n g_j}
          ar += Fg[j].x * c - Fg[j].y * s;
          ai += Fg[j].x * s + Fg[j].y * c;
        }
        ar *= 0.2;
        ai *= 0.2;
        // e^{i n theta_k}
        double er, ei;
        sincos((double)nn * thk, &ei, &er);
        cre[a][t] = ar * er - ai * ei;
        cim[a][t] = ar * ei + ai * er;
      }
    } else {
      const RIFT_CONST double* ax = P->arms[k][0];
      const RIFT_CONST double* ay = P->arms[k][1];
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
    double u = (tk - P->t0) * P->inv_dt;
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
    // data term: Re sum_a conj(C~_a) sum_i conj(Y_i) Qhat_{a,i}
    for (int a = 0; a < n_a; ++a) {
      double zr = 0.0, zi = 0.0;
#pragma unroll
      for (int j = 0; j < WIDE_MAX_MODES; ++j) {
        if (j < M) {
          const RIFT_GLOBAL double* q =
              as_global(P->Q) + 2 * ((((int64_t)k * n_a + a) * M + P->perm[j]) * (int64_t)n_t);
          double qr = 0.0, qi = 0.0;
#pragma unroll
          for (int tap = 0; tap < 4; ++tap) {
            const int node = j0 + tap;
            if (node >= 0 && node < n_t) {
              qr += w[tap] * q[2 * node];
              qi += w[tap] * q[2 * node + 1];
            }
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
    const RIFT_CONST double* Uk = as_const(P->U) + 2 * (int64_t)k * A * A;
    const RIFT_CONST double* Vk = as_const(P->V) + 2 * (int64_t)k * A * A;
    for (int a = 0; a < n_a; ++a) {
      for (int b = a; b < n_a; ++b) {
        double g[4] = {0.0, 0.0, 0.0, 0.0};  // Re G, Im G, Re H, Im H
        PairForms<0>::run(P, Uk, Vk, A, a, b, M, yr, yi, g);
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
  const double x = P->d_ref / dist;
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
__global__ void k_wide_merge(const WideDesc* __restrict__ P, const double* __restrict__ part, int nb,
                             double* __restrict__ lnZ, double* __restrict__ neff) {
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
    else z = r.m + log(r.s) - P->lnN;
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
  } else if (pt->response == RIFT_RESP_ARMS) {
    if (pt->n_terms < 1 || pt->n_terms > WIDE_MAX_TERMS || !pt->det_arms) return RIFT_EINVAL;
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
  const int64_t nb = (n + WIDE_BLOCK - 1) / WIDE_BLOCK;
  if (nb > 0x7fffffff) return RIFT_EUNSUPPORTED;
  WideDesc D;
  memset(&D, 0, sizeof(D));
  D.K = pt->n_det;
  D.M = pt->n_modes;
  D.n_t = pt->n_t;
  D.n_a = pt->n_terms;
  D.response = pt->response;
  D.t0 = pt->t0;
  D.inv_dt = 1.0 / pt->dt;
  D.gmst = pt->gmst_rad;
  D.omega = pt->response == RIFT_RESP_ROTATION ? pt->omega : 0.0;
  D.d_ref = pt->d_ref;
  D.lnN = log((double)n);
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
  D.U = pt->U;
  D.V = pt->V;
  hipStream_t st = (hipStream_t)stream;
  WideDesc* d_desc = nullptr;
  double* d_part = nullptr;
  if (hipMalloc(&d_desc, sizeof(WideDesc)) != hipSuccess) return RIFT_ENOMEM;
  if (lnZ && hipMalloc(&d_part, sizeof(double) * 2 * nb) != hipSuccess) {
    (void)hipFree(d_desc);
    return RIFT_ENOMEM;
  }
  rc = RIFT_OK;
  if (hipMemcpyAsync(d_desc, &D, sizeof(WideDesc), hipMemcpyHostToDevice, st) != hipSuccess) rc = RIFT_EDEVICE;
  if (!rc) {
    hipLaunchKernelGGL(k_wide, dim3((unsigned)nb), dim3(WIDE_BLOCK), 0, st, (const WideDesc*)d_desc, theta, n, lnw,
                       lnL, d_part);
    if (lnZ)
      hipLaunchKernelGGL(k_wide_merge, dim3(1), dim3(WIDE_BLOCK), 0, st, (const WideDesc*)d_desc,
                         (const double*)d_part, (int)nb, lnZ, neff);
    if (hipGetLastError() != hipSuccess) rc = RIFT_EDEVICE;
  }
  // the host copy of the description and the device buffers live until the work is done
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = RIFT_EDEVICE;
  (void)hipFree(d_desc);
  if (d_part) (void)hipFree(d_part);
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
