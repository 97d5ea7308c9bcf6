// Hand-written gradient of the factored log-likelihood (FP64): lnL and
// d lnL / d(ra, dec, psi, incl or cos incl, phiref, tref, dist or ln dist)
// (Sec. "The differentiable likelihood": the same closed form, differentiated).
//
// With gha = gmst - ra, the rotating-frame identities used below are
//   dN/dgha = -cos(dec) e_a,  de_a/dgha = cos(dec) N - sin(dec) e_d,  de_d/dgha = sin(dec) e_a,
//   dN/ddec = e_d,            de_a/ddec = 0,                          de_d/ddec = -N,
// so that dX/dgha = -cos(psi) cos(dec) N + sin(dec) Y, dY/dgha = sin(psi) cos(dec) N - sin(dec) X,
// dX/ddec = -sin(psi) N, dY/ddec = -cos(psi) N, dF/dpsi = -2i F.  With
// S_NX = 2 N.D.X and S_NY = 2 N.D.Y:
//   dF+/dgha = -cpsi cdec S_NX - spsi cdec S_NY + 2 sdec Fx
//   dFx/dgha = -cpsi cdec S_NY + spsi cdec S_NX - 2 sdec F+
//   dF+/ddec = -spsi S_NX + cpsi S_NY,   dFx/ddec = -spsi S_NY - cpsi S_NX
//   dt_k/dgha = cdec r_k.e_a,  dt_k/ddec = -r_k.e_d,  dt_k/dtref = 1.
// The table read contributes dQ/dt from the derivative of the Lagrange weights
// (the derivative within the cell; the cubic is only C0 at the nodes).
#pragma once

#include "ile_device.h"

namespace rift {

// Coordinates of rows 3 and 6 of theta, for the input and for the gradient
// (bit 0: cos(incl) instead of incl; bit 1: ln(dist) instead of dist).
enum : int { COORD_COS_INCL = 1, COORD_LN_DIST = 2 };

// Rows 3 and 6 of a sample in the coordinates `coords` -> (incl, dist).  A
// cos(incl) outside [-1, 1] is not a point of the sky: the sample is poisoned.
__device__ __forceinline__ bool theta_coords(int coords, double& incl, double& dist) {
  bool ok = true;
  if (coords & COORD_COS_INCL) {
    ok = fabs(incl) <= 1.0;
    incl = acos(fmin(fmax(incl, -1.0), 1.0));
  }
  if (coords & COORD_LN_DIST) dist = exp(dist);
  return ok;
}

// The last step of both gradient forms: from the derivatives along incl (g3)
// and ln(dist) (g6) to the coordinates `coords`, given row 3 as the caller
// passed it (c3) and the distance:
//   d/d cos(incl) = -d/d incl / sin(incl), sin(incl) = sqrt((1 - c)(1 + c))
//   (exactly 0 at c = +-1, where the derivative is infinite or NaN: the
//   likelihood is not differentiable in cos(incl) at the poles);
//   d/d dist = d/d ln(dist) / dist.
__device__ __forceinline__ void grad_coords(int coords, double c3, double dist, double& g3, double& g6) {
  if (coords & COORD_COS_INCL) g3 = -g3 / sqrt((1.0 - c3) * (1.0 + c3));
  if (!(coords & COORD_LN_DIST)) g6 = g6 / dist;
}

// The distance factors of both epilogues.  lnL = x data - x^2 quad in
// x = d_ref / D, and every derivative along the other coordinates is
// x d(data) - x^2 d(quad).  At the sample's distance: m1 = x, m2 = x^2.  For
// the likelihood marginalised over distance (`marg`, Eq. (ap:dgh)):
// ln L_d by the rule, and d ln L_d = <x> d(data) - <x^2> d(quad) with the
// moments under the distance posterior taken by the rule's node weights
// W_i p_x(x_i), p_x ~ x^-4; where the model has no power (R = 2 quad <= 0)
// the prior's moments of x; no node inside the prior: `none` (derivative 0).
struct DistFactors {
  double m1, m2, lnL;
  bool none;
};
__device__ __forceinline__ DistFactors dist_factors(PDesc P, double dist, double data, double quad, bool bad,
                                                    const DistRule& G, bool marg) {
  DistFactors f;
  f.none = false;
  if (!marg) {
    const double x = P->d_ref / dist;
    const double x2 = x * x;
    f.m1 = x;
    f.m2 = x2;
    f.lnL = x * data - x2 * quad;
    return f;
  }
  const double d_ref = P->d_ref;
  Terms t;
  t.data = data;
  t.quad = quad;
  t.wq = 0.0;
  t.bad = bad;
  f.lnL = dist_marginal(G, d_ref, t);
  const double a = d_ref / G.d_max, b = d_ref / G.d_min;
  const double Rd = 2.0 * quad;
  if (!(Rd > 0.0)) {
    const double i3 = 1.0 / (a * a * a) - 1.0 / (b * b * b);
    f.m1 = 1.5 * (1.0 / (a * a) - 1.0 / (b * b)) / i3;
    f.m2 = 3.0 * (1.0 / a - 1.0 / b) / i3;
    return f;
  }
  const double xs = data / Rd, sig = 1.0 / sqrt(Rd);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int k = 0; k < G.n; ++k) {
    const double x = fma(G.xi[k], sig, xs);
    if (x >= a && x <= b) {
      const double r = d_ref / x;
      const double w = G.w[k] * (r * r) * (r * r);
      s0 += w;
      s1 = fma(w, x, s1);
      s2 = fma(w * x, x, s2);
    }
  }
  f.none = !(s0 > 0.0);
  f.m1 = s1 / s0;
  f.m2 = s2 / s0;
  return f;
}

template <int KT, int L, bool MARG = false>
__device__ __forceinline__ double eval_grad(PDesc P, double* __restrict__ trig, int ts, double ra,
                                            double dec, double psi, double incl, double phi,
                                            double tref, double dist, double g[7], const DistRule* dm = nullptr) {
  typedef Cls<L> CL;
  constexpr int NI = CL::NI;
  constexpr int NY = CL::NY;
  const int M = P->M;
  const int n_t = P->n_t;
  const RIFT_GLOBAL double* Qt = as_global(P->Q64);

  double sg, cg, sd, cd, sp, cp;
  sincos(P->gmst - ra, &sg, &cg);
  sincos(dec, &sd, &cd);
  sincos(psi, &sp, &cp);
  const double N[3] = {cd * cg, -cd * sg, sd};
  const double ea[3] = {sg, cg, 0.0};
  const double ed[3] = {-sd * cg, sd * sg, cd};
  double X[3], Y[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    X[a] = -cp * ea[a] + sp * ed[a];
    Y[a] = sp * ea[a] + cp * ed[a];
  }

  // harmonics in incl (registers up to l, scratch column up to 2l)
  double si, ci;
  sincos(incl, &si, &ci);
  double cn[NY], sn[NY];
  {
    double c0 = 1.0, c1 = ci, s0 = 0.0, s1 = si;
#pragma unroll
    for (int n = 0; n <= NI; ++n) {
      const double c = (n == 0) ? c0 : c1;
      const double s = (n == 0) ? s0 : s1;
      if (n < NY) {
        cn[n] = c;
        sn[n] = s;
      }
      trig[n * ts] = c;
      trig[(NI + 1 + n) * ts] = s;
      if (n > 0) {
        const double c2 = 2.0 * ci * c1 - c0, s2 = 2.0 * ci * s1 - s0;
        c0 = c1;
        c1 = c2;
        s0 = s1;
        s1 = s2;
      }
    }
  }
  double sf, cf;
  sincos(phi, &sf, &cf);

  // antenna factors, their derivatives and the stencils
  double Fp[KT], Fx[KT], dFg[KT][2], dFd[KT][2], dtg[KT], dtd[KT];
  double w[KT][4], wd[KT][4];
  int soff[KT];
  const int ntp = n_t + 2 * QPAD;
  const int NGR = q_groups(M, QW64);
  bool bad = false;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const RIFT_CONST double* dt6 = P->dten[k];
    const double D00 = dt6[0], D11 = dt6[1], D22 = dt6[2];
    const double D01 = 0.5 * dt6[3], D02 = 0.5 * dt6[4], D12 = 0.5 * dt6[5];
    double DX[3], DY[3];
    DX[0] = D00 * X[0] + D01 * X[1] + D02 * X[2];
    DX[1] = D01 * X[0] + D11 * X[1] + D12 * X[2];
    DX[2] = D02 * X[0] + D12 * X[1] + D22 * X[2];
    DY[0] = D00 * Y[0] + D01 * Y[1] + D02 * Y[2];
    DY[1] = D01 * Y[0] + D11 * Y[1] + D12 * Y[2];
    DY[2] = D02 * Y[0] + D12 * Y[1] + D22 * Y[2];
    const double fp = X[0] * DX[0] + X[1] * DX[1] + X[2] * DX[2] - (Y[0] * DY[0] + Y[1] * DY[1] + Y[2] * DY[2]);
    const double fx = 2.0 * (X[0] * DY[0] + X[1] * DY[1] + X[2] * DY[2]);
    const double SNX = 2.0 * (N[0] * DX[0] + N[1] * DX[1] + N[2] * DX[2]);
    const double SNY = 2.0 * (N[0] * DY[0] + N[1] * DY[1] + N[2] * DY[2]);
    Fp[k] = fp;
    Fx[k] = fx;
    dFg[k][0] = -cp * cd * SNX - sp * cd * SNY + 2.0 * sd * fx;
    dFg[k][1] = -cp * cd * SNY + sp * cd * SNX - 2.0 * sd * fp;
    dFd[k][0] = -sp * SNX + cp * SNY;
    dFd[k][1] = -sp * SNY - cp * SNX;

    const RIFT_CONST double* r = P->rpos[k];
    const double tk = tref - (r[0] * N[0] + r[1] * N[1] + r[2] * N[2]);
    dtg[k] = cd * (r[0] * ea[0] + r[1] * ea[1]);
    dtd[k] = -(r[0] * ed[0] + r[1] * ed[1] + r[2] * ed[2]);
    double u = (tk - P->t0) * P->inv_dt;
    if (!stencil_u(u, n_t)) bad = true;
    const double jf = floor(u);
    const double s = u - jf;
    int j0 = (int)jf - 1;
    j0 = j0 < -QPAD ? -QPAD : (j0 > n_t ? n_t : j0);
    soff[k] = j0 + QPAD;
    const double s2 = s * s;
    const double idt = P->inv_dt;
    w[k][0] = -s * (s - 1.0) * (s - 2.0) / 6.0;
    w[k][1] = (s + 1.0) * (s - 1.0) * (s - 2.0) * 0.5;
    w[k][2] = -(s + 1.0) * s * (s - 2.0) * 0.5;
    w[k][3] = (s + 1.0) * s * (s - 1.0) / 6.0;
    wd[k][0] = -(3.0 * s2 - 6.0 * s + 2.0) / 6.0 * idt;
    wd[k][1] = (3.0 * s2 - 4.0 * s - 1.0) * 0.5 * idt;
    wd[k][2] = -(3.0 * s2 - 2.0 * s - 2.0) * 0.5 * idt;
    wd[k][3] = (3.0 * s2 - 1.0) / 6.0 * idt;
  }

  // data term and its derivatives: loop over modes
  C2<double> Z[KT], Zt[KT], Zi[KT], Zf[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) Z[k].x = Z[k].y = Zt[k].x = Zt[k].y = Zi[k].x = Zi[k].y = Zf[k].x = Zf[k].y = 0.0;
  {
    C2<double> ph;
    ph.x = 1.0;
    ph.y = 0.0;
    const int mmin = P->m_min;
    for (int t = 0; t < -mmin; ++t) {
      const double a = ph.x * cf + ph.y * sf, bb = ph.y * cf - ph.x * sf;
      ph.x = a;
      ph.y = bb;
    }
    int mc = mmin < 0 ? mmin : 0;
    for (int i = 0; i < M; ++i) {
      const int mi = P->m[i];
      while (mc < mi) {
        const double a = ph.x * cf - ph.y * sf, bb = ph.y * cf + ph.x * sf;
        ph.x = a;
        ph.y = bb;
        ++mc;
      }
      double d = 0.0, dd = 0.0;
      if (P->odd[i]) {
#pragma unroll
        for (int n = 1; n < NY; ++n) {
          d += P->ycoef[i][n] * sn[n];
          dd += P->ycoef[i][n] * (double)n * cn[n];
        }
      } else {
#pragma unroll
        for (int n = 0; n < NY; ++n) {
          d += P->ycoef[i][n] * cn[n];
          dd -= P->ycoef[i][n] * (double)n * sn[n];
        }
      }
      const double yx = d * ph.x, yy = d * ph.y, ix = dd * ph.x, iy = dd * ph.y;
      const double mv = (double)mi;
#pragma unroll
      for (int k = 0; k < KT; ++k) {
        const RIFT_GLOBAL double* ser = Qt + 2 * ((int64_t)(k * NGR + i / QW64) * ntp * QW64 + i % QW64);
        const C2<double> q0 = ldq(ser, soff[k] * QW64), q1 = ldq(ser, (soff[k] + 1) * QW64);
        const C2<double> q2 = ldq(ser, (soff[k] + 2) * QW64), q3 = ldq(ser, (soff[k] + 3) * QW64);
        const double qx = w[k][0] * q0.x + w[k][1] * q1.x + w[k][2] * q2.x + w[k][3] * q3.x;
        const double qy = w[k][0] * q0.y + w[k][1] * q1.y + w[k][2] * q2.y + w[k][3] * q3.y;
        const double tx = wd[k][0] * q0.x + wd[k][1] * q1.x + wd[k][2] * q2.x + wd[k][3] * q3.x;
        const double ty = wd[k][0] * q0.y + wd[k][1] * q1.y + wd[k][2] * q2.y + wd[k][3] * q3.y;
        const double zx = yx * qx + yy * qy;  // conj(Y) q
        const double zy = yx * qy - yy * qx;
        Z[k].x += zx;
        Z[k].y += zy;
        Zt[k].x += yx * tx + yy * ty;
        Zt[k].y += yx * ty - yy * tx;
        Zi[k].x += ix * qx + iy * qy;
        Zi[k].y += ix * qy - iy * qx;
        // d/dphi conj(Y) = -i m conj(Y): (-i m)(zx + i zy) = m zy - i m zx
        Zf[k].x += mv * zy;
        Zf[k].y -= mv * zx;
      }
    }
  }
  double data = 0.0, gg = 0.0, gdec = 0.0, gpsi = 0.0, gi = 0.0, gf = 0.0, gt = 0.0;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const double fp = Fp[k], fx = Fx[k];
    data += fp * Z[k].x + fx * Z[k].y;
    const double dt_term = fp * Zt[k].x + fx * Zt[k].y;
    gg += dFg[k][0] * Z[k].x + dFg[k][1] * Z[k].y + dt_term * dtg[k];
    gdec += dFd[k][0] * Z[k].x + dFd[k][1] * Z[k].y + dt_term * dtd[k];
    gpsi += 2.0 * fx * Z[k].x - 2.0 * fp * Z[k].y;  // dF/dpsi = (2 Fx, -2 F+)
    gi += fp * Zi[k].x + fx * Zi[k].y;
    gf += fp * Zf[k].x + fx * Zf[k].y;
    gt += dt_term;
  }

  // model-norm term and its incl/phi derivatives: loop over basis rows.  For
  // T_n = cos or sin(n incl) and T'_n its incl-derivative, a pair of basis
  // functions T_n cos(q phi), T_n sin(q phi) has derivatives
  // (T'_n cos, -q T_n sin) and (T'_n sin, q T_n cos).
  const RIFT_CONST double* Cc = as_const(P->C64);
  double R[3 * KT], Ri[3 * KT], Rf[3 * KT];
#pragma unroll
  for (int c = 0; c < 3 * KT; ++c) R[c] = Ri[c] = Rf[c] = 0.0;
#pragma unroll 1
  for (int n = 0; n <= NI; ++n) {
    const double v = trig[n * ts], vi = -(double)n * trig[(NI + 1 + n) * ts];
    const RIFT_CONST double* cr = Cc + n * 3 * KT;
#pragma unroll
    for (int c = 0; c < 3 * KT; ++c) {
      R[c] += cr[c] * v;
      Ri[c] += cr[c] * vi;
    }
  }
  {
    int b = NI + 1;
    C2<double> eq;
    eq.x = cf;
    eq.y = sf;
#pragma unroll 1
    for (int q = 1; q <= NI; ++q) {
      const int odd = q & 1;
      const double qd = (double)q;
#pragma unroll 1
      for (int n = odd; n <= NI; ++n, b += 2) {
        const double nd = (double)n;
        const double t = odd ? trig[(NI + 1 + n) * ts] : trig[n * ts];
        const double tp = odd ? nd * trig[n * ts] : -nd * trig[(NI + 1 + n) * ts];
        const double v1 = t * eq.x, i1 = tp * eq.x, f1 = -qd * t * eq.y;
        const double v2 = t * eq.y, i2 = tp * eq.y, f2 = qd * t * eq.x;
        const RIFT_CONST double* cr = Cc + b * 3 * KT;
#pragma unroll
        for (int c = 0; c < 3 * KT; ++c) {
          const double c1 = cr[c], c2 = cr[3 * KT + c];
          R[c] += c1 * v1 + c2 * v2;
          Ri[c] += c1 * i1 + c2 * i2;
          Rf[c] += c1 * f1 + c2 * f2;
        }
      }
      const double ex_ = eq.x * cf - eq.y * sf, ey_ = eq.x * sf + eq.y * cf;
      eq.x = ex_;
      eq.y = ey_;
    }
  }
  double quad = 0.0, qg = 0.0, qdec = 0.0, qpsi = 0.0, qi = 0.0, qf = 0.0;
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const double a = Fp[k], c = Fx[k];
    const double w0 = a * a + c * c, w1 = a * a - c * c, w2 = 2.0 * a * c;
    quad += w0 * R[3 * k] + w1 * R[3 * k + 1] + w2 * R[3 * k + 2];
    qi += w0 * Ri[3 * k] + w1 * Ri[3 * k + 1] + w2 * Ri[3 * k + 2];
    qf += w0 * Rf[3 * k] + w1 * Rf[3 * k + 1] + w2 * Rf[3 * k + 2];
    // weights' change for a change (da, dc) of (F+, Fx)
    {
      const double da = dFg[k][0], dc = dFg[k][1];
      qg += 2.0 * (a * da + c * dc) * R[3 * k] + 2.0 * (a * da - c * dc) * R[3 * k + 1] +
            2.0 * (da * c + a * dc) * R[3 * k + 2];
    }
    {
      const double da = dFd[k][0], dc = dFd[k][1];
      qdec += 2.0 * (a * da + c * dc) * R[3 * k] + 2.0 * (a * da - c * dc) * R[3 * k + 1] +
              2.0 * (da * c + a * dc) * R[3 * k + 2];
    }
    {
      const double da = 2.0 * c, dc = -2.0 * a;
      qpsi += 2.0 * (a * da + c * dc) * R[3 * k] + 2.0 * (a * da - c * dc) * R[3 * k + 1] +
              2.0 * (da * c + a * dc) * R[3 * k + 2];
    }
  }

  double x, x2, lnL;
  bool none = false;
  if constexpr (MARG) {
    const DistFactors Df = dist_factors(P, dist, data, quad, bad, *dm, true);
    x = Df.m1;
    x2 = Df.m2;
    lnL = Df.lnL;
    none = Df.none;
  } else {
    x = P->d_ref / dist;
    x2 = x * x;
    lnL = x * data - x2 * quad;
  }
  g[0] = -(x * gg - x2 * qg);          // d/dra = -d/dgha
  g[1] = x * gdec - x2 * qdec;
  g[2] = x * gpsi - x2 * qpsi;
  g[3] = x * gi - x2 * qi;             // d/d incl
  g[4] = x * gf - x2 * qf;
  g[5] = x * gt;
  g[6] = MARG ? 0.0 : -x * data + 2.0 * x2 * quad;  // d/d ln(dist), x = D_ref e^{-ln dist}
  if (none) {
#pragma unroll
    for (int a = 0; a < 6; ++a) g[a] = 0.0;
  }
  if (bad) {
    const double nan = __builtin_nan("");
#pragma unroll
    for (int a = 0; a < 7; ++a) g[a] = nan;
    return nan;
  }
  return lnL;
}

// The same value and gradient with a group of G lanes (a power of two, at
// most 64) per sample, for batches too small to fill the GPU one lane per
// sample.  The group shares its sample's tables through `tab` (GRAD_TAB(L, KT)
// doubles of LDS per group):
//   cos/sin(n incl) and cos/sin(q phi) for n, q = 0..2L;
//   per detector: F+, Fx, dF/dgha (2), dF/ddec (2), dt/dgha, dt/ddec, stencil
//   row and fraction, a bad flag, and the model-norm weights (|F|^2,
//   Re F^2, Im F^2) with their changes along gha, dec and psi (12 values).
// The (detector, mode) pairs of the data term and the basis rows of the
// model-norm contraction are spread over the group's lanes; 14 group sums
// finish it.  Every lane of the group returns the value and g[].  The whole
// wavefront calls this together (one sample per group).
#define GRAD_TAB(L, KT) (4 * (2 * (L) + 1) + 24 * (KT))
template <int G>
__device__ __forceinline__ double gsum(double v) {
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
template <int KT, int L, int G, bool MARG = false>
__device__ __forceinline__ double eval_grad_group(PDesc P, double ra, double dec, double psi, double incl,
                                                  double phi, double tref, double dist, double* tab,
                                                  double g[7], const DistRule* dm = nullptr) {
  constexpr int NI = 2 * L;
  constexpr int NY = L + 1;
  const int lg = (int)(threadIdx.x & (G - 1));
  const int K = P->K, M = P->M, n_t = P->n_t;
  double* ctab = tab;
  double* stab = tab + (NI + 1);
  double* cq = tab + 2 * (NI + 1);
  double* sq = tab + 3 * (NI + 1);
  double* det = tab + 4 * (NI + 1);
  for (int n = lg; n <= NI; n += G) {
    double s, c;
    sincos((double)n * incl, &s, &c);
    ctab[n] = c;
    stab[n] = s;
    sincos((double)n * phi, &s, &c);
    cq[n] = c;
    sq[n] = s;
  }
  for (int k = lg; k < KT; k += G) {
    double* dk = det + 24 * k;
    if (k < K) {
      double sg, cg, sd, cd, sp, cp;
      sincos(P->gmst - ra, &sg, &cg);
      sincos(dec, &sd, &cd);
      sincos(psi, &sp, &cp);
      const double N[3] = {cd * cg, -cd * sg, sd};
      const double ea[3] = {sg, cg, 0.0};
      const double ed[3] = {-sd * cg, sd * sg, cd};
      double X[3], Y[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        X[a] = -cp * ea[a] + sp * ed[a];
        Y[a] = sp * ea[a] + cp * ed[a];
      }
      const RIFT_CONST double* dt6 = P->dten[k];
      const double D00 = dt6[0], D11 = dt6[1], D22 = dt6[2];
      const double D01 = 0.5 * dt6[3], D02 = 0.5 * dt6[4], D12 = 0.5 * dt6[5];
      double DX[3], DY[3];
      DX[0] = D00 * X[0] + D01 * X[1] + D02 * X[2];
      DX[1] = D01 * X[0] + D11 * X[1] + D12 * X[2];
      DX[2] = D02 * X[0] + D12 * X[1] + D22 * X[2];
      DY[0] = D00 * Y[0] + D01 * Y[1] + D02 * Y[2];
      DY[1] = D01 * Y[0] + D11 * Y[1] + D12 * Y[2];
      DY[2] = D02 * Y[0] + D12 * Y[1] + D22 * Y[2];
      const double fp = X[0] * DX[0] + X[1] * DX[1] + X[2] * DX[2] - (Y[0] * DY[0] + Y[1] * DY[1] + Y[2] * DY[2]);
      const double fx = 2.0 * (X[0] * DY[0] + X[1] * DY[1] + X[2] * DY[2]);
      const double SNX = 2.0 * (N[0] * DX[0] + N[1] * DX[1] + N[2] * DX[2]);
      const double SNY = 2.0 * (N[0] * DY[0] + N[1] * DY[1] + N[2] * DY[2]);
      const double gA = -cp * cd * SNX - sp * cd * SNY + 2.0 * sd * fx;
      const double gC = -cp * cd * SNY + sp * cd * SNX - 2.0 * sd * fp;
      const double dA = -sp * SNX + cp * SNY;
      const double dC = -sp * SNY - cp * SNX;
      const RIFT_CONST double* r = P->rpos[k];
      const double tk = tref - (r[0] * N[0] + r[1] * N[1] + r[2] * N[2]);
      double u = (tk - P->t0) * P->inv_dt;
      const double bad = stencil_u(u, n_t) ? 0.0 : 1.0;
      const double jf = floor(u);
      int j0 = (int)jf - 1;
      j0 = j0 < -QPAD ? -QPAD : (j0 > n_t ? n_t : j0);
      dk[0] = fp;
      dk[1] = fx;
      dk[2] = gA;
      dk[3] = gC;
      dk[4] = dA;
      dk[5] = dC;
      dk[6] = cd * (r[0] * ea[0] + r[1] * ea[1]);
      dk[7] = -(r[0] * ed[0] + r[1] * ed[1] + r[2] * ed[2]);
      dk[8] = (double)(j0 + QPAD);
      dk[9] = u - jf;
      dk[10] = bad;
      dk[11] = 0.0;
      // weights (|F|^2, F+^2 - Fx^2, 2 F+ Fx) and their changes along a
      // change (da, dc) of (F+, Fx): 2 (a da + c dc), 2 (a da - c dc), 2 (da c + a dc)
      const double a = fp, c = fx;
      dk[12] = a * a + c * c;
      dk[13] = a * a - c * c;
      dk[14] = 2.0 * a * c;
      const double dirs[3][2] = {{gA, gC}, {dA, dC}, {2.0 * c, -2.0 * a}};
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        const double da = dirs[v][0], dc = dirs[v][1];
        dk[15 + 3 * v] = 2.0 * (a * da + c * dc);
        dk[16 + 3 * v] = 2.0 * (a * da - c * dc);
        dk[17 + 3 * v] = 2.0 * (da * c + a * dc);
      }
    } else {
#pragma unroll
      for (int v = 0; v < 24; ++v) dk[v] = 0.0;
      dk[8] = (double)QPAD;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // data term and its derivatives: pairs (k, i)
  const RIFT_GLOBAL double* Q = as_global(P->Q64);
  const int64_t ntp = n_t + 2 * QPAD;
  const int NGR = q_groups(M, QW64);
  const double idt = P->inv_dt;
  double data = 0.0, gg = 0.0, gdec = 0.0, gpsi = 0.0, gi = 0.0, gf = 0.0, gt = 0.0;
  for (int pr = lg; pr < K * M; pr += G) {
    const int k = pr / M, i = pr % M;
    const double* dk = det + 24 * k;
    const double s = dk[9], s2 = s * s;
    double w[4], wd[4];
    w[0] = -s * (s - 1.0) * (s - 2.0) / 6.0;
    w[1] = (s + 1.0) * (s - 1.0) * (s - 2.0) * 0.5;
    w[2] = -(s + 1.0) * s * (s - 2.0) * 0.5;
    w[3] = (s + 1.0) * s * (s - 1.0) / 6.0;
    wd[0] = -(3.0 * s2 - 6.0 * s + 2.0) / 6.0 * idt;
    wd[1] = (3.0 * s2 - 4.0 * s - 1.0) * 0.5 * idt;
    wd[2] = -(3.0 * s2 - 2.0 * s - 2.0) * 0.5 * idt;
    wd[3] = (3.0 * s2 - 1.0) / 6.0 * idt;
    const RIFT_GLOBAL double* q =
        Q + 2 * ((((int64_t)k * NGR + i / QW64) * ntp + (int64_t)dk[8]) * QW64 + i % QW64);
    double qx = 0.0, qy = 0.0, tx = 0.0, ty = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double vx = q[2 * QW64 * j], vy = q[2 * QW64 * j + 1];
      qx += w[j] * vx;
      qy += w[j] * vy;
      tx += wd[j] * vx;
      ty += wd[j] * vy;
    }
    const int m = P->m[i];
    double d = 0.0, dd = 0.0;
    if (P->odd[i]) {
      for (int n = 1; n < NY; ++n) {
        d += P->ycoef[i][n] * stab[n];
        dd += P->ycoef[i][n] * (double)n * ctab[n];
      }
    } else {
      for (int n = 0; n < NY; ++n) {
        d += P->ycoef[i][n] * ctab[n];
        dd -= P->ycoef[i][n] * (double)n * stab[n];
      }
    }
    const int am = m < 0 ? -m : m;
    const double ex = cq[am], ey = m < 0 ? -sq[am] : sq[am];  // e^{i m phi}
    const double yx = d * ex, yy = d * ey, ix = dd * ex, iy = dd * ey;
    const double zx = yx * qx + yy * qy, zy = yx * qy - yy * qx;  // conj(Y) Qhat
    const double ztx = yx * tx + yy * ty, zty = yx * ty - yy * tx;
    const double zix = ix * qx + iy * qy, ziy = ix * qy - iy * qx;
    const double mv = (double)m;
    const double fp = dk[0], fx = dk[1];
    data += fp * zx + fx * zy;
    const double dt_term = fp * ztx + fx * zty;
    gg += dk[2] * zx + dk[3] * zy + dt_term * dk[6];
    gdec += dk[4] * zx + dk[5] * zy + dt_term * dk[7];
    gpsi += 2.0 * fx * zx - 2.0 * fp * zy;
    gi += fp * zix + fx * ziy;
    gf += fp * (mv * zy) + fx * (-mv * zx);
    gt += dt_term;
  }
  // model-norm term and its derivatives: basis rows b over the lanes, the
  // 3 KT columns (3 k + c) of each row in turn
  double quad = 0.0, qg = 0.0, qdec = 0.0, qpsi = 0.0, qi = 0.0, qf = 0.0;
  const RIFT_GLOBAL double* C = as_global(P->C64);
  constexpr int W = 3 * KT;
  for (int b = lg; b < Cls<L>::B; b += G) {
    const int rb = basis_row<L>(b);
    const int kind = rb & 15, n = (rb >> 4) & 255, qq = rb >> 12;
    // T_n(incl) and its incl-derivative
    const double T = (kind >= 3) ? stab[n] : ctab[n];
    const double Tp = (kind >= 3) ? (double)n * ctab[n] : -(double)n * stab[n];
    double beta = T, bi = Tp, bf = 0.0;
    if (kind != 0) {
      const double cqv = cq[qq], sqv = sq[qq], qd = (double)qq;
      if ((kind & 1) == 1) {  // cos(q phi)
        beta = T * cqv;
        bi = Tp * cqv;
        bf = -qd * T * sqv;
      } else {  // sin(q phi)
        beta = T * sqv;
        bi = Tp * sqv;
        bf = qd * T * cqv;
      }
    }
    const RIFT_GLOBAL double* cr = C + (int64_t)b * W;
#pragma unroll
    for (int col = 0; col < W; ++col) {
      const int k = col / 3, c = col - 3 * k;
      const double* dk = det + 24 * k;
      const double cj = cr[col];
      const double cb = cj * beta;
      quad += cb * dk[12 + c];
      qi += cj * bi * dk[12 + c];
      qf += cj * bf * dk[12 + c];
      qg += cb * dk[15 + c];
      qdec += cb * dk[18 + c];
      qpsi += cb * dk[21 + c];
    }
  }
  double bad = 0.0;
  for (int k = lg; k < K; k += G) bad += det[24 * k + 10];
  data = gsum<G>(data);
  gg = gsum<G>(gg);
  gdec = gsum<G>(gdec);
  gpsi = gsum<G>(gpsi);
  gi = gsum<G>(gi);
  gf = gsum<G>(gf);
  gt = gsum<G>(gt);
  quad = gsum<G>(quad);
  qg = gsum<G>(qg);
  qdec = gsum<G>(qdec);
  qpsi = gsum<G>(qpsi);
  qi = gsum<G>(qi);
  qf = gsum<G>(qf);
  bad = gsum<G>(bad);
  double x, x2, lnL;
  bool none = false;
  if constexpr (MARG) {
    const DistFactors Df = dist_factors(P, dist, data, quad, bad != 0.0, *dm, true);
    x = Df.m1;
    x2 = Df.m2;
    lnL = Df.lnL;
    none = Df.none;
  } else {
    x = P->d_ref / dist;
    x2 = x * x;
    lnL = x * data - x2 * quad;
  }
  g[0] = -(x * gg - x2 * qg);
  g[1] = x * gdec - x2 * qdec;
  g[2] = x * gpsi - x2 * qpsi;
  g[3] = x * gi - x2 * qi;
  g[4] = x * gf - x2 * qf;
  g[5] = x * gt;
  g[6] = MARG ? 0.0 : -x * data + 2.0 * x2 * quad;
  if (none) {
#pragma unroll
    for (int a = 0; a < 6; ++a) g[a] = 0.0;
  }
  if (bad != 0.0) {
    const double nan = __builtin_nan("");
#pragma unroll
    for (int a = 0; a < 7; ++a) g[a] = nan;
    return nan;
  }
  return lnL;
}

}  // namespace rift
