// Plain FP64 CPU oracle for the factored extrinsic likelihood and its
// Monte-Carlo evidence reduction.
//
// TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link,
// load or call this file.  It exists to be the slow, obviously correct
// reference that the HIP kernels are compared against, and it shares no code
// with them.
//
// Everything here follows the paper's own order of operations:
//   * antenna response and arrival time:   Sec. "Review of the RIFT likelihood"
//     (static response paragraph: constant F+, Fx; t_k = t_c - x_k . n)
//   * spin-weighted harmonics -2Y_lm:      Eq. (strain_mode)
//   * four-point cubic read of Q on the fine grid:  Eq. (q-time-pregrid)
//   * factored log-likelihood:             Eq. (def:lnL:Decomposed)
//   * Monte-Carlo marginal likelihood:     Eq. (lnL:MonteCarlo)
//   * effective sample size:               Eq. (neff)
//   * gradient (the differentiable path):  Sec. "The differentiable likelihood"
//   * composite-index likelihood (Earth rotation, Path A; finite arms, Path D):
//     Sec. "A generalized detector response", Eqs. (slowrot:Fharm),
//     (slowrot:postphase), (slowrot:lnL:Decomposed), (fsize:bp)
//   * the distance-free terms K, R of lnL(x) = K x - R x^2 / 2:  Eq. (ap:dexp)
//     (the adaptive Gauss-Hermite marginal over distance built on them,
//     Eqs. (ap:dpeak), (ap:dgh), is in the Python layer of the oracle)
//
// Readings where the paper is silent or inconsistent (all listed in the
// design notes of the repository):
//   * complex antenna factor F = F+ + i Fx (the strain is h = h+ - i hx, and
//     the response h_k = F+ h+ + Fx hx must equal Re[F h]);
//   * arrival time t_k = t_ref - r_k . N, with N pointing to the source and r_k
//     in light-seconds;
//   * "four-point cubic" = 4-point Lagrange interpolation on nodes j-1..j+2,
//     with taps outside the stored window reading zero;
//   * the V term carries Re(...), as in Eq. (def:lnL:Decomposed);
//   * ln Z normalised by 1/N with caller-supplied ln(p/p_s).
//
// Build: g++ -O2 -fopenmp -shared -fPIC oracle.cpp -o liboracle.so
// Precision: IEEE double throughout, libm transcendentals.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <limits>
#include <omp.h>

namespace {

// ---------------------------------------------------------------------------
// Forward-mode dual number with NT tangents, for the oracle gradient.
// ---------------------------------------------------------------------------
template <int NT>
struct Dual {
  double v;
  double d[NT];
  Dual() : v(0) { for (int i = 0; i < NT; ++i) d[i] = 0; }
  Dual(double x) : v(x) { for (int i = 0; i < NT; ++i) d[i] = 0; }
};
template <int NT> Dual<NT> operator+(const Dual<NT>& a, const Dual<NT>& b) {
  Dual<NT> r; r.v = a.v + b.v; for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int NT> Dual<NT> operator-(const Dual<NT>& a, const Dual<NT>& b) {
  Dual<NT> r; r.v = a.v - b.v; for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int NT> Dual<NT> operator-(const Dual<NT>& a) {
  Dual<NT> r; r.v = -a.v; for (int i = 0; i < NT; ++i) r.d[i] = -a.d[i]; return r; }
template <int NT> Dual<NT> operator*(const Dual<NT>& a, const Dual<NT>& b) {
  Dual<NT> r; r.v = a.v * b.v; for (int i = 0; i < NT; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int NT> Dual<NT> operator/(const Dual<NT>& a, const Dual<NT>& b) {
  Dual<NT> r; r.v = a.v / b.v;
  for (int i = 0; i < NT; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r; }
template <int NT> Dual<NT> operator+(const Dual<NT>& a, double b) { return a + Dual<NT>(b); }
template <int NT> Dual<NT> operator+(double a, const Dual<NT>& b) { return Dual<NT>(a) + b; }
template <int NT> Dual<NT> operator-(const Dual<NT>& a, double b) { return a - Dual<NT>(b); }
template <int NT> Dual<NT> operator-(double a, const Dual<NT>& b) { return Dual<NT>(a) - b; }
template <int NT> Dual<NT> operator*(const Dual<NT>& a, double b) { return a * Dual<NT>(b); }
template <int NT> Dual<NT> operator*(double a, const Dual<NT>& b) { return Dual<NT>(a) * b; }
template <int NT> Dual<NT> operator/(const Dual<NT>& a, double b) { return a / Dual<NT>(b); }
template <int NT> Dual<NT> operator/(double a, const Dual<NT>& b) { return Dual<NT>(a) / b; }
template <int NT> Dual<NT> sin(const Dual<NT>& a) {
  Dual<NT> r;
  r.v = std::sin(a.v);
  double c = std::cos(a.v);
  for (int i = 0; i < NT; ++i) r.d[i] = c * a.d[i];
  return r;
}
template <int NT> Dual<NT> cos(const Dual<NT>& a) {
  Dual<NT> r;
  r.v = std::cos(a.v);
  double s = -std::sin(a.v);
  for (int i = 0; i < NT; ++i) r.d[i] = s * a.d[i];
  return r;
}
template <int NT> Dual<NT> exp(const Dual<NT>& a) {
  Dual<NT> r;
  r.v = std::exp(a.v);
  for (int i = 0; i < NT; ++i) r.d[i] = r.v * a.d[i];
  return r;
}
template <int NT> Dual<NT> acos(const Dual<NT>& a) {
  Dual<NT> r;
  r.v = std::acos(a.v);
  double g = -1.0 / std::sqrt(1.0 - a.v * a.v);
  for (int i = 0; i < NT; ++i) r.d[i] = g * a.d[i];
  return r;
}
using std::sin;
using std::cos;
using std::exp;
using std::acos;
template <int NT> double value(const Dual<NT>& a) { return a.v; }
inline double value(double a) { return a; }

// Minimal complex type usable with both double and Dual.
template <class T>
struct Cx {
  T re, im;
};
template <class T> Cx<T> cmul(const Cx<T>& a, const Cx<T>& b) {
  return Cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
template <class T> Cx<T> cconj(const Cx<T>& a) { return Cx<T>{a.re, T(0.0) - a.im}; }

double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

// ---------------------------------------------------------------------------
// Point description (paper order of every array).
// ---------------------------------------------------------------------------
struct Point {
  int32_t K, M, n_t;
  const int32_t* lm;      // [M][2] (l, m)
  double t0, dt;          // Q grid: t_j = t0 + j dt  (seconds)
  const double* Q;        // [K][M][n_t] complex interleaved
  const double* U;        // [K][M][M] complex interleaved, U_{k, i, j}
  const double* V;        // [K][M][M] complex interleaved
  const double* det_tensor;  // [K][3][3]
  const double* det_pos;     // [K][3] light-seconds
  double gmst;            // Greenwich sidereal angle at the reference epoch (rad)
  double d_ref;           // reference distance of Eq. (strain_mode)
};

// -2Y_lm(iota, phi): Wigner-d sum (Goldberg et al. 1967 form), spin weight -2,
// i.e. (-1)^s sqrt((2l+1)/4pi) d^l_{m,s}(iota) e^{i m phi} with s = 2.
template <class T>
Cx<T> ylm_m2(int l, int m, const T& iota, const T& phi) {
  const int s = 2;
  T c = cos(iota * 0.5);
  T sn = sin(iota * 0.5);
  T d(0.0);
  int kmin = (m - s > 0) ? (m - s) : 0;
  int kmax = (l + m < l - s) ? (l + m) : (l - s);
  double pref = std::sqrt(factorial(l + m) * factorial(l - m) * factorial(l + s) * factorial(l - s));
  for (int k = kmin; k <= kmax; ++k) {
    double coef = ((k % 2) ? -1.0 : 1.0) * pref /
                  (factorial(l + m - k) * factorial(l - s - k) * factorial(k) * factorial(k + s - m));
    int pc = 2 * l + m - s - 2 * k;
    int ps = 2 * k + s - m;
    T term(coef);
    for (int i = 0; i < pc; ++i) term = term * c;
    for (int i = 0; i < ps; ++i) term = term * sn;
    d = d + term;
  }
  double norm = ((s % 2) ? -1.0 : 1.0) * std::sqrt((2.0 * l + 1.0) / (4.0 * M_PI));
  T amp = d * norm;
  T ang = phi * double(m);
  return Cx<T>{amp * cos(ang), amp * sin(ang)};
}

// Source direction N (towards the source) and polarisation axes X, Y in the
// Earth-fixed frame (x: Greenwich meridian on the equator, z: north pole).
template <class T>
void sky_frame(const T& ra, const T& dec, const T& psi, double gmst, T N[3], T X[3], T Y[3]) {
  T gha = gmst - ra;
  T cg = cos(gha), sg = sin(gha), cd = cos(dec), sd = sin(dec), cp = cos(psi), sp = sin(psi);
  N[0] = cd * cg; N[1] = T(0.0) - cd * sg; N[2] = sd;
  T ea[3] = {sg, cg, T(0.0)};
  T ed[3] = {T(0.0) - sd * cg, sd * sg, cd};
  for (int i = 0; i < 3; ++i) {
    X[i] = T(0.0) - cp * ea[i] + sp * ed[i];
    Y[i] = sp * ea[i] + cp * ed[i];
  }
}

// F = F+ + i Fx with F+ = D : (X X^T - Y Y^T) and Fx = D : (X Y^T + Y X^T).
template <class T>
Cx<T> antenna(const double* D, const T X[3], const T Y[3]) {
  T fp(0.0), fx(0.0);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double dij = D[3 * i + j];
      fp = fp + dij * (X[i] * X[j] - Y[i] * Y[j]);
      fx = fx + dij * (X[i] * Y[j] + Y[i] * X[j]);
    }
  return Cx<T>{fp, fx};
}

// Four-point Lagrange read of a uniformly sampled complex series.  The
// stencil is nodes j-1, j, j+1, j+2 around u = (t - t0)/dt, j = floor(u);
// nodes outside [0, n_t) contribute zero.
template <class T>
Cx<T> interp_lagrange4(const double* q, int n_t, double t0, double dt, const T& t) {
  T u = (t - t0) / dt;
  if (!std::isfinite(value(u))) {  // a non-finite time poisons the read
    const double nan = std::numeric_limits<double>::quiet_NaN();
    return Cx<T>{T(nan), T(nan)};
  }
  double j = std::floor(value(u));
  T s = u - j;
  T w[4];
  w[0] = T(0.0) - s * (s - 1.0) * (s - 2.0) / 6.0;
  w[1] = (s + 1.0) * (s - 1.0) * (s - 2.0) / 2.0;
  w[2] = T(0.0) - (s + 1.0) * s * (s - 2.0) / 2.0;
  w[3] = (s + 1.0) * s * (s - 1.0) / 6.0;
  Cx<T> out{T(0.0), T(0.0)};
  for (int i = 0; i < 4; ++i) {
    double node = j - 1.0 + i;
    if (!(node >= 0.0 && node < (double)n_t)) continue;  // zero extension (also NaN)
    int64_t n = (int64_t)node;
    out.re = out.re + w[i] * q[2 * n];
    out.im = out.im + w[i] * q[2 * n + 1];
  }
  return out;
}

// Factored log-likelihood, Eq. (def:lnL:Decomposed), given F_k, Y_lm, x = D_ref/D
// and the Q values already read at t_k.
// The two terms of Eq. (def:lnL:Decomposed) at the reference distance:
// data = Re sum_k sum_lm conj(F_k Y_lm) Qhat_{k,lm} and
// quad = sum_k [|F_k|^2 Y^H U_k Y + Re(F_k^2 Y^T V_k Y)], so that
// lnL(x) = x data - x^2 quad / 4 with x = D_ref / D.
template <class T>
void terms_factored(int K, int M, const Cx<T>* F, const Cx<T>* Y, const Cx<T>* Qhat, const double* U,
                    const double* V, T* data_out, T* quad_out) {
  T data(0.0), quad(0.0);
  for (int k = 0; k < K; ++k) {
    for (int i = 0; i < M; ++i) {
      Cx<T> c = cconj(cmul(F[k], Y[i]));
      Cx<T> q = Qhat[k * M + i];
      data = data + (c.re * q.re - c.im * q.im);
    }
    Cx<T> a{T(0.0), T(0.0)}, b{T(0.0), T(0.0)};
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j) {
        const double* u = U + 2 * ((size_t)(k * M + i) * M + j);
        const double* v = V + 2 * ((size_t)(k * M + i) * M + j);
        Cx<T> uu{T(u[0]), T(u[1])}, vv{T(v[0]), T(v[1])};
        Cx<T> ta = cmul(cmul(cconj(Y[i]), uu), Y[j]);
        Cx<T> tb = cmul(cmul(Y[i], vv), Y[j]);
        a.re = a.re + ta.re; a.im = a.im + ta.im;
        b.re = b.re + tb.re; b.im = b.im + tb.im;
      }
    T f2abs = F[k].re * F[k].re + F[k].im * F[k].im;
    Cx<T> f2 = cmul(F[k], F[k]);
    quad = quad + f2abs * a.re + (f2.re * b.re - f2.im * b.im);
  }
  *data_out = data;
  *quad_out = quad;
}

template <class T>
T lnL_factored(int K, int M, const Cx<T>* F, const Cx<T>* Y, const T& x,
               const Cx<T>* Qhat, const double* U, const double* V) {
  T data, quad;
  terms_factored(K, M, F, Y, Qhat, U, V, &data, &quad);
  return x * data - x * x * quad * 0.25;
}

// The per-sample terms (data, quad) of the likelihood, at the reference
// distance, from the extrinsic parameters other than the distance.
void terms_one(const Point& p, double ra, double dec, double psi, double iota, double phi, double tref,
               double* data, double* quad) {
  double N[3], X[3], Y3[3];
  sky_frame(ra, dec, psi, p.gmst, N, X, Y3);
  std::vector<Cx<double>> F(p.K), Y(p.M), Qhat((size_t)p.K * p.M);
  for (int k = 0; k < p.K; ++k) {
    F[k] = antenna(p.det_tensor + 9 * k, X, Y3);
    const double* r = p.det_pos + 3 * k;
    double tk = tref - (r[0] * N[0] + r[1] * N[1] + r[2] * N[2]);
    for (int i = 0; i < p.M; ++i)
      Qhat[(size_t)k * p.M + i] =
          interp_lagrange4(p.Q + 2 * ((size_t)(k * p.M + i) * p.n_t), p.n_t, p.t0, p.dt, tk);
  }
  for (int i = 0; i < p.M; ++i) Y[i] = ylm_m2(p.lm[2 * i], p.lm[2 * i + 1], iota, phi);
  terms_factored(p.K, p.M, F.data(), Y.data(), Qhat.data(), p.U, p.V, data, quad);
}

// Full per-sample likelihood from the extrinsic parameters.
template <class T>
T lnL_one(const Point& p, const T& ra, const T& dec, const T& psi, const T& iota,
          const T& phi, const T& tref, const T& dist) {
  T N[3], X[3], Y3[3];
  sky_frame(ra, dec, psi, p.gmst, N, X, Y3);
  std::vector<Cx<T>> F(p.K), Y(p.M), Qhat((size_t)p.K * p.M);
  for (int k = 0; k < p.K; ++k) {
    F[k] = antenna(p.det_tensor + 9 * k, X, Y3);
    const double* r = p.det_pos + 3 * k;
    T tk = tref - (r[0] * N[0] + r[1] * N[1] + r[2] * N[2]);
    for (int i = 0; i < p.M; ++i)
      Qhat[(size_t)k * p.M + i] =
          interp_lagrange4(p.Q + 2 * ((size_t)(k * p.M + i) * p.n_t), p.n_t, p.t0, p.dt, tk);
  }
  for (int i = 0; i < p.M; ++i) Y[i] = ylm_m2(p.lm[2 * i], p.lm[2 * i + 1], iota, phi);
  T x = p.d_ref / dist;
  return lnL_factored(p.K, p.M, F.data(), Y.data(), x, Qhat.data(), p.U, p.V);
}

// ---------------------------------------------------------------------------
// Generalised (composite-index) response, Sec. "A generalized detector
// response": the mode index widens to A = (a, lm) and the antenna factor F_k
// to a coefficient C~^k_a per composite term a.  Two responses:
//   rotation (Path A, "Earth rotation: a slowly time-varying response"):
//     a <-> sidereal harmonic n = a - 2 in -2..2.  F_k as a function of the
//     Greenwich hour angle g is a trigonometric polynomial of degree 2,
//     F_k(g) = sum_n A_n e^{i n g} (Eq. (slowrot:Fharm)), with A_n depending on
//     dec and psi only.  C^k_n = A_n e^{i n g(t_ref)} and the arrival-time
//     post-phase of Eq. (slowrot:postphase) gives C~^k_n = C^k_n e^{i n W (t_k - t_ref)}.
//     g(t) = gmst + W t - ra, t on the axis of t_ref (W the sidereal rate);
//     the delay is held at t_k = t_ref - r_k . N(g(t_ref)) (Path A).
//   arms (Path D, "Long arms: a frequency-dependent response"):
//     a <-> order p = a of the arm-projection expansion, Eq. (fsize:bp):
//     b^k_p = 1/2 [ (x.N)^p e:xx - (y.N)^p e:yy ] with x, y the arm unit
//     vectors, N towards the source and e = e+ + i ex the complex polarisation
//     tensor of the reading F = F+ + i Fx (so b_0 = D : e = F_k for
//     D = (x x^T - y y^T)/2).  Static sky frame.
// The likelihood is Eq. (slowrot:lnL:Decomposed) with Q, U, V over the
// composite index (layout [k][a][lm][n_t] and [k][a M + i][a' M + j]).
// ---------------------------------------------------------------------------
struct PointWide {
  int32_t K, M, n_t;
  const int32_t* lm;
  double t0, dt;
  int32_t response;        // 1: rotation, 2: arms
  int32_t n_a;             // composite terms per detector
  const double* Q;         // [K][n_a][M][n_t] complex
  const double* U;         // [K][n_a M][n_a M] complex
  const double* V;         // [K][n_a M][n_a M] complex
  const double* det_tensor;  // [K][3][3]
  const double* det_pos;     // [K][3] light-seconds
  const double* det_arms;    // [K][2][3] arm unit vectors (arms response)
  double gmst;             // Greenwich sidereal angle at t = 0 (rad)
  double omega;            // sidereal rate (rad/s), rotation response
  double d_ref;
};

// The five sidereal Fourier coefficients A_n (n = -2..2) of F_k(g) at fixed
// dec and psi: the exact 5-point discrete Fourier transform of the degree-2
// trigonometric polynomial F_k over g.
void rotation_harmonics(const double* det_tensor, double dec, double psi, Cx<double> A[5]) {
  const double two_pi = 2.0 * M_PI;
  Cx<double> Fg[5];
  for (int j = 0; j < 5; ++j) {
    const double g = two_pi * j / 5.0;
    double N[3], X[3], Y[3];
    // hour angle g = gmst - ra with gmst = g, ra = 0
    sky_frame<double>(0.0, dec, psi, g, N, X, Y);
    Fg[j] = antenna<double>(det_tensor, X, Y);
  }
  for (int n = -2; n <= 2; ++n) {
    Cx<double> acc{0.0, 0.0};
    for (int j = 0; j < 5; ++j) {
      const double g = two_pi * j / 5.0;
      const Cx<double> e{std::cos(n * g), -std::sin(n * g)};
      const Cx<double> t = cmul(Fg[j], e);
      acc.re += t.re;
      acc.im += t.im;
    }
    A[n + 2] = Cx<double>{acc.re / 5.0, acc.im / 5.0};
  }
}

// Composite coefficients C~[k][a] and arrival times t_k of one sample.
void wide_coefficients(const PointWide& p, double ra, double dec, double psi, double tref,
                       std::vector<Cx<double>>& C, std::vector<double>& tk) {
  C.assign((size_t)p.K * p.n_a, Cx<double>{0.0, 0.0});
  tk.assign(p.K, 0.0);
  const double gm = (p.response == 1 || p.response == 3) ? p.gmst + p.omega * tref : p.gmst;
  double N[3], X[3], Y[3];
  sky_frame<double>(ra, dec, psi, gm, N, X, Y);
  for (int k = 0; k < p.K; ++k) {
    const double* r = p.det_pos + 3 * k;
    tk[k] = tref - (r[0] * N[0] + r[1] * N[1] + r[2] * N[2]);
    if (p.response == 1) {
      Cx<double> A[5];
      rotation_harmonics(p.det_tensor + 9 * k, dec, psi, A);
      const double gref = gm - ra;  // g(t_ref)
      for (int a = 0; a < p.n_a; ++a) {
        const int n = a - 2;
        const double ph = n * gref + n * p.omega * (tk[k] - tref);
        C[(size_t)k * p.n_a + a] = cmul(A[a], Cx<double>{std::cos(ph), std::sin(ph)});
      }
    } else if (p.response == 3) {
      // rotation with the delay drift to order P (Path B), n_a = (P + 1)(P + 5):
      // index a = P(4 + P) offset of order p, then n~ = -(2 + p) .. 2 + p.
      // The delay tau(g) = -r . N(g) over the hour angle g carries the
      // harmonics 0, +-1; -dt(phi) = -(tau(g_ref + phi) - tau(g_ref)) in the
      // modulation phase phi = Omega (t - t_ref):
      //   m = 0: -cos(dec) Re(rho e^{i g_ref}),  m = +1: cos(dec)/2 rho e^{i g_ref},
      //   m = -1: cos(dec)/2 conj(rho e^{i g_ref}),  rho = r_x + i r_y.
      // C_(p, n~) = (1/p!) sum_{n + m = n~} A_n e^{i n g_ref} [(-dt)^{*p}]_m
      // (Eq. (slowrot:master)), then the post-phase e^{i n~ Omega (t_k - t_ref)}.
      int P = 0;
      while ((P + 1) * (P + 5) < p.n_a) ++P;
      Cx<double> A[5];
      rotation_harmonics(p.det_tensor + 9 * k, dec, psi, A);
      const double gref = gm - ra;
      const Cx<double> eg{std::cos(gref), std::sin(gref)};
      const Cx<double> re = cmul(Cx<double>{r[0], r[1]}, eg);
      const double cdec = std::cos(dec);
      // harmonics of -dt, index m + 1
      const Cx<double> D1[3] = {Cx<double>{0.5 * cdec * re.re, -0.5 * cdec * re.im}, Cx<double>{-cdec * re.re, 0.0},
                                Cx<double>{0.5 * cdec * re.re, 0.5 * cdec * re.im}};
      std::vector<Cx<double>> pw(1, Cx<double>{1.0, 0.0});  // (-dt)^p, index m + p
      double fact = 1.0;
      int base = 0;
      for (int pp = 0; pp <= P; ++pp) {
        if (pp > 0) {
          std::vector<Cx<double>> nx(2 * pp + 1, Cx<double>{0.0, 0.0});
          for (int m = -(pp - 1); m <= pp - 1; ++m)
            for (int d = -1; d <= 1; ++d) {
              const Cx<double> t = cmul(pw[m + pp - 1], D1[d + 1]);
              nx[m + d + pp].re += t.re;
              nx[m + d + pp].im += t.im;
            }
          pw.swap(nx);
          fact *= pp;
        }
        for (int nt = -(2 + pp); nt <= 2 + pp; ++nt) {
          Cx<double> acc{0.0, 0.0};
          for (int n = -2; n <= 2; ++n) {
            const int m = nt - n;
            if (m < -pp || m > pp) continue;
            const Cx<double> an = cmul(A[n + 2], Cx<double>{std::cos(n * gref), std::sin(n * gref)});
            const Cx<double> t = cmul(an, pw[m + pp]);
            acc.re += t.re;
            acc.im += t.im;
          }
          const double ph = nt * p.omega * (tk[k] - tref);
          const Cx<double> c = cmul(acc, Cx<double>{std::cos(ph) / fact, std::sin(ph) / fact});
          C[(size_t)k * p.n_a + base + nt + 2 + pp] = c;
        }
        base += 5 + 2 * pp;
      }
    } else {
      const double* ax = p.det_arms + 6 * k;
      const double* ay = ax + 3;
      // e : a a = (X.a + i Y.a)^2 for a unit arm vector a
      const double xX = X[0] * ax[0] + X[1] * ax[1] + X[2] * ax[2];
      const double xY = Y[0] * ax[0] + Y[1] * ax[1] + Y[2] * ax[2];
      const double yX = X[0] * ay[0] + X[1] * ay[1] + X[2] * ay[2];
      const double yY = Y[0] * ay[0] + Y[1] * ay[1] + Y[2] * ay[2];
      const Cx<double> ex = cmul(Cx<double>{xX, xY}, Cx<double>{xX, xY});
      const Cx<double> ey = cmul(Cx<double>{yX, yY}, Cx<double>{yX, yY});
      const double ux = N[0] * ax[0] + N[1] * ax[1] + N[2] * ax[2];
      const double uy = N[0] * ay[0] + N[1] * ay[1] + N[2] * ay[2];
      double px = 1.0, py = 1.0;
      for (int a = 0; a < p.n_a; ++a) {
        C[(size_t)k * p.n_a + a] = Cx<double>{0.5 * (px * ex.re - py * ey.re), 0.5 * (px * ex.im - py * ey.im)};
        px *= ux;
        py *= uy;
      }
    }
  }
}

// Eq. (slowrot:lnL:Decomposed) for one sample: plain loops over detectors,
// composite terms and modes.
double lnL_wide_one(const PointWide& p, double ra, double dec, double psi, double iota, double phi,
                    double tref, double dist) {
  std::vector<Cx<double>> C, Y(p.M);
  std::vector<double> tk;
  wide_coefficients(p, ra, dec, psi, tref, C, tk);
  for (int i = 0; i < p.M; ++i) Y[i] = ylm_m2<double>(p.lm[2 * i], p.lm[2 * i + 1], iota, phi);
  const int A = p.n_a * p.M;
  std::vector<Cx<double>> c(A);
  double data = 0.0, quad = 0.0;
  for (int k = 0; k < p.K; ++k) {
    for (int a = 0; a < p.n_a; ++a)
      for (int i = 0; i < p.M; ++i) c[a * p.M + i] = cmul(C[(size_t)k * p.n_a + a], Y[i]);
    // data term: Re sum_A conj(c_A) Q_{k,A}(t_k)
    for (int a = 0; a < p.n_a; ++a)
      for (int i = 0; i < p.M; ++i) {
        const double* q = p.Q + 2 * ((((size_t)k * p.n_a + a) * p.M + i) * p.n_t);
        const Cx<double> qh = interp_lagrange4<double>(q, p.n_t, p.t0, p.dt, tk[k]);
        const Cx<double> t = cmul(cconj(c[a * p.M + i]), qh);
        data += t.re;
      }
    // quadratic term: c^H U c + Re(c^T V c)
    Cx<double> cu{0.0, 0.0}, cv{0.0, 0.0};
    for (int I = 0; I < A; ++I)
      for (int J = 0; J < A; ++J) {
        const double* u = p.U + 2 * (((size_t)k * A + I) * A + J);
        const double* v = p.V + 2 * (((size_t)k * A + I) * A + J);
        const Cx<double> tu = cmul(cmul(cconj(c[I]), Cx<double>{u[0], u[1]}), c[J]);
        const Cx<double> tv = cmul(cmul(c[I], Cx<double>{v[0], v[1]}), c[J]);
        cu.re += tu.re; cu.im += tu.im;
        cv.re += tv.re; cv.im += tv.im;
      }
    quad += cu.re + cv.re;
  }
  const double x = p.d_ref / dist;
  return x * data - x * x * quad * 0.25;
}

}  // namespace

extern "C" {

int oracle_version() { return 1; }

// Sidereal harmonics A_n (n = -2..2) of one detector's F(g): out[5][2].
void oracle_rotation_harmonics(const double* det_tensor, double dec, double psi, double* out) {
  Cx<double> A[5];
  rotation_harmonics(det_tensor, dec, psi, A);
  for (int n = 0; n < 5; ++n) { out[2 * n] = A[n].re; out[2 * n + 1] = A[n].im; }
}

// Composite coefficients C~[K][n_a][2] and arrival times tk[K] of one sample
// theta[7] (ra, dec, psi, incl, phiref, tref, dist).
void oracle_wide_coef(const PointWide* p, const double* theta, double* C, double* tk) {
  std::vector<Cx<double>> c;
  std::vector<double> t;
  wide_coefficients(*p, theta[0], theta[1], theta[2], theta[5], c, t);
  for (size_t i = 0; i < c.size(); ++i) { C[2 * i] = c[i].re; C[2 * i + 1] = c[i].im; }
  for (int k = 0; k < p->K; ++k) tk[k] = t[k];
}

// lnL of the composite-index likelihood for n samples (SoA [7][n]).
void oracle_lnL_wide(const PointWide* p, int64_t n, const double* theta, double* lnL, int nthreads) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    lnL[i] = lnL_wide_one(*p, theta[i], theta[n + i], theta[2 * n + i], theta[3 * n + i], theta[4 * n + i],
                          theta[5 * n + i], theta[6 * n + i]);
}

// -2Y_lm(iota, phi) -> out[2] = (re, im)
void oracle_ylm(int l, int m, double iota, double phi, double* out) {
  Cx<double> y = ylm_m2<double>(l, m, iota, phi);
  out[0] = y.re; out[1] = y.im;
}

// Complex antenna factor of one detector; out[2] = (F+, Fx).  N_out[3] (may be
// NULL) receives the unit vector towards the source.
void oracle_antenna(const double* det_tensor, double ra, double dec, double psi, double gmst,
                    double* out, double* N_out) {
  double N[3], X[3], Y[3];
  sky_frame<double>(ra, dec, psi, gmst, N, X, Y);
  Cx<double> f = antenna<double>(det_tensor, X, Y);
  out[0] = f.re; out[1] = f.im;
  if (N_out) for (int i = 0; i < 3; ++i) N_out[i] = N[i];
}

// Arrival time at a detector at position r (light-seconds).
double oracle_arrival_time(const double* r, double ra, double dec, double gmst, double tref) {
  double N[3], X[3], Y[3];
  sky_frame<double>(ra, dec, 0.0, gmst, N, X, Y);
  return tref - (r[0] * N[0] + r[1] * N[1] + r[2] * N[2]);
}

// Four-point Lagrange read of one complex series q[n_t][2] at times t[n].
void oracle_interp(const double* q, int n_t, double t0, double dt, int64_t n, const double* t,
                   double* out) {
  for (int64_t i = 0; i < n; ++i) {
    Cx<double> v = interp_lagrange4<double>(q, n_t, t0, dt, t[i]);
    out[2 * i] = v.re; out[2 * i + 1] = v.im;
  }
}

// Eq. (def:lnL:Decomposed) from given F[K][2], Y[M][2], x, Qhat[K][M][2].
double oracle_lnL_factored(int K, int M, const double* F, const double* Y, double x,
                           const double* Qhat, const double* U, const double* V) {
  std::vector<Cx<double>> f(K), y(M), q((size_t)K * M);
  for (int k = 0; k < K; ++k) f[k] = Cx<double>{F[2 * k], F[2 * k + 1]};
  for (int i = 0; i < M; ++i) y[i] = Cx<double>{Y[2 * i], Y[2 * i + 1]};
  for (size_t i = 0; i < (size_t)K * M; ++i) q[i] = Cx<double>{Qhat[2 * i], Qhat[2 * i + 1]};
  return lnL_factored<double>(K, M, f.data(), y.data(), x, q.data(), U, V);
}

// lnL for n samples; theta is SoA [7][n]: ra, dec, psi, incl, phiref, tref, dist.
void oracle_lnL(const Point* p, int64_t n, const double* theta, double* lnL, int nthreads) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    lnL[i] = lnL_one<double>(*p, theta[i], theta[n + i], theta[2 * n + i], theta[3 * n + i],
                             theta[4 * n + i], theta[5 * n + i], theta[6 * n + i]);
  }
}

// The distance-free terms of n samples: K_i = data_i and R_i = quad_i / 2, so
// that lnL_i(x) = K_i x - R_i x^2 / 2 exactly (Eq. (ap:dexp)); the distance
// row of theta is not read.
void oracle_lnL_terms(const Point* p, int64_t n, const double* theta, double* Kout, double* Rout, int nthreads) {
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double data, quad;
    terms_one(*p, theta[i], theta[n + i], theta[2 * n + i], theta[3 * n + i], theta[4 * n + i], theta[5 * n + i],
              &data, &quad);
    Kout[i] = data;
    Rout[i] = 0.5 * quad;
  }
}

// lnL and its gradient with respect to (ra, dec, psi, cos incl, phiref, tref, ln dist),
// grad SoA [7][n].  Forward-mode dual numbers over the same code as oracle_lnL.
void oracle_grad(const Point* p, int64_t n, const double* theta, double* lnL, double* grad,
                 int nthreads) {
  typedef Dual<7> D7;
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    D7 v[7];
    for (int a = 0; a < 7; ++a) v[a] = D7(theta[a * n + i]);
    // independent coordinates: ra, dec, psi, cos(incl), phiref, tref, ln(dist)
    D7 ra = v[0], dec = v[1], psi = v[2], phi = v[4], tref = v[5];
    ra.d[0] = 1; dec.d[1] = 1; psi.d[2] = 1; phi.d[4] = 1; tref.d[5] = 1;
    D7 cosi(std::cos(theta[3 * n + i])); cosi.d[3] = 1;
    D7 iota = acos(cosi);
    iota.v = theta[3 * n + i];  // keep the caller's angle exactly; tangent from acos
    D7 lnd(std::log(theta[6 * n + i])); lnd.d[6] = 1;
    D7 dist = exp(lnd);
    dist.v = theta[6 * n + i];
    D7 r = lnL_one<D7>(*p, ra, dec, psi, iota, phi, tref, dist);
    lnL[i] = r.v;
    for (int a = 0; a < 7; ++a) grad[a * n + i] = r.d[a];
  }
}

// Eq. (lnL:MonteCarlo) in log form and Eq. (neff):
//   lnZ = ln[(1/N) sum_i exp(lnL_i + lnw_i)],  neff = sum_i p_i / max_i p_i.
// lnw may be NULL (all zero).  Any NaN makes both outputs NaN.
void oracle_lnZ(int64_t n, const double* lnL, const double* lnw, double* lnZ, double* neff) {
  const double ninf = -std::numeric_limits<double>::infinity();
  double m = ninf;
  bool nan = false;
  for (int64_t i = 0; i < n; ++i) {
    double l = lnL[i] + (lnw ? lnw[i] : 0.0);
    if (std::isnan(l)) nan = true;
    else if (l > m) m = l;
  }
  if (nan || n <= 0) {
    *lnZ = std::numeric_limits<double>::quiet_NaN();
    *neff = std::numeric_limits<double>::quiet_NaN();
    return;
  }
  if (m == ninf) { *lnZ = ninf; *neff = 0.0; return; }
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += std::exp(lnL[i] + (lnw ? lnw[i] : 0.0) - m);
  *lnZ = m + std::log(s) - std::log((double)n);
  *neff = s;
}

}  // extern "C"
