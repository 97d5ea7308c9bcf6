// Host-side helpers shared by the translation units of the library.
#pragma once

#include <algorithm>
#include <cmath>

#include "ile_device.h"

namespace rift {

inline double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

// Wigner d^l_{m,s}(beta), explicit sum over k (s = 2 for spin weight -2):
// the form of Goldberg et al. (1967) behind the -2Y_lm of Eq. (strain_mode).
inline double wigner_d(int l, int m, int s, double beta) {
  const double c = cos(0.5 * beta), sn = sin(0.5 * beta);
  const int k0 = std::max(0, m - s), k1 = std::min(l + m, l - s);
  const double pre = sqrt(factorial(l + m) * factorial(l - m) * factorial(l + s) * factorial(l - s));
  double d = 0.0;
  for (int k = k0; k <= k1; ++k) {
    const double den = factorial(l + m - k) * factorial(l - s - k) * factorial(k) * factorial(k + s - m);
    d += ((k & 1) ? -1.0 : 1.0) * pre / den * pow(c, 2 * l + m - s - 2 * k) * pow(sn, 2 * k + s - m);
  }
  return d;
}

// Fourier coefficients in incl of sqrt((2l+1)/4pi) d^l_{m,2}(incl): a cosine
// series for even m, a sine series for odd m, degree <= l (exact by a 32-point
// DFT since l <= 8).
inline void ylm_fourier(int l, int m, double* out /* [LMAXC+1] */) {
  const int N = 32;
  const double two_pi = 6.283185307179586476925286766559;
  const double norm = sqrt((2.0 * l + 1.0) / (2.0 * two_pi));
  for (int n = 0; n <= LMAXC; ++n) out[n] = 0.0;
  for (int n = 0; n <= l; ++n) {
    double acc = 0.0;
    for (int p = 0; p < N; ++p) {
      const double b = two_pi * p / N;
      const double d = wigner_d(l, m, 2, b);
      acc += d * ((m & 1) ? sin(n * b) : cos(n * b));
    }
    out[n] = norm * acc * ((n == 0) ? 1.0 : 2.0) / N;
  }
  if (m & 1) out[0] = 0.0;
}

}  // namespace rift
