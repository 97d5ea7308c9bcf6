// Fourier refinement of sampled correlation series on the device,
// Eq. (q-time-pregrid): each series q[0..n-1] (spacing h) is extended by its
// reversed copy to a continuous period of L = 2n samples, its spectrum is
// zero-padded by r (the Nyquist bin split in halves between +L/2 and -L/2)
// and transformed back, giving (n-1) r + 1 samples at spacing h / r that
// reproduce the nodes.
//
// That chain is linear with real coefficients, so the refined series is one
// dense contraction shared by every series:
//   fine[j] = sum_{i<n} T(j, i) q[i],
//   T(j, i) = D(j/r - i) + D(j/r - (2n-1-i)),
//   D(u)    = (1/L) sum over the padded spectrum of e^{2 pi i k u / L}
//           = sin(pi u) cot(pi u / L) / L     (the Nyquist half-bins add cos(pi u)),
// D(0) = 1 and D = 0 at the other integers.  With j = a r + b (phase b), the
// kernel depends on (a - i) and (a + i + 1 - 2n) only, so one table per
// phase, g_b(m) = D(m + b / r) for m in [-(2n-1), n-1], serves every entry.
// Its values are exact to rounding: sin(pi (m + b/r)) = (-1)^m sin(pi b / r)
// and the argument of cot is the rational (m r + b) / (2 n r), reduced in
// integers before the division.
//
// The contraction is VALU work in FP64 (the FP64 matrix units have the
// vector unit's peak on this chip): one lane per refined sample and four
// series per one-wavefront workgroup (a table set has only 10^4 refined
// samples per series, so the grid is made of many small workgroups to fill
// the chip), the series' native samples uniform across the workgroup (scalar
// loads), the two table reads per tap per lane coalesced within a phase and
// four taps in flight.  (Staging a phase's table in LDS, with one phase per
// workgroup, measured slower: 0.56 ms against 0.24 ms for the headline
// table set.)

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/rift_ile.h"

namespace {

constexpr int PG_BLOCK = 64;
constexpr int PG_S = 4;  // series per workgroup

// g[b][m + 2n - 1] = D(m + b / r), b < r, m in [-(2n-1), n-1].
__global__ void k_pregrid_table(int n, int r, double* __restrict__ g) {
  const int W = 3 * n - 1;
  const int64_t total = (int64_t)r * W;
  const int64_t Q = 2 * (int64_t)n * r;  // the period in units of 1/r samples
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(e / W);
    const int m = (int)(e - (int64_t)b * W) - (2 * n - 1);
    double v;
    if (b == 0) {
      v = (m == 0) ? 1.0 : 0.0;  // the nodes (m = -2n, the next multiple of L, is outside the range)
    } else {
      // u / L = p / Q with p = m r + b, reduced to (-Q, Q]
      int64_t p = (int64_t)m * r + b;
      p %= 2 * Q;
      if (p > Q) p -= 2 * Q;
      if (p <= -Q) p += 2 * Q;
      const double x = (double)p / (double)Q;
      const double sgn = (m & 1) ? -1.0 : 1.0;
      v = sgn * sinpi((double)b / (double)r) * cospi(x) / (sinpi(x) * (double)(2 * n));
    }
    g[e] = v;
  }
}

__global__ void __launch_bounds__(PG_BLOCK) k_pregrid(const double* __restrict__ q, int64_t S, int n, int r,
                                                      const double* __restrict__ g, double* __restrict__ fine) {
  const int64_t Nf = (int64_t)(n - 1) * r + 1;
  const int64_t j0 = (int64_t)blockIdx.x * PG_BLOCK + threadIdx.x;
  const bool live = j0 < Nf;
  const int64_t j = live ? j0 : Nf - 1;
  const int a = (int)(j / r), b = (int)(j - (int64_t)(j / r) * r);
  const int W = 3 * n - 1;
  const double* gb = g + (int64_t)b * W + (2 * n - 1);  // gb[m], m in [-(2n-1), n-1]
  const int64_t s0 = (int64_t)blockIdx.y * PG_S;
  const int ns = (int)std::min<int64_t>(PG_S, S - s0);
  double acc[2 * PG_S];
#pragma unroll
  for (int c = 0; c < 2 * PG_S; ++c) acc[c] = 0.0;
  const double* qs = q + 2 * s0 * (int64_t)n;
  int i = 0;
  for (; i + 4 <= n; i += 4) {
    double t[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) t[u] = gb[a - (i + u)] + gb[a + (i + u) + 1 - 2 * n];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int c = 0; c < PG_S; ++c) {
        if (c < ns) {
          acc[2 * c] = fma(t[u], qs[2 * ((int64_t)c * n + i + u)], acc[2 * c]);
          acc[2 * c + 1] = fma(t[u], qs[2 * ((int64_t)c * n + i + u) + 1], acc[2 * c + 1]);
        }
      }
  }
  for (; i < n; ++i) {
    const double t = gb[a - i] + gb[a + i + 1 - 2 * n];
#pragma unroll
    for (int c = 0; c < PG_S; ++c) {
      if (c < ns) {
        acc[2 * c] = fma(t, qs[2 * ((int64_t)c * n + i)], acc[2 * c]);
        acc[2 * c + 1] = fma(t, qs[2 * ((int64_t)c * n + i) + 1], acc[2 * c + 1]);
      }
    }
  }
  if (!live) return;
#pragma unroll
  for (int c = 0; c < PG_S; ++c) {
    if (c < ns) {
      double* o = fine + 2 * ((s0 + c) * Nf + j);
      o[0] = acc[2 * c];
      o[1] = acc[2 * c + 1];
    }
  }
}

}  // namespace

extern "C" int rift_ile_pregrid(const double* q, int64_t n_series, int32_t n, int32_t r, double* fine, void* stream) {
  if (n_series < 0 || n < 2 || r < 1 || r > 64) return RIFT_EINVAL;
  if ((int64_t)(n - 1) * r + 1 > ((int64_t)1 << 28) || n > (1 << 24)) return RIFT_EINVAL;
  if (n_series == 0) return RIFT_OK;
  if (!q || !fine || (((uintptr_t)q) & 7u) || (((uintptr_t)fine) & 7u)) return RIFT_EINVAL;
  const int64_t Nf = (int64_t)(n - 1) * r + 1;
  const int64_t gy = (n_series + PG_S - 1) / PG_S;
  if (gy > 65535) return RIFT_EUNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  const int64_t tab = (int64_t)r * (3 * n - 1);
  double* g = nullptr;
  if (hipMallocAsync((void**)&g, sizeof(double) * tab, st) != hipSuccess) return RIFT_ENOMEM;
  hipLaunchKernelGGL(k_pregrid_table, dim3((unsigned)std::min<int64_t>((tab + 255) / 256, 4096)), dim3(256), 0, st, n,
                     r, g);
  hipLaunchKernelGGL(k_pregrid, dim3((unsigned)((Nf + PG_BLOCK - 1) / PG_BLOCK), (unsigned)gy), dim3(PG_BLOCK), 0,
                     st, q, n_series, (int)n, (int)r, (const double*)g, fine);
  int rc = hipGetLastError() == hipSuccess ? RIFT_OK : RIFT_EDEVICE;
  if (hipFreeAsync(g, st) != hipSuccess && !rc) rc = RIFT_EDEVICE;
  return rc;
}
