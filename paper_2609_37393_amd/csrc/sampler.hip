// Building block of gradient-based samplers on the likelihood's gradient
// (Sec. "Sampling the differentiable extrinsic likelihood"): the position
// update (drift) of a leapfrog step in the sampler's coordinates
// (ra, dec, psi, cos incl, phiref, tref, ln dist), theta += step * p, with a
// reflecting boundary on cos incl: a state that leaves [-1, 1] is folded back
// (a triangle wave of period 4) and its momentum in cos incl changes sign
// after an odd number of folds, which keeps the dynamics reversible and
// volume-preserving on the bounded coordinate.
#include <hip/hip_runtime.h>

#include <cmath>

#include "../../include/rift_ile.h"

namespace {

struct Step7 {
  double s[7];
};

__global__ void k_drift(int64_t n, double* __restrict__ theta, double* __restrict__ p, Step7 step) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      double q = theta[a * n + i] + step.s[a] * p[a * n + i];
      if (a == 3 && !(fabs(q) <= 1.0) && q == q && fabs(q) < 1.0e300) {
        // fold onto [-1, 1]: c' = 1 - |((c + 1) mod 4) - 2|
        double r = fmod(q + 1.0, 4.0);
        if (r < 0.0) r += 4.0;
        q = 1.0 - fabs(r - 2.0);
        if (r > 2.0) p[a * n + i] = -p[a * n + i];
      }
      theta[a * n + i] = q;
    }
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
