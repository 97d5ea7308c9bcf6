// Evaluation kernels of the factored extrinsic likelihood (templates).  Each
// instance set is compiled in its own translation unit (inst.hip) and reached
// from the host code through the getters declared at the end of this file.
#pragma once

#include "ile_device.h"
#include "ile_grad.h"

namespace rift {

// ---------------------------------------------------------------------------
// Evaluation kernels
// ---------------------------------------------------------------------------
enum : int { MODE_LSE64 = 0, MODE_PASS32 = 1 };

struct TileArgs {
  const PointDesc* descs;
  const Tile* tiles;
  int32_t n_tiles;
  int32_t persistent;
  int32_t* counter;
  const double* theta;  // [7][N]
  const double* lnw;    // [N] or null
  int64_t N;
  double* lnL;          // [N] or null
  float* bnd;           // [N] (pass32)
  double* part;         // [n_tiles][2]: (max, sum) (lse64)
  double* tmax;         // [n_tiles]: max(lnL + lnw - bound) (pass32)
  // sorted mode: samples read from the records theta_aos[pos][8] (ra, dec,
  // psi, incl, phiref, tref, dist, int64 bits whose upper 48 hold the sample
  // index) and results
  // written to that sample index; the reductions then run in input order in
  // a separate pass
  const double* theta_aos;
};

// One tile: every sample's lnL (and bound), then a block reduction.
template <class R, int KT, int L, int MODE>
__device__ __forceinline__ void run_tile(const TileArgs& a, int tidx, MS* sh, double* shd, R* trig) {
  const Tile t = a.tiles[tidx];
  const PointDesc* P = a.descs + __builtin_amdgcn_readfirstlane(t.p);
  const RIFT_GLOBAL double* theta = as_global(a.theta);
  const RIFT_GLOBAL double* lnw = as_global(a.lnw);
  RIFT_GLOBAL double* lnL = as_global_w(a.lnL);
  MS acc;
  acc.m = -__builtin_inf();
  acc.s = 0.0;
  double tm = -__builtin_inf();
  const int64_t N = a.N;
  if (a.theta_aos) {
    const RIFT_GLOBAL double* aos = as_global(a.theta_aos);
    for (int o = threadIdx.x; o < t.cnt; o += blockDim.x) {
      const int64_t pos = t.s + o;
      const RIFT_GLOBAL double* th = aos + 8 * pos;
      const Eval e = eval_sample<R, KT, L, MODE == MODE_PASS32>(opaque(P), trig, blockDim.x, th[0], th[1],
                                                                th[2], th[3], th[4], th[5], th[6]);
      const int64_t i = (int64_t)__double_as_longlong(th[7]) >> 16;
      lnL[i] = e.lnL;
      if (MODE == MODE_PASS32) as_global_w(a.bnd)[i] = e.bound;
    }
    return;
  }
  for (int o = threadIdx.x; o < t.cnt; o += blockDim.x) {
    const int64_t i = t.s + o;
    const RIFT_GLOBAL double* th = theta + i;
    const Eval e = eval_sample<R, KT, L, MODE == MODE_PASS32>(opaque(P), trig, blockDim.x, th[0], th[N],
                                                              th[2 * N], th[3 * N], th[4 * N], th[5 * N],
                                                              th[6 * N]);
    const double w = lnw ? lnw[i] : 0.0;
    if (lnL) lnL[i] = e.lnL;
    if (MODE == MODE_LSE64) {
      acc = ms_push(acc, e.lnL + w);
    } else {
      as_global_w(a.bnd)[i] = e.bound;
      const double v = e.lnL + w - (double)e.bound;
      if (v == v) tm = fmax(tm, v);
    }
  }
  if (MODE == MODE_LSE64) {
    const MS r = ms_block(acc, sh);
    if (threadIdx.x == 0) {
      a.part[2 * tidx] = r.m;
      a.part[2 * tidx + 1] = r.s;
    }
  } else {
    tm = dmax_wave(tm);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) shd[threadIdx.x >> 6] = tm;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = shd[0];
      for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, shd[w]);
      a.tmax[tidx] = r;
    }
  }
}

// Class sets compiled into one kernel (bit 0: L=2, 1: L=3, 2: L=4, 3: L=8).
template <class R, int KT, int LSET, int MODE>
__device__ __forceinline__ void dispatch_tile(const TileArgs& a, int tidx, MS* sh, double* shd, R* trig) {
  const int L = __builtin_amdgcn_readfirstlane(as_const(a.descs)[as_const(a.tiles)[tidx].p].L);
  if ((LSET & 1) && L == 2) run_tile<R, KT, 2, MODE>(a, tidx, sh, shd, trig);
  else if ((LSET & 2) && L == 3) run_tile<R, KT, 3, MODE>(a, tidx, sh, shd, trig);
  else if ((LSET & 4) && L == 4) run_tile<R, KT, 4, MODE>(a, tidx, sh, shd, trig);
  else if ((LSET & 8) && L == 8) run_tile<R, KT, 8, MODE>(a, tidx, sh, shd, trig);
}

// Per-lane scratch column for cos/sin(n incl), n <= 2 L: 2 (2 L + 1) values.
__host__ __device__ constexpr int trig_rows(int lset) { return (lset & 8) ? 34 : ((lset & 4) ? 18 : ((lset & 2) ? 14 : 10)); }

// Persistent (work queue over tiles) or one block per tile.
template <class R, int KT, int LSET, int MODE>
__global__ void __launch_bounds__(512) k_tiles(TileArgs a) {
  __shared__ MS sh[8];
  __shared__ double shd[8];
  __shared__ int s_t;
  extern __shared__ __align__(16) unsigned char smem[];
  R* trig = reinterpret_cast<R*>(smem) + threadIdx.x;
  // one code path for both launch forms: the non-persistent form runs the
  // body once with its block index as the tile
  int t = blockIdx.x;
  for (;;) {
    if (a.persistent) {
      __syncthreads();
      if (threadIdx.x == 0) s_t = atomicAdd(a.counter, 1);
      __syncthreads();
      t = s_t;
    }
    if (t >= a.n_tiles) break;
    dispatch_tile<R, KT, LSET, MODE>(a, t, sh, shd, trig);
    if (!a.persistent) break;
  }
}

// FP64 recompute of the refine list of point blockIdx.y.
template <int KT, int L>
__device__ __forceinline__ void refine_point(const PointDesc* P, const double* theta, int64_t N,
                                             const int32_t* cnt, const int32_t* list, double* lnL,
                                             int p, double* trig) {
  const int c = as_const(cnt)[p];
  const int64_t s0 = as_const(P)->s0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < c; e += gridDim.x * blockDim.x) {
    const int64_t i = s0 + as_global(list)[s0 + e];
    const RIFT_GLOBAL double* th = as_global(theta) + i;
    const Eval r = eval_sample<double, KT, L, false>(opaque(P), trig, blockDim.x, th[0], th[N], th[2 * N],
                                                     th[3 * N], th[4 * N], th[5 * N], th[6 * N]);
    as_global_w(lnL)[i] = r.lnL;
  }
}

template <int KT, int LSET>
__global__ void __launch_bounds__(256) k_refine(const PointDesc* __restrict__ descs,
                                                const double* __restrict__ theta, int64_t N,
                                                const int32_t* __restrict__ cnt,
                                                const int32_t* __restrict__ list, double* lnL) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* trig = reinterpret_cast<double*>(smem) + threadIdx.x;
  const int p = blockIdx.y;
  const PointDesc* P = descs + p;
  const int L = __builtin_amdgcn_readfirstlane(as_const(P)->L);
  if ((LSET & 1) && L == 2) refine_point<KT, 2>(P, theta, N, cnt, list, lnL, p, trig);
  else if ((LSET & 2) && L == 3) refine_point<KT, 3>(P, theta, N, cnt, list, lnL, p, trig);
  else if ((LSET & 4) && L == 4) refine_point<KT, 4>(P, theta, N, cnt, list, lnL, p, trig);
  else if ((LSET & 8) && L == 8) refine_point<KT, 8>(P, theta, N, cnt, list, lnL, p, trig);
}

// Gradient: one lane per sample, grid-stride.
template <int KT, int L>
__global__ void __launch_bounds__(256) k_grad(const PointDesc* __restrict__ P,
                                              const double* __restrict__ theta, int64_t n,
                                              double* __restrict__ lnL, double* __restrict__ grad) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* trig = reinterpret_cast<double*>(smem) + threadIdx.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const RIFT_GLOBAL double* th = as_global(theta) + i;
    double g[7];
    const double l = eval_grad<KT, L>(opaque(P), trig, blockDim.x, th[0], th[n], th[2 * n], th[3 * n],
                                      th[4 * n], th[5 * n], th[6 * n], g);
    if (lnL) as_global_w(lnL)[i] = l;
#pragma unroll
    for (int a = 0; a < 7; ++a) as_global_w(grad)[a * n + i] = g[a];
  }
}


typedef void (*tile_fn)(TileArgs);
typedef void (*refine_fn)(const PointDesc*, const double*, int64_t, const int32_t*, const int32_t*, double*);
typedef void (*grad_fn)(const PointDesc*, const double*, int64_t, double*, double*);

// Getters (one translation unit per detector class and kernel kind).
#define RIFT_DECL_GETTERS(KT)                        \
  tile_fn get_tiles64_kt##KT(int lset);              \
  tile_fn get_tiles32_kt##KT(int lset);              \
  refine_fn get_refine_kt##KT(int lset);             \
  grad_fn get_grad_kt##KT(int L);
RIFT_DECL_GETTERS(2)
RIFT_DECL_GETTERS(3)
RIFT_DECL_GETTERS(5)
RIFT_DECL_GETTERS(8)
#undef RIFT_DECL_GETTERS

}  // namespace rift
