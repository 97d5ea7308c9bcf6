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
// MODE_LSE64: FP64 lnL and the tile's (max, sum); MODE_PASS32: the FP32 pass
// of the mixed path; MODE_DMARG64: FP64, the likelihood marginalised over
// distance (Eq. (ap:dgh)) in place of lnL, and its tile (max, sum);
// MODE_TMARG64: FP64, the likelihood marginalised over geocentric time by the
// fixed-spacing rule (Eq. (ap:tfixed)) in place of lnL, and its tile pair.
// MODE_PMARG64: FP64, the likelihood marginalised over polarisation
// (Eqs. (ap:psiexp), (ap:psilaplace)) in place of lnL, and its tile pair.
// MODE_TBAND64: FP64, the data pass of the band-limited time rule
// (Eq. (ap:tband)): x kappa at every node into `kap`, the time-independent
// remainder in place of lnL, and no reduction (a later pass finishes the
// rule per sample and reduces).
// MODE_ERAI64: FP64, the data pass of the joint phiref / psi marginal by
// exact reconstruction: the angular coefficients at their sampling angles
// into `ang`, NaN or 0 (poisoned or not) in place of lnL, no reduction.
enum : int { MODE_LSE64 = 0, MODE_PASS32 = 1, MODE_DMARG64 = 2, MODE_TMARG64 = 3, MODE_PMARG64 = 4,
             MODE_TBAND64 = 5, MODE_ERAI64 = 6 };
constexpr bool mode_reduces(int mode) { return mode != MODE_TBAND64 && mode != MODE_ERAI64; }

struct TileArgs {
  const PointDesc* descs;
  const Tile* tiles;
  int32_t n_tiles;
  int32_t persistent;
  int32_t* counter;  // [0]: next tile, [1]: finished blocks (persistent form; both 0 at launch)
  const double* theta;  // [7][N]
  const double* lnw;    // [N] or null
  int64_t N;
  double* lnL;          // [N] or null
  float* bnd;           // [N] (pass32)
  double* part;         // [n_tiles][2]: (max, sum) (lse64)
  double* tmax;         // [n_tiles]: max(lnL + lnw - bound) (pass32)
  int32_t* cnt;         // [n_points]: refine-list lengths, zeroed here (pass32)
  // sorted mode: samples read from the records theta_aos[pos][8] (ra, dec,
  // psi, incl, phiref, tref, dist, int64 bits whose upper 48 hold the sample
  // index) and results
  // written to that sample index; the reductions then run in input order in
  // a separate pass
  const double* theta_aos;
  DistRule dm;  // MODE_DMARG64: the distance rule and prior
  TimeRule tm;  // MODE_TMARG64, MODE_TBAND64: the time nodes
  PsiRule pm;   // MODE_PMARG64: the polarisation rule
  double* kap;  // MODE_TBAND64: [tm.n][N], x kappa at the nodes
  AngleRule am; // MODE_ERAI64: the sampling angles
  double* ang;  // MODE_ERAI64: [2 nd + 3 nq][N], the angular coefficients
};

// One tile: every sample's lnL (and bound), then a block reduction.
// The sample loops run whole wavefronts (the data term reads cooperatively):
// lanes past the end of the tile evaluate its last sample and drop the result.
template <class R, int KT, int L, int MODE>
__device__ __forceinline__ void run_tile(const TileArgs& a, int tidx, MS* sh, double* shd, R* trig,
                                         RIFT_LDS unsigned char* stage) {
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
  // the point's refine list starts empty for the selection that follows
  if (MODE == MODE_PASS32 && threadIdx.x == 0 && t.s == as_const(P)->s0) a.cnt[t.p] = 0;
  const int wbase = (int)(threadIdx.x & ~63u);
  const int lane = (int)threadIdx.x - wbase;
  if (a.theta_aos) {
    const RIFT_GLOBAL double* aos = as_global(a.theta_aos);
    for (int ob = wbase; ob < t.cnt; ob += blockDim.x) {
      const int o = ob + lane;
      const bool live = o < t.cnt;
      const int64_t pos = t.s + (live ? o : t.cnt - 1);
      const RIFT_GLOBAL double* th = aos + 8 * pos;
      const int64_t i = (int64_t)__double_as_longlong(th[7]) >> 16;
      Eval e;
      if constexpr (MODE == MODE_TBAND64) {
        e.lnL = eval_tkappa<R, KT, L>(opaque(P), trig, blockDim.x, stage, th[0], th[1], th[2], th[3], th[4], th[6],
                                      a.tm, as_global_w(a.kap), N, i, live);
      } else if constexpr (MODE == MODE_ERAI64) {
        e.lnL = eval_erai<R, KT, L>(opaque(P), trig, blockDim.x, stage, th[0], th[1], th[2], th[3], th[4], th[5],
                                    th[6], a.am, as_global_w(a.ang), N, i, live)
                    ? __builtin_nan("")
                    : 0.0;
      } else if constexpr (MODE == MODE_DMARG64) {
        const Terms tm = eval_terms<R, KT, L>(opaque(P), trig, blockDim.x, stage, th[0], th[1], th[2], th[3],
                                              th[4], th[5]);
        e.lnL = dist_marginal(a.dm, as_const(P)->d_ref, tm);
      } else if constexpr (MODE == MODE_TMARG64) {
        e.lnL = eval_tmarg<R, KT, L>(opaque(P), trig, blockDim.x, stage, th[0], th[1], th[2], th[3], th[4], th[6],
                                     a.tm);
      } else if constexpr (MODE == MODE_PMARG64) {
        e.lnL = eval_pmarg<R, KT, L>(opaque(P), trig, blockDim.x, stage, th[0], th[1], th[2], th[3], th[4], th[5],
                                     th[6], a.pm);
      } else {
        e = eval_sample<R, KT, L, MODE == MODE_PASS32>(opaque(P), trig, blockDim.x, stage, th[0], th[1], th[2],
                                                       th[3], th[4], th[5], th[6]);
      }
      if (live) {
        lnL[i] = e.lnL;
        if (MODE == MODE_PASS32) as_global_w(a.bnd)[i] = e.bound;
      }
    }
    return;
  }
  for (int ob = wbase; ob < t.cnt; ob += blockDim.x) {
    const int o = ob + lane;
    const bool live = o < t.cnt;
    const int64_t i = t.s + (live ? o : t.cnt - 1);
    const RIFT_GLOBAL double* th = theta + i;
    Eval e;
    if constexpr (MODE == MODE_TBAND64) {
      e.lnL = eval_tkappa<R, KT, L>(opaque(P), trig, blockDim.x, stage, th[0], th[N], th[2 * N], th[3 * N],
                                    th[4 * N], th[6 * N], a.tm, as_global_w(a.kap), N, i, live);
    } else if constexpr (MODE == MODE_ERAI64) {
      e.lnL = eval_erai<R, KT, L>(opaque(P), trig, blockDim.x, stage, th[0], th[N], th[2 * N], th[3 * N],
                                  th[4 * N], th[5 * N], th[6 * N], a.am, as_global_w(a.ang), N, i, live)
                  ? __builtin_nan("")
                  : 0.0;
    } else if constexpr (MODE == MODE_DMARG64) {
      const Terms tm = eval_terms<R, KT, L>(opaque(P), trig, blockDim.x, stage, th[0], th[N], th[2 * N],
                                            th[3 * N], th[4 * N], th[5 * N]);
      e.lnL = dist_marginal(a.dm, as_const(P)->d_ref, tm);
    } else if constexpr (MODE == MODE_TMARG64) {
      e.lnL = eval_tmarg<R, KT, L>(opaque(P), trig, blockDim.x, stage, th[0], th[N], th[2 * N], th[3 * N],
                                   th[4 * N], th[6 * N], a.tm);
    } else if constexpr (MODE == MODE_PMARG64) {
      e.lnL = eval_pmarg<R, KT, L>(opaque(P), trig, blockDim.x, stage, th[0], th[N], th[2 * N], th[3 * N],
                                   th[4 * N], th[5 * N], th[6 * N], a.pm);
    } else {
      e = eval_sample<R, KT, L, MODE == MODE_PASS32>(opaque(P), trig, blockDim.x, stage, th[0], th[N],
                                                     th[2 * N], th[3 * N], th[4 * N], th[5 * N], th[6 * N]);
    }
    if (!live) continue;
    const double w = lnw ? lnw[i] : 0.0;
    if (lnL) lnL[i] = e.lnL;
    if (!mode_reduces(MODE)) continue;
    if (MODE != MODE_PASS32) {
      acc = ms_push(acc, e.lnL + w);
    } else {
      as_global_w(a.bnd)[i] = e.bound;
      const double v = e.lnL + w - (double)e.bound;
      if (v == v) tm = fmax(tm, v);
    }
  }
  if (!mode_reduces(MODE)) return;
  if (MODE != MODE_PASS32) {
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
__device__ __forceinline__ void dispatch_tile(const TileArgs& a, int tidx, MS* sh, double* shd, R* trig,
                                              RIFT_LDS unsigned char* stage) {
  const int L = __builtin_amdgcn_readfirstlane(as_const(a.descs)[as_const(a.tiles)[tidx].p].L);
  if ((LSET & 1) && L == 2) run_tile<R, KT, 2, MODE>(a, tidx, sh, shd, trig, stage);
  else if ((LSET & 2) && L == 3) run_tile<R, KT, 3, MODE>(a, tidx, sh, shd, trig, stage);
  else if ((LSET & 4) && L == 4) run_tile<R, KT, 4, MODE>(a, tidx, sh, shd, trig, stage);
  else if ((LSET & 8) && L == 8) run_tile<R, KT, 8, MODE>(a, tidx, sh, shd, trig, stage);
}

// Per-lane scratch column for cos/sin(n incl), n <= 2 L: 2 (2 L + 1) values.
__host__ __device__ constexpr int trig_rows(int lset) { return (lset & 8) ? 34 : ((lset & 4) ? 18 : ((lset & 2) ? 14 : 10)); }

// Persistent (work queue over tiles) or one block per tile.
template <class R, int KT, int LSET, int MODE>
__global__ void __launch_bounds__(512) k_tiles(TileArgs a) {
  __shared__ MS sh[8];
  __shared__ double shd[8];
  __shared__ int s_t;
  // dynamic LDS: the wavefronts' staging buffers, then (l <= 8 class) the
  // per-lane trig columns
  extern __shared__ __align__(16) unsigned char smem[];
  RIFT_LDS unsigned char* stage = (RIFT_LDS unsigned char*)smem + (threadIdx.x >> 6) * STAGE_WAVE;
  R* trig = reinterpret_cast<R*>(smem + (blockDim.x >> 6) * STAGE_WAVE) + threadIdx.x;
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
    dispatch_tile<R, KT, LSET, MODE>(a, t, sh, shd, trig, stage);
    if (!a.persistent) break;
  }
  // persistent form: the last block to finish leaves the queue at 0 for the
  // next launch (every other block has taken its last tile by then)
  if (a.persistent && threadIdx.x == 0) {
    const int done = atomicAdd(a.counter + 1, 1);
    if (done == (int)gridDim.x - 1) {
      atomicExch(a.counter, 0);
      atomicExch(a.counter + 1, 0);
    }
  }
}

// One sample evaluated by a whole wavefront (FP64): the same definition as
// eval_sample, split over the lanes for latency.  Lanes below 2 L + 1 fill
// the wavefront's table of cos/sin(n incl) and cos/sin(q phi), n, q <= 2 L;
// lanes below K fill detector k's antenna factor, norm weights and stencil.
// Then lane l takes the (detector, mode) pairs l, l+64, ... of the data term
// and the coefficients l, l+64, ... of the model-norm contraction; the shares
// meet in wavefront sums.  tab: this wavefront's LDS scratch of
// WIDE_TAB(L, KT) doubles.  Every lane returns the sample's lnL.
#define WIDE_TAB(L, KT) (4 * (2 * (L) + 1) + 8 * (KT))
template <int KT, int L>
__device__ __forceinline__ double eval_wide(PDesc P, double ra, double dec, double psi, double incl,
                                            double phi, double tref, double dist, double* tab) {
  constexpr int NI = 2 * L;
  constexpr int NY = L + 1;
  const int lane = threadIdx.x & 63;
  const int K = P->K, M = P->M, n_t = P->n_t;
  double* ctab = tab;
  double* stab = tab + (NI + 1);
  double* cq = tab + 2 * (NI + 1);
  double* sq = tab + 3 * (NI + 1);
  double* det = tab + 4 * (NI + 1);  // per detector: fp, fx, f2, g2r, g2i, row, s, bad
  if (lane <= NI) {
    double s, c;
    sincos((double)lane * incl, &s, &c);
    ctab[lane] = c;
    stab[lane] = s;
    sincos((double)lane * phi, &s, &c);
    cq[lane] = c;
    sq[lane] = s;
  }
  if (lane < K) {
    const int k = lane;
    double sg, cg, sd, cd, sp, cp;
    sincos(P->gmst - ra, &sg, &cg);
    sincos(dec, &sd, &cd);
    sincos(psi, &sp, &cp);
    const double N0 = cd * cg, N1 = -cd * sg, N2 = sd;
    const double ed0 = -sd * cg, ed1 = sd * sg, ed2 = cd;
    const double X0 = -cp * sg + sp * ed0, X1 = -cp * cg + sp * ed1, X2 = sp * ed2;
    const double Y0 = sp * sg + cp * ed0, Y1 = sp * cg + cp * ed1, Y2 = cp * ed2;
    const double ep[6] = {X0 * X0 - Y0 * Y0, X1 * X1 - Y1 * Y1, X2 * X2 - Y2 * Y2,
                          X0 * X1 - Y0 * Y1, X0 * X2 - Y0 * Y2, X1 * X2 - Y1 * Y2};
    const double ex[6] = {2 * X0 * Y0, 2 * X1 * Y1, 2 * X2 * Y2,
                          X0 * Y1 + Y0 * X1, X0 * Y2 + Y0 * X2, X1 * Y2 + Y1 * X2};
    double fp = 0.0, fx = 0.0;
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      fp += P->dten[k][a] * ep[a];
      fx += P->dten[k][a] * ex[a];
    }
    const double tk = tref - (P->rpos[k][0] * N0 + P->rpos[k][1] * N1 + P->rpos[k][2] * N2);
    double u = (tk - P->t0) * P->inv_dt;
    const double bad = stencil_u(u, n_t) ? 0.0 : 1.0;
    const double jf = floor(u);
    int j0 = (int)jf - 1;
    j0 = j0 < -QPAD ? -QPAD : (j0 > n_t ? n_t : j0);
    double* dk = det + 8 * k;
    dk[0] = fp;
    dk[1] = fx;
    dk[2] = fp * fp + fx * fx;
    dk[3] = fp * fp - fx * fx;
    dk[4] = 2 * fp * fx;
    dk[5] = (double)(j0 + QPAD);
    dk[6] = u - jf;
    dk[7] = bad;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // data term: pairs (k, i)
  const RIFT_GLOBAL double* Q = as_global(P->Q64);
  const int64_t ntp = n_t + 2 * QPAD;
  const int NGR = q_groups(M, QW64);
  double data = 0.0;
  for (int pr = lane; pr < K * M; pr += 64) {
    const int k = pr / M, i = pr % M;
    const double* dk = det + 8 * k;
    double w[4];
    lagrange4(dk[6], w);
    const RIFT_GLOBAL double* q =
        Q + 2 * ((((int64_t)k * NGR + i / QW64) * ntp + (int64_t)dk[5]) * QW64 + i % QW64);
    double qx = 0.0, qy = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      qx += w[j] * q[2 * QW64 * j];
      qy += w[j] * q[2 * QW64 * j + 1];
    }
    // Y_i = d_i(incl) e^{i m_i phi}
    const int m = P->m[i];
    double d = 0.0;
    if (P->odd[i]) {
      for (int n = 1; n < NY; ++n) d += P->ycoef[i][n] * stab[n];
    } else {
      for (int n = 0; n < NY; ++n) d += P->ycoef[i][n] * ctab[n];
    }
    const int am = m < 0 ? -m : m;
    const double yx = d * cq[am], yy = d * (m < 0 ? -sq[am] : sq[am]);
    // Re[conj(F) conj(Y) Qhat]
    data += dk[0] * (yx * qx + yy * qy) + dk[1] * (yx * qy - yy * qx);
  }
  // model-norm term: coefficient j = b * 3 KT + 3 k + c, weights |F|^2,
  // Re F^2, Im F^2 for c = 0, 1, 2; basis rows over the lanes, each row's
  // 3 KT coefficients read together
  double quad = 0.0;
  const RIFT_GLOBAL double* C = as_global(P->C64);
  constexpr int W = 3 * KT;
  for (int b = lane; b < Cls<L>::B; b += 64) {
    const int rb = basis_row<L>(b);
    const int kind = rb & 15, n = (rb >> 4) & 255, qq = rb >> 12;
    double beta = (kind >= 3) ? stab[n] : ctab[n];
    if (kind != 0) beta *= ((kind & 1) == 1) ? cq[qq] : sq[qq];
    const RIFT_GLOBAL double* cr = C + (int64_t)b * W;
    double cv[W];
#pragma unroll
    for (int col = 0; col < W; ++col) cv[col] = cr[col];
#pragma unroll
    for (int col = 0; col < W; ++col) {
      const int k = col / 3, c = col - 3 * k;
      const double wt = (k < K) ? det[8 * k + 2 + c] : 0.0;
      quad += cv[col] * beta * wt;
    }
  }
  double bad = (lane < K) ? det[8 * lane + 7] : 0.0;
  data = dsum_wave(data);
  quad = dsum_wave(quad);
  bad = dsum_wave(bad);
  const double x = P->d_ref / dist;
  double l = x * data - x * x * quad;
  if (bad != 0.0) l = __builtin_nan("");
  return l;
}

// FP64 recompute of the refine list of point blockIdx.y: a whole wavefront
// per sample while the list is short (latency), one lane per sample when it
// is long (throughput).
template <int KT, int L>
__device__ __forceinline__ void refine_point(const PointDesc* P, const double* theta, int64_t N,
                                             const int32_t* cnt, const int32_t* list, double* lnL,
                                             int p, double* trig, double* wtab, RIFT_LDS unsigned char* stage) {
  const int c = as_const(cnt)[p];
  const int64_t s0 = as_const(P)->s0;
  const int waves = gridDim.x * (blockDim.x >> 6);
  if (c <= waves) {
    const int wv = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    double* tab = wtab + (threadIdx.x >> 6) * WIDE_TAB(L, KT);
    for (int e = wv; e < c; e += waves) {
      const int64_t i = s0 + as_global(list)[s0 + e];
      const RIFT_GLOBAL double* th = as_global(theta) + i;
      const double l = eval_wide<KT, L>(opaque(P), th[0], th[N], th[2 * N], th[3 * N], th[4 * N], th[5 * N],
                                        th[6 * N], tab);
      if ((threadIdx.x & 63) == 0) as_global_w(lnL)[i] = l;
    }
    return;
  }
  // whole wavefronts (cooperative reads): lanes past the end repeat the last entry
  const int lane = (int)(threadIdx.x & 63u);
  for (int eb = blockIdx.x * blockDim.x + (int)(threadIdx.x & ~63u); eb < c; eb += gridDim.x * blockDim.x) {
    const int e = eb + lane < c ? eb + lane : c - 1;
    const int64_t i = s0 + as_global(list)[s0 + e];
    const RIFT_GLOBAL double* th = as_global(theta) + i;
    const Eval r = eval_sample<double, KT, L, false>(opaque(P), trig, blockDim.x, stage, th[0], th[N],
                                                     th[2 * N], th[3 * N], th[4 * N], th[5 * N], th[6 * N]);
    if (eb + lane < c) as_global_w(lnL)[i] = r.lnL;
  }
}

template <int KT, int LSET>
__global__ void __launch_bounds__(256) k_refine(const PointDesc* __restrict__ descs,
                                                const double* __restrict__ theta, int64_t N,
                                                const int32_t* __restrict__ cnt,
                                                const int32_t* __restrict__ list, double* lnL) {
  // dynamic LDS: staging buffers (4 wavefronts), then the trig columns
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double wtab[4 * WIDE_TAB(8, KT)];  // per wavefront, for the largest class
  RIFT_LDS unsigned char* stage = (RIFT_LDS unsigned char*)smem + (threadIdx.x >> 6) * STAGE_WAVE;
  double* trig = reinterpret_cast<double*>(smem + 4 * STAGE_WAVE) + threadIdx.x;
  const int p = blockIdx.y;
  const PointDesc* P = descs + p;
  const int L = __builtin_amdgcn_readfirstlane(as_const(P)->L);
  if ((LSET & 1) && L == 2) refine_point<KT, 2>(P, theta, N, cnt, list, lnL, p, trig, wtab, stage);
  else if ((LSET & 2) && L == 3) refine_point<KT, 3>(P, theta, N, cnt, list, lnL, p, trig, wtab, stage);
  else if ((LSET & 4) && L == 4) refine_point<KT, 4>(P, theta, N, cnt, list, lnL, p, trig, wtab, stage);
  else if ((LSET & 8) && L == 8) refine_point<KT, 8>(P, theta, N, cnt, list, lnL, p, trig, wtab, stage);
}

// Gradient: one lane per sample, grid-stride.
template <int KT, int L, bool MARG>
__device__ __forceinline__ void grad_lanes(const PointDesc* __restrict__ P, const double* __restrict__ theta,
                                           int64_t n, double* __restrict__ lnL, double* __restrict__ grad,
                                           int coords, const DistRule* dm) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* trig = reinterpret_cast<double*>(smem) + threadIdx.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const RIFT_GLOBAL double* th = as_global(theta) + i;
    const double c3 = th[3 * n];
    double incl = c3, dist = th[6 * n];
    const bool ok = theta_coords(coords, incl, dist);
    double g[7];
    double l = eval_grad<KT, L, MARG>(opaque(P), trig, blockDim.x, th[0], th[n], th[2 * n], incl, th[4 * n],
                                      th[5 * n], dist, g, dm);
    grad_coords(coords, c3, dist, g[3], g[6]);
    if (!ok) {
      l = __builtin_nan("");
#pragma unroll
      for (int a = 0; a < 7; ++a) g[a] = l;
    }
    if (lnL) as_global_w(lnL)[i] = l;
#pragma unroll
    for (int a = 0; a < 7; ++a) as_global_w(grad)[a * n + i] = g[a];
  }
}

template <int KT, int L>
__global__ void __launch_bounds__(256) k_grad(const PointDesc* __restrict__ P,
                                              const double* __restrict__ theta, int64_t n,
                                              double* __restrict__ lnL, double* __restrict__ grad,
                                              int coords) {
  grad_lanes<KT, L, false>(P, theta, n, lnL, grad, coords, nullptr);
}

// The same for the likelihood marginalised over distance under the rule `dm`
// (ln L_d and its gradient; row 6 of theta is not used).
template <int KT, int L>
__global__ void __launch_bounds__(256) k_grad_dm(const PointDesc* __restrict__ P,
                                                 const double* __restrict__ theta, int64_t n,
                                                 double* __restrict__ lnL, double* __restrict__ grad,
                                                 int coords, DistRule dm) {
  grad_lanes<KT, L, true>(P, theta, n, lnL, grad, coords, &dm);
}


// Gradient, a group of GRAD_G lanes per sample (batches too small to fill the
// GPU one lane per sample).  A wavefront holds 64 / GRAD_G samples; groups
// past the end repeat the last sample and drop it.  Lanes 0..6 of a group
// write the seven components.
constexpr int GRAD_G = 16;
template <int KT, int L, bool MARG>
__device__ __forceinline__ void grad_groups(const PointDesc* __restrict__ P, const double* __restrict__ theta,
                                            int64_t n, double* __restrict__ lnL, double* __restrict__ grad,
                                            int coords, const DistRule* dm) {
  constexpr int SPW = 64 / GRAD_G;  // samples per wavefront
  __shared__ double tabs[4 * SPW * GRAD_TAB(L, KT)];
  const int lg = (int)(threadIdx.x & (GRAD_G - 1));
  const int gw = (int)((threadIdx.x & 63u) / GRAD_G);
  double* tab = tabs + ((threadIdx.x >> 6) * SPW + gw) * GRAD_TAB(L, KT);
  const int64_t per_launch = (int64_t)gridDim.x * (blockDim.x >> 6) * SPW;
  for (int64_t ib = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * SPW; ib < n;
       ib += per_launch) {
    const bool live = ib + gw < n;
    const int64_t i = live ? ib + gw : n - 1;
    const RIFT_GLOBAL double* th = as_global(theta) + i;
    const double c3 = th[3 * n];
    double incl = c3, dist = th[6 * n];
    const bool ok = theta_coords(coords, incl, dist);
    double g[7];
    double l = eval_grad_group<KT, L, GRAD_G, MARG>(opaque(P), th[0], th[n], th[2 * n], incl, th[4 * n],
                                                    th[5 * n], dist, tab, g, dm);
    grad_coords(coords, c3, dist, g[3], g[6]);
    if (!ok) {
      l = __builtin_nan("");
#pragma unroll
      for (int a = 0; a < 7; ++a) g[a] = l;
    }
    if (live) {
      if (lg == 0 && lnL) as_global_w(lnL)[i] = l;
      double v = g[0];
#pragma unroll
      for (int a = 1; a < 7; ++a) v = (lg == a) ? g[a] : v;
      if (lg < 7) as_global_w(grad)[lg * n + i] = v;
    }
  }
}

template <int KT, int L>
__global__ void __launch_bounds__(256) k_grad_wide(const PointDesc* __restrict__ P,
                                                   const double* __restrict__ theta, int64_t n,
                                                   double* __restrict__ lnL, double* __restrict__ grad,
                                                   int coords) {
  grad_groups<KT, L, false>(P, theta, n, lnL, grad, coords, nullptr);
}

template <int KT, int L>
__global__ void __launch_bounds__(256) k_grad_wide_dm(const PointDesc* __restrict__ P,
                                                      const double* __restrict__ theta, int64_t n,
                                                      double* __restrict__ lnL, double* __restrict__ grad,
                                                      int coords, DistRule dm) {
  grad_groups<KT, L, true>(P, theta, n, lnL, grad, coords, &dm);
}

typedef void (*tile_fn)(TileArgs);
typedef void (*refine_fn)(const PointDesc*, const double*, int64_t, const int32_t*, const int32_t*, double*);
typedef void (*grad_fn)(const PointDesc*, const double*, int64_t, double*, double*, int);
typedef void (*grad_dm_fn)(const PointDesc*, const double*, int64_t, double*, double*, int, DistRule);

// Getters (one translation unit per detector class and kernel kind).
#define RIFT_DECL_GETTERS(KT)                        \
  tile_fn get_tiles64_kt##KT(int lset);              \
  tile_fn get_tiles32_kt##KT(int lset);              \
  tile_fn get_tilesdm_kt##KT(int lset);              \
  tile_fn get_tilestm_kt##KT(int lset);              \
  tile_fn get_tilespm_kt##KT(int lset);              \
  tile_fn get_tilestb_kt##KT(int lset);              \
  tile_fn get_tilesea_kt##KT(int lset);              \
  refine_fn get_refine_kt##KT(int lset);             \
  grad_fn get_grad_kt##KT(int L);                   \
  grad_fn get_gradw_kt##KT(int L);                  \
  grad_dm_fn get_graddm_kt##KT(int L);              \
  grad_dm_fn get_gradwdm_kt##KT(int L);
RIFT_DECL_GETTERS(2)
RIFT_DECL_GETTERS(3)
RIFT_DECL_GETTERS(5)
RIFT_DECL_GETTERS(8)
#undef RIFT_DECL_GETTERS

}  // namespace rift
