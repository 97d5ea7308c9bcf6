// Instances of the evaluation kernels for one detector class RIFT_KT and one
// kernel kind RIFT_KIND (0: FP64 tiles, 1: FP32 tiles, 2: FP64 refine,
// 3: gradient, a lane or a group of lanes per sample, 4: FP64 tiles of the
// distance marginal, 5: FP64 tiles of the time marginal, 6: FP64 tiles of
// the polarisation marginal, 7: FP64 data pass of the band-limited time
// rule, 8: FP64 data pass of the joint phiref / psi marginal).  The build compiles
// this file once per (class, kind) so the instances build in parallel.
#include "ile_kernels.h"

#if !defined(RIFT_KT) || !defined(RIFT_KIND)
#error "RIFT_KT and RIFT_KIND must be defined"
#endif

#define RIFT_CAT_(a, b) a##b
#define RIFT_CAT(a, b) RIFT_CAT_(a, b)

namespace rift {

// Mode-class sets: 1 (l<=2), 2 (l=3), 4 (l=4), 8 (l<=8), 7 (l<=4 mixed).
#if RIFT_KIND == 0 || RIFT_KIND == 1 || RIFT_KIND == 4 || RIFT_KIND == 5 || RIFT_KIND == 6 || RIFT_KIND == 7 || \
    RIFT_KIND == 8
#if RIFT_KIND == 0
#define RIFT_R double
#define RIFT_MODE MODE_LSE64
#define RIFT_NAME RIFT_CAT(get_tiles64_kt, RIFT_KT)
#elif RIFT_KIND == 4
#define RIFT_R double
#define RIFT_MODE MODE_DMARG64
#define RIFT_NAME RIFT_CAT(get_tilesdm_kt, RIFT_KT)
#elif RIFT_KIND == 5
#define RIFT_R double
#define RIFT_MODE MODE_TMARG64
#define RIFT_NAME RIFT_CAT(get_tilestm_kt, RIFT_KT)
#elif RIFT_KIND == 6
#define RIFT_R double
#define RIFT_MODE MODE_PMARG64
#define RIFT_NAME RIFT_CAT(get_tilespm_kt, RIFT_KT)
#elif RIFT_KIND == 7
#define RIFT_R double
#define RIFT_MODE MODE_TBAND64
#define RIFT_NAME RIFT_CAT(get_tilestb_kt, RIFT_KT)
#elif RIFT_KIND == 8
#define RIFT_R double
#define RIFT_MODE MODE_ERAI64
#define RIFT_NAME RIFT_CAT(get_tilesea_kt, RIFT_KT)
#else
#define RIFT_R float
#define RIFT_MODE MODE_PASS32
#define RIFT_NAME RIFT_CAT(get_tiles32_kt, RIFT_KT)
#endif
tile_fn RIFT_NAME(int lset) {
  switch (lset) {
    case 1: return k_tiles<RIFT_R, RIFT_KT, 1, RIFT_MODE>;
    case 2: return k_tiles<RIFT_R, RIFT_KT, 2, RIFT_MODE>;
    case 4: return k_tiles<RIFT_R, RIFT_KT, 4, RIFT_MODE>;
    case 7: return k_tiles<RIFT_R, RIFT_KT, 7, RIFT_MODE>;
    case 8: return k_tiles<RIFT_R, RIFT_KT, 8, RIFT_MODE>;
    default: return nullptr;
  }
}
#elif RIFT_KIND == 2
refine_fn RIFT_CAT(get_refine_kt, RIFT_KT)(int lset) {
  switch (lset) {
    case 1: return k_refine<RIFT_KT, 1>;
    case 2: return k_refine<RIFT_KT, 2>;
    case 4: return k_refine<RIFT_KT, 4>;
    case 7: return k_refine<RIFT_KT, 7>;
    case 8: return k_refine<RIFT_KT, 8>;
    default: return nullptr;
  }
}
#elif RIFT_KIND == 3
grad_fn RIFT_CAT(get_grad_kt, RIFT_KT)(int L) {
  switch (L) {
    case 2: return k_grad<RIFT_KT, 2>;
    case 3: return k_grad<RIFT_KT, 3>;
    case 4: return k_grad<RIFT_KT, 4>;
    case 8: return k_grad<RIFT_KT, 8>;
    default: return nullptr;
  }
}
grad_fn RIFT_CAT(get_gradw_kt, RIFT_KT)(int L) {
  switch (L) {
    case 2: return k_grad_wide<RIFT_KT, 2>;
    case 3: return k_grad_wide<RIFT_KT, 3>;
    case 4: return k_grad_wide<RIFT_KT, 4>;
    case 8: return k_grad_wide<RIFT_KT, 8>;
    default: return nullptr;
  }
}
grad_dm_fn RIFT_CAT(get_graddm_kt, RIFT_KT)(int L) {
  switch (L) {
    case 2: return k_grad_dm<RIFT_KT, 2>;
    case 3: return k_grad_dm<RIFT_KT, 3>;
    case 4: return k_grad_dm<RIFT_KT, 4>;
    case 8: return k_grad_dm<RIFT_KT, 8>;
    default: return nullptr;
  }
}
grad_dm_fn RIFT_CAT(get_gradwdm_kt, RIFT_KT)(int L) {
  switch (L) {
    case 2: return k_grad_wide_dm<RIFT_KT, 2>;
    case 3: return k_grad_wide_dm<RIFT_KT, 3>;
    case 4: return k_grad_wide_dm<RIFT_KT, 4>;
    case 8: return k_grad_wide_dm<RIFT_KT, 8>;
    default: return nullptr;
  }
}
#endif

}  // namespace rift
