// The separable form's phi transforms in reduced precision: the FP64 tile
// engine (yyg_tile.h) with its LDS stages converted on the way in, to FP32
// (kGemmLpF32) or to three BF16 parts (kGemmLpBF3), FP32-accumulating 16x16
// MFMAs and an FP64 flush after every 16-wide stage.  The density, the
// coefficients and the bases stay FP64 in memory, so these kernels move the
// same bytes as the FP64 ones and spend a quarter (FP32) or a fraction
// (BF16 x 3: six 16x16x16 products per 16-wide stage instead of four
// 16x16x4 FP64 ones) of the matrix-core time.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>

#include "yyg_internal.h"
#include "yyg_tile.h"

namespace yyg {

namespace {

template <int PREC>
constexpr int lp_bit() {
  return PREC == 1 ? kGemmLpF32 : kGemmLpBF3;
}

// phi analysis (C column-major, transposed tile so that a store covers 16
// rows) and phi synthesis (A k-major), folded or not, as the FP64 roles
template <int PREC>
constexpr int sep_lp_mode(int phase, bool fold) {
  return lp_bit<PREC>() | (phase == 0 ? (kGemmCTrans | kGemmDT | (fold ? kGemmFoldA : 0))
                                      : (kGemmATrans | (fold ? kGemmFoldC | kGemmNFast : 0)));
}

template <int PREC, int BM, int BN, int WGM, int WGN>
hipError_t launch_sep_lp_t(int phase, bool fold, const GemmF64Args &a, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0 || a.batch <= 0) return hipSuccess;
  GemmF64Args g = a;
  g.tiles_m = (g.M + BM - 1) / BM;
  const int per = g.tiles_m * ((g.N + BN - 1) / BN);
  const long total = (long)per * g.batch;
  if (total > INT_MAX) return hipErrorInvalidValue;
  dim3 grid((unsigned)total), block(64 * WGM * WGN);
  if (phase == 0) {
    if (fold)
      hipLaunchKernelGGL((gemm_nt_f64_batched<0, BM, BN, WGM, WGN, sep_lp_mode<PREC>(0, true)>), grid, block, 0, s, g,
                         per, (int)total);
    else
      hipLaunchKernelGGL((gemm_nt_f64_batched<0, BM, BN, WGM, WGN, sep_lp_mode<PREC>(0, false)>), grid, block, 0, s,
                         g, per, (int)total);
  } else if (phase == 4) {
    if (fold)
      hipLaunchKernelGGL((gemm_nt_f64_batched<1, BM, BN, WGM, WGN, sep_lp_mode<PREC>(4, true)>), grid, block, 0, s, g,
                         per, (int)total);
    else
      hipLaunchKernelGGL((gemm_nt_f64_batched<1, BM, BN, WGM, WGN, sep_lp_mode<PREC>(4, false)>), grid, block, 0, s,
                         g, per, (int)total);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

typedef hipError_t (*sep_lp_fn)(int, bool, const GemmF64Args &, hipStream_t);
struct SepLpTile {
  int bm, bn, wm, wn;
  sep_lp_fn fn[2];  // FP32, BF16 x 3
};
#define YYG_SEP_LP_TILE(BM, BN, WM, WN) \
  { BM, BN, WM, WN, {launch_sep_lp_t<1, BM, BN, WM, WN>, launch_sep_lp_t<2, BM, BN, WM, WN>} }

const SepLpTile kSepLpTiles[] = {
    YYG_SEP_LP_TILE(64, 80, 4, 1), YYG_SEP_LP_TILE(128, 48, 4, 1), YYG_SEP_LP_TILE(64, 64, 4, 2),
    YYG_SEP_LP_TILE(64, 32, 2, 2), YYG_SEP_LP_TILE(32, 32, 2, 2),  YYG_SEP_LP_TILE(128, 80, 4, 1),
};

}  // namespace

int sep_lp_tile_count() { return (int)(sizeof(kSepLpTiles) / sizeof(kSepLpTiles[0])); }

hipError_t launch_sep_lp_phase(int prec, int tile, int phase, bool fold, const GemmF64Args &phi, hipStream_t s) {
  if (prec < 1 || prec > 2 || tile < 0 || tile >= sep_lp_tile_count()) return hipErrorInvalidValue;
  return kSepLpTiles[tile].fn[prec - 1](phase, fold, phi, s);
}

int sep_lp_kernel_name(int prec, int tile, int phase, bool fold, char *buf, size_t n) {
  if (prec < 1 || prec > 2 || tile < 0 || tile >= sep_lp_tile_count() || (phase != 0 && phase != 4)) return -1;
  const SepLpTile &t = kSepLpTiles[tile];
  const int mode = prec == 1 ? sep_lp_mode<1>(phase, fold) : sep_lp_mode<2>(phase, fold);
  return snprintf(buf, n, "yyg::gemm_nt_f64_batched<%d, %d, %d, %d, %d, %d>", phase == 0 ? 0 : 1, t.bm, t.bn, t.wm,
                  t.wn, mode) < 0 ? -1 : 0;
}

}  // namespace yyg
