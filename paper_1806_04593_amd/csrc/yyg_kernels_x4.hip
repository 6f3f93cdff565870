// The separable form's contractions on v_mfma_f64_4x4x4f64 (kGemmX4).
//
// On MI355X (gfx950) the FP64 16x16x4 MFMA sustains about 49 TFLOP/s, 62%
// of the 78.6 TFLOP/s FP64 matrix peak, while the 4x4x4 form (four
// independent 4 x 4 x 4 products per instruction) sustains about 72 TFLOP/s
// (measured with back-to-back independent instructions at 1-8 waves per
// SIMD).  The price is operand traffic: each instruction reads one value per
// lane of each operand for a quarter of the 16x16x4 form's work, and the
// four-wide side of every product is the same in all four blocks.  These
// tiles keep that side narrow per wave (16 or 32) and the sixteen-wide side
// wide, with the same LDS staging, prefetch and epilogues as the 16x16x4
// tiles (yyg_tile.h).
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>

#include "yyg_internal.h"
#include "yyg_tile.h"

namespace yyg {

namespace {

// Phase modes (phase 0 the phi analysis, 4 the phi synthesis, folded or
// not; 1 theta analysis, 2 rotation, 3 theta synthesis), as for the 16x16x4
// tiles, with kGemmX4.  DTA: the phi analysis accumulates the transposed
// tile (the four-wide side is then its N, the azimuthal columns).
template <int DTA>
constexpr int phi_ana_mode(bool fold) {
  return kGemmX4 | kGemmCTrans | (DTA ? kGemmDT : 0) | (fold ? kGemmFoldA : 0);
}
constexpr int phi_syn_mode(bool fold) { return kGemmX4 | kGemmATrans | (fold ? kGemmFoldC : 0); }
constexpr int kSepMode1 = kGemmX4 | 1 | kGemmATrans | kGemmDT;
constexpr int kSepMode2 = kGemmX4 | 1 | kGemmATrans | kGemmBTrans | kGemmDT | kGemmAccInit;
constexpr int kSepMode3 = kGemmX4 | kGemmBTrans;

template <int BM, int BN, int WGM, int WGN, int MODE>
hipError_t launch_batched_x4(const GemmF64Args &a, int role, hipStream_t s) {
  GemmF64Args g = a;
  g.tiles_m = (g.M + BM - 1) / BM;
  const int per = g.tiles_m * ((g.N + BN - 1) / BN);
  const long total = (long)per * g.batch;
  if (total > INT_MAX) return hipErrorInvalidValue;
  if (role == 0)
    hipLaunchKernelGGL((gemm_nt_f64_batched<0, BM, BN, WGM, WGN, MODE>), dim3((unsigned)total), dim3(64 * WGM * WGN),
                       0, s, g, per, (int)total);
  else
    hipLaunchKernelGGL((gemm_nt_f64_batched<1, BM, BN, WGM, WGN, MODE>), dim3((unsigned)total), dim3(64 * WGM * WGN),
                       0, s, g, per, (int)total);
  return hipGetLastError();
}

template <int BM, int BN, int WGM, int WGN, int DEEP, int DTA>
hipError_t launch_x4_t(int phase, bool fold, const GemmF64Args &phi, const SepPhaseArgs &a, hipStream_t s) {
  constexpr int D = DEEP ? kGemmDeep : 0;
  if (phase == 0) {
    if (phi.M <= 0 || phi.N <= 0 || phi.batch <= 0) return hipSuccess;
    return fold ? launch_batched_x4<BM, BN, WGM, WGN, phi_ana_mode<DTA>(true) | D>(phi, 0, s)
                : launch_batched_x4<BM, BN, WGM, WGN, phi_ana_mode<DTA>(false) | D>(phi, 0, s);
  }
  if (phase == 4) {
    if (phi.M <= 0 || phi.N <= 0 || phi.batch <= 0) return hipSuccess;
    return fold ? launch_batched_x4<BM, BN, WGM, WGN, phi_syn_mode(true) | D>(phi, 1, s)
                : launch_batched_x4<BM, BN, WGM, WGN, phi_syn_mode(false) | D>(phi, 1, s);
  }
  if (a.nR <= 0) return hipSuccess;
  const long Mr = (long)a.P * a.nR;
  long mmax, nmax;
  int nz;
  if (phase == 1) {
    mmax = Mr, nmax = a.L + 1, nz = 2 * a.L + 1;
  } else if (phase == 2) {
    if (a.P != 2) return hipSuccess;  // one patch: nothing to rotate
    mmax = a.nR, nmax = 2 * a.L + 1, nz = 2 * (a.L + 1);
  } else if (phase == 3) {
    mmax = a.nt, nmax = Mr, nz = 2 * a.L + 1;
  } else {
    return hipErrorInvalidValue;
  }
  if ((mmax + BM - 1) / BM > INT_MAX || (nmax + BN - 1) / BN > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)((mmax + BM - 1) / BM), (unsigned)((nmax + BN - 1) / BN), nz), block(64 * WGM * WGN);
  if (phase == 1)
    hipLaunchKernelGGL((gemm_f64_sep_phase<1, BM, BN, WGM, WGN, kSepMode1 | D>), grid, block, 0, s, a);
  else if (phase == 2)
    hipLaunchKernelGGL((gemm_f64_sep_phase<2, BM, BN, WGM, WGN, kSepMode2 | D>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((gemm_f64_sep_phase<3, BM, BN, WGM, WGN, kSepMode3 | D>), grid, block, 0, s, a);
  return hipGetLastError();
}

typedef hipError_t (*x4_fn)(int, bool, const GemmF64Args &, const SepPhaseArgs &, hipStream_t);

struct X4Variant {
  int bm, bn, wm, wn, deep, dta;
  x4_fn fn;
};

#define YYG_X4_VARIANT(BM, BN, WM, WN, DEEP, DTA) \
  { BM, BN, WM, WN, DEEP, DTA, launch_x4_t<BM, BN, WM, WN, DEEP, DTA> }

// Per wave: (BM / WM) x (BN / WN); the four-wide side is the wave's rows
// (its columns for the transposed phases 1, 2 and, DTA, the phi analysis).
const X4Variant kX4Variants[] = {
    YYG_X4_VARIANT(64, 64, 4, 1, 0, 0),  YYG_X4_VARIANT(64, 80, 4, 1, 0, 0),  YYG_X4_VARIANT(128, 64, 4, 1, 0, 0),
    YYG_X4_VARIANT(64, 128, 4, 1, 0, 0), YYG_X4_VARIANT(32, 64, 2, 1, 0, 0),  YYG_X4_VARIANT(64, 48, 4, 1, 0, 0),
    YYG_X4_VARIANT(128, 32, 4, 1, 0, 0), YYG_X4_VARIANT(64, 32, 2, 2, 0, 1),  YYG_X4_VARIANT(128, 32, 4, 2, 0, 1),
    YYG_X4_VARIANT(64, 64, 4, 1, 1, 0),  YYG_X4_VARIANT(64, 80, 4, 1, 1, 0),  YYG_X4_VARIANT(64, 32, 2, 2, 1, 1),
};
constexpr int kNX4 = (int)(sizeof(kX4Variants) / sizeof(kX4Variants[0]));

// Folded phi transforms with one block over both halves of its rows:
//  phase 0: kGemmFoldAB, every basis slot (cos half then sin half) in one
//           tile of BN >= the slots, so the density is read once;
//  phase 4: kGemmFoldC with the tiles numbered cell-fastest, so the blocks
//           that read the same coefficient rows run together.
// X4 = 1: the 4x4x4 MFMA (rows on the four-wide side), else 16x16x4 (for
// phase 0 with the transposed tile).
template <int PHASE, int BM, int BN, int WGM, int WGN, int X4, int DEEP>
hipError_t launch_phi_both_t(const GemmF64Args &phi, hipStream_t s) {
  if (phi.M <= 0 || phi.N <= 0 || phi.batch <= 0) return hipSuccess;
  constexpr int D = DEEP ? kGemmDeep : 0;
  constexpr int XM = X4 ? kGemmX4 : 0;
  if constexpr (PHASE == 0)
    return launch_batched_x4<BM, BN, WGM, WGN, XM | kGemmCTrans | kGemmFoldAB | (X4 ? 0 : kGemmDT) | D>(phi, 0, s);
  else
    return launch_batched_x4<BM, BN, WGM, WGN, XM | kGemmATrans | kGemmFoldC | kGemmNFast | D>(phi, 1, s);
}

typedef hipError_t (*both_fn)(const GemmF64Args &, hipStream_t);
struct BothVariant {
  int bm, bn, wm, wn, x4, deep;
  both_fn fn;
};
#define YYG_BOTH_VARIANT(PH, BM, BN, WM, WN, X4, DEEP) \
  { BM, BN, WM, WN, X4, DEEP, launch_phi_both_t<PH, BM, BN, WM, WN, X4, DEEP> }

const BothVariant kPhiAnaBoth[] = {
    YYG_BOTH_VARIANT(0, 64, 144, 4, 1, 1, 0), YYG_BOTH_VARIANT(0, 32, 144, 2, 1, 1, 0),
    YYG_BOTH_VARIANT(0, 64, 96, 4, 1, 1, 0),  YYG_BOTH_VARIANT(0, 64, 64, 4, 1, 1, 0),
    YYG_BOTH_VARIANT(0, 64, 144, 4, 1, 0, 0), YYG_BOTH_VARIANT(0, 64, 96, 4, 1, 0, 0),
    YYG_BOTH_VARIANT(0, 64, 64, 4, 1, 0, 0),  YYG_BOTH_VARIANT(0, 64, 144, 4, 1, 1, 1),
};
const BothVariant kPhiSynBoth[] = {
    YYG_BOTH_VARIANT(4, 64, 64, 4, 1, 1, 0),  YYG_BOTH_VARIANT(4, 128, 64, 4, 1, 1, 0),
    YYG_BOTH_VARIANT(4, 64, 128, 4, 1, 1, 0), YYG_BOTH_VARIANT(4, 128, 48, 4, 1, 0, 0),
    YYG_BOTH_VARIANT(4, 64, 64, 2, 2, 0, 0),  YYG_BOTH_VARIANT(4, 128, 64, 2, 2, 0, 0),
};
constexpr int kNAna = (int)(sizeof(kPhiAnaBoth) / sizeof(kPhiAnaBoth[0]));
constexpr int kNSyn = (int)(sizeof(kPhiSynBoth) / sizeof(kPhiSynBoth[0]));

}  // namespace

int x4_variant_count(int phase) { return kNX4 + (phase == 0 ? kNAna : phase == 4 ? kNSyn : 0); }

int x4_fold_only(int phase, int variant) { return variant >= kNX4 && variant < x4_variant_count(phase); }

hipError_t launch_x4_sep_phase(int variant, int phase, bool fold, const GemmF64Args &phi, const GemmF64Args &phi_ab,
                               const SepPhaseArgs &a, hipStream_t s) {
  if (variant < 0 || variant >= x4_variant_count(phase) || phase < 0 || phase > 4) return hipErrorInvalidValue;
  if (variant < kNX4) return kX4Variants[variant].fn(phase, fold, phi, a, s);
  if (!fold) return hipErrorInvalidValue;
  return phase == 0 ? kPhiAnaBoth[variant - kNX4].fn(phi_ab, s) : kPhiSynBoth[variant - kNX4].fn(phi, s);
}

int x4_kernel_name(int variant, int phase, bool fold, char *buf, size_t n) {
  if (variant < 0 || variant >= x4_variant_count(phase) || phase < 0 || phase > 4) return -1;
  if (variant >= kNX4) {
    if (!fold) return -1;
    const BothVariant &v = phase == 0 ? kPhiAnaBoth[variant - kNX4] : kPhiSynBoth[variant - kNX4];
    const int xm = v.x4 ? kGemmX4 : 0, d = v.deep ? kGemmDeep : 0;
    const int mode = phase == 0 ? xm | kGemmCTrans | kGemmFoldAB | (v.x4 ? 0 : kGemmDT) | d
                                : xm | kGemmATrans | kGemmFoldC | kGemmNFast | d;
    return snprintf(buf, n, "yyg::gemm_nt_f64_batched<%d, %d, %d, %d, %d, %d>", phase == 0 ? 0 : 1, v.bm, v.bn, v.wm,
                    v.wn, mode) < 0 ? -1 : 0;
  }
  const X4Variant &v = kX4Variants[variant];
  const int deep = v.deep ? kGemmDeep : 0;
  int mode;
  if (phase == 0 || phase == 4) {
    mode = (phase == 0 ? (v.dta ? phi_ana_mode<1>(fold) : phi_ana_mode<0>(fold)) : phi_syn_mode(fold)) | deep;
    return snprintf(buf, n, "yyg::gemm_nt_f64_batched<%d, %d, %d, %d, %d, %d>", phase == 0 ? 0 : 1, v.bm, v.bn, v.wm,
                    v.wn, mode) < 0 ? -1 : 0;
  }
  mode = (phase == 1 ? kSepMode1 : phase == 2 ? kSepMode2 : kSepMode3) | deep;
  return snprintf(buf, n, "yyg::gemm_f64_sep_phase<%d, %d, %d, %d, %d, %d>", phase, v.bm, v.bn, v.wm, v.wn, mode) < 0
             ? -1
             : 0;
}

}  // namespace yyg
