// Batched separable solves: each phase of the separable form as one
// persistent launch over the work items of every plan in the batch (the
// tables of each plan computed once, the density-dependent work of all
// fields in one sweep per phase).
#include <hip/hip_runtime.h>

#include <cstdio>

#include "yyg_internal.h"
#include "yyg_tile.h"

namespace yyg {

namespace {

// the phases' tile modes, as in the per-plan separable launches
constexpr int kAna = kGemmCTrans | kGemmDT | kGemmBatch;
constexpr int kAnaFold = kAna | kGemmFoldA;
constexpr int kSyn = kGemmATrans | kGemmBatch;
constexpr int kSynFold = kSyn | kGemmFoldC;
constexpr int kTh1 = 1 | kGemmATrans | kGemmDT;
constexpr int kTh2 = 1 | kGemmATrans | kGemmBTrans | kGemmDT | kGemmAccInit;
constexpr int kTh3 = kGemmBTrans;

template <int BM, int BN, int WGM, int WGN>
hipError_t launch_sep_batch_t(int phase, bool fold, const GemmF64Args *phi, const SepPhaseArgs *args,
                              const int4 *items, int n_items, int n_blocks, hipStream_t s) {
  dim3 grid(n_blocks), block(64 * WGM * WGN);
  switch (phase) {
    case 0:
      if (fold)
        hipLaunchKernelGGL((gemm_nt_f64_grouped<0, BM, BN, WGM, WGN, kAnaFold>), grid, block, 0, s, phi, items, n_items);
      else
        hipLaunchKernelGGL((gemm_nt_f64_grouped<0, BM, BN, WGM, WGN, kAna>), grid, block, 0, s, phi, items, n_items);
      break;
    case 1:
      hipLaunchKernelGGL((gemm_f64_sep_grouped<1, BM, BN, WGM, WGN, kTh1>), grid, block, 0, s, args, items, n_items);
      break;
    case 2:
      hipLaunchKernelGGL((gemm_f64_sep_grouped<2, BM, BN, WGM, WGN, kTh2>), grid, block, 0, s, args, items, n_items);
      break;
    case 3:
      hipLaunchKernelGGL((gemm_f64_sep_grouped<3, BM, BN, WGM, WGN, kTh3>), grid, block, 0, s, args, items, n_items);
      break;
    case 4:
      if (fold)
        hipLaunchKernelGGL((gemm_nt_f64_grouped<1, BM, BN, WGM, WGN, kSynFold>), grid, block, 0, s, phi, items, n_items);
      else
        hipLaunchKernelGGL((gemm_nt_f64_grouped<1, BM, BN, WGM, WGN, kSyn>), grid, block, 0, s, phi, items, n_items);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

typedef hipError_t (*sep_batch_fn)(int, bool, const GemmF64Args *, const SepPhaseArgs *, const int4 *, int, int,
                                   hipStream_t);
struct SepBatchTile {
  int bm, bn, wm, wn;
  sep_batch_fn fn;
};
#define YYG_SEP_BATCH_TILE(BM, BN, WM, WN) \
  { BM, BN, WM, WN, launch_sep_batch_t<BM, BN, WM, WN> }

// the shapes the per-plan autotuner picks most often on the separable phases
const SepBatchTile kSepBatchTiles[] = {
    YYG_SEP_BATCH_TILE(32, 32, 2, 2), YYG_SEP_BATCH_TILE(64, 32, 2, 2), YYG_SEP_BATCH_TILE(64, 64, 4, 2),
    YYG_SEP_BATCH_TILE(64, 80, 4, 1), YYG_SEP_BATCH_TILE(128, 48, 4, 1),
};

int mode_of(int phase, bool fold) {
  switch (phase) {
    case 0: return fold ? kAnaFold : kAna;
    case 1: return kTh1;
    case 2: return kTh2;
    case 3: return kTh3;
    default: return fold ? kSynFold : kSyn;
  }
}

}  // namespace

int sep_batch_tile_count() { return (int)(sizeof(kSepBatchTiles) / sizeof(kSepBatchTiles[0])); }

void sep_batch_tile(int t, int *bm, int *bn, int *threads) {
  *bm = kSepBatchTiles[t].bm;
  *bn = kSepBatchTiles[t].bn;
  *threads = 64 * kSepBatchTiles[t].wm * kSepBatchTiles[t].wn;
}

hipError_t launch_sep_batch_phase(int t, int phase, bool fold, const GemmF64Args *phi, const SepPhaseArgs *args,
                                  const int4 *items, int n_items, int n_blocks, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (t < 0 || t >= sep_batch_tile_count() || n_blocks <= 0) return hipErrorInvalidValue;
  return kSepBatchTiles[t].fn(phase, fold, phi, args, items, n_items, n_blocks, s);
}

int sep_batch_kernel_name(int t, int phase, bool fold, char *buf, size_t n) {
  if (t < 0 || t >= sep_batch_tile_count() || phase < 0 || phase > 4) return -1;
  const SepBatchTile &v = kSepBatchTiles[t];
  const int mode = mode_of(phase, fold);  // the kernel's template argument
  if (phase == 0 || phase == 4)
    return snprintf(buf, n, "yyg::gemm_nt_f64_grouped<%d, %d, %d, %d, %d, %d>", phase == 0 ? 0 : 1, v.bm, v.bn, v.wm,
                    v.wn, mode) < 0 ? -1 : 0;
  return snprintf(buf, n, "yyg::gemm_f64_sep_grouped<%d, %d, %d, %d, %d, %d>", phase, v.bm, v.bn, v.wm, v.wn, mode) < 0
             ? -1
             : 0;
}

}  // namespace yyg
