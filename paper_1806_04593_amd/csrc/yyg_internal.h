// Internal launch interface between the C-ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace yyg {

// Arguments of one FP64 NT GEMM problem (grouped launches read an array).
struct GemmF64Args {
  int M, N, K;
  const double *A;
  long lda;
  const double *B;
  long ldb;
  double *C;
  long ldc;             // row stride of C
  long c_split_stride;
  int k_per_split;      // multiple of the stage width (16)
  int tiles_m;
  long ldc_c = 1;       // column stride of C
  int c_sq = -1;        // >= 0: column n of C lands at (n + c_sq)^2 (degree-major q index)
  int c_add = 0;        // 1: C += A.B^T instead of C = A.B^T
  // strided batch (launch_gemm_f64_batched): problem z reads A + z a_batch,
  // B + z b_batch and writes C + z c_split_stride
  int batch = 1;
  long a_batch = 0, b_batch = 0;
};

// Operand layouts (bit flags of the tile kernel):
//  kGemmATrans  A is stored k-major: element (m, k) at A[k * lda + m]
//  kGemmCTrans  C is stored column-major: element (m, n) at C[n * ldc + m]
//  kGemmBatch   the split index selects a problem of a strided batch
enum { kGemmATrans = 2, kGemmCTrans = 4, kGemmBatch = 8 };

// Strided batch of g.batch equal-shape problems, whole K each: role 0
// stores C column-major, role 1 reads A k-major (plain epilogue otherwise).
hipError_t launch_gemm_f64_batched(int variant, int role, const GemmF64Args &g, hipStream_t s);

// FP64 NT GEMM C = A . B^T in one of several tile shapes ("variants");
// role 0 = analysis, 1 = synthesis (separate kernel symbols).
int gemm_f64_variant_count();
void gemm_f64_variant_tile(int variant, int *bm, int *bn);
hipError_t launch_gemm_nt_f64(int variant, int role, int M, int N, int K, const double *A, long lda, const double *B,
                              long ldb, double *C, long ldc, int nsplit, long c_split_stride, hipStream_t s);

// Persistent grouped FP64 GEMM: n_blocks blocks walk `items` = (problem,
// tm, tn, split) over the problems' tiles of the variant's shape.  role 0/1
// = analysis / synthesis with the plain epilogue, 2/3 with the general one
// (ldc_c, c_sq, c_add honoured), 4 = synthesis with the general epilogue
// and A stored k-major (kGemmATrans), 5 = analysis with the general
// epilogue and A stored k-major.
hipError_t launch_gemm_f64_grouped(int variant, int role, const GemmF64Args *probs, const int4 *items, int n_items,
                                  int n_blocks, hipStream_t s);

// Arguments of one radial scan (see launch_radial_scan).
struct ScanArgs {
  const double *part;
  int nsplit;
  long split_stride;
  double *Ahat;
  const double *coef;
  const int *qdeg;
  int nR, Q, L;
  double negG;
  double *U;
  long ldu;
  int cross;  // also write each row into the other patch's cross columns [Q, 2Q)
  double *Ut = nullptr;  // if set: write U to Ut[mc][l][row] (q = l^2 + mc) instead
  long ut_rows = 0;      // rows of Ut (patches x nR)
};

// Grouped scan over several plans (each n_r <= 1024): items = (problem,
// 16-column block, patch); blocks of 16 x 64 threads.
hipError_t launch_radial_scan_grouped(const ScanArgs *probs, const int4 *items, int n_items, int n_blocks,
                                      hipStream_t s);

// patches = 2 (Yin-Yang: rows of patch p also land in the cross columns of
// the other patch's rows) or 1 (polar grid: own columns only)
// Ahat may be null (no copy of the reduced moments).  With Ut set the
// potential coefficients go to Ut[mc][l][row] (azimuthal-column-major,
// rows contiguous) instead of U; needs nR <= 1024.
hipError_t launch_radial_scan(const double *part, int nsplit, long split_stride, double *Ahat, const double *coef,
                              const int *qdeg, int nR, int Q, int L, double negG, double *U, long ldu, int patches,
                              hipStream_t s, double *Ut = nullptr);

hipError_t launch_expand_analysis_basis(const double *w, const double *Tt, const double *CS, int n_t, int n_p,
                                        int Q, double *Bt, long ldb, hipStream_t s);

hipError_t launch_expand_self_basis(const double *P, const double *Tr, int n_t, int n_p, int Q, double *Y, long ldy,
                                    int kend, hipStream_t s);

// Reduced-precision contractions (prec 1 = FP32, 2 = BF16 x 3, 3 = FP16 x 2):
// A and B as pre-split planes of the operand type ([rows][ld] each, plane
// strides apart, k zero-padded to the stage width, rows scaled by 2^-e),
// FP32 MFMA accumulation flushed to FP64.
struct GemmLpArgs {
  int M, N, K;
  const void *A;  // planes [parts][M][lda], a_plane elements apart
  long lda, a_plane;
  const int *eA;  // row exponents of A (nullable)
  const void *B;  // planes [parts][N][ldb]
  long ldb, b_plane;
  const int *eB;
  double *C;
  long ldc, c_split_stride;
  int k_per_split;  // multiple of the stage width
  int tiles_m;
};

int gemm_lp_variant_count();
void gemm_lp_variant_tile(int variant, int *bm, int *bn);
int lp_parts(int prec);
int lp_elem_bytes(int prec);
int lp_stage_k(int prec);
hipError_t launch_gemm_nt_lp(int prec, int variant, int role, int M, int N, int K, const void *A, long lda,
                             long a_plane, const int *eA, const void *B, long ldb, long b_plane, const int *eB,
                             double *C, long ldc, int nsplit, long c_split_stride, hipStream_t s);
hipError_t launch_gemm_lp_grouped(int prec, int variant, int role, const GemmLpArgs *probs, const int4 *items,
                                 int n_items, int n_blocks, hipStream_t s);
hipError_t launch_row_exponent(const double *X, long ldx, int rows, int ncols, int *e, hipStream_t s);

// Grouped row split over several matrices: items = (problem, row).  With
// `e` non-null the row's power-of-two exponent is computed first (and
// stored), otherwise rows are not scaled.
struct SplitArgs {
  const double *X;
  long ldx;
  int ncols;
  int *e;
  void *P;
  long ldp, plane;
};
hipError_t launch_split_rows_grouped(int prec, const SplitArgs *probs, const int2 *items, int n_items, int n_blocks,
                                     hipStream_t s);
hipError_t launch_split_rows(int prec, const double *X, long ldx, int rows, int ncols, const int *e, void *P,
                             long ldp, long plane_stride, hipStream_t s);

// Separable-form kernels (see yyg_kernels.hip).
// At[row][q] = A[row][q] + the other patch's moments of the same shell
// rotated degree by degree (rows: 2 nR, Yin then Yang); dofs[l] = offset of
// the transposed rotation block of degree l in Dt.
hipError_t launch_rotate_moments(const double *A, int nR, int L, const int *dofs, const double *Dt, double *At,
                                 hipStream_t s);
int gemm_f64_variant_threads(int v);


// Split-K factor for an output of `tiles` block tiles and K columns.
int choose_split(long tiles, long K);

}  // namespace yyg
