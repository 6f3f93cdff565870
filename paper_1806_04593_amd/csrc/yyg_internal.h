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
  int c_sq = -1;        // >= 0: column n of C lands at column (n + c_sq)^2 (degree-major q index)
  // kGemmFoldC: the first contraction index of the odd part
  int k_split = 0;
  // kGemmAccInit: the accumulators' initial values, addressed like C
  const double *Cin = nullptr;
  // strided batch (launch_gemm_f64_batched): problem z reads A + z a_batch,
  // B + z b_batch and writes C + z c_split_stride
  int batch = 1;
  long a_batch = 0, b_batch = 0;
  // folded phi transforms (kGemmFoldA / kGemmFoldC): the unfolded row
  // length and the number of azimuthal columns
  int fold_k = 0, fold_mc = 0;
};

// Operand layouts (bit flags of the tile kernel):
//  kGemmATrans  A is stored k-major: element (m, k) at A[k * lda + m]
//  kGemmCTrans  C is stored column-major: element (m, n) at C[n * ldc + m]
//  kGemmBatch   the split index selects a problem of a strided batch
//  kGemmBTrans  B is stored k-major: element (n, k) at B[k * ldb + n]
//  kGemmDeep    three stages of loads in flight instead of one (short K)
//  kGemmFoldA   phi analysis folded about the middle of each row: batched
//               problem z = 2 j + g reads A(m, k) = X(m, k) +/- X(m,
//               fold_k - 1 - k) (+ for g = 0, - for g = 1) at A + j a_batch,
//               B at B + z b_batch, and stores output column c of group g
//               at azimuthal column mc = max(2c - 1, 0) (g = 0) or 2c + 2
//               (g = 1), if mc < fold_mc, of the column-major C + j
//               c_split_stride
//  kGemmFoldC   phi synthesis folded: A (k-major) row k is the azimuthal
//               column max(2k - 1, 0) for k < k_split, 2 (k - k_split) + 2
//               beyond (clamped below fold_mc); stages below k_split sum the
//               even part e, the rest the odd part o; output column c gets
//               e + o, column fold_k - 1 - c gets e - o
//  kGemmDT      accumulate the transposed tile (B A^T): each store then
//               covers 16 consecutive rows, for C stored column-major
//  kGemmAccInit (with the general epilogue) the accumulators start from
//               Cin (same strides as C) instead of zero
//  kGemmFoldAB  phi analysis folded, both halves in one block: batched
//               problem z = j reads A(m, k) = X(m, k) +/- X(m, fold_k - 1 - k)
//               (LDS holds both), B rows (slots) below k_split are the cos
//               half (cos m at slot m) and take the sum, the rest the sin half
//               (sin m at slot k_split + m - 1) and take the difference; slot
//               s stores azimuthal column mc (if mc < fold_mc) of the
//               column-major C + j c_split_stride
//  kGemmNFast   strided batch: a problem's tiles are numbered N-fastest (the
//               blocks that share an A tile run together and share L2)
//  kGemmLpF32   the operands rounded to FP32 on their way into LDS, FP32
//               MFMA (16x16x4) with FP32 accumulation over each 16-wide stage,
//               flushed into FP64 accumulators after every stage
//  kGemmLpBF3   the same with each operand split into three BF16 parts
//               (x = x0 + x1 + x2, each the rounding of the remainder) and the
//               six part products of order < 3 on the 16x16x16 BF16 MFMA
//  kGemmX4      v_mfma_f64_4x4x4f64 instead of the 16x16x4 form: measured on
//               MI355X it runs at ~92% of the FP64 matrix peak where the
//               16x16x4 form stops at ~62%, for four times the operand
//               traffic per flop (each 4 x 4 operand is replicated over the
//               instruction's four blocks)
enum {
  kGemmATrans = 2,
  kGemmCTrans = 4,
  kGemmBatch = 8,
  kGemmBTrans = 16,
  kGemmDeep = 32,
  kGemmFoldA = 128,
  kGemmFoldC = 256,
  kGemmDT = 512,
  kGemmAccInit = 1024,
  kGemmX4 = 2048,
  kGemmFoldAB = 4096,
  kGemmNFast = 8192,
  kGemmLpF32 = 16384,
  kGemmLpBF3 = 32768,
  // FOLDA: the column n0 + BN, when it is the last (N - 1), summed on the
  // vector units from the stage already in LDS, so that an N of one past a
  // multiple of BN needs no further MFMA tile
  kGemmXCol = 65536
};
// role offset of the kGemmDeep forms of the batched roles
constexpr int kRoleDeep = 16;

// The separable form's theta phases and moment rotation (one launch each;
// problem z of a phase derives its operands from these arguments).
struct SepPhaseArgs {
  int L, nR, P, nt;  // degree, shells, patches, colatitudes
  long ldl;          // row stride of P2
  const double *X2;  // phi-analysis output [mc][j][row]
  const double *T2;  // theta-analysis basis [mc][l][n_t]
  const double *P2;  // theta-synthesis basis [mc][j][ldl]
  const double *Ut;  // potential coefficients [mc][l][row]
  const double *D;   // per degree l: D_l (d x d, row k the input column), one after the other
  double *Ahat;      // column-major moments [Q][row] (theta analysis output)
  double *At;        // own + rotated other moments [Q][row] (Yin-Yang)
  double *V;         // theta-synthesis output [mc][j][row]
};
// Phi transforms of the separable form with the basis staged in LDS and
// the data streamed into MFMA fragments (one launch over all colatitudes).
//  analysis:  C = X2[mc][j][row] (N = 2L+1 columns mc) from X = rho
//             [row][j][k] (K = n_p) and bas = W [j][mc][ldb] (bas_batch =
//             N ldb);
//  synthesis: C = phi[row][j][k] (N = n_p) from X = V [mc][j][row] (K = 2L+1)
//             and bas = trig [k][ldb] (bas_batch = 0).
// The folded forms (launch_phi_fold) run over h = ceil(n_p / 2) cells:
//  analysis:  N = the folded basis rows (cos m at row m, sin m at row kc +
//             m - 1; kc a multiple of 16), K = h, bas = [j][N][ldb];
//  synthesis: N = h, K = the contraction slots (cos m at slot m, sin m at
//             slot kc + m - 1; kc a multiple of 4), bas = [h][ldb]
//             (bas_batch = 0);
// with np = n_p and nmc = 2L+1 the azimuthal columns.
struct PhiDirectArgs {
  const double *X, *bas;
  double *C;
  int M, nt, N, K;  // rows, colatitudes, basis rows, contraction length
  long ldb, bas_batch;
  int np = 0, kc = 0, nmc = 0;  // folded forms only
};
int phi_direct_variant_count();
hipError_t launch_phi_direct(int variant, bool analysis, const PhiDirectArgs &a, hipStream_t s);
int phi_fold_variant_count();
hipError_t launch_phi_fold(int variant, bool analysis, const PhiDirectArgs &a, hipStream_t s);

// Folded phi synthesis with every wave loading its MFMA fragments straight
// from memory (no LDS): phi[row][j][k] for k < h = ceil(n_p / 2) and the
// mirror n_p - 1 - k, from V[mc][j][row] and the slot-major basis Bk[s][hp]
// (slot s < kc: cos m = s; s >= kc: sin m = s - kc + 1; zero at padding
// slots and cells k >= h).
struct PhiLeanArgs {
  const double *V, *Bk;
  double *C;
  int M, nt, np, h, hp;  // rows, colatitudes, cells per row, folded cells, padded row (multiple of 32, >= h)
  int ns, kc, nmc;       // slots and cos slots (multiples of 4), azimuthal columns (2L+1)
};
int phi_lean_variant_count();
hipError_t launch_phi_syn_lean(int variant, const PhiLeanArgs &a, hipStream_t s);

// FP64 tiles on v_mfma_f64_4x4x4f64 (kGemmX4) for the separable phases:
// x4_variant_count() shapes; phase 0 / 4 are the phi transforms (folded
// when `fold`, as launch_gemm_f64_batched roles 2 / 3, else roles 0 / 1),
// phases 1-3 as launch_gemm_f64_sep.
// x4_variant_count(phase) of them: the generic tiles first, then (phases 0
// and 4, mirror-symmetric grids only: x4_fold_only) the folded phi
// transforms with both halves per block, phase 0 reading phi_ab
// (kGemmFoldAB), phase 4 phi (kGemmFoldC, tiles cell-fastest).
int x4_variant_count(int phase);
int x4_fold_only(int phase, int variant);
hipError_t launch_x4_sep_phase(int variant, int phase, bool fold, const GemmF64Args &phi, const GemmF64Args &phi_ab,
                               const SepPhaseArgs &a, hipStream_t s);
int x4_kernel_name(int variant, int phase, bool fold, char *buf, size_t n);

// phase 1 theta analysis, 2 rotation (two patches), 3 theta synthesis;
// deep = kGemmDeep.
hipError_t launch_gemm_f64_sep(int variant, int phase, bool deep, const SepPhaseArgs &a, hipStream_t s);

// Strided batch of g.batch equal-shape problems, whole K each: role 0
// stores C column-major, role 1 reads A k-major (plain epilogue otherwise),
// role 2 = role 0 with kGemmFoldA, role 3 = role 1 with kGemmFoldC; roles
// + kRoleDeep: the same with kGemmDeep.
hipError_t launch_gemm_f64_batched(int variant, int role, const GemmF64Args &g, hipStream_t s);
// folded phi analysis tiles with the last output column summed on the vector
// units (kGemmXCol); g as for role 2 of launch_gemm_f64_batched
int fold_xcol_variant_count();
hipError_t launch_fold_xcol(int v, const GemmF64Args &g, hipStream_t s);
int fold_xcol_kernel_name(int v, char *buf, size_t n);

// FP64 NT GEMM C = A . B^T in one of several tile shapes ("variants");
// role 0 = analysis, 1 = synthesis (separate kernel symbols).
int gemm_f64_variant_count();
void gemm_f64_variant_tile(int variant, int *bm, int *bn);
hipError_t launch_gemm_nt_f64(int variant, int role, int M, int N, int K, const double *A, long lda, const double *B,
                              long ldb, double *C, long ldc, int nsplit, long c_split_stride, hipStream_t s);

// Persistent grouped FP64 GEMM: n_blocks blocks walk `items` = (problem,
// tm, tn, split) over the problems' tiles of the variant's shape.  role 0/1
// = analysis / synthesis with the plain epilogue, 2/3 with the general one
// (ldc_c and c_sq honoured).
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
};

// Grouped scan over several plans (each n_r <= 1024): items = (problem,
// 16-column block, patch); blocks of 16 x 64 threads.
hipError_t launch_radial_scan_grouped(const ScanArgs *probs, const int4 *items, int n_items, int n_blocks,
                                      hipStream_t s);

// patches = 2 (Yin-Yang: rows of patch p also land in the cross columns of
// the other patch's rows) or 1 (polar grid: own columns only)
// Ahat may be null (no copy of the reduced moments; nsplit must be 1).
hipError_t launch_radial_scan(const double *part, int nsplit, long split_stride, double *Ahat, const double *coef,
                              const int *qdeg, int nR, int Q, int L, double negG, double *U, long ldu, int patches,
                              hipStream_t s);

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
// Radial scan of column-major moments X[q][patches nR] (one block per
// column, one wave per patch) into Ut[mc][l][patches nR]; coefS = the
// recurrence coefficients as [L+1][4][nR].  The column and its coefficients
// sit in LDS: radial_scan_q_lds bytes, at most kScanQMaxLds
// (hipErrorInvalidValue beyond).
constexpr size_t kScanQMaxLds = 160 * 1024;
size_t radial_scan_q_lds(int nR, int patches);
// n_r the column scan takes (n_r <= 3413 with two patches, 4032 with one)
bool radial_scan_q_supports(int nR, int patches);
hipError_t launch_radial_scan_q(const double *X, const double *coefS, const int *qdeg, int nR, int L, double negG,
                                int patches, double *Ut, hipStream_t s);

// The separable form's phi transforms in a reduced precision (prec 1 = FP32,
// 2 = BF16 x 3; the operands are FP64 in memory and converted in the tile):
// sep_lp_tile_count() tile shapes; phase 0 / 4 as launch_gemm_f64_batched
// roles 2 / 3 (fold) or 0 / 1.
int sep_lp_tile_count();
hipError_t launch_sep_lp_phase(int prec, int tile, int phase, bool fold, const GemmF64Args &phi, hipStream_t s);
int sep_lp_kernel_name(int prec, int tile, int phase, bool fold, char *buf, size_t n);

// Batched separable solves: one plan's column scan (as launch_radial_scan_q)
// per entry; chunk = ((nR + 63) / 64) | 1, P patches.
struct ScanQArgs {
  const double *X, *coefS;
  const int *qdeg;
  int nR, L, chunk, P;
  double negG;
  double *Ut;
};
// items = (plan, column q); blocks of 128 threads with the LDS of the
// largest plan (max_nR shells).
hipError_t launch_radial_scan_q_grouped(const ScanQArgs *args, const int2 *items, int n_items, int n_blocks,
                                        int max_nR, hipStream_t s);
// Grouped separable phases over several plans with one of
// sep_batch_tile_count() tile shapes: phase 0 / 4 the phi transforms
// (folded or not; items (plan, tile row, tile column, batch index z) over
// the plans' GemmF64Args), 1-3 the theta phases and rotation (items (plan,
// tile row, tile column, problem z) over the plans' SepPhaseArgs).
int sep_batch_tile_count();
void sep_batch_tile(int t, int *bm, int *bn, int *threads);
hipError_t launch_sep_batch_phase(int t, int phase, bool fold, const GemmF64Args *phi, const SepPhaseArgs *args,
                                  const int4 *items, int n_items, int n_blocks, hipStream_t s);
int sep_batch_kernel_name(int t, int phase, bool fold, char *buf, size_t n);

// Kernel symbol (as profilers print it) of variant v of separable phase
// `phase`, with the phi phases folded (fold) or not; 0, or -1 for an
// invalid phase / variant.
int sep_kernel_name(int phase, int v, bool fold, char *buf, size_t n);


// Split-K factor for an output of `tiles` block tiles and K columns.
int choose_split(long tiles, long K);

// Allocation-free solve: the fixed-size device scratch array of the current
// device (yyg_noalloc.hip).
constexpr size_t kScratchBytes = 64UL << 20;
hipError_t scratch_region(int device, double **ptr, size_t *bytes);

// *flag (device int) = 1 if x[0..n) holds a NaN or an infinity, else 0
hipError_t launch_check_finite(const double *x, long n, int *flag, hipStream_t s);

// Folded phi synthesis, streaming form (yyg_phi_stream.hip): for every
// row (patch, shell) and colatitude j, phi[row][j][s] = e + o and
// phi[row][j][np - 1 - s] = e - o over the folded cells s < h, with e the
// cosine part (V columns 0, 1, 3, .., 2L - 1 against TF columns 0..L) and o
// the sine part (V columns 2, 4, .., 2L against TF columns ks..ks + L - 1).
struct PhiStreamArgs {
  const double *V;   // [2L + 1][nt][Mr] theta-synthesis output
  const double *TF;  // [h][ldtf] folded basis
  double *phi;       // [Mr][nt][np] rows of ldc = nt * np
  long MJ, ldc;      // nt * Mr; nt * np
  int Mr, nt, np, h, L, nmc, ldtf, ks;
};
int phi_stream_variant_count();
// whether variant v holds the basis panel of degree L in LDS
bool phi_stream_supports(int v, int L);
int phi_stream_kernel_name(int v, char *buf, size_t n);
// cus: compute units of the device (the persistent grid's size)
hipError_t launch_phi_syn_stream(int v, const PhiStreamArgs &a, int cus, hipStream_t s);
// the same with FP32 basis panels and FP32 MFMAs flushed to FP64 every 16
// columns (the separable form's FP32 precision)
int phi_stream32_variant_count();
bool phi_stream32_supports(int v, int L);
int phi_stream32_kernel_name(int v, char *buf, size_t n);
hipError_t launch_phi_syn_stream32(int v, const PhiStreamArgs &a, int cus, hipStream_t s);

// Folded phi analysis, streaming form (yyg_phi_stream.hip): for every row
// (patch, shell) and colatitude j, X2[mc][j][row] = sum_{k < h} a_k CSF[c][k]
// with a_k = w[j][k] (rho[row][j][k] + rho[row][j][np - 1 - k]) for the
// cosine outputs c < 16 nte (m = c, column mc = max(2m - 1, 0)) and
// a_k = w[j][k] (rho_k - rho_mirror) for the sine outputs (m = c - 16 nte + 1,
// column 2m), m <= L.
struct PhiAnaStreamArgs {
  const double *rho;   // [Mr][nt][np]
  const double *CSF;   // [16 (nte + nto)][ldcs] folded basis, zero past h and past L
  const double *Wt;    // [nt][ldcs] folded overlap weights (middle cell halved), zero past h
  double *X2;          // [2L + 1][nt][Mr]
  long MJ, ldr;        // nt * Mr; nt * np
  int Mr, nt, np, h, L, nmc, ldcs, nte, nto;
};
int phi_ana_stream_variant_count();
// whether variant v holds the basis panel of h folded points in LDS
bool phi_ana_stream_supports(int v, int h, int np);
int phi_ana_stream_kernel_name(int v, char *buf, size_t n);
hipError_t launch_phi_ana_stream(int v, const PhiAnaStreamArgs &a, int cus, hipStream_t s);
// the same with an FP32 basis panel and FP32 MFMAs added to FP64 sums every
// 16 points (the separable form's FP32 precision)
int phi_ana_stream32_variant_count();
bool phi_ana_stream32_supports(int v, int h, int np);
int phi_ana_stream32_kernel_name(int v, char *buf, size_t n);
hipError_t launch_phi_ana_stream32(int v, const PhiAnaStreamArgs &a, int cus, hipStream_t s);

}  // namespace yyg
