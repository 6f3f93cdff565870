/*
 * yyg — Yin-Yang multipole gravity on MI355X (gfx950).
 *
 * Solves for the Newtonian potential Phi of a cell-averaged density rho on
 * the two patches of a Yin-Yang grid with the multipole method of
 * Almanstoetter, Melson, Janka & Mueller (2018), "Parallelized solution
 * method of the three-dimensional gravitational potential on the Yin-Yang
 * grid":
 *
 *   1. angular analysis into per-shell moments A_C, A_S     (Eqs. 21-22, 26-27)
 *   2. radial inner/outer cumulative sums at the interfaces (Eqs. 11-12, 16-17, 19-20)
 *   3. synthesis on every cell of both patches, both patches' moments
 *      contributing to each (Eqs. 5, 28-29).
 *
 * The same plan type also runs the single-patch method on the full-sphere
 * spherical polar grid that the paper starts from (Sect. 2, Eqs. 5, 13-22):
 * desc.kind = YYG_GRID_POLAR.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Return value: YYG_OK (0) or a negative yyg_status.  Errors never abort
 *   the process; yyg_status_string() names them.
 * - Density and potential arrays are FP64, C order [P][n_r][n_theta][n_phi]
 *   with P = 2 patches on the Yin-Yang grid: patch 0 (Yin) first, then
 *   patch 1 (Yang), each in its own local coordinates (identical local
 *   axes, Sect. 4); P = 1 on the polar grid.  rho[p][i][j][k] is the
 *   average over radial cell i (between r_edges[i] and r_edges[i+1]) and
 *   angular cell (j, k).  phi[p][n][j][k] is the potential at the outer
 *   interface r_edges[n+1] and at the midpoint of angular cell (j, k).
 * - Yin-Yang: each patch covers theta in [pi/4 - delta_theta, 3pi/4 +
 *   delta_theta] and phi in [-3pi/4 - delta_phi, 3pi/4 + delta_phi] with
 *   n_theta x n_phi equal cells (Sect. 4).  Polar: theta in [0, pi] and phi
 *   in [0, 2pi] with n_theta x n_phi equal cells (Sect. 2).
 * - Spherical-harmonic columns are ordered q(l,0) = l*l,
 *   q(l,m,cos) = l*l + 2m - 1, q(l,m,sin) = l*l + 2m (m >= 1), so
 *   Q = (lmax+1)^2 columns.
 * - Device pointers are HIP device addresses valid on the stream passed in;
 *   `stream` is a hipStream_t (NULL = legacy default stream).  The library
 *   never frees caller memory.
 * - A grid handle is not thread-safe; distinct handles are independent.
 * - Device memory cap: when the environment variable YYG_MAX_DEVICE_BYTES
 *   holds a decimal byte count (> 0), an allocation that would take the
 *   device memory the library holds in this process (every plan and batch
 *   together; see yyg_device_bytes) past it fails with
 *   YYG_ERR_OUT_OF_MEMORY before the HIP runtime is asked, and the call
 *   that needed it releases what it had allocated.  Read at every
 *   allocation; unset, 0 or not a plain number: no cap.  Pinned host
 *   memory and the allocation-free solve's scratch array are not counted.
 */
#ifndef YYG_H
#define YYG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  YYG_OK = 0,
  YYG_ERR_INVALID_ARG = -1,   /* a size, pointer or descriptor field is invalid  */
  YYG_ERR_OUT_OF_MEMORY = -2, /* device or host allocation failed                */
  YYG_ERR_DEVICE = -3,        /* a HIP runtime call or kernel launch failed       */
  YYG_ERR_NOT_READY = -4,     /* solve before upload, or precision not prepared  */
  YYG_ERR_UNSUPPORTED = -5,   /* valid request this build does not implement     */
  YYG_ERR_NONFINITE = -6      /* the density holds a NaN or an infinity (the check
                                 of yyg_set_check_finite, off by default)          */
} yyg_status;

/* Arithmetic of the two angular contractions (analysis and synthesis).  The
 * radial sums always run in FP64.  FP64 is the reference path; the others
 * trade accuracy for throughput and must be prepared first. */
typedef enum {
  YYG_FP64 = 0,   /* FP64 MFMA                                                   */
  YYG_FP32 = 1,   /* FP32 MFMA operands and accumulation                         */
  YYG_BF16X3 = 2, /* three-term BF16 operand split, FP32 MFMA accumulation       */
  YYG_FP16X2 = 3  /* two-term FP16 operand split with power-of-two scaling       */
} yyg_precision;

#define YYG_LMAX_CAP 128

/* Angular grid of a plan. */
enum {
  YYG_GRID_YINYANG = 0, /* two patches with overlap weights (Sect. 4)           */
  YYG_GRID_POLAR = 1    /* one full-sphere spherical polar patch (Sect. 2)      */
};

/* Zero-initialise and fill; kind 0 is the Yin-Yang grid. */
typedef struct {
  int n_r;                  /* radial cells, >= 1                                  */
  const double *r_edges;    /* host, n_r + 1 strictly increasing radii, r_edges[0] >= 0 */
  int n_theta, n_phi;       /* angular cells per patch, >= 1 each                  */
  double delta_theta;       /* Yin-Yang patch buffer widths [rad], 0 <= delta < pi/4;
                               must be 0 on the polar grid                          */
  double delta_phi;
  int lmax;                 /* 0 <= lmax <= YYG_LMAX_CAP                           */
  double G;                 /* gravitational constant (units of the caller)        */
  int kind;                 /* YYG_GRID_YINYANG or YYG_GRID_POLAR                  */
} yyg_grid_desc;

typedef struct yyg_grid yyg_grid;
typedef struct yyg_batch yyg_batch;

/* Build a grid plan on HIP device `device`: every density-independent table
 * of the method, computed once (Sect. 3, last paragraph): overlap weights
 * w_jk (Sect. 4, Eq. 25), polar integrals T_j^(lm) (Eq. 18), azimuthal
 * integrals C_k^(m), S_k^(m) (Eqs. 14-15), radial recurrence coefficients
 * from Eqs. (16)-(17), and the synthesis bases P_l^m cos/sin(m phi) at the
 * own and at the other patch's cell midpoints (Eqs. 5, 23-24).  On the
 * polar grid the weights are 1 and there is no other patch.  Host tables
 * are FP64.  Allocates device memory (about 8 n_theta n_phi (P+1) Q +
 * 20 P n_r Q bytes); `*out` receives the handle, to be released by
 * yyg_grid_destroy. */
int yyg_grid_create(const yyg_grid_desc *desc, int device, yyg_grid **out);

/* Same, Yin-Yang grid with the patch cells derived from an angular
 * resolution in degrees: n = ceil(span/res) + 2 cells of exactly `res_deg`
 * (span 90 deg in theta, 270 deg in phi), the surplus split evenly into the
 * two buffer widths. */
int yyg_grid_create_res(int n_r, const double *r_edges, double res_deg, int lmax,
                        double G, int device, yyg_grid **out);

/* Sizes of a plan.  Any output pointer may be NULL. */
int yyg_grid_dims(const yyg_grid *g, int *n_r, int *n_theta, int *n_phi, int *Q);

/* Grid kind (YYG_GRID_YINYANG or YYG_GRID_POLAR) and patch count P of a
 * plan.  Either output pointer may be NULL. */
int yyg_grid_kind(const yyg_grid *g, int *kind, int *patches);

/* Build the extra tables a reduced-precision path needs (no-op for FP64):
 * the analysis and synthesis bases split into 1 (FP32), 3 (BF16) or 2
 * (FP16) planes of the operand type, each basis row scaled by a power of
 * two.  Allocates; call before timing or capturing solves. */
int yyg_prepare(yyg_grid *g, int precision);

/* Solution method of yyg_solve (the separable form in FP64, FP32 or
 * BF16 x 3; see yyg_solve).
 *  YYG_METHOD_DENSE      the two angular contractions as dense MFMA
 *                        contractions over all angular cells (Eqs. 26-27 and
 *                        5, 28-29 written as matrix products): 2Q + 4Q flops
 *                        per cell.
 *  YYG_METHOD_SEPARABLE  the same sums factored along the tensor structure
 *                        of the tables: the analysis as a transform over phi
 *                        (w_jk C/S_k^(m), a GEMM per colatitude row) followed
 *                        by one over theta (T_j^(lm)); the potential of the
 *                        other patch's moments at this patch's points as the
 *                        potential of those moments rotated degree by degree
 *                        into this patch's frame (exact rotation blocks of
 *                        the real harmonics under the Yin <-> Yang map,
 *                        computed once), then one synthesis over theta and
 *                        one over phi.  On a grid that is mirror-symmetric
 *                        about the patch's central meridian (every Yin-Yang
 *                        and polar grid this library builds) each phi
 *                        transform folds into even and odd halves of
 *                        ceil(n_phi/2) points.  Equal to the dense result up
 *                        to rounding; about 2(2L+1) + 4Q/n_phi flops per
 *                        cell.  Needs 8(4 n_r + P(n_r + 1)) bytes of LDS
 *                        for its radial scan (P patches) and at most 63
 *                        shells per lane: YYG_ERR_UNSUPPORTED beyond
 *                        (n_r > 3413 on a Yin-Yang grid, 4032 polar).
 * Switching to the separable form builds its tables (allocates). */
enum { YYG_METHOD_DENSE = 0, YYG_METHOD_SEPARABLE = 1 };
int yyg_set_method(yyg_grid *g, int method);

/* Hand the density to the plan: the cell averages rho_ijk of Eq. (10), one
 * array per patch stacked as [P][n_r][n_theta][n_phi] (Yin first; Sect. 4:
 * both patches in their own local coordinates).  rho_is_device != 0: `rho` is a device
 * array that the plan borrows (no copy) and that must stay valid until the
 * next yyg_solve on `stream` completes.  rho_is_device == 0: host array,
 * copied into plan-owned device memory on `stream`. */
int yyg_upload_rho(yyg_grid *g, const double *rho, int rho_is_device, void *stream);

/* Solve Phi for the last uploaded density: the per-patch weighted moments
 * of Eqs. (21)-(22) with the overlap weights of Eqs. (26)-(27), the inner
 * and outer radial sums of Eqs. (19)-(20) at the interfaces, and the
 * synthesis of Eq. (5) with its normalisation (Eqs. 8-9), both patches'
 * moments contributing at every point (Eqs. 28-29).  Output layout as rho.
 * Precisions: the dense method any that yyg_prepare enabled (FP64 always
 * is); the separable method FP64, and FP32 or BF16 x 3 for its two phi
 * transforms (operands converted inside the kernels, FP32 accumulation over
 * 16-wide stages flushed to FP64; the theta transforms, the rotation and the
 * radial sums stay FP64; no yyg_prepare needed), YYG_ERR_UNSUPPORTED for
 * FP16 x 2 (its exponent range would need a per-row scaling the separable
 * phi transforms do not apply).  Asynchronous on `stream` when
 * phi_is_device != 0 (no host synchronisation, no allocation); with a host
 * `phi` the call copies back and synchronises the stream.  `precision` is a
 * yyg_precision that yyg_prepare has enabled (FP64 always is).  Returns
 * YYG_ERR_NOT_READY before any upload. */
int yyg_solve(yyg_grid *g, double *phi, int phi_is_device, int precision, void *stream);

/* Allocation-free separable solve, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels as yyg_solve in the separable form
 * (FP64), with every intermediate (phi and theta transform outputs,
 * moments, rotated moments, radial sums) in a fixed device scratch array of
 * 64 MiB that the library holds on each GPU it runs on until the process
 * ends, instead of the plan's own work buffers.  `rho` and `phi` are device
 * arrays in the layout of yyg_upload_rho / yyg_solve (the density is read
 * directly; no upload is needed or used); asynchronous on `stream`; no
 * allocation, no host synchronisation, no events.  YYG_ERR_NOT_READY when
 * the plan is not in the separable form (yyg_set_method);
 * YYG_ERR_UNSUPPORTED when its intermediates (sizes below) exceed the
 * scratch array; the result equals
 * yyg_solve's bit for bit.  Every call on one GPU shares that GPU's array:
 * calls that overlap in time on one GPU (concurrent streams or threads)
 * race and must be serialised by the caller.  yyg_get_moments keeps
 * reporting the last yyg_solve.  The intermediates take
 * 8 [2 (2L+1) n_theta M + (2L+1)(L+1) M + P' M Q] bytes (M = P n_r rows,
 * P' = 2 on a Yin-Yang grid, 1 on the polar grid), each part rounded up to
 * 256 bytes: e.g. 48 MB at n_r 400, 2 deg, lmax 25. */
int yyg_solve_noalloc(yyg_grid *g, const double *rho, double *phi, void *stream);

/* Opt-in input check (engineering safeguard, not part of the method):
 * with on != 0, yyg_solve, yyg_solve_noalloc and yyg_batch_solve (for each
 * field whose plan has it on) first scan the density for NaN and infinite
 * values on the solve's stream and return YYG_ERR_NONFINITE without
 * touching phi if they find one.  The check reads the density once more
 * (8 bytes per cell) and waits for its one-int result, so such a solve
 * synchronises the stream.  Turning it on allocates a 4-byte device flag
 * (YYG_ERR_OUT_OF_MEMORY / YYG_ERR_DEVICE on failure); off (the default)
 * costs nothing. */
int yyg_set_check_finite(yyg_grid *g, int on);

/* Bytes of device memory the library holds in this process (plans, their
 * work buffers and batches; the figure YYG_MAX_DEVICE_BYTES caps). */
int yyg_device_bytes(size_t *held);

/* Debug/test export after a synchronised solve: the angular moments
 * A[p][i][q] of Eqs. (26)-(27) (A_C in cos columns, A_S in sin columns) for
 * patch p and radial cell i, unnormalised as the paper defines them.  Host
 * array of P*n_r*Q doubles. */
int yyg_get_moments(yyg_grid *g, double *A_host);

/* Overlap weights w[j][k] of the plan (Sect. 4; all 1 on the polar grid);
 * host array n_theta*n_phi. */
int yyg_get_weights(const yyg_grid *g, double *w_host);

/* Release a plan and its device memory (not the caller's arrays). */
int yyg_grid_destroy(yyg_grid *g);

/* Host-only table builders, callable without a GPU (used by the CPU tests of
 * the plan logic).  `which` selects the table; `out` is a host array of
 * exactly `n` doubles:
 *   YYG_TABLE_WEIGHTS   w[j][k] (1 on the polar grid)   n = n_theta*n_phi
 *   YYG_TABLE_THETA     T_j^(lm) (unnormalised, Eq. 18) at [j][q], the
 *                       same value in the cos and sin columns     n = n_theta*Q
 *   YYG_TABLE_PHI       C_k^(m) / S_k^(m) at [k][q] (Eqs. 14-15) n = n_phi*Q
 *   YYG_TABLE_RADIAL    per radial index n (0-based) and degree l, the
 *                       four coefficients alpha, beta, gamma, kappa of the
 *                       recurrences U_n = I_n + O_n,
 *                         I_n = alpha I_(n-1) + beta A_n,
 *                         O_n = gamma O_(n+1) + kappa A_(n+1),
 *                       which reproduce r^-(l+1) sum_(i<=n) R_in,i A_i and
 *                       r^l sum_(i>n) R_out,i A_i of Eqs. (19)-(20) at
 *                       r = r_edges[n+1]; layout [n][l][4]   n = 4*n_r*(lmax+1)
 *   YYG_TABLE_CROSS     for every angular cell a = j*n_phi + k: cos theta',
 *                       sin theta', phi' of its midpoint in the other patch's
 *                       frame (Eqs. 23-24); layout [a][3]      n = 3*n_theta*n_phi
 *                       (YYG_ERR_UNSUPPORTED on the polar grid)
 *   YYG_TABLE_ROTATION  the rotation blocks of the separable form: for each
 *                       l the (2l+1)^2 matrix D_l, row-major, blocks in
 *                       order of l, with Ybar_q(R x) = sum_q' D_l[q][q']
 *                       Ybar_q'(x) for the map R: (x,y,z) -> (-x,z,y) and
 *                       Ybar_q = sqrt(N^(lm)) P_l^m cos/sin(m phi)
 *                                                  n = sum_l (2l+1)^2
 */
enum {
  YYG_TABLE_WEIGHTS = 0,
  YYG_TABLE_THETA = 1,
  YYG_TABLE_PHI = 2,
  YYG_TABLE_RADIAL = 3,
  YYG_TABLE_CROSS = 4,
  YYG_TABLE_ROTATION = 5
};
int yyg_host_table(const yyg_grid_desc *desc, int which, double *out, size_t n);

/* Per-kernel timing with HIP events recorded on the solve stream around
 * every launch of yyg_solve while enabled.  Kernel slots: 0 analysis
 * contraction, 1 radial scan, 2 synthesis contraction, 3 operand
 * conversion (reduced precisions); separable form: 4 phi analysis,
 * 5 theta analysis and the rotation of the other patch's moments,
 * 6 theta synthesis, 7 phi synthesis (and 1 its radial scan).
 * yyg_get_timing synchronises the recorded events and returns the summed
 * milliseconds and launch counts per slot (arrays of `n_slots` entries,
 * n_slots <= 8); enabling again clears the sums. */
int yyg_set_timing(yyg_grid *g, int enable);
int yyg_get_timing(yyg_grid *g, double *ms, long *counts, int n_slots);

/* Choose the launch configuration of the plan's current method by timing
 * every candidate on the plan's own shapes (HIP events on `stream`; blocks
 * until done).  Dense method: the tile shape and split-K factor of both
 * angular contractions of `precision`.  Separable method (FP64): the tile
 * variant of each of its five phases, each timed inside whole solves; FP32
 * or BF16 x 3: the tile shape of the reduced-precision phi transforms.  Allocates scratch memory for the
 * duration of the call and may grow the plan's partial-moment buffer.  With
 * the environment variable YYG_TUNE_CACHE naming a file, earlier choices
 * for the same (precision, shape) are read from it and new ones appended.
 * Without autotuning a plan uses a fixed heuristic.  Results do not depend
 * on the choice beyond FP64 summation order. */
int yyg_autotune(yyg_grid *g, int precision, void *stream);

/* Set the launch configuration of one precision by hand (tile variants as
 * numbered by yyg_plan_info, split-K factor 1..64 of the analysis).  May
 * allocate a larger partial-moment buffer; for tests and expert tuning.
 * YYG_ERR_NOT_READY for a reduced precision that is not prepared. */
int yyg_plan_config(yyg_grid *g, int precision, int var_ana, int split_ana, int var_syn);

/* Current launch configuration of one precision: info[0..6] = analysis
 * tile variant, its split-K factor, synthesis tile variant, analysis tile
 * rows/cols, synthesis tile rows/cols (first n entries are written). */
int yyg_plan_info(const yyg_grid *g, int precision, int *info, int n);

/* Tile variant (numbered as for yyg_plan_info) of one phase of the
 * separable form: 0 phi analysis, 1 theta analysis, 2 rotation of the other
 * patch's moments (Yin-Yang grids; no work on a polar grid), 3 theta
 * synthesis, 4 phi synthesis.  variant in [0, 2V), V = the number of FP64
 * tile variants: V + v is tile v with three stages of operand loads in
 * flight instead of one; the phi phases also take [2V, 2V + 6), kernels
 * that keep the phi basis in LDS and stream the data straight into MFMA
 * fragments (unfolded), and [2V + 6, 2V + 14), the same kernels folded
 * about the patch's central meridian (h = ceil(n_phi / 2) cells per row;
 * YYG_ERR_UNSUPPORTED on a grid whose rows are not mirror-symmetric, the
 * condition under which the tile variants of the phi phases fold too); the
 * phi synthesis also [2V + 14, 2V + 18), folded kernels in which every wave
 * loads its matrix-core operands straight from memory (no LDS; the same
 * mirror-symmetry condition).  Every phase then takes 12 further variants
 * at the end of its range: tiles on the 4x4x4 FP64 matrix instruction, for
 * the phi phases folded whenever the grid is mirror-symmetric; after them
 * the phi analysis takes 8 and the phi synthesis 6 folded variants in which
 * one block covers both halves of its rows (the analysis reading each
 * density value once, the synthesis its tiles ordered along the cells;
 * mirror-symmetric grids only, else YYG_ERR_UNSUPPORTED).  Last, the phi
 * synthesis takes 16 folded streaming kernels: each block keeps one panel of
 * the folded basis in LDS for its whole life and its waves sweep row tiles
 * on their own, loading the coefficients straight into 16x16x4 FP64 MFMA
 * operands several steps ahead (persistent grid of one to three blocks per
 * compute unit; the eighth to tenth, the thirteenth, fourteenth and
 * fifteenth number the row tiles colatitude row fastest, so that a block's
 * waves write neighbouring rows of the same planes; the last two give each
 * wave two row tiles of 16 rows, which share every basis fragment read from
 * LDS); the seventh holds lmax <= 131, the others lmax <= 67
 * (YYG_ERR_UNSUPPORTED beyond, and on grids that are not mirror-symmetric).
 * The phi analysis likewise takes 8 streaming kernels (the
 * colatitude-independent folded C/S basis in LDS, the overlap weights
 * applied to the density pairs as they load; folded point counts
 * h <= 416 for the sixth, h <= 272 for the others), and last 8 folded
 * tiles (64 x 64 with 4 x 1 and 2 x 2 waves, 64 x 32, 128 x 64, the two
 * 64 x 64 with three stages of loads in flight, 128 x 64 with 2 x 2 waves,
 * 64 x 64 with 4 x 2 waves) that sum the last output column on
 * the vector units when it falls just past their MFMA tiles (lmax a
 * multiple of the tile width: cos lmax, the 65th column of the even half
 * at lmax 64, then costs no MFMA tile of its own; mirror-symmetric grids
 * only).
 * yyg_sep_variant_count gives the length of each phase's range.
 * Needs the separable form built (yyg_set_method); synchronises the
 * device.  For tests and expert tuning; yyg_autotune chooses all of them. */
int yyg_sep_config(yyg_grid *g, int phase, int variant);

/* Number of variants of separable phase `phase` (0-4) that yyg_sep_config
 * numbers, or YYG_ERR_INVALID_ARG for another phase.  No device work. */
int yyg_sep_variant_count(int phase);

/* variants[0..4] = the separable form's tile variant per phase (-1 for
 * phase 2 on a polar grid, and for every phase before the form is built). */
int yyg_sep_info(const yyg_grid *g, int *variants, int n);

/* The kernel that runs separable phase `phase` (0-4, as for yyg_sep_config)
 * with the current variant, named as profilers print it (e.g.
 * "yyg::gemm_nt_f64_batched<0, 64, 32, 2, 2, 644>"), NUL-terminated into
 * name[0..n) (truncated if longer); the empty string for phase 2 on a polar
 * grid.  For matching profiles to a plan.  Needs the separable form built. */
int yyg_sep_kernel(const yyg_grid *g, int phase, char *name, size_t n);

/* The kernel that runs phi transform `phase` (0 analysis, 4 synthesis) of
 * the separable form in `precision` (YYG_FP32 or YYG_BF16X3), named as
 * profilers print it, NUL-terminated into name[0..n).  Needs the separable
 * form built. */
int yyg_sep_lp_kernel(const yyg_grid *g, int precision, int phase, char *name, size_t n);

/* Set the tile of reduced-precision phi transform `phase` (0 or 4) of the
 * separable form for `precision` (YYG_FP32 or YYG_BF16X3) by hand: tile in
 * [0, 6) (64 x 80, 128 x 48, 64 x 64, 64 x 32, 32 x 32, 128 x 80).  In FP32
 * on a mirror-symmetric grid the phi synthesis also takes [6, 15), the
 * streaming kernel of yyg_sep_config's phi synthesis with an FP32 basis
 * panel and FP32 products added to FP64 sums every 16 columns (tiles 10 and
 * 12 for lmax <= 131, the others for lmax <= 67; tiles 11, 12 and 14 number
 * the row tiles colatitude row fastest), and the phi analysis [6, 13),
 * the streaming analysis with an FP32 basis panel (a degree up to 64 in one
 * panel of 9 tiles for all but the second and third, so that each density
 * row is read once; FP64 sums every 16 points; h <= 272) — YYG_ERR_UNSUPPORTED beyond
 * these limits and on other grids.  For tests and expert tuning; yyg_autotune chooses them.
 * Needs the separable form built. */
int yyg_sep_lp_config(yyg_grid *g, int precision, int phase, int tile);

/* Launch one phase (0-4, as for yyg_sep_config) of the separable solve on
 * `stream`, asynchronously, reading what the earlier phases of the last
 * yyg_solve left in the plan's buffers (the density of the last
 * yyg_upload_rho for phase 0) and writing that phase's output (phi, a device
 * buffer laid out as for yyg_solve, for phase 4).  Repeated after a solve,
 * each phase recomputes the same output, so that a phase can be timed or
 * profiled alone.  YYG_ERR_NOT_READY without the separable form or a
 * density; before the first solve the intermediate buffers hold no defined
 * values (no fault, meaningless output). */
int yyg_sep_phase(yyg_grid *g, int phase, double *phi, void *stream);

/* Batched solves of several plans (uneven n_r, angular sizes and lmax
 * allowed) for fields that each have their own density and potential
 * arrays: the tables of every plan are built once (Sect. 3, last
 * paragraph), the density-dependent work of all fields runs together.
 * When every plan is in the separable form (yyg_set_method) and
 * `precision` is FP64, one batched solve is six persistent grouped
 * launches, the separable form's phases over every field's problems: phi
 * analysis, theta analysis, rotation of the other patch's moments, the
 * column scans, theta synthesis, phi synthesis (n_r as the plans'
 * separable form allows).  Otherwise it is the dense form's three (five
 * with the reduced-precision operand splits): all fields' analysis tiles,
 * then all radial scans, then all synthesis tiles (n_r <= 1024).  Each
 * launch's blocks walk a device work list.  Yin-Yang and polar plans may
 * be mixed.
 * The launches, together with the copy of the
 * per-field arguments, are recorded once into a HIP graph and replayed.
 * `grids` are borrowed and must outlive the batch; all on one device; for
 * a reduced precision every plan must be prepared for it.  The batch uses
 * the plans' work buffers, so a plan must not be solved on its own while a
 * batched solve that includes it is in flight.  yyg_autotune or
 * yyg_plan_config may move a plan's work buffer; a batch built before that
 * returns YYG_ERR_NOT_READY from yyg_batch_solve and must be re-created. */
int yyg_batch_create(yyg_grid *const *grids, int n, int precision, yyg_batch **out);

/* Choose the tile variant of each grouped contraction by timing them on the
 * batch (blocks until done).  Needs one earlier yyg_batch_solve (the timed
 * launches reuse its densities and rewrite its potentials with the same
 * values); YYG_ERR_NOT_READY otherwise.  The next solve records a new graph. */
int yyg_batch_autotune(yyg_batch *b, void *stream);

/* info[0..5] = fields, precision, analysis variant, synthesis variant,
 * analysis work items, synthesis work items; for a separable batch the
 * variants and items are those of the phi analysis and phi synthesis, and
 * info[6..8] the tiles of the theta analysis, rotation and theta synthesis
 * (-1 for a dense batch).  Writes the first n entries (n <= 9). */
int yyg_batch_info(const yyg_batch *b, int *info, int n);

/* Solve every field: d_rho[f] / d_phi[f] are device arrays of field f in
 * the layout above (host arrays of n pointers).  Asynchronous on `stream`;
 * with the default (NULL) stream the graph runs on a blocking stream of the
 * batch, which the default stream orders against.
 * The first call on a stream records the graph; later calls replay it.
 * Passing pointers different from the previous call waits for that call
 * to finish before the argument arrays are rewritten. */
int yyg_batch_solve(yyg_batch *b, const double *const *d_rho, double *const *d_phi, void *stream);

/* Run the launches of the last batched solve once more, eagerly (not from
 * the graph), with HIP events between the phases on `stream`; blocks and
 * writes the milliseconds of ms[0] analysis, ms[1] radial scans, ms[2]
 * synthesis, ms[3] operand splits (first n entries; a separable batch:
 * phi + theta analysis and rotation, scans, theta + phi synthesis, 0).
 * Needs one earlier yyg_batch_solve. */
int yyg_batch_profile(yyg_batch *b, void *stream, double *ms, int n);
int yyg_batch_destroy(yyg_batch *b);

/* Static string naming a status code. */
const char *yyg_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* YYG_H */
