// HIP kernels of the Yin-Yang multipole solve on gfx950 (CDNA4).
//
//  * gemm_nt_f64: C[M x N] (+)= A[M x K] . B[N x K]^T, FP64 MFMA 16x16x4,
//    128 x 128 block tile, four waves of 64 x 64, LDS double buffering and
//    optional split-K (partials written side by side, reduced in a fixed
//    order by the consumer).  Serves the angular analysis (Eqs. 26-27: rows
//    are (patch, shell), K the angular cells, N the (l, m, cos/sin) columns)
//    and the synthesis (Eqs. 5, 28-29: K the 2Q self + cross columns, N the
//    angular cells).
//  * radial_scan: the inner/outer radial sums of Eqs. (19)-(20) as two
//    first-order recurrences per (patch, column), chunked over radius across
//    the waves of a workgroup, FP64 throughout.
//  * table expansion kernels that build the separable analysis and
//    self-synthesis bases from their FP64 factors.
#include <hip/hip_runtime.h>

#include "yyg_internal.h"

namespace yyg {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kBK = 16, kPad = 2, kLDK = kBK + kPad;

// Logical tile of a block so that the blocks one XCD receives (the hardware
// hands blocks to the 8 XCDs round-robin) form a contiguous run of tiles in
// M-fastest order: the M tiles that share a B tile then share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int total) {
  const int per = total / 8, rem = total % 8;
  const int x = b % 8, i = b / 8;
  return x * per + min(x, rem) + i;
}

}  // namespace

// Block tile BM x BN, WGM x WGN waves, each wave a (BM/WGM) x (BN/WGN) grid
// of 16 x 16 MFMA tiles; computes output tile (tm, tn) over split z.
// GEN selects the general epilogue (column stride, degree-major column
// index, accumulate); the plain one writes C[row * ldc + col].
template <int BM, int BN, int WGM, int WGN, bool GEN>
__device__ __forceinline__ void gemm_f64_tile(const GemmF64Args &g, int tm, int tn, int z) {
  const int M = g.M, N = g.N, K = g.K;
  const double *__restrict__ A = g.A;
  const double *__restrict__ B = g.B;
  double *__restrict__ C = g.C;
  const long lda = g.lda, ldb = g.ldb, ldc = g.ldc;
  constexpr int NT = 64 * WGM * WGN;
  constexpr int TI = BM / WGM / 16, TJ = BN / WGN / 16;
  static_assert(TI >= 1 && TJ >= 1 && TI * 16 * WGM == BM && TJ * 16 * WGN == BN, "tile/wave mismatch");
  // Stage loads.  When a thread's share of a tile stage divides the 16-wide
  // stage, it reads one contiguous run of k in one row (one row pointer);
  // otherwise element e = tid + i*NT sits at row e / 16, column e % 16.
  constexpr bool RUN_A = (BM * kBK) % NT == 0 && kBK % ((BM * kBK) / NT) == 0;
  constexpr bool RUN_B = (BN * kBK) % NT == 0 && kBK % ((BN * kBK) / NT) == 0;
  constexpr int EA = RUN_A ? (BM * kBK) / NT : (BM * kBK + NT - 1) / NT;
  constexpr int EB = RUN_B ? (BN * kBK) / NT : (BN * kBK + NT - 1) / NT;
  __shared__ double As[2][BM * kLDK];
  __shared__ double Bs[2][BN * kLDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = tm * BM, n0 = tn * BN;
  const int kbeg = z * g.k_per_split;
  const int kend = min(K, kbeg + g.k_per_split);
  C += (long)z * g.c_split_stride;

  const int wm = wave % WGM, wn = wave / WGM;

  dbl4 acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  double ra[EA], rb[EB];
  // run mapping: this thread's row and first column
  const int arow = RUN_A ? tid / (kBK / EA) : 0, acol = RUN_A ? (tid % (kBK / EA)) * EA : 0;
  const int brow = RUN_B ? tid / (kBK / EB) : 0, bcol = RUN_B ? (tid % (kBK / EB)) * EB : 0;
  const double *pa = A + (long)min(m0 + arow, M - 1) * lda;
  const double *pb = B + (long)min(n0 + brow, N - 1) * ldb;
  const bool va = m0 + arow < M, vb = n0 + brow < N;
  auto load = [&](int k0) {
    if constexpr (RUN_A) {
#pragma unroll
      for (int i = 0; i < EA; ++i) {
        const int kk = k0 + acol + i;
        ra[i] = (va && kk < kend) ? pa[kk] : 0.0;
      }
    } else {
#pragma unroll
      for (int i = 0; i < EA; ++i) {
        const int e = tid + i * NT, row = e / kBK, kk = k0 + e % kBK;
        const int gr = m0 + row;
        ra[i] = (e < BM * kBK && gr < M && kk < kend) ? A[(long)gr * lda + kk] : 0.0;
      }
    }
    if constexpr (RUN_B) {
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int kk = k0 + bcol + i;
        rb[i] = (vb && kk < kend) ? pb[kk] : 0.0;
      }
    } else {
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int e = tid + i * NT, row = e / kBK, kk = k0 + e % kBK;
        const int gr = n0 + row;
        rb[i] = (e < BN * kBK && gr < N && kk < kend) ? B[(long)gr * ldb + kk] : 0.0;
      }
    }
  };
  auto stash = [&](int buf) {
    if constexpr (RUN_A) {
#pragma unroll
      for (int i = 0; i < EA; ++i) As[buf][arow * kLDK + acol + i] = ra[i];
    } else {
#pragma unroll
      for (int i = 0; i < EA; ++i) {
        const int e = tid + i * NT;
        if (e < BM * kBK) As[buf][(e / kBK) * kLDK + e % kBK] = ra[i];
      }
    }
    if constexpr (RUN_B) {
#pragma unroll
      for (int i = 0; i < EB; ++i) Bs[buf][brow * kLDK + bcol + i] = rb[i];
    } else {
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int e = tid + i * NT;
        if (e < BN * kBK) Bs[buf][(e / kBK) * kLDK + e % kBK] = rb[i];
      }
    }
  };

  const int nk = (kend - kbeg + kBK - 1) / kBK;
  if (nk > 0) {
    load(kbeg);
    stash(0);
  }
  __syncthreads();

  const int frow = lane & 15, fk = 4 * (lane >> 4);
  for (int it = 0; it < nk; ++it) {
    const int buf = it & 1;
    const bool more = it + 1 < nk;
    if (more) load(kbeg + (it + 1) * kBK);
    // Each lane holds four consecutive k of its row; MFMA step s uses the
    // s-th of them, so the four steps cover the 16 k of the stage once.
    double af[TI][4], bf[TJ][4];
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      const double *s = &As[buf][(wm * (BM / WGM) + i * 16 + frow) * kLDK + fk];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) af[i][s4] = s[s4];
    }
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const double *s = &Bs[buf][(wn * (BN / WGN) + j * 16 + frow) * kLDK + fk];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) bf[j][s4] = s[s4];
    }
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i][s4], bf[j][s4], acc[i][j], 0, 0, 0);
    if (more) stash(buf ^ 1);
    __syncthreads();
  }

  // D layout of the 16x16x4 f64 MFMA: lane l, element r -> row l/16 + 4r,
  // col l%16 (one row per output group, unlike the f32 variant's four).
  const int orow = lane >> 4, ocol = lane & 15;
#pragma unroll
  for (int i = 0; i < TI; ++i) {
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int col = n0 + wn * (BN / WGN) + j * 16 + ocol;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * (BM / WGM) + i * 16 + orow + 4 * r;
        if (row < M && col < N) {
          if constexpr (GEN) {
            const long cc = g.c_sq < 0 ? (long)col * g.ldc_c : (long)(col + g.c_sq) * (col + g.c_sq);
            double *c = &C[(long)row * ldc + cc];
            *c = g.c_add ? *c + acc[i][j][r] : acc[i][j][r];
          } else {
            C[(long)row * ldc + col] = acc[i][j][r];
          }
        }
      }
    }
  }
}

// ROLE only separates the analysis (0) and synthesis (1) instantiations so
// that profilers list them apart.
template <int ROLE, int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_nt_f64_kernel(GemmF64Args g, int tiles_total) {
  const int tile = xcd_tile(blockIdx.x, tiles_total);
  gemm_f64_tile<BM, BN, WGM, WGN, false>(g, tile % g.tiles_m, tile / g.tiles_m, blockIdx.y);
}

// Persistent grouped form: blocks walk a list of (problem, tm, tn, split)
// work items over several independent contractions of one phase.
template <int ROLE, int BM, int BN, int WGM, int WGN, bool GEN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_nt_f64_grouped(const GemmF64Args *__restrict__ probs,
                                                                      const int4 *__restrict__ items, int n_items) {
  for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
    const int4 it = items[w];
    __syncthreads();  // the previous item's LDS reads are done
    gemm_f64_tile<BM, BN, WGM, WGN, GEN>(probs[it.x], it.y, it.z, it.w);
  }
}

// Radial sums of Eqs. (19)-(20) for every (patch, column), with the split-K
// partial moments reduced first (fixed order over the splits).
//   I_n = alpha_n I_(n-1) + beta_n A_n            (I_(-1) = 0)
//   O_n = gamma_n O_(n+1) + kappa_n A_(n+1)       (O_(nR-1) = 0)
// Block: 64 columns x nw waves; wave w owns a contiguous chunk of radii.
// General form for any number of shells (the register form below covers
// n_r <= 1024).
// Chunk summaries (product of multipliers, local value) combine in LDS.
// Output Ucat[(p, n)][q] = -G U[p, n, q] and Ucat[(pbar, n)][Q + q] = the same
// value, i.e. the synthesis operand [self | other] of Eqs. (28)-(29).
__global__ __launch_bounds__(1024) void radial_scan_loop_kernel(
    const double *__restrict__ part, int nsplit, long split_stride, double *__restrict__ Ahat,
    const double *__restrict__ coef, const int *__restrict__ qdeg, int nR, int Q, int L, double negG,
    double *__restrict__ U, long ldu, int cross) {
  __shared__ double sI[16][64], sPa[16][64], sO[16][64], sPg[16][64];
  const int lane = threadIdx.x, w = threadIdx.y, nw = blockDim.y;
  const int q = blockIdx.x * 64 + lane;
  const int p = blockIdx.y;
  const bool ok = q < Q;
  const int qq = ok ? q : 0;
  const int l = ok ? qdeg[q] : 0;
  const int chunk = (nR + nw - 1) / nw;
  const int n0 = min(nR, w * chunk), n1 = min(nR, n0 + chunk);
  const long rbase = (long)p * nR;
  const long rbar = (long)(1 - p) * nR;
  const double *cf = coef + (long)l * 4;
  const long cstride = (long)(L + 1) * 4;

  double I = 0.0, Pa = 1.0;
  if (ok) {
#pragma unroll 4
    for (int n = n0; n < n1; ++n) {
      const long row = rbase + n;
      double a = 0.0;
      for (int z = 0; z < nsplit; ++z) a += part[z * split_stride + row * Q + qq];
      Ahat[row * Q + qq] = a;
      const double *c = cf + n * cstride;
      I = c[0] * I + c[1] * a;
      Pa *= c[0];
    }
  }
  __syncthreads();
  double O = 0.0, Pg = 1.0;
  if (ok) {
#pragma unroll 4
    for (int n = n1 - 1; n >= n0; --n) {
      const double *c = cf + n * cstride;
      const double an = (n + 1 < nR) ? Ahat[(rbase + n + 1) * Q + qq] : 0.0;
      O = c[2] * O + c[3] * an;
      Pg *= c[2];
    }
  }
  sI[w][lane] = I;
  sPa[w][lane] = Pa;
  sO[w][lane] = O;
  sPg[w][lane] = Pg;
  __syncthreads();
  if (!ok) return;
  double Iin = 0.0, Oin = 0.0;
  for (int c = 0; c < w; ++c) Iin = sPa[c][lane] * Iin + sI[c][lane];
  for (int c = nw - 1; c > w; --c) Oin = sPg[c][lane] * Oin + sO[c][lane];

  I = Iin;
#pragma unroll 4
  for (int n = n0; n < n1; ++n) {
    const double *c = cf + n * cstride;
    I = c[0] * I + c[1] * Ahat[(rbase + n) * Q + q];
    U[(rbase + n) * ldu + q] = I;
  }
  O = Oin;
#pragma unroll 4
  for (int n = n1 - 1; n >= n0; --n) {
    const double *c = cf + n * cstride;
    const double an = (n + 1 < nR) ? Ahat[(rbase + n + 1) * Q + q] : 0.0;
    O = c[2] * O + c[3] * an;
    const double v = negG * (U[(rbase + n) * ldu + q] + O);
    U[(rbase + n) * ldu + q] = v;
    if (cross) U[(rbar + n) * ldu + Q + q] = v;
  }
}


// Register form of the radial scan for n_r <= 64 * CMAX.  Block = 16 columns
// x 64 radial chunks (one thread per (column, chunk)); each thread keeps its
// chunk's moments in registers, so every pass after the first load is
// register/LDS work.  Same recurrences, outputs and reduction order as the
// loop form.
template <int CMAX>
__device__ __forceinline__ void radial_scan_block(const ScanArgs &sa, int colblock, int p) {
  const double *__restrict__ part = sa.part;
  const int nsplit = sa.nsplit;
  const long split_stride = sa.split_stride;
  double *__restrict__ Ahat = sa.Ahat;
  const double *__restrict__ coef = sa.coef;
  const int *__restrict__ qdeg = sa.qdeg;
  const int nR = sa.nR, Q = sa.Q, L = sa.L;
  const double negG = sa.negG;
  double *__restrict__ U = sa.U;
  const long ldu = sa.ldu;
  __shared__ double sI[64][16], sPa[64][16], sO[64][16], sPg[64][16];
  const int x = threadIdx.x, y = threadIdx.y;
  const int q = colblock * 16 + x;
  const bool ok = q < Q;
  const int qq = ok ? q : 0;
  const int l = qdeg[qq];
  const int chunk = (nR + 63) / 64;
  const int n0 = min(nR, y * chunk), n1 = min(nR, n0 + chunk);
  const int len = n1 - n0;
  const long rbase = (long)p * nR;
  const double *cf = coef + (long)l * 4;
  const long cstride = (long)(L + 1) * 4;

  // a[i] = A at radius n0 + i, i <= len (the element past the chunk feeds
  // the outer recurrence); zero beyond the grid.
  double a[CMAX + 1];
#pragma unroll
  for (int i = 0; i <= CMAX; ++i) {
    double v = 0.0;
    if (ok && i <= len && n0 + i < nR) {
      const long off = (rbase + n0 + i) * Q + qq;
      for (int zz = 0; zz < nsplit; ++zz) v += part[zz * split_stride + off];
    }
    a[i] = v;
  }
  if (ok) {
#pragma unroll
    for (int i = 0; i < CMAX; ++i)
      if (i < len) Ahat[(rbase + n0 + i) * Q + qq] = a[i];
  }
  double I = 0.0, Pa = 1.0, O = 0.0, Pg = 1.0;
#pragma unroll
  for (int i = 0; i < CMAX; ++i) {
    if (i < len) {
      const double *c = cf + (n0 + i) * cstride;
      I = c[0] * I + c[1] * a[i];
      Pa *= c[0];
    }
  }
#pragma unroll
  for (int i = CMAX - 1; i >= 0; --i) {
    if (i < len) {
      const double *c = cf + (n0 + i) * cstride;
      O = c[2] * O + c[3] * a[i + 1];
      Pg *= c[2];
    }
  }
  sI[y][x] = I;
  sPa[y][x] = Pa;
  sO[y][x] = O;
  sPg[y][x] = Pg;
  __syncthreads();
  if (!ok) return;
  double Iin = 0.0, Oin = 0.0;
  for (int c = 0; c < y; ++c) Iin = sPa[c][x] * Iin + sI[c][x];
  for (int c = 63; c > y; --c) Oin = sPg[c][x] * Oin + sO[c][x];

  double Iv[CMAX];
  I = Iin;
#pragma unroll
  for (int i = 0; i < CMAX; ++i) {
    if (i < len) {
      const double *c = cf + (n0 + i) * cstride;
      I = c[0] * I + c[1] * a[i];
    }
    Iv[i] = I;
  }
  const long rbar = (long)(1 - p) * nR;
  O = Oin;
#pragma unroll
  for (int i = CMAX - 1; i >= 0; --i) {
    if (i < len) {
      const double *c = cf + (n0 + i) * cstride;
      O = c[2] * O + c[3] * a[i + 1];
      const double v = negG * (Iv[i] + O);
      U[(rbase + n0 + i) * ldu + q] = v;
      if (sa.cross) U[(rbar + n0 + i) * ldu + Q + q] = v;
    }
  }
}

template <int CMAX>
__global__ __launch_bounds__(1024) void radial_scan_kernel(ScanArgs sa) {
  radial_scan_block<CMAX>(sa, blockIdx.x, blockIdx.y);
}

// Grouped form over several plans: items = (problem, column block, patch).
__global__ __launch_bounds__(1024) void radial_scan_grouped(const ScanArgs *__restrict__ probs,
                                                            const int4 *__restrict__ items, int n_items) {
  for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
    const int4 it = items[w];
    __syncthreads();  // LDS summaries of the previous item are consumed
    radial_scan_block<16>(probs[it.x], it.y, it.z);
  }
}

// Bt[q][a] = w[a] Tbar[j][q] CS[k][q], a = j*n_p + k (analysis basis,
// Eqs. 26-27 with sqrt(N^(lm)) folded in); zero in the padding columns.
__global__ void expand_analysis_basis_kernel(const double *__restrict__ w, const double *__restrict__ Tt,
                                             const double *__restrict__ CS, int n_t, int n_p, int Q,
                                             double *__restrict__ Bt, long ldb) {
  const long a = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (a >= ldb) return;
  const long nang = (long)n_t * n_p;
  double v = 0.0;
  if (a < nang) {
    const int j = (int)(a / n_p), k = (int)(a % n_p);
    v = w[a] * Tt[(long)j * Q + q] * CS[(long)k * Q + q];
  }
  Bt[(long)q * ldb + a] = v;
}

// Ycat[a][q] = Pbar[j][q] trig[k][q] for q < Q (self-synthesis basis at the
// patch's own cell midpoints, Eq. 5); columns >= kend (padding past the
// cross columns, or past the own columns on a single-patch grid) are zeroed.
__global__ void expand_self_basis_kernel(const double *__restrict__ P, const double *__restrict__ Tr, int n_t,
                                         int n_p, int Q, double *__restrict__ Y, long ldy, int kend) {
  const int a = blockIdx.x;
  const int j = a / n_p, k = a % n_p;
  for (int q = threadIdx.x; q < ldy; q += blockDim.x) {
    if (q < Q)
      Y[(long)a * ldy + q] = P[(long)j * Q + q] * Tr[(long)k * Q + q];
    else if (q >= kend)
      Y[(long)a * ldy + q] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Separable form.  The analysis basis factors as T_j^(lm) x (w_jk C/S_k^(m))
// and the self-synthesis basis as P_l^m(cos t_j) x cos/sin(m phi_k), so each
// contraction splits into a transform over phi (a GEMM per colatitude row j)
// and one over theta (a GEMM per azimuthal column mc), both run as grouped
// launches of gemm_f64_tile.  The other patch's moments enter the synthesis
// rotated into this patch's frame, degree by degree (kernel below).
// Azimuthal column mc: 0 for m = 0, 2m-1 (cos) / 2m (sin); q = l^2 + mc.

// Ut[mc][row][l] = U[row][l^2 + mc]: own moments in azimuthal-column-major
// order; the rotated moments of the other patch are added by grouped GEMMs
// (one per degree l, with the transposed rotation block).
__global__ void scatter_moments_kernel(const double *__restrict__ U, long ldu, const int *__restrict__ qdeg, int Q,
                                       long M, double *__restrict__ Ut, long ldl) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const long row = blockIdx.y;
  if (q >= Q) return;
  const int l = qdeg[q];
  Ut[((long)(q - l * l) * M + row) * ldl + l] = U[row * ldu + q];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

namespace {

template <int BM, int BN, int WGM, int WGN>
hipError_t launch_gemm_variant(int role, int M, int N, int K, const double *A, long lda, const double *B, long ldb,
                               double *C, long ldc, int nsplit, long c_split_stride, hipStream_t s) {
  GemmF64Args g;
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = A;
  g.lda = lda;
  g.B = B;
  g.ldb = ldb;
  g.C = C;
  g.ldc = ldc;
  g.c_split_stride = c_split_stride;
  g.tiles_m = (M + BM - 1) / BM;
  const int tiles_n = (N + BN - 1) / BN;
  int kps = (K + nsplit - 1) / nsplit;
  g.k_per_split = ((kps + kBK - 1) / kBK) * kBK;
  dim3 grid(g.tiles_m * tiles_n, nsplit), block(64 * WGM * WGN);
  if (role == 0)
    hipLaunchKernelGGL((gemm_nt_f64_kernel<0, BM, BN, WGM, WGN>), grid, block, 0, s, g, g.tiles_m * tiles_n);
  else
    hipLaunchKernelGGL((gemm_nt_f64_kernel<1, BM, BN, WGM, WGN>), grid, block, 0, s, g, g.tiles_m * tiles_n);
  return hipGetLastError();
}

template <int BM, int BN, int WGM, int WGN>
hipError_t launch_grouped_variant(int role, const GemmF64Args *probs, const int4 *items, int n_items, int n_blocks,
                                  hipStream_t s) {
  dim3 grid(n_blocks), block(64 * WGM * WGN);
  // roles 0/1: analysis / synthesis with the plain epilogue; 2/3: the same
  // with the general epilogue
  switch (role) {
    case 0:
      hipLaunchKernelGGL((gemm_nt_f64_grouped<0, BM, BN, WGM, WGN, false>), grid, block, 0, s, probs, items, n_items);
      break;
    case 1:
      hipLaunchKernelGGL((gemm_nt_f64_grouped<1, BM, BN, WGM, WGN, false>), grid, block, 0, s, probs, items, n_items);
      break;
    case 2:
      hipLaunchKernelGGL((gemm_nt_f64_grouped<0, BM, BN, WGM, WGN, true>), grid, block, 0, s, probs, items, n_items);
      break;
    default:
      hipLaunchKernelGGL((gemm_nt_f64_grouped<1, BM, BN, WGM, WGN, true>), grid, block, 0, s, probs, items, n_items);
      break;
  }
  return hipGetLastError();
}

typedef hipError_t (*gemm_f64_fn)(int, int, int, int, const double *, long, const double *, long, double *, long, int,
                                  long, hipStream_t);

typedef hipError_t (*grouped_f64_fn)(int, const GemmF64Args *, const int4 *, int, int, hipStream_t);

struct F64Variant {
  int bm, bn, threads;
  gemm_f64_fn fn;
  grouped_f64_fn grouped;
};

#define YYG_F64_VARIANT(BM, BN, WM, WN) \
  { BM, BN, 64 * WM * WN, launch_gemm_variant<BM, BN, WM, WN>, launch_grouped_variant<BM, BN, WM, WN> }

const F64Variant kF64Variants[] = {
    YYG_F64_VARIANT(128, 128, 2, 2), YYG_F64_VARIANT(64, 128, 2, 2),  YYG_F64_VARIANT(128, 64, 2, 2),
    YYG_F64_VARIANT(64, 64, 2, 2),   YYG_F64_VARIANT(256, 128, 4, 2), YYG_F64_VARIANT(128, 256, 2, 4),
    // narrow-N shapes for the transforms whose N is 2L+1 or a degree block
    YYG_F64_VARIANT(128, 48, 4, 1),  YYG_F64_VARIANT(128, 96, 4, 1),  YYG_F64_VARIANT(128, 144, 4, 1),
    YYG_F64_VARIANT(64, 32, 2, 2),
};

}  // namespace

int gemm_f64_variant_count() { return (int)(sizeof(kF64Variants) / sizeof(kF64Variants[0])); }

void gemm_f64_variant_tile(int v, int *bm, int *bn) {
  *bm = kF64Variants[v].bm;
  *bn = kF64Variants[v].bn;
}

hipError_t launch_gemm_f64_grouped(int variant, int role, const GemmF64Args *probs, const int4 *items, int n_items,
                                  int n_blocks, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (variant < 0 || variant >= gemm_f64_variant_count()) return hipErrorInvalidValue;
  return kF64Variants[variant].grouped(role, probs, items, n_items, n_blocks, s);
}

hipError_t launch_gemm_nt_f64(int variant, int role, int M, int N, int K, const double *A, long lda, const double *B,
                              long ldb, double *C, long ldc, int nsplit, long c_split_stride, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (variant < 0 || variant >= gemm_f64_variant_count()) return hipErrorInvalidValue;
  return kF64Variants[variant].fn(role, M, N, K, A, lda, B, ldb, C, ldc, nsplit, c_split_stride, s);
}

hipError_t launch_radial_scan(const double *part, int nsplit, long split_stride, double *Ahat, const double *coef,
                              const int *qdeg, int nR, int Q, int L, double negG, double *U, long ldu, int patches,
                              hipStream_t s) {
  if (patches != 1 && patches != 2) return hipErrorInvalidValue;
  const int cross = patches == 2 ? 1 : 0;
  ScanArgs sa{part, nsplit, split_stride, Ahat, coef, qdeg, nR, Q, L, negG, U, ldu, cross};
  if (nR <= 64 * 4) {
    hipLaunchKernelGGL(radial_scan_kernel<4>, dim3((Q + 15) / 16, patches), dim3(16, 64), 0, s, sa);
  } else if (nR <= 64 * 16) {
    hipLaunchKernelGGL(radial_scan_kernel<16>, dim3((Q + 15) / 16, patches), dim3(16, 64), 0, s, sa);
  } else {
    int nw = 16;
    while (nw > 1 && nR / nw < 8) nw >>= 1;
    dim3 block(64, nw), grid((Q + 63) / 64, patches);
    hipLaunchKernelGGL(radial_scan_loop_kernel, grid, block, 0, s, part, nsplit, split_stride, Ahat, coef, qdeg, nR,
                       Q, L, negG, U, ldu, cross);
  }
  return hipGetLastError();
}

hipError_t launch_radial_scan_grouped(const ScanArgs *probs, const int4 *items, int n_items, int n_blocks,
                                      hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(radial_scan_grouped, dim3(n_blocks), dim3(16, 64), 0, s, probs, items, n_items);
  return hipGetLastError();
}

hipError_t launch_expand_analysis_basis(const double *w, const double *Tt, const double *CS, int n_t, int n_p,
                                        int Q, double *Bt, long ldb, hipStream_t s) {
  dim3 grid((unsigned)((ldb + 255) / 256), Q);
  hipLaunchKernelGGL(expand_analysis_basis_kernel, grid, dim3(256), 0, s, w, Tt, CS, n_t, n_p, Q, Bt, ldb);
  return hipGetLastError();
}

hipError_t launch_expand_self_basis(const double *P, const double *Tr, int n_t, int n_p, int Q, double *Y, long ldy,
                                    int kend, hipStream_t s) {
  hipLaunchKernelGGL(expand_self_basis_kernel, dim3(n_t * n_p), dim3(256), 0, s, P, Tr, n_t, n_p, Q, Y, ldy, kend);
  return hipGetLastError();
}

hipError_t launch_scatter_moments(const double *U, long ldu, const int *qdeg, int M, int Q, double *Ut, long ldl,
                                  hipStream_t s) {
  hipLaunchKernelGGL(scatter_moments_kernel, dim3((Q + 127) / 128, M), dim3(128), 0, s, U, ldu, qdeg, Q, (long)M, Ut,
                     ldl);
  return hipGetLastError();
}

int gemm_f64_variant_threads(int v) { return kF64Variants[v].threads; }

}  // namespace yyg
