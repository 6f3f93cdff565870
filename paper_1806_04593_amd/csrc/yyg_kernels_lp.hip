// Reduced-precision forms of the two angular contractions (analysis and
// synthesis): the same NT GEMM C[M x N] = A[M x K] . B[N x K]^T as the FP64
// path, with
//   * A (the density, or the radial-scan output) split into NP parts of the
//     operand type: x = x0 + x1 (+ x2), each part the rounding of the
//     remainder (exact residuals in FP64);
//   * B (the analysis / synthesis basis) split the same way into NP planes;
//   * every product term with part orders i + j < NP on MFMA with FP32
//     accumulation, flushed into FP64 accumulators every kFlush stages;
//   * optional power-of-two scaling of A rows and B rows (needed for FP16's
//     narrow exponent range), undone exactly in the FP64 epilogue.
// PREC 1 = FP32 (one part), 2 = BF16 x 3 parts, 3 = FP16 x 2 parts.
// The FP64 operands are split into planes by split_rows_kernel before the
// contraction (the density once per solve, the bases once per plan).
#include <hip/hip_runtime.h>

#include "yyg_internal.h"

namespace yyg {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double dbl4lp __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

namespace {

template <int PREC>
struct LpTraits;

template <>
struct LpTraits<1> {
  typedef float T;
  static constexpr int NP = 1, BK = 16, PAD = 4;
};
template <>
struct LpTraits<2> {
  typedef __bf16 T;
  static constexpr int NP = 3, BK = 32, PAD = 8;
};
template <>
struct LpTraits<3> {
  typedef _Float16 T;
  static constexpr int NP = 2, BK = 32, PAD = 8;
};

constexpr int kFlush = 4;  // stages per FP32 accumulation chunk

__device__ __forceinline__ int xcd_tile_lp(int b, int total) {
  const int per = total / 8, rem = total % 8;
  const int x = b % 8, i = b / 8;
  return x * per + min(x, rem) + i;
}

// Split x into NP parts of type T with x = sum(parts) + (tail below the last part).
template <class T, int NP>
__device__ __forceinline__ void split_parts(double x, T (&p)[NP]) {
  double r = x;
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    p[i] = (T)r;
    r -= (double)p[i];
  }
}

template <int PREC>
__device__ __forceinline__ f32x4 mfma_lp(const typename LpTraits<PREC>::T *a, const typename LpTraits<PREC>::T *b,
                                         f32x4 c);

}  // namespace

// Both operands arrive as pre-split planes of the operand type: plane p of A
// is [M][lda], of B [N][ldb], plane_stride elements apart, zero-padded to a
// multiple of the stage width in k (so a stage never needs a k bound).  Rows
// carry power-of-two exponents eA / eB (nullable) undone in the epilogue.
template <int PREC, int BM, int BN, int WGM, int WGN>
__device__ __forceinline__ void gemm_lp_tile(const GemmLpArgs &g, int tm, int tn, int z) {
  typedef typename LpTraits<PREC>::T Te;
  const int M = g.M, N = g.N, K = g.K;
  const Te *__restrict__ A = static_cast<const Te *>(g.A);
  const Te *__restrict__ B = static_cast<const Te *>(g.B);
  const int *__restrict__ eA = g.eA;
  const int *__restrict__ eB = g.eB;
  double *__restrict__ C = g.C;
  const long lda = g.lda, ldb = g.ldb, ldc = g.ldc, a_plane = g.a_plane, b_plane = g.b_plane;
  typedef typename LpTraits<PREC>::T T;
  typedef uint4 V;                                     // 16-byte chunk
  constexpr int NP = LpTraits<PREC>::NP, BK = LpTraits<PREC>::BK, LDK = BK + LpTraits<PREC>::PAD;
  constexpr int EPC = 16 / sizeof(T);                  // elements per chunk
  constexpr int CPR = BK / EPC;                        // chunks per row per stage
  constexpr int NT = 64 * WGM * WGN;
  constexpr int TI = BM / WGM / 16, TJ = BN / WGN / 16;
  constexpr int CA = NP * BM * CPR / NT, CB = NP * BN * CPR / NT;  // chunks per thread
  static_assert(CA * NT == NP * BM * CPR && CB * NT == NP * BN * CPR, "tile/thread mismatch");
  constexpr int FK = (PREC == 1) ? 4 : 8;
  __shared__ __attribute__((aligned(16))) T As[2][NP][BM * LDK];
  __shared__ __attribute__((aligned(16))) T Bs[2][NP][BN * LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = tm * BM, n0 = tn * BN;
  const int kbeg = z * g.k_per_split;
  const int kend = min(K, kbeg + g.k_per_split);
  C += (long)z * g.c_split_stride;
  const int wm = wave % WGM, wn = wave / WGM;

  f32x4 facc[TI][TJ];
  dbl4lp dacc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      facc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      dacc[i][j] = dbl4lp{0.0, 0.0, 0.0, 0.0};
    }

  // chunk c of this thread: plane, row, chunk-in-row
  V ra[CA], rb[CB];
  auto load = [&](int k0) {
#pragma unroll
    for (int c = 0; c < CA; ++c) {
      const int id = tid + c * NT;
      const int p = id / (BM * CPR), rem = id % (BM * CPR), row = rem / CPR, cc = rem % CPR;
      const int gr = m0 + row;
      // clamped, valid address; rows past M are zeroed by stash (a load
      // under a condition would be waited for before the next one issues)
      const V *src = reinterpret_cast<const V *>(A + p * a_plane + (long)min(gr, M - 1) * lda + k0 + cc * EPC);
      ra[c] = *src;
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int id = tid + c * NT;
      const int p = id / (BN * CPR), rem = id % (BN * CPR), row = rem / CPR, cc = rem % CPR;
      const int gr = n0 + row;
      const V *src = reinterpret_cast<const V *>(B + p * b_plane + (long)min(gr, N - 1) * ldb + k0 + cc * EPC);
      rb[c] = *src;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int c = 0; c < CA; ++c) {
      const int id = tid + c * NT;
      const int p = id / (BM * CPR), rem = id % (BM * CPR), row = rem / CPR, cc = rem % CPR;
      *reinterpret_cast<V *>(&As[buf][p][row * LDK + cc * EPC]) = m0 + row < M ? ra[c] : V{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int c = 0; c < CB; ++c) {
      const int id = tid + c * NT;
      const int p = id / (BN * CPR), rem = id % (BN * CPR), row = rem / CPR, cc = rem % CPR;
      *reinterpret_cast<V *>(&Bs[buf][p][row * LDK + cc * EPC]) = n0 + row < N ? rb[c] : V{0u, 0u, 0u, 0u};
    }
  };

  const int nk = (kend - kbeg + BK - 1) / BK;
  if (nk > 0) {
    load(kbeg);
    stash(0);
  }
  __syncthreads();

  const int frow = lane & 15, fk = FK * (lane >> 4);
  for (int it = 0; it < nk; ++it) {
    const int buf = it & 1;
    const bool more = it + 1 < nk;
    if (more) load(kbeg + (it + 1) * BK);
    T af[NP][TI][FK], bf[NP][TJ][FK];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        const V v = *reinterpret_cast<const V *>(&As[buf][p][(wm * (BM / WGM) + i * 16 + frow) * LDK + fk]);
        __builtin_memcpy(&af[p][i][0], &v, sizeof(V));
      }
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        const V v = *reinterpret_cast<const V *>(&Bs[buf][p][(wn * (BN / WGN) + j * 16 + frow) * LDK + fk]);
        __builtin_memcpy(&bf[p][j][0], &v, sizeof(V));
      }
    }
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        // part pairs with order pa + pb < NP, smallest terms first
#pragma unroll
        for (int ord = NP - 1; ord >= 0; --ord)
#pragma unroll
          for (int p = 0; p <= ord; ++p) facc[i][j] = mfma_lp<PREC>(af[p][i], bf[ord - p][j], facc[i][j]);
      }
    if ((it + 1) % kFlush == 0 || it + 1 == nk) {
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) dacc[i][j][r] += (double)facc[i][j][r];
          facc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
  }

  // D layout of the FP32-accumulating 16x16 MFMAs: lane l, element r ->
  // row 4(l/16) + r, col l%16.
  const int orow = 4 * (lane >> 4), ocol = lane & 15;
#pragma unroll
  for (int i = 0; i < TI; ++i) {
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int col = n0 + wn * (BN / WGN) + j * 16 + ocol;
      const int ebc = (eB && col < N) ? eB[col] : 0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * (BM / WGM) + i * 16 + orow + r;
        if (row < M && col < N) {
          const int e = ebc + (eA ? eA[row] : 0);
          C[(long)row * ldc + col] = ldexp(dacc[i][j][r], e);
        }
      }
    }
  }
}

template <int ROLE, int PREC, int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_nt_lp_kernel(GemmLpArgs g, int tiles_total) {
  const int tile = xcd_tile_lp(blockIdx.x, tiles_total);
  gemm_lp_tile<PREC, BM, BN, WGM, WGN>(g, tile % g.tiles_m, tile / g.tiles_m, blockIdx.y);
}

template <int ROLE, int PREC, int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_nt_lp_grouped(const GemmLpArgs *__restrict__ probs,
                                                                     const int4 *__restrict__ items, int n_items) {
  for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
    const int4 it = items[w];
    __syncthreads();  // the previous item's LDS reads are done
    gemm_lp_tile<PREC, BM, BN, WGM, WGN>(probs[it.x], it.y, it.z, it.w);
  }
}

namespace {

template <>
__device__ __forceinline__ f32x4 mfma_lp<1>(const float *a, const float *b, f32x4 c) {
  // four k-steps: lane holds k = 4 (l/16) + s for step s, A and B alike
#pragma unroll
  for (int s = 0; s < 4; ++s) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], c, 0, 0, 0);
  return c;
}
template <>
__device__ __forceinline__ f32x4 mfma_lp<2>(const __bf16 *a, const __bf16 *b, f32x4 c) {
  bf16x8 va, vb;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    va[e] = a[e];
    vb[e] = b[e];
  }
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(va, vb, c, 0, 0, 0);
}
template <>
__device__ __forceinline__ f32x4 mfma_lp<3>(const _Float16 *a, const _Float16 *b, f32x4 c) {
  f16x8 va, vb;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    va[e] = a[e];
    vb[e] = b[e];
  }
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(va, vb, c, 0, 0, 0);
}

}  // namespace

// Power-of-two exponent e of each row's largest magnitude (|x| 2^-e < 1),
// 0 for an all-zero row.  One block per row.
__global__ void row_exponent_kernel(const double *__restrict__ X, long ldx, int ncols, int *__restrict__ e) {
  __shared__ double red[256];
  const long row = blockIdx.x;
  double m = 0.0;
  for (int c = threadIdx.x; c < ncols; c += blockDim.x) m = fmax(m, fabs(X[row * ldx + c]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int ex = 0;
    if (red[0] > 0.0) frexp(red[0], &ex);
    e[row] = ex;
  }
}

// Split an FP64 matrix [rows][ncols] (leading dimension ldx) into NP planes
// of T, [rows][ldp] each (zero past ncols), rows scaled by 2^-e[row].
template <int PREC>
__global__ void split_rows_kernel(const double *__restrict__ X, long ldx, int ncols, const int *__restrict__ e,
                                  typename LpTraits<PREC>::T *__restrict__ P, long ldp, long plane_stride) {
  typedef typename LpTraits<PREC>::T T;
  constexpr int NP = LpTraits<PREC>::NP;
  const long row = blockIdx.y;
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ldp) return;
  const double x = (c < ncols) ? ldexp(X[row * ldx + c], -(e ? e[row] : 0)) : 0.0;
  T parts[NP];
  split_parts<T, NP>(x, parts);
#pragma unroll
  for (int p = 0; p < NP; ++p) P[p * plane_stride + row * ldp + c] = parts[p];
}

// Grouped row split: one block per (problem, row) item; optionally the row's
// exponent first (max-reduction in LDS), then the planes.
template <int PREC>
__global__ __launch_bounds__(256) void split_rows_grouped_kernel(const SplitArgs *__restrict__ probs,
                                                                 const int2 *__restrict__ items, int n_items) {
  typedef typename LpTraits<PREC>::T T;
  constexpr int NP = LpTraits<PREC>::NP;
  __shared__ double red[256];
  for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
    const int2 it = items[w];
    const SplitArgs a = probs[it.x];
    const long row = it.y;
    const double *x = a.X + row * a.ldx;
    int ex = 0;
    if (a.e) {
      double m = 0.0;
      for (int c = threadIdx.x; c < a.ncols; c += blockDim.x) m = fmax(m, fabs(x[c]));
      __syncthreads();  // previous item's reads of red[] are done
      red[threadIdx.x] = m;
      __syncthreads();
      for (int st = blockDim.x / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
      }
      if (red[0] > 0.0) frexp(red[0], &ex);
      if (threadIdx.x == 0) a.e[row] = ex;
    }
    T *P = static_cast<T *>(a.P);
    for (long c = threadIdx.x; c < a.ldp; c += blockDim.x) {
      const double v = (c < a.ncols) ? ldexp(x[c], -ex) : 0.0;
      T parts[NP];
      split_parts<T, NP>(v, parts);
#pragma unroll
      for (int pp = 0; pp < NP; ++pp) P[pp * a.plane + row * a.ldp + c] = parts[pp];
    }
  }
}

namespace {

template <int PREC, int BM, int BN, int WGM, int WGN>
hipError_t launch_lp_variant(int role, int M, int N, int K, const void *A, long lda, long a_plane, const int *eA,
                             const void *B, long ldb, long b_plane, const int *eB, double *C, long ldc, int nsplit,
                             long c_split_stride, hipStream_t s) {
  constexpr int BK = LpTraits<PREC>::BK;
  GemmLpArgs g;
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = A;
  g.lda = lda;
  g.a_plane = a_plane;
  g.eA = eA;
  g.B = B;
  g.ldb = ldb;
  g.b_plane = b_plane;
  g.eB = eB;
  g.C = C;
  g.ldc = ldc;
  g.c_split_stride = c_split_stride;
  g.tiles_m = (M + BM - 1) / BM;
  const int tiles_n = (N + BN - 1) / BN;
  int kps = (K + nsplit - 1) / nsplit;
  g.k_per_split = ((kps + BK - 1) / BK) * BK;
  dim3 grid(g.tiles_m * tiles_n, nsplit), block(64 * WGM * WGN);
  if (role == 0)
    hipLaunchKernelGGL((gemm_nt_lp_kernel<0, PREC, BM, BN, WGM, WGN>), grid, block, 0, s, g, g.tiles_m * tiles_n);
  else
    hipLaunchKernelGGL((gemm_nt_lp_kernel<1, PREC, BM, BN, WGM, WGN>), grid, block, 0, s, g, g.tiles_m * tiles_n);
  return hipGetLastError();
}

template <int PREC, int BM, int BN, int WGM, int WGN>
hipError_t launch_lp_grouped(int role, const GemmLpArgs *probs, const int4 *items, int n_items, int n_blocks,
                             hipStream_t s) {
  dim3 grid(n_blocks), block(64 * WGM * WGN);
  if (role == 0)
    hipLaunchKernelGGL((gemm_nt_lp_grouped<0, PREC, BM, BN, WGM, WGN>), grid, block, 0, s, probs, items, n_items);
  else
    hipLaunchKernelGGL((gemm_nt_lp_grouped<1, PREC, BM, BN, WGM, WGN>), grid, block, 0, s, probs, items, n_items);
  return hipGetLastError();
}

typedef hipError_t (*gemm_lp_fn)(int, int, int, int, const void *, long, long, const int *, const void *, long,
                                 long, const int *, double *, long, int, long, hipStream_t);

typedef hipError_t (*grouped_lp_fn)(int, const GemmLpArgs *, const int4 *, int, int, hipStream_t);

struct LpVariant {
  int bm, bn, threads;
  gemm_lp_fn fn[3];  // FP32, BF16x3, FP16x2
  grouped_lp_fn grouped[3];
};

#define YYG_LP_VARIANT(BM, BN, WM, WN)                                                                         \
  {                                                                                                            \
    BM, BN, 64 * WM * WN,                                                                                      \
        {launch_lp_variant<1, BM, BN, WM, WN>, launch_lp_variant<2, BM, BN, WM, WN>,                           \
         launch_lp_variant<3, BM, BN, WM, WN>},                                                                \
    {                                                                                                          \
      launch_lp_grouped<1, BM, BN, WM, WN>, launch_lp_grouped<2, BM, BN, WM, WN>,                              \
          launch_lp_grouped<3, BM, BN, WM, WN>                                                                 \
    }                                                                                                          \
  }

const LpVariant kLpVariants[] = {
    YYG_LP_VARIANT(64, 64, 2, 2),
    YYG_LP_VARIANT(128, 64, 2, 2),
    YYG_LP_VARIANT(64, 128, 2, 2),
    YYG_LP_VARIANT(128, 128, 2, 2),
    YYG_LP_VARIANT(128, 128, 4, 2),
};

}  // namespace

int gemm_lp_variant_count() { return (int)(sizeof(kLpVariants) / sizeof(kLpVariants[0])); }

void gemm_lp_variant_tile(int v, int *bm, int *bn) {
  *bm = kLpVariants[v].bm;
  *bn = kLpVariants[v].bn;
}

int lp_parts(int prec) { return prec == 1 ? 1 : (prec == 2 ? 3 : 2); }
int lp_elem_bytes(int prec) { return prec == 1 ? 4 : 2; }
int lp_stage_k(int prec) { return prec == 1 ? LpTraits<1>::BK : LpTraits<2>::BK; }

hipError_t launch_gemm_nt_lp(int prec, int variant, int role, int M, int N, int K, const void *A, long lda,
                             long a_plane, const int *eA, const void *B, long ldb, long b_plane, const int *eB,
                             double *C, long ldc, int nsplit, long c_split_stride, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (prec < 1 || prec > 3 || variant < 0 || variant >= gemm_lp_variant_count()) return hipErrorInvalidValue;
  return kLpVariants[variant].fn[prec - 1](role, M, N, K, A, lda, a_plane, eA, B, ldb, b_plane, eB, C, ldc, nsplit,
                                           c_split_stride, s);
}

hipError_t launch_gemm_lp_grouped(int prec, int variant, int role, const GemmLpArgs *probs, const int4 *items,
                                 int n_items, int n_blocks, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (prec < 1 || prec > 3 || variant < 0 || variant >= gemm_lp_variant_count()) return hipErrorInvalidValue;
  return kLpVariants[variant].grouped[prec - 1](role, probs, items, n_items, n_blocks, s);
}

hipError_t launch_row_exponent(const double *X, long ldx, int rows, int ncols, int *e, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(row_exponent_kernel, dim3(rows), dim3(256), 0, s, X, ldx, ncols, e);
  return hipGetLastError();
}

hipError_t launch_split_rows_grouped(int prec, const SplitArgs *probs, const int2 *items, int n_items, int n_blocks,
                                     hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  switch (prec) {
    case 1:
      hipLaunchKernelGGL(split_rows_grouped_kernel<1>, dim3(n_blocks), dim3(256), 0, s, probs, items, n_items);
      break;
    case 2:
      hipLaunchKernelGGL(split_rows_grouped_kernel<2>, dim3(n_blocks), dim3(256), 0, s, probs, items, n_items);
      break;
    case 3:
      hipLaunchKernelGGL(split_rows_grouped_kernel<3>, dim3(n_blocks), dim3(256), 0, s, probs, items, n_items);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_split_rows(int prec, const double *X, long ldx, int rows, int ncols, const int *e, void *P,
                             long ldp, long plane_stride, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  dim3 grid((unsigned)((ldp + 255) / 256), rows);
  switch (prec) {
    case 1:
      hipLaunchKernelGGL(split_rows_kernel<1>, grid, dim3(256), 0, s, X, ldx, ncols, e, static_cast<float *>(P), ldp,
                         plane_stride);
      break;
    case 2:
      hipLaunchKernelGGL(split_rows_kernel<2>, grid, dim3(256), 0, s, X, ldx, ncols, e, static_cast<__bf16 *>(P),
                         ldp, plane_stride);
      break;
    case 3:
      hipLaunchKernelGGL(split_rows_kernel<3>, grid, dim3(256), 0, s, X, ldx, ncols, e,
                         static_cast<_Float16 *>(P), ldp, plane_stride);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace yyg
