// FP64 MFMA tile engine shared by the kernel sources: one block tile of
// C = A . B^T staged through LDS, and the kernels built on it (plain, strided
// batch, separable theta phases, grouped).  Included by yyg_kernels.hip and
// yyg_kernels_x4.hip; everything here is a template or internal.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "yyg_internal.h"

namespace yyg {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {

// x where keep holds, else 0, as an FP multiply by 1 or 0: the compiler
// cannot move the load of x under a branch on keep (x * 0 is NaN for a
// non-finite x), so the loads of a loop stay unconditional and in flight
// together.  x must be finite: it is read from a clamped, valid address.
__device__ __forceinline__ double keep_if(bool keep, double x) { return x * (keep ? 1.0 : 0.0); }

constexpr int kBK = 16, kPad = 2, kLDK = kBK + kPad;
// Stages of A and B held in registers ahead of the LDS stage being
// multiplied: a stage's global loads are issued kPF stages before its LDS
// store.  Measured on MI355X, three stages were slower than one for the
// long dense contractions (the registers cost occupancy); the short
// contractions of the separable form (K of a few stages) can ask for
// kDeepPF with the kGemmDeep mode bit, so that their loads are in flight
// together.
constexpr int kPF = 1, kDeepPF = 3;

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
// MODE bit 1 selects the general epilogue (column stride, degree-major
// column index); the plain one writes C[row * ldc + col].  The other bits
// change the operand layouts and the prefetch depth as documented with
// GemmF64Args.
template <int BM, int BN, int WGM, int WGN, int MODE>
__device__ __forceinline__ void gemm_f64_tile(const GemmF64Args &g, int tm, int tn, int z) {
  constexpr bool GEN = (MODE & 1) != 0;
  constexpr bool AT = (MODE & kGemmATrans) != 0;
  constexpr bool CT = (MODE & kGemmCTrans) != 0;
  constexpr bool BATCH = (MODE & kGemmBatch) != 0;
  constexpr bool BT = (MODE & kGemmBTrans) != 0;
  constexpr bool ACCINIT = (MODE & kGemmAccInit) != 0;
  constexpr bool FOLDA = (MODE & kGemmFoldA) != 0;
  constexpr bool FOLDAB = (MODE & kGemmFoldAB) != 0;
  constexpr bool FLD = FOLDA || FOLDAB;  // the loads keep front and mirror values
  constexpr bool FOLDC = (MODE & kGemmFoldC) != 0;
  constexpr bool DT = (MODE & kGemmDT) != 0;
  constexpr bool X4 = (MODE & kGemmX4) != 0;
  constexpr bool LPF32 = (MODE & kGemmLpF32) != 0;
  constexpr bool LPBF3 = (MODE & kGemmLpBF3) != 0;
  constexpr bool LP = LPF32 || LPBF3;
  constexpr bool XCOL = (MODE & kGemmXCol) != 0;
  static_assert(!ACCINIT || GEN, "the initial accumulator is addressed like C");
  static_assert(!LP || (!X4 && !FOLDAB && !ACCINIT && !(LPF32 && LPBF3)), "reduced precision: the 16x16 phi forms");
  static_assert(!DT || !FOLDC, "the folded synthesis stores rows");
  static_assert(!FOLDA || (BATCH && CT && !AT && !GEN), "folded analysis: batched, row-major A, C column-major");
  static_assert(!FOLDC || (BATCH && AT && !CT && !GEN), "folded synthesis: batched, A k-major");
  static_assert(!FOLDAB || (BATCH && CT && !AT && !GEN && !FOLDA && (X4 ? !DT : DT)),
                "both folded halves: batched, row-major A, C column-major, rows on the coalesced side");

  const int M = g.M, N = g.N, K = g.K;
  // FOLDA: problem z = 2 zj + group (group 0 the even, 1 the odd half), so
  // that the two halves of a row tile run close together and share L2
  const int fgrp = FOLDA ? (z & 1) : 0;
  const int zj = FOLDA ? (z >> 1) : z;
  const double fsign = fgrp ? -1.0 : 1.0;
  const double *__restrict__ A = g.A + (BATCH ? zj * g.a_batch : 0L);
  const double *__restrict__ B = g.B + (BATCH ? z * g.b_batch : 0L);
  double *__restrict__ C = g.C;
  const long lda = g.lda, ldb = g.ldb, ldc = g.ldc;
  constexpr int NT = 64 * WGM * WGN;
  constexpr int TI = BM / WGM / 16, TJ = BN / WGN / 16;
  static_assert(!XCOL || (FOLDA && !X4 && !LP && NT % BM == 0 && kBK % (NT / BM) == 0),
                "extra column: folded analysis FP64 16x16 tiles, whole threads per row");
  static_assert(TI >= 1 && TJ >= 1 && TI * 16 * WGM == BM && TJ * 16 * WGN == BN, "tile/wave mismatch");
  // X4 (v_mfma_f64_4x4x4f64): the wave tile as R4 four-wide by S16
  // sixteen-wide products; the four-wide side is M (N with DT).
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int R4 = X4 ? (DT ? WN : WM) / 4 : 1, S16 = X4 ? (DT ? WM : WN) / 16 : 1;
  // Stage loads.  When a thread's share of a tile stage divides the 16-wide
  // stage, it reads one contiguous run of k in one row (one row pointer);
  // otherwise element e = tid + i*NT sits at row e / 16, column e % 16.
  // An operand stored k-major loads along m (n) instead: element
  // e = tid + i*NT at k = e / BM, m = e % BM.
  constexpr bool RUN_A = !AT && (BM * kBK) % NT == 0 && kBK % ((BM * kBK) / NT) == 0;
  constexpr bool RUN_B = !BT && (BN * kBK) % NT == 0 && kBK % ((BN * kBK) / NT) == 0;
  constexpr int EA = RUN_A ? (BM * kBK) / NT : (BM * kBK + NT - 1) / NT;
  constexpr int EB = RUN_B ? (BN * kBK) / NT : (BN * kBK + NT - 1) / NT;
  __shared__ double As[LP ? 1 : 2][LP ? 1 : BM * kLDK];
  __shared__ double Ao[FOLDAB ? 2 : 1][FOLDAB ? BM * kLDK : 1];  // FOLDAB: the odd half of A
  __shared__ double Bs[LP ? 1 : 2][LP ? 1 : BN * kLDK];
  // reduced precisions: the stages as FP32 values, or as three BF16 planes
  // (bit patterns) with rows of kLDH
  constexpr int kLDH = kBK + 4;
  __shared__ float AsF[LPF32 ? 2 : 1][LPF32 ? BM * kLDK : 1];
  __shared__ float BsF[LPF32 ? 2 : 1][LPF32 ? BN * kLDK : 1];
  __shared__ __attribute__((aligned(16))) short AsH[LPBF3 ? 2 : 1][LPBF3 ? 3 : 1][LPBF3 ? BM * kLDH : 1];
  __shared__ __attribute__((aligned(16))) short BsH[LPBF3 ? 2 : 1][LPBF3 ? 3 : 1][LPBF3 ? BN * kLDH : 1];
  // store one stage element (row, column within the stage) of A / B
  auto bf16_bits = [](double x) -> short {
    // round to nearest even of the FP32 rounding of x (|x| within FP32's
    // range; the remainders of a split are exact in FP64)
    const float f = (float)x;
    unsigned u = __builtin_bit_cast(unsigned, f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
  };
  auto bf16_val = [](short h) -> double {
    return (double)__builtin_bit_cast(float, (unsigned)(unsigned short)h << 16);
  };
  auto put = [&](auto &F64, auto &F32, auto &H, int buf, int row, int col, double v) {
    if constexpr (LPF32) {
      F32[buf][row * kLDK + col] = (float)v;
    } else if constexpr (LPBF3) {
      const short h0 = bf16_bits(v);
      const double r1 = v - bf16_val(h0);
      const short h1 = bf16_bits(r1);
      const short h2 = bf16_bits(r1 - bf16_val(h1));
      H[buf][0][row * kLDH + col] = h0;
      H[buf][1][row * kLDH + col] = h1;
      H[buf][2][row * kLDH + col] = h2;
    } else {
      F64[buf][row * kLDK + col] = v;
    }
  };
  auto putA = [&](int buf, int row, int col, double v) { put(As, AsF, AsH, buf, row, col, v); };
  auto putB = [&](int buf, int row, int col, double v) { put(Bs, BsF, BsH, buf, row, col, v); };

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = tm * BM, n0 = tn * BN;
  // z is the split-K slice, or with BATCH the problem of a strided batch
  const int kbeg = BATCH ? 0 : z * g.k_per_split;
  const int kend = BATCH ? K : min(K, kbeg + g.k_per_split);
  C += (long)zj * g.c_split_stride;

  const int wm = wave % WGM, wn = wave / WGM;

  // XCOL: output column nx = n0 + BN (active when it is N - 1, uniform over
  // the block): XTPR threads per row of the tile each sum XSPT of a stage's
  // 16 contraction points, from A's stage in LDS and the column's basis
  // values staged beside it
  constexpr int XTPR = XCOL ? NT / BM : 1, XSPT = kBK / XTPR;
  __shared__ double Bx[XCOL ? 2 : 1][XCOL ? kBK : 1];
  const int nx = n0 + BN;
  const bool xon = XCOL && nx == N - 1;
  const int xr = tid / XTPR, xq = tid % XTPR;
  double xacc = 0.0;

  // FOLDC: acc sums the stages below k_split (the even part), acc2 the rest
  // (acc4 / acc4b in the X4 form: one value per lane and product)
  constexpr int TIa = X4 ? 1 : TI, TJa = X4 ? 1 : TJ;
  dbl4 acc[TIa][TJa], acc2[FOLDC ? TIa : 1][FOLDC ? TJa : 1];
  double acc4[R4][S16], acc4b[FOLDC ? R4 : 1][FOLDC ? S16 : 1];
#pragma unroll
  for (int i = 0; i < TIa; ++i)
#pragma unroll
    for (int j = 0; j < TJa; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  if constexpr (FOLDC) {
#pragma unroll
    for (int i = 0; i < TIa; ++i)
#pragma unroll
      for (int j = 0; j < TJa; ++j) acc2[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  }
#pragma unroll
  for (int r = 0; r < R4; ++r)
#pragma unroll
    for (int c = 0; c < S16; ++c) acc4[r][c] = 0.0;
  if constexpr (FOLDC) {
#pragma unroll
    for (int r = 0; r < R4; ++r)
#pragma unroll
      for (int c = 0; c < S16; ++c) acc4b[r][c] = 0.0;
  }
  // X4 lane roles: lane = 16 xu + 4 xb + xv; product (r, c) of a wave holds
  // the four-wide index 4 r + xu and the sixteen-wide index 16 c + 4 xb + xv
  const int xu = lane >> 4, xb = (lane >> 2) & 3, xv = lane & 3;
  auto x4_row = [&](int r, int c) {
    return m0 + wm * WM + (DT ? 16 * c + 4 * xb + xv : 4 * r + xu);
  };
  auto x4_col = [&](int r, int c) {
    return n0 + wn * WN + (DT ? 4 * r + xu : 16 * c + 4 * xb + xv);
  };
  if constexpr (ACCINIT && X4) {
#pragma unroll
    for (int r = 0; r < R4; ++r)
#pragma unroll
      for (int c = 0; c < S16; ++c) {
        const int row = x4_row(r, c), col = x4_col(r, c);
        const double v = g.Cin[(long)min(row, M - 1) * ldc + (long)min(col, N - 1) * g.ldc_c];
        acc4[r][c] = (row < M && col < N) ? v : 0.0;
      }
  } else if constexpr (ACCINIT) {
    // start from Cin, element by element in the D layout of the epilogue
    // (clamped addresses; entries outside the matrix start at zero)
    const int ln = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < TIa; ++i)
#pragma unroll
      for (int j = 0; j < TJa; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + (wv % WGM) * (BM / WGM) + i * 16 + (DT ? (ln & 15) : (ln >> 4) + 4 * r);
          const int col = n0 + (wv / WGM) * (BN / WGN) + j * 16 + (DT ? (ln >> 4) + 4 * r : (ln & 15));
          const double v = g.Cin[(long)min(row, M - 1) * ldc + (long)min(col, N - 1) * g.ldc_c];
          acc[i][j][r] = (row < M && col < N) ? v : 0.0;
        }
  }

  constexpr int PF = (MODE & kGemmDeep) ? kDeepPF : kPF;
  // FOLDA keeps the raw front and mirror values (ra[i], ra[EA + i]) until
  // the stash: folding them at load time would wait for the loads there
  constexpr int EAR = FLD ? 2 * EA : EA;
  double ra[PF][EAR], rb[PF][EB], rx[PF];
  // run mapping: this thread's row and first column
  const int arow = RUN_A ? tid / (kBK / EA) : 0, acol = RUN_A ? (tid % (kBK / EA)) * EA : 0;
  const int brow = RUN_B ? tid / (kBK / EB) : 0, bcol = RUN_B ? (tid % (kBK / EB)) * EB : 0;
  const double *pa = A + (long)min(m0 + arow, M - 1) * lda;
  const double *pb = B + (long)min(n0 + brow, N - 1) * ldb;
  const bool va = m0 + arow < M, vb = n0 + brow < N;
  // load: every global load reads a clamped, valid address (a load under a
  // condition would be waited for before the next one issues); stash: the
  // entries outside the matrix or the stage's k range are zeroed on the way
  // into LDS, after the stage's MFMA work, so the loads overlap it.
  // FOLDA: A(m, k) = X(m, k) + sign X(m, fold_k - 1 - k), the even (odd)
  // half of a row about its middle
  auto aload = [&](double (&ra)[EAR], int i, const double *row, int kc) {
    ra[i] = row[kc];
    if constexpr (FLD) ra[EA + i] = row[g.fold_k - 1 - kc];
  };
  // FOLDA, a run of EA (even) values per thread: pairs of neighbours as one
  // 16-byte load each at the front and at the mirror.  K = h < fold_k, so a
  // pair starting at a clamped kc <= K - 1 stays inside the row on both sides
  // (its second value, past K, is zeroed at the stash like every value past K).
  typedef double dbl2u __attribute__((ext_vector_type(2), aligned(8)));
  auto apairs = [&](double (&ra)[EAR], const double *row, int k0) {
#pragma unroll
    for (int i = 0; i < EA; i += 2) {
      const int kc = min(k0 + acol + i, K - 1);
      const dbl2u f = *reinterpret_cast<const dbl2u *>(row + kc);
      const dbl2u b = *reinterpret_cast<const dbl2u *>(row + (g.fold_k - 2 - kc));
      ra[i] = f.x;
      ra[i + 1] = f.y;
      ra[EA + i] = b.y;
      ra[EA + i + 1] = b.x;
    }
  };
  auto aval = [&](const double (&ra)[EAR], int i) { return FLD ? ra[i] + fsign * ra[(FLD ? EA : 0) + i] : ra[i]; };
  // FOLDAB: the odd half, front minus mirror
  auto aval_o = [&](const double (&ra)[EAR], int i) { return FLD ? ra[i] - ra[(FLD ? EA : 0) + i] : ra[i]; };
  auto load = [&](double (&ra)[EAR], double (&rb)[EB], int k0) {
    if constexpr (RUN_A && FLD && EA % 2 == 0) {
      apairs(ra, pa, k0);
    } else if constexpr (RUN_A) {
#pragma unroll
      for (int i = 0; i < EA; ++i) aload(ra, i, pa, min(k0 + acol + i, K - 1));
    } else if constexpr (AT) {
#pragma unroll
      for (int i = 0; i < EA; ++i) {
        const int e = tid + i * NT, gm = m0 + e % BM;
        int kc = min(k0 + e / BM, K - 1);
        if constexpr (FOLDC) {
          // contraction index -> azimuthal column: cos m at k = m, sin m at
          // k_split + m - 1 (padding clamps; its basis entries are zero)
          kc = min(kc < g.k_split ? max(2 * kc - 1, 0) : 2 * (kc - g.k_split) + 2, g.fold_mc - 1);
        }
        ra[i] = A[(long)kc * lda + min(gm, M - 1)];
      }
    } else {
#pragma unroll
      for (int i = 0; i < EA; ++i) {
        const int e = tid + i * NT, row = e / kBK, kk = k0 + e % kBK;
        aload(ra, i, A + (long)min(m0 + row, M - 1) * lda, min(kk, K - 1));
      }
    }
    if constexpr (RUN_B) {
#pragma unroll
      for (int i = 0; i < EB; ++i) rb[i] = pb[min(k0 + bcol + i, K - 1)];
    } else if constexpr (BT) {
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int e = tid + i * NT, kk = k0 + e / BN, gn = n0 + e % BN;
        rb[i] = B[(long)min(kk, K - 1) * ldb + min(gn, N - 1)];
      }
    } else {
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int e = tid + i * NT, row = e / kBK, kk = k0 + e % kBK;
        rb[i] = B[(long)min(n0 + row, N - 1) * ldb + min(kk, K - 1)];
      }
    }
  };
  auto stash = [&](const double (&ra)[EAR], const double (&rb)[EB], int buf, int k0) {
    if constexpr (RUN_A) {
#pragma unroll
      for (int i = 0; i < EA; ++i) {
        const bool ok = va && k0 + acol + i < kend;
        putA(buf, arow, acol + i, ok ? aval(ra, i) : 0.0);
        if constexpr (FOLDAB) Ao[FOLDAB ? buf : 0][arow * kLDK + acol + i] = ok ? aval_o(ra, i) : 0.0;
      }
    } else if constexpr (AT) {
#pragma unroll
      for (int i = 0; i < EA; ++i) {
        const int e = tid + i * NT, kk = k0 + e / BM, gm = m0 + e % BM;
        if (e < BM * kBK) putA(buf, e % BM, e / BM, (gm < M && kk < kend) ? ra[i] : 0.0);
      }
    } else {
#pragma unroll
      for (int i = 0; i < EA; ++i) {
        const int e = tid + i * NT, row = e / kBK, kk = k0 + e % kBK;
        if (e < BM * kBK) {
          const bool ok = m0 + row < M && kk < kend;
          putA(buf, row, e % kBK, ok ? aval(ra, i) : 0.0);
          if constexpr (FOLDAB) Ao[FOLDAB ? buf : 0][row * kLDK + e % kBK] = ok ? aval_o(ra, i) : 0.0;
        }
      }
    }
    if constexpr (RUN_B) {
#pragma unroll
      for (int i = 0; i < EB; ++i) putB(buf, brow, bcol + i, (vb && k0 + bcol + i < kend) ? rb[i] : 0.0);
    } else if constexpr (BT) {
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int e = tid + i * NT, kk = k0 + e / BN, gn = n0 + e % BN;
        if (e < BN * kBK) putB(buf, e % BN, e / BN, (gn < N && kk < kend) ? rb[i] : 0.0);
      }
    } else {
#pragma unroll
      for (int i = 0; i < EB; ++i) {
        const int e = tid + i * NT, row = e / kBK, kk = k0 + e % kBK;
        if (e < BN * kBK) putB(buf, row, e % kBK, (n0 + row < N && kk < kend) ? rb[i] : 0.0);
      }
    }
  };

  // XCOL: every thread loads (a clamped, valid address); the first kBK
  // store the stage's basis values of column nx
  auto xload = [&](double &x, int k0) {
    if constexpr (XCOL) x = B[(long)min(nx, N - 1) * ldb + min(k0 + (tid & (kBK - 1)), K - 1)];
  };
  auto xstash = [&](double x, int buf, int k0) {
    if constexpr (XCOL) {
      if (tid < kBK) Bx[XCOL ? buf : 0][tid] = (xon && k0 + tid < kend) ? x : 0.0;
    }
  };
  auto xcompute = [&](int buf) {
    if constexpr (XCOL) {
      if (xon) {  // uniform
        const double *ap = &As[buf][xr * kLDK + xq * XSPT];
        const double *bx = &Bx[XCOL ? buf : 0][xq * XSPT];
#pragma unroll
        for (int s = 0; s < XSPT; ++s) xacc = __builtin_fma(ap[s], bx[s], xacc);
      }
    }
  };

  const int frow = lane & 15, fk = 4 * (lane >> 4);
  // X4: at step s lane (xu, xb, xv) supplies row 4 r + xv of the four-wide
  // side (the same in each block) and row 16 c + 4 xb + xv of the
  // sixteen-wide side, both at contraction index 4 xu + s of the stage, so
  // the four steps cover the 16 k once, as in the 16 x 16 path.
  auto compute4 = [&](int buf, bool second) {
    const double *__restrict__ s4p = DT ? Bs[buf] : As[buf];
    const double *__restrict__ s16p = DT ? As[buf] : Bs[buf];
    const double *__restrict__ s4o = Ao[FOLDAB ? buf : 0];
    const int b4 = DT ? wn * WN : wm * WM, b16 = DT ? wm * WM : wn * WN;
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      double rf[R4], sf[S16], ro[FOLDAB ? R4 : 1];
#pragma unroll
      for (int r = 0; r < R4; ++r) rf[r] = s4p[(b4 + 4 * r + xv) * kLDK + 4 * xu + s4];
      if constexpr (FOLDAB) {
#pragma unroll
        for (int r = 0; r < R4; ++r) ro[FOLDAB ? r : 0] = s4o[(b4 + 4 * r + xv) * kLDK + 4 * xu + s4];
      }
#pragma unroll
      for (int c = 0; c < S16; ++c) sf[c] = s16p[(b16 + 16 * c + 4 * xb + xv) * kLDK + 4 * xu + s4];
      if (FOLDC && second) {  // uniform: the whole stage is past k_split
#pragma unroll
        for (int r = 0; r < R4; ++r)
#pragma unroll
          for (int c = 0; c < S16; ++c)
            acc4b[FOLDC ? r : 0][FOLDC ? c : 0] =
                __builtin_amdgcn_mfma_f64_4x4x4f64(rf[r], sf[c], acc4b[FOLDC ? r : 0][FOLDC ? c : 0], 0, 0, 0);
      } else {
#pragma unroll
        for (int r = 0; r < R4; ++r)
#pragma unroll
          for (int c = 0; c < S16; ++c) {
            // FOLDAB: slot tiles at or past k_split are the odd half (uniform)
            const double a = (FOLDAB && n0 + b16 + 16 * c >= g.k_split) ? ro[FOLDAB ? r : 0] : rf[r];
            acc4[r][c] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, sf[c], acc4[r][c], 0, 0, 0);
          }
      }
    }
  };
  auto compute16 = [&](int buf, bool second) {
    // Each lane holds four consecutive k of its row; MFMA step s uses the
    // s-th of them, so the four steps cover the 16 k of the stage once.
    double af[TIa][4], bf[TJa][4], ao[FOLDAB ? TIa : 1][4];
#pragma unroll
    for (int i = 0; i < TIa; ++i) {
      const double *sp = &As[buf][(wm * (BM / WGM) + i * 16 + frow) * kLDK + fk];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) af[i][s4] = sp[s4];
      if constexpr (FOLDAB) {
        const double *so = &Ao[FOLDAB ? buf : 0][(wm * (BM / WGM) + i * 16 + frow) * kLDK + fk];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) ao[FOLDAB ? i : 0][s4] = so[s4];
      }
    }
#pragma unroll
    for (int j = 0; j < TJa; ++j) {
      const double *sp = &Bs[buf][(wn * (BN / WGN) + j * 16 + frow) * kLDK + fk];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) bf[j][s4] = sp[s4];
    }
    if (FOLDC && second) {  // uniform: the whole stage is past k_split
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int i = 0; i < TIa; ++i)
#pragma unroll
          for (int j = 0; j < TJa; ++j)
            acc2[FOLDC ? i : 0][FOLDC ? j : 0] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                af[i][s4], bf[j][s4], acc2[FOLDC ? i : 0][FOLDC ? j : 0], 0, 0, 0);
    } else {
      // DT: the transposed tile B A^T, so that a store covers 16 rows
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int i = 0; i < TIa; ++i)
#pragma unroll
          for (int j = 0; j < TJa; ++j) {
            // FOLDAB: column tiles at or past k_split take the odd half (uniform)
            const double a = (FOLDAB && n0 + wn * (BN / WGN) + 16 * j >= g.k_split) ? ao[FOLDAB ? i : 0][s4]
                                                                                    : af[i][s4];
            acc[i][j] = DT ? __builtin_amdgcn_mfma_f64_16x16x4f64(bf[j][s4], a, acc[i][j], 0, 0, 0)
                           : __builtin_amdgcn_mfma_f64_16x16x4f64(a, bf[j][s4], acc[i][j], 0, 0, 0);
          }
    }
  };
  // reduced precisions: FP32-accumulating 16x16 MFMAs over the stage, then
  // the stage's sums added to the FP64 accumulators (D layout of these
  // MFMAs: lane l, element r -> row 4 (l/16) + r, col l % 16; DT swaps)
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  typedef short s16x4 __attribute__((ext_vector_type(4)));
  auto compute_lp = [&](int buf, bool second) {
    f32x4 lacc[TIa][TJa];
#pragma unroll
    for (int i = 0; i < TIa; ++i)
#pragma unroll
      for (int j = 0; j < TJa; ++j) lacc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (LPF32) {
      float af[TIa][4], bf[TJa][4];
#pragma unroll
      for (int i = 0; i < TIa; ++i)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) af[i][s4] = AsF[buf][(wm * (BM / WGM) + i * 16 + frow) * kLDK + fk + s4];
#pragma unroll
      for (int j = 0; j < TJa; ++j)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) bf[j][s4] = BsF[buf][(wn * (BN / WGN) + j * 16 + frow) * kLDK + fk + s4];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int i = 0; i < TIa; ++i)
#pragma unroll
          for (int j = 0; j < TJa; ++j)
            lacc[i][j] = DT ? __builtin_amdgcn_mfma_f32_16x16x4f32(bf[j][s4], af[i][s4], lacc[i][j], 0, 0, 0)
                            : __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][s4], bf[j][s4], lacc[i][j], 0, 0, 0);
    } else if constexpr (LPBF3) {
      // each lane's four consecutive k of its row are one 16x16x16 operand
      s16x4 ah[TIa][3], bh[TJa][3];
#pragma unroll
      for (int i = 0; i < TIa; ++i)
#pragma unroll
        for (int p = 0; p < 3; ++p)
          ah[i][p] = *reinterpret_cast<const s16x4 *>(&AsH[buf][p][(wm * (BM / WGM) + i * 16 + frow) * kLDH + fk]);
#pragma unroll
      for (int j = 0; j < TJa; ++j)
#pragma unroll
        for (int p = 0; p < 3; ++p)
          bh[j][p] = *reinterpret_cast<const s16x4 *>(&BsH[buf][p][(wn * (BN / WGN) + j * 16 + frow) * kLDH + fk]);
#pragma unroll
      for (int i = 0; i < TIa; ++i)
#pragma unroll
        for (int j = 0; j < TJa; ++j)
          // part pairs (pa, pb) of order pa + pb < 3, smallest terms first
#pragma unroll
          for (int ord = 2; ord >= 0; --ord)
#pragma unroll
            for (int pa = 0; pa <= ord; ++pa)
              lacc[i][j] = DT ? __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(bh[j][ord - pa], ah[i][pa], lacc[i][j], 0, 0, 0)
                              : __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i][pa], bh[j][ord - pa], lacc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < TIa; ++i)
#pragma unroll
      for (int j = 0; j < TJa; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (FOLDC && second)
            acc2[FOLDC ? i : 0][FOLDC ? j : 0][r] += (double)lacc[i][j][r];
          else
            acc[i][j][r] += (double)lacc[i][j][r];
        }
  };
  auto compute = [&](int buf, bool second) {
    if constexpr (X4)
      compute4(buf, second);
    else if constexpr (LP)
      compute_lp(buf, second);
    else
      compute16(buf, second);
  };

  const int nk = (kend - kbeg + kBK - 1) / kBK;
#pragma unroll
  for (int p = 0; p < PF; ++p)
    if (p < nk) {
      load(ra[p], rb[p], kbeg + p * kBK);
      xload(rx[p], kbeg + p * kBK);
    }
  if (nk > 0) {
    stash(ra[0], rb[0], 0, kbeg);
    xstash(rx[0], 0, kbeg);
  }
  __syncthreads();

  // Stage `it` sits in LDS buffer it & 1 and register slot it % PF; the
  // loop is unrolled by PF so that every slot index is a constant.  With
  // PF = 1 the stage loaded this iteration is the one stored after it.
  // Steady state first, where every step refills its slot: no condition
  // around the loads, so that each slot is refilled in its own registers
  // and the stash waits for its own stage only (not for the later stages
  // in flight); then the last stages with their conditions.
  int base0 = 0;
  for (; base0 + 2 * PF - 1 < nk; base0 += PF) {
#pragma unroll
    for (int sl = 0; sl < PF; ++sl) {
      const int it = base0 + sl, buf = it & 1;
      __builtin_amdgcn_sched_barrier(0);
      load(ra[sl], rb[sl], kbeg + (it + PF) * kBK);
      xload(rx[sl], kbeg + (it + PF) * kBK);
      compute(buf, FOLDC && kbeg + it * kBK >= g.k_split);
      xcompute(buf);
      stash(ra[(sl + 1) % PF], rb[(sl + 1) % PF], buf ^ 1, kbeg + (it + 1) * kBK);
      xstash(rx[(sl + 1) % PF], buf ^ 1, kbeg + (it + 1) * kBK);
      __syncthreads();
    }
  }
  for (int base = base0; base < nk; base += PF) {
#pragma unroll
    for (int sl = 0; sl < PF; ++sl) {
      const int it = base + sl;
      if (it < nk) {  // uniform across the block
        const int buf = it & 1;
        if (it + PF < nk) {
          load(ra[sl], rb[sl], kbeg + (it + PF) * kBK);
          xload(rx[sl], kbeg + (it + PF) * kBK);
        }
        compute(buf, FOLDC && kbeg + it * kBK >= g.k_split);
        xcompute(buf);
        if (it + 1 < nk) {
          stash(ra[(sl + 1) % PF], rb[(sl + 1) % PF], buf ^ 1, kbeg + (it + 1) * kBK);
          xstash(rx[(sl + 1) % PF], buf ^ 1, kbeg + (it + 1) * kBK);
        }
        __syncthreads();
      }
    }
  }

  // store one output element (and, FOLDC, its odd part) in C's layout
  auto emit = [&](int row, int col, double v, double v2) {
    if (row < M && col < N) {
      if constexpr (GEN) {
        const long cc = g.c_sq < 0 ? (long)col : (long)(col + g.c_sq) * (col + g.c_sq);
        C[(long)row * ldc + cc * g.ldc_c] = v;
      } else if constexpr (FOLDA) {
        // output column -> azimuthal column: cos m (group 0, col m), sin m
        // (group 1, col m - 1)
        const int mc = max(2 * col + (fgrp ? 2 : -1), 0);
        if (mc < g.fold_mc) C[(long)mc * ldc + row] = v;
      } else if constexpr (FOLDAB) {
        // slot -> azimuthal column: cos m at slot m, sin m at k_split + m - 1
        const int mc = col < g.k_split ? max(2 * col - 1, 0) : 2 * (col - g.k_split) + 2;
        if (mc < g.fold_mc) C[(long)mc * ldc + row] = v;
      } else if constexpr (CT) {
        C[(long)col * ldc + row] = v;
      } else if constexpr (FOLDC) {
        // the even part plus / minus the odd part, at col and its mirror
        const int cm = g.fold_k - 1 - col;
        C[(long)row * ldc + col] = v + v2;
        if (cm != col) C[(long)row * ldc + cm] = v - v2;
      } else {
        C[(long)row * ldc + col] = v;
      }
    }
  };
  if constexpr (XCOL) {
    if (xon) {  // uniform: the row's partial sums meet in its first thread
#pragma unroll
      for (int o = 1; o < XTPR; o <<= 1) xacc += __shfl_xor(xacc, o);
      if (xq == 0) emit(m0 + xr, nx, xacc, 0.0);
    }
  }
  if constexpr (X4) {
#pragma unroll
    for (int r = 0; r < R4; ++r)
#pragma unroll
      for (int c = 0; c < S16; ++c) emit(x4_row(r, c), x4_col(r, c), acc4[r][c], FOLDC ? acc4b[FOLDC ? r : 0][FOLDC ? c : 0] : 0.0);
    return;
  }
  // D layout of the 16x16x4 f64 MFMA: lane l, element r -> row l/16 + 4r,
  // col l%16 (one row per output group, unlike the f32 variant's four);
  // with DT the roles of row and column swap.
  const int orow = lane >> 4, ocol = lane & 15;
#pragma unroll
  for (int i = 0; i < TIa; ++i) {
#pragma unroll
    for (int j = 0; j < TJa; ++j) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // FP64 MFMA: row l/16 + 4r; FP32-accumulating (LP): row 4 (l/16) + r
        const int dr = LP ? 4 * orow + r : orow + 4 * r;
        const int row = m0 + wm * (BM / WGM) + i * 16 + (DT ? ocol : dr);
        const int col = n0 + wn * (BN / WGN) + j * 16 + (DT ? dr : ocol);
        emit(row, col, acc[i][j][r], FOLDC ? acc2[FOLDC ? i : 0][FOLDC ? j : 0][r] : 0.0);
      }
    }
  }
}

// ROLE only separates the analysis (0) and synthesis (1) instantiations so
// that profilers list them apart.
template <int ROLE, int BM, int BN, int WGM, int WGN, int MODE = 0>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_nt_f64_kernel(GemmF64Args g, int tiles_total) {
  const int tile = xcd_tile(blockIdx.x, tiles_total);
  gemm_f64_tile<BM, BN, WGM, WGN, MODE>(g, tile % g.tiles_m, tile / g.tiles_m, blockIdx.y);
}

// Strided batch of equal-shape problems, one block per (problem, tile),
// problem-major after the XCD remapping.
template <int ROLE, int BM, int BN, int WGM, int WGN, int MODE>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_nt_f64_batched(GemmF64Args g, int per_problem,
                                                                      int tiles_total) {
  const int t = xcd_tile(blockIdx.x, tiles_total);
  int z, tile;
  if constexpr ((MODE & kGemmFoldA) != 0) {
    // the even and odd halves (z = 2 j, 2 j + 1) of one row tile back to
    // back on one XCD: the second reads the same density rows from its L2
    const int u = t >> 1, zj = u / per_problem;
    tile = u - zj * per_problem;
    z = 2 * zj + (t & 1);
  } else {
    z = t / per_problem;
    tile = t - z * per_problem;
  }
  if constexpr ((MODE & kGemmNFast) != 0) {
    const int tiles_n = per_problem / g.tiles_m;
    gemm_f64_tile<BM, BN, WGM, WGN, MODE | kGemmBatch>(g, tile / tiles_n, tile % tiles_n, z);
  } else {
    gemm_f64_tile<BM, BN, WGM, WGN, MODE | kGemmBatch>(g, tile % g.tiles_m, tile / g.tiles_m, z);
  }
}

// The theta phases and the moment rotation of the separable form: one
// problem per blockIdx.z, its shapes and operands derived from the phase
// arguments (no descriptor loads ahead of the operand loads).
//  PHASE 1, theta analysis, z = mc (m = (mc + 1) / 2): the column-major
//    moments A[(l^2 + mc)][row] = sum_j X2[mc][j][row] T2[mc][l][j], l >= m.
//  PHASE 2, rotation, z = 2 (L - l) + p: At[l^2 + b][p nR + n] =
//    A_own(n, b) + sum_{k < d} A_other(n, k) D_l[k][b], d = 2l + 1, with
//    A_own / A_other this / the other patch's rows of degree l's columns;
//    the accumulators start from A_own (kGemmAccInit).
//  PHASE 3, theta synthesis, z = mc: V[mc][j][row] =
//    sum_{l >= m} P2[mc][j][l] Ut[mc][l][row].
template <int PHASE>
__device__ __forceinline__ GemmF64Args sep_problem(const SepPhaseArgs &a, int z) {
  const long Mr = (long)a.P * a.nR, MJ = Mr * a.nt;
  GemmF64Args g{};
  if constexpr (PHASE == 1) {
    const int mc = z, m = (mc + 1) >> 1;
    g.M = (int)Mr;
    g.N = a.L + 1 - m;
    g.K = a.nt;
    g.A = a.X2 + mc * MJ;
    g.lda = Mr;
    g.B = a.T2 + ((long)mc * (a.L + 1) + m) * a.nt;
    g.ldb = a.nt;
    g.C = a.Ahat + mc * Mr;
    g.ldc = 1;
    g.ldc_c = Mr;
    g.c_sq = m;
  } else if constexpr (PHASE == 2) {
    const int l = a.L - (z >> 1), p = z & 1, d = 2 * l + 1;
    g.M = a.nR;
    g.N = d;
    g.K = d;
    g.A = a.Ahat + (long)l * l * Mr + (long)(1 - p) * a.nR;  // the other patch's rows
    g.lda = Mr;
    g.B = a.D + (long)l * (4 * (long)l * l - 1) / 3;  // D_l after the blocks of degrees below l
    g.ldb = d;
    g.C = a.At + (long)l * l * Mr + (long)p * a.nR;
    g.Cin = a.Ahat + (long)l * l * Mr + (long)p * a.nR;  // this patch's own moments
    g.ldc = 1;
    g.ldc_c = Mr;
  } else {
    const int mc = z, m = (mc + 1) >> 1;
    g.M = a.nt;
    g.N = (int)Mr;
    g.K = a.L + 1 - m;
    g.A = a.P2 + (long)mc * a.nt * a.ldl + m;
    g.lda = a.ldl;
    g.B = a.Ut + ((long)mc * (a.L + 1) + m) * Mr;
    g.ldb = Mr;
    g.C = a.V + mc * MJ;
    g.ldc = Mr;
  }
  g.k_per_split = (g.K + kBK - 1) / kBK * kBK;
  g.tiles_m = 1;
  return g;
}

template <int PHASE, int BM, int BN, int WGM, int WGN, int MODE>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_f64_sep_phase(SepPhaseArgs a) {
  const GemmF64Args g = sep_problem<PHASE>(a, blockIdx.z);
  if ((int)blockIdx.x * BM >= g.M || (int)blockIdx.y * BN >= g.N) return;  // uniform: past this problem's tiles
  gemm_f64_tile<BM, BN, WGM, WGN, MODE>(g, blockIdx.x, blockIdx.y, 0);
}

// The same over the problems of several plans (batched separable solves):
// blocks walk work items (plan, tile row, tile column, problem z).
template <int PHASE, int BM, int BN, int WGM, int WGN, int MODE>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_f64_sep_grouped(const SepPhaseArgs *__restrict__ args,
                                                                       const int4 *__restrict__ items, int n_items) {
  for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
    const int4 it = items[w];
    __syncthreads();  // the previous item's LDS reads are done
    const GemmF64Args g = sep_problem<PHASE>(args[it.x], it.w);
    gemm_f64_tile<BM, BN, WGM, WGN, MODE>(g, it.y, it.z, 0);
  }
}

// Persistent grouped form: blocks walk a list of (problem, tm, tn, split)
// work items over several independent contractions of one phase.
template <int ROLE, int BM, int BN, int WGM, int WGN, int MODE>
__global__ __launch_bounds__(64 * WGM * WGN) void gemm_nt_f64_grouped(const GemmF64Args *__restrict__ probs,
                                                                      const int4 *__restrict__ items, int n_items) {
  for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
    const int4 it = items[w];
    __syncthreads();  // the previous item's LDS reads are done
    gemm_f64_tile<BM, BN, WGM, WGN, MODE>(probs[it.x], it.y, it.z, it.w);
  }
}

}  // namespace yyg
