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

#include <algorithm>
#include <climits>
#include <cstdio>

#include "yyg_internal.h"
#include "yyg_tile.h"

namespace yyg {

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
  // reduced moments for the later passes: the copy in Ahat, or the single
  // partial buffer itself when no copy is kept (nsplit == 1 then)
  const double *__restrict__ Ared = Ahat ? Ahat : part;

  double I = 0.0, Pa = 1.0;
  if (ok) {
#pragma unroll 4
    for (int n = n0; n < n1; ++n) {
      const long row = rbase + n;
      double a = 0.0;
      for (int z = 0; z < nsplit; ++z) a += part[z * split_stride + row * Q + qq];
      if (Ahat) Ahat[row * Q + qq] = a;
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
      const double an = (n + 1 < nR) ? Ared[(rbase + n + 1) * Q + qq] : 0.0;
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
    I = c[0] * I + c[1] * Ared[(rbase + n) * Q + q];
    U[(rbase + n) * ldu + q] = I;
  }
  O = Oin;
#pragma unroll 4
  for (int n = n1 - 1; n >= n0; --n) {
    const double *c = cf + n * cstride;
    const double an = (n + 1 < nR) ? Ared[(rbase + n + 1) * Q + q] : 0.0;
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
  // the outer recurrence); zero beyond the grid.  Every load goes to a
  // clamped, valid address and is masked afterwards, so that all of a
  // thread's loads are in flight together (a conditional load would be
  // waited for before the next one is issued).
  double a[CMAX + 1];
#pragma unroll
  for (int i = 0; i <= CMAX; ++i) a[i] = 0.0;
  for (int zz = 0; zz < nsplit; ++zz) {
    const double *__restrict__ pz = part + zz * split_stride + rbase * Q + qq;
    // batches of 8 loads, all in flight before the first use
#pragma unroll
    for (int h0 = 0; h0 <= CMAX; h0 += 8) {
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (h0 + u <= CMAX) t[u] = pz[(long)min(n0 + h0 + u, nR - 1) * Q];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (h0 + u <= CMAX) a[h0 + u] += keep_if(h0 + u <= len && n0 + h0 + u < nR, t[u]);
    }
  }
  // This thread's recurrence coefficients, clamped the same way, fetched
  // H rows at a time (pair o, o+1 of the four per row) with all loads of a
  // batch in flight together.
  constexpr int H = CMAX < 8 ? CMAX : (CMAX > 8 ? 4 : 8);  // fewer in flight at CMAX 16: registers
  auto coef_pair = [&](int h, int o, double (&x)[H], double (&y)[H]) {
#pragma unroll
    for (int u = 0; u < H; ++u) {
      const double *c = cf + (long)min(n0 + h * H + u, nR - 1) * cstride;
      x[u] = c[o];
      y[u] = c[o + 1];
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  if (ok && Ahat) {
#pragma unroll
    for (int i = 0; i < CMAX; ++i)
      if (i < len) Ahat[(rbase + n0 + i) * Q + qq] = a[i];
  }
  double I = 0.0, Pa = 1.0, O = 0.0, Pg = 1.0;
#pragma unroll
  for (int h = 0; h < CMAX / H; ++h) {
    double c0[H], c1[H];
    coef_pair(h, 0, c0, c1);
#pragma unroll
    for (int u = 0; u < H; ++u) {
      const int i = h * H + u;
      if (i < len) {
        I = c0[u] * I + c1[u] * a[i];
        Pa *= c0[u];
      }
    }
  }
#pragma unroll
  for (int h = CMAX / H - 1; h >= 0; --h) {
    double c2[H], c3[H];
    coef_pair(h, 2, c2, c3);
#pragma unroll
    for (int u = H - 1; u >= 0; --u) {
      const int i = h * H + u;
      if (i < len) {
        O = c2[u] * O + c3[u] * a[i + 1];
        Pg *= c2[u];
      }
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
  for (int h = 0; h < CMAX / H; ++h) {
    double c0[H], c1[H];
    coef_pair(h, 0, c0, c1);
#pragma unroll
    for (int u = 0; u < H; ++u) {
      const int i = h * H + u;
      if (i < len) I = c0[u] * I + c1[u] * a[i];
      Iv[i] = I;
    }
  }
  const long rbar = (long)(1 - p) * nR;
  O = Oin;
#pragma unroll
  for (int h = CMAX / H - 1; h >= 0; --h) {
    double c2[H], c3[H];
    coef_pair(h, 2, c2, c3);
#pragma unroll
    for (int u = H - 1; u >= 0; --u) {
      const int i = h * H + u;
      if (i < len) {
        O = c2[u] * O + c3[u] * a[i + 1];
        const double v = negG * (Iv[i] + O);
        U[(rbase + n0 + i) * ldu + q] = v;
        if (sa.cross) U[(rbar + n0 + i) * ldu + Q + q] = v;
      }
    }
  }
}

template <int CMAX>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4, 4))) void radial_scan_kernel(ScanArgs sa) {
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
// contraction splits into a transform over phi (a strided batch over the
// colatitudes j) and one over theta (a grouped GEMM, one problem per
// azimuthal column mc).  The other patch's moments enter the synthesis
// rotated into this patch's frame, degree by degree (a grouped GEMM, one
// problem per degree and patch), before the radial scan below.
// Azimuthal column mc: 0 for m = 0, 2m-1 (cos) / 2m (sin); q = l^2 + mc.

// Phi transforms with the basis in LDS and the data streamed straight into
// MFMA fragments.  Block = WAVES waves of 16 data rows each, one colatitude
// j (blockIdx.y) and a group of G = 16 NT basis rows (blockIdx.z); the
// basis passes through LDS in chunks of 64 along the contraction (NBUF = 2:
// double buffered, one barrier per chunk; NBUF = 1: one buffer and two
// barriers per chunk, for wide groups whose contraction is mostly one
// chunk); each wave keeps the
// next PF stages (16 contraction values each) of its data fragments in
// registers.  Every basis entry outside the matrix is zeroed on its way into
// LDS, so the data loads only clamp their addresses.
//  analysis  (ANA): X2[mc][j][row] = sum_k W_j[mc][k] rho[row][j][k]; the
//            MFMA's A side is the basis (rows mc), the B side the data.
//  synthesis:       phi[row][j][k] = sum_mc V[mc][j][row] trig[k][mc]; the
//            A side is the data (rows), the B side the basis (rows k).
// FOLD: every row of n_p cells is even (cos) / odd (sin) about its middle,
// so the transforms run over h = ceil(n_p / 2) cells (the kGemmFoldA /
// kGemmFoldC forms, without their padding of each half to 16):
//  analysis:  basis rows kc (a multiple of 16) apart: row i < kc is cos m =
//             i, row i >= kc sin m = i - kc + 1 (W_j folded, K = h); a cos
//             tile multiplies rho[k] + rho[n_p - 1 - k], a sin tile
//             rho[k] - rho[n_p - 1 - k]; row i lands at azimuthal column mc
//             (dropped when mc >= nmc);
//  synthesis: contraction slots in steps of 4 consecutive slots, slot s < kc
//             (a multiple of 4) cos m = s, beyond sin m = s - kc + 1; the data
//             of a slot is V's azimuthal column mc (clamped below nmc; the
//             basis is zero at padding slots); the cos steps sum the even
//             part e, the sin steps the odd part o, and cell k < h gets
//             e + o, its mirror n_p - 1 - k gets e - o.
template <bool ANA, int WAVES, int NT, int NBUF, bool FOLD>
__global__ __launch_bounds__(64 * WAVES) void phi_direct_kernel(PhiDirectArgs a) {
  constexpr int G = 16 * NT, KC = 64, NTH = 64 * WAVES, PF = 4;
  constexpr bool FA = FOLD && ANA, FS = FOLD && !ANA;
  constexpr int EL = (G * KC + NTH - 1) / NTH;  // basis chunk elements per thread
  __shared__ __align__(16) double sB[NBUF][G][KC + 2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  const int j = blockIdx.y, g0 = blockIdx.z * G;
  const int r0 = blockIdx.x * (16 * WAVES) + 16 * wave;
  const int M = a.M, N = a.N, K = a.K, nt = a.nt;
  const int np = FOLD ? a.np : (ANA ? K : N);  // cells per row
  const double *__restrict__ bas = a.bas + (long)j * a.bas_batch;
  // this lane's data row (clamped) and its view of the contraction index
  const int row = min(r0 + lr, M - 1);
  const double *__restrict__ xr =
      ANA ? a.X + (long)row * ((long)nt * np) + (long)j * np : a.X + (long)j * M + row;
  const long xk = ANA ? 1 : (long)nt * M;  // stride of the contraction index
  // contraction slot of step s of stage st: each lane four consecutive
  // slots (one per step) or, FS, each step four consecutive slots
  auto slot = [&](int st, int s) { return FS ? 16 * st + 4 * s + lg : 16 * st + 4 * lg + s; };
  double xs[PF][4], xm[FA ? PF : 1][4];
  double stg[EL];
  // FS: acc sums the cos slots (even part), acc2 the sin slots (odd part)
  dbl4 acc[NT], acc2[FS ? NT : 1];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = dbl4{0.0, 0.0, 0.0, 0.0};
  if constexpr (FS) {
#pragma unroll
    for (int t = 0; t < NT; ++t) acc2[FS ? t : 0] = dbl4{0.0, 0.0, 0.0, 0.0};
  }

  // The contraction over slots [kb, kb + kn) into ac: data fragments PF
  // stages ahead in registers, the basis in chunks of KC slots through LDS.
  auto run = [&](dbl4 (&ac)[NT], int kb, int kn) {
    auto xload = [&](int st, int q) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = kb + min(slot(st, s), kn - 1);
        if constexpr (FS) {
          const int m = k < a.kc ? k : k - a.kc + 1;
          const int mc = min(k < a.kc ? max(2 * m - 1, 0) : 2 * m, a.nmc - 1);
          xs[q][s] = xr[(long)mc * xk];
        } else {
          xs[q][s] = xr[(long)k * xk];
          if constexpr (FA) xm[FA ? q : 0][s] = xr[np - 1 - k];
        }
      }
    };
    auto bload = [&](int c) {
#pragma unroll
      for (int u = 0; u < EL; ++u) {
        const int e = min(tid + NTH * u, G * KC - 1), br = e / KC, kk = e % KC;
        stg[u] = bas[(long)min(g0 + br, N - 1) * a.ldb + kb + min(c * KC + kk, kn - 1)];
      }
    };
    auto bstore = [&](int c, int buf) {
#pragma unroll
      for (int u = 0; u < EL; ++u) {
        const int e = tid + NTH * u, br = e / KC, kk = e % KC;
        if (e < G * KC) sB[buf][br][kk] = keep_if(g0 + br < N && c * KC + kk < kn, stg[u]);
      }
    };
    const int nst = (kn + 15) / 16, nch = (kn + KC - 1) / KC;
#pragma unroll
    for (int p = 0; p < PF; ++p) xload(min(p, nst - 1), p);
    bload(0);
    __builtin_amdgcn_sched_barrier(0);
    bstore(0, 0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
      const int buf = NBUF == 2 ? (c & 1) : 0;
      if (c + 1 < nch) bload(c + 1);
      // the chunk's four stages; stage st = 4c + q sits in register slot q
#pragma unroll
      for (int q = 0; q < KC / 16; ++q) {
        const int st = c * (KC / 16) + q;
        if (st < nst) {  // uniform
          double bf[NT][4];
#pragma unroll
          for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int s = 0; s < 4; ++s) bf[t][s] = sB[buf][16 * t + lr][slot(q, s)];
          if constexpr (FA) {
            // the even and odd parts of the data; a tile is all cos or all sin
            double de[4], dd[4];
#pragma unroll
            for (int s = 0; s < 4; ++s) {
              de[s] = xs[q][s] + xm[FA ? q : 0][s];
              dd[s] = xs[q][s] - xm[FA ? q : 0][s];
            }
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
              for (int t = 0; t < NT; ++t)
                ac[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[t][s], g0 + 16 * t < a.kc ? de[s] : dd[s], ac[t], 0,
                                                             0, 0);
          } else if constexpr (FS) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
              if (16 * st + 4 * s < kn) {  // uniform: steps past the end skipped
#pragma unroll
                for (int t = 0; t < NT; ++t)
                  ac[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[q][s], bf[t][s], ac[t], 0, 0, 0);
              }
          } else {
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
              for (int t = 0; t < NT; ++t)
                ac[t] = ANA ? __builtin_amdgcn_mfma_f64_16x16x4f64(bf[t][s], xs[q][s], ac[t], 0, 0, 0)
                            : __builtin_amdgcn_mfma_f64_16x16x4f64(xs[q][s], bf[t][s], ac[t], 0, 0, 0);
          }
          if (st + PF < nst) xload(st + PF, q);
        }
      }
      if (c + 1 < nch) {
        if (NBUF == 1) __syncthreads();  // every wave is done with the one buffer
        bstore(c + 1, NBUF == 2 ? buf ^ 1 : 0);
      }
      __syncthreads();
    }
  };
  if constexpr (FS) {
    run(acc, 0, a.kc);
    if (K > a.kc) run(acc2, a.kc, K - a.kc);  // none at L = 0
  } else {
    run(acc, 0, K);
  }
  // D layout: lane l, element e -> MFMA row l/16 + 4e, column l%16
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (ANA) {
        const int br = g0 + 16 * t + lg + 4 * e, r = r0 + lr;
        int mc = br;
        if constexpr (FA) {
          const int m = br < a.kc ? br : br - a.kc + 1;
          mc = br < a.kc ? max(2 * m - 1, 0) : 2 * m;
        }
        if (br < N && mc < (FA ? a.nmc : N) && r < M) a.C[(long)mc * ((long)nt * M) + (long)j * M + r] = acc[t][e];
      } else {
        const int r = r0 + lg + 4 * e, k = g0 + 16 * t + lr;
        if (r < M && k < N) {
          double *__restrict__ cr = a.C + (long)r * ((long)nt * np) + (long)j * np;
          if constexpr (FS) {
            const double ev = acc[t][e], od = acc2[FS ? t : 0][e];
            cr[k] = ev + od;
            if (np - 1 - k != k) cr[np - 1 - k] = ev - od;
          } else {
            cr[k] = acc[t][e];
          }
        }
      }
    }
}

// Folded phi synthesis with no LDS and no barrier: every wave owns 16 rows
// and CT column tiles of 16 folded cells of one colatitude, loads its data
// and basis fragments straight from memory in MFMA layout (S steps of 4
// contraction slots at a time, the next S in flight behind them) and
// stores its cells and their mirrors.  The waves are numbered column group
// fastest, then row tile, then colatitude; a block holds 4 of them.
//   data:  V[mc][j][row] (slot s: cos m = s for s < kc, sin m = s - kc + 1;
//          its azimuthal column mc clamped below nmc);
//   basis: Bk[s][n] (slot-major, n < hp, zero at padding slots and cells);
//   out:   phi[row][j][k] = e + o (k < h), phi[row][j][n_p - 1 - k] = e - o.
template <int CT, int S>
__global__ __launch_bounds__(256) void phi_syn_lean_kernel(PhiLeanArgs a) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int M = a.M, nt = a.nt, ncg = (a.h + 16 * CT - 1) / (16 * CT), nrt = (M + 15) / 16;
  const long w = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int cg = (int)(w % ncg), rt = (int)((w / ncg) % nrt), j = (int)(w / ((long)ncg * nrt));
  if (j >= nt) return;  // uniform across the wave; no barrier below
  const int row0 = rt * 16, n0 = cg * 16 * CT;
  const double *__restrict__ xr = a.V + (long)j * M + min(row0 + lr, M - 1);
  const long xk = (long)nt * M;
  dbl4 acc[CT], acc2[CT];
#pragma unroll
  for (int c = 0; c < CT; ++c) acc[c] = acc2[c] = dbl4{0.0, 0.0, 0.0, 0.0};
  // steps s0 / 4 .. s0 / 4 + S - 1 of the slots [.., se): lane group lg
  // takes slot 4t + lg of step t
  auto load = [&](double (&xa)[S], double (&xb)[CT][S], int s0, int se) {
#pragma unroll
    for (int t = 0; t < S; ++t) {
      const int sl = min(s0 + 4 * t + lg, se - 1);
      const int m = sl < a.kc ? sl : sl - a.kc + 1;
      const int mc = min(sl < a.kc ? max(2 * m - 1, 0) : 2 * m, a.nmc - 1);
      xa[t] = xr[(long)mc * xk];
#pragma unroll
      for (int c = 0; c < CT; ++c) xb[c][t] = a.Bk[(long)sl * a.hp + n0 + 16 * c + lr];
    }
  };
  auto mma = [&](dbl4 (&ac)[CT], const double (&xa)[S], const double (&xb)[CT][S], int s0, int se) {
#pragma unroll
    for (int t = 0; t < S; ++t)
      if (s0 + 4 * t < se) {  // uniform
#pragma unroll
        for (int c = 0; c < CT; ++c) ac[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[t], xb[c][t], ac[c], 0, 0, 0);
      }
  };
  // the slots [sb, se) into ac, two register sets of S steps in turn, the
  // first (xa0, xb0) already loaded
  auto run = [&](dbl4 (&ac)[CT], double (&xa0)[S], double (&xb0)[CT][S], int sb, int se) {
    double xa1[S], xb1[CT][S];
    for (int s0 = sb; s0 < se; s0 += 8 * S) {
      if (s0 + 4 * S < se) load(xa1, xb1, s0 + 4 * S, se);
      mma(ac, xa0, xb0, s0, se);
      if (s0 + 4 * S >= se) break;
      if (s0 + 8 * S < se) load(xa0, xb0, s0 + 8 * S, se);
      mma(ac, xa1, xb1, s0 + 4 * S, se);
    }
  };
  // the first register sets of the cos and of the sin slots load together,
  // so that the sin pass does not start with a wait of its own
  const bool odd = a.ns > a.kc;  // no sin slots at L = 0
  double ca[S], cb[CT][S], sa[S], sb[CT][S];
  load(ca, cb, 0, a.kc);
  if (odd) load(sa, sb, a.kc, a.ns);
  run(acc, ca, cb, 0, a.kc);
  if (odd) run(acc2, sa, sb, a.kc, a.ns);
  // D layout: lane l, element e -> row l/16 + 4e, column l%16
  const int np = a.np;
#pragma unroll
  for (int c = 0; c < CT; ++c) {
    const int k = n0 + 16 * c + lr;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = row0 + lg + 4 * e;
      if (r < M && k < a.h) {
        double *__restrict__ cr = a.C + ((long)r * nt + j) * np;
        const double ev = acc[c][e], od = acc2[c][e];
        cr[k] = ev + od;
        if (np - 1 - k != k) cr[np - 1 - k] = ev - od;
      }
    }
  }
}

// Radial sums of Eqs. (19)-(20) (the recurrences above) on column-major
// moments X[q][p nR + n]: one block per column q, one wave per patch.  The
// column (and its degree's recurrence coefficients, coefS[l][4][nR], shared
// by the waves) is staged
// in LDS; lane i owns the radial chunk [i c, i c + c) (c odd, so that the
// chunk-strided LDS reads spread over the banks); the chunk summaries
// (product of multipliers, local value) combine across the wave with
// shuffles, and the potential coefficients -G U_n^(q) go back through the
// column's LDS (once every lane has read it) to Ut[mc][l][p nR + n]
// (q = l^2 + mc), rows contiguous.
// CMAX bounds the chunk length: the chunk loops unroll with every LDS read
// at a clamped index, so that the reads issue ahead of the recurrences.
// Column q of one plan's scan; waves p >= P (a one-patch plan in a block
// sized for two) take part in the barriers only.  NCOL = 2: the block's
// waves 0..P-1 scan column q, waves P..2P-1 column q2 of the same degree
// (its recurrence coefficients staged once for both; q2 < 0: those waves
// take part in the barriers only).
template <int CMAX, int NCOL = 1>
__device__ __forceinline__ void radial_scan_q_body(const double *__restrict__ X, const double *__restrict__ coefS,
                                                   const int *__restrict__ qdeg, int nR, int L, int chunk,
                                                   double negG, double *__restrict__ Ut, int q, int P,
                                                   double *smem, int q2 = -1) {
  const int l = qdeg[q];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int col = NCOL > 1 ? w / P : 0, p = NCOL > 1 ? w - col * P : w;
  const bool active = p < P && (col == 0 || q2 >= 0);
  const int pa = p < P ? p : 0;                       // an inactive wave addresses patch 0 and stores nothing
  if (col == 1 && q2 >= 0) q = q2;
  const long M = (long)P * nR;
  double *sc = smem;                                  // [4][nR]: c0, c1, c2, c3 over n
  // [nR + 1]: the moments, zero at nR; then the outputs
  double *sx = smem + 4L * nR + (long)(col * P + pa) * (nR + 1);
  {
    // staging: batches of CB coefficient and XB moment loads from clamped
    // addresses, all in flight before the first LDS store (one batch covers
    // n_r <= 512 with two patches)
    constexpr int CB = 16, XB = 8;
    const double *__restrict__ cl = coefS + (long)l * 4 * nR;
    const double *__restrict__ xp = X + (long)q * M + (long)pa * nR;
    const int nt = blockDim.x;
    for (int c0 = 0, x0 = 0; c0 < 4 * nR || x0 <= nR; c0 += CB * nt, x0 += XB * 64) {
      double tc[CB], tx[XB];
#pragma unroll
      for (int u = 0; u < CB; ++u) tc[u] = cl[min(c0 + u * nt + tid, 4 * nR - 1)];
#pragma unroll
      for (int u = 0; u < XB; ++u) tx[u] = xp[min(x0 + u * 64 + lane, nR - 1)];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < CB; ++u)
        if (c0 + u * nt + tid < 4 * nR) sc[c0 + u * nt + tid] = tc[u];
#pragma unroll
      for (int u = 0; u < XB; ++u) {
        const int e = x0 + u * 64 + lane;
        if (active && e <= nR) sx[e] = keep_if(e < nR, tx[u]);
      }
    }
  }
  __syncthreads();
  const double *c0 = sc, *c1 = sc + nR, *c2 = sc + 2L * nR, *c3 = sc + 3L * nR;
  const int n0 = min(nR, lane * chunk), len = min(nR, n0 + chunk) - n0;
  // chunk summaries: I_out = Pa I_in + I, O_out = Pg O_in + O
  double I = 0.0, Pa = 1.0, O = 0.0, Pg = 1.0;
#pragma unroll
  for (int i = 0; i < CMAX; ++i) {
    const int n = min(n0 + i, nR - 1);
    const double a = c0[n], b = c1[n] * sx[n];
    if (i < len) {
      I = a * I + b;
      Pa *= a;
    }
  }
#pragma unroll
  for (int i = CMAX - 1; i >= 0; --i) {
    const int n = min(n0 + i, nR - 1);
    const double a = c2[n], b = c3[n] * sx[n + 1];
    if (i < len) {
      O = a * O + b;
      Pg *= a;
    }
  }
  // inclusive scans across the wave: inner sums from the left, outer sums
  // from the right
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double Pp = __shfl_up(Pa, off), Ip = __shfl_up(I, off);
    const double Pn = __shfl_down(Pg, off), On = __shfl_down(O, off);
    if (lane >= off) {
      I = Pa * Ip + I;
      Pa *= Pp;
    }
    if (lane + off < 64) {
      O = Pg * On + O;
      Pg *= Pn;
    }
  }
  double Iin = __shfl_up(I, 1), Oin = __shfl_down(O, 1);
  if (lane == 0) Iin = 0.0;
  if (lane == 63) Oin = 0.0;
  double Iv[CMAX];
  I = Iin;
#pragma unroll
  for (int i = 0; i < CMAX; ++i) {
    const int n = min(n0 + i, nR - 1);
    const double a = c0[n], b = c1[n] * sx[n];
    if (i < len) I = a * I + b;
    Iv[i] = I;
  }
  O = Oin;
#pragma unroll
  for (int i = CMAX - 1; i >= 0; --i) {
    const int n = min(n0 + i, nR - 1);
    const double a = c2[n], b = c3[n] * sx[n + 1];
    if (i < len) {
      O = a * O + b;
      Iv[i] = negG * (Iv[i] + O);  // the output of shell n
    }
  }
  __syncthreads();  // every lane has read the column: its space takes the outputs
#pragma unroll
  for (int i = 0; i < CMAX; ++i)
    if (active && i < len) sx[n0 + i] = Iv[i];
  __syncthreads();
  const int mc = q - l * l;
  double *__restrict__ ut = Ut + ((long)mc * (L + 1) + l) * M + (long)pa * nR;
  if (active)
    for (int e = lane; e < nR; e += 64) ut[e] = sx[e];
}

template <int CMAX>
__global__ __launch_bounds__(128) void radial_scan_q_kernel(const double *__restrict__ X, const double *__restrict__ coefS,
                                                            const int *__restrict__ qdeg, int nR, int L, int chunk,
                                                            double negG, double *__restrict__ Ut) {
  extern __shared__ double smem[];
  radial_scan_q_body<CMAX>(X, coefS, qdeg, nR, L, chunk, negG, Ut, blockIdx.x, blockDim.x / 64, smem);
}

// Two columns of one degree per block (P waves each): block b of degree l
// (l (l + 1) / 2 <= b < (l + 1) (l + 2) / 2) takes columns l^2 + 2 j and
// l^2 + 2 j + 1, j = b - l (l + 1) / 2, the second absent for j = l (the
// degree's 2l + 1 columns are odd in number).
template <int CMAX>
__global__ __launch_bounds__(256) void radial_scan_q2_kernel(const double *__restrict__ X,
                                                             const double *__restrict__ coefS,
                                                             const int *__restrict__ qdeg, int nR, int L, int chunk,
                                                             double negG, double *__restrict__ Ut, int P) {
  extern __shared__ double smem[];
  const int b = blockIdx.x;
  int l = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
  while (l * (l + 1) / 2 > b) --l;            // exact for any rounding of the square root
  while ((l + 1) * (l + 2) / 2 <= b) ++l;
  const int j = b - l * (l + 1) / 2, q = l * l + 2 * j;
  radial_scan_q_body<CMAX, 2>(X, coefS, qdeg, nR, L, chunk, negG, Ut, q, P, smem, j < l ? q + 1 : -1);
}

// The same over the columns of several plans (batched separable solves):
// blocks of two waves walk work items (plan, column q).
template <int CMAX>
__global__ __launch_bounds__(128) void radial_scan_q_grouped(const ScanQArgs *__restrict__ args,
                                                             const int2 *__restrict__ items, int n_items) {
  extern __shared__ double smem[];
  for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
    const int2 it = items[w];
    const ScanQArgs a = args[it.x];
    __syncthreads();  // the previous item's LDS reads are done
    radial_scan_q_body<CMAX>(a.X, a.coefS, a.qdeg, a.nR, a.L, a.chunk, a.negG, a.Ut, it.y, a.P, smem);
  }
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
      hipLaunchKernelGGL((gemm_nt_f64_grouped<0, BM, BN, WGM, WGN, 0>), grid, block, 0, s, probs, items, n_items);
      break;
    case 1:
      hipLaunchKernelGGL((gemm_nt_f64_grouped<1, BM, BN, WGM, WGN, 0>), grid, block, 0, s, probs, items, n_items);
      break;
    case 2:
      hipLaunchKernelGGL((gemm_nt_f64_grouped<0, BM, BN, WGM, WGN, 1>), grid, block, 0, s, probs, items, n_items);
      break;
    case 3:
      hipLaunchKernelGGL((gemm_nt_f64_grouped<1, BM, BN, WGM, WGN, 1>), grid, block, 0, s, probs, items, n_items);
      break;

    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Strided batch (see gemm_nt_f64_batched): role 0 stores C column-major
// (kGemmCTrans), role 1 reads A k-major (kGemmATrans), roles 2 and 3 the
// same with kGemmFoldA / kGemmFoldC; + kRoleDeep: with kGemmDeep.
template <int BM, int BN, int WGM, int WGN>
hipError_t launch_batch_variant(int role, const GemmF64Args &a, hipStream_t s) {
  GemmF64Args g = a;
  g.tiles_m = (g.M + BM - 1) / BM;
  const int per = g.tiles_m * ((g.N + BN - 1) / BN);
  const long total = (long)per * g.batch;
  if (total > INT_MAX) return hipErrorInvalidValue;
  dim3 grid((unsigned)total), block(64 * WGM * WGN);
  // column-major C: the transposed accumulation (kGemmDT) stores 16 rows at once
  if (role == 0)
    hipLaunchKernelGGL((gemm_nt_f64_batched<0, BM, BN, WGM, WGN, kGemmCTrans | kGemmDT>), grid, block, 0, s, g, per,
                       (int)total);
  else if (role == 1)
    hipLaunchKernelGGL((gemm_nt_f64_batched<1, BM, BN, WGM, WGN, kGemmATrans>), grid, block, 0, s, g, per,
                       (int)total);
  else if (role == kRoleDeep)
    hipLaunchKernelGGL((gemm_nt_f64_batched<0, BM, BN, WGM, WGN, kGemmCTrans | kGemmDT | kGemmDeep>), grid, block, 0, s,
                       g, per, (int)total);
  else if (role == 1 + kRoleDeep)
    hipLaunchKernelGGL((gemm_nt_f64_batched<1, BM, BN, WGM, WGN, kGemmATrans | kGemmDeep>), grid, block, 0, s, g, per,
                       (int)total);
  else if (role == 2)
    hipLaunchKernelGGL((gemm_nt_f64_batched<0, BM, BN, WGM, WGN, kGemmCTrans | kGemmDT | kGemmFoldA>), grid, block, 0,
                       s, g, per, (int)total);
  else if (role == 3)
    hipLaunchKernelGGL((gemm_nt_f64_batched<1, BM, BN, WGM, WGN, kGemmATrans | kGemmFoldC>), grid, block, 0, s, g,
                       per, (int)total);
  else if (role == 2 + kRoleDeep)
    hipLaunchKernelGGL((gemm_nt_f64_batched<0, BM, BN, WGM, WGN, kGemmCTrans | kGemmDT | kGemmFoldA | kGemmDeep>), grid,
                       block, 0, s, g, per, (int)total);
  else if (role == 3 + kRoleDeep)
    hipLaunchKernelGGL((gemm_nt_f64_batched<1, BM, BN, WGM, WGN, kGemmATrans | kGemmFoldC | kGemmDeep>), grid, block,
                       0, s, g, per, (int)total);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Separable theta phases and rotation (see gemm_f64_sep_phase).
template <int BM, int BN, int WGM, int WGN>
hipError_t launch_sep_variant(int phase, bool deep, const SepPhaseArgs &a, hipStream_t s) {
  const long Mr = (long)a.P * a.nR;
  long mmax, nmax;
  int nz;
  if (phase == 1) {
    mmax = Mr, nmax = a.L + 1, nz = 2 * a.L + 1;
  } else if (phase == 2) {
    mmax = a.nR, nmax = 2 * a.L + 1, nz = 2 * (a.L + 1);
  } else if (phase == 3) {
    mmax = a.nt, nmax = Mr, nz = 2 * a.L + 1;
  } else {
    return hipErrorInvalidValue;
  }
  if ((mmax + BM - 1) / BM > INT_MAX || (nmax + BN - 1) / BN > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)((mmax + BM - 1) / BM), (unsigned)((nmax + BN - 1) / BN), nz), block(64 * WGM * WGN);
  // phases 1 and 2 store column-major (ldc = 1): transposed accumulation
  constexpr int A1 = 1 | kGemmATrans | kGemmDT, A2 = 1 | kGemmATrans | kGemmBTrans | kGemmDT | kGemmAccInit,
                A3 = kGemmBTrans;
#define YYG_SEP_GO(P, M)                                                                                     \
  hipLaunchKernelGGL((gemm_f64_sep_phase<P, BM, BN, WGM, WGN, M>), grid, block, 0, s, a);                  \
  break
  switch (phase * 2 + (deep ? 1 : 0)) {
    case 2: YYG_SEP_GO(1, A1);
    case 3: YYG_SEP_GO(1, A1 | kGemmDeep);
    case 4: YYG_SEP_GO(2, A2);
    case 5: YYG_SEP_GO(2, A2 | kGemmDeep);
    case 6: YYG_SEP_GO(3, A3);
    default: YYG_SEP_GO(3, A3 | kGemmDeep);
  }
#undef YYG_SEP_GO
  return hipGetLastError();
}

typedef hipError_t (*gemm_f64_fn)(int, int, int, int, const double *, long, const double *, long, double *, long, int,
                                  long, hipStream_t);
typedef hipError_t (*batch_f64_fn)(int, const GemmF64Args &, hipStream_t);
typedef hipError_t (*sep_f64_fn)(int, bool, const SepPhaseArgs &, hipStream_t);

typedef hipError_t (*grouped_f64_fn)(int, const GemmF64Args *, const int4 *, int, int, hipStream_t);

struct F64Variant {
  int bm, bn, threads, wm, wn;
  gemm_f64_fn fn;
  grouped_f64_fn grouped;
  batch_f64_fn batch;
  sep_f64_fn sep;
};

#define YYG_F64_VARIANT(BM, BN, WM, WN)                                                                   \
  {                                                                                                        \
    BM, BN, 64 * WM * WN, WM, WN, launch_gemm_variant<BM, BN, WM, WN>, launch_grouped_variant<BM, BN, WM, WN>, \
        launch_batch_variant<BM, BN, WM, WN>, launch_sep_variant<BM, BN, WM, WN>                          \
  }

const F64Variant kF64Variants[] = {
    YYG_F64_VARIANT(128, 128, 2, 2), YYG_F64_VARIANT(64, 128, 2, 2),  YYG_F64_VARIANT(128, 64, 2, 2),
    YYG_F64_VARIANT(64, 64, 2, 2),   YYG_F64_VARIANT(256, 128, 4, 2), YYG_F64_VARIANT(128, 256, 2, 4),
    // narrow-N shapes for the transforms whose N is 2L+1 or a degree block
    YYG_F64_VARIANT(128, 48, 4, 1),  YYG_F64_VARIANT(128, 96, 4, 1),  YYG_F64_VARIANT(128, 144, 4, 1),
    YYG_F64_VARIANT(64, 32, 2, 2),
    // more waves per tile for the short contractions of the separable form
    YYG_F64_VARIANT(32, 32, 2, 2),   YYG_F64_VARIANT(64, 64, 4, 2),
    // five MFMA columns per wave: folded phi transforms whose N is one or a
    // few past a multiple of 32 or 64 (L + 1 = 65, h = 69)
    YYG_F64_VARIANT(32, 80, 2, 1),   YYG_F64_VARIANT(64, 80, 4, 1),
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

namespace {

template <bool ANA, int WAVES, int NT, int NBUF, bool FOLD>
hipError_t launch_phi_direct_t(const PhiDirectArgs &a, hipStream_t s) {
  dim3 grid((a.M + 16 * WAVES - 1) / (16 * WAVES), a.nt, (a.N + 16 * NT - 1) / (16 * NT));
  hipLaunchKernelGGL((phi_direct_kernel<ANA, WAVES, NT, NBUF, FOLD>), grid, dim3(64 * WAVES), 0, s, a);
  return hipGetLastError();
}

template <bool ANA>
hipError_t launch_phi_direct_v(int variant, const PhiDirectArgs &a, hipStream_t s) {
  switch (variant) {
    case 0: return launch_phi_direct_t<ANA, 8, 4, 2, false>(a, s);
    case 1: return launch_phi_direct_t<ANA, 8, 3, 2, false>(a, s);
    case 2: return launch_phi_direct_t<ANA, 8, 2, 2, false>(a, s);
    case 3: return launch_phi_direct_t<ANA, 4, 4, 2, false>(a, s);
    case 4: return launch_phi_direct_t<ANA, 4, 3, 2, false>(a, s);
    case 5: return launch_phi_direct_t<ANA, 4, 2, 2, false>(a, s);
  }
  return hipErrorInvalidValue;
}

template <bool ANA>
hipError_t launch_phi_fold_v(int variant, const PhiDirectArgs &a, hipStream_t s) {
  switch (variant) {
    case 0: return launch_phi_direct_t<ANA, 2, 4, 1, true>(a, s);
    case 1: return launch_phi_direct_t<ANA, 4, 4, 1, true>(a, s);
    case 2: return launch_phi_direct_t<ANA, 8, 4, 1, true>(a, s);
    case 3: return launch_phi_direct_t<ANA, 2, 5, 1, true>(a, s);
    case 4: return launch_phi_direct_t<ANA, 4, 5, 1, true>(a, s);
    case 5: return launch_phi_direct_t<ANA, 8, 5, 1, true>(a, s);
    case 6: return launch_phi_direct_t<ANA, 4, 4, 2, true>(a, s);
    case 7: return launch_phi_direct_t<ANA, 4, 5, 2, true>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

// (waves per block, basis tiles per block, LDS buffers) of each variant
// (measured on MI355X: single-buffered groups of 96-144 basis rows were
// slower than these at 2L+1 = 51 and n_p = 137)
const int kPhiDirect[][3] = {{8, 4, 2}, {8, 3, 2}, {8, 2, 2}, {4, 4, 2}, {4, 3, 2}, {4, 2, 2}};
// the same for the folded form
const int kPhiFold[][3] = {{2, 4, 1}, {4, 4, 1}, {8, 4, 1}, {2, 5, 1}, {4, 5, 1}, {8, 5, 1}, {4, 4, 2}, {4, 5, 2}};

int phi_direct_variant_count() { return (int)(sizeof(kPhiDirect) / sizeof(kPhiDirect[0])); }
int phi_fold_variant_count() { return (int)(sizeof(kPhiFold) / sizeof(kPhiFold[0])); }

hipError_t launch_phi_direct(int variant, bool analysis, const PhiDirectArgs &a, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0 || a.nt <= 0) return hipSuccess;
  if (a.K <= 0 || a.nt > 65535 || (a.N + 31) / 32 > 65535) return hipErrorInvalidValue;
  return analysis ? launch_phi_direct_v<true>(variant, a, s) : launch_phi_direct_v<false>(variant, a, s);
}

hipError_t launch_phi_fold(int variant, bool analysis, const PhiDirectArgs &a, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0 || a.nt <= 0) return hipSuccess;
  if (a.K <= 0 || a.nt > 65535 || (a.N + 31) / 32 > 65535 || a.nmc < 1) return hipErrorInvalidValue;
  // the cos / sin boundary: whole basis tiles (analysis), whole steps (synthesis)
  if (a.kc < 0 || a.kc % (analysis ? 16 : 4) != 0) return hipErrorInvalidValue;
  // analysis: K = h cells of the n_p per row; synthesis: N = h
  if ((analysis ? a.K : a.N) != (a.np + 1) / 2) return hipErrorInvalidValue;
  return analysis ? launch_phi_fold_v<true>(variant, a, s) : launch_phi_fold_v<false>(variant, a, s);
}

namespace {

template <int CT, int S>
hipError_t launch_phi_syn_lean_t(const PhiLeanArgs &a, hipStream_t s) {
  const long waves = (long)a.nt * ((a.M + 15) / 16) * ((a.h + 16 * CT - 1) / (16 * CT));
  if ((waves + 3) / 4 > INT_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((phi_syn_lean_kernel<CT, S>), dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace

// (column tiles per wave, steps per register set) of each variant
const int kPhiLean[][2] = {{1, 4}, {1, 8}, {2, 4}, {2, 8}};

int phi_lean_variant_count() { return (int)(sizeof(kPhiLean) / sizeof(kPhiLean[0])); }

hipError_t launch_phi_syn_lean(int variant, const PhiLeanArgs &a, hipStream_t s) {
  if (a.M <= 0 || a.nt <= 0 || a.h <= 0) return hipSuccess;
  if (a.nmc < 1 || a.ns < 4 || a.ns % 4 || a.kc < 4 || a.kc % 4 || a.kc > a.ns || a.h != (a.np + 1) / 2 ||
      a.hp % 32 || a.hp < a.h)
    return hipErrorInvalidValue;
  switch (variant) {
    case 0: return launch_phi_syn_lean_t<1, 4>(a, s);
    case 1: return launch_phi_syn_lean_t<1, 8>(a, s);
    case 2: return launch_phi_syn_lean_t<2, 4>(a, s);
    case 3: return launch_phi_syn_lean_t<2, 8>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_f64_sep(int variant, int phase, bool deep, const SepPhaseArgs &a, hipStream_t s) {
  if (a.nR <= 0) return hipSuccess;
  if (variant < 0 || variant >= gemm_f64_variant_count()) return hipErrorInvalidValue;
  return kF64Variants[variant].sep(phase, deep, a, s);
}

hipError_t launch_gemm_f64_batched(int variant, int role, const GemmF64Args &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  if (variant < 0 || variant >= gemm_f64_variant_count()) return hipErrorInvalidValue;
  return kF64Variants[variant].batch(role, g, s);
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
  if (!Ahat && nsplit != 1) return hipErrorInvalidValue;
  ScanArgs sa{part, nsplit, split_stride, Ahat, coef, qdeg, nR, Q, L, negG, U, ldu, cross};
  if (nR <= 64 * 4) {
    hipLaunchKernelGGL(radial_scan_kernel<4>, dim3((Q + 15) / 16, patches), dim3(16, 64), 0, s, sa);
  } else if (nR <= 64 * 8) {
    hipLaunchKernelGGL(radial_scan_kernel<8>, dim3((Q + 15) / 16, patches), dim3(16, 64), 0, s, sa);
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


size_t radial_scan_q_lds(int nR, int patches) { return (4UL * nR + (size_t)patches * (nR + 1UL)) * sizeof(double); }

// the paired form: the coefficients once, two columns of every patch
static size_t radial_scan_q2_lds(int nR, int patches) {
  return (4UL * nR + 2UL * patches * (nR + 1UL)) * sizeof(double);
}

// the column and its coefficients fit in LDS and a lane's chunk in the
// largest instance (63 shells)
bool radial_scan_q_supports(int nR, int patches) {
  return nR >= 1 && radial_scan_q_lds(nR, patches) <= kScanQMaxLds && (((nR + 63) / 64) | 1) <= 63;
}

hipError_t launch_radial_scan_q(const double *X, const double *coefS, const int *qdeg, int nR, int L, double negG,
                                int patches, double *Ut, hipStream_t s) {
  if (nR <= 0) return hipSuccess;
  if (patches < 1 || patches > 2) return hipErrorInvalidValue;
  const size_t lds = radial_scan_q_lds(nR, patches);
  if (lds > kScanQMaxLds) return hipErrorInvalidValue;
  const int chunk = ((nR + 63) / 64) | 1;
  const int Q = (L + 1) * (L + 1);
  auto go = [&](auto kern) {
    if (lds > 64 * 1024 &&
        hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
      return hipGetLastError();
    hipLaunchKernelGGL(kern, dim3(Q), dim3(64 * patches), lds, s, X, coefS, qdeg, nR, L, chunk, negG, Ut);
    return hipGetLastError();
  };
  // two columns per block where they fit in LDS (the coefficients staged
  // once for both) ...; the unrolled chunk loops run CMAX steps: an instance
  // close to the chunk (n_r 550: 9, n_r 1000: 17) keeps the dependent
  // recurrences short
  // (with enough columns: Q / 2 blocks must still fill the device; at
  // lmax 25, 351 paired blocks ran slower than 676 single ones)
  const size_t lds2 = radial_scan_q2_lds(nR, patches);
  if (lds2 <= kScanQMaxLds && Q >= 1024) {
    const int blocks = (L + 1) * (L + 2) / 2;
    auto go2 = [&](auto kern) {
      if (lds2 > 64 * 1024 &&
          hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds2) != hipSuccess)
        return hipGetLastError();
      hipLaunchKernelGGL(kern, dim3(blocks), dim3(128 * patches), lds2, s, X, coefS, qdeg, nR, L, chunk, negG, Ut,
                         patches);
      return hipGetLastError();
    };
    if (chunk <= 7) return go2(radial_scan_q2_kernel<7>);
    if (chunk <= 9) return go2(radial_scan_q2_kernel<9>);
    if (chunk <= 11) return go2(radial_scan_q2_kernel<11>);
    if (chunk <= 15) return go2(radial_scan_q2_kernel<15>);
    if (chunk <= 17) return go2(radial_scan_q2_kernel<17>);
    if (chunk <= 23) return go2(radial_scan_q2_kernel<23>);
    if (chunk <= 31) return go2(radial_scan_q2_kernel<31>);
    return go2(radial_scan_q2_kernel<63>);
  }
  if (chunk <= 7) return go(radial_scan_q_kernel<7>);
  if (chunk <= 9) return go(radial_scan_q_kernel<9>);
  if (chunk <= 11) return go(radial_scan_q_kernel<11>);
  if (chunk <= 15) return go(radial_scan_q_kernel<15>);
  if (chunk <= 17) return go(radial_scan_q_kernel<17>);
  if (chunk <= 23) return go(radial_scan_q_kernel<23>);
  if (chunk <= 31) return go(radial_scan_q_kernel<31>);
  if (chunk <= 63) return go(radial_scan_q_kernel<63>);
  return hipErrorInvalidValue;
}

hipError_t launch_radial_scan_q_grouped(const ScanQArgs *args, const int2 *items, int n_items, int n_blocks,
                                        int max_nR, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  const size_t lds = radial_scan_q_lds(max_nR, 2);
  if (lds > kScanQMaxLds) return hipErrorInvalidValue;
  const int chunk = ((max_nR + 63) / 64) | 1;
  auto go = [&](auto kern) {
    if (lds > 64 * 1024 &&
        hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds) != hipSuccess)
      return hipGetLastError();
    hipLaunchKernelGGL(kern, dim3(n_blocks), dim3(128), lds, s, args, items, n_items);
    return hipGetLastError();
  };
  if (chunk <= 7) return go(radial_scan_q_grouped<7>);
  if (chunk <= 15) return go(radial_scan_q_grouped<15>);
  if (chunk <= 31) return go(radial_scan_q_grouped<31>);
  if (chunk <= 63) return go(radial_scan_q_grouped<63>);
  return hipErrorInvalidValue;
}

namespace {

// Folded phi analysis with the last output column on the vector units
// (kGemmXCol): N - 1 columns in MFMA tiles of BN, the column N - 1 beside
// them when N - 1 is a multiple of BN (L + 1 = 65 outputs per half in
// 64-wide tiles, where an MFMA tile for the one column would double the work).
template <int BM, int BN, int WGM, int WGN, bool DEEP>
hipError_t launch_fold_xcol_t(const GemmF64Args &a, hipStream_t s) {
  GemmF64Args g = a;
  g.tiles_m = (g.M + BM - 1) / BM;
  const int tiles_n = std::max(1, (g.N - 1 + BN - 1) / BN);
  const long per = (long)g.tiles_m * tiles_n, total = per * g.batch;
  if (total > INT_MAX || g.batch % 2) return hipErrorInvalidValue;
  constexpr int MODE = kGemmCTrans | kGemmDT | kGemmFoldA | kGemmXCol | (DEEP ? kGemmDeep : 0);
  hipLaunchKernelGGL((gemm_nt_f64_batched<0, BM, BN, WGM, WGN, MODE>), dim3((unsigned)total), dim3(64 * WGM * WGN), 0,
                     s, g, (int)per, (int)total);
  return hipGetLastError();
}

struct XColVariant {
  int bm, bn, wm, wn, deep;
  hipError_t (*fn)(const GemmF64Args &, hipStream_t);
};

#define YYG_XCOL(BM, BN, WM, WN, D) \
  { BM, BN, WM, WN, D, launch_fold_xcol_t<BM, BN, WM, WN, D> }

const XColVariant kXCol[] = {
    YYG_XCOL(64, 64, 4, 1, false), YYG_XCOL(64, 64, 2, 2, false), YYG_XCOL(64, 32, 4, 1, false),
    YYG_XCOL(128, 64, 4, 1, false), YYG_XCOL(64, 64, 4, 1, true), YYG_XCOL(64, 64, 2, 2, true),
    YYG_XCOL(128, 64, 2, 2, false), YYG_XCOL(64, 64, 4, 2, false),
};

#undef YYG_XCOL

}  // namespace

int fold_xcol_variant_count() { return (int)(sizeof(kXCol) / sizeof(kXCol[0])); }

hipError_t launch_fold_xcol(int v, const GemmF64Args &g, hipStream_t s) {
  if (v < 0 || v >= fold_xcol_variant_count()) return hipErrorInvalidValue;
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  return kXCol[v].fn(g, s);
}

int fold_xcol_kernel_name(int v, char *buf, size_t n) {
  if (v < 0 || v >= fold_xcol_variant_count()) return -1;
  const XColVariant &x = kXCol[v];
  const int mode = kGemmCTrans | kGemmDT | kGemmFoldA | kGemmXCol | (x.deep ? kGemmDeep : 0);
  return snprintf(buf, n, "yyg::gemm_nt_f64_batched<0, %d, %d, %d, %d, %d>", x.bm, x.bn, x.wm, x.wn, mode) < 0 ? -1
                                                                                                               : 0;
}

int sep_kernel_name(int phase, int v, bool fold, char *buf, size_t n) {
  const int nv = gemm_f64_variant_count(), nd = phi_direct_variant_count(), nf = phi_fold_variant_count();
  const int nl = phase == 4 ? phi_lean_variant_count() : 0;
  const bool phi = phase == 0 || phase == 4;
  if (phase < 0 || phase > 4 || v < 0 || v >= 2 * nv + (phi ? nd + nf : 0) + nl) return -1;
  if (v >= 2 * nv + nd + nf) {
    if (!fold) return -1;
    const int *d = kPhiLean[v - 2 * nv - nd - nf];
    return snprintf(buf, n, "yyg::phi_syn_lean_kernel<%d, %d>", d[0], d[1]) < 0 ? -1 : 0;
  }
  if (v >= 2 * nv) {
    const bool fd = v >= 2 * nv + nd;
    if (fd && !fold) return -1;
    const int *d = fd ? kPhiFold[v - 2 * nv - nd] : kPhiDirect[v - 2 * nv];
    return snprintf(buf, n, "yyg::phi_direct_kernel<%s, %d, %d, %d, %s>", phase == 0 ? "true" : "false", d[0], d[1],
                    d[2], fd ? "true" : "false") < 0 ? -1 : 0;
  }
  const F64Variant &f = kF64Variants[v % nv];
  const int deep = v >= nv ? kGemmDeep : 0;
  if (phase == 0 || phase == 4) {
    const int mode =
        phase == 0 ? kGemmCTrans | kGemmDT | (fold ? kGemmFoldA : 0) : kGemmATrans | (fold ? kGemmFoldC : 0);
    return snprintf(buf, n, "yyg::gemm_nt_f64_batched<%d, %d, %d, %d, %d, %d>", phase == 0 ? 0 : 1, f.bm, f.bn, f.wm,
                    f.wn, mode | deep) < 0 ? -1 : 0;
  }
  const int mode = phase == 1   ? 1 | kGemmATrans | kGemmDT
                   : phase == 2 ? 1 | kGemmATrans | kGemmBTrans | kGemmDT | kGemmAccInit
                                : kGemmBTrans;
  return snprintf(buf, n, "yyg::gemm_f64_sep_phase<%d, %d, %d, %d, %d, %d>", phase, f.bm, f.bn, f.wm, f.wn,
                  mode | deep) < 0 ? -1 : 0;
}

}  // namespace yyg
