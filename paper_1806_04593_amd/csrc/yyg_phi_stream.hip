// Folded phi synthesis of the separable form, streaming variant: the block
// keeps one panel of the folded azimuthal basis in LDS for its whole life
// and its waves sweep row tiles independently, loading the coefficients of
// the theta synthesis straight into registers in the 16x16x4 FP64 MFMA
// operand layout a few steps ahead of their use (no LDS staging, no
// barrier after the panel fill).
//
// For colatitude j and row (patch, shell) the potential at the azimuthal
// cell s of the folded half and at its mirror n_phi - 1 - s is e + o and
// e - o, with e = sum_m c_m TF_cos(s, m) over the cosine columns (m = 0..L)
// and o = sum_m s_m TF_sin(s, m) over the sine columns (m = 1..L): the
// synthesis of Eqs. (5) and (28)-(29) along one colatitude row, split into
// its parts even and odd about the central meridian.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdio>

#include "yyg_internal.h"

namespace yyg {

typedef double dbl4s __attribute__((ext_vector_type(4)));

// TI row tiles of 16 rows per wave, a basis panel of TJ tiles of 16 folded
// azimuthal cells per block, NW waves per block, P steps of coefficient
// loads in flight, LDB the panel's row capacity (at least 8 ceil((L+1)/4)).
// One step takes four cosine and four sine columns: the wave's accumulators
// e and o each gain a 16 x 16 x 4 product per basis tile.
// The wave's sweep for a panel of TJR basis tiles (TJR <= TJ: the last panel
// of a row may hold fewer), once its panel is in LDS.
// Row tile tt -> (colatitude row jl, tile rt of 16 TI (patch, shell) rows):
// CF false numbers the (patch, shell) tiles fastest, CF true the colatitude
// rows, so that the waves of a block then write neighbouring rows of the
// same planes (whose shared cache lines meet in L2 before they are evicted).
template <bool CF>
__device__ __forceinline__ void tile_split(int tt, int tiles_j, int nt, int &jl, int &rt) {
  if (CF) {
    rt = tt / nt;
    jl = tt - rt * nt;
  } else {
    jl = tt / tiles_j;
    rt = tt - jl * tiles_j;
  }
}

// Lane groups (16 lanes) 2 and 3 of a trade places with groups 0 and 1 of
// b, both 32-bit halves of the doubles (v_permlane32_swap).
__device__ __forceinline__ void swap_half_waves(double &a, double &b) {
  const unsigned long long ua = __builtin_bit_cast(unsigned long long, a);
  const unsigned long long ub = __builtin_bit_cast(unsigned long long, b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  a = __builtin_bit_cast(double, ((unsigned long long)hi[0] << 32) | lo[0]);
  b = __builtin_bit_cast(double, ((unsigned long long)hi[1] << 32) | lo[1]);
}

// Stores a finished row tile (rows row0 + [0, 16 TI) of colatitude row jl,
// folded cells slot0 + [0, 16 TJ)): e + o at each cell and e - o at its
// mirror, then clears the sums.  Lane group g, element r of a product holds
// row F32 ? 4 g + r : g + 4 r (the FP32 and FP64 16x16x4 D layouts), cell
// r16.  Tiles go in pairs (j, j + 1): after swapping half-waves between
// their values, lane group g holds tile j + g / 2 of two rows, so that one
// store instruction writes two rows x 32 consecutive cells rather than four
// rows x 16 (fewer cache lines, since the rows are not 128-byte aligned).
// `live` is uniform; every lane takes part in the swaps.
template <int TI, int TJ, bool F32>
__device__ __forceinline__ void store_row_tile(const PhiStreamArgs &a, dbl4s (&accE)[TI][TJ],
                                               dbl4s (&accO)[TI][TJ], int row0, int jl, int slot0, int g,
                                               int r16, bool live) {
  auto rowof = [](int sg, int r) { return F32 ? 4 * sg + r : sg + 4 * r; };
  double *const base = a.phi + (long)jl * a.np;
  auto put = [&](int row, int slot, double sum, double dif) {
    if (live && row < a.Mr && slot < a.h) {
      double *o = base + (long)row * a.ldc;
      o[slot] = sum;
      const int cm = a.np - 1 - slot;
      if (cm != slot) o[cm] = dif;
    }
  };
#pragma unroll
  for (int i = 0; i < TI; ++i) {
#pragma unroll
    for (int j = 0; j + 1 < TJ; j += 2)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double s0 = accE[i][j][r] + accO[i][j][r], d0 = accE[i][j][r] - accO[i][j][r];
        double s1 = accE[i][j + 1][r] + accO[i][j + 1][r], d1 = accE[i][j + 1][r] - accO[i][j + 1][r];
        swap_half_waves(s0, s1);
        swap_half_waves(d0, d1);
        const int slot = slot0 + 16 * (j + (g >> 1)) + r16;
        put(row0 + 16 * i + rowof(g & 1, r), slot, s0, d0);
        put(row0 + 16 * i + rowof(2 + (g & 1), r), slot, s1, d1);
      }
    if constexpr ((TJ & 1) != 0)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        put(row0 + 16 * i + rowof(g, r), slot0 + 16 * (TJ - 1) + r16, accE[i][TJ - 1][r] + accO[i][TJ - 1][r],
            accE[i][TJ - 1][r] - accO[i][TJ - 1][r]);
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      accE[i][j] = dbl4s{0.0, 0.0, 0.0, 0.0};
      accO[i][j] = dbl4s{0.0, 0.0, 0.0, 0.0};
    }
  }
}

template <int TI, int TJR, int NW, int P, bool CF>
__device__ __forceinline__ void phi_syn_stream_sweep(const PhiStreamArgs &a, const double *Bs, int ldb, int NQ,
                                                     int KE, int slot0, int groups, int grp, int xcd,
                                                     int tiles_j, int tiles_total) {
  constexpr int TJ = TJR;
  const int NQO = (a.L + 3) / 4;   // sine steps that hold a column (the last step may hold none)
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, r16 = lane & 15;
  const int per = tiles_total / 8, rem = tiles_total % 8;
  const int t_beg = xcd * per + min(xcd, rem), t_end = t_beg + per + (xcd < rem ? 1 : 0);
  const int stride = groups * NW;
  int t = t_beg + grp * NW + wave;
  if (t >= t_end) return;
  // element offsets stay below 2^31 (checked by the launcher)
  auto rowbase = [&](int tt, int i) -> int {
    tt = min(tt, tiles_total - 1);
    int jl, rt;
    tile_split<CF>(tt, tiles_j, a.nt, jl, rt);
    return jl * a.Mr + min(rt * 16 * TI + 16 * i + r16, a.Mr - 1);
  };
  const int MJ = (int)a.MJ;
  // azimuthal columns of step q for lane group g (clamped: past L the basis is zero)
  auto offE = [&](int q) { return min(max(8 * q + 2 * g - 1, 0), a.nmc - 1) * MJ; };
  auto offO = [&](int q) { return min(8 * q + 2 * g + 2, a.nmc - 1) * MJ; };
  dbl4s accE[TI][TJ], accO[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      accE[i][j] = dbl4s{0.0, 0.0, 0.0, 0.0};
      accO[i][j] = dbl4s{0.0, 0.0, 0.0, 0.0};
    }
  // the steps of every tile of this wave, padded to whole rings: the
  // surplus steps read clamped addresses and their sums are never stored
  const int n_my = (t_end - t + stride - 1) / stride;
  const int total = (n_my * NQ + P - 1) / P * P;
  // load cursor (tile tl, step ql), P steps ahead of the compute cursor
  int tl = t, ql = 0;
  int rbl[TI];
#pragma unroll
  for (int i = 0; i < TI; ++i) rbl[i] = rowbase(tl, i);
  // without a branch: the loads that refill a ring slot then stay after
  // the reads of its values (a load hoisted above them would need other
  // registers and a copy, after a wait for every load in flight, at the
  // end of each ring)
  auto advance_load = [&]() {
    const bool next = ++ql == NQ;
    ql = next ? 0 : ql;
    tl += next ? stride : 0;
#pragma unroll
    for (int i = 0; i < TI; ++i) rbl[i] = rowbase(tl, i);
  };
  double raE[P][TI], raO[P][TI];
  auto refill = [&](int p) {
    const int oe = offE(ql), oo = offO(ql);
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      raE[p][i] = a.V[oe + rbl[i]];
      raO[p][i] = a.V[oo + rbl[i]];
    }
    advance_load();
  };
  // slots filled in order (the waits in the loop count on slot p's loads
  // being older than slot p + 1's)
#pragma unroll
  for (int p = 0; p < P; ++p) {
    refill(p);
    __builtin_amdgcn_sched_barrier(0);
  }
  // basis fragments of the current step, read one step ahead (up to 6
  // tiles; wider panels read them at the step, for registers): lane
  // (g, r16) holds cell 16 j + r16 of the panel at column 4 q + g
  constexpr bool BPF = TJ <= 6;
  const double *bp = &Bs[r16 * ldb + g];
  double bE[TJ], bO[TJ];
  if constexpr (BPF) {
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      bE[j] = bp[16 * j * ldb];
      bO[j] = bp[16 * j * ldb + KE];
    }
  }
  int q = 0;
  for (int base = 0; base < total; base += P) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      double nE[BPF ? TJ : 1], nO[BPF ? TJ : 1];
      if constexpr (BPF) {
        const int qn = q + 1 == NQ ? 0 : q + 1;
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          nE[j] = bp[16 * j * ldb + 4 * qn];
          nO[j] = bp[16 * j * ldb + KE + 4 * qn];
        }
      } else {
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          bE[j] = bp[16 * j * ldb + 4 * q];
          bO[j] = bp[16 * j * ldb + KE + 4 * q];
        }
      }
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
          accE[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(raE[p][i], bE[j], accE[i][j], 0, 0, 0);
      if (q < NQO) {  // uniform: a sine step past L adds nothing
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j)
            accO[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(raO[p][i], bO[j], accO[i][j], 0, 0, 0);
      }
      // the slot's refill P steps ahead, after its values have gone into
      // this step's products: into the same registers, no copy
      __builtin_amdgcn_sched_barrier(0);
      refill(p);
      if constexpr (BPF) {
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
          bE[j] = nE[j];
          bO[j] = nO[j];
        }
      }
      if (++q == NQ) {
        // tile t done
        int jl, rt;
        tile_split<CF>(t, tiles_j, a.nt, jl, rt);
        store_row_tile<TI, TJ, false>(a, accE, accO, rt * 16 * TI, jl, slot0, g, r16, t < t_end);
        q = 0;
        t += stride;
      }
    }
  }
}

template <int TI, int TJ, int NW, int P, int LDB, bool CF>
__device__ __forceinline__ void phi_syn_stream_body(const PhiStreamArgs &a, int n_panels, int tiles_j,
                                                    int tiles_total) {
  __shared__ double Bs[TJ * 16 * LDB];
  const int NQ = (a.L + 4) / 4;   // steps: cosine columns m = 4q + g (m <= L), sine m = 4q + g + 1
  const int KE = 4 * NQ;          // panel row: cosine part [0, KE), sine part [KE, 2 KE)
  const int ldb = 2 * KE + 2;     // row stride: 16 rows x 2 lanes land on distinct LDS bank pairs
  // blocks of one XCD (blockIdx % 8, the hardware's round-robin) share one
  // contiguous run of row tiles; within it, block ib serves panel ib % n_panels
  const int xcd = blockIdx.x & 7, ib = blockIdx.x >> 3, nbx = (int)(gridDim.x >> 3);
  const int panel = ib % n_panels, grp = ib / n_panels;
  const int groups = (nbx - panel + n_panels - 1) / n_panels;
  const int slot0 = panel * TJ * 16;
  for (int e = threadIdx.x; e < TJ * 16 * 2 * KE; e += 64 * NW) {
    const int sl = e / (2 * KE), kk = e - sl * (2 * KE), slot = slot0 + sl;
    double v = 0.0;
    if (slot < a.h) {
      if (kk < KE) {
        if (kk <= a.L) v = a.TF[(long)slot * a.ldtf + kk];
      } else if (kk - KE < a.L) {
        v = a.TF[(long)slot * a.ldtf + a.ks + (kk - KE)];
      }
    }
    Bs[sl * ldb + kk] = v;
  }
  __syncthreads();
  // the last panel of a row runs with the tiles it holds when that is one
  // fewer (the other cases keep the full panel; its surplus tiles are zero)
  if (TJ > 1 && a.h - slot0 <= 16 * (TJ - 1))
    phi_syn_stream_sweep<TI, (TJ > 1 ? TJ - 1 : 1), NW, P, CF>(a, Bs, ldb, NQ, KE, slot0, groups, grp, xcd,
                                                               tiles_j, tiles_total);
  else
    phi_syn_stream_sweep<TI, TJ, NW, P, CF>(a, Bs, ldb, NQ, KE, slot0, groups, grp, xcd, tiles_j, tiles_total);
}

template <int TI, int TJ, int NW, int P, int LDB>
__global__ __launch_bounds__(64 * NW) void phi_syn_stream(PhiStreamArgs a, int n_panels, int tiles_j,
                                                          int tiles_total) {
  phi_syn_stream_body<TI, TJ, NW, P, LDB, false>(a, n_panels, tiles_j, tiles_total);
}

// the same with the row tiles numbered colatitude row fastest
template <int TI, int TJ, int NW, int P, int LDB>
__global__ __launch_bounds__(64 * NW) void phi_syn_stream_cf(PhiStreamArgs a, int n_panels, int tiles_j,
                                                             int tiles_total) {
  phi_syn_stream_body<TI, TJ, NW, P, LDB, true>(a, n_panels, tiles_j, tiles_total);
}

// FP32 form (the separable solve's FP32 precision): the basis panel in LDS
// as FP32, the coefficients converted to FP32 as they enter the MFMA, FP32
// 16x16x4 products accumulated over FL steps (FL 4: 16 cosine and 16 sine
// columns, as the reduced-precision tiles flush every 16-wide stage) and then
// added to FP64 accumulators.  D layout of the FP32 MFMA: lane l, element r
// -> row 4 (l / 16) + r, cell l % 16.
template <int TI, int TJR, int NW, int P, bool CF>
__device__ __forceinline__ void phi_syn_stream32_sweep(const PhiStreamArgs &a, const float *Bs, int ldb, int NQ,
                                                       int KE, int slot0, int groups, int grp, int xcd,
                                                       int tiles_j, int tiles_total) {
  constexpr int TJ = TJR, FL = 4;
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  const int NQO = (a.L + 3) / 4;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, r16 = lane & 15;
  const int per = tiles_total / 8, rem = tiles_total % 8;
  const int t_beg = xcd * per + min(xcd, rem), t_end = t_beg + per + (xcd < rem ? 1 : 0);
  const int stride = groups * NW;
  int t = t_beg + grp * NW + wave;
  if (t >= t_end) return;
  auto rowbase = [&](int tt, int i) -> int {
    tt = min(tt, tiles_total - 1);
    int jl, rt;
    tile_split<CF>(tt, tiles_j, a.nt, jl, rt);
    return jl * a.Mr + min(rt * 16 * TI + 16 * i + r16, a.Mr - 1);
  };
  const int MJ = (int)a.MJ;
  auto offE = [&](int q) { return min(max(8 * q + 2 * g - 1, 0), a.nmc - 1) * MJ; };
  auto offO = [&](int q) { return min(8 * q + 2 * g + 2, a.nmc - 1) * MJ; };
  dbl4s accE[TI][TJ], accO[TI][TJ];
  f32x4 fE[TI][TJ], fO[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      accE[i][j] = dbl4s{0.0, 0.0, 0.0, 0.0};
      accO[i][j] = dbl4s{0.0, 0.0, 0.0, 0.0};
      fE[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
      fO[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  auto flush = [&]() {
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          accE[i][j][r] += (double)fE[i][j][r];
          accO[i][j][r] += (double)fO[i][j][r];
          fE[i][j][r] = 0.f;
          fO[i][j][r] = 0.f;
        }
  };
  const int n_my = (t_end - t + stride - 1) / stride;
  const int total = (n_my * NQ + P - 1) / P * P;
  int tl = t, ql = 0;
  int rbl[TI];
#pragma unroll
  for (int i = 0; i < TI; ++i) rbl[i] = rowbase(tl, i);
  // without a branch: the loads that refill a ring slot then stay after
  // the reads of its values (a load hoisted above them would need other
  // registers and a copy, after a wait for every load in flight, at the
  // end of each ring)
  auto advance_load = [&]() {
    const bool next = ++ql == NQ;
    ql = next ? 0 : ql;
    tl += next ? stride : 0;
#pragma unroll
    for (int i = 0; i < TI; ++i) rbl[i] = rowbase(tl, i);
  };
  double raE[P][TI], raO[P][TI];
  auto refill = [&](int p) {
    const int oe = offE(ql), oo = offO(ql);
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      raE[p][i] = a.V[oe + rbl[i]];
      raO[p][i] = a.V[oo + rbl[i]];
    }
    advance_load();
  };
  // slots filled in order (the waits in the loop count on slot p's loads
  // being older than slot p + 1's)
#pragma unroll
  for (int p = 0; p < P; ++p) {
    refill(p);
    __builtin_amdgcn_sched_barrier(0);
  }
  const float *bp = &Bs[r16 * ldb + g];
  float bE[TJ], bO[TJ];
#pragma unroll
  for (int j = 0; j < TJ; ++j) {
    bE[j] = bp[16 * j * ldb];
    bO[j] = bp[16 * j * ldb + KE];
  }
  int q = 0;
  for (int base = 0; base < total; base += P) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      float nE[TJ], nO[TJ];
      const int qn = q + 1 == NQ ? 0 : q + 1;
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        nE[j] = bp[16 * j * ldb + 4 * qn];
        nO[j] = bp[16 * j * ldb + KE + 4 * qn];
      }
      float aE[TI], aO[TI];
#pragma unroll
      for (int i = 0; i < TI; ++i) {
        aE[i] = (float)raE[p][i];
        aO[i] = (float)raO[p][i];
      }
      // the slot's refill after its values are converted, into the same
      // registers
      __builtin_amdgcn_sched_barrier(0);
      refill(p);
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) fE[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(aE[i], bE[j], fE[i][j], 0, 0, 0);
      if (q < NQO) {
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j) fO[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(aO[i], bO[j], fO[i][j], 0, 0, 0);
      }
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        bE[j] = nE[j];
        bO[j] = nO[j];
      }
      ++q;
      if (q % FL == 0 || q == NQ) flush();  // uniform
      if (q == NQ) {
        int jl, rt;
        tile_split<CF>(t, tiles_j, a.nt, jl, rt);
        store_row_tile<TI, TJ, true>(a, accE, accO, rt * 16 * TI, jl, slot0, g, r16, t < t_end);
        q = 0;
        t += stride;
      }
    }
  }
}

template <int TI, int TJ, int NW, int P, int LDB, bool CF>
__device__ __forceinline__ void phi_syn_stream32_body(const PhiStreamArgs &a, int n_panels, int tiles_j,
                                                      int tiles_total) {
  __shared__ float Bs[TJ * 16 * LDB];
  const int NQ = (a.L + 4) / 4;
  const int KE = 4 * NQ;
  const int ldb = 2 * KE + 2;     // 32 lanes of a 4-byte read on distinct banks
  const int xcd = blockIdx.x & 7, ib = blockIdx.x >> 3, nbx = (int)(gridDim.x >> 3);
  const int panel = ib % n_panels, grp = ib / n_panels;
  const int groups = (nbx - panel + n_panels - 1) / n_panels;
  const int slot0 = panel * TJ * 16;
  for (int e = threadIdx.x; e < TJ * 16 * 2 * KE; e += 64 * NW) {
    const int sl = e / (2 * KE), kk = e - sl * (2 * KE), slot = slot0 + sl;
    double v = 0.0;
    if (slot < a.h) {
      if (kk < KE) {
        if (kk <= a.L) v = a.TF[(long)slot * a.ldtf + kk];
      } else if (kk - KE < a.L) {
        v = a.TF[(long)slot * a.ldtf + a.ks + (kk - KE)];
      }
    }
    Bs[sl * ldb + kk] = (float)v;
  }
  __syncthreads();
  if (TJ > 1 && a.h - slot0 <= 16 * (TJ - 1))
    phi_syn_stream32_sweep<TI, (TJ > 1 ? TJ - 1 : 1), NW, P, CF>(a, Bs, ldb, NQ, KE, slot0, groups, grp, xcd,
                                                                 tiles_j, tiles_total);
  else
    phi_syn_stream32_sweep<TI, TJ, NW, P, CF>(a, Bs, ldb, NQ, KE, slot0, groups, grp, xcd, tiles_j, tiles_total);
}

template <int TI, int TJ, int NW, int P, int LDB>
__global__ __launch_bounds__(64 * NW) void phi_syn_stream32(PhiStreamArgs a, int n_panels, int tiles_j,
                                                            int tiles_total) {
  phi_syn_stream32_body<TI, TJ, NW, P, LDB, false>(a, n_panels, tiles_j, tiles_total);
}

// the same with the row tiles numbered colatitude row fastest
template <int TI, int TJ, int NW, int P, int LDB>
__global__ __launch_bounds__(64 * NW) void phi_syn_stream32_cf(PhiStreamArgs a, int n_panels, int tiles_j,
                                                               int tiles_total) {
  phi_syn_stream32_body<TI, TJ, NW, P, LDB, true>(a, n_panels, tiles_j, tiles_total);
}

// Folded phi analysis (Eqs. 14-15 and 21-22 along one colatitude row, the
// overlap weights of Eq. 25): each block keeps TJ tiles of 16 outputs of the
// colatitude-independent folded basis in LDS; its waves sweep row tiles of
// 16 TI rows, each lane loading its four contraction points of a 16-wide
// stage as one 32-byte run at the front and one at the mirror of the row
// (16 rows x 128 bytes per load), weighting the sum (cosine outputs) or the
// difference (sine outputs) as it enters the MFMA.  The products are the
// transposed tile, basis x data, so that a store covers 16 consecutive rows
// of the column-major output.
template <int TI, int TJR, int NW, int P>
__device__ __forceinline__ void phi_ana_stream_sweep(const PhiAnaStreamArgs &a, const double *Bs, int ldb, int NS,
                                                     int tile0, int groups, int grp, int xcd, int tiles_j,
                                                     int tiles_total) {
  constexpr int TJ = TJR;
  typedef double dbl2u __attribute__((ext_vector_type(2), aligned(8)));
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, r16 = lane & 15;
  const int per = tiles_total / 8, rem = tiles_total % 8;
  const int t_beg = xcd * per + min(xcd, rem), t_end = t_beg + per + (xcd < rem ? 1 : 0);
  const int stride = groups * NW;
  int t = t_beg + grp * NW + wave;
  if (t >= t_end) return;
  // element offsets of a row tile's density rows and weights (below 2^31,
  // checked by the launcher)
  auto rowbase = [&](int tt, int i) -> int {
    tt = min(tt, tiles_total - 1);
    const int jl = tt / tiles_j, rt = tt - jl * tiles_j;
    return min(rt * 16 * TI + 16 * i + r16, a.Mr - 1) * (int)a.ldr + jl * a.np;
  };
  auto wbase = [&](int tt) -> int { return (min(tt, tiles_total - 1) / tiles_j) * a.ldcs; };
  bool isE[TJ];
#pragma unroll
  for (int j = 0; j < TJ; ++j) isE[j] = tile0 + j < a.nte;
  dbl4s acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = dbl4s{0.0, 0.0, 0.0, 0.0};
  const int n_my = (t_end - t + stride - 1) / stride;
  const int total = (n_my * NS + P - 1) / P * P;
  int tl = t, sl = 0;
  int rbl[TI], wbl = wbase(tl);
#pragma unroll
  for (int i = 0; i < TI; ++i) rbl[i] = rowbase(tl, i);
  // without a branch: arithmetic on the ring's values is then not moved
  // past the loads that refill the ring (which would need other registers)
  auto advance_load = [&]() {
    const bool next = ++sl == NS;
    sl = next ? 0 : sl;
    tl += next ? stride : 0;
#pragma unroll
    for (int i = 0; i < TI; ++i) rbl[i] = rowbase(tl, i);
    wbl = wbase(tl);
  };
  // stage registers: front and mirror runs of each row tile, the weights
  double rf[P][TI][4], rb[P][TI][4], rw[P][4];
  auto load = [&](int p) {
    const int k = 16 * sl + 4 * g;
    const int kf = min(k, a.np - 4), kb = max(a.np - 4 - k, 0);  // clamped runs stay inside the row
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      const dbl2u f0 = *reinterpret_cast<const dbl2u *>(a.rho + rbl[i] + kf);
      const dbl2u f1 = *reinterpret_cast<const dbl2u *>(a.rho + rbl[i] + kf + 2);
      const dbl2u b0 = *reinterpret_cast<const dbl2u *>(a.rho + rbl[i] + kb);
      const dbl2u b1 = *reinterpret_cast<const dbl2u *>(a.rho + rbl[i] + kb + 2);
      rf[p][i][0] = f0.x;
      rf[p][i][1] = f0.y;
      rf[p][i][2] = f1.x;
      rf[p][i][3] = f1.y;
      // the mirror of point k + s is element 3 - s of the run
      rb[p][i][3] = b0.x;
      rb[p][i][2] = b0.y;
      rb[p][i][1] = b1.x;
      rb[p][i][0] = b1.y;
    }
    const dbl2u w0 = *reinterpret_cast<const dbl2u *>(a.Wt + wbl + k);
    const dbl2u w1 = *reinterpret_cast<const dbl2u *>(a.Wt + wbl + k + 2);
    rw[p][0] = w0.x;
    rw[p][1] = w0.y;
    rw[p][2] = w1.x;
    rw[p][3] = w1.y;
  };
  // slots filled in order (the waits in the loop count on slot p's loads
  // being older than slot p + 1's)
#pragma unroll
  for (int p = 0; p < P; ++p) {
    load(p);
    advance_load();
    __builtin_amdgcn_sched_barrier(0);
  }
  // lane (g, r16) reads output r16 of each tile at points 16 s + 4 g .. + 3
  const double *bp = &Bs[r16 * ldb + 4 * g];
  int st = 0;
  for (int base = 0; base < total; base += P) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      double bf[TJ][4];
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        const dbl2u v0 = *reinterpret_cast<const dbl2u *>(bp + 16 * j * ldb + 16 * st);
        const dbl2u v1 = *reinterpret_cast<const dbl2u *>(bp + 16 * j * ldb + 16 * st + 2);
        bf[j][0] = v0.x;
        bf[j][1] = v0.y;
        bf[j][2] = v1.x;
        bf[j][3] = v1.y;
      }
      double ae[TI][4], ao[TI][4];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          ae[i][s4] = rw[p][s4] * (rf[p][i][s4] + rb[p][i][s4]);
          ao[i][s4] = rw[p][s4] * (rf[p][i][s4] - rb[p][i][s4]);
        }
      // the slot's loads after its values are used, into the same registers
      __builtin_amdgcn_sched_barrier(0);
      load(p);
      advance_load();
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[j][s4], isE[j] ? ae[i][s4] : ao[i][s4], acc[i][j], 0,
                                                             0, 0);
      if (++st == NS) {
        // tile t done: lane l, element r -> output l / 16 + 4 r of the
        // tile, row l % 16
        const int jl = t / tiles_j, rt = t - jl * tiles_j;
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = rt * 16 * TI + 16 * i + r16, o = g + 4 * r;
              const int m = isE[j] ? 16 * (tile0 + j) + o : 16 * (tile0 + j - a.nte) + o + 1;
              const int mc = isE[j] ? max(2 * m - 1, 0) : 2 * m;
              if (t < t_end && row < a.Mr && m <= a.L && tile0 + j < a.nte + a.nto)
                a.X2[(long)mc * a.MJ + (long)jl * a.Mr + row] = acc[i][j][r];
              acc[i][j][r] = 0.0;
            }
        st = 0;
        t += stride;
      }
    }
  }
}

template <int TI, int TJ, int NW, int P, int LDB>
__global__ __launch_bounds__(64 * NW) void phi_ana_stream(PhiAnaStreamArgs a, int n_panels, int tiles_j,
                                                          int tiles_total) {
  __shared__ double Bs[TJ * 16 * LDB];
  const int NS = (a.h + 15) / 16;   // 16-wide stages over the folded points
  const int ldb = 16 * NS + 4;      // row stride: the 32-byte reads of 8 lanes hit distinct banks
  const int xcd = blockIdx.x & 7, ib = blockIdx.x >> 3, nbx = (int)(gridDim.x >> 3);
  const int panel = ib % n_panels, grp = ib / n_panels;
  const int groups = (nbx - panel + n_panels - 1) / n_panels;
  const int tile0 = panel * TJ, ntiles = a.nte + a.nto;
  for (int e = threadIdx.x; e < TJ * 16 * 16 * NS; e += 64 * NW) {
    const int sl = e / (16 * NS), kk = e - sl * (16 * NS), c = 16 * tile0 + sl;
    Bs[sl * ldb + kk] = (c < 16 * ntiles && kk < a.ldcs) ? a.CSF[(long)c * a.ldcs + kk] : 0.0;
  }
  __syncthreads();
  if (TJ > 1 && ntiles - tile0 <= TJ - 1)
    phi_ana_stream_sweep<TI, (TJ > 1 ? TJ - 1 : 1), NW, P>(a, Bs, ldb, NS, tile0, groups, grp, xcd, tiles_j,
                                                           tiles_total);
  else
    phi_ana_stream_sweep<TI, TJ, NW, P>(a, Bs, ldb, NS, tile0, groups, grp, xcd, tiles_j, tiles_total);
}

// FP32 form of the streaming analysis (the separable solve's FP32
// precision): the basis panel in LDS as FP32 (all 16 (nte + nto) outputs of
// a degree up to 64 fit in one panel, so each density row is read once),
// the weighted density pairs converted to FP32 as they enter the MFMA, the
// FP32 16x16x4 products of one 16-wide stage added to FP64 sums.  D layout
// of the FP32 MFMA: lane l, element r -> output 4 (l / 16) + r, row l % 16.
template <int TI, int TJR, int NW, int P>
__device__ __forceinline__ void phi_ana_stream32_sweep(const PhiAnaStreamArgs &a, const float *Bs, int ldb, int NS,
                                                       int tile0, int groups, int grp, int xcd, int tiles_j,
                                                       int tiles_total) {
  constexpr int TJ = TJR;
  typedef double dbl2u __attribute__((ext_vector_type(2), aligned(8)));
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, r16 = lane & 15;
  const int per = tiles_total / 8, rem = tiles_total % 8;
  const int t_beg = xcd * per + min(xcd, rem), t_end = t_beg + per + (xcd < rem ? 1 : 0);
  const int stride = groups * NW;
  int t = t_beg + grp * NW + wave;
  if (t >= t_end) return;
  auto rowbase = [&](int tt, int i) -> int {
    tt = min(tt, tiles_total - 1);
    const int jl = tt / tiles_j, rt = tt - jl * tiles_j;
    return min(rt * 16 * TI + 16 * i + r16, a.Mr - 1) * (int)a.ldr + jl * a.np;
  };
  auto wbase = [&](int tt) -> int { return (min(tt, tiles_total - 1) / tiles_j) * a.ldcs; };
  bool isE[TJ];
#pragma unroll
  for (int j = 0; j < TJ; ++j) isE[j] = tile0 + j < a.nte;
  dbl4s acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = dbl4s{0.0, 0.0, 0.0, 0.0};
  const int n_my = (t_end - t + stride - 1) / stride;
  const int total = (n_my * NS + P - 1) / P * P;
  int tl = t, sl = 0;
  int rbl[TI], wbl = wbase(tl);
#pragma unroll
  for (int i = 0; i < TI; ++i) rbl[i] = rowbase(tl, i);
  // without a branch: arithmetic on the ring's values is then not moved
  // past the loads that refill the ring (which would need other registers)
  auto advance_load = [&]() {
    const bool next = ++sl == NS;
    sl = next ? 0 : sl;
    tl += next ? stride : 0;
#pragma unroll
    for (int i = 0; i < TI; ++i) rbl[i] = rowbase(tl, i);
    wbl = wbase(tl);
  };
  double rf[P][TI][4], rb[P][TI][4], rw[P][4];
  auto load = [&](int p) {
    const int k = 16 * sl + 4 * g;
    const int kf = min(k, a.np - 4), kb = max(a.np - 4 - k, 0);
#pragma unroll
    for (int i = 0; i < TI; ++i) {
      const dbl2u f0 = *reinterpret_cast<const dbl2u *>(a.rho + rbl[i] + kf);
      const dbl2u f1 = *reinterpret_cast<const dbl2u *>(a.rho + rbl[i] + kf + 2);
      const dbl2u b0 = *reinterpret_cast<const dbl2u *>(a.rho + rbl[i] + kb);
      const dbl2u b1 = *reinterpret_cast<const dbl2u *>(a.rho + rbl[i] + kb + 2);
      rf[p][i][0] = f0.x;
      rf[p][i][1] = f0.y;
      rf[p][i][2] = f1.x;
      rf[p][i][3] = f1.y;
      rb[p][i][3] = b0.x;
      rb[p][i][2] = b0.y;
      rb[p][i][1] = b1.x;
      rb[p][i][0] = b1.y;
    }
    const dbl2u w0 = *reinterpret_cast<const dbl2u *>(a.Wt + wbl + k);
    const dbl2u w1 = *reinterpret_cast<const dbl2u *>(a.Wt + wbl + k + 2);
    rw[p][0] = w0.x;
    rw[p][1] = w0.y;
    rw[p][2] = w1.x;
    rw[p][3] = w1.y;
  };
  // slots filled in order (the waits in the loop count on slot p's loads
  // being older than slot p + 1's)
#pragma unroll
  for (int p = 0; p < P; ++p) {
    load(p);
    advance_load();
    __builtin_amdgcn_sched_barrier(0);
  }
  const float *bp = &Bs[r16 * ldb + 4 * g];
  int st = 0;
  for (int base = 0; base < total; base += P) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      float ae[TI][4], ao[TI][4];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          ae[i][s4] = (float)(rw[p][s4] * (rf[p][i][s4] + rb[p][i][s4]));
          ao[i][s4] = (float)(rw[p][s4] * (rf[p][i][s4] - rb[p][i][s4]));
        }
      // the slot's loads after its values are used, into the same
      // registers: a load hoisted above them would need other registers and
      // a copy (after a wait for every load in flight) at the loop's end
      __builtin_amdgcn_sched_barrier(0);
      load(p);
      advance_load();
      // tiles in groups of G: the group's basis fragments first, then its
      // TI x G independent product chains interleaved step by step (the
      // matrix pipe does not wait on one chain), then its FP32 sums added
      // to the FP64 ones; a small group keeps registers for the ring
      constexpr int G = TJ < 3 ? TJ : 3;
#pragma unroll
      for (int j0 = 0; j0 < TJ; j0 += G) {
        f32x4 bf[G], f[TI][G];
#pragma unroll
        for (int u = 0; u < G; ++u)
          if (j0 + u < TJ) bf[u] = *reinterpret_cast<const f32x4 *>(bp + 16 * (j0 + u) * ldb + 16 * st);
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
          for (int i = 0; i < TI; ++i)
#pragma unroll
            for (int u = 0; u < G; ++u)
              if (j0 + u < TJ)
                f[i][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                    bf[u][s4], isE[j0 + u] ? ae[i][s4] : ao[i][s4], s4 == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : f[i][u],
                    0, 0, 0);
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int u = 0; u < G; ++u)
            if (j0 + u < TJ)
#pragma unroll
              for (int r = 0; r < 4; ++r) acc[i][j0 + u][r] += (double)f[i][u][r];
      }
      if (++st == NS) {
        const int jl = t / tiles_j, rt = t - jl * tiles_j;
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = rt * 16 * TI + 16 * i + r16, o = 4 * g + r;
              const int m = isE[j] ? 16 * (tile0 + j) + o : 16 * (tile0 + j - a.nte) + o + 1;
              const int mc = isE[j] ? max(2 * m - 1, 0) : 2 * m;
              if (t < t_end && row < a.Mr && m <= a.L && tile0 + j < a.nte + a.nto)
                a.X2[(long)mc * a.MJ + (long)jl * a.Mr + row] = acc[i][j][r];
              acc[i][j][r] = 0.0;
            }
        st = 0;
        t += stride;
      }
    }
  }
}

template <int TI, int TJ, int NW, int P, int LDB>
__global__ __launch_bounds__(64 * NW) void phi_ana_stream32(PhiAnaStreamArgs a, int n_panels, int tiles_j,
                                                            int tiles_total) {
  __shared__ float Bs[TJ * 16 * LDB];
  const int NS = (a.h + 15) / 16;
  const int ldb = 16 * NS + 4;      // floats: the 16-byte reads of 8 lanes hit distinct banks
  const int xcd = blockIdx.x & 7, ib = blockIdx.x >> 3, nbx = (int)(gridDim.x >> 3);
  const int panel = ib % n_panels, grp = ib / n_panels;
  const int groups = (nbx - panel + n_panels - 1) / n_panels;
  const int tile0 = panel * TJ, ntiles = a.nte + a.nto;
  for (int e = threadIdx.x; e < TJ * 16 * 16 * NS; e += 64 * NW) {
    const int sl = e / (16 * NS), kk = e - sl * (16 * NS), c = 16 * tile0 + sl;
    Bs[sl * ldb + kk] = (c < 16 * ntiles && kk < a.ldcs) ? (float)a.CSF[(long)c * a.ldcs + kk] : 0.f;
  }
  __syncthreads();
  if (TJ > 1 && ntiles - tile0 <= TJ - 1)
    phi_ana_stream32_sweep<TI, (TJ > 1 ? TJ - 1 : 1), NW, P>(a, Bs, ldb, NS, tile0, groups, grp, xcd, tiles_j,
                                                             tiles_total);
  else
    phi_ana_stream32_sweep<TI, TJ, NW, P>(a, Bs, ldb, NS, tile0, groups, grp, xcd, tiles_j, tiles_total);
}

namespace {

struct StreamVariant {
  int ti, tj, nw, p, ldb, bpc;
  void (*kernel)(PhiStreamArgs, int, int, int);
  const char *name;
};

#define YYG_STREAM(TI, TJ, NW, P, LDB, BPC)                                                             \
  {                                                                                                     \
    TI, TJ, NW, P, LDB, BPC, phi_syn_stream<TI, TJ, NW, P, LDB>,                                        \
        "yyg::phi_syn_stream<" #TI ", " #TJ ", " #NW ", " #P ", " #LDB ">"                              \
  }

#define YYG_STREAM_CF(TI, TJ, NW, P, LDB, BPC)                                                          \
  {                                                                                                     \
    TI, TJ, NW, P, LDB, BPC, phi_syn_stream_cf<TI, TJ, NW, P, LDB>,                                     \
        "yyg::phi_syn_stream_cf<" #TI ", " #TJ ", " #NW ", " #P ", " #LDB ">"                           \
  }

// a variant serves the degrees whose panel rows (8 ceil((L+1)/4) + 2
// doubles) fit its LDB: L <= 67 at 138, L <= 131 at 266
const StreamVariant kStream[] = {
    YYG_STREAM(1, 6, 8, 4, 138, 1), YYG_STREAM(1, 4, 8, 8, 138, 1), YYG_STREAM(1, 3, 4, 8, 138, 3),
    YYG_STREAM(1, 6, 8, 8, 138, 1), YYG_STREAM(1, 9, 8, 4, 138, 1), YYG_STREAM(1, 9, 8, 2, 138, 1),
    YYG_STREAM(1, 3, 8, 4, 266, 1), YYG_STREAM_CF(1, 9, 8, 4, 138, 1), YYG_STREAM_CF(1, 6, 8, 4, 138, 1),
    YYG_STREAM_CF(1, 9, 8, 2, 138, 1), YYG_STREAM(1, 9, 8, 8, 138, 1), YYG_STREAM(1, 6, 8, 12, 138, 1),
    YYG_STREAM_CF(1, 6, 8, 8, 138, 1), YYG_STREAM_CF(1, 9, 8, 8, 138, 1),
    YYG_STREAM_CF(2, 6, 4, 4, 138, 1), YYG_STREAM(2, 6, 4, 4, 138, 1),
};

#define YYG_STREAM32(TI, TJ, NW, P, LDB, BPC)                                                           \
  {                                                                                                     \
    TI, TJ, NW, P, LDB, BPC, phi_syn_stream32<TI, TJ, NW, P, LDB>,                                      \
        "yyg::phi_syn_stream32<" #TI ", " #TJ ", " #NW ", " #P ", " #LDB ">"                            \
  }

#define YYG_STREAM32_CF(TI, TJ, NW, P, LDB, BPC)                                                        \
  {                                                                                                     \
    TI, TJ, NW, P, LDB, BPC, phi_syn_stream32_cf<TI, TJ, NW, P, LDB>,                                   \
        "yyg::phi_syn_stream32_cf<" #TI ", " #TJ ", " #NW ", " #P ", " #LDB ">"                         \
  }

// FP32 panels: LDB floats per row (L <= 67 at 138, L <= 131 at 266)
const StreamVariant kStream32[] = {
    YYG_STREAM32(1, 6, 8, 4, 138, 1), YYG_STREAM32(1, 4, 4, 8, 138, 2), YYG_STREAM32(1, 5, 8, 4, 138, 1),
    YYG_STREAM32(1, 3, 4, 4, 138, 2), YYG_STREAM32(1, 6, 8, 4, 266, 1), YYG_STREAM32_CF(1, 6, 8, 4, 138, 1),
    YYG_STREAM32_CF(1, 6, 8, 4, 266, 1), YYG_STREAM32(1, 6, 8, 8, 138, 1), YYG_STREAM32_CF(1, 6, 8, 8, 138, 1),
};

struct AnaVariant {
  int ti, tj, nw, p, ldb, bpc;
  void (*kernel)(PhiAnaStreamArgs, int, int, int);
  const char *name;
};

#define YYG_ANA_STREAM(TI, TJ, NW, P, LDB, BPC)                                                         \
  {                                                                                                     \
    TI, TJ, NW, P, LDB, BPC, phi_ana_stream<TI, TJ, NW, P, LDB>,                                        \
        "yyg::phi_ana_stream<" #TI ", " #TJ ", " #NW ", " #P ", " #LDB ">"                              \
  }

// panels of TJ tiles x LDB points (16 ceil(h / 16) + 4 <= LDB: h <= 272 at 276)
const AnaVariant kAna[] = {
    YYG_ANA_STREAM(2, 3, 8, 2, 276, 1), YYG_ANA_STREAM(1, 3, 8, 2, 276, 1), YYG_ANA_STREAM(1, 3, 8, 4, 276, 1),
    YYG_ANA_STREAM(2, 2, 8, 2, 276, 1), YYG_ANA_STREAM(2, 3, 4, 2, 276, 1), YYG_ANA_STREAM(1, 2, 4, 4, 420, 1),
    YYG_ANA_STREAM(1, 3, 8, 6, 276, 1), YYG_ANA_STREAM(2, 2, 8, 3, 276, 1),
};

#define YYG_ANA_STREAM32(TI, TJ, NW, P, LDB, BPC)                                                       \
  {                                                                                                     \
    TI, TJ, NW, P, LDB, BPC, phi_ana_stream32<TI, TJ, NW, P, LDB>,                                      \
        "yyg::phi_ana_stream32<" #TI ", " #TJ ", " #NW ", " #P ", " #LDB ">"                            \
  }

// FP32 panels: 9 tiles (lmax <= 64 in one panel) x 276 floats (h <= 272)
const AnaVariant kAna32[] = {
    YYG_ANA_STREAM32(1, 9, 8, 1, 276, 1), YYG_ANA_STREAM32(1, 5, 8, 2, 276, 1), YYG_ANA_STREAM32(1, 5, 8, 1, 276, 1),
    YYG_ANA_STREAM32(1, 9, 4, 4, 276, 1), YYG_ANA_STREAM32(1, 9, 4, 3, 276, 1), YYG_ANA_STREAM32(1, 9, 4, 2, 276, 1),
    YYG_ANA_STREAM32(1, 9, 8, 2, 276, 1),
};

}  // namespace

int phi_ana_stream32_variant_count() { return (int)(sizeof(kAna32) / sizeof(kAna32[0])); }

bool phi_ana_stream32_supports(int v, int h, int np) {
  return v >= 0 && v < phi_ana_stream32_variant_count() && np >= 8 && 16 * ((h + 15) / 16) + 4 <= kAna32[v].ldb;
}

int phi_ana_stream32_kernel_name(int v, char *buf, size_t n) {
  if (v < 0 || v >= phi_ana_stream32_variant_count()) return -1;
  return snprintf(buf, n, "%s", kAna32[v].name) < 0 ? -1 : 0;
}

int phi_ana_stream_variant_count() { return (int)(sizeof(kAna) / sizeof(kAna[0])); }

bool phi_ana_stream_supports(int v, int h, int np) {
  return v >= 0 && v < phi_ana_stream_variant_count() && np >= 8 && 16 * ((h + 15) / 16) + 4 <= kAna[v].ldb;
}

int phi_ana_stream_kernel_name(int v, char *buf, size_t n) {
  if (v < 0 || v >= phi_ana_stream_variant_count()) return -1;
  return snprintf(buf, n, "%s", kAna[v].name) < 0 ? -1 : 0;
}

namespace {

hipError_t launch_ana(const AnaVariant &k, const PhiAnaStreamArgs &a, int cus, hipStream_t s) {
  if (a.Mr <= 0 || a.nt <= 0 || a.h <= 0) return hipSuccess;
  // 32-bit element offsets of the density in the kernel
  if ((long)a.Mr * a.ldr >= INT_MAX || (long)a.nt * a.ldcs >= INT_MAX) return hipErrorInvalidValue;
  const int rows = 16 * k.ti;
  const long tj = (a.Mr + rows - 1) / rows, tt = tj * a.nt;
  if (tt >= INT_MAX / 2) return hipErrorInvalidValue;
  const int n_panels = (a.nte + a.nto + k.tj - 1) / k.tj;
  int per_xcd = std::max(n_panels, k.bpc * std::max(cus, 8) / 8);
  const dim3 grid(8 * per_xcd), block(64 * k.nw);
  hipLaunchKernelGGL(k.kernel, grid, block, 0, s, a, n_panels, (int)tj, (int)tt);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_phi_ana_stream(int v, const PhiAnaStreamArgs &a, int cus, hipStream_t s) {
  if (!phi_ana_stream_supports(v, a.h, a.np)) return hipErrorInvalidValue;
  return launch_ana(kAna[v], a, cus, s);
}

hipError_t launch_phi_ana_stream32(int v, const PhiAnaStreamArgs &a, int cus, hipStream_t s) {
  if (!phi_ana_stream32_supports(v, a.h, a.np)) return hipErrorInvalidValue;
  return launch_ana(kAna32[v], a, cus, s);
}

int phi_stream32_variant_count() { return (int)(sizeof(kStream32) / sizeof(kStream32[0])); }

bool phi_stream32_supports(int v, int L) {
  return v >= 0 && v < phi_stream32_variant_count() && L >= 0 && 8 * ((L + 4) / 4) + 2 <= kStream32[v].ldb;
}

int phi_stream32_kernel_name(int v, char *buf, size_t n) {
  if (v < 0 || v >= phi_stream32_variant_count()) return -1;
  return snprintf(buf, n, "%s", kStream32[v].name) < 0 ? -1 : 0;
}

int phi_stream_variant_count() { return (int)(sizeof(kStream) / sizeof(kStream[0])); }

bool phi_stream_supports(int v, int L) {
  return v >= 0 && v < phi_stream_variant_count() && L >= 0 && 8 * ((L + 4) / 4) + 2 <= kStream[v].ldb;
}

int phi_stream_kernel_name(int v, char *buf, size_t n) {
  if (v < 0 || v >= phi_stream_variant_count()) return -1;
  return snprintf(buf, n, "%s", kStream[v].name) < 0 ? -1 : 0;
}

namespace {

hipError_t launch_stream(const StreamVariant &k, const PhiStreamArgs &a, int cus, hipStream_t s) {
  if (a.Mr <= 0 || a.nt <= 0 || a.h <= 0) return hipSuccess;
  // element offsets of the coefficients are 32-bit in the kernel
  if ((long)a.nmc * a.MJ >= INT_MAX) return hipErrorInvalidValue;
  const int rows = 16 * k.ti;
  const long tj = (a.Mr + rows - 1) / rows, tt = tj * a.nt;
  if (tt >= INT_MAX / 2) return hipErrorInvalidValue;
  const int n_panels = (a.h + 16 * k.tj - 1) / (16 * k.tj);
  // a whole number of blocks per XCD, at least one per panel on each
  int per_xcd = std::max(n_panels, k.bpc * std::max(cus, 8) / 8);
  const dim3 grid(8 * per_xcd), block(64 * k.nw);
  hipLaunchKernelGGL(k.kernel, grid, block, 0, s, a, n_panels, (int)tj, (int)tt);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_phi_syn_stream(int v, const PhiStreamArgs &a, int cus, hipStream_t s) {
  if (!phi_stream_supports(v, a.L)) return hipErrorInvalidValue;
  return launch_stream(kStream[v], a, cus, s);
}

hipError_t launch_phi_syn_stream32(int v, const PhiStreamArgs &a, int cus, hipStream_t s) {
  if (!phi_stream32_supports(v, a.L)) return hipErrorInvalidValue;
  return launch_stream(kStream32[v], a, cus, s);
}

}  // namespace yyg
