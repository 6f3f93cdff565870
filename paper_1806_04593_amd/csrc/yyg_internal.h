// Internal launch interface between the C-ABI layer and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace yyg {

// FP64 NT GEMM C = A . B^T in one of several tile shapes ("variants");
// role 0 = analysis, 1 = synthesis (separate kernel symbols).
int gemm_f64_variant_count();
void gemm_f64_variant_tile(int variant, int *bm, int *bn);
hipError_t launch_gemm_nt_f64(int variant, int role, int M, int N, int K, const double *A, long lda, const double *B,
                              long ldb, double *C, long ldc, int nsplit, long c_split_stride, hipStream_t s);

hipError_t launch_radial_scan(const double *part, int nsplit, long split_stride, double *Ahat, const double *coef,
                              const int *qdeg, int nR, int Q, int L, double negG, double *U, long ldu,
                              hipStream_t s);

hipError_t launch_expand_analysis_basis(const double *w, const double *Tt, const double *CS, int n_t, int n_p,
                                        int Q, double *Bt, long ldb, hipStream_t s);

hipError_t launch_expand_self_basis(const double *P, const double *Tr, int n_t, int n_p, int Q, double *Y, long ldy,
                                    hipStream_t s);

// Split-K factor for an output of `tiles` block tiles and K columns.
int choose_split(long tiles, long K);

}  // namespace yyg
