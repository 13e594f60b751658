// Batched dense products and elementwise steps of the Laplace cascade
// (internal; kernels in jk_gemm.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace jk {

// C[b] = alpha op(A[b]) op(B[b]) + beta C[b] for b < batch; row-major with
// leading dimensions lda, ldb, ldc and batch strides sa, sb, sc (elements;
// 0 repeats one matrix); op(A) is M x K (A[k][m] read when ta), op(B) K x N
// (B[n][k] read when tb).  With gcols > 0 the columns of C come in groups of
// gcols, group g starting gstride elements after group g - 1 (column n of
// row m at m ldc + (n / gcols) gstride + n % gcols).  With klast > 0 the
// last batch sums over its first klast values of k only (a split-K
// product whose last piece is shorter).
struct GemmArgs {
    const double* A;
    const double* B;
    double* C;
    int M, N, K, ta, tb, lda, ldb, ldc;
    long long sa, sb, sc;
    double alpha, beta;
    int gcols;
    long long gstride;
    int klast;
};
hipError_t launch_gemm(const GemmArgs& g, int batch, hipStream_t s);

constexpr int kMaxTaus = 64;
struct ScaleTaus {
    double t[kMaxTaus];
    int n;
};
// out[k][i][c] = C[i][c0 + c] exp(sign eps[c0 + c] tau_k), C row-major [n][nmo]
hipError_t launch_scale_cols(const double* Cm, int n, int nmo, int c0, int ncols, const double* eps,
                             const ScaleTaus& taus, double sign, double* out, hipStream_t s);
// out = a x + b y
hipError_t launch_axpby(long long n, double a, const double* x, double b, const double* y, double* out, hipStream_t s);

}  // namespace jk
