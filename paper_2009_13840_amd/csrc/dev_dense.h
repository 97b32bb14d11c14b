// Block-cooperative dense factorisations (one workgroup, any address space).
#pragma once

#include <hip/hip_runtime.h>

namespace hho {

// In-place lower Cholesky of A (n x n, leading dimension lda).  Sets *bad when a
// pivot is not positive.
__device__ inline void blk_chol(double *A, int n, int lda, int *bad) {
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      double v = A[j * lda + j];
      if (!(v > 0.0)) {
        *bad = 1;
        v = 1.0;
      }
      A[j * lda + j] = sqrt(v);
    }
    __syncthreads();
    const double ljj = A[j * lda + j];
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) A[i * lda + j] /= ljj;
    __syncthreads();
    const int r = n - j - 1;
    for (int idx = threadIdx.x; idx < r * r; idx += blockDim.x) {
      const int i = j + 1 + idx / r, k = j + 1 + idx % r;
      if (k <= i) A[i * lda + k] -= A[i * lda + j] * A[k * lda + j];
    }
    __syncthreads();
  }
}

// Forward substitution L y = b on ncol columns of B (column c at B + c*cs, rows
// strided by rs), one column per thread.
__device__ inline void blk_fwd(const double *L, int n, int lda, double *B, int ncol, int64_t cs, int64_t rs) {
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
    double *b = B + c * cs;
    for (int i = 0; i < n; ++i) {
      double v = b[i * rs];
      for (int k = 0; k < i; ++k) v -= L[i * lda + k] * b[k * rs];
      b[i * rs] = v / L[i * lda + i];
    }
  }
}

// Backward substitution L^T y = b on ncol columns of B (layout as blk_fwd).
__device__ inline void blk_bwd(const double *L, int n, int lda, double *B, int ncol, int64_t cs, int64_t rs) {
  for (int c = threadIdx.x; c < ncol; c += blockDim.x) {
    double *b = B + c * cs;
    for (int i = n - 1; i >= 0; --i) {
      double v = b[i * rs];
      for (int k = i + 1; k < n; ++k) v -= L[k * lda + i] * b[k * rs];
      b[i * rs] = v / L[i * lda + i];
    }
  }
}

// X = (L L^T)^{-1} (n x n, leading dimension ldx), one column per thread.
__device__ inline void blk_chol_inverse(const double *L, int n, int lda, double *X, int ldx) {
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    for (int i = 0; i < n; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) v -= L[i * lda + k] * X[k * ldx + c];
      X[i * ldx + c] = v / L[i * lda + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double v = X[i * ldx + c];
      for (int k = i + 1; k < n; ++k) v -= L[k * lda + i] * X[k * ldx + c];
      X[i * ldx + c] = v / L[i * lda + i];
    }
  }
  __syncthreads();
}

}  // namespace hho
