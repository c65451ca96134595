// Workgroup-level dense linear algebra for the batched local problems of
// the hierarchy setup (one workgroup per aggregate or coarse interface).
// Matrices are row-major with a leading dimension; all threads of the block
// call each routine; results are complete after the call returns.
#pragma once

#include <hip/hip_runtime.h>

namespace spfas {

__device__ inline void wg_sync() { __syncthreads(); }

__device__ inline void wg_fill(double* a, int n, double v) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) a[i] = v;
  wg_sync();
}

// In-place lower Cholesky A = L L^T (upper part left untouched).  Returns
// false (in every thread) when a pivot is not positive.
__device__ inline bool wg_chol(double* A, int n, int ld, int* flag) {
  if (threadIdx.x == 0) *flag = 0;
  wg_sync();
  for (int k = 0; k < n; ++k) {
    const double d = A[k * ld + k];
    if (!(d > 0.0)) {
      if (threadIdx.x == 0) *flag = k + 1;   // 1-based index of the failing pivot
      wg_sync();
      return false;
    }
    const double s = sqrt(d);
    wg_sync();
    if (threadIdx.x == 0) A[k * ld + k] = s;
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) A[i * ld + k] /= s;
    wg_sync();
    const int rem = n - k - 1;
    for (int e = threadIdx.x; e < rem * rem; e += blockDim.x) {
      const int i = k + 1 + e / rem, j = k + 1 + e % rem;
      if (j <= i) A[i * ld + j] -= A[i * ld + k] * A[j * ld + k];
    }
    wg_sync();
  }
  return *flag == 0;
}

// B <- (L L^T)^{-1} B for B of n rows and nrhs columns (row-major, ldb).
__device__ inline void wg_chol_solve(const double* L, int n, int ld, double* B, int nrhs, int ldb) {
  for (int k = 0; k < n; ++k) {
    const double d = L[k * ld + k];
    for (int c = threadIdx.x; c < nrhs; c += blockDim.x) B[k * ldb + c] /= d;
    wg_sync();
    const int rem = n - k - 1;
    for (int e = threadIdx.x; e < rem * nrhs; e += blockDim.x) {
      const int i = k + 1 + e / nrhs, c = e % nrhs;
      B[i * ldb + c] -= L[i * ld + k] * B[k * ldb + c];
    }
    wg_sync();
  }
  for (int k = n - 1; k >= 0; --k) {
    const double d = L[k * ld + k];
    for (int c = threadIdx.x; c < nrhs; c += blockDim.x) B[k * ldb + c] /= d;
    wg_sync();
    for (int e = threadIdx.x; e < k * nrhs; e += blockDim.x) {
      const int i = e / nrhs, c = e % nrhs;
      B[i * ldb + c] -= L[k * ld + i] * B[k * ldb + c];
    }
    wg_sync();
  }
}

// C (m x n) = op(A) op(B) with op = transpose when the flag is set.
// A is (m x k) or (k x m), B is (k x n) or (n x k).
__device__ inline void wg_gemm(const double* A, int lda, bool ta, const double* B, int ldb, bool tb, double* C,
                               int ldc, int m, int n, int k, double beta = 0.0) {
  for (int e = threadIdx.x; e < m * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    double s = 0.0;
    for (int q = 0; q < k; ++q) {
      const double a = ta ? A[q * lda + i] : A[i * lda + q];
      const double b = tb ? B[j * ldb + q] : B[q * ldb + j];
      s += a * b;
    }
    // C is not read when beta == 0: it may hold any bit pattern (NaN included)
    C[i * ldc + j] = (beta == 0.0) ? s : beta * C[i * ldc + j] + s;
  }
  wg_sync();
}

// Symmetric eigen-decomposition by the cyclic Jacobi method with the
// round-robin (tournament) ordering, so that n/2 disjoint rotations are
// applied in parallel.  A (n x n) is overwritten (diagonal = eigenvalues,
// unsorted); V receives the eigenvectors as columns.  `cs` needs 2*(n/2+1)
// doubles and `pr` 2*(n/2+1) ints of scratch (shared or global).
__device__ inline void wg_jacobi_eig(double* A, int lda, double* V, int ldv, int n, double* cs, int* pr,
                                     double* red, int max_sweeps = 40) {
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) V[(e / n) * ldv + e % n] = ((e / n) == (e % n)) ? 1.0 : 0.0;
  wg_sync();
  if (n < 2) return;
  const int np = (n + 1) / 2;          // pairs per round
  const int nn = 2 * np;               // padded size (a dummy index n when n is odd)
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    // Frobenius norm and off-diagonal norm
    double fro = 0.0, off = 0.0;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
      const int i = e / n, j = e % n;
      const double a = A[i * lda + j];
      fro += a * a;
      if (i != j) off += a * a;
    }
    // block reduction through `red`
    red[threadIdx.x] = fro;
    red[blockDim.x + threadIdx.x] = off;
    wg_sync();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o) {
        red[threadIdx.x] += red[threadIdx.x + o];
        red[blockDim.x + threadIdx.x] += red[blockDim.x + threadIdx.x + o];
      }
      wg_sync();
    }
    fro = red[0];
    off = red[blockDim.x];
    wg_sync();
    if (off <= 1e-30 * fro || fro == 0.0) break;
    const double tiny = 1e-18 * sqrt(fro);
    for (int round = 0; round < nn - 1; ++round) {
      // tournament pairing: position 0 fixed, the others rotate
      for (int q = threadIdx.x; q < np; q += blockDim.x) {
        int a = (q == 0) ? 0 : 1 + (q - 1 + round) % (nn - 1);
        int b = 1 + (nn - 2 - q + round) % (nn - 1);
        if (a > b) { const int t = a; a = b; b = t; }
        double c = 1.0, s = 0.0;
        if (b < n) {
          const double apq = A[a * lda + b];
          if (fabs(apq) > tiny) {
            const double app = A[a * lda + a], aqq = A[b * lda + b];
            const double tau = (aqq - app) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
          }
        }
        pr[2 * q] = a;
        pr[2 * q + 1] = b;
        cs[2 * q] = c;
        cs[2 * q + 1] = s;
      }
      wg_sync();
      // rows: A <- J^T A
      for (int e = threadIdx.x; e < np * n; e += blockDim.x) {
        const int q = e / n, j = e % n;
        const int a = pr[2 * q], b = pr[2 * q + 1];
        const double s = cs[2 * q + 1];
        if (b >= n || s == 0.0) continue;
        const double c = cs[2 * q];
        const double x = A[a * lda + j], y = A[b * lda + j];
        A[a * lda + j] = c * x - s * y;
        A[b * lda + j] = s * x + c * y;
      }
      wg_sync();
      // columns: A <- A J, V <- V J
      for (int e = threadIdx.x; e < np * n; e += blockDim.x) {
        const int q = e / n, i = e % n;
        const int a = pr[2 * q], b = pr[2 * q + 1];
        const double s = cs[2 * q + 1];
        if (b >= n || s == 0.0) continue;
        const double c = cs[2 * q];
        const double x = A[i * lda + a], y = A[i * lda + b];
        A[i * lda + a] = c * x - s * y;
        A[i * lda + b] = s * x + c * y;
        const double u = V[i * ldv + a], w = V[i * ldv + b];
        V[i * ldv + a] = c * u - s * w;
        V[i * ldv + b] = s * u + c * w;
      }
      wg_sync();
    }
  }
}

}  // namespace spfas
