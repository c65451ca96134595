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

// The routines below assume blockDim.x == 256 (the setup kernels' block).
constexpr int kGemmTile = 64;   // output tile edge of the tiled product
constexpr int kGemmKc = 16;     // depth of one staged slice
constexpr int kCholNb = 32;     // panel width of the blocked factorisation and solves

// C (m x n) = alpha op(A) op(B) + beta C, op = transpose when the flag is set
// (A is m x k or k x m, B is k x n or n x k).  64 x 64 output tiles, 4 x 4
// per thread, depth-16 slices of A and B staged in LDS.  lower_only skips
// the tiles strictly above the diagonal (updates whose upper part is never
// read).  C is not read when beta == 0: it may hold any bit pattern.
__device__ inline void wg_gemm_acc(const double* A, int lda, bool ta, const double* B, int ldb, bool tb, double* C,
                                   int ldc, int m, int n, int k, double alpha, double beta, bool lower_only) {
  __shared__ double As[kGemmKc][kGemmTile + 1];
  __shared__ double Bs[kGemmKc][kGemmTile + 1];
  const int t = threadIdx.x;
  const int tr = t >> 4, tc = t & 15;
  for (int i0 = 0; i0 < m; i0 += kGemmTile)
    for (int j0 = 0; j0 < n; j0 += kGemmTile) {
      if (lower_only && j0 > i0) continue;
      double acc[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
      for (int q0 = 0; q0 < k; q0 += kGemmKc) {
        for (int e = t; e < kGemmKc * kGemmTile; e += 256) {
          // contiguous memory runs along the fastest-varying index of the thread
          int q, i;
          if (ta) { q = e / kGemmTile; i = e % kGemmTile; } else { i = e / kGemmKc; q = e % kGemmKc; }
          const int gi = i0 + i, gq = q0 + q;
          As[q][i] = (gi < m && gq < k) ? (ta ? A[(size_t)gq * lda + gi] : A[(size_t)gi * lda + gq]) : 0.0;
          int j, q2;
          if (tb) { j = e / kGemmKc; q2 = e % kGemmKc; } else { q2 = e / kGemmTile; j = e % kGemmTile; }
          const int gj = j0 + j, gq2 = q0 + q2;
          Bs[q2][j] = (gj < n && gq2 < k) ? (tb ? B[(size_t)gj * ldb + gq2] : B[(size_t)gq2 * ldb + gj]) : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int q = 0; q < kGemmKc; ++q) {
          double av[4], bv[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) av[r] = As[q][tr * 4 + r];
#pragma unroll
          for (int c = 0; c < 4; ++c) bv[c] = Bs[q][tc * 4 + c];
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] += av[r] * bv[c];
        }
        __syncthreads();
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int gi = i0 + tr * 4 + r, gj = j0 + tc * 4 + c;
          if (gi < m && gj < n) {
            double* cp = C + (size_t)gi * ldc + gj;
            *cp = (beta == 0.0) ? alpha * acc[r][c] : beta * *cp + alpha * acc[r][c];
          }
        }
    }
  __syncthreads();
}

// C (m x n) = op(A) op(B) (+ beta C); see wg_gemm_acc.
__device__ inline void wg_gemm(const double* A, int lda, bool ta, const double* B, int ldb, bool tb, double* C,
                               int ldc, int m, int n, int k, double beta = 0.0) {
  wg_gemm_acc(A, lda, ta, B, ldb, tb, C, ldc, m, n, k, 1.0, beta, false);
}

// Unblocked in-place lower Cholesky of an n x n block; on a non-positive
// pivot sets *flag = base + (1-based pivot index) and returns false.
__device__ inline bool wg_chol_unblocked(double* A, int n, int ld, int* flag, int base) {
  for (int k = 0; k < n; ++k) {
    const double d = A[k * ld + k];
    if (!(d > 0.0)) {
      if (threadIdx.x == 0) *flag = base + k + 1;
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
  return true;
}

// In-place lower Cholesky A = L L^T (upper part left untouched): right-
// looking with 32-column panels; the trailing updates run on the tiled
// product.  Returns false (in every thread) when a pivot is not positive,
// with *flag = 1-based index of that pivot.
__device__ inline bool wg_chol(double* A, int n, int ld, int* flag) {
  if (threadIdx.x == 0) *flag = 0;
  wg_sync();
  for (int k0 = 0; k0 < n; k0 += kCholNb) {
    const int kb = min(kCholNb, n - k0);
    double* A11 = A + (size_t)k0 * ld + k0;
    if (!wg_chol_unblocked(A11, kb, ld, flag, k0)) return false;
    const int rem = n - k0 - kb;
    if (rem <= 0) break;
    // panel: every row below solves x L11^T = a
    for (int i = threadIdx.x; i < rem; i += blockDim.x) {
      double* row = A + (size_t)(k0 + kb + i) * ld + k0;
      for (int j = 0; j < kb; ++j) {
        double v = row[j];
        for (int l = 0; l < j; ++l) v -= row[l] * A11[j * ld + l];
        row[j] = v / A11[j * ld + j];
      }
    }
    wg_sync();
    double* L21 = A + (size_t)(k0 + kb) * ld + k0;
    wg_gemm_acc(L21, ld, false, L21, ld, true, A + (size_t)(k0 + kb) * ld + k0 + kb, ld, rem, rem, kb, -1.0, 1.0,
                true);
  }
  return *flag == 0;
}

// B <- (L L^T)^{-1} B for B of n rows and nrhs columns (row-major, ldb):
// forward then backward substitution in 32-row blocks, the off-diagonal
// block updates on the tiled product.
__device__ inline void wg_chol_solve(const double* L, int n, int ld, double* B, int nrhs, int ldb) {
  for (int k0 = 0; k0 < n; k0 += kCholNb) {
    const int kb = min(kCholNb, n - k0);
    const double* L11 = L + (size_t)k0 * ld + k0;
    for (int c = threadIdx.x; c < nrhs; c += blockDim.x)
      for (int j = 0; j < kb; ++j) {
        double v = B[(size_t)(k0 + j) * ldb + c];
        for (int l = 0; l < j; ++l) v -= L11[j * ld + l] * B[(size_t)(k0 + l) * ldb + c];
        B[(size_t)(k0 + j) * ldb + c] = v / L11[j * ld + j];
      }
    wg_sync();
    const int rem = n - k0 - kb;
    if (rem > 0)
      wg_gemm_acc(L + (size_t)(k0 + kb) * ld + k0, ld, false, B + (size_t)k0 * ldb, ldb, false,
                  B + (size_t)(k0 + kb) * ldb, ldb, rem, nrhs, kb, -1.0, 1.0, false);
  }
  const int nblk = (n + kCholNb - 1) / kCholNb;
  for (int bk = nblk - 1; bk >= 0; --bk) {
    const int k0 = bk * kCholNb;
    const int kb = min(kCholNb, n - k0);
    const double* L11 = L + (size_t)k0 * ld + k0;
    for (int c = threadIdx.x; c < nrhs; c += blockDim.x)
      for (int j = kb - 1; j >= 0; --j) {
        double v = B[(size_t)(k0 + j) * ldb + c];
        for (int l = j + 1; l < kb; ++l) v -= L11[l * ld + j] * B[(size_t)(k0 + l) * ldb + c];
        B[(size_t)(k0 + j) * ldb + c] = v / L11[j * ld + j];
      }
    wg_sync();
    if (k0 > 0)
      wg_gemm_acc(L + (size_t)k0 * ld, ld, true, B + (size_t)k0 * ldb, ldb, false, B, ldb, k0, nrhs, kb, -1.0, 1.0,
                  false);
  }
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


// ------------------------------------------------------------------ smallest eigenpairs

constexpr int kSubMax = 16;   // largest block of the subspace iteration

// Y (n x nb, ld nb) <- Y - q (q^T Y) for a unit vector q.
__device__ inline void wg_project_out(const double* q, double* Y, int n, int nb) {
  __shared__ double dots[kSubMax];
  for (int c = threadIdx.x; c < nb; c += blockDim.x) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += q[i] * Y[i * nb + c];
    dots[c] = s;
  }
  wg_sync();
  for (int e = threadIdx.x; e < n * nb; e += blockDim.x) Y[e] -= q[e / nb] * dots[e % nb];
  wg_sync();
}

// Orthonormal columns by Cholesky QR: G = Y^T Y = R^T R, Y <- Y R^{-1}.
// Returns false when G is not numerically positive definite.
__device__ inline bool wg_cholqr(double* Y, int n, int nb, double* G, int* flag) {
  wg_gemm(Y, nb, true, Y, nb, false, G, nb, nb, nb, n);
  if (threadIdx.x == 0) *flag = 0;
  wg_sync();
  if (!wg_chol_unblocked(G, nb, nb, flag, 0)) return false;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double* row = Y + i * nb;
    for (int j = 0; j < nb; ++j) {
      double v = row[j];
      for (int l = 0; l < j; ++l) v -= row[l] * G[j * nb + l];
      row[j] = v / G[j * nb + j];
    }
  }
  wg_sync();
  return true;
}

// Smallest eigenpairs, other than the null vector, of a symmetric positive
// semidefinite L (n x n, row-major) whose null space is spanned by the unit
// vector q: block inverse iteration on Lreg = L + rho q q^T (C = its lower
// Cholesky factor) with a Rayleigh-Ritz step every iteration; the nb
// iterated vectors are kept orthogonal to q.  On success X (n x nb, ld nb)
// holds the Ritz vectors and theta[0..nb) the Ritz values, ascending, and
// the first nev pairs satisfy ||L x - theta x||_2 <= tol * rho.  Returns
// false when that is not reached within maxit iterations (or the block
// loses rank).  Scratch: Y, LX (n x nb), G, W (nb x nb); cs, pr, red as for
// wg_jacobi_eig.
__device__ inline bool wg_subspace_eig(const double* L, const double* C, const double* q, int n, int nb, int nev,
                                       double rho, double tol, int maxit, double* X, double* Y, double* LX, double* G,
                                       double* W, double* theta, double* cs, int* pr, double* red, int* flag) {
  __shared__ int ord[kSubMax];
  __shared__ int done;
  // deterministic start: distinct low-discrepancy columns, then orthogonal to q
  for (int e = threadIdx.x; e < n * nb; e += blockDim.x) {
    const int i = e / nb, j = e % nb;
    const double u = (double)((i + 1) * (2 * j + 3) % 97) / 97.0;
    X[e] = u - 0.5 + 0.01 * (double)(j + 1) * (double)((i % (j + 2)) == 0);
  }
  wg_sync();
  wg_project_out(q, X, n, nb);
  if (!wg_cholqr(X, n, nb, G, flag)) return false;
  for (int it = 0; it < maxit; ++it) {
    for (int e = threadIdx.x; e < n * nb; e += blockDim.x) Y[e] = X[e];
    wg_sync();
    wg_chol_solve(C, n, n, Y, nb, nb);
    wg_project_out(q, Y, n, nb);
    if (!wg_cholqr(Y, n, nb, G, flag) || !wg_cholqr(Y, n, nb, G, flag)) return false;
    // Rayleigh-Ritz: G = Y^T L Y, eigenvectors W
    wg_gemm(L, n, false, Y, nb, false, LX, nb, n, nb, n);
    wg_gemm(Y, nb, true, LX, nb, false, G, nb, nb, nb, n);
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
      const int i = e / nb, j = e % nb;
      if (i < j) {
        const double sy = 0.5 * (G[i * nb + j] + G[j * nb + i]);
        G[i * nb + j] = sy;
        G[j * nb + i] = sy;
      }
    }
    wg_sync();
    wg_jacobi_eig(G, nb, W, nb, nb, cs, pr, red);
    if (threadIdx.x == 0) {
      for (int i = 0; i < nb; ++i) ord[i] = i;
      for (int i = 1; i < nb; ++i) {
        const int oi = ord[i];
        int j = i - 1;
        while (j >= 0 && G[ord[j] * nb + ord[j]] > G[oi * nb + oi]) { ord[j + 1] = ord[j]; --j; }
        ord[j + 1] = oi;
      }
      for (int i = 0; i < nb; ++i) theta[i] = G[ord[i] * nb + ord[i]];
    }
    wg_sync();
    // X = Y W, LX = (L Y) W with the columns of W in ascending order
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) G[e] = W[(e / nb) * nb + ord[e % nb]];
    wg_sync();
    wg_gemm(Y, nb, false, G, nb, false, X, nb, n, nb, nb);
    wg_gemm(LX, nb, false, G, nb, false, Y, nb, n, nb, nb);   // Y <- L X
    if (threadIdx.x == 0) done = 1;
    wg_sync();
    for (int c = threadIdx.x; c < nev; c += blockDim.x) {
      double r2 = 0.0;
      for (int i = 0; i < n; ++i) {
        const double d = Y[i * nb + c] - theta[c] * X[i * nb + c];
        r2 += d * d;
      }
      if (!(sqrt(r2) <= tol * rho)) done = 0;
    }
    wg_sync();
    if (done) return true;
  }
  return false;
}

}  // namespace spfas
