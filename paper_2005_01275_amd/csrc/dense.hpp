// Workgroup-level dense linear algebra for the batched local problems of
// the hierarchy setup (one workgroup per aggregate or coarse interface).
// Matrices are row-major with a leading dimension; all threads of the block
// call each routine; results are complete after the call returns.
#pragma once

#include <hip/hip_runtime.h>

#include "kern.hpp"

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
// (A is m x k or k x m, B is k x n or n x k).  64 x 64 output tiles; depth-16
// slices of A and B staged in LDS; each of the 4 waves computes one 32 x 32
// quadrant as 2 x 2 FP64 matrix-core products (v_mfma_f64_16x16x4f64, four
// per slice and sub-tile).  Operand layout of that instruction: A[i][k] in
// lane i + 16k, B[k][j] in lane j + 16k, D[i][j] in lane j + 16 (i mod 4),
// accumulator register i / 4.  lower_only skips the tiles strictly above the
// diagonal (updates whose upper part is never read).  C is not read when
// beta == 0: it may hold any bit pattern.
typedef double dbl4 __attribute__((ext_vector_type(4)));

__device__ inline void wg_gemm_acc(const double* A, int lda, bool ta, const double* B, int ldb, bool tb, double* C,
                                   int ldc, int m, int n, int k, double alpha, double beta, bool lower_only) {
  __shared__ double As[kGemmKc][kGemmTile + 1];
  __shared__ double Bs[kGemmKc][kGemmTile + 1];
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int wr = wv >> 1, wc = wv & 1;          // quadrant of this wave
  const int li = lane & 15, lk = lane >> 4;     // row/column and depth index of the operands
  for (int i0 = 0; i0 < m; i0 += kGemmTile)
    for (int j0 = 0; j0 < n; j0 += kGemmTile) {
      if (lower_only && j0 > i0) continue;
      dbl4 acc[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = dbl4{0.0, 0.0, 0.0, 0.0};
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
#pragma unroll
        for (int ks = 0; ks < kGemmKc; ks += 4) {
          double af[2], bf[2];
#pragma unroll
          for (int a = 0; a < 2; ++a) af[a] = As[ks + lk][32 * wr + 16 * a + li];
#pragma unroll
          for (int b = 0; b < 2; ++b) bf[b] = Bs[ks + lk][32 * wc + 16 * b + li];
#pragma unroll
          for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
        __syncthreads();
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int gi = i0 + 32 * wr + 16 * a + 4 * r + lk, gj = j0 + 32 * wc + 16 * b + li;
            if (gi < m && gj < n) {
              double* cp = C + (size_t)gi * ldc + gj;
              *cp = (beta == 0.0) ? alpha * acc[a][b][r] : beta * *cp + alpha * acc[a][b][r];
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
// block updates on the tiled product.  Diagonal blocks: with few right-hand
// sides (nrhs <= kFewRhs) 32-lane groups solve one column each (8 at a time
// per block of 256 threads: lane r holds row r, each solved entry is
// broadcast by a shuffle, no barrier inside the block); with more, a thread
// per column substitutes sequentially.
constexpr int kFewRhs = 32;

__device__ inline void wg_chol_solve(const double* L, int n, int ld, double* B, int nrhs, int ldb) {
  const int r = threadIdx.x & 31, grp = threadIdx.x >> 5, ngrp = blockDim.x >> 5;
  const bool few = nrhs <= kFewRhs;
  for (int k0 = 0; k0 < n; k0 += kCholNb) {
    const int kb = min(kCholNb, n - k0);
    const double* L11 = L + (size_t)k0 * ld + k0;
    if (!few)
      for (int c = threadIdx.x; c < nrhs; c += blockDim.x)
        for (int j = 0; j < kb; ++j) {
          double v = B[(size_t)(k0 + j) * ldb + c];
          for (int l = 0; l < j; ++l) v -= L11[j * ld + l] * B[(size_t)(k0 + l) * ldb + c];
          B[(size_t)(k0 + j) * ldb + c] = v / L11[j * ld + j];
        }
    for (int c = grp; few && c < nrhs; c += ngrp) {
      double b = r < kb ? B[(size_t)(k0 + r) * ldb + c] : 0.0;
      for (int j = 0; j < kb; ++j) {
        const double xj = __shfl(b, j, 32) / L11[j * ld + j];
        if (r == j) b = xj;
        else if (r > j && r < kb) b -= L11[r * ld + j] * xj;
      }
      if (r < kb) B[(size_t)(k0 + r) * ldb + c] = b;
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
    if (!few)
      for (int c = threadIdx.x; c < nrhs; c += blockDim.x)
        for (int j = kb - 1; j >= 0; --j) {
          double v = B[(size_t)(k0 + j) * ldb + c];
          for (int l = j + 1; l < kb; ++l) v -= L11[l * ld + j] * B[(size_t)(k0 + l) * ldb + c];
          B[(size_t)(k0 + j) * ldb + c] = v / L11[j * ld + j];
        }
    for (int c = grp; few && c < nrhs; c += ngrp) {
      double b = r < kb ? B[(size_t)(k0 + r) * ldb + c] : 0.0;
      for (int j = kb - 1; j >= 0; --j) {
        const double xj = __shfl(b, j, 32) / L11[j * ld + j];
        if (r == j) b = xj;
        else if (r < j) b -= L11[j * ld + r] * xj;
      }
      if (r < kb) B[(size_t)(k0 + r) * ldb + c] = b;
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

constexpr int kSubMax = 16;   // most eigenvectors per aggregate taken by the tridiagonal route

}  // namespace spfas

// ------------------------------------------------------------------ tridiagonal route

namespace spfas {

// Householder reduction of the symmetric A (n x n, row-major, full storage,
// overwritten) to the tridiagonal T = Q^T A Q with Q = H_0 H_1 ... H_{n-3},
// H_k = I - tau_k v_k v_k^T acting on entries k+1 .. n-1, v_k[k+1] = 1 and
// v_k[i] = A[i][k] for i > k+1 on return.  d[0..n) and e[0..n-1) receive
// T's diagonal and subdiagonal, tau[0..n-2) the reflector scales.  vb, pb:
// n doubles of scratch each; red: blockDim doubles of shared memory.
__device__ inline void wg_tridiag(double* A, int n, double* d, double* e, double* tau, double* vb, double* pb,
                                  double* red) {
  __shared__ double sc[3];
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;                  // trailing block rows/cols k+1 .. n-1
    double* a22 = A + (size_t)(k + 1) * n + (k + 1);
    double s = 0.0;
    for (int i = 1 + threadIdx.x; i < m; i += blockDim.x) {
      const double x = A[(size_t)(k + 1 + i) * n + k];
      s += x * x;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
      const double x0 = A[(size_t)(k + 1) * n + k];
      double beta = x0, t = 0.0, scale = 0.0;
      if (s > 0.0) {
        beta = -copysign(sqrt(x0 * x0 + s), x0);
        t = (beta - x0) / beta;
        scale = 1.0 / (x0 - beta);
      }
      e[k] = beta;
      tau[k] = t;
      sc[0] = t;
      sc[1] = scale;
    }
    wg_sync();
    const double t = sc[0], scale = sc[1];
    if (t == 0.0) continue;                    // already reduced in this column (uniform branch)
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
      double v = 1.0;
      if (i > 0) {
        v = A[(size_t)(k + 1 + i) * n + k] * scale;
        A[(size_t)(k + 1 + i) * n + k] = v;
      }
      vb[i] = v;
    }
    wg_sync();
    // p = tau A22 v, K = tau/2 v^T p
    double kv = 0.0;
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
      const double* row = a22 + (size_t)i * n;
      double acc = 0.0;
      for (int j = 0; j < m; ++j) acc = fma(row[j], vb[j], acc);
      acc *= t;
      pb[i] = acc;
      kv = fma(vb[i], acc, kv);
    }
    kv = block_sum(kv, red);
    if (threadIdx.x == 0) sc[2] = 0.5 * t * kv;
    wg_sync();
    const double K = sc[2];
    // A22 -= v w^T + w v^T with w = p - K v
    for (int q = threadIdx.x; q < m * m; q += blockDim.x) {
      const int i = q / m, j = q % m;
      const double wi = pb[i] - K * vb[i], wj = pb[j] - K * vb[j];
      a22[(size_t)i * n + j] -= vb[i] * wj + wi * vb[j];
    }
    wg_sync();
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) d[i] = A[(size_t)i * n + i];
  if (threadIdx.x == 0 && n >= 2) e[n - 2] = A[(size_t)(n - 1) * n + (n - 2)];
  wg_sync();
}

// Number of eigenvalues of the tridiagonal (d, e) below x (Sturm sequence of
// the LDL^T pivots; a zero pivot is replaced by -tiny).
__device__ inline int tri_count(const double* d, const double* e, int n, double x, double tiny) {
  int c = 0;
  double q = d[0] - x;
  for (int i = 0;; ++i) {
    if (q == 0.0) q = -tiny;
    if (q < 0.0) ++c;
    if (i + 1 == n) break;
    q = d[i + 1] - x - e[i] * e[i] / q;
  }
  return c;
}

// The j-th smallest eigenvalue (0-based) of the tridiagonal (d, e) by
// bisection on [lo, hi] (Gershgorin bounds) to the rounding level.
__device__ inline double tri_bisect(const double* d, const double* e, int n, int j, double lo, double hi,
                                    double tiny) {
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (hi - lo <= 4.4e-16 * fmax(fabs(lo), fabs(hi)) + tiny) break;
    if (tri_count(d, e, n, mid, tiny) > j) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

// Eigenvector of the tridiagonal (d, e) for the eigenvalue lam by inverse
// iteration (three solves of (T - lam I) y = y with Gaussian elimination
// and partial pivoting; zero pivots replaced by tiny), unit 2-norm.
// w: 5n doubles of scratch (u0, u1, u2, l, pivot flags).
__device__ inline void tri_invit(const double* d, const double* e, int n, double lam, double tiny, double* y,
                                 double* w) {
  double *u0 = w, *u1 = w + n, *u2 = w + 2 * n, *l = w + 3 * n, *pv = w + 4 * n;
  for (int i = 0; i < n; ++i) {
    u0[i] = d[i] - lam;
    u1[i] = i + 1 < n ? e[i] : 0.0;
    u2[i] = 0.0;
  }
  for (int i = 0; i + 1 < n; ++i) {
    const double s = e[i], a0 = u0[i], a1 = u1[i], b0 = u0[i + 1], b1 = u1[i + 1];
    if (fabs(a0) >= fabs(s)) {
      const double li = a0 != 0.0 ? s / a0 : 0.0;
      l[i] = li;
      pv[i] = 0.0;
      u0[i + 1] = b0 - li * a1;
    } else {
      const double li = a0 / s;
      l[i] = li;
      pv[i] = 1.0;
      u0[i] = s;
      u1[i] = b0;
      u2[i] = b1;
      u0[i + 1] = a1 - li * b0;
      u1[i + 1] = -li * b1;
    }
    if (u0[i] == 0.0) u0[i] = tiny;
  }
  if (u0[n - 1] == 0.0) u0[n - 1] = tiny;
  for (int i = 0; i < n; ++i) y[i] = 1.0 + 0.01 * (double)(i % 7);
  for (int it = 0; it < 3; ++it) {
    for (int i = 0; i + 1 < n; ++i) {
      if (pv[i] != 0.0) { const double t = y[i]; y[i] = y[i + 1]; y[i + 1] = t; }
      y[i + 1] -= l[i] * y[i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double v = y[i];
      if (i + 1 < n) v -= u1[i] * y[i + 1];
      if (i + 2 < n) v -= u2[i] * y[i + 2];
      y[i] = v / u0[i];
    }
    double mx = 0.0;
    for (int i = 0; i < n; ++i) mx = fmax(mx, fabs(y[i]));
    const double inv = mx > 0.0 ? 1.0 / mx : 1.0;
    for (int i = 0; i < n; ++i) y[i] *= inv;
  }
  double nn = 0.0;
  for (int i = 0; i < n; ++i) nn += y[i] * y[i];
  const double inv = 1.0 / sqrt(nn);
  for (int i = 0; i < n; ++i) y[i] *= inv;
}

// Y (n x nc, ld ldy) <- Q Y with Q = H_0 ... H_{n-3} from wg_tridiag (the
// reflectors applied last to first).  Column dot products are wave
// reductions (fixed order).
__device__ inline void wg_tridiag_backtransform(const double* A, int n, const double* tau, double* Y, int nc,
                                                int ldy) {
  __shared__ double dots[kSubMax];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int k = n - 3; k >= 0; --k) {
    const double t = tau[k];
    if (t == 0.0) continue;
    const int m = n - k - 1;
    for (int c = wv; c < nc; c += nw) {
      double s = 0.0;
      for (int i = lane; i < m; i += 64) {
        const double v = i == 0 ? 1.0 : A[(size_t)(k + 1 + i) * n + k];
        s = fma(v, Y[(size_t)(k + 1 + i) * ldy + c], s);
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
      if (lane == 0) dots[c] = t * s;
    }
    wg_sync();
    for (int q = threadIdx.x; q < m * nc; q += blockDim.x) {
      const int i = q / nc, c = q % nc;
      const double v = i == 0 ? 1.0 : A[(size_t)(k + 1 + i) * n + k];
      Y[(size_t)(k + 1 + i) * ldy + c] -= dots[c] * v;
    }
    wg_sync();
  }
}

}  // namespace spfas
