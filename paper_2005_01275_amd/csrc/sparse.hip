// Sparse linear solvers: SpMV, classical and aggregation AMG, dense
// coarsest level, PCG and BiCGStab with device-resident scalars (see
// sparse.hpp).
#include "sparse.hpp"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <numeric>

#include "amg_host.hpp"
#include "kern.hpp"
#include "prof.hpp"
#include "sell_layout.hpp"

namespace spfas {

// ------------------------------------------------------------------ kernels

template <class F>
static void timed(KernelProf* prof, int id, double bytes, hipStream_t s, F&& fn) {
  if (prof && id >= 0) prof->run(id, bytes, s, fn);
  else fn();
}

__global__ void __launch_bounds__(kBlock) k_spmv(CsrView A, const double* __restrict__ x, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  double acc = A.diag[i] * x[i];
  for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) acc += A.val[k] * x[A.col[k]];
  y[i] = acc;
}

void launch_spmv(const CsrView& A, const double* x, double* y, hipStream_t s) {
  if (!A.n) return;
  hipLaunchKernelGGL(k_spmv, dim3(grid_for(A.n, kBlock)), dim3(kBlock), 0, s, A, x, y);
  LAUNCHCHECK();
}

// Row products of the two matrix layouts the Krylov solvers read.
// Products are summed in FP64 whatever the storage of values and vectors.
template <class T>
__device__ inline double row_dot(const CsrView& A, int i, const T* __restrict__ x) {
  double a = A.diag[i] * (double)x[i];
  for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) a += A.val[k] * (double)x[A.col[k]];
  return a;
}

template <class Mat, class T>
__device__ inline double row_dot_sell(const Mat& A, int i, const T* __restrict__ x) {
  const int sl = i >> 6;
  const int a0 = A.sptr[sl];
  const int width = (A.sptr[sl + 1] - a0) >> 6;
  int e = a0 + (i & 63);
  double a = 0.0;
#pragma unroll 4
  for (int k = 0; k < width; ++k, e += 64) a += (double)ld_stream(A.val + e) * (double)x[ld_stream(A.col + e)];
  return a;
}

template <class T>
__device__ inline double row_dot(const Sell64View& A, int i, const T* __restrict__ x) { return row_dot_sell(A, i, x); }
// Row-sum form (entry 0 is the row sum, see Sell32View)
template <class T>
__device__ inline double row_dot(const Sell32View& A, int i, const T* __restrict__ x) {
  const int sl = i >> 6;
  const int a0 = A.sptr[sl];
  const int width = (A.sptr[sl + 1] - a0) >> 6;
  int e = a0 + (i & 63);
  const double xi = (double)x[i];
  double a = (double)ld_stream(A.val + e) * xi;
  e += 64;
#pragma unroll 4
  for (int k = 1; k < width; ++k, e += 64) a += (double)ld_stream(A.val + e) * ((double)x[ld_stream(A.col + e)] - xi);
  return a;
}

// Rows [lo, hi) of the logical block: contiguous chunks (multiples of
// `align` rows) in XCD-aware order.
__device__ inline void block_rows(int n, int& lb, int& lo, int& hi, int align = kBlock) {
  const int G = (int)gridDim.x;
  lb = xcd_block();
  const int chunk = ((n + G - 1) / G + align - 1) / align * align;
  lo = lb * chunk;
  hi = min(n, lo + chunk);
}

// Threads per block of the Krylov products: 512 on the level-0 SELL-64
// matrix (about 6 % faster there than 256 or 1024), kBlock elsewhere.
template <class Mat> struct SpmvBlock { static constexpr int v = kBlock; };
template <> struct SpmvBlock<Sell64View> { static constexpr int v = 512; };
template <> struct SpmvBlock<Sell32View> { static constexpr int v = 512; };

// y = A x; parts = sum_i w_i y_i (w may be x itself or another vector).
// The template flag only separates the finest-level launches by name.
template <class Mat, bool Finest, class T>
__global__ void __launch_bounds__(SpmvBlock<Mat>::v) k_spmv_dot(Mat A, const T* __restrict__ x,
                                                                T* __restrict__ y, const T* __restrict__ w,
                                                                double* __restrict__ parts) {
  __shared__ double sh[SpmvBlock<Mat>::v / 64];
  int lb, lo, hi;
  block_rows(A.n, lb, lo, hi, 64);
  double acc = 0.0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += blockDim.x) {
    const T a = (T)row_dot(A, i, x);
    y[i] = a;
    acc += (double)w[i] * (double)a;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) parts[lb] = acc;
}

// y = A x; parts0 = sum w0*y, parts1 = sum y*y
template <class Mat, bool Finest, class T>
__global__ void __launch_bounds__(SpmvBlock<Mat>::v) k_spmv_dot2(Mat A, const T* __restrict__ x,
                                                                 T* __restrict__ y,
                                                                 const T* __restrict__ w0,
                                                                 double* __restrict__ parts0,
                                                                 double* __restrict__ parts1) {
  __shared__ double sh[SpmvBlock<Mat>::v / 64];
  int lb, lo, hi;
  block_rows(A.n, lb, lo, hi, 64);
  double a0 = 0.0, a1 = 0.0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += blockDim.x) {
    const T a = (T)row_dot(A, i, x);
    y[i] = a;
    a0 += (double)w0[i] * (double)a;
    a1 += (double)a * (double)a;
  }
  a0 = block_sum(a0, sh);
  a1 = block_sum(a1, sh);
  if (threadIdx.x == 0) { parts0[lb] = a0; parts1[lb] = a1; }
}

// r = b - A x in FP64 with r stored in FP32 (the right-hand side of a
// refinement step of mixed precision); parts[lb] = r.r, parts[G + lb] = b.b
template <class Mat>
__global__ void __launch_bounds__(SpmvBlock<Mat>::v) k_resid64(Mat A, const double* __restrict__ x,
                                                               const double* __restrict__ b, float* __restrict__ r,
                                                               double* __restrict__ parts) {
  __shared__ double sh[SpmvBlock<Mat>::v / 64];
  int lb, lo, hi;
  block_rows(A.n, lb, lo, hi, 64);
  double rr = 0.0, bb = 0.0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += blockDim.x) {
    const double bi = b[i];
    const double ri = bi - row_dot(A, i, x);
    r[i] = (float)ri;
    rr += ri * ri;
    bb += bi * bi;
  }
  rr = block_sum(rr, sh);
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    parts[lb] = rr;
    parts[gridDim.x + lb] = bb;
  }
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_dot(int n, const T* __restrict__ a, const T* __restrict__ b,
                                                double* __restrict__ parts) {
  __shared__ double sh[kBlock / 64];
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    acc += (double)a[i] * (double)b[i];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) parts[blockIdx.x] = acc;
}

// scal[slot] = sum of parts (fixed order)
__global__ void __launch_bounds__(kBlock) k_finalize(const double* __restrict__ parts, int G, double* scal, int slot) {
  __shared__ double sh[kBlock / 64];
  double v = reduce_parts(parts, G, sh);
  if (threadIdx.x == 0) scal[slot] = v;
}

// Krylov scalar slots
enum { S_RZ0 = 0, S_RZ1, S_PQ, S_RR, S_BB, S_RHO0, S_RHO1, S_RV, S_TS, S_TT, S_ALPHA, S_OMEGA, S_NSLOT };

// Sum of parts[0..G) computed by every block in the same fixed order (so all
// blocks, and k_finalize, obtain the same value); valid in every thread.
__device__ inline double all_parts(const double* __restrict__ parts, int G, double* sh, double* bc) {
  const double v = reduce_parts(parts, G, sh);
  if (threadIdx.x == 0) *bc = v;
  __syncthreads();
  return *bc;
}

// PCG with the reductions folded in: rz = sum of the r.z partials (block 0
// stores it in slot `cur`), beta = rz / scal[old] (0 on the first
// iteration), p = z + beta p (p = z on the first iteration, whatever p
// held before).
template <class T>
__global__ void __launch_bounds__(kBlock) k_pcg_p2(int n, const double* __restrict__ prz, int G, double* scal, int cur,
                                                   int old, int first, const T* __restrict__ z,
                                                   T* __restrict__ p) {
  __shared__ double sh[kBlock / 64];
  __shared__ double bc;
  const double rz = all_parts(prz, G, sh, &bc);
  if (blockIdx.x == 0 && threadIdx.x == 0) scal[cur] = rz;
  const double ro = scal[old];
  const double beta = (first || ro == 0.0) ? 0.0 : rz / ro;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = first ? z[i] : (T)((double)z[i] + beta * (double)p[i]);
}

// Takes back the last PCG update of x: x -= (rz / pq) p with the alpha
// k_pcg_xr2 used (rz in scal[rz_slot], pq its p.q).
template <class T>
__global__ void __launch_bounds__(kBlock) k_pcg_undo(int n, const double* __restrict__ scal, int rz_slot, double pq,
                                                     T* __restrict__ x, const T* __restrict__ p) {
  const double alpha = pq != 0.0 ? scal[rz_slot] / pq : 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    x[i] = (T)((double)x[i] - alpha * (double)p[i]);
}

// pq = sum of the p.q partials (block 0 stores it in S_PQ and in *hpq),
// alpha = rz / pq, x += alpha p, r -= alpha q, r.r partials.
template <class T>
__global__ void __launch_bounds__(kBlock) k_pcg_xr2(int n, const double* __restrict__ ppq, int G, double* scal, int rz,
                                                    T* __restrict__ x, T* __restrict__ r,
                                                    const T* __restrict__ p, const T* __restrict__ q,
                                                    double* __restrict__ parts, double* __restrict__ hpq) {
  __shared__ double sh[kBlock / 64];
  __shared__ double bc;
  const double pq = all_parts(ppq, G, sh, &bc);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[S_PQ] = pq;
    *hpq = pq;
  }
  const double alpha = pq != 0.0 ? scal[rz] / pq : 0.0;
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    x[i] = (T)((double)x[i] + alpha * (double)p[i]);
    const T ri = (T)((double)r[i] - alpha * (double)q[i]);
    r[i] = ri;
    acc += (double)ri * (double)ri;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) parts[blockIdx.x] = acc;
}

// BiCGStab: p = r + beta (p - omega v), beta = (rho/rho_old)(alpha/omega)
template <class T>
__global__ void __launch_bounds__(kBlock) k_bicg_p(int n, const double* __restrict__ scal, int rho, int rho_old,
                                                   int first, const T* __restrict__ r, T* __restrict__ p,
                                                   const T* __restrict__ v) {
  double beta = 0.0, omega = 0.0;
  if (!first) {
    beta = (scal[rho] / scal[rho_old]) * (scal[S_ALPHA] / scal[S_OMEGA]);
    omega = scal[S_OMEGA];
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = first ? r[i] : (T)((double)r[i] + beta * ((double)p[i] - omega * (double)v[i]));
}

// alpha = rho / (rh.v); s = r - alpha v (into s); writes alpha to scal
template <class T>
__global__ void __launch_bounds__(kBlock) k_bicg_s(int n, double* __restrict__ scal, int rho, const T* __restrict__ r,
                                                   const T* __restrict__ v, T* __restrict__ s) {
  const double alpha = scal[rho] / scal[S_RV];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    s[i] = (T)((double)r[i] - alpha * (double)v[i]);
  if (blockIdx.x == 0 && threadIdx.x == 0) scal[S_ALPHA] = alpha;
}

// scal[slot0] = sum parts0, scal[slot1] = sum parts1 (fixed order); with
// omega != 0 also scal[S_OMEGA] = TS / TT from the two new values; the first
// value also to *hout (host-mapped) if hout is non-null.
__global__ void __launch_bounds__(kBlock) k_finalize2(const double* __restrict__ parts0,
                                                      const double* __restrict__ parts1, int G, double* scal,
                                                      int slot0, int slot1, int omega, double* hout) {
  __shared__ double sh[kBlock / 64];
  const double v0 = reduce_parts(parts0, G, sh);
  const double v1 = reduce_parts(parts1, G, sh);
  if (threadIdx.x == 0) {
    scal[slot0] = v0;
    scal[slot1] = v1;
    if (hout) *hout = v0;
    if (omega) scal[S_OMEGA] = v1 > 0.0 ? v0 / v1 : 0.0;
  }
}

// BiCGStab start: x = 0, r = rh = b, parts = b.b
template <class T>
__global__ void __launch_bounds__(kBlock) k_bicg_init(int n, const T* __restrict__ b, T* __restrict__ x,
                                                      T* __restrict__ r, T* __restrict__ rh,
                                                      double* __restrict__ parts) {
  __shared__ double sh[kBlock / 64];
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const T bi = b[i];
    x[i] = (T)0;
    r[i] = bi;
    rh[i] = bi;
    acc += (double)bi * (double)bi;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) parts[blockIdx.x] = acc;
}

// x += alpha y + omega z; r = s - omega t; parts0 = r.r, parts1 = rh.r
template <class T>
__global__ void __launch_bounds__(kBlock) k_bicg_xr(int n, const double* __restrict__ scal, T* __restrict__ x,
                                                    const T* __restrict__ y, const T* __restrict__ z,
                                                    T* __restrict__ r, const T* __restrict__ s,
                                                    const T* __restrict__ t, const T* __restrict__ rh,
                                                    double* __restrict__ parts0, double* __restrict__ parts1) {
  __shared__ double sh[kBlock / 64];
  const double alpha = scal[S_ALPHA];
  const double omega = scal[S_OMEGA];
  double a0 = 0.0, a1 = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    x[i] = (T)((double)x[i] + (alpha * (double)y[i] + omega * (double)z[i]));
    const T ri = (T)((double)s[i] - omega * (double)t[i]);
    r[i] = ri;
    a0 += (double)ri * (double)ri;
    a1 += (double)rh[i] * (double)ri;
  }
  a0 = block_sum(a0, sh);
  a1 = block_sum(a1, sh);
  if (threadIdx.x == 0) { parts0[blockIdx.x] = a0; parts1[blockIdx.x] = a1; }
}


template <class T>
__global__ void __launch_bounds__(kBlock) k_copy(int n, const T* __restrict__ a, T* __restrict__ b) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) b[i] = a[i];
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_zero(int n, T* __restrict__ b) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) b[i] = 0.0;
}

// ------------------------------------------------------------------ AMG kernels



// ------------------------------------------------------------------ SELL-64 cycle kernels

// First stored entry and width of row i of a SELL-64 matrix.
__device__ inline void sell_row(const SellView& A, int i, int& e, int& width) {
  const int sl = i >> 6;
  const int a = A.sptr[sl];
  e = a + (i & 63);
  width = (A.sptr[sl + 1] - a) >> 6;
}

// Two Jacobi sweeps from x = 0 in one pass: x1 = w b, x2 = x1 + w (b - A x1).
// The template flag only separates the finest-level launches by name.
template <bool Finest>
__global__ void __launch_bounds__(kBlock) k_amg_pre(SellView A, const double* __restrict__ w,
                                                    const double* __restrict__ b, double* __restrict__ x2) {
  const int i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  int e, width;
  sell_row(A, i, e, width);
  double acc = 0.0;
#pragma unroll 4
  for (int k = 0; k < width; ++k, e += 64) {
    const int j = A.col[e];
    acc += (double)A.val[e] * (w[j] * b[j]);
  }
  const double wi = w[i], bi = b[i];
  x2[i] = wi * bi + wi * (bi - acc);
}

// r = b - A x
template <bool Finest>
__global__ void __launch_bounds__(kBlock) k_amg_resid(SellView A, const double* __restrict__ b,
                                                      const double* __restrict__ x, double* __restrict__ r) {
  const int i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  int e, width;
  sell_row(A, i, e, width);
  double acc = 0.0;
#pragma unroll 4
  for (int k = 0; k < width; ++k, e += 64) acc += (double)A.val[e] * x[A.col[e]];
  r[i] = b[i] - acc;
}

// Prolongation of the coarse correction and one sweep in one pass:
// y = x + ec[agg], out = y + w (b - A y).
template <bool Finest>
__global__ void __launch_bounds__(kBlock) k_amg_post1(SellView A, const double* __restrict__ w,
                                                      const double* __restrict__ b, const double* __restrict__ x,
                                                      const int* __restrict__ agg, const double* __restrict__ ec,
                                                      double* __restrict__ out) {
  const int i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  int e, width;
  sell_row(A, i, e, width);
  double acc = 0.0;
#pragma unroll 4
  for (int k = 0; k < width; ++k, e += 64) {
    const int j = A.col[e];
    acc += (double)A.val[e] * (x[j] + ec[agg[j]]);
  }
  out[i] = (x[i] + ec[agg[i]]) + w[i] * (b[i] - acc);
}

// out = x + w (b - A x)
template <bool Finest>
__global__ void __launch_bounds__(kBlock) k_amg_post2(SellView A, const double* __restrict__ w,
                                                      const double* __restrict__ b, const double* __restrict__ x,
                                                      double* __restrict__ out) {
  const int i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  int e, width;
  sell_row(A, i, e, width);
  double acc = 0.0;
#pragma unroll 4
  for (int k = 0; k < width; ++k, e += 64) acc += (double)A.val[e] * x[A.col[e]];
  out[i] = x[i] + w[i] * (b[i] - acc);
}

// Group-per-row variants for the small coarse levels, whose rows are wide
// and few: kVecG lanes share a row of the FP64 DIA+CSR matrix, so the
// dependent column-then-value loads of a long row run in parallel instead of
// as one serial chain per thread.  Lane 0 of each group writes the row.
constexpr int kVecG = 8;

__device__ inline double group_sum(double v) {
#pragma unroll
  for (int o = kVecG / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kVecG);
  return v;
}

__global__ void __launch_bounds__(kBlock) k_amgv_pre(CsrView A, const double* __restrict__ w,
                                                     const double* __restrict__ b, double* __restrict__ x2) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = t / kVecG, g = t % kVecG;
  if (i >= A.n) return;   // the whole group leaves together
  double acc = 0.0;
  for (int k = A.ptr[i] + g; k < A.ptr[i + 1]; k += kVecG) {
    const int j = A.col[k];
    acc += A.val[k] * (w[j] * b[j]);
  }
  acc = group_sum(acc);
  if (g == 0) {
    const double wi = w[i], bi = b[i], x1 = wi * bi;
    x2[i] = x1 + wi * (bi - (A.diag[i] * x1 + acc));
  }
}

__global__ void __launch_bounds__(kBlock) k_amgv_resid(CsrView A, const double* __restrict__ b,
                                                       const double* __restrict__ x, double* __restrict__ r) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = t / kVecG, g = t % kVecG;
  if (i >= A.n) return;
  double acc = 0.0;
  for (int k = A.ptr[i] + g; k < A.ptr[i + 1]; k += kVecG) acc += A.val[k] * x[A.col[k]];
  acc = group_sum(acc);
  if (g == 0) r[i] = b[i] - (A.diag[i] * x[i] + acc);
}

__global__ void __launch_bounds__(kBlock) k_amgv_post1(CsrView A, const double* __restrict__ w,
                                                       const double* __restrict__ b, const double* __restrict__ x,
                                                       const int* __restrict__ agg, const double* __restrict__ ec,
                                                       double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = t / kVecG, g = t % kVecG;
  if (i >= A.n) return;
  double acc = 0.0;
  for (int k = A.ptr[i] + g; k < A.ptr[i + 1]; k += kVecG) {
    const int j = A.col[k];
    acc += A.val[k] * (x[j] + ec[agg[j]]);
  }
  acc = group_sum(acc);
  if (g == 0) {
    const double yi = x[i] + ec[agg[i]];
    out[i] = yi + w[i] * (b[i] - (A.diag[i] * yi + acc));
  }
}

__global__ void __launch_bounds__(kBlock) k_amgv_post2(CsrView A, const double* __restrict__ w,
                                                       const double* __restrict__ b, const double* __restrict__ x,
                                                       double* __restrict__ out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = t / kVecG, g = t % kVecG;
  if (i >= A.n) return;
  double acc = 0.0;
  for (int k = A.ptr[i] + g; k < A.ptr[i + 1]; k += kVecG) acc += A.val[k] * x[A.col[k]];
  acc = group_sum(acc);
  if (g == 0) out[i] = x[i] + w[i] * (b[i] - (A.diag[i] * x[i] + acc));
}

// smoother weights 1 / (|a_ii| + 0.5 sum_j |a_ij|), a lane group per row
__global__ void __launch_bounds__(kBlock) k_invd(CsrView A, double* __restrict__ invd) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = t / kVecG, g = t % kVecG;
  if (i >= A.n) return;
  double s = 0.0;
  for (int k = A.ptr[i] + g; k < A.ptr[i + 1]; k += kVecG) s += fabs(A.val[k]);
  s = group_sum(s);
  if (g == 0) {
    const double d = fabs(A.diag[i]) + 0.5 * s;
    invd[i] = d > 0.0 ? 1.0 / d : 0.0;
  }
}

// bc[I] = sum of r over the members of coarse node I, a lane group per node
__global__ void __launch_bounds__(kBlock) k_restrict_vec(int nc, const int* __restrict__ mptr,
                                                         const int* __restrict__ mem, const double* __restrict__ r,
                                                         double* __restrict__ bc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int I = t / kVecG, g = t % kVecG;
  if (I >= nc) return;
  double s = 0.0;
  for (int k = mptr[I] + g; k < mptr[I + 1]; k += kVecG) s += r[mem[k]];
  s = group_sum(s);
  if (g == 0) bc[I] = s;
}

// DIA+CSR values of a level from its FP64 SELL copy (the inverse of
// k_sell_fill; padding slots are skipped).
template <class V>
__global__ void __launch_bounds__(kBlock) k_sell_to_csr(int ne, const int* __restrict__ smap,
                                                        const V* __restrict__ val, double* __restrict__ diag,
                                                        double* __restrict__ off);

// FP32 SELL values from the FP64 DIA+CSR values of the level.
constexpr int kSellPad = INT_MIN;
__global__ void __launch_bounds__(kBlock) k_sell_fill(int ne, const int* __restrict__ smap,
                                                      const double* __restrict__ diag, const double* __restrict__ off,
                                                      float* __restrict__ val, double* __restrict__ val64) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int m = smap[e];
  double v = 0.0;
  if (m >= 0) v = off[m];
  else if (m != kSellPad) v = diag[-1 - m];
  if (val) val[e] = (float)v;
  if (val64) val64[e] = v;
}

__global__ void __launch_bounds__(kBlock) k_restrict(int nc, const int* __restrict__ mptr, const int* __restrict__ mem,
                                                     const double* __restrict__ r, double* __restrict__ bc) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  double s = 0.0;
  for (int k = mptr[I]; k < mptr[I + 1]; ++k) s += r[mem[k]];
  bc[I] = s;
}

__global__ void __launch_bounds__(kBlock) k_galerkin_off(int nnz, const int* __restrict__ gp, const int* __restrict__ gi,
                                                         const double* __restrict__ fval, double* __restrict__ cval) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  double s = 0.0;
  for (int k = gp[e]; k < gp[e + 1]; ++k) s += fval[gi[k]];
  cval[e] = s;
}

__global__ void __launch_bounds__(kBlock) k_galerkin_diag(int nc, const int* __restrict__ gp, const int* __restrict__ gi,
                                                          const double* __restrict__ fdiag,
                                                          const double* __restrict__ fval, double* __restrict__ cdiag) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  double s = 0.0;
  for (int k = gp[I]; k < gp[I + 1]; ++k) {
    const int c = gi[k];
    s += (c & 1) ? fval[c >> 1] : fdiag[c >> 1];
  }
  cdiag[I] = s;
}

// ------------------------------------------------------------------ classical AMG kernels

// A P values: the products of each entry, summed in a fixed order.
// Product codes address the DIA+CSR matrix (dia_code / off_code).
__global__ void __launch_bounds__(kBlock) k_ap_numeric(int ne, const int* __restrict__ lptr,
                                                       const int* __restrict__ la, const int* __restrict__ lp,
                                                       CsrView A, const double* __restrict__ pval,
                                                       double* __restrict__ apv) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double s = 0.0;
  for (int t = lptr[e]; t < lptr[e + 1]; ++t) {
    const int c = la[t];
    const double a = (c & 1) ? A.val[c >> 1] : A.diag[c >> 1];
    s += a * pval[lp[t]];
  }
  apv[e] = s;
}

// P^T (A P): entries [0, noff) are the next level's off-diagonal values,
// [noff, noff + nc) its diagonal.
__global__ void __launch_bounds__(kBlock) k_rap_numeric(int noff, int nc, const int* __restrict__ lptr,
                                                        const int* __restrict__ lr, const int* __restrict__ lq,
                                                        const double* __restrict__ pval,
                                                        const double* __restrict__ apv, double* __restrict__ cval,
                                                        double* __restrict__ cdiag) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= noff + nc) return;
  double s = 0.0;
  for (int t = lptr[e]; t < lptr[e + 1]; ++t) s += pval[lr[t]] * apv[lq[t]];
  if (e < noff) cval[e] = s;
  else cdiag[e - noff] = s;
}

// Stored slots of row i of a cycle operator: e, e + step, ... < end.
template <bool Sell>
__device__ inline void cyc_row(const CycView& M, int i, int& e, int& end, int& step) {
  if constexpr (Sell) {
    const int sl = i >> 6;
    const int a = M.ptr[sl];
    e = a + (i & 63);
    end = e + (M.ptr[sl + 1] - a);
    step = 64;
  } else {
    e = M.ptr[i];
    end = M.ptr[i + 1];
    step = 1;
  }
}

// FP16 value of an operator entry, saturated to the finite FP16 range
__device__ inline cyc_t to_cyc(double v) { return (cyc_t)fmin(fmax(v, -65504.0), 65504.0); }

// A diag(w) in FP16, one thread per stored slot: a(src) * w[col]
__global__ void __launch_bounds__(kBlock) k_fill_aw(int ne, const int* __restrict__ col, const int* __restrict__ src,
                                                    CsrView A, const double* __restrict__ w, cyc_t* __restrict__ val) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int c = src[e];
  double v = 0.0;
  if (c >= 0) v = ((c & 1) ? A.val[c >> 1] : A.diag[c >> 1]) * w[col[e]];
  val[e] = to_cyc(v);
}

// P - diag(w) A P in FP16 on the pattern of A P (which contains that of P):
// SELL thread per row, CSR lane group per row.
__device__ inline cyc_t cm_value(int q, const int* __restrict__ appidx, const double* __restrict__ pval,
                                 const double* __restrict__ apv, double wi) {
  if (q < 0) return (cyc_t)0.0;
  const int pi = appidx[q];
  return to_cyc((pi >= 0 ? pval[pi] : 0.0) - wi * apv[q]);
}

__global__ void __launch_bounds__(kBlock) k_fill_cm(CycView M, const int* __restrict__ src,
                                                    const int* __restrict__ appidx, const double* __restrict__ pval,
                                                    const double* __restrict__ apv, const double* __restrict__ w,
                                                    cyc_t* __restrict__ val) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M.n) return;
  int e, end, step;
  cyc_row<true>(M, i, e, end, step);
  const double wi = w[i];
  for (; e < end; e += step) val[e] = cm_value(src[e], appidx, pval, apv, wi);
}

__global__ void __launch_bounds__(kBlock) k_fill_cmv(CycView M, const int* __restrict__ src,
                                                     const int* __restrict__ appidx, const double* __restrict__ pval,
                                                     const double* __restrict__ apv, const double* __restrict__ w,
                                                     cyc_t* __restrict__ val) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = t / kVecG, g = t % kVecG;
  if (i >= M.n) return;
  const double wi = w[i];
  for (int e = M.ptr[i] + g; e < M.ptr[i + 1]; e += kVecG) val[e] = cm_value(src[e], appidx, pval, apv, wi);
}

// G = P^T (I - A diag(w)) in FP16, one thread per entry (CSR order):
// G_cj = P_jc - w_j sum_i P_ic a_ij over the entry's product list
__global__ void __launch_bounds__(kBlock) k_fill_g(int ne, const int* __restrict__ col, const int* __restrict__ rt,
                                                   const int* __restrict__ lptr, const int* __restrict__ lp,
                                                   const int* __restrict__ la, CsrView A,
                                                   const double* __restrict__ pval, const double* __restrict__ w,
                                                   cyc_t* __restrict__ val) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  double s = 0.0;
  for (int t = lptr[e]; t < lptr[e + 1]; ++t) {
    const int c = la[t];
    s += pval[lp[t]] * ((c & 1) ? A.val[c >> 1] : A.diag[c >> 1]);
  }
  val[e] = to_cyc((rt[e] >= 0 ? pval[rt[e]] : 0.0) - w[col[e]] * s);
}

// R = P^T in FP16 (filled once at setup), one thread per stored slot
__global__ void __launch_bounds__(kBlock) k_fill_rm(int ne, const int* __restrict__ src,
                                                    const double* __restrict__ pval, cyc_t* __restrict__ val) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  val[e] = src[e] >= 0 ? to_cyc(pval[src[e]]) : (cyc_t)0.0;
}

// The three kernels of a classical V(1,1) level, on SELL-64 (thread per row):
//   Op 0: y = b - M b               pre-sweep from zero + residual, M = A diag(w)
//   Op 1: y = M x                   restriction, M = P^T
//   Op 2: y = w (b + r) + M x       prolongation + post-sweep, M = P - diag(w) A P
// (with x1 = w b and r = b - A x1, the post-sweep of y = x1 + P e is
// y + w (b - A y) = w (b + r) + (P - diag(w) A P) e).  The template flag
// only separates the finest-level launches by name.
// Vectors inside the classical cycle are FP32 (residuals, restricted
// right-hand sides, coarse corrections); the cycle's input b and output on
// level 0 are the Krylov solver's FP64 vectors (TB, TY); products and sums
// are FP64.  Op 0 gathers x = b; Ops 1 and 2 gather FP32 vectors.
template <int Op, class TB>
using CycX = std::conditional_t<Op == 0, TB, float>;

template <int Op, bool Finest, class TB, class TY>
__global__ void __launch_bounds__(kBlock) k_cyc(CycView M, const CycX<Op, TB>* __restrict__ x,
                                                const TB* __restrict__ b, const float* __restrict__ r,
                                                const double* __restrict__ w, TY* __restrict__ y) {
  const int i = xcd_block() * blockDim.x + threadIdx.x;
  if (i >= M.n) return;
  int e, end, step;
  cyc_row<true>(M, i, e, end, step);
  double acc = 0.0;
#pragma unroll 4
  for (; e < end; e += 64) acc += (double)ld_stream(M.val + e) * (double)x[ld_stream(M.col + e)];
  if constexpr (Op == 0) y[i] = (TY)((double)b[i] - acc);
  else if constexpr (Op == 1) y[i] = (TY)acc;
  else y[i] = (TY)(w[i] * ((double)b[i] + (double)r[i]) + acc);
}

// The same on CSR with a group of LG lanes per row (smaller levels).
template <int Op, int LG, class TB, class TY>
__global__ void __launch_bounds__(kBlock) k_cycv(CycView M, const CycX<Op, TB>* __restrict__ x,
                                                 const TB* __restrict__ b, const float* __restrict__ r,
                                                 const double* __restrict__ w, TY* __restrict__ y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = t / LG, g = t % LG;
  if (i >= M.n) return;   // the whole group leaves together
  double acc = 0.0;
  for (int e = M.ptr[i] + g; e < M.ptr[i + 1]; e += LG) acc += (double)M.val[e] * (double)x[M.col[e]];
#pragma unroll
  for (int o = LG / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, LG);
  if (g == 0) {
    if constexpr (Op == 0) y[i] = (TY)((double)b[i] - acc);
    else if constexpr (Op == 1) y[i] = (TY)acc;
    else y[i] = (TY)(w[i] * ((double)b[i] + (double)r[i]) + acc);
  }
}

// The down leg of a small level in one launch: rows [0, n) y = b - M b
// (pre-sweep from zero + residual, M = A diag(w)), rows [n, n + nc)
// yc = G b with G = P^T (I - A diag(w)), the restriction of that residual.
template <int LG>
__global__ void __launch_bounds__(kBlock) k_cycv_down(CycView M, CycView G, const float* __restrict__ b,
                                                      float* __restrict__ y, float* __restrict__ yc) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = t / LG, g = t % LG;
  if (i >= M.n + G.n) return;   // the whole group leaves together
  const bool fine = i < M.n;
  const int row = fine ? i : i - M.n;
  const int* ptr = fine ? M.ptr : G.ptr;
  const int* col = fine ? M.col : G.col;
  const cyc_t* val = fine ? M.val : G.val;
  double acc = 0.0;
  for (int e = ptr[row] + g; e < ptr[row + 1]; e += LG) acc += (double)val[e] * (double)b[col[e]];
#pragma unroll
  for (int o = LG / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, LG);
  if (g == 0) {
    if (fine) y[row] = (float)((double)b[row] - acc);
    else yc[row] = (float)acc;
  }
}

// dense row-major copy of a small DIA+CSR matrix
__global__ void __launch_bounds__(kBlock) k_dense_fill(CsrView A, double* __restrict__ M, int nd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  double* row = M + (size_t)i * nd;
  for (int j = 0; j < nd; ++j) row[j] = 0.0;
  row[i] = A.diag[i];
  for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) row[A.col[k]] += A.val[k];
}

// In-place inverse of a dense nd x nd row-major matrix by LU with partial
// pivoting (one block), then column-by-column substitution into `inv`.
// `M` is overwritten by the LU factors; flag[0] = 1 on a zero pivot.
__global__ void __launch_bounds__(kBlock) k_dense_inverse(double* __restrict__ M, double* __restrict__ inv,
                                                          int* __restrict__ piv, int nd, int* __restrict__ flag) {
  __shared__ double sv[kBlock];
  __shared__ int si[kBlock];
  const int tid = threadIdx.x;
  for (int k = 0; k < nd; ++k) {
    double best = -1.0;
    int bi = k;
    for (int i = k + tid; i < nd; i += blockDim.x) {
      const double a = fabs(M[(size_t)i * nd + k]);
      if (a > best) { best = a; bi = i; }
    }
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
      if (tid < o) {
        if (sv[tid + o] > sv[tid] || (sv[tid + o] == sv[tid] && si[tid + o] < si[tid])) {
          sv[tid] = sv[tid + o];
          si[tid] = si[tid + o];
        }
      }
      __syncthreads();
    }
    const int p = si[0];
    if (tid == 0) {
      piv[k] = p;
      if (!(sv[0] > 0.0)) flag[0] = 1;
    }
    if (p != k)
      for (int j = tid; j < nd; j += blockDim.x) {
        const double a = M[(size_t)k * nd + j];
        M[(size_t)k * nd + j] = M[(size_t)p * nd + j];
        M[(size_t)p * nd + j] = a;
      }
    __syncthreads();
    const double pv = M[(size_t)k * nd + k];
    const double ipv = pv != 0.0 ? 1.0 / pv : 0.0;
    for (int i = k + 1 + tid; i < nd; i += blockDim.x) M[(size_t)i * nd + k] *= ipv;
    __syncthreads();
    const int rem = nd - k - 1;
    for (int e = tid; e < rem * rem; e += blockDim.x) {
      const int i = k + 1 + e / rem, j = k + 1 + e % rem;
      M[(size_t)i * nd + j] -= M[(size_t)i * nd + k] * M[(size_t)k * nd + j];
    }
    __syncthreads();
  }
  // columns of the inverse: solve L U x = P e_c
  for (int c = tid; c < nd; c += blockDim.x) {
    // x = P e_c held in column c of inv (row-major, strided)
    for (int i = 0; i < nd; ++i) inv[(size_t)i * nd + c] = (i == c) ? 1.0 : 0.0;
    for (int k = 0; k < nd; ++k) {
      const int p = piv[k];
      if (p != k) {
        const double a = inv[(size_t)k * nd + c];
        inv[(size_t)k * nd + c] = inv[(size_t)p * nd + c];
        inv[(size_t)p * nd + c] = a;
      }
    }
    for (int i = 0; i < nd; ++i) {
      double s = inv[(size_t)i * nd + c];
      for (int j = 0; j < i; ++j) s -= M[(size_t)i * nd + j] * inv[(size_t)j * nd + c];
      inv[(size_t)i * nd + c] = s;
    }
    for (int i = nd - 1; i >= 0; --i) {
      double s = inv[(size_t)i * nd + c];
      for (int j = i + 1; j < nd; ++j) s -= M[(size_t)i * nd + j] * inv[(size_t)j * nd + c];
      const double d = M[(size_t)i * nd + i];
      inv[(size_t)i * nd + c] = d != 0.0 ? s / d : 0.0;
    }
  }
}

// In-place Gauss-Jordan inverse with partial pivoting of an nd x nd
// row-major matrix held entirely in LDS (nd <= kDenseLds, one block).  Row
// interchanges are undone as column interchanges in reverse order at the end.
__global__ void __launch_bounds__(kBlock) k_dense_inverse_lds(const double* __restrict__ A, double* __restrict__ inv,
                                                              int nd, int* __restrict__ flag) {
  __shared__ double a[kDenseLds * kDenseLds];
  __shared__ double fcol[kDenseLds];
  __shared__ int perm[kDenseLds];
  const int tid = threadIdx.x;
  const int nn = nd * nd;
  for (int e = tid; e < nn; e += blockDim.x) a[e] = A[e];
  __syncthreads();
  for (int k = 0; k < nd; ++k) {
    if (tid < 64) {   // pivot search by wave 0; ties go to the lowest row
      double best = -1.0;
      int bi = k;
      for (int i = k + tid; i < nd; i += 64) {
        const double v = fabs(a[i * nd + k]);
        if (v > best) { best = v; bi = i; }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_down(best, o, 64);
        const int oi = __shfl_down(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) {
        perm[k] = bi;
        if (!(best > 0.0)) flag[0] = 1;
      }
    }
    __syncthreads();
    const int p = perm[k];
    if (p != k)
      for (int j = tid; j < nd; j += blockDim.x) {
        const double t = a[k * nd + j];
        a[k * nd + j] = a[p * nd + j];
        a[p * nd + j] = t;
      }
    __syncthreads();
    const double pv = a[k * nd + k];
    const double ipv = pv != 0.0 ? 1.0 / pv : 0.0;
    __syncthreads();
    for (int j = tid; j < nd; j += blockDim.x) a[k * nd + j] = (j == k) ? ipv : a[k * nd + j] * ipv;
    for (int i = tid; i < nd; i += blockDim.x)
      if (i != k) fcol[i] = a[i * nd + k];
    __syncthreads();
    for (int i = tid >> 5; i < nd; i += kBlock / 32) {   // 8 rows x 32 columns per pass
      if (i == k) continue;
      const double fi = fcol[i];
      for (int j = tid & 31; j < nd; j += 32) {
        const double base = (j == k) ? 0.0 : a[i * nd + j];
        a[i * nd + j] = base - fi * a[k * nd + j];
      }
    }
    __syncthreads();
  }
  for (int k = nd - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k)
      for (int i = tid; i < nd; i += blockDim.x) {
        const double t = a[i * nd + k];
        a[i * nd + k] = a[i * nd + p];
        a[i * nd + p] = t;
      }
    __syncthreads();
  }
  for (int e = tid; e < nn; e += blockDim.x) inv[e] = a[e];
}

// x = inv b, one wave per row (coalesced row reads)
template <class TB, class TY>
__global__ void __launch_bounds__(kBlock) k_dense_gemv(int nd, const double* __restrict__ inv, const TB* __restrict__ b,
                                                       TY* __restrict__ x) {
  const int row = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= nd) return;
  const double* r = inv + (size_t)row * nd;
  double s = 0.0;
  for (int j = lane; j < nd; j += 64) s += r[j] * (double)b[j];
  s = wave_sum(s);
  if (lane == 0) x[row] = (TY)s;
}

// ------------------------------------------------------------------ AMG host

namespace {

// Plain aggregation with row-relative strength |a_ij| >= theta max_k |a_ik|
// (a threshold relative to the diagonal turns the wide stencils of coarse
// Galerkin rows into all-weak rows and stalls the coarsening).
int aggregate(const HostCsr& A, double theta, std::vector<int>& agg) {
  const int n = A.n;
  agg.assign(n, -1);
  std::vector<double> rowmax(n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (A.col[k] != i) rowmax[i] = std::max(rowmax[i], std::fabs(A.val[k]));
  auto strong = [&](int i, int k) {
    const int j = A.col[k];
    if (j == i) return false;
    return rowmax[i] > 0.0 && std::fabs(A.val[k]) >= theta * rowmax[i];
  };
  int nc = 0;
  std::vector<char> phase1(n, 0);
  for (int i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    bool ok = true;
    bool any = false;
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (strong(i, k)) {
        any = true;
        if (agg[A.col[k]] >= 0) { ok = false; break; }
      }
    if (!ok || !any) continue;
    agg[i] = nc;
    phase1[i] = 1;
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (strong(i, k)) { agg[A.col[k]] = nc; phase1[A.col[k]] = 1; }
    ++nc;
  }
  std::vector<int> agg1(agg);
  for (int i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    double best = -1.0;
    int bj = -1;
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const int j = A.col[k];
      if (strong(i, k) && phase1[j] && std::fabs(A.val[k]) > best) { best = std::fabs(A.val[k]); bj = j; }
    }
    if (bj >= 0) agg[i] = agg1[bj];
  }
  for (int i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    agg[i] = nc;
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) {
      const int j = A.col[k];
      if (strong(i, k) && agg[j] < 0) agg[j] = nc;
    }
    ++nc;
  }
  return nc;
}

// SELL-64 pattern of a level (diagonal first in every row) and the map from
// each stored entry to its FP64 source value.
void build_sell(const HostCsr& H, AmgLevel& F, hipStream_t s) {
  const int n = H.n;
  std::vector<int> sptr, col, map;
  sell_matrix_layout(n, H.ptr, H.col, kSellPad, sptr, col, map);
  const int ne = (int)col.size();
  F.sptr.upload(sptr, s);
  F.scol.upload(col, s);
  F.smap.upload(map, s);
  F.sval.alloc(ne);
  F.sell.n = n;
  F.sell.sptr = F.sptr.p;
  F.sell.col = F.scol.p;
  F.sell.val = F.sval.p;
  F.sell_nnz = (long long)n + H.ptr[n];
}

// Lanes per row of the CSR cycle products: 8, 16 above 24 stored entries per
// row on average, 32 above 36 (the long rows of the middle AMG levels; more
// lanes shorten each lane's chain of dependent loads).  Measured on the
// 60x220x85 hierarchy: 7 % less time in these kernels than 8 lanes throughout,
// while 4 lanes for short rows was slower.
static int cyc_lanes(double mean) { return mean > 36.0 ? 32 : mean > 24.0 ? 16 : 8; }

// Cycle operator from CSR rows (col, src per entry): SELL-64 for at least
// kSellRows rows, else CSR.  Padding slots read column `pad_col` of their
// row (its first column, or 0 for an empty row) with value 0.
void build_cyc(int n, const std::vector<int>& ptr, const std::vector<int>& col, const std::vector<int>& src,
               CycMat& M, hipStream_t s) {
  M.n = n;
  M.nnz = ptr[n];
  M.sell = n >= kSellRows;
  M.lanes = cyc_lanes(n ? (double)M.nnz / n : 0.0);
  if (!M.sell) {
    M.ptr.upload(ptr, s);
    M.col.upload(col, s);
    M.src.upload(src, s);
    M.val.alloc(std::max<size_t>(col.size(), 1));
    return;
  }
  std::vector<int> sptr, scol, ssrc;
  sell_cyc_layout(n, ptr, col, src, sptr, scol, ssrc);
  const int ne = (int)scol.size();
  M.ptr.upload(sptr, s);
  M.col.upload(scol, s);
  M.src.upload(ssrc, s);
  M.val.alloc(ne);
}

CycView cyc_view(const CycMat& M) { return CycView{M.n, M.ptr.p, M.col.p, M.val.p}; }

// Pattern and product lists of G = P^T (I - A diag(w)) for the fused down
// leg: row c of G collects, for every fine row i of P^T's row c (P entry
// pe), the P^T term at column i and the products pe x a_ij over row i of A
// (diagonal first, then the off-diagonal entries in CSR order); columns
// ascending, each entry's products in that traversal order.
void build_fused(const HostCsr& A, const ClassicalLevel& CL, AmgLevel& F, hipStream_t s) {
  const int nc = CL.nc;
  // rows of G in 16 ordered chunks on host threads, joined in row order
  constexpr int kChunks = 16;
  struct GChunk {
    std::vector<int> col, rt, nprod, lp, la, rowlen;
  };
  std::vector<GChunk> gch(kChunks);
  const int per = (nc + kChunks - 1) / kChunks;
  parallel_ranges(kChunks, [&](int64_t tlo, int64_t thi) {
    std::vector<int> slot(A.n, -1), cols, rt, cnt, start, order;
    struct Item { int q, pe, code; };
    std::vector<Item> items;
    std::vector<std::pair<int, int>> grouped;
    for (int64_t t = tlo; t < thi; ++t) {
      GChunk& ch = gch[t];
      for (int c = std::min(nc, (int)t * per); c < std::min(nc, (int)(t + 1) * per); ++c) {
        cols.clear();
        rt.clear();
        items.clear();
        auto at = [&](int j) -> int {
          if (slot[j] < 0) {
            slot[j] = (int)cols.size();
            cols.push_back(j);
            rt.push_back(-1);
          }
          return slot[j];
        };
        for (int e = CL.rptr[c]; e < CL.rptr[c + 1]; ++e) {
          const int i = CL.rcol[e], pe = CL.rsrc[e];
          const int qi = at(i);
          rt[qi] = pe;
          items.push_back({qi, pe, dia_code(i)});
          for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k) items.push_back({at(A.col[k]), pe, off_code(k)});
        }
        // products grouped by column, in generation order within a column
        cnt.assign(cols.size() + 1, 0);
        for (const Item& it : items) cnt[it.q + 1]++;
        for (size_t q = 0; q < cols.size(); ++q) cnt[q + 1] += cnt[q];
        start.assign(cnt.begin(), cnt.end() - 1);
        grouped.resize(items.size());
        for (const Item& it : items) grouped[start[it.q]++] = {it.pe, it.code};
        order.resize(cols.size());
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(), [&](int x, int y) { return cols[x] < cols[y]; });
        for (int q : order) {
          ch.col.push_back(cols[q]);
          ch.rt.push_back(rt[q]);
          ch.nprod.push_back(cnt[q + 1] - cnt[q]);
          for (int k = cnt[q]; k < cnt[q + 1]; ++k) {
            ch.lp.push_back(grouped[k].first);
            ch.la.push_back(grouped[k].second);
          }
        }
        for (int j : cols) slot[j] = -1;
        ch.rowlen.push_back((int)cols.size());
      }
    }
  }, (int64_t)A.n + A.ptr[A.n]);
  std::vector<int> gptr(nc + 1, 0), gcol, grt, glptr(1, 0), glp, gla, src;
  {
    int row = 0;
    for (const GChunk& ch : gch) {
      for (int len : ch.rowlen) { gptr[row + 1] = gptr[row] + len; ++row; }
      gcol.insert(gcol.end(), ch.col.begin(), ch.col.end());
      grt.insert(grt.end(), ch.rt.begin(), ch.rt.end());
      glp.insert(glp.end(), ch.lp.begin(), ch.lp.end());
      gla.insert(gla.end(), ch.la.begin(), ch.la.end());
      for (int np : ch.nprod) glptr.push_back(glptr.back() + np);
    }
  }
  src.resize(gcol.size());
  std::iota(src.begin(), src.end(), 0);
  build_cyc(nc, gptr, gcol, src, F.gm, s);
  require(!F.gm.sell, "fused restriction operator on SELL");
  F.grt.upload(grt, s);
  F.glptr.upload(glptr, s);
  F.glp.upload(glp, s);
  F.gla.upload(gla, s);
  F.fused = true;
}

// device storage of a coarse level's DIA+CSR matrix (values filled by numeric())
void coarse_storage(AmgLevel& Cl, const HostCsr& C, hipStream_t s) {
  Cl.n = C.n;
  Cl.diag.alloc(C.n);
  Cl.ptr.upload(C.ptr, s);
  Cl.col.upload(C.col, s);
  Cl.val.alloc(C.col.size());
  Cl.view.n = C.n;
  Cl.view.diag = Cl.diag.p;
  Cl.view.ptr = Cl.ptr.p;
  Cl.view.col = Cl.col.p;
  Cl.view.val = Cl.val.p;
}

}  // namespace

void Amg::setup(const CsrView& A0, hipStream_t s, bool sell64, int dense_max, bool classical_) {
  if (trace_level() >= 2) {
    lvprof = std::make_shared<KernelProf>(64);
    lvprof->on = true;
  }
  lv.clear();
  lv.reserve(32);
  lv.emplace_back();
  lv[0].n = A0.n;
  lv[0].view = A0;
  HostCsr H;
  H.n = A0.n;
  H.diag.resize(A0.n);
  H.ptr.resize(A0.n + 1);
  HIPCHECK(hipMemcpyAsync(H.diag.data(), A0.diag, A0.n * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipMemcpyAsync(H.ptr.data(), A0.ptr, (A0.n + 1) * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  const int nnz0 = H.ptr[A0.n];
  H.col.resize(nnz0);
  H.val.resize(nnz0);
  if (nnz0) {
    HIPCHECK(hipMemcpyAsync(H.col.data(), A0.col, nnz0 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(H.val.data(), A0.val, nnz0 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
  }
  classical = classical_;
  double t_prod = 0.0, t_ops = 0.0;   // host coarsening and product lists; operators and uploads
  while (classical && H.n > dense_max) {
    ClassicalLevel CL;
    const double t0 = wall_ms();
    if (!classical_level(H, kClassicalStrength, 0x5EED0000ULL + lv.size(), CL)) break;
    const double t1 = wall_ms();
    t_prod += t1 - t0;
    AmgLevel& F = lv.back();
    {   // A diag(w): every row as [diagonal, off-diagonal entries]
      std::vector<int> p, c, src;
      aw_rows(H.n, H.ptr, H.col, p, c, src, dia_code, off_code);
      build_cyc(H.n, p, c, src, F.aw, s);
    }
    build_cyc(CL.nc, CL.rptr, CL.rcol, CL.rsrc, F.rm, s);
    if (lv.size() > 1 && H.n <= kFuseRows && H.n < kSellRows) build_fused(H, CL, F, s);
    {
      std::vector<int> src(CL.apcol.size());
      std::iota(src.begin(), src.end(), 0);
      build_cyc(H.n, CL.apptr, CL.apcol, src, F.cm, s);
    }
    if (sell64 && lv.size() == 1) {   // FP64 SELL copy of level 0 for the Krylov products
      build_sell(H, F, s);
      F.sval.release();
      F.sell.val = nullptr;
      F.sval64.alloc(F.scol.n);
      F.sell64.n = F.n;
      F.sell64.sptr = F.sptr.p;
      F.sell64.col = F.scol.p;
      F.sell64.val = F.sval64.p;
    }
    F.pval.upload(CL.pval, s);
    F.aplptr.upload(CL.aplptr.data(), CL.aplptr.size(), s);
    F.apla.upload(CL.apla.data(), CL.apla.size(), s);
    F.aplp.upload(CL.aplp.data(), CL.aplp.size(), s);
    F.appidx.upload(CL.appidx.data(), CL.appidx.size(), s);
    F.apv.alloc(std::max<size_t>(CL.apcol.size(), 1));
    F.clptr.upload(CL.clptr.data(), CL.clptr.size(), s);
    F.clr.upload(CL.clr.data(), CL.clr.size(), s);
    F.clq.upload(CL.clq.data(), CL.clq.size(), s);
    hipLaunchKernelGGL(k_fill_rm, dim3(grid_for(F.rm.src.n, kBlock)), dim3(kBlock), 0, s, (int)F.rm.src.n,
                       F.rm.src.p, F.pval.p, F.rm.val.p);
    LAUNCHCHECK();
    lv.emplace_back();
    coarse_storage(lv.back(), CL.C, s);
    HIPCHECK(hipStreamSynchronize(s));
    H = std::move(CL.C);
    t_ops += wall_ms() - t1;
  }
  if (classical && trace_level() > 0)
    std::fprintf(stderr, "[spfas] classical AMG setup: coarsening and product lists %.1f ms, operators and uploads %.1f ms\n",
                 t_prod, t_ops);
  if (classical && lv.size() == 1 && H.n > dense_max) classical = false;   // no classical coarsening: aggregation
  while (!classical && H.n > dense_max) {
    std::vector<int> agg;
    const int nc = aggregate(H, kStrength, agg);
    if (nc >= H.n || nc * 10 > H.n * 9) break;   // coarsening stalled
    AmgLevel& F = lv.back();
    F.vec = H.n < kVecRows;
    if (!F.vec) {
      build_sell(H, F, s);
      if (sell64 && lv.size() == 1) {
        F.sval64.alloc(F.sval.n);
        F.sell64.n = F.n;
        F.sell64.sptr = F.sptr.p;
        F.sell64.col = F.scol.p;
        F.sell64.val = F.sval64.p;
      }
    }
    // members
    std::vector<int> mptr(nc + 1, 0), mem(H.n);
    for (int i = 0; i < H.n; ++i) mptr[agg[i] + 1]++;
    for (int I = 0; I < nc; ++I) mptr[I + 1] += mptr[I];
    {
      std::vector<int> fill(mptr.begin(), mptr.end() - 1);
      for (int i = 0; i < H.n; ++i) mem[fill[agg[i]]++] = i;
    }
    // coarse pattern and contributor lists
    HostCsr C;
    C.n = nc;
    C.diag.assign(nc, 0.0);
    C.ptr.assign(nc + 1, 0);
    std::vector<std::vector<std::pair<int, int>>> rows(nc);   // (J, fine off index)
    std::vector<std::vector<int>> dg(nc);                     // encoded diag contributors
    for (int I = 0; I < nc; ++I)
      for (int q = mptr[I]; q < mptr[I + 1]; ++q) {
        const int i = mem[q];
        dg[I].push_back(i << 1);
        C.diag[I] += H.diag[i];
        for (int k = H.ptr[i]; k < H.ptr[i + 1]; ++k) {
          const int J = agg[H.col[k]];
          if (J == I) {
            dg[I].push_back((k << 1) | 1);
            C.diag[I] += H.val[k];
          } else {
            rows[I].emplace_back(J, k);
          }
        }
      }
    std::vector<int> gptr(1, 0), gidx;
    for (int I = 0; I < nc; ++I) {
      auto& r = rows[I];
      std::stable_sort(r.begin(), r.end(), [](const std::pair<int, int>& a, const std::pair<int, int>& b) {
        return a.first < b.first;
      });
      size_t q = 0;
      while (q < r.size()) {
        const int J = r[q].first;
        double v = 0.0;
        while (q < r.size() && r[q].first == J) {
          gidx.push_back(r[q].second);
          v += H.val[r[q].second];
          ++q;
        }
        C.col.push_back(J);
        C.val.push_back(v);
        gptr.push_back((int)gidx.size());
      }
      C.ptr[I + 1] = (int)C.col.size();
    }
    std::vector<int> gdptr(1, 0), gdidx;
    for (int I = 0; I < nc; ++I) {
      for (int c : dg[I]) gdidx.push_back(c);
      gdptr.push_back((int)gdidx.size());
    }
    F.agg.upload(agg, s);
    F.mptr.upload(mptr, s);
    F.mem.upload(mem, s);
    F.goff_ptr.upload(gptr, s);
    F.goff_idx.upload(gidx, s);
    F.gdiag_ptr.upload(gdptr, s);
    F.gdiag_idx.upload(gdidx, s);
    lv.emplace_back();
    AmgLevel& Cl = lv.back();
    Cl.n = nc;
    Cl.diag.alloc(nc);
    Cl.ptr.upload(C.ptr, s);
    Cl.col.upload(C.col, s);
    Cl.val.alloc(C.col.size());
    Cl.view.n = nc;
    Cl.view.diag = Cl.diag.p;
    Cl.view.ptr = Cl.ptr.p;
    Cl.view.col = Cl.col.p;
    Cl.view.val = Cl.val.p;
    HIPCHECK(hipStreamSynchronize(s));
    H = std::move(C);
  }
  nd = lv.back().n;
  require(nd <= 4096, "AMG coarsening stalled above the dense limit");
  lu.alloc((size_t)nd * nd);
  for (auto& L : lv) {
    L.invd.alloc(L.n);
    L.t.alloc(L.n);
    if (classical) {
      L.x32.alloc(L.n);
      L.b32.alloc(L.n);
      L.r32.alloc(L.n);
    } else {
      L.x.alloc(L.n);
      L.b.alloc(L.n);
      L.r.alloc(L.n);
    }
  }
  lv.back().t.alloc((size_t)nd * nd);   // dense inverse of the coarsest matrix
  piv.alloc(nd);
  flag.alloc(1);
}

std::string Amg::level_times() {
  if (!lvprof) return "";
  lvprof->collect();
  std::string out = "AMG ms (down/up):";
  char buf[64];
  for (int k = 0; k + 1 < (int)lv.size(); ++k) {
    std::snprintf(buf, sizeof buf, " %.1f/%.1f", lvprof->ms[3 * k], lvprof->ms[3 * k + 1]);
    out += buf;
  }
  std::snprintf(buf, sizeof buf, " dense %.1f", lvprof->ms[63]);
  out += buf;
  lvprof->reset();
  return out;
}

std::string Amg::describe() const {
  std::string out;
  for (const AmgLevel& L : lv) {
    long long nnz = 0;
    if (&L != &lv[0]) nnz = (long long)L.val.n;
    out += std::to_string(L.n) + "/" + std::to_string(nnz) + " ";
  }
  out += "dense " + std::to_string(nd);
  return out;
}

void Amg::numeric(hipStream_t s) {
  if (classical) {
    numeric_classical(s);
    return;
  }
  if (sell_source) sell_to_csr(s);
  for (size_t k = 0; k + 1 < lv.size(); ++k) {
    AmgLevel& F = lv[k];
    AmgLevel& C = lv[k + 1];
    const int nnz = (int)C.val.n;
    if (nnz) {
      hipLaunchKernelGGL(k_galerkin_off, dim3(grid_for(nnz, kBlock)), dim3(kBlock), 0, s, nnz, F.goff_ptr.p,
                         F.goff_idx.p, F.view.val, C.val.p);
      LAUNCHCHECK();
    }
    hipLaunchKernelGGL(k_galerkin_diag, dim3(grid_for(C.n, kBlock)), dim3(kBlock), 0, s, C.n, F.gdiag_ptr.p,
                       F.gdiag_idx.p, F.view.diag, F.view.val, C.diag.p);
    LAUNCHCHECK();
  }
  for (auto& L : lv) {
    hipLaunchKernelGGL(k_invd, dim3(grid_for((size_t)L.n * kVecG, kBlock)), dim3(kBlock), 0, s, L.view, L.invd.p);
    LAUNCHCHECK();
  }
  for (size_t k = 0; k + 1 < lv.size(); ++k) {
    AmgLevel& F = lv[k];
    if (F.vec) continue;
    const int ne = (int)F.sval.n;
    hipLaunchKernelGGL(k_sell_fill, dim3(grid_for(ne, kBlock)), dim3(kBlock), 0, s, ne, F.smap.p, F.view.diag,
                       F.view.val, F.sval.p, F.sval64.p);
    LAUNCHCHECK();
  }
  dense_numeric(s);
}

__global__ void __launch_bounds__(kBlock) k_sell_to_csr(int ne, const int* __restrict__ smap,
                                                        const double* __restrict__ val, double* __restrict__ diag,
                                                        double* __restrict__ off) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  const int m = smap[e];
  if (m >= 0) off[m] = val[e];
  else if (m != kSellPad) diag[-1 - m] = val[e];
}

void Amg::sell_to_csr(hipStream_t s) {
  AmgLevel& F = lv[0];
  const int ne = (int)F.sval64.n;
  require(ne > 0, "sell_to_csr without a SELL copy");
  double* diag = const_cast<double*>(F.view.diag);
  double* off = const_cast<double*>(F.view.val);
  hipLaunchKernelGGL(k_sell_to_csr, dim3(grid_for(ne, kBlock)), dim3(kBlock), 0, s, ne, F.smap.p, F.sval64.p, diag,
                     off);
  LAUNCHCHECK();
}

void Amg::operator_values(hipStream_t s) {
  AmgLevel& F = lv[0];
  if (!F.sval64.n || sell_source) return;   // SELL source: the Krylov operator is already current
  const int ne = (int)F.sval64.n;
  hipLaunchKernelGGL(k_sell_fill, dim3(grid_for(ne, kBlock)), dim3(kBlock), 0, s, ne, F.smap.p, F.view.diag,
                     F.view.val, (float*)nullptr, F.sval64.p);
  LAUNCHCHECK();
}

void Amg::numeric_classical(hipStream_t s) {
  const int L = (int)lv.size();
  if (sell_source) sell_to_csr(s);
  for (int k = 0; k + 1 < L; ++k) {
    AmgLevel& F = lv[k];
    AmgLevel& C = lv[k + 1];
    const int ne = (int)(F.aplptr.n - 1);
    if (ne > 0) {
      hipLaunchKernelGGL(k_ap_numeric, dim3(grid_for(ne, kBlock)), dim3(kBlock), 0, s, ne, F.aplptr.p, F.apla.p,
                         F.aplp.p, F.view, F.pval.p, F.apv.p);
      LAUNCHCHECK();
    }
    const int noff = (int)C.col.n;
    hipLaunchKernelGGL(k_rap_numeric, dim3(grid_for(noff + C.n, kBlock)), dim3(kBlock), 0, s, noff, C.n, F.clptr.p,
                       F.clr.p, F.clq.p, F.pval.p, F.apv.p, C.val.p, C.diag.p);
    LAUNCHCHECK();
  }
  for (auto& Lv : lv) {
    hipLaunchKernelGGL(k_invd, dim3(grid_for((size_t)Lv.n * kVecG, kBlock)), dim3(kBlock), 0, s, Lv.view, Lv.invd.p);
    LAUNCHCHECK();
  }
  for (int k = 0; k + 1 < L; ++k) {
    AmgLevel& F = lv[k];
    hipLaunchKernelGGL(k_fill_aw, dim3(grid_for(F.aw.src.n, kBlock)), dim3(kBlock), 0, s, (int)F.aw.src.n,
                       F.aw.col.p, F.aw.src.p, F.view, F.invd.p, F.aw.val.p);
    LAUNCHCHECK();
    if (F.fused) {
      const int ne = (int)F.gm.nnz;
      if (ne > 0)
        hipLaunchKernelGGL(k_fill_g, dim3(grid_for(ne, kBlock)), dim3(kBlock), 0, s, ne, F.gm.col.p, F.grt.p,
                           F.glptr.p, F.glp.p, F.gla.p, F.view, F.pval.p, F.invd.p, F.gm.val.p);
      LAUNCHCHECK();
    }
    if (F.cm.sell)
      hipLaunchKernelGGL(k_fill_cm, dim3(grid_for(F.n, kBlock)), dim3(kBlock), 0, s, cyc_view(F.cm), F.cm.src.p,
                         F.appidx.p, F.pval.p, F.apv.p, F.invd.p, F.cm.val.p);
    else
      hipLaunchKernelGGL(k_fill_cmv, dim3(grid_for((size_t)F.n * kVecG, kBlock)), dim3(kBlock), 0, s, cyc_view(F.cm),
                         F.cm.src.p, F.appidx.p, F.pval.p, F.apv.p, F.invd.p, F.cm.val.p);
    LAUNCHCHECK();
    if (F.sval64.n) {
      const int ne = (int)F.sval64.n;
      hipLaunchKernelGGL(k_sell_fill, dim3(grid_for(ne, kBlock)), dim3(kBlock), 0, s, ne, F.smap.p, F.view.diag,
                         F.view.val, (float*)nullptr, F.sval64.p);
      LAUNCHCHECK();
    }
  }
  dense_numeric(s);
}

void Amg::dense_numeric(hipStream_t s) {
  AmgLevel& Lc = lv.back();
  hipLaunchKernelGGL(k_dense_fill, dim3(grid_for(nd, kBlock)), dim3(kBlock), 0, s, Lc.view, lu.p, nd);
  LAUNCHCHECK();
  flag.zero(s);
  if (nd <= kDenseLds)
    hipLaunchKernelGGL(k_dense_inverse_lds, dim3(1), dim3(kBlock), 0, s, lu.p, Lc.t.p, nd, flag.p);
  else
    hipLaunchKernelGGL(k_dense_inverse, dim3(1), dim3(kBlock), 0, s, lu.p, Lc.t.p, piv.p, nd, flag.p);
  LAUNCHCHECK();
}

// One cycle product on operator M: SELL-64 (thread per row; the `Finest`
// flag only names the level-0 launches apart) or CSR with the lane-group
// width chosen for the operator.
template <int Op, class TB, class TY>
static void launch_cyc(const CycMat& M, bool finest, const CycX<Op, TB>* x, const TB* b, const float* r,
                       const double* w, TY* y, hipStream_t s) {
  const CycView v = cyc_view(M);
  if (M.sell) {
    const unsigned g = grid_for(M.n, kBlock);
    if (finest) hipLaunchKernelGGL((k_cyc<Op, true, TB, TY>), dim3(g), dim3(kBlock), 0, s, v, x, b, r, w, y);
    else hipLaunchKernelGGL((k_cyc<Op, false, TB, TY>), dim3(g), dim3(kBlock), 0, s, v, x, b, r, w, y);
    return;
  }
  const unsigned g = grid_for((size_t)M.n * M.lanes, kBlock);
  switch (M.lanes) {
    case 16: hipLaunchKernelGGL((k_cycv<Op, 16, TB, TY>), dim3(g), dim3(kBlock), 0, s, v, x, b, r, w, y); break;
    case 32: hipLaunchKernelGGL((k_cycv<Op, 32, TB, TY>), dim3(g), dim3(kBlock), 0, s, v, x, b, r, w, y); break;
    default: hipLaunchKernelGGL((k_cycv<Op, 8, TB, TY>), dim3(g), dim3(kBlock), 0, s, v, x, b, r, w, y); break;
  }
}

// The fused down leg of a small level (k_cycv_down), with the lane group of
// the longer rows of the two operators.
static void launch_cyc_down(const CycMat& M, const CycMat& G, const float* b, float* y, float* yc, hipStream_t s) {
  require(!M.sell && !G.sell, "fused down leg on SELL operators");
  const int lanes = std::max(M.lanes, G.lanes);
  const unsigned g = grid_for((size_t)(M.n + G.n) * lanes, kBlock);
  const CycView vm = cyc_view(M), vg = cyc_view(G);
  switch (lanes) {
    case 16: hipLaunchKernelGGL(k_cycv_down<16>, dim3(g), dim3(kBlock), 0, s, vm, vg, b, y, yc); break;
    case 32: hipLaunchKernelGGL(k_cycv_down<32>, dim3(g), dim3(kBlock), 0, s, vm, vg, b, y, yc); break;
    default: hipLaunchKernelGGL(k_cycv_down<8>, dim3(g), dim3(kBlock), 0, s, vm, vg, b, y, yc); break;
  }
}

// One V(1,1) cycle of the classical hierarchy, three kernels per level:
// down [pre-sweep + residual] [restriction], up [prolongation + post-sweep].
// FP64 b and x on level 0, FP32 vectors on the levels below and for the
// level-0 residual.
template <class T>
void Amg::apply_classical(const T* b, T* x, hipStream_t s) {
  const int L = (int)lv.size();
  if (L == 1) {   // dense solve only
    timed(lvprof.get(), 63, 0.0, s, [&] {
      hipLaunchKernelGGL((k_dense_gemv<T, T>), dim3(grid_for(nd, kBlock / 64)), dim3(kBlock), 0, s, nd,
                         lv.back().t.p, b, x);
    });
    LAUNCHCHECK();
    return;
  }
  for (int k = 0; k < L - 1; ++k) {
    AmgLevel& F = lv[k];
    AmgLevel& C = lv[k + 1];
    timed(lvprof.get(), 3 * k, 0.0, s, [&] {
      const double n = (double)F.n;
      if (F.fused) {   // residual and its restriction in one launch (k >= 1)
        timed(hook.prof, hook.tail_down_id, 6.0 * (double)(F.aw.nnz + F.gm.nnz) + 8.0 * n + 4.0 * C.n, s, [&] {
          launch_cyc_down(F.aw, F.gm, F.b32.p, F.r32.p, C.b32.p, s);
        });
        return;
      }
      // r = b - A diag(w) b: b read (sizeof(T) bytes on level 0, 4 below), r written in FP32
      const double bsz = k == 0 ? (double)sizeof(T) : 4.0;
      timed(hook.prof, k == 0 ? hook.down_id : hook.tail_down_id, 6.0 * (double)F.aw.nnz + (bsz + 4.0) * n, s, [&] {
        if (k == 0) launch_cyc<0, T, float>(F.aw, true, b, b, nullptr, nullptr, F.r32.p, s);
        else launch_cyc<0, float, float>(F.aw, false, F.b32.p, F.b32.p, nullptr, nullptr, F.r32.p, s);
      });
      timed(hook.prof, k == 0 ? hook.restrict_id : hook.tail_restrict_id,
            6.0 * (double)F.rm.nnz + 4.0 * n + 4.0 * C.n, s, [&] {
        launch_cyc<1, float, float>(F.rm, k == 0, F.r32.p, nullptr, nullptr, nullptr, C.b32.p, s);
      });
    });
    LAUNCHCHECK();
  }
  timed(lvprof.get(), 63, 0.0, s, [&] {
    hipLaunchKernelGGL((k_dense_gemv<float, float>), dim3(grid_for(nd, kBlock / 64)), dim3(kBlock), 0, s, nd,
                       lv.back().t.p, lv.back().b32.p, lv.back().x32.p);
  });
  LAUNCHCHECK();
  for (int k = L - 2; k >= 0; --k) {
    AmgLevel& F = lv[k];
    AmgLevel& C = lv[k + 1];
    timed(lvprof.get(), 3 * k + 1, 0.0, s, [&] {
      // w (8), b, r (4), x per row: b and x sizeof(T) on level 0, 4 below; e gathered in FP32
      const double vsz = k == 0 ? (double)sizeof(T) : 4.0;
      timed(hook.prof, k == 0 ? hook.up_id : hook.tail_up_id,
            6.0 * (double)F.cm.nnz + (12.0 + 2.0 * vsz) * F.n + 4.0 * C.n, s, [&] {
        if (k == 0) launch_cyc<2, T, T>(F.cm, true, C.x32.p, b, F.r32.p, F.invd.p, x, s);
        else launch_cyc<2, float, float>(F.cm, false, C.x32.p, F.b32.p, F.r32.p, F.invd.p, F.x32.p, s);
      });
    });
    LAUNCHCHECK();
  }
}

void Amg::apply(const float* b, float* x, hipStream_t s) {
  require(classical, "FP32 preconditioner input needs the classical AMG");
  apply_classical<float>(b, x, s);
}

void Amg::apply(const double* b, double* x, hipStream_t s) {
  if (classical) {
    apply_classical<double>(b, x, s);
    return;
  }
  // level 0 uses the caller's b and x; V(2,2) with the sweep pairs fused:
  // down: [two sweeps from zero] [residual] [restriction];
  // up:   [prolongation + sweep] [sweep].
  const int L = (int)lv.size();
  const double* bl = b;
  for (int k = 0; k < L - 1; ++k) {
    AmgLevel& F = lv[k];
    AmgLevel& C = lv[k + 1];
    const unsigned g = grid_for(F.n, kBlock);
    KernelProf* pf = k == 0 ? hook.prof : nullptr;
    const double E = 8.0 * (double)F.sell_nnz, n = (double)F.n;
    if (F.vec) {
      timed(lvprof.get(), 3 * k, 0.0, s, [&] {
        const unsigned gv = grid_for((size_t)F.n * kVecG, kBlock);
        hipLaunchKernelGGL(k_amgv_pre, dim3(gv), dim3(kBlock), 0, s, F.view, F.invd.p, bl, F.t.p);
        hipLaunchKernelGGL(k_amgv_resid, dim3(gv), dim3(kBlock), 0, s, F.view, bl, F.t.p, F.r.p);
        hipLaunchKernelGGL(k_restrict_vec, dim3(grid_for((size_t)C.n * kVecG, kBlock)), dim3(kBlock), 0, s, C.n,
                           F.mptr.p, F.mem.p, F.r.p, C.b.p);
      });
      LAUNCHCHECK();
      bl = C.b.p;
      continue;
    }
    timed(lvprof.get(), 3 * k, 0.0, s, [&] {
    timed(pf, hook.down_id, 2.0 * E + 48.0 * n, s, [&] {
      if (pf) hipLaunchKernelGGL(k_amg_pre<true>, dim3(g), dim3(kBlock), 0, s, F.sell, F.invd.p, bl, F.t.p);
      else hipLaunchKernelGGL(k_amg_pre<false>, dim3(g), dim3(kBlock), 0, s, F.sell, F.invd.p, bl, F.t.p);
      if (pf) hipLaunchKernelGGL(k_amg_resid<true>, dim3(g), dim3(kBlock), 0, s, F.sell, bl, F.t.p, F.r.p);
      else hipLaunchKernelGGL(k_amg_resid<false>, dim3(g), dim3(kBlock), 0, s, F.sell, bl, F.t.p, F.r.p);
    });
    timed(pf, hook.restrict_id, 12.0 * n + 8.0 * C.n, s, [&] {
      hipLaunchKernelGGL(k_restrict, dim3(grid_for(C.n, kBlock)), dim3(kBlock), 0, s, C.n, F.mptr.p, F.mem.p, F.r.p,
                         C.b.p);
    });
    LAUNCHCHECK();
    });
    bl = C.b.p;
  }
  double* xl = L == 1 ? x : lv.back().x.p;
  timed(lvprof.get(), 63, 0.0, s, [&] {
    hipLaunchKernelGGL((k_dense_gemv<double, double>), dim3(grid_for(nd, kBlock / 64)), dim3(kBlock), 0, s, nd,
                       lv.back().t.p, bl, xl);
  });
  LAUNCHCHECK();
  for (int k = L - 2; k >= 0; --k) {
    AmgLevel& F = lv[k];
    AmgLevel& C = lv[k + 1];
    const unsigned g = grid_for(F.n, kBlock);
    double* xf = (k == 0) ? x : F.x.p;
    const double* bf = (k == 0) ? b : F.b.p;
    KernelProf* pf = k == 0 ? hook.prof : nullptr;
    const double E = 8.0 * (double)F.sell_nnz, n = (double)F.n;
    if (F.vec) {
      timed(lvprof.get(), 3 * k + 1, 0.0, s, [&] {
        const unsigned gv = grid_for((size_t)F.n * kVecG, kBlock);
        hipLaunchKernelGGL(k_amgv_post1, dim3(gv), dim3(kBlock), 0, s, F.view, F.invd.p, bf, F.t.p, F.agg.p, C.x.p,
                           F.r.p);
        hipLaunchKernelGGL(k_amgv_post2, dim3(gv), dim3(kBlock), 0, s, F.view, F.invd.p, bf, F.r.p, xf);
      });
      LAUNCHCHECK();
      continue;
    }
    timed(lvprof.get(), 3 * k + 1, 0.0, s, [&] {
    timed(pf, hook.up_id, 2.0 * E + 68.0 * n, s, [&] {
      if (pf)
        hipLaunchKernelGGL(k_amg_post1<true>, dim3(g), dim3(kBlock), 0, s, F.sell, F.invd.p, bf, F.t.p, F.agg.p,
                           C.x.p, F.r.p);
      else
        hipLaunchKernelGGL(k_amg_post1<false>, dim3(g), dim3(kBlock), 0, s, F.sell, F.invd.p, bf, F.t.p, F.agg.p,
                           C.x.p, F.r.p);
      if (pf) hipLaunchKernelGGL(k_amg_post2<true>, dim3(g), dim3(kBlock), 0, s, F.sell, F.invd.p, bf, F.r.p, xf);
      else hipLaunchKernelGGL(k_amg_post2<false>, dim3(g), dim3(kBlock), 0, s, F.sell, F.invd.p, bf, F.r.p, xf);
    });
    });
    LAUNCHCHECK();
  }
}

// ------------------------------------------------------------------ Krylov

template <class Mat, bool Fin, class T>
static void spmv_dot_as(const Mat& A, int G, hipStream_t st, const T* x, T* y, const T* w, double* P) {
  hipLaunchKernelGGL((k_spmv_dot<Mat, Fin, T>), dim3(G), dim3(SpmvBlock<Mat>::v), 0, st, A, x, y, w, P);
}

template <class Mat, bool Fin, class T>
static void spmv_dot2_as(const Mat& A, int G, hipStream_t st, const T* x, T* y, const T* w, double* P0, double* P1) {
  hipLaunchKernelGGL((k_spmv_dot2<Mat, Fin, T>), dim3(G), dim3(SpmvBlock<Mat>::v), 0, st, A, x, y, w, P0, P1);
}

// y = A x and one partial dot product w.y per block (G blocks)
template <class T, class SellT>
static void spmv_dot(const CsrView& A, const SellT* As, bool fin, int G, hipStream_t st, const T* x, T* y,
                     const T* w, double* P) {
  if (As) {
    if (fin) spmv_dot_as<SellT, true>(*As, G, st, x, y, w, P);
    else spmv_dot_as<SellT, false>(*As, G, st, x, y, w, P);
  } else {
    if (fin) spmv_dot_as<CsrView, true>(A, G, st, x, y, w, P);
    else spmv_dot_as<CsrView, false>(A, G, st, x, y, w, P);
  }
  LAUNCHCHECK();
}

// y = A x, partials of w.y and y.y per block
template <class T, class SellT>
static void spmv_dot2(const CsrView& A, const SellT* As, bool fin, int G, hipStream_t st, const T* x, T* y,
                      const T* w, double* P0, double* P1) {
  if (As) {
    if (fin) spmv_dot2_as<SellT, true>(*As, G, st, x, y, w, P0, P1);
    else spmv_dot2_as<SellT, false>(*As, G, st, x, y, w, P0, P1);
  } else {
    if (fin) spmv_dot2_as<CsrView, true>(A, G, st, x, y, w, P0, P1);
    else spmv_dot2_as<CsrView, false>(A, G, st, x, y, w, P0, P1);
  }
  LAUNCHCHECK();
}

// doubles of Krylov::hlag
constexpr int kLagDoubles = 2 + 3 * kMaxParts;

template <class T>
KrylovT<T>::~KrylovT() {
  if (hlag) (void)hipHostFree(hlag);
  for (hipEvent_t& e : ev)
    if (e) (void)hipEventDestroy(e);
}

template <class T>
void KrylovT<T>::alloc(int n_) {
  if (n == n_ && hlag) return;
  n = n_;
  r.alloc(n); z.alloc(n); p.alloc(n); q.alloc(n); rh.alloc(n); v.alloc(n); s.alloc(n); t.alloc(n); y.alloc(n);
  w.alloc(n);
  parts.alloc(kMaxParts * 3);
  scal.alloc(S_NSLOT);
  if (!hlag) {   // coherent host-mapped: the kernels write what the host checks there directly
    HIPCHECK(hipHostMalloc((void**)&hlag, kLagDoubles * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
    HIPCHECK(hipHostGetDevicePointer((void**)&dlag, hlag, 0));
  }
  for (hipEvent_t& e : ev)
    if (!e) HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

template <class T>
int KrylovT<T>::pcg(const CsrView& A, Amg* M, const T* b, T* x, double rtol, int maxit, hipStream_t st, int stall) {
  alloc(A.n);
  const int G = reduce_grid(n);
  const unsigned g1 = grid_for(n, kBlock);
  double* P0 = parts.p;
  double* P1 = parts.p + kMaxParts;
  require(G <= kMaxParts, "reduction grid larger than the partial-sum buffers");
  // host-mapped: [p.q of the last two iterations | b.b partials | r.r
  // partials of the last two iterations], written by the kernels
  const volatile double* hl = hlag;
  double* d_bb = dlag + 2;
  double* d_rr = dlag + 2 + kMaxParts;
  hipLaunchKernelGGL(k_zero<T>, dim3(G), dim3(kBlock), 0, st, n, x);
  hipLaunchKernelGGL(k_copy<T>, dim3(G), dim3(kBlock), 0, st, n, b, r.p);
  hipLaunchKernelGGL(k_dot<T>, dim3(G), dim3(kBlock), 0, st, n, b, b, d_bb);
  LAUNCHCHECK();
  // b.b reaches the host with the scalars of iteration 0 (no wait of its own)
  failed = false;
  converged = false;
  double tol2 = 0.0;
  bool have_bb = false;
  int it = 0;
  int cur = S_RZ0, old = S_RZ1;
  static_assert(S_RR == S_PQ + 1 && S_BB == S_RR + 1, "p.Ap, r.r and b.b are read together");
  // While the residual is far above the tolerance, the residual of
  // iteration k is checked while iteration k + 1 is already queued, so the
  // device never waits for the host; within a factor 10 of the tolerance
  // each iteration is checked as soon as it completes, so the solve stops
  // at the first iteration that meets it (or one later, if it jumps there).
  auto host_total = [&](const volatile double* v) {   // partials in block order
    double t = 0.0;
    for (int i = 0; i < G; ++i) t += v[i];
    return t;
  };
  auto lagged = [&](int k, double& pq, double& rr) {
    HIPCHECK(hipEventSynchronize(ev[k & 1]));
    pq = hl[k & 1];
    rr = host_total(hl + 2 + kMaxParts * (1 + (k & 1)));
    if (!have_bb) {
      have_bb = true;
      const double bb = host_total(hl + 2);
      tol2 = rtol * rtol * bb;
      return !std::isfinite(bb) ? 2 : (bb == 0.0 ? 1 : 0);   // 2: non-finite b, 1: b = 0
    }
    return 0;
  };
  auto bad = [&](double pq, double rr) { return !std::isfinite(rr) || !(pq > 0.0); };
  // stall > 0: give up (neither converged nor failed) once r.r of an
  // iteration is above a quarter of its value `stall` iterations earlier
  std::vector<double> hist;
  auto stalled = [&](int k, double rr) {
    if (stall <= 0) return false;
    if ((int)hist.size() <= k) hist.resize(k + 1, HUGE_VAL);
    hist[k] = rr;
    return k >= stall && rr > 0.25 * hist[k - stall];
  };
  bool stop = false;
  bool near = false;   // within a factor 10 of the tolerance: check every iteration at once
  for (; it < maxit; ++it) {
    if (M) M->apply(r.p, z.p, st);
    else hipLaunchKernelGGL(k_copy<T>, dim3(G), dim3(kBlock), 0, st, n, r.p, z.p);
    // partial sums: P0 r.z, P1 p.q (each consumed by the next kernel), r.r
    // (host-mapped, for the host's check)
    hipLaunchKernelGGL(k_dot<T>, dim3(G), dim3(kBlock), 0, st, n, r.p, z.p, P0);
    hipLaunchKernelGGL(k_pcg_p2<T>, dim3(G), dim3(kBlock), 0, st, n, P0, G, scal.p, cur, old, it == 0 ? 1 : 0, z.p, p.p);
    timed(hook.prof, hook.spmv_id, hook.spmv_bytes, st,
          [&] { spmv_dot(A, sell, hook.prof != nullptr, G, st, p.p, q.p, p.p, P1); });
    hipLaunchKernelGGL(k_pcg_xr2<T>, dim3(G), dim3(kBlock), 0, st, n, P1, G, scal.p, cur, x, r.p, p.p, q.p,
                       d_rr + kMaxParts * (it & 1), dlag + (it & 1));
    LAUNCHCHECK();
    std::swap(cur, old);
    HIPCHECK(hipEventRecord(ev[it & 1], st));
    double pq, rr;
    if (!near && it > 0) {
      lagged(it - 1, pq, rr);
      if (bad(pq, rr)) { failed = true; ++it; break; }
      if (rr <= tol2) {
        // iteration it is already in x: keep it only if its p.Ap is sound
        // (Newton systems are not symmetric, so p.Ap can be <= 0), else take
        // it back and return the iterate that met the tolerance
        converged = true;
        HIPCHECK(hipEventSynchronize(ev[it & 1]));
        const double pq_it = hl[it & 1];
        if (!std::isfinite(pq_it)) {
          failed = true;
          converged = false;
        } else if (!(pq_it > 0.0)) {
          hipLaunchKernelGGL(k_pcg_undo<T>, dim3(G), dim3(kBlock), 0, st, n, scal.p, old, pq_it, x, p.p);
          LAUNCHCHECK();
          break;   // `it` iterations were kept
        }
        ++it;
        break;
      }
      if (stalled(it - 1, rr)) { stop = true; ++it; break; }
      near = rr <= 100.0 * tol2;
    }
    if (near || it == 0) {
      const int zb = lagged(it, pq, rr);   // it == 0 always comes here first
      if (zb == 2) { failed = true; it = 0; break; }
      if (zb == 1) { converged = true; it = 0; break; }   // b = 0: x = 0 (alpha was 0)
      if (bad(pq, rr)) { failed = true; ++it; break; }
      if (rr <= tol2) { converged = true; ++it; break; }
      if (stalled(it, rr)) { stop = true; ++it; break; }
      near = rr <= 100.0 * tol2;
    }
  }
  if (!failed && !converged && !stop && it > 0 && !near) {   // the last iteration has not been checked yet
    double pq, rr;
    lagged(it - 1, pq, rr);
    if (bad(pq, rr)) failed = true;
    else if (rr <= tol2) converged = true;
  }
  if (failed) {   // breakdown (p.Ap <= 0) or non-finite operator: x = 0
    hipLaunchKernelGGL(k_zero<T>, dim3(G), dim3(kBlock), 0, st, n, x);
    LAUNCHCHECK();
  }
  (void)g1;
  iters += it;
  return it;
}

template <class T>
int KrylovT<T>::bicgstab(const CsrView& A, Amg* M, const T* b, T* x, double rtol, int maxit, hipStream_t st) {
  alloc(A.n);
  const int G = reduce_grid(n);
  double* P0 = parts.p;
  double* P1 = parts.p + kMaxParts;
  int cur = S_RHO0, old = S_RHO1;
  // the host's checks: b.b, then r.r of each iteration (host-mapped)
  const volatile double* hl = hlag;
  // x = 0, r = rh = b; ||b||^2 is also rho_0 = rh.r
  hipLaunchKernelGGL(k_bicg_init<T>, dim3(G), dim3(kBlock), 0, st, n, b, x, r.p, rh.p, P0);
  hipLaunchKernelGGL(k_finalize2, dim3(1), dim3(kBlock), 0, st, P0, P0, G, scal.p, (int)S_BB, cur, 0, dlag);
  LAUNCHCHECK();
  HIPCHECK(hipStreamSynchronize(st));
  const double bb = hl[0];
  failed = !std::isfinite(bb);
  converged = bb == 0.0;
  if (!(bb > 0.0) || failed) return 0;
  const double tol2 = rtol * rtol * bb;
  int it = 0;
  for (; it < maxit; ++it) {
    hipLaunchKernelGGL(k_bicg_p<T>, dim3(G), dim3(kBlock), 0, st, n, scal.p, cur, old, it == 0 ? 1 : 0, r.p, p.p, v.p);
    LAUNCHCHECK();
    if (M) M->apply(p.p, y.p, st);
    else hipLaunchKernelGGL(k_copy<T>, dim3(G), dim3(kBlock), 0, st, n, p.p, y.p);
    timed(hook.prof, hook.spmv_id, hook.spmv_bytes, st,
          [&] { spmv_dot(A, sell, hook.prof != nullptr, G, st, y.p, v.p, rh.p, P0); });
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, st, P0, G, scal.p, (int)S_RV);
    hipLaunchKernelGGL(k_bicg_s<T>, dim3(G), dim3(kBlock), 0, st, n, scal.p, cur, r.p, v.p, s.p);
    LAUNCHCHECK();
    if (M) M->apply(s.p, z.p, st);
    else hipLaunchKernelGGL(k_copy<T>, dim3(G), dim3(kBlock), 0, st, n, s.p, z.p);
    timed(hook.prof, hook.spmv2_id, hook.spmv_bytes, st,
          [&] { spmv_dot2(A, sell, hook.prof != nullptr, G, st, z.p, t.p, s.p, P0, P1); });
    // TS, TT and omega = TS / TT in one launch
    hipLaunchKernelGGL(k_finalize2, dim3(1), dim3(kBlock), 0, st, P0, P1, G, scal.p, (int)S_TS, (int)S_TT, 1,
                       nullptr);
    hipLaunchKernelGGL(k_bicg_xr<T>, dim3(G), dim3(kBlock), 0, st, n, scal.p, x, y.p, z.p, r.p, s.p, t.p, rh.p, P0, P1);
    // ||r||^2 and the next rho = rh.r (into the slot of the previous rho)
    hipLaunchKernelGGL(k_finalize2, dim3(1), dim3(kBlock), 0, st, P0, P1, G, scal.p, (int)S_RR, old, 0, dlag);
    LAUNCHCHECK();
    std::swap(cur, old);
    HIPCHECK(hipStreamSynchronize(st));
    const double rr = hl[0];
    if (!std::isfinite(rr)) {   // breakdown or non-finite operator: report, leave x = 0
      failed = true;
      hipLaunchKernelGGL(k_zero<T>, dim3(G), dim3(kBlock), 0, st, n, x);
      ++it;
      break;
    }
    if (rr <= tol2) { ++it; converged = true; break; }
  }
  iters += it;
  return it;
}

template struct KrylovT<double>;
template struct KrylovT<float>;

int launch_resid64(const CsrView& A, const Sell64View* As, const double* x, const double* b, float* r, double* parts,
                   hipStream_t s) {
  const int G = reduce_grid(A.n);
  if (As) {
    require(As->n == A.n, "SELL copy of another matrix");
    hipLaunchKernelGGL(k_resid64<Sell64View>, dim3(G), dim3(SpmvBlock<Sell64View>::v), 0, s, *As, x, b, r, parts);
  } else {
    hipLaunchKernelGGL(k_resid64<CsrView>, dim3(G), dim3(SpmvBlock<CsrView>::v), 0, s, A, x, b, r, parts);
  }
  LAUNCHCHECK();
  return G;
}

}  // namespace spfas
