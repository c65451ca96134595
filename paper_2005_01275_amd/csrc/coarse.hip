// Coarse levels in the solve phase (Sections 3.2-3.4 of the paper):
//   * the level operator assembled cell by cell from the static local
//     matrices scaled by 1/kappa of the aggregate-average pressure (Prop. 1),
//   * Picard/Newton linearisation (Props. 2 and 3: E_c = D_c^T +
//     (M_c sigma_c) kinv'(pbar_c) w_c^T) solved by algebraic hybridisation:
//     local saddle blocks inverted cell by cell, multipliers on the
//     interfaces between cells, H lambda = xi, local back-substitution,
//   * restriction R = P^T, projection Q and prolongation P between levels.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "coarse_kern.hpp"
#include "hier.hpp"
#include "kappa.hpp"
#include "kern.hpp"

namespace spfas {

// ------------------------------------------------------------------ residual

struct CView {
  int n, np, nf;
  const int *pptr, *lfptr, *lfidx, *mptr, *dptr, *fcell, *floc;
  const double *M, *D, *w;
  const double* z;   // shift of kappa per cell (volume mean of the level-0 shift), nullptr: none
};

static CView cview(const CoarseLevel& C) {
  CView v;
  v.n = C.n; v.np = C.np; v.nf = C.nf;
  v.pptr = C.pptr.p; v.lfptr = C.lfptr.p; v.lfidx = C.lfidx.p; v.mptr = C.mptr.p; v.dptr = C.dptr.p;
  v.fcell = C.fcell.p; v.floc = C.floc.p; v.M = C.M.p; v.D = C.D.p; v.w = C.w.p;
  v.z = C.has_shift ? C.zbar.p : nullptr;
  return v;
}

// One residual row (coarse flux `it` < nf, or the m_c pressure rows of cell
// it - nf) at NT step lengths: acc[t] += the squares of its entries of
// r(x + s_t dx).  Shared by the single-step and the multi-step kernels, with
// every multiply-add written as an explicit fma, so a step gives the same
// bits in both whatever the compiler would contract.
template <bool STEP, int NT>
__device__ inline void coarse_row(const CView& v, const KappaFam& kf, int it, const double* __restrict__ sig,
                                  const double* __restrict__ p, const double* __restrict__ dsig,
                                  const double* __restrict__ dp, const double* steps,
                                  const double* __restrict__ b, double* __restrict__ r, double* acc) {
  // value of component i at step t: a_i + s_t d_i (explicit fma)
  auto stp = [&](double a, double d, int t) { return STEP ? fma(steps[t], d, a) : a; };
  if (it < v.nf) {
    const int j = it;
    double val[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) val[t] = 0.0;
    for (int slot = 0; slot < 2; ++slot) {
      const int c = v.fcell[2 * j + slot];
      if (c < 0) continue;
      const int li = v.floc[2 * j + slot];
      const int k = v.lfptr[c + 1] - v.lfptr[c];
      const int p0 = v.pptr[c], m = v.pptr[c + 1] - p0;
      const double* Mr = v.M + v.mptr[c] + li * k;
      const int* lf = v.lfidx + v.lfptr[c];
      // every sum runs over its index in the same order for each step, so a
      // step gives the same bits whatever NT is; each datum is loaded once
      double pbar[NT], ms[NT], dtp[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) pbar[t] = ms[t] = dtp[t] = 0.0;
      for (int q = 0; q < m; ++q) {
        const double wq = v.w[p0 + q], dq = v.D[v.dptr[c] + q * k + li];
        const double a = p[p0 + q], d = STEP ? dp[p0 + q] : 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          pbar[t] = fma(wq, stp(a, d, t), pbar[t]);
          dtp[t] = fma(dq, stp(a, d, t), dtp[t]);
        }
      }
      for (int i = 0; i < k; ++i) {
        const double mi = Mr[i];
        const int f = lf[i];
        const double a = sig[f], d = STEP ? dsig[f] : 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) ms[t] = fma(mi, stp(a, d, t), ms[t]);
      }
#pragma unroll
      for (int t = 0; t < NT; ++t) val[t] = val[t] + fma(kap_inv(kf, kap_psi(v.z, pbar[t], c)), ms[t], dtp[t]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const double ri = val[t] - b[j];
      if (r) r[j] = ri;
      acc[t] = fma(ri, ri, acc[t]);
    }
  } else {
    const int c = it - v.nf;
    const int k = v.lfptr[c + 1] - v.lfptr[c];
    const int p0 = v.pptr[c], m = v.pptr[c + 1] - p0;
    const int* lf = v.lfidx + v.lfptr[c];
    for (int q = 0; q < m; ++q) {
      const double* Dr = v.D + v.dptr[c] + q * k;
      double dv[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) dv[t] = 0.0;
      for (int i = 0; i < k; ++i) {
        const double di = Dr[i];
        const int f = lf[i];
        const double a = sig[f], d = STEP ? dsig[f] : 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) dv[t] = fma(di, stp(a, d, t), dv[t]);
      }
      const double bq = b[v.nf + p0 + q];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const double ri = dv[t] - bq;
        if (r) r[v.nf + p0 + q] = ri;
        acc[t] = fma(ri, ri, acc[t]);
      }
    }
  }
}

template <bool STEP>
__global__ void __launch_bounds__(kBlock) k_coarse_resid(CView v, KappaFam kf, const double* __restrict__ x,
                                                         const double* __restrict__ dx, double step,
                                                         const double* __restrict__ b, double* __restrict__ r,
                                                         double* __restrict__ parts) {
  __shared__ double sh[kBlock / 64];
  double acc[1] = {0.0};
  const int ntot = v.nf + v.n;
  for (int it = blockIdx.x * blockDim.x + threadIdx.x; it < ntot; it += gridDim.x * blockDim.x)
    coarse_row<STEP, 1>(v, kf, it, x, x + v.nf, dx, STEP ? dx + v.nf : nullptr, &step, b, r, acc);
  const double a = block_sum(acc[0], sh);
  if (threadIdx.x == 0) parts[blockIdx.x] = a;
}

struct CoarseSteps {
  double s[kMaxTrials];
};

// Sums of squares of r(x + s_t dx) for NT step lengths in one pass:
// parts[t * gridDim.x + block].
template <int NT>
__global__ void __launch_bounds__(kBlock) k_coarse_resid_trials(CView v, KappaFam kf, const double* __restrict__ x,
                                                                const double* __restrict__ dx, CoarseSteps st,
                                                                const double* __restrict__ b,
                                                                double* __restrict__ parts) {
  __shared__ double sh[kBlock / 64];
  double acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = 0.0;
  const int ntot = v.nf + v.n;
  for (int it = blockIdx.x * blockDim.x + threadIdx.x; it < ntot; it += gridDim.x * blockDim.x)
    coarse_row<true, NT>(v, kf, it, x, x + v.nf, dx, dx + v.nf, st.s, b, nullptr, acc);
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const double a = block_sum(acc[t], sh);
    if (threadIdx.x == 0) parts[t * gridDim.x + blockIdx.x] = a;
  }
}

int launch_coarse_resid_trials(const CoarseLevel& C, const KappaFam& kf, const double* x, const double* dx,
                               const double* steps, int nt, const double* b, double* parts, hipStream_t s) {
  require(nt >= 1 && nt <= kMaxTrials, "number of trial steps out of range");
  const int G = reduce_grid(C.nf + C.n);
  CView v = cview(C);
  CoarseSteps cs{};
  for (int t = 0; t < nt; ++t) cs.s[t] = steps[t];
  switch (nt) {
    case 1: hipLaunchKernelGGL(k_coarse_resid_trials<1>, dim3(G), dim3(kBlock), 0, s, v, kf, x, dx, cs, b, parts); break;
    case 2: hipLaunchKernelGGL(k_coarse_resid_trials<2>, dim3(G), dim3(kBlock), 0, s, v, kf, x, dx, cs, b, parts); break;
    case 3: hipLaunchKernelGGL(k_coarse_resid_trials<3>, dim3(G), dim3(kBlock), 0, s, v, kf, x, dx, cs, b, parts); break;
    default: hipLaunchKernelGGL(k_coarse_resid_trials<4>, dim3(G), dim3(kBlock), 0, s, v, kf, x, dx, cs, b, parts); break;
  }
  LAUNCHCHECK();
  return G;
}

int launch_coarse_resid(const CoarseLevel& C, const KappaFam& kf, const double* x, const double* dx, double step,
                        const double* b, double* r, double* parts, hipStream_t s) {
  const int G = reduce_grid(C.nf + C.n);
  CView v = cview(C);
  if (dx)
    hipLaunchKernelGGL(k_coarse_resid<true>, dim3(G), dim3(kBlock), 0, s, v, kf, x, dx, step, b, r, parts);
  else
    hipLaunchKernelGGL(k_coarse_resid<false>, dim3(G), dim3(kBlock), 0, s, v, kf, x, dx, step, b, r, parts);
  LAUNCHCHECK();
  return G;
}

// ------------------------------------------------------------------ hybridisation

struct HView {
  CView v;
  const int *zptr, *invptr, *lam_of;   // lam_of: multiplier index of a flux unknown, -1 if none
  double *inv, *tmp, *z;
};

// ---- block elimination with the static M_c^{-1} (cells with m_c <= kLocM)
//
// A_c = [[sc M_c, E_c], [D_c, 0]] with sc = 1/kappa(pbar_c) and E_c = D_c^T
// (Picard) or D_c^T + (M_c sigma_c) dsc w_c^T (Newton, dsc = d sc / d pbar).
// M_c is static, so with Minv = M_c^{-1}, G = Minv D_c^T and DG = D_c G kept
// from setup:  Y = (sc M_c)^{-1} E_c = (G + sigma_c dsc w_c^T) / sc,
// S = D_c Y = (DG + (D_c sigma_c) dsc w_c^T) / sc, and
//   A_c^{-1} = [[Minv/sc - Y S^{-1} G^T/sc, Y S^{-1}], [S^{-1} G^T/sc, -S^{-1}]].
constexpr int kLocM = 8;

struct LocStatic {
  const int* gptr;       // offset of G_c (k_c x m_c, row-major)
  const int* sgptr;      // offset of DG_c (m_c x m_c)
  const double* Minv;    // at mptr[c], k_c x k_c
  const double* G;
  const double* DG;
};

__device__ inline double wave_allsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Setup: Minv (Gauss-Jordan without pivoting; M_c is symmetric positive
// definite, a non-positive pivot sets *flag), symmetrised; G; DG.  One wave
// per cell, rows padded to 65 doubles in LDS (no bank conflicts).
__global__ void __launch_bounds__(64) k_local_static(CView v, LocStatic ls, double* __restrict__ Minv,
                                                     double* __restrict__ G, double* __restrict__ DG,
                                                     int* __restrict__ flag) {
  __shared__ double a[64 * 65];
  const int c = blockIdx.x, lane = threadIdx.x;
  const int k = v.lfptr[c + 1] - v.lfptr[c];
  const int p0 = v.pptr[c], m = v.pptr[c + 1] - p0;
  const double* Mc = v.M + v.mptr[c];
  const double* Dc = v.D + v.dptr[c];
  for (int i = 0; i < k; ++i)
    if (lane < k) a[i * 65 + lane] = Mc[i * k + lane];
  __syncthreads();
  for (int kk = 0; kk < k; ++kk) {
    const double pv = a[kk * 65 + kk];
    const double f = (lane < k && lane != kk) ? a[lane * 65 + kk] : 0.0;
    __syncthreads();
    if (lane == 0 && !(pv > 0.0)) flag[0] = 1;
    const double ip = 1.0 / pv;
    if (lane < k && lane != kk) {
      for (int j = 0; j < k; ++j)
        if (j != kk) a[lane * 65 + j] -= f * ip * a[kk * 65 + j];
      a[lane * 65 + kk] = -f * ip;
    }
    __syncthreads();
    if (lane < k) a[kk * 65 + lane] = lane == kk ? ip : a[kk * 65 + lane] * ip;
    __syncthreads();
  }
  double* Mi = Minv + v.mptr[c];
  for (int i = 0; i < k; ++i)
    if (lane < k) Mi[i * k + lane] = 0.5 * (a[i * 65 + lane] + a[lane * 65 + i]);
  __syncthreads();
  // G = Minv D^T (row `lane`), DG = D G
  double g[kLocM];
#pragma unroll
  for (int q = 0; q < kLocM; ++q) g[q] = 0.0;
  if (lane < k)
    for (int j = 0; j < k; ++j) {
      const double mij = 0.5 * (a[lane * 65 + j] + a[j * 65 + lane]);
#pragma unroll
      for (int q = 0; q < kLocM; ++q)
        if (q < m) g[q] += mij * Dc[q * k + j];
    }
  double* Gc = G + ls.gptr[c];
#pragma unroll
  for (int q = 0; q < kLocM; ++q)
    if (q < m && lane < k) Gc[lane * m + q] = g[q];
  double* DGc = DG + ls.sgptr[c];
#pragma unroll
  for (int q = 0; q < kLocM; ++q)
#pragma unroll
    for (int r = 0; r < kLocM; ++r)
      if (q < m && r < m) {
        const double t = wave_allsum(lane < k ? Dc[q * k + lane] * g[r] : 0.0);
        if (lane == 0) DGc[q * m + r] = t;
      }
}

// Per cell (one wave): A_c^{-1} by block elimination, z_c = A_c^{-1} g_c with
// g = [-r_hat; -r_p] (r_hat keeps r_sigma on the first owner only).
__global__ void __launch_bounds__(kBlock) k_coarse_local(HView hv, LocStatic ls, KappaFam kf, int newton,
                                                         const double* __restrict__ x, const double* __restrict__ r) {
  __shared__ double sT[kBlock / 64][64 * kLocM];
  __shared__ double sS[kBlock / 64][kLocM * kLocM];
  __shared__ double sg[kBlock / 64][64];
  const CView& v = hv.v;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.x * (kBlock / 64) + wv;
  const bool act = c < v.n;
  int k = 0, m = 0, p0 = 0;
  double isc = 1.0, dsc = 0.0;
  double Gj[kLocM], Yj[kLocM], z2[kLocM];
  if (act) {
    k = v.lfptr[c + 1] - v.lfptr[c];
    p0 = v.pptr[c];
    m = v.pptr[c + 1] - p0;
    const int* lf = v.lfidx + v.lfptr[c];
    const double* sig = x;
    const double* p = x + v.nf;
    const double* w = v.w + p0;
    double pbar = 0.0;
    for (int q = 0; q < m; ++q) pbar += w[q] * p[p0 + q];
    const double ps = kap_psi(v.z, pbar, c);
    const double sc = kap_inv(kf, ps);
    dsc = kap_dinv(kf, ps, sc);
    isc = 1.0 / sc;
    double sj = 0.0, g1 = 0.0;
#pragma unroll
    for (int q = 0; q < kLocM; ++q) Gj[q] = 0.0;
    if (lane < k) {
      const int fj = lf[lane];
      if (newton) sj = sig[fj];
      g1 = (v.fcell[2 * fj] == c) ? -r[fj] : 0.0;
      const double* Gr = ls.G + ls.gptr[c] + lane * m;
#pragma unroll
      for (int q = 0; q < kLocM; ++q)
        if (q < m) Gj[q] = Gr[q];
    }
    sg[wv][lane] = g1;
    // D sigma and G^T g1 (wave sums; m is uniform over the wave)
    double dsig[kLocM], u[kLocM];
#pragma unroll
    for (int q = 0; q < kLocM; ++q) {
      dsig[q] = 0.0;
      u[q] = 0.0;
      if (q < m) {
        dsig[q] = wave_allsum(lane < k ? v.D[v.dptr[c] + q * k + lane] * sj : 0.0);
        u[q] = wave_allsum(Gj[q] * g1) * isc + r[v.nf + p0 + q];   // G^T g1 / sc - g2
      }
    }
    // S, padded with the identity to kLocM, inverted in place (Gauss-Jordan)
    const double* DG = ls.DG + ls.sgptr[c];
    double S[kLocM][kLocM];
#pragma unroll
    for (int q = 0; q < kLocM; ++q)
#pragma unroll
      for (int j = 0; j < kLocM; ++j)
        S[q][j] = (q < m && j < m) ? (DG[q * m + j] + dsig[q] * dsc * w[j]) * isc : (q == j ? 1.0 : 0.0);
#pragma unroll
    for (int kk = 0; kk < kLocM; ++kk) {
      const double ip = 1.0 / S[kk][kk];
      S[kk][kk] = 1.0;
#pragma unroll
      for (int j = 0; j < kLocM; ++j) S[kk][j] *= ip;
#pragma unroll
      for (int q = 0; q < kLocM; ++q) {
        if (q == kk) continue;
        const double f = S[q][kk];
        S[q][kk] = 0.0;
#pragma unroll
        for (int j = 0; j < kLocM; ++j) S[q][j] -= f * S[kk][j];
      }
    }
    // Y row, T = Y S^{-1} row, z2 = S^{-1} (G^T g1 / sc - g2)
#pragma unroll
    for (int q = 0; q < kLocM; ++q) Yj[q] = q < m ? (Gj[q] + sj * dsc * w[q]) * isc : 0.0;
    if (lane < k) {
#pragma unroll
      for (int j = 0; j < kLocM; ++j) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < kLocM; ++q) t += Yj[q] * S[q][j];
        sT[wv][lane * kLocM + j] = t;
      }
    }
#pragma unroll
    for (int q = 0; q < kLocM; ++q) {
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < kLocM; ++j) t += S[q][j] * u[j];
      z2[q] = t;
    }
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < kLocM; ++q)
#pragma unroll
        for (int j = 0; j < kLocM; ++j) sS[wv][q * kLocM + j] = S[q][j];
    }
  }
  __syncthreads();
  if (!act) return;
  const int nc = k + m;
  double* inv = hv.inv + hv.invptr[c];
  const double* Mi = ls.Minv + v.mptr[c];
  double h = 0.0;   // (Minv g1)[lane]: Minv is symmetric
  for (int i = 0; i < k; ++i) {
    const double* Ti = &sT[wv][i * kLocM];
    if (lane < k) {
      const double mij = Mi[i * k + lane];
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < kLocM; ++j) t += Ti[j] * Gj[j];
      inv[i * nc + lane] = (mij - t) * isc;
      h += mij * sg[wv][i];
    } else if (lane < nc) {
      inv[i * nc + lane] = Ti[lane - k];
    }
  }
  for (int q = 0; q < m; ++q) {
    const double* Sq = &sS[wv][q * kLocM];
    if (lane < k) {
      double t = 0.0;
#pragma unroll
      for (int j = 0; j < kLocM; ++j) t += Sq[j] * Gj[j];
      inv[(k + q) * nc + lane] = t * isc;
    } else if (lane < nc) {
      inv[(k + q) * nc + lane] = -Sq[lane - k];
    }
  }
  double* z = hv.z + hv.zptr[c];
  if (lane < k) {
    double t = h * isc;
#pragma unroll
    for (int q = 0; q < kLocM; ++q) t -= Yj[q] * z2[q];
    z[lane] = t;
  } else if (lane < nc) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kLocM; ++q)
      if (lane - k == q) t = z2[q];
    z[lane] = t;
  }
}

// ---- general cells: LU of the whole saddle block
// Per cell: build A_c, invert it (LU with partial pivoting, then the columns
// of the inverse), z_c = A_c^{-1} g_c.
__global__ void __launch_bounds__(kBlock) k_coarse_local_lu(HView hv, KappaFam kf, int newton, const double* __restrict__ x,
                                                         const double* __restrict__ r) {
  const CView& v = hv.v;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= v.n) return;
  const int k = v.lfptr[c + 1] - v.lfptr[c];
  const int p0 = v.pptr[c], m = v.pptr[c + 1] - p0;
  const int nc = k + m;
  const int* lf = v.lfidx + v.lfptr[c];
  const double* Mc = v.M + v.mptr[c];
  const double* Dc = v.D + v.dptr[c];
  const double* sig = x;
  const double* p = x + v.nf;
  double pbar = 0.0;
  for (int q = 0; q < m; ++q) pbar += v.w[p0 + q] * p[p0 + q];
  const double ps = kap_psi(v.z, pbar, c);
  const double sc = kap_inv(kf, ps);
  const double dsc = kap_dinv(kf, ps, sc);
  double* A = hv.tmp + hv.invptr[c];
  double* inv = hv.inv + hv.invptr[c];
  for (int i = 0; i < k; ++i) {
    double ms = 0.0;
    if (newton)
      for (int j = 0; j < k; ++j) ms += Mc[i * k + j] * sig[lf[j]];
    for (int j = 0; j < k; ++j) A[i * nc + j] = sc * Mc[i * k + j];
    for (int q = 0; q < m; ++q) A[i * nc + k + q] = Dc[q * k + i] + (newton ? ms * dsc * v.w[p0 + q] : 0.0);
  }
  for (int q = 0; q < m; ++q) {
    for (int j = 0; j < k; ++j) A[(k + q) * nc + j] = Dc[q * k + j];
    for (int j = 0; j < m; ++j) A[(k + q) * nc + k + j] = 0.0;
  }
  int piv[64];
  for (int kk = 0; kk < nc; ++kk) {
    int pr = kk;
    double best = fabs(A[kk * nc + kk]);
    for (int i = kk + 1; i < nc; ++i)
      if (fabs(A[i * nc + kk]) > best) { best = fabs(A[i * nc + kk]); pr = i; }
    piv[kk] = pr;
    if (pr != kk)
      for (int j = 0; j < nc; ++j) { const double t = A[kk * nc + j]; A[kk * nc + j] = A[pr * nc + j]; A[pr * nc + j] = t; }
    const double d = A[kk * nc + kk];
    const double id = d != 0.0 ? 1.0 / d : 0.0;
    for (int i = kk + 1; i < nc; ++i) {
      const double l = A[i * nc + kk] * id;
      A[i * nc + kk] = l;
      for (int j = kk + 1; j < nc; ++j) A[i * nc + j] -= l * A[kk * nc + j];
    }
  }
  for (int col = 0; col < nc; ++col) {
    for (int i = 0; i < nc; ++i) inv[i * nc + col] = (i == col) ? 1.0 : 0.0;
    for (int kk = 0; kk < nc; ++kk)
      if (piv[kk] != kk) {
        const double t = inv[kk * nc + col];
        inv[kk * nc + col] = inv[piv[kk] * nc + col];
        inv[piv[kk] * nc + col] = t;
      }
    for (int i = 0; i < nc; ++i) {
      double s = inv[i * nc + col];
      for (int j = 0; j < i; ++j) s -= A[i * nc + j] * inv[j * nc + col];
      inv[i * nc + col] = s;
    }
    for (int i = nc - 1; i >= 0; --i) {
      double s = inv[i * nc + col];
      for (int j = i + 1; j < nc; ++j) s -= A[i * nc + j] * inv[j * nc + col];
      const double d = A[i * nc + i];
      inv[i * nc + col] = d != 0.0 ? s / d : 0.0;
    }
  }
  // z_c = A_c^{-1} g_c, g = [-r_hat; -r_p]; r_hat keeps r_sigma on the first owner only
  double* z = hv.z + hv.zptr[c];
  for (int i = 0; i < nc; ++i) {
    double s = 0.0;
    for (int j = 0; j < nc; ++j) {
      double g;
      if (j < k) {
        const int fj = lf[j];
        g = (v.fcell[2 * fj] == c) ? -r[fj] : 0.0;
      } else {
        g = -r[v.nf + p0 + (j - k)];
      }
      s += inv[i * nc + j] * g;
    }
    z[i] = s;
  }
}

void launch_coarse_local(CoarseLevel& C, const KappaFam& kf, bool newton, const double* x, const double* r,
                         hipStream_t s) {
  HView hv;
  hv.v = cview(C);
  hv.zptr = C.zptr.p;
  hv.invptr = C.invptr.p;
  hv.lam_of = nullptr;
  hv.inv = C.inv.p;
  hv.tmp = C.t.p;
  hv.z = C.z.p;
  if (C.fast_local) {
    const LocStatic ls{C.gptr.p, C.sgptr.p, C.Minv.p, C.G.p, C.DG.p};
    hipLaunchKernelGGL(k_coarse_local, dim3(grid_for(C.n, kBlock / 64)), dim3(kBlock), 0, s, hv, ls, kf,
                       newton ? 1 : 0, x, r);
  } else {
    hipLaunchKernelGGL(k_coarse_local_lu, dim3(grid_for(C.n, kBlock)), dim3(kBlock), 0, s, hv, kf, newton ? 1 : 0,
                       x, r);
  }
  LAUNCHCHECK();
}

// H_{ll'} = sum_c sgn sgn' X_c[i][i'] (X_c: flux block of A_c^{-1});
// xi_l = z_{c1}[i1] - z_{c2}[i2].  Multiplier l lives on flux l (interfaces
// come first in the canonical flux order).
__global__ void __launch_bounds__(kBlock) k_H_assemble(CView v, const int* __restrict__ zptr, const int* __restrict__ invptr,
                                                       const double* __restrict__ inv, const double* __restrict__ z,
                                                       int nl, const int* __restrict__ Hptr, const int* __restrict__ Hoc,
                                                       const int* __restrict__ Hoi, const int* __restrict__ Hoj,
                                                       const int8_t* __restrict__ Hos, double* __restrict__ Hdiag,
                                                       double* __restrict__ Hoff, double* __restrict__ xi) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nl) return;
  double d = 0.0, x0 = 0.0;
  for (int slot = 0; slot < 2; ++slot) {
    const int c = v.fcell[2 * l + slot];
    if (c < 0) continue;
    const int li = v.floc[2 * l + slot];
    const int nc = (v.lfptr[c + 1] - v.lfptr[c]) + (v.pptr[c + 1] - v.pptr[c]);
    d += inv[invptr[c] + li * nc + li];
    x0 += (slot == 0 ? 1.0 : -1.0) * z[zptr[c] + li];
  }
  Hdiag[l] = d;
  xi[l] = x0;
  for (int e = Hptr[l]; e < Hptr[l + 1]; ++e) {
    const int c = Hoc[e];
    const int nc = (v.lfptr[c + 1] - v.lfptr[c]) + (v.pptr[c + 1] - v.pptr[c]);
    Hoff[e] = (double)Hos[e] * inv[invptr[c] + Hoi[e] * nc + Hoj[e]];
  }
}

void launch_H_assemble(CoarseLevel& C, hipStream_t s) {
  if (C.nl == 0) return;
  hipLaunchKernelGGL(k_H_assemble, dim3(grid_for(C.nl, kBlock)), dim3(kBlock), 0, s, cview(C), C.zptr.p, C.invptr.p,
                     C.inv.p, C.z.p, C.nl, C.Hptr.p, C.Hoc.p, C.Hoi.p, C.Hoj.p, C.Hos.p, C.Hdiag.p, C.Hoff.p, C.xi.p);
  LAUNCHCHECK();
}

// [dsigma_c; dp_c] = z_c - A_c^{-1} [C_c^T lambda; 0]; each flux takes the
// value of its first owner.  One wave per cell, a lane per local row; the
// per-block maximum of |Pi~ dp_c| over the block's cells goes to parts.
constexpr int kBacksubBlock = 1024;

__global__ void __launch_bounds__(kBacksubBlock) k_coarse_backsub(CView v, const int* __restrict__ zptr,
                                                                  const int* __restrict__ invptr,
                                                                  const double* __restrict__ inv,
                                                                  const double* __restrict__ z, int nl,
                                                                  const double* __restrict__ lam,
                                                                  double* __restrict__ dx, double* __restrict__ parts) {
  __shared__ double sh[kBacksubBlock / 64];
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * (kBacksubBlock / 64) + (threadIdx.x >> 6);
  double mx = 0.0;
  if (c < v.n) {
    const int k = v.lfptr[c + 1] - v.lfptr[c];
    const int p0 = v.pptr[c], m = v.pptr[c + 1] - p0;
    const int nc = k + m;
    const int* lf = v.lfidx + v.lfptr[c];
    double pbv = 0.0;
    if (lane < nc) {
      const double* Ai = inv + invptr[c] + lane * nc;
      double s = z[zptr[c] + lane];
      for (int j = 0; j < k; ++j) {
        const int fj = lf[j];
        if (fj < nl) s -= Ai[j] * ((v.fcell[2 * fj] == c) ? lam[fj] : -lam[fj]);
      }
      if (lane < k) {
        if (v.fcell[2 * lf[lane]] == c) dx[lf[lane]] = s;
      } else {
        dx[v.nf + p0 + (lane - k)] = s;
        pbv = v.w[p0 + (lane - k)] * s;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) pbv += __shfl_xor(pbv, o, 64);
    mx = pbv == pbv ? fabs(pbv) : HUGE_VAL;   // a NaN counts as non-finite (fmax would drop it)
  }
  mx = block_max(mx, sh);
  if (threadIdx.x == 0) parts[blockIdx.x] = mx;
}

int launch_coarse_backsub(CoarseLevel& C, const double* lam, double* dx, double* parts, hipStream_t s) {
  const unsigned G = grid_for(C.n, kBacksubBlock / 64);
  require(G <= (unsigned)kMaxParts * 4, "too many coarse cells for one reduction");
  hipLaunchKernelGGL(k_coarse_backsub, dim3(G), dim3(kBacksubBlock), 0, s, cview(C), C.zptr.p, C.invptr.p, C.inv.p,
                     C.z.p, C.nl, lam, dx, parts);
  LAUNCHCHECK();
  return (int)G;
}

// ------------------------------------------------------------------ divergence

__global__ void __launch_bounds__(kBlock) k_div_coarse(CView v, const double* __restrict__ sig, double* __restrict__ div) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= v.n) return;
  const int k = v.lfptr[c + 1] - v.lfptr[c];
  const int p0 = v.pptr[c], m = v.pptr[c + 1] - p0;
  const int* lf = v.lfidx + v.lfptr[c];
  for (int q = 0; q < m; ++q) {
    double acc = 0.0;
    for (int i = 0; i < k; ++i) acc += v.D[v.dptr[c] + q * k + i] * sig[lf[i]];
    div[p0 + q] = acc;
  }
}

__global__ void __launch_bounds__(kBlock) k_div_fine(int64_t n, const int* __restrict__ cfptr, const int* __restrict__ cfcode,
                                                     const double* __restrict__ sig, double* __restrict__ div) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double acc = 0.0;
  for (int k = cfptr[c]; k < cfptr[c + 1]; ++k) {
    const int code = cfcode[k];
    acc += (code & 1) ? sig[code >> 1] : -sig[code >> 1];
  }
  div[c] = acc;
}

void launch_div_coarse(const CoarseLevel& C, const double* sigma, double* div, hipStream_t s) {
  hipLaunchKernelGGL(k_div_coarse, dim3(grid_for(C.n, kBlock)), dim3(kBlock), 0, s, cview(C), sigma, div);
  LAUNCHCHECK();
}

void launch_div_fine(int64_t n, const int* cfptr, const int* cfcode, const double* sigma, double* div,
                     hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_div_fine, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, n, cfptr, cfcode, sigma, div);
  LAUNCHCHECK();
}

// ------------------------------------------------------------------ transfers

struct TView {
  int n_agg, nf_f, np_f, nf_c, n_int_total;
  const int *pd_ptr, *pd_list, *dof_ptr, *dof_list, *n_int, *mA, *fgrp_ptr, *fgrp_list, *Pptr, *Eptr;
  const int *pd_agg, *pd_row, *int_agg, *int_row, *int_pos, *grp_of, *bub0;
  const double *P, *E, *trace, *omega;
  // coarse
  const int *pptr, *lfptr, *lfidx, *fcell, *floc;
  const int8_t* kind;
};

static TView tview(const TransferDev& T, const CoarseLevel& C) {
  TView t;
  t.n_agg = T.n_agg; t.nf_f = T.nf_fine; t.np_f = T.np_fine; t.nf_c = C.nf; t.n_int_total = T.n_int_total;
  t.pd_ptr = T.pd_ptr.p; t.pd_list = T.pd_list.p; t.dof_ptr = T.dof_ptr.p; t.dof_list = T.dof_list.p;
  t.n_int = T.n_int.p; t.mA = T.mA.p; t.fgrp_ptr = T.fgrp_ptr.p; t.fgrp_list = T.fgrp_list.p; t.Pptr = T.Pptr.p;
  t.Eptr = T.Eptr.p; t.pd_agg = T.pd_agg.p; t.pd_row = T.pd_row.p; t.int_agg = T.int_agg.p; t.int_row = T.int_row.p;
  t.int_pos = T.int_pos.p; t.grp_of = T.grp_of.p; t.bub0 = T.bub0.p; t.P = T.P.p; t.E = T.E.p; t.trace = T.trace.p;
  t.omega = T.omega.p; t.pptr = C.pptr.p; t.lfptr = C.lfptr.p; t.lfidx = C.lfidx.p; t.fcell = C.fcell.p;
  t.floc = C.floc.p; t.kind = C.kind.p;
  return t;
}

// out = P^T in (R), or out = Q in (Q: flux moments on interfaces, divergence
// moments of the NPV columns on bubbles) -- items: coarse flux unknowns, then
// aggregates (pressure coefficients).  One wave per item: the lanes split the
// item's sums (fine fluxes of the group, interior dofs of the adjacent
// aggregates, cells of the aggregate) and a fixed-order wave reduction
// combines them.
__device__ inline double wave_allsum_t(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <bool PROJECT>
__global__ void __launch_bounds__(kBlock) k_restrict_t(TView t, const double* __restrict__ in, const double* __restrict__ divf,
                                                       double* __restrict__ out) {
  const int it = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (it >= t.nf_c + t.n_agg) return;   // whole wave
  const double* in_s = in;
  const double* in_p = in + t.nf_f;
  if (it < t.nf_c) {
    const int J = it;
    double acc = 0.0;
    if (t.kind[J] != 2)
      for (int q = t.fgrp_ptr[J] + lane; q < t.fgrp_ptr[J + 1]; q += 64) {
        const int g = t.fgrp_list[q];
        acc += (PROJECT ? t.omega[g] : t.trace[g]) * in_s[g];
      }
    if (!PROJECT) {
      for (int slot = 0; slot < 2; ++slot) {
        const int A = t.fcell[2 * J + slot];
        if (A < 0) continue;
        const int loc = t.floc[2 * J + slot];
        const int kA = t.lfptr[A + 1] - t.lfptr[A];
        const double* EA = t.E + t.Eptr[A];
        const int* dl = t.dof_list + t.dof_ptr[A];
        const int nI = t.n_int[A];
        for (int q = lane; q < nI; q += 64) acc += EA[q * kA + loc] * in_s[dl[q]];
      }
    } else if (t.kind[J] == 2) {
      const int A = t.fcell[2 * J];
      const int j = 1 + (J - t.bub0[A]);
      const int mA = t.mA[A];
      const double* PA = t.P + t.Pptr[A];
      const int* pl = t.pd_list + t.pd_ptr[A];
      const int npA = t.pd_ptr[A + 1] - t.pd_ptr[A];
      for (int r = lane; r < npA; r += 64) acc += PA[r * mA + j] * divf[pl[r]];
    }
    acc = wave_allsum_t(acc);
    if (lane == 0) out[J] = acc;
  } else {
    const int A = it - t.nf_c;
    const int mA = t.mA[A];
    const double* PA = t.P + t.Pptr[A];
    const int* pl = t.pd_list + t.pd_ptr[A];
    const int npA = t.pd_ptr[A + 1] - t.pd_ptr[A];
    for (int i = 0; i < mA; ++i) {
      double acc = 0.0;
      for (int r = lane; r < npA; r += 64) acc += PA[r * mA + i] * in_p[pl[r]];
      acc = wave_allsum_t(acc);
      if (lane == 0) out[t.nf_c + t.pptr[A] + i] = acc;
    }
  }
}

// out[A] = sum over the level-l cells c of A of vol_l[c] z_l[c], over vol_c[A]
// (the cells in the plan's list order, a thread per aggregate)
__global__ void k_volume_mean(int n_agg, const int* __restrict__ cell_ptr, const int* __restrict__ cell_list,
                              const double* __restrict__ vol_l, const double* __restrict__ z_l,
                              const double* __restrict__ vol_c, double* __restrict__ out) {
  const int A = blockIdx.x * blockDim.x + threadIdx.x;
  if (A >= n_agg) return;
  double acc = 0.0;
  for (int i = cell_ptr[A]; i < cell_ptr[A + 1]; ++i) {
    const int c = cell_list[i];
    acc = fma(vol_l[c], z_l[c], acc);
  }
  out[A] = acc / vol_c[A];
}

void launch_volume_mean(const TransferDev& T, const double* vol_l, const double* z_l, const double* vol_c,
                        double* out, hipStream_t s) {
  if (T.n_agg == 0) return;
  hipLaunchKernelGGL(k_volume_mean, dim3(grid_for(T.n_agg, kBlock)), dim3(kBlock), 0, s, T.n_agg, T.cell_ptr.p,
                     T.cell_list.p, vol_l, z_l, vol_c, out);
  LAUNCHCHECK();
}

void launch_restrict(const TransferDev& T, const CoarseLevel& Cc, const double* rf, double* out, hipStream_t s) {
  TView t = tview(T, Cc);
  hipLaunchKernelGGL(k_restrict_t<false>, dim3(grid_for(t.nf_c + t.n_agg, kBlock / 64)), dim3(kBlock), 0, s, t, rf,
                     (const double*)nullptr, out);
  LAUNCHCHECK();
}

void launch_project(const TransferDev& T, const CoarseLevel& Cc, const double* xf, const double* divf, double* out,
                    hipStream_t s) {
  TView t = tview(T, Cc);
  hipLaunchKernelGGL(k_restrict_t<true>, dim3(grid_for(t.nf_c + t.n_agg, kBlock / 64)), dim3(kBlock), 0, s, t, xf,
                     divf, out);
  LAUNCHCHECK();
}

// outf = P e: items = pressure unknowns of the aggregates, interior flux
// rows, then every fine flux of an interface/Dirichlet group.
__global__ void __launch_bounds__(kBlock) k_prolong_t(TView t, const double* __restrict__ e, double* __restrict__ outf) {
  const int npl = t.pd_ptr[t.n_agg];
  const int ntot = npl + t.n_int_total + t.nf_f;
  const double* e_s = e;
  const double* e_p = e + t.nf_c;
  double* o_s = outf;
  double* o_p = outf + t.nf_f;
  for (int it = blockIdx.x * blockDim.x + threadIdx.x; it < ntot; it += gridDim.x * blockDim.x) {
    if (it < npl) {
      const int A = t.pd_agg[it], row = t.pd_row[it];
      const int mA = t.mA[A];
      const double* PA = t.P + t.Pptr[A] + row * mA;
      double acc = 0.0;
      for (int i = 0; i < mA; ++i) acc += PA[i] * e_p[t.pptr[A] + i];
      o_p[t.pd_list[it]] = acc;
    } else if (it < npl + t.n_int_total) {
      const int q = it - npl;
      const int A = t.int_agg[q], row = t.int_row[q];
      const int kA = t.lfptr[A + 1] - t.lfptr[A];
      const double* EA = t.E + t.Eptr[A] + row * kA;
      const int* lf = t.lfidx + t.lfptr[A];
      double acc = 0.0;
      for (int k = 0; k < kA; ++k) acc += EA[k] * e_s[lf[k]];
      o_s[t.dof_list[t.int_pos[q]]] = acc;
    } else {
      const int j = it - npl - t.n_int_total;
      const int J = t.grp_of[j];
      if (J >= 0) o_s[j] = t.trace[j] * e_s[J];
    }
  }
}

void launch_prolong(const TransferDev& T, const CoarseLevel& Cc, const double* e, double* outf, hipStream_t s) {
  TView t = tview(T, Cc);
  const int64_t ntot = (int64_t)T.h_pd_ptr.back() + T.n_int_total + T.nf_fine;
  hipLaunchKernelGGL(k_prolong_t, dim3(grid_for(ntot, kBlock)), dim3(kBlock), 0, s, t, e, outf);
  LAUNCHCHECK();
}

// ------------------------------------------------------------------ solver setup

void setup_coarse_solver(Hierarchy& h, int l) {
  hipStream_t s = h.stream;
  CoarseLevel& C = *h.coarse[l - 1];
  const int n = C.n, nf = C.nf, np = C.np;
  C.x.alloc(nf + np);
  C.dx.alloc(nf + np);
  C.b.alloc(nf + np);
  C.r.alloc(nf + np);
  C.div.alloc(np);
  C.x0.alloc(nf + np);
  C.ax.alloc(nf + np);
  C.zeros.alloc(nf + np);
  C.zeros.zero(s);
  // offsets of local systems
  std::vector<int> zptr(n + 1, 0), invptr(n + 1, 0);
  int mxn = 0;
  for (int c = 0; c < n; ++c) {
    const int nc = (C.h_lfptr[c + 1] - C.h_lfptr[c]) + (C.h_pptr[c + 1] - C.h_pptr[c]);
    mxn = std::max(mxn, nc);
    zptr[c + 1] = zptr[c] + nc;
    invptr[c + 1] = invptr[c] + nc * nc;
  }
  require(mxn <= 64, "coarse cell with more than 64 local unknowns");
  // static parts of the block elimination (cells with at most kLocM pressure unknowns)
  {
    std::vector<int> gptr(n + 1, 0), sgptr(n + 1, 0);
    int mxm = 0;
    for (int c = 0; c < n; ++c) {
      const int k = C.h_lfptr[c + 1] - C.h_lfptr[c], m = C.h_pptr[c + 1] - C.h_pptr[c];
      mxm = std::max(mxm, m);
      gptr[c + 1] = gptr[c] + k * m;
      sgptr[c + 1] = sgptr[c] + m * m;
    }
    C.fast_local = false;
    if (mxm <= kLocM && n > 0) {
      C.gptr.upload(gptr, s);
      C.sgptr.upload(sgptr, s);
      C.Minv.alloc(C.M.n);
      C.G.alloc(std::max(gptr[n], 1));
      C.DG.alloc(std::max(sgptr[n], 1));
      DVec<int> flag;
      flag.alloc(1);
      flag.zero(s);
      const LocStatic ls{C.gptr.p, C.sgptr.p, C.Minv.p, C.G.p, C.DG.p};
      hipLaunchKernelGGL(k_local_static, dim3(n), dim3(64), 0, s, cview(C), ls, C.Minv.p, C.G.p, C.DG.p, flag.p);
      LAUNCHCHECK();
      C.fast_local = flag.download(s)[0] == 0;   // otherwise LU of the whole local block
    }
  }
  C.nsum = zptr[n];
  C.zptr.upload(zptr, s);
  C.invptr.upload(invptr, s);
  C.inv.alloc(invptr[n]);
  C.t.alloc(std::max(invptr[n], nf + np));
  C.z.alloc(zptr[n]);
  // multipliers: the interior interfaces, which come first
  int nl = 0;
  while (nl < nf && C.h_kind[nl] == FK_INTERIOR) ++nl;
  C.nl = nl;
  std::vector<int> fcell(2 * nf), floc(2 * nf);
  {
    std::vector<int> a = C.fcell.download(s), b = C.floc.download(s);
    fcell = a;
    floc = b;
  }
  std::vector<int> Hptr(nl + 1, 0), Hcol, Hoc, Hoi, Hoj;
  std::vector<int8_t> Hos;
  for (int L = 0; L < nl; ++L) {
    std::vector<std::tuple<int, int, int, int, int>> ent;   // (col, cell, li, lj, sign)
    for (int slot = 0; slot < 2; ++slot) {
      const int c = fcell[2 * L + slot];
      if (c < 0) continue;
      const int li = floc[2 * L + slot];
      const int sgi = slot == 0 ? 1 : -1;
      for (int q = C.h_lfptr[c]; q < C.h_lfptr[c + 1]; ++q) {
        const int J = C.h_lfidx[q];
        if (J == L || J >= nl) continue;
        const int lj = q - C.h_lfptr[c];
        const int sgj = (fcell[2 * J] == c) ? 1 : -1;
        ent.emplace_back(J, c, li, lj, sgi * sgj);
      }
    }
    std::sort(ent.begin(), ent.end());
    for (auto& e : ent) {
      Hcol.push_back(std::get<0>(e));
      Hoc.push_back(std::get<1>(e));
      Hoi.push_back(std::get<2>(e));
      Hoj.push_back(std::get<3>(e));
      Hos.push_back((int8_t)std::get<4>(e));
    }
    Hptr[L + 1] = (int)Hcol.size();
  }
  C.Hptr.upload(Hptr, s);
  C.Hcol.upload(Hcol, s);
  C.Hoc.upload(Hoc, s);
  C.Hoi.upload(Hoi, s);
  C.Hoj.upload(Hoj, s);
  C.Hos.upload(Hos, s);
  C.Hdiag.alloc(nl);
  C.Hoff.alloc(Hcol.size());
  C.xi.alloc(nl);
  C.lam.alloc(nl);
  C.H.n = nl;
  C.H.diag = C.Hdiag.p;
  C.H.ptr = C.Hptr.p;
  C.H.col = C.Hcol.p;
  C.H.val = C.Hoff.p;
  if (nl > 0) {
    // aggregation matrix: Picard at x = 0 (kappa = 1)
    C.x.zero(s);
    C.r.zero(s);
    launch_coarse_local(C, KappaFam{}, false, C.x.p, C.r.p, s);   // exp(0 psi) = 1
    launch_H_assemble(C, s);
    HIPCHECK(hipStreamSynchronize(s));
    C.amg.setup(C.H, s);
    if (trace_level() > 0)
      std::fprintf(stderr, "[spfas] hybridised system of level %d AMG: %s\n", l, C.amg.describe().c_str());
  }
}

}  // namespace spfas
