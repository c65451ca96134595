// Fine-level (level 0) kernels: half-transmissibilities, the mixed TPFA
// residual, the Picard/Newton linearisation with exact elimination of the
// (diagonal) flux block, and the flux back-substitution.
//
// Layout (renumbered order: cells contiguous per aggregate, faces grouped
// inside-aggregate / per interface / Dirichlet):
//   state x = [sigma (nf) | p (n)], contiguous FP64
//   faces:  K[j], L[j] (L = -1 on a Dirichlet face), TKi[j] = 1/Tb_K,
//           TLi[j] = 1/Tb_L (0 on Dirichlet faces), g[j] (g_D or 0)
//   cells:  f[c] (|tau| f + Neumann inflow), cell->face list cfptr/cfcode
//           with code = (face << 1) | side, side 0: cell is K (D = -1),
//           side 1: cell is L (D = +1); nb[k] = cell across that face
//           (the cell itself on a Dirichlet face).
#include "fine.hpp"
#include "kappa.hpp"

#include <type_traits>

#include "kern.hpp"

namespace spfas {

// ------------------------------------------------------------------ setup

// Tb_{i,eps} = |eps| n_i . K0_i . (x_eps - x_i) / ||x_eps - x_i||^2 with
// n_K = n_eps, n_L = -n_eps (eq. half-transmissibility).  Input order.
__global__ void k_halftrans(int64_t nf, int dim, const int* __restrict__ fc, const double* __restrict__ area,
                            const double* __restrict__ nrm, const double* __restrict__ pt,
                            const double* __restrict__ cen, const double* __restrict__ k0,
                            double* __restrict__ TK, double* __restrict__ TL, int* __restrict__ bad) {
  int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int nbad = 0;
  for (int side = 0; side < 2; ++side) {
    const int c = fc[2 * f + side];
    if (c < 0) {
      if (side == 1) TL[f] = 0.0;
      continue;
    }
    const double sg = side == 0 ? 1.0 : -1.0;
    double d[3], kd[3];
    double dd = 0.0;
    for (int a = 0; a < dim; ++a) {
      d[a] = pt[f * dim + a] - cen[(int64_t)c * dim + a];
      dd += d[a] * d[a];
    }
    double num = 0.0;
    for (int a = 0; a < dim; ++a) {
      kd[a] = 0.0;
      for (int b = 0; b < dim; ++b) kd[a] += k0[((int64_t)c * dim + a) * dim + b] * d[b];
      num += sg * nrm[f * dim + a] * kd[a];
    }
    const double t = area[f] * num / dd;
    if (!(t > 0.0) || !(dd > 0.0)) nbad++;
    if (side == 0) TK[f] = t; else TL[f] = t;
  }
  if (nbad) atomicAdd(bad, nbad);
}

void launch_halftrans(int64_t nf, int dim, const int* fc, const double* area, const double* nrm,
                      const double* pt, const double* cen, const double* k0, double* TK, double* TL,
                      int* bad, hipStream_t s) {
  if (nf == 0) return;
  hipLaunchKernelGGL(k_halftrans, dim3(grid_for(nf, kBlock)), dim3(kBlock), 0, s, nf, dim, fc, area, nrm, pt,
                     cen, k0, TK, TL, bad);
  LAUNCHCHECK();
}

// ------------------------------------------------------------------ residual

// r(x + s dx) = A(x + s dx) - b with b = -[g; f] (eqs. fine_level_residual,
// FV_matrix); items [0, nf) are faces (flux rows), [nf, nf+n) cells
// (mass-balance rows).  The row values come from the two routines below,
// shared by the single-step and the multi-step kernels (multiply-adds as
// explicit fma) so that a trial step gives the same bits in both.
// 1/kappa at a cell value p and its derivative: with GK false the
// exponential family without shift, exp(-alpha p) as written; otherwise
// the general family of KappaFam at p - z_c.
template <bool GK>
__device__ inline double fine_kinv(const FineView& v, double p, int c) {
  if constexpr (GK) return kap_inv(v.kf, kap_psi(v.z, p, c));
  else return exp(-v.kf.alpha * p);
}
template <bool GK>
__device__ inline double fine_dkinv(const FineView& v, double p, int c, double kinv) {
  if constexpr (GK) return kap_dinv(v.kf, kap_psi(v.z, p, c), kinv);
  else return -v.kf.alpha * kinv;
}

// kernels instantiated for the general kappa family when the problem is not
// the exponential without shift
inline bool general_kappa(const FineView& v) { return v.kf.kind != 0 || v.z != nullptr; }

template <bool GK>
__device__ inline double flux_row(const FineView& v, int64_t i, double pK, double pL, double sj) {
  const int L = v.L[i];
  double m = fine_kinv<GK>(v, pK, GK ? v.K[i] : 0) * v.TKi[i];
  double dtp = -pK;
  if (L >= 0) {
    m = fma(fine_kinv<GK>(v, pL, L), v.TLi[i], m);
    dtp += pL;
  }
  return fma(m, sj, dtp) + v.g[i];
}

// x + s dx component: explicit fma, the same in every kernel
__device__ inline double stepped(double a, double s, double d) { return fma(s, d, a); }

// Writes r if `r` is non-null and the per-block sum of squares to
// parts[blockIdx.x].
template <bool STEP, bool GK>
__global__ void __launch_bounds__(kBlock) k_fine_resid(FineView v, const double* __restrict__ x,
                                                       const double* __restrict__ dx, double s,
                                                       double* __restrict__ r, double* __restrict__ parts) {
  __shared__ double sh[kBlock / 64];
  const int64_t nf = v.nf, ntot = v.nf + v.n;
  const double* sig = x;
  const double* p = x + nf;
  const double* dsig = dx;
  const double* dp = dx + nf;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ntot; i += (int64_t)gridDim.x * blockDim.x) {
    double ri;
    if (i < nf) {
      const int K = v.K[i], L = v.L[i];
      double pK = p[K], pL = L >= 0 ? p[L] : 0.0, sj = sig[i];
      if (STEP) {
        pK = stepped(pK, s, dp[K]);
        if (L >= 0) pL = stepped(pL, s, dp[L]);
        sj = stepped(sj, s, dsig[i]);
      }
      ri = flux_row<GK>(v, i, pK, pL, sj);
    } else {
      const int64_t c = i - nf;
      double div = 0.0;
      for (int k = v.cfptr[c]; k < v.cfptr[c + 1]; ++k) {
        const int code = v.cfcode[k];
        const int j = code >> 1;
        double sj = sig[j];
        if (STEP) sj = stepped(sj, s, dsig[j]);
        div += (code & 1) ? sj : -sj;
      }
      ri = div + v.f[c];
    }
    if (r) r[i] = ri;
    acc = fma(ri, ri, acc);
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) parts[blockIdx.x] = acc;
}

// The same sums of squares at NT step lengths in one pass over the data
// (the remaining trials of Alg. 1): parts[t * gridDim.x + block].
struct TrialSteps {
  double s[kMaxTrials];
};

template <int NT, bool GK>
__global__ void __launch_bounds__(kBlock) k_fine_resid_trials(FineView v, const double* __restrict__ x,
                                                              const double* __restrict__ dx, TrialSteps st,
                                                              double* __restrict__ parts) {
  __shared__ double sh[kBlock / 64];
  const int64_t nf = v.nf, ntot = v.nf + v.n;
  const double* sig = x;
  const double* p = x + nf;
  const double* dsig = dx;
  const double* dp = dx + nf;
  double acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ntot; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < nf) {
      const int K = v.K[i], L = v.L[i];
      const double pK0 = p[K], dK = dp[K], sj0 = sig[i], ds = dsig[i];
      const double pL0 = L >= 0 ? p[L] : 0.0, dL = L >= 0 ? dp[L] : 0.0;
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const double pL = L >= 0 ? stepped(pL0, st.s[t], dL) : 0.0;
        const double ri = flux_row<GK>(v, i, stepped(pK0, st.s[t], dK), pL, stepped(sj0, st.s[t], ds));
        acc[t] = fma(ri, ri, acc[t]);
      }
    } else {
      const int64_t c = i - nf;
      double div[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) div[t] = 0.0;
      for (int k = v.cfptr[c]; k < v.cfptr[c + 1]; ++k) {
        const int code = v.cfcode[k];
        const int j = code >> 1;
        const double s0 = sig[j], d0 = dsig[j];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const double sj = stepped(s0, st.s[t], d0);
          div[t] += (code & 1) ? sj : -sj;
        }
      }
      const double fc = v.f[c];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const double ri = div[t] + fc;
        acc[t] = fma(ri, ri, acc[t]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const double a = block_sum(acc[t], sh);
    if (threadIdx.x == 0) parts[(int64_t)t * gridDim.x + blockIdx.x] = a;
  }
}

int launch_fine_resid_trials(const FineView& v, const double* x, const double* dx, const double* steps, int nt,
                             double* parts, hipStream_t st) {
  require(nt >= 1 && nt <= kMaxTrials, "number of trial steps out of range");
  const int G = reduce_grid(v.nf + v.n);
  TrialSteps ts{};
  for (int t = 0; t < nt; ++t) ts.s[t] = steps[t];
  if (general_kappa(v)) {
    switch (nt) {
      case 1: hipLaunchKernelGGL((k_fine_resid_trials<1, true>), dim3(G), dim3(kBlock), 0, st, v, x, dx, ts, parts); break;
      case 2: hipLaunchKernelGGL((k_fine_resid_trials<2, true>), dim3(G), dim3(kBlock), 0, st, v, x, dx, ts, parts); break;
      case 3: hipLaunchKernelGGL((k_fine_resid_trials<3, true>), dim3(G), dim3(kBlock), 0, st, v, x, dx, ts, parts); break;
      default: hipLaunchKernelGGL((k_fine_resid_trials<4, true>), dim3(G), dim3(kBlock), 0, st, v, x, dx, ts, parts); break;
    }
  } else {
    switch (nt) {
      case 1: hipLaunchKernelGGL((k_fine_resid_trials<1, false>), dim3(G), dim3(kBlock), 0, st, v, x, dx, ts, parts); break;
      case 2: hipLaunchKernelGGL((k_fine_resid_trials<2, false>), dim3(G), dim3(kBlock), 0, st, v, x, dx, ts, parts); break;
      case 3: hipLaunchKernelGGL((k_fine_resid_trials<3, false>), dim3(G), dim3(kBlock), 0, st, v, x, dx, ts, parts); break;
      default: hipLaunchKernelGGL((k_fine_resid_trials<4, false>), dim3(G), dim3(kBlock), 0, st, v, x, dx, ts, parts); break;
    }
  }
  LAUNCHCHECK();
  return G;
}

int launch_fine_resid(const FineView& v, const double* x, const double* dx, double s, double* r, double* parts,
                      hipStream_t st) {
  const int G = reduce_grid(v.nf + v.n);
  const bool gk = general_kappa(v);
  if (dx && gk)
    hipLaunchKernelGGL((k_fine_resid<true, true>), dim3(G), dim3(kBlock), 0, st, v, x, dx, s, r, parts);
  else if (dx)
    hipLaunchKernelGGL((k_fine_resid<true, false>), dim3(G), dim3(kBlock), 0, st, v, x, dx, s, r, parts);
  else if (gk)
    hipLaunchKernelGGL((k_fine_resid<false, true>), dim3(G), dim3(kBlock), 0, st, v, x, dx, s, r, parts);
  else
    hipLaunchKernelGGL((k_fine_resid<false, false>), dim3(G), dim3(kBlock), 0, st, v, x, dx, s, r, parts);
  LAUNCHCHECK();
  return G;
}

// ------------------------------------------------------------------ linearisation

// Linearisation (Section 3.3) with the flux block eliminated (M is diagonal
// on level 0): S = D M^{-1} E (Picard: E = D^T; Newton:
// E = N(sigma) kinv'(p) + D^T, Prop. 3 on level 0) and rhs = r_p -
// D M^{-1} r_sigma of the eliminated system S dp = rhs.  With m_j the diagonal of M on face j, E_K
// and E_L the entries of E on its cells and r_j its flux residual, the face
// contributes u_K = E_K / m_j, u_L = E_L / m_j and v = sigma_j - r_j / m_j
// with the orientation d = -1 (cell K) or +1 (cell L): diag += d u_own,
// off = d u_other, rhs += d v.
// One pass over the cells, a group of kLinG lanes per cell, each lane
// taking every kLinG-th incidence (4 lanes measured 15 % faster than one
// lane per incidence with 8): each lane evaluates the coefficients of a face
// (a face's m, E_K, E_L and r are computed by both of its cells instead of
// being stored and gathered back) and writes its entry of the cell's row
// of S straight into the layout the Krylov products read: the SELL-64 slots
// of the level-0 matrix (diagonal in entry 0, the incidences in list order
// in entries 1, 2, ...), or the DIA+CSR arrays when there is no SELL copy.
// The diagonal and the right-hand side are group sums (fixed order).
constexpr int kLinG = 4;

// TV: storage of the SELL values and of the right-hand side (FP64, or FP32
// in mixed precision); everything is computed in FP64.
template <bool NEWTON, bool SELL, class TV, bool GK>
__global__ void __launch_bounds__(kBlock) k_fine_lin_cells(FineView v, const double* __restrict__ x,
                                                           const int* __restrict__ sptr, double* __restrict__ diag,
                                                           double* __restrict__ off, TV* __restrict__ sval,
                                                           TV* __restrict__ rhs, double* __restrict__ sval64,
                                                           double* __restrict__ rhs64) {
  // FP32 values also go out in FP64 (the refinement residual of mixed precision)
  constexpr bool DUAL = std::is_same_v<TV, float>;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = t / kLinG;
  const int g = (int)(t % kLinG);
  if (c >= v.n) return;   // the whole group leaves together
  const double* sig = x;
  const double* p = x + v.nf;
  const int k0 = v.cfptr[c], k1 = v.cfptr[c + 1];
  TV* row = nullptr;
  double* row64 = nullptr;
  if constexpr (SELL) row = sval + sptr[c >> 6] + (c & 63);   // slot k of the row: row[64 k]
  if constexpr (SELL && DUAL) row64 = sval64 + sptr[c >> 6] + (c & 63);
  double dg = 0.0, rh = 0.0, so = 0.0;   // so: sum of the off-diagonal entries (FP32 row-sum form)
  for (int k = k0 + g; k < k1; k += kLinG) {
    const int code = v.cfcode[k];
    const int j = code >> 1;
    const int K = v.K[j], L = v.L[j];
    const double pK = p[K];
    const double iK = fine_kinv<GK>(v, pK, K);
    const double eK = iK * v.TKi[j];
    double eL = 0.0, pL = 0.0, iL = 0.0;
    if (L >= 0) {
      pL = p[L];
      iL = fine_kinv<GK>(v, pL, L);
      eL = iL * v.TLi[j];
    }
    const double m = eK + eL;
    const double sj = sig[j];
    const double rs = m * sj + (L >= 0 ? pL : 0.0) - pK + v.g[j];
    double EK = -1.0, EL = 1.0;
    if (NEWTON) {   // d r_sigma / d p_K = d(1/kappa_K)/dp Tbar_K^{-1} sigma - 1 (Prop. 3 on level 0)
      EK += fine_dkinv<GK>(v, pK, K, iK) * v.TKi[j] * sj;
      if (L >= 0) EL += fine_dkinv<GK>(v, pL, L, iL) * v.TLi[j] * sj;
    }
    const double ainv = 1.0 / m;
    const double uk = ainv * EK, ul = ainv * EL, vs = sj - ainv * rs;
    double o;
    if (code & 1) {   // this cell is L
      dg += ul;
      o = uk;
      rh += vs;
    } else {          // this cell is K
      dg -= uk;
      o = L >= 0 ? -ul : 0.0;
      rh -= vs;
    }
    if constexpr (SELL) {
      row[(size_t)(1 + k - k0) << 6] = (TV)o;
      if constexpr (DUAL) {
        row64[(size_t)(1 + k - k0) << 6] = o;
        so += o;
      }
    } else {
      off[k] = o;
    }
  }
#pragma unroll
  for (int o = kLinG / 2; o > 0; o >>= 1) {
    dg += __shfl_xor(dg, o, kLinG);
    rh += __shfl_xor(rh, o, kLinG);
    if constexpr (SELL && DUAL) so += __shfl_xor(so, o, kLinG);
  }
  if (g == 0) {
    if constexpr (SELL && DUAL) {   // FP32 rows keep the row sum in slot 0 (Sell32View)
      row[0] = (TV)(dg + so);
      row64[0] = dg;
    } else if constexpr (SELL) {
      row[0] = (TV)dg;
    } else {
      diag[c] = dg;
    }
    const double b = v.f[c] + rh;
    rhs[c] = (TV)b;
    if constexpr (DUAL) rhs64[c] = b;
  }
}

template <class TV, bool GK>
static void lin_cells_launch(const FineView& v, bool newton, const double* x, const int* sell_ptr, TV* sell_val,
                             double* diag, double* off, TV* rhs, double* sell64, double* rhs64, hipStream_t s) {
  const dim3 g(grid_for((size_t)v.n * kLinG, kBlock)), b(kBlock);
  if (sell_ptr) {
    if (newton)
      hipLaunchKernelGGL((k_fine_lin_cells<true, true, TV, GK>), g, b, 0, s, v, x, sell_ptr, nullptr, nullptr,
                         sell_val, rhs, sell64, rhs64);
    else
      hipLaunchKernelGGL((k_fine_lin_cells<false, true, TV, GK>), g, b, 0, s, v, x, sell_ptr, nullptr, nullptr,
                         sell_val, rhs, sell64, rhs64);
  } else {
    if (newton)
      hipLaunchKernelGGL((k_fine_lin_cells<true, false, TV, GK>), g, b, 0, s, v, x, nullptr, diag, off, nullptr, rhs,
                         nullptr, rhs64);
    else
      hipLaunchKernelGGL((k_fine_lin_cells<false, false, TV, GK>), g, b, 0, s, v, x, nullptr, diag, off, nullptr,
                         rhs, nullptr, rhs64);
  }
  LAUNCHCHECK();
}

template <class TV>
static void lin_cells(const FineView& v, bool newton, const double* x, const int* sell_ptr, TV* sell_val,
                      double* diag, double* off, TV* rhs, double* sell64, double* rhs64, hipStream_t s) {
  if (v.n == 0) return;
  if (general_kappa(v)) lin_cells_launch<TV, true>(v, newton, x, sell_ptr, sell_val, diag, off, rhs, sell64, rhs64, s);
  else lin_cells_launch<TV, false>(v, newton, x, sell_ptr, sell_val, diag, off, rhs, sell64, rhs64, s);
}

void launch_fine_linearize_cells(const FineView& v, bool newton, const double* x, const int* sell_ptr,
                                 double* sell_val, double* diag, double* off, double* rhs, hipStream_t s) {
  lin_cells<double>(v, newton, x, sell_ptr, sell_val, diag, off, rhs, nullptr, nullptr, s);
}

void launch_fine_linearize_cells(const FineView& v, bool newton, const double* x, const int* sell_ptr,
                                 float* sell_val, double* sell_val64, double* diag, double* off, float* rhs,
                                 double* rhs64, hipStream_t s) {
  require(rhs64 && (!sell_ptr || sell_val64), "mixed linearisation without its FP64 outputs");
  lin_cells<float>(v, newton, x, sell_ptr, sell_val, diag, off, rhs, sell_val64, rhs64, s);
}

template <bool ADD>
__global__ void __launch_bounds__(kBlock) k_widen(int64_t n, const float* __restrict__ a, double* __restrict__ b) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (ADD) b[i] += (double)a[i];
    else b[i] = (double)a[i];
  }
}

void launch_widen(int64_t n, const float* a, double* b, hipStream_t s, bool add) {
  if (!n) return;
  if (add) hipLaunchKernelGGL(k_widen<true>, dim3(reduce_grid(n)), dim3(kBlock), 0, s, n, a, b);
  else hipLaunchKernelGGL(k_widen<false>, dim3(reduce_grid(n)), dim3(kBlock), 0, s, n, a, b);
  LAUNCHCHECK();
}

// dsigma = -M^{-1} (r_sigma + E dp) on faces; per-block max |dp| on cells.
template <bool NEWTON, bool GK>
__global__ void __launch_bounds__(kBlock) k_fine_backsub(FineView v, const double* __restrict__ x,
                                                         double* __restrict__ dx, double* __restrict__ parts) {
  __shared__ double sh[kBlock / 64];
  const int64_t nf = v.nf, ntot = v.nf + v.n;
  const double* sig = x;
  const double* p = x + nf;
  const double* dp = dx + nf;
  double mx = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ntot; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < nf) {
      const int K = v.K[i], L = v.L[i];
      const double pK = p[K];
      const double iK = fine_kinv<GK>(v, pK, K);
      const double eK = iK * v.TKi[i];
      double eL = 0.0, pL = 0.0, dpL = 0.0, iL = 0.0;
      if (L >= 0) {
        pL = p[L];
        iL = fine_kinv<GK>(v, pL, L);
        eL = iL * v.TLi[i];
        dpL = dp[L];
      }
      const double m = eK + eL;
      const double sj = sig[i];
      const double rs = m * sj + (L >= 0 ? pL : 0.0) - pK + v.g[i];
      double EK = -1.0, EL = 1.0;
      if (NEWTON) {
        EK += fine_dkinv<GK>(v, pK, K, iK) * v.TKi[i] * sj;
        if (L >= 0) EL += fine_dkinv<GK>(v, pL, L, iL) * v.TLi[i] * sj;
      }
      dx[i] = -(rs + EK * dp[K] + (L >= 0 ? EL * dpL : 0.0)) / m;
    } else {
      const double d = fabs(dp[i - nf]);
      mx = d == d ? fmax(mx, d) : HUGE_VAL;   // a NaN counts as non-finite (fmax would drop it)
    }
  }
  mx = block_max(mx, sh);
  if (threadIdx.x == 0) parts[blockIdx.x] = mx;
}

int launch_fine_backsub(const FineView& v, bool newton, const double* x, double* dx, double* parts,
                        hipStream_t s) {
  const int G = reduce_grid(v.nf + v.n);
  const bool gk = general_kappa(v);
  if (newton && gk)
    hipLaunchKernelGGL((k_fine_backsub<true, true>), dim3(G), dim3(kBlock), 0, s, v, x, dx, parts);
  else if (newton)
    hipLaunchKernelGGL((k_fine_backsub<true, false>), dim3(G), dim3(kBlock), 0, s, v, x, dx, parts);
  else if (gk)
    hipLaunchKernelGGL((k_fine_backsub<false, true>), dim3(G), dim3(kBlock), 0, s, v, x, dx, parts);
  else
    hipLaunchKernelGGL((k_fine_backsub<false, false>), dim3(G), dim3(kBlock), 0, s, v, x, dx, parts);
  LAUNCHCHECK();
  return G;
}

// ------------------------------------------------------------------ problem data

// f_K = |tau_K| f_K (input order source -> internal order), then the
// Neumann inflow |eps| g_N is added by k_neumann_fold.
__global__ void k_fine_rhs(int64_t n, const int* __restrict__ cell_in, const double* __restrict__ vol,
                           const double* __restrict__ src, double* __restrict__ f) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) f[c] = vol[c] * src[cell_in[c]];
}

// Neumann faces of each internal cell as a CSR list (deterministic order).
__global__ void k_neumann_fold(int64_t n, const int* __restrict__ nptr, const int* __restrict__ nface,
                               const double* __restrict__ narea, const double* __restrict__ gN,
                               double* __restrict__ f) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double acc = 0.0;
  for (int k = nptr[c]; k < nptr[c + 1]; ++k) acc += narea[k] * gN[nface[k]];
  f[c] += acc;
}

__global__ void k_fine_g(int64_t nf, const int* __restrict__ flux_in, const int* __restrict__ L,
                         const double* __restrict__ gD, double* __restrict__ g) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < nf) g[j] = (L[j] < 0 && gD) ? gD[flux_in[j]] : 0.0;
}

void launch_fine_problem(const FineView& v, const int* cell_in, const int* flux_in, const double* vol,
                         const int* nptr, const int* nface, const double* narea, const double* src,
                         const double* gD, const double* gN, double* f, double* g, hipStream_t s) {
  if (v.n) {
    hipLaunchKernelGGL(k_fine_rhs, dim3(grid_for(v.n, kBlock)), dim3(kBlock), 0, s, v.n, cell_in, vol, src, f);
    LAUNCHCHECK();
    if (gN) {
      hipLaunchKernelGGL(k_neumann_fold, dim3(grid_for(v.n, kBlock)), dim3(kBlock), 0, s, v.n, nptr, nface, narea,
                         gN, f);
      LAUNCHCHECK();
    }
  }
  if (v.nf) {
    hipLaunchKernelGGL(k_fine_g, dim3(grid_for(v.nf, kBlock)), dim3(kBlock), 0, s, v.nf, flux_in, v.L, gD, g);
    LAUNCHCHECK();
  }
}

// ------------------------------------------------------------------ layout maps

__global__ void k_gather(int64_t n, const int* __restrict__ map, const double* __restrict__ in,
                         double* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[map[i]];
}
__global__ void k_scatter(int64_t n, const int* __restrict__ map, const double* __restrict__ in,
                          double* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[map[i]] = in[i];
}
__global__ void k_fill(int64_t n, double v, double* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v;
}
// sigma = -|eps| g_N on Neumann faces (input order)
__global__ void k_neumann_flux(int64_t nn, const int* __restrict__ nface_in, const double* __restrict__ narea_in,
                               const double* __restrict__ gN, double* __restrict__ sig_out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nn) sig_out[nface_in[i]] = gN ? -narea_in[i] * gN[nface_in[i]] : 0.0;
}

void launch_gather(int64_t n, const int* map, const double* in, double* out, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_gather, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, n, map, in, out);
  LAUNCHCHECK();
}
void launch_scatter(int64_t n, const int* map, const double* in, double* out, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_scatter, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, n, map, in, out);
  LAUNCHCHECK();
}
void launch_fill(int64_t n, double v, double* out, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(n, kBlock)), dim3(kBlock), 0, s, n, v, out);
  LAUNCHCHECK();
}
void launch_neumann_flux(int64_t nn, const int* nface_in, const double* narea_in, const double* gN, double* sig,
                         hipStream_t s) {
  if (!nn) return;
  hipLaunchKernelGGL(k_neumann_flux, dim3(grid_for(nn, kBlock)), dim3(kBlock), 0, s, nn, nface_in, narea_in, gN, sig);
  LAUNCHCHECK();
}

}  // namespace spfas
