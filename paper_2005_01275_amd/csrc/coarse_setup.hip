// Batched hierarchy setup on the device (Appendix A of the paper):
//   phase A, one workgroup per coarse interface: PV trace t_F from the
//     local mixed problem on the union of its two aggregates (one-sided on
//     Dirichlet groups);
//   phase B, one workgroup per aggregate: local Laplacian
//     L_A = D_int M_int^{-1} D_int^T (static matrices), full Jacobi
//     eigen-decomposition, P_A = [q_PV, v_2..v_m], bubbles and trace
//     extensions through the pseudo-inverse of L_A, the static coarse local
//     matrices M^{l+1}_A = P_sigma,A^T M_A P_sigma,A and
//     D^{l+1}_A = P_A^T D_A P_sigma,A (Prop. 1), the flux-moment weights of
//     Q_sigma and the weights of the piecewise-constant projector (App. B).
// Host code orchestrates the levels and builds the index plans.
#include <algorithm>
#include <cstdlib>
#include <cstdio>
#include <chrono>
#include <cmath>
#include <numeric>

#include "coarse_kern.hpp"
#include "dense.hpp"
#include "hier.hpp"
#include "kern.hpp"

namespace spfas {

// ------------------------------------------------------------------ local matrix access

__device__ inline int lv_k(const LocalView& v, int c) {
  return v.level0 ? v.cfptr[c + 1] - v.cfptr[c] : v.lfptr[c + 1] - v.lfptr[c];
}
__device__ inline int lv_m(const LocalView& v, int c) { return v.level0 ? 1 : v.pptr[c + 1] - v.pptr[c]; }
__device__ inline double lv_M(const LocalView& v, int c, int i, int j) {
  if (v.level0) {
    if (i != j) return 0.0;
    const int code = v.cfcode[v.cfptr[c] + i];
    return (code & 1) ? v.TLi[code >> 1] : v.TKi[code >> 1];
  }
  const int k = v.lfptr[c + 1] - v.lfptr[c];
  return v.M[v.mptr[c] + i * k + j];
}
__device__ inline double lv_D(const LocalView& v, int c, int r, int i) {
  if (v.level0) return (v.cfcode[v.cfptr[c] + i] & 1) ? 1.0 : -1.0;
  const int k = v.lfptr[c + 1] - v.lfptr[c];
  return v.D[v.dptr[c] + r * k + i];
}

struct PlanView {
  const int *cell_ptr, *cell_list, *pd_ptr, *pd_list, *dof_ptr, *dof_list, *n_int, *mA;
  const int *fgrp_ptr, *fgrp_list, *grp_pos_A, *grp_pos_B, *smap_ptr, *smap;
};

// ------------------------------------------------------------------ phase A

struct ScratchA {
  size_t mu, du, t, l, y;   // sizes in doubles
  size_t total;
};

// Position of local flux i of a cell of side `side` (0: A, 1: B) among the
// unknowns of the union problem [int(A), int(B), F], or -1 when the flux is
// not one of them (faces to other aggregates, Dirichlet faces).
__device__ inline int union_pos(const int* sm, int i, int side, int nIA, int nIB, int nF, int gA, int gB) {
  const int q = sm[i];
  if (side == 0) {
    if (q < nIA) return q;
    if (q >= gA && q < gA + nF) return nIA + nIB + (q - gA);
    return -1;
  }
  if (q < nIB) return nIA + q;
  if (q >= gB && q < gB + nF) return nIA + nIB + (q - gB);
  return -1;
}

// Level 0 (M diagonal, one pressure unknown per cell, D entries -1 / +1):
// L = D M^{-1} D^T of the union problem is assembled from the two incidences
// of each flux, without the dense D, M^{-1} D^T and their product.  `inc`
// holds per flux the two (row, sign) pairs [row0 | sign0 | row1 | sign1],
// row -1 when absent.
__device__ inline void pv_union_level0(const LocalView& lv, const PlanView& pl, int A, int B, int nIA, int nIB, int nF,
                                       int gA, int gB, int ns, int npA, int npU, double* Mu, double* inc, double* L) {
  for (int s = threadIdx.x; s < ns; s += blockDim.x) {
    Mu[s] = 0.0;
    inc[s] = -1.0;
    inc[ns + s] = 0.0;
    inc[2 * ns + s] = -1.0;
    inc[3 * ns + s] = 0.0;
  }
  wg_sync();
  int row = 0;
  for (int side = 0; side < (B >= 0 ? 2 : 1); ++side) {
    const int X = side == 0 ? A : B;
    for (int ci = pl.cell_ptr[X]; ci < pl.cell_ptr[X + 1]; ++ci, ++row) {
      const int c = pl.cell_list[ci];
      const int k = lv_k(lv, c);
      const int* sm = pl.smap + pl.smap_ptr[ci];
      // a cell's local fluxes are distinct, so the threads touch distinct pi
      for (int i = threadIdx.x; i < k; i += blockDim.x) {
        const int pi = union_pos(sm, i, side, nIA, nIB, nF, gA, gB);
        if (pi < 0) continue;
        Mu[pi] += lv_M(lv, c, i, i);
        const int slot = inc[pi] < 0.0 ? 0 : 2 * ns;
        inc[slot + pi] = (double)row;
        inc[slot + ns + pi] = lv_D(lv, c, 0, i);
      }
      wg_sync();
    }
  }
  // row r of L from the fluxes of its cell, in the cell's local order
  for (int r = threadIdx.x; r < npU; r += blockDim.x) {
    const int side = r < npA ? 0 : 1;
    const int ci = side == 0 ? pl.cell_ptr[A] + r : pl.cell_ptr[B] + (r - npA);
    const int c = pl.cell_list[ci];
    const int k = lv_k(lv, c);
    const int* sm = pl.smap + pl.smap_ptr[ci];
    double* Lr = L + (size_t)r * npU;
    for (int q = 0; q < npU; ++q) Lr[q] = 0.0;
    for (int i = 0; i < k; ++i) {
      const int pi = union_pos(sm, i, side, nIA, nIB, nF, gA, gB);
      if (pi < 0) continue;
      const double w = 1.0 / Mu[pi];
      const bool first = (int)inc[pi] == r;
      const double sr = first ? inc[ns + pi] : inc[3 * ns + pi];
      const int o = (int)(first ? inc[2 * ns + pi] : inc[pi]);
      Lr[r] += w;
      if (o >= 0) Lr[o] += w * sr * (first ? inc[3 * ns + pi] : inc[ns + pi]);
    }
  }
  wg_sync();
}

// order: the interfaces in processing order (largest first, so that the
// workgroups that take a second interface take small ones), or null.
__global__ void __launch_bounds__(kBlock) k_pv_trace(LocalView lv, PlanView pl, int n_faces, const int* __restrict__ order,
                                                     const int* __restrict__ fc1,
                                                     const int* __restrict__ fc2, const double* __restrict__ ones,
                                                     double* __restrict__ trace, double* __restrict__ scratch,
                                                     ScratchA sa, int* __restrict__ bad) {
  __shared__ int flag;
  double* Mu = scratch + (size_t)blockIdx.x * sa.total;
  double* Du = Mu + sa.mu;
  double* T = Du + sa.du;
  double* L = T + sa.t;
  double* y = L + sa.l;
  for (int Fi = blockIdx.x; Fi < n_faces; Fi += gridDim.x) {
    const int F = order ? order[Fi] : Fi;
    const int A = fc1[F], B = fc2[F];
    const int nIA = pl.n_int[A], nIB = B >= 0 ? pl.n_int[B] : 0;
    const int nF = pl.fgrp_ptr[F + 1] - pl.fgrp_ptr[F];
    const int ns = nIA + nIB + nF;
    const int npA = pl.pd_ptr[A + 1] - pl.pd_ptr[A];
    const int npB = B >= 0 ? pl.pd_ptr[B + 1] - pl.pd_ptr[B] : 0;
    const int npU = npA + npB;
    const int gA = pl.grp_pos_A[F], gB = B >= 0 ? pl.grp_pos_B[F] : -1;
    if (lv.level0) {
      pv_union_level0(lv, pl, A, B, nIA, nIB, nF, gA, gB, ns, npA, npU, Mu, Du, L);
    } else {
      const int ldm = ns;
      wg_fill(Mu, ns * ns, 0.0);
      wg_fill(Du, npU * ns, 0.0);
      // assemble cell by cell (deterministic: cells in order, entries of one cell in parallel)
      int rowbase = 0;
      for (int side = 0; side < (B >= 0 ? 2 : 1); ++side) {
        const int X = side == 0 ? A : B;
        for (int ci = pl.cell_ptr[X]; ci < pl.cell_ptr[X + 1]; ++ci) {
          const int c = pl.cell_list[ci];
          const int k = lv_k(lv, c), m = lv_m(lv, c);
          const int* sm = pl.smap + pl.smap_ptr[ci];
          for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
            const int i = e / k, j = e % k;
            const int pi = union_pos(sm, i, side, nIA, nIB, nF, gA, gB);
            const int pj = union_pos(sm, j, side, nIA, nIB, nF, gA, gB);
            if (pi >= 0 && pj >= 0) Mu[pi * ldm + pj] += lv_M(lv, c, i, j);
          }
          for (int e = threadIdx.x; e < m * k; e += blockDim.x) {
            const int r = e / k, i = e % k;
            const int pi = union_pos(sm, i, side, nIA, nIB, nF, gA, gB);
            if (pi >= 0) Du[(rowbase + r) * ns + pi] += lv_D(lv, c, r, i);
          }
          rowbase += m;
          wg_sync();
        }
      }
      // T = Mu^{-1} Du^T  (ns x npU)
      for (int e = threadIdx.x; e < ns * npU; e += blockDim.x) {
        const int s = e / npU, r = e % npU;
        T[s * npU + r] = Du[r * ns + s];
      }
      wg_sync();
      if (!wg_chol(Mu, ns, ns, &flag)) {
        if (threadIdx.x == 0) { atomicAdd(bad, 1); bad[1] = 1; bad[2] = F; bad[3] = flag; }
        continue;
      }
      wg_chol_solve(Mu, ns, ns, T, npU, npU);
      // L = Du T
      wg_gemm(Du, ns, false, T, npU, false, L, npU, npU, npU, ns);
    }
    // right-hand side -f_F and the regularisation rho u u^T on interior
    // interfaces (pure Neumann union)
    double na = 0.0, nb = 0.0;
    for (int r = 0; r < npA; ++r) { const double o = ones[pl.pd_list[pl.pd_ptr[A] + r]]; na += o * o; }
    for (int r = 0; r < npB; ++r) { const double o = ones[pl.pd_list[pl.pd_ptr[B] + r]]; nb += o * o; }
    for (int r = threadIdx.x; r < npU; r += blockDim.x) {
      const double o = r < npA ? ones[pl.pd_list[pl.pd_ptr[A] + r]] : ones[pl.pd_list[pl.pd_ptr[B] + r - npA]];
      y[r] = r < npA ? o / na : -o / nb;   // -f_F
    }
    if (B >= 0) {
      double rho = 0.0;
      for (int r = 0; r < npU; ++r) rho = fmax(rho, L[r * npU + r]);
      wg_sync();   // every thread has read the diagonal before any update below
      const double nu = na + nb;
      for (int e = threadIdx.x; e < npU * npU; e += blockDim.x) {
        const int r = e / npU, q = e % npU;
        const double ur = r < npA ? ones[pl.pd_list[pl.pd_ptr[A] + r]] : ones[pl.pd_list[pl.pd_ptr[B] + r - npA]];
        const double uq = q < npA ? ones[pl.pd_list[pl.pd_ptr[A] + q]] : ones[pl.pd_list[pl.pd_ptr[B] + q - npA]];
        L[e] += rho * ur * uq / nu;
      }
    }
    wg_sync();
    if (!wg_chol(L, npU, npU, &flag)) {
      if (threadIdx.x == 0) { atomicAdd(bad, 1); bad[1] = 2; bad[2] = F; bad[3] = flag; }
      continue;
    }
    wg_chol_solve(L, npU, npU, y, 1, 1);
    // sigma = -M^{-1} D^T p, restricted to F
    for (int q = threadIdx.x; q < nF; q += blockDim.x) {
      const int s = nIA + nIB + q;
      double acc = 0.0;
      if (lv.level0) {
        const double* inc = Du;
        acc = inc[ns + s] * y[(int)inc[s]];
        if (inc[2 * ns + s] >= 0.0) acc += inc[3 * ns + s] * y[(int)inc[2 * ns + s]];
        acc /= Mu[s];
      } else {
        for (int r = 0; r < npU; ++r) acc += T[s * npU + r] * y[r];
      }
      trace[pl.fgrp_list[pl.fgrp_ptr[F] + q]] = -acc;
    }
    wg_sync();
  }
}

// ------------------------------------------------------------------ phase B

struct ScratchB {
  size_t ma, da, ci, t, l, v, pl, tmp, vec, ev;
  size_t total;
};

// Local problems with more pressure unknowns than this take the tridiagonal
// route for their smallest eigenpairs (falling back to the full Jacobi
// decomposition if the shifted Cholesky factorisation fails); smaller ones
// use Jacobi.
constexpr int kSmallEig = 32;

struct CoarseOut {
  const int* lfptr;     // coarse local flux lists
  const int* lfidx;
  const int* c1;        // coarse flux cells
  const int* pptr;
  const int* mptr;
  const int* dptr;
  double* M;
  double* D;
  double* w;
  double* ones;
  double* u;
  double* vol;
};

__global__ void __launch_bounds__(kBlock) k_agg_setup(LocalView lv, PlanView pl, int n_agg, const double* __restrict__ ones,
                                                      const double* __restrict__ uvec, const double* __restrict__ vol,
                                                      const double* __restrict__ trace, double* __restrict__ omega,
                                                      const int* __restrict__ Pptr, double* __restrict__ P,
                                                      const int* __restrict__ Eptr, double* __restrict__ E,
                                                      double* __restrict__ eig, double* __restrict__ lmax,
                                                      CoarseOut co,
                                                      double* __restrict__ scratch, ScratchB sb, int* __restrict__ bad,
                                                      unsigned long long* __restrict__ phase_ns) {
  __shared__ int flag;
  __shared__ double red[2 * kBlock];
  __shared__ double cs[2 * (kBlock + 1)];
  __shared__ int prs[2 * (kBlock + 1)];
  __shared__ int idx_small[64];
  __shared__ double scal[8];
  double* MA = scratch + (size_t)blockIdx.x * sb.total;
  double* DA = MA + sb.ma;
  double* Ci = DA + sb.da;
  double* T = Ci + sb.ci;
  double* L = T + sb.t;
  double* V = L + sb.l;
  double* Pl = V + sb.v;
  double* tmp = Pl + sb.pl;
  double* vec = tmp + sb.tmp;   // 4 vectors of length npA + one of length nd
  double* EX = vec + sb.vec;     // subspace iteration: X, Y, LX (npA x kSubMax), G, W, theta
  double* EY = EX + 2 * kBlock * kSubMax;
  double* ELX = EY + 2 * kBlock * kSubMax;
  double* EG = ELX + 2 * kBlock * kSubMax;
  double* EW = EG + kSubMax * kSubMax;
  double* Eth = EW + kSubMax * kSubMax;
  double* TRI = Eth + kSubMax + 8;   // tridiagonal route: diagonal, subdiagonal, reflector scales
  // optional phase timing (diagnostics): wall-clock ticks (10 ns) per phase, summed by thread 0
  unsigned long long tick = wall_clock64();
  auto phase = [&](int id) {
    if (!phase_ns) return;
    wg_sync();
    if (threadIdx.x == 0) {
      const unsigned long long now = wall_clock64();
      atomicAdd(phase_ns + id, (now - tick) * 10ull);
      tick = now;
    }
  };
  for (int A = blockIdx.x; A < n_agg; A += gridDim.x) {
    const int nI = pl.n_int[A];
    const int nd = pl.dof_ptr[A + 1] - pl.dof_ptr[A];
    const int npA = pl.pd_ptr[A + 1] - pl.pd_ptr[A];
    const int mA = pl.mA[A];
    const int kA = co.lfptr[A + 1] - co.lfptr[A];
    const int nbub = mA - 1;
    const int nface = kA - nbub;
    const int* pdA = pl.pd_list + pl.pd_ptr[A];
    double* y0 = vec;
    double* y1 = vec + npA;
    double* q = vec + 2 * npA;
    double* yc = vec + 3 * npA;   // length >= nd
    const int ldm = lv.level0 ? 1 : nd;
    // 1. assemble M_A (over dofs(A)) and D_A
    wg_fill(MA, lv.level0 ? nd : nd * nd, 0.0);
    wg_fill(DA, npA * nd, 0.0);
    int rowbase = 0;
    for (int ci = pl.cell_ptr[A]; ci < pl.cell_ptr[A + 1]; ++ci) {
      const int c = pl.cell_list[ci];
      const int k = lv_k(lv, c), m = lv_m(lv, c);
      const int* sm = pl.smap + pl.smap_ptr[ci];
      if (lv.level0) {
        for (int i = threadIdx.x; i < k; i += blockDim.x) MA[sm[i]] += lv_M(lv, c, i, i);
      } else {
        for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
          const int i = e / k, j = e % k;
          MA[sm[i] * ldm + sm[j]] += lv_M(lv, c, i, j);
        }
      }
      for (int e = threadIdx.x; e < m * k; e += blockDim.x) {
        const int r = e / k, i = e % k;
        DA[(rowbase + r) * nd + sm[i]] += lv_D(lv, c, r, i);
      }
      rowbase += m;
      wg_sync();
    }
    phase(0);
    // 2-3. T = M_int^{-1} D_int^T  (nI x npA)
    for (int e = threadIdx.x; e < nI * npA; e += blockDim.x) {
      const int s = e / npA, r = e % npA;
      T[s * npA + r] = lv.level0 ? DA[r * nd + s] / MA[s] : DA[r * nd + s];
    }
    if (!lv.level0)
      for (int e = threadIdx.x; e < nI * nI; e += blockDim.x) Ci[e] = MA[(e / nI) * nd + e % nI];
    wg_sync();
    if (!lv.level0 && nI > 0) {
      if (!wg_chol(Ci, nI, nI, &flag)) {
        if (threadIdx.x == 0) { atomicAdd(bad, 1); bad[1] = 3; bad[2] = A; bad[3] = flag; }
        continue;
      }
      wg_chol_solve(Ci, nI, nI, T, npA, npA);
    }
    // L = D_int T; on level 0 from the nonzeros only (each row of T holds
    // the two incidences of its flux), row r from the fluxes of its cell
    if (lv.level0) {
      for (int r = threadIdx.x; r < npA; r += blockDim.x) {
        const int ci = pl.cell_ptr[A] + r;
        const int k = lv_k(lv, pl.cell_list[ci]);
        const int* sm = pl.smap + pl.smap_ptr[ci];
        double* Lr = L + (size_t)r * npA;
        for (int q2 = 0; q2 < npA; ++q2) Lr[q2] = 0.0;
        for (int i = 0; i < k; ++i) {
          const int sf = sm[i];
          if (sf >= nI) continue;
          const double d = DA[r * nd + sf];
          const double* Ts = T + (size_t)sf * npA;
          for (int q2 = 0; q2 < npA; ++q2)
            if (Ts[q2] != 0.0) Lr[q2] += d * Ts[q2];
        }
      }
      wg_sync();
    } else {
      wg_gemm(DA, nd, false, T, npA, false, L, npA, npA, npA, nI);
    }
    // symmetrise
    for (int e = threadIdx.x; e < npA * npA; e += blockDim.x) {
      const int i = e / npA, j = e % npA;
      if (i < j) {
        const double s = 0.5 * (L[i * npA + j] + L[j * npA + i]);
        L[i * npA + j] = s;
        L[j * npA + i] = s;
      }
    }
    wg_sync();
    phase(1);
    // q_PV = 1^l|_A / ||1^l|_A||
    if (threadIdx.x == 0) {
      double nn = 0.0;
      for (int r = 0; r < npA; ++r) nn += ones[pdA[r]] * ones[pdA[r]];
      scal[0] = sqrt(nn);
      double rho = 0.0;
      for (int r = 0; r < npA; ++r) rho = fmax(rho, L[r * npA + r]);
      scal[4] = rho;
    }
    wg_sync();
    for (int r = threadIdx.x; r < npA; r += blockDim.x) q[r] = ones[pdA[r]] / scal[0];
    wg_sync();
    // 4-5. the mA smallest eigenpairs of L_A.  Larger problems: Householder
    // reduction to tridiagonal form (L is overwritten), bisection on Sturm
    // counts for the eigenvalues (and the largest one), inverse iteration on
    // the tridiagonal for the eigenvectors 2..mA (the first is the null
    // vector q), back-transformation by the reflectors; the pseudo-inverse of
    // L_A is applied through the Cholesky factor of L_A + rho q q^T (in V).
    // Small problems, or a factorisation that fails, take the full Jacobi
    // decomposition.
    const int nev = mA - 1;
    const int nbs = min(npA - 1, min(kSubMax, nev + 6));
    bool sub = false;
    double* lam = eig + pl.pd_ptr[A];
    if (npA > kSmallEig && nev >= 1 && nev <= kSubMax) {
      const double rho = scal[4];
      for (int e = threadIdx.x; e < npA * npA; e += blockDim.x) V[e] = L[e] + rho * q[e / npA] * q[e % npA];
      wg_sync();
      if (wg_chol(V, npA, npA, &flag)) {
        double* td = TRI;
        double* te = TRI + npA;
        double* tt = TRI + 2 * npA;
        wg_tridiag(L, npA, td, te, tt, y0, y1, red);
        if (threadIdx.x == 0) {   // Gershgorin interval of the tridiagonal
          double lo = td[0], hi = td[0];
          for (int i = 0; i < npA; ++i) {
            const double r = (i > 0 ? fabs(te[i - 1]) : 0.0) + (i + 1 < npA ? fabs(te[i]) : 0.0);
            lo = fmin(lo, td[i] - r);
            hi = fmax(hi, td[i] + r);
          }
          EG[0] = lo;
          EG[1] = hi;
          EG[2] = 1e-16 * (fabs(lo) + fabs(hi)) + 1e-300;
        }
        wg_sync();
        const double glo = EG[0], ghi = EG[1], tiny = EG[2];
        // eigenvalues 0..nev, one thread each; the largest by the last thread
        for (int j = threadIdx.x; j <= nev; j += blockDim.x) {
          const double v = tri_bisect(td, te, npA, j, glo, ghi, tiny);
          if (j == 0) lam[0] = v;
          else Eth[j - 1] = v;
        }
        if (threadIdx.x == blockDim.x - 1) scal[5] = tri_bisect(td, te, npA, npA - 1, glo, ghi, tiny);
        wg_sync();
        // eigenvectors of the tridiagonal, as many at a time as the scratch
        // (6 npA doubles each) holds
        const int grp = max(1, (int)((4 * kBlock * kSubMax) / (6 * npA)));
        for (int c0 = 0; c0 < nev; c0 += grp) {
          const int c = c0 + (int)threadIdx.x;
          if ((int)threadIdx.x < grp && c < nev) {
            double* y = EY + (size_t)threadIdx.x * 6 * npA;
            tri_invit(td, te, npA, Eth[c], 2.2e-16 * (fabs(glo) + fabs(ghi)), y, y + npA);
            for (int r = 0; r < npA; ++r) EX[r * nbs + c] = y[r];
          }
          wg_sync();
        }
        // close eigenvalues: Gram-Schmidt within the cluster (ascending order)
        if (threadIdx.x == 0) {
          const double ctol = 1e-3 * (fabs(glo) + fabs(ghi));
          for (int c = 1; c < nev; ++c) {
            bool any = false;
            for (int b = 0; b < c; ++b) {
              if (!(fabs(Eth[c] - Eth[b]) < ctol)) continue;
              any = true;
              double dd = 0.0;
              for (int r = 0; r < npA; ++r) dd += EX[r * nbs + b] * EX[r * nbs + c];
              for (int r = 0; r < npA; ++r) EX[r * nbs + c] -= dd * EX[r * nbs + b];
            }
            if (any) {
              double nn = 0.0;
              for (int r = 0; r < npA; ++r) nn += EX[r * nbs + c] * EX[r * nbs + c];
              const double inv = 1.0 / sqrt(nn);
              for (int r = 0; r < npA; ++r) EX[r * nbs + c] *= inv;
            }
          }
          for (int j = 1; j < mA; ++j) lam[j] = Eth[j - 1];
          for (int j = 0; j < mA && j < 64; ++j) idx_small[j] = j;
        }
        wg_sync();
        wg_tridiag_backtransform(L, npA, tt, EX, nev, nbs);
        sub = true;
      }
    }
    if (!sub) {
      wg_jacobi_eig(L, npA, V, npA, npA, cs, prs, red);
      // order the spectrum (thread 0; small sizes)
      if (threadIdx.x == 0) {
        int* ord = (int*)tmp;
        for (int i = 0; i < npA; ++i) ord[i] = i;
        for (int i = 1; i < npA; ++i) {
          const int oi = ord[i];
          const double li = L[oi * npA + oi];
          int j = i - 1;
          while (j >= 0 && L[ord[j] * npA + ord[j]] > li) { ord[j + 1] = ord[j]; --j; }
          ord[j + 1] = oi;
        }
        for (int i = 0; i < mA; ++i) lam[i] = L[ord[i] * npA + ord[i]];
        for (int i = 0; i < mA && i < 64; ++i) idx_small[i] = ord[i];
      }
    }
    wg_sync();
    if (lmax) {
      // counting pass of the eigenvalue-threshold rule: the mA smallest
      // eigenvalues are in eig; the largest is the top of the Jacobi
      // spectrum, or the bisection's (tridiagonal route, already in scal[5])
      if (!sub && threadIdx.x == 0) {
        double mx = L[0];
        for (int i = 1; i < npA; ++i) mx = fmax(mx, L[i * npA + i]);
        scal[5] = mx;
      }
      wg_sync();
      if (threadIdx.x == 0) lmax[A] = scal[5];
      wg_sync();
      continue;
    }
    const int i0 = idx_small[0];
    // eigenvector j >= 1 of the ascending order, entry r
    auto evec = [&](int r, int j) -> double { return sub ? EX[r * nbs + (j - 1)] : V[r * npA + idx_small[j]]; };
    phase(2);
    // 6. P_A = [q_PV, v_2..v_m]
    double* PA = P + Pptr[A];
    for (int r = threadIdx.x; r < npA; r += blockDim.x) PA[r * mA] = q[r];
    for (int j = 1; j < mA; ++j) {
      if (threadIdx.x == 0) {
        double d = 0.0;
        for (int r = 0; r < npA; ++r) d += q[r] * evec(r, j);
        scal[1] = d;
      }
      wg_sync();
      for (int r = threadIdx.x; r < npA; r += blockDim.x) y0[r] = evec(r, j) - scal[1] * q[r];
      wg_sync();
      if (threadIdx.x == 0) {
        double nn = 0.0, mx = 0.0;
        for (int r = 0; r < npA; ++r) { nn += y0[r] * y0[r]; mx = fmax(mx, fabs(y0[r])); }
        const double thr = 1e-8 * mx;
        int k = 0;
        while (k < npA && !(fabs(y0[k]) > thr)) ++k;
        const double sg = (k < npA && y0[k] < 0.0) ? -1.0 : 1.0;
        scal[2] = sg / sqrt(nn);
      }
      wg_sync();
      for (int r = threadIdx.x; r < npA; r += blockDim.x) PA[r * mA + j] = y0[r] * scal[2];
      wg_sync();
    }
    // pseudo-inverse of L_A on a vector: out = sum_{i != i0} V_i (V_i . in) / lambda_i
    // (Jacobi path), or out = P (L_A + rho q q^T)^{-1} P in with P = I - q q^T
    auto lplus = [&](const double* in, double* out) {
      if (sub) {
        if (threadIdx.x == 0) {
          double d = 0.0;
          for (int r = 0; r < npA; ++r) d += q[r] * in[r];
          scal[5] = d;
        }
        wg_sync();
        for (int r = threadIdx.x; r < npA; r += blockDim.x) out[r] = in[r] - scal[5] * q[r];
        wg_sync();
        wg_chol_solve(V, npA, npA, out, 1, 1);
        if (threadIdx.x == 0) {
          double d = 0.0;
          for (int r = 0; r < npA; ++r) d += q[r] * out[r];
          scal[5] = d;
        }
        wg_sync();
        for (int r = threadIdx.x; r < npA; r += blockDim.x) out[r] -= scal[5] * q[r];
        wg_sync();
        return;
      }
      for (int i = threadIdx.x; i < npA; i += blockDim.x) {
        double s = 0.0;
        if (i != i0) {
          for (int r = 0; r < npA; ++r) s += V[r * npA + i] * in[r];
          s /= L[i * npA + i];
        }
        y1[i] = s;
      }
      wg_sync();
      for (int r = threadIdx.x; r < npA; r += blockDim.x) {
        double s = 0.0;
        for (int i = 0; i < npA; ++i) s += V[r * npA + i] * y1[i];
        out[r] = s;
      }
      wg_sync();
    };
    phase(3);
    // 7-9. columns of P_sigma restricted to dofs(A): Pl (nd x kA)
    wg_fill(Pl, nd * kA, 0.0);
    for (int j = 1; j < mA; ++j) {
      // bubble: b = T L^+ v_j
      for (int r = threadIdx.x; r < npA; r += blockDim.x) y0[r] = PA[r * mA + j];
      wg_sync();
      lplus(y0, yc);
      const int col = nface + j - 1;
      for (int s = threadIdx.x; s < nI; s += blockDim.x) {
        double acc = 0.0;
        for (int r = 0; r < npA; ++r) acc += T[s * npA + r] * yc[r];
        Pl[s * kA + col] = acc;
      }
      wg_sync();
    }
    phase(4);
    for (int kf = 0; kf < nface; ++kf) {
      const int J = co.lfidx[co.lfptr[A] + kf];
      const int gpos = (co.c1[J] == A) ? pl.grp_pos_A[J] : pl.grp_pos_B[J];
      const int nF = pl.fgrp_ptr[J + 1] - pl.fgrp_ptr[J];
      const int* grp = pl.fgrp_list + pl.fgrp_ptr[J];
      // trace on the group rows
      for (int i = threadIdx.x; i < nF; i += blockDim.x) Pl[(gpos + i) * kA + kf] = trace[grp[i]];
      // DF = D_{A,F} t  and c = q . DF
      for (int r = threadIdx.x; r < npA; r += blockDim.x) {
        double acc = 0.0;
        for (int i = 0; i < nF; ++i) acc += DA[r * nd + gpos + i] * trace[grp[i]];
        y0[r] = acc;
      }
      wg_sync();
      if (threadIdx.x == 0) {
        double c = 0.0;
        for (int r = 0; r < npA; ++r) c += q[r] * y0[r];
        scal[3] = c;
      }
      wg_sync();
      const double cA = scal[3];
      // g1 = -M_{int,F} t ; h = M_int^{-1} g1 (coarse levels only)
      double* h = Pl;   // reuse: write h into column kf of the interior rows
      if (!lv.level0) {
        for (int s = threadIdx.x; s < nI; s += blockDim.x) {
          double acc = 0.0;
          for (int i = 0; i < nF; ++i) acc -= MA[s * nd + gpos + i] * trace[grp[i]];
          h[s * kA + kf] = acc;
        }
        wg_sync();
        // T^T g1  (before solving: D_int M_int^{-1} g1 = T^T g1)
        for (int r = threadIdx.x; r < npA; r += blockDim.x) {
          double acc = 0.0;
          for (int s = 0; s < nI; ++s) acc += T[s * npA + r] * h[s * kA + kf];
          yc[r] = acc;
        }
        wg_sync();
        if (nI > 0) wg_chol_solve(Ci, nI, nI, h + kf, 1, kA);
      } else {
        for (int r = threadIdx.x; r < npA; r += blockDim.x) yc[r] = 0.0;
        wg_sync();
      }
      // rhs = T^T g1 - (c q - DF); pp = L^+ rhs
      for (int r = threadIdx.x; r < npA; r += blockDim.x) yc[r] = yc[r] - (cA * q[r] - y0[r]);
      wg_sync();
      lplus(yc, y0);
      // sigma_int = h - T pp
      for (int s = threadIdx.x; s < nI; s += blockDim.x) {
        double acc = 0.0;
        for (int r = 0; r < npA; ++r) acc += T[s * npA + r] * y0[r];
        Pl[s * kA + kf] = (lv.level0 ? 0.0 : Pl[s * kA + kf]) - acc;
      }
      wg_sync();
      // Q_sigma weights (lower aggregate of an interface, or the only one of a Dirichlet group)
      if (co.c1[J] == A) {
        for (int i = threadIdx.x; i < nF; i += blockDim.x) {
          double acc = 0.0;
          for (int r = 0; r < npA; ++r) acc += q[r] * DA[r * nd + gpos + i];
          omega[grp[i]] = acc / cA;
        }
      }
      wg_sync();
    }
    phase(5);
    // 10. M^{l+1}_A = Pl^T M_A Pl
    double* Mc = co.M + co.mptr[A];
    if (lv.level0) {
      for (int e = threadIdx.x; e < kA * kA; e += blockDim.x) {
        const int a = e / kA, b = e % kA;
        double acc = 0.0;
        for (int s = 0; s < nd; ++s) acc += Pl[s * kA + a] * MA[s] * Pl[s * kA + b];
        Mc[e] = acc;
      }
      wg_sync();
    } else {
      wg_gemm(MA, nd, false, Pl, kA, false, tmp, kA, nd, kA, nd);
      wg_gemm(Pl, kA, true, tmp, kA, false, Mc, kA, kA, kA, nd);
    }
    // 11. D^{l+1}_A = P_A^T D_A Pl
    wg_gemm(DA, nd, false, Pl, kA, false, tmp, kA, npA, kA, nd);
    wg_gemm(PA, mA, true, tmp, kA, false, co.D + co.dptr[A], kA, mA, kA, npA);
    // 12. interior block of P_sigma
    double* EA = E + Eptr[A];
    for (int e = threadIdx.x; e < nI * kA; e += blockDim.x) EA[e] = Pl[e];
    phase(6);
    // 14. projector weights and coarse 1, u, volume
    for (int i = threadIdx.x; i < mA; i += blockDim.x) {
      double so = 0.0, su = 0.0;
      for (int r = 0; r < npA; ++r) {
        so += PA[r * mA + i] * ones[pdA[r]];
        su += PA[r * mA + i] * uvec[pdA[r]];
      }
      co.ones[co.pptr[A] + i] = so;
      co.u[co.pptr[A] + i] = su;
    }
    if (threadIdx.x == 0) {
      double v = 0.0;
      for (int ci = pl.cell_ptr[A]; ci < pl.cell_ptr[A + 1]; ++ci) v += vol[pl.cell_list[ci]];
      co.vol[A] = v;
    }
    wg_sync();
    for (int i = threadIdx.x; i < mA; i += blockDim.x) co.w[co.pptr[A] + i] = co.u[co.pptr[A] + i] / co.vol[A];
    wg_sync();
    phase(7);
  }
}

// ------------------------------------------------------------------ host orchestration

static PlanView plan_view(const TransferDev& t) {
  PlanView p;
  p.cell_ptr = t.cell_ptr.p; p.cell_list = t.cell_list.p; p.pd_ptr = t.pd_ptr.p; p.pd_list = t.pd_list.p;
  p.dof_ptr = t.dof_ptr.p; p.dof_list = t.dof_list.p; p.n_int = t.n_int.p; p.mA = t.mA.p;
  p.fgrp_ptr = t.fgrp_ptr.p; p.fgrp_list = t.fgrp_list.p; p.grp_pos_A = t.grp_pos_A.p; p.grp_pos_B = t.grp_pos_B.p;
  p.smap_ptr = t.smap_ptr.p; p.smap = t.smap.p;
  return p;
}

template <class T>
static std::vector<int> to_int(const std::vector<T>& v) {
  std::vector<int> r(v.size());
  for (size_t i = 0; i < v.size(); ++i) r[i] = (int)v[i];
  return r;
}

static size_t slots_for(size_t per_slot_doubles, int items) {
  const size_t budget = (size_t)6 << 30;   // bytes of setup scratch
  size_t s = budget / std::max<size_t>(1, per_slot_doubles * sizeof(double));
  s = std::max<size_t>(1, std::min<size_t>(s, 4096));
  return std::min<size_t>(s, (size_t)std::max(1, items));
}

void setup_coarse_levels(Hierarchy& h) {
  hipStream_t s = h.stream;
  const int L = h.n_levels;
  if (L < 2) return;
  h.eigvals.assign(L - 1, {});
  // device view of level 0
  FineDev& f = h.fine;
  std::vector<int> cfptr0 = f.cfptr.download(s), cfcode0 = f.cfcode.download(s);
  std::vector<int> cell_in0 = f.cell_in.download(s);   // internal -> canonical cell id on level 0
  const Topo& t0 = h.topo[0];
  const int64_t n0 = t0.n_cells, nf0 = t0.n_flux;
  // canonical -> device ids on level 0
  std::vector<int64_t> dev_cell0(n0), dev_flux0(nf0);
  for (int64_t i = 0; i < n0; ++i) dev_cell0[cell_in0[i]] = i;
  for (int64_t i = 0; i < nf0; ++i) dev_flux0[t0.flux_order[i]] = i;
  DVec<double> ones0;
  ones0.alloc(n0);
  launch_fill(n0, 1.0, ones0.p, s);
  // eigenvalue-threshold count: each level first runs the aggregate kernel
  // in its counting mode on the provisional coarse topology, then (when the
  // counts differ) rebuilds the coarser topologies and runs again
  std::vector<char> counted(L, 0);
  const bool trace = trace_level() > 0;
  for (int l = 0; l + 1 < L; ++l) {
    const double t_level = wall_ms();
    const bool counting = h.copts.eig_threshold > 0.0 && !counted[l];
    const Topo& tf = h.topo[l];
    const Topo& tc = h.topo[l + 1];
    std::vector<int64_t> dev_cell, dev_p, dev_flux, dcfptr, dcfidx;
    if (l == 0) {
      dev_cell = dev_cell0;
      dev_p = dev_cell0;
      dev_flux = dev_flux0;
      dcfptr.assign(cfptr0.begin(), cfptr0.end());
      dcfidx.resize(cfcode0.size());
      for (size_t k = 0; k < cfcode0.size(); ++k) dcfidx[k] = cfcode0[k] >> 1;
    } else {
      dev_cell.resize(tf.n_cells);
      std::iota(dev_cell.begin(), dev_cell.end(), 0);
      dev_p.resize(tf.n_p());
      std::iota(dev_p.begin(), dev_p.end(), 0);
      dev_flux.resize(tf.n_flux);
      std::iota(dev_flux.begin(), dev_flux.end(), 0);
      dcfptr = tf.cfptr;
      dcfidx = tf.cfidx;
    }
    TransferPlan plan = make_plan(tf, tc, dev_cell, dev_p, dev_flux, dcfptr, dcfidx);
    if (trace) std::fprintf(stderr, "[spfas] setup level %d->%d host: plan at %.1f ms\n", l, l + 1, wall_ms() - t_level);
    auto tr = std::make_unique<TransferDev>();
    TransferDev& T = *tr;
    T.n_agg = (int)plan.n_agg;
    T.nf_fine = (int)tf.n_flux;
    T.np_fine = (int)tf.n_p();
    T.cell_ptr.upload(to_int(plan.cell_ptr), s);
    T.cell_list.upload(to_int(plan.cell_list), s);
    T.pd_ptr.upload(to_int(plan.pd_ptr), s);
    T.pd_list.upload(to_int(plan.pd_list), s);
    T.dof_ptr.upload(to_int(plan.dof_ptr), s);
    T.dof_list.upload(to_int(plan.dof_list), s);
    T.n_int.upload(plan.n_int, s);
    T.mA.upload(plan.mA, s);
    T.fgrp_ptr.upload(to_int(plan.fgrp_ptr), s);
    T.fgrp_list.upload(to_int(plan.fgrp_list), s);
    T.grp_pos_A.upload(to_int(plan.grp_pos_A), s);
    T.grp_pos_B.upload(to_int(plan.grp_pos_B), s);
    T.smap_ptr.upload(to_int(plan.smap_ptr), s);
    T.smap.upload(plan.smap, s);
    T.h_pd_ptr = to_int(plan.pd_ptr);
    T.h_mA = plan.mA;
    T.h_nint = plan.n_int;
    // ---- coarse level topology on the device
    auto cl = std::make_unique<CoarseLevel>();
    CoarseLevel& C = *cl;
    C.n = (int)tc.n_cells;
    C.np = (int)tc.n_p();
    C.nf = (int)tc.n_flux;
    C.h_pptr = to_int(tc.pptr);
    C.h_lfptr = to_int(tc.cfptr);
    C.h_lfidx = to_int(tc.cfidx);
    C.h_c1 = to_int(tc.c1);
    C.h_c2 = to_int(tc.c2);
    C.h_kind = tc.kind;
    C.h_mptr.assign(C.n + 1, 0);
    C.h_dptr.assign(C.n + 1, 0);
    for (int c = 0; c < C.n; ++c) {
      const int k = C.h_lfptr[c + 1] - C.h_lfptr[c], m = C.h_pptr[c + 1] - C.h_pptr[c];
      C.h_mptr[c + 1] = C.h_mptr[c] + k * k;
      C.h_dptr[c + 1] = C.h_dptr[c] + m * k;
    }
    C.pptr.upload(C.h_pptr, s);
    C.lfptr.upload(C.h_lfptr, s);
    C.lfidx.upload(C.h_lfidx, s);
    C.mptr.upload(C.h_mptr, s);
    C.dptr.upload(C.h_dptr, s);
    C.c1.upload(C.h_c1, s);
    C.c2.upload(C.h_c2, s);
    C.kind.upload(C.h_kind, s);
    C.M.alloc(C.h_mptr[C.n]);
    C.D.alloc(C.h_dptr[C.n]);
    C.w.alloc(C.np);
    C.ones.alloc(C.np);
    C.u.alloc(C.np);
    C.vol.alloc(C.n);
    // contributors of each coarse flux: (cell, local index)
    {
      std::vector<int> fcell(2 * C.nf, -1), floc(2 * C.nf, -1);
      for (int c = 0; c < C.n; ++c)
        for (int q = C.h_lfptr[c]; q < C.h_lfptr[c + 1]; ++q) {
          const int J = C.h_lfidx[q];
          const int slot = (C.h_c1[J] == c) ? 0 : 1;
          fcell[2 * J + slot] = c;
          floc[2 * J + slot] = q - C.h_lfptr[c];
        }
      C.fcell.upload(fcell, s);
      C.floc.upload(floc, s);
    }
    // ---- numeric buffers of the transfer
    std::vector<int> Pptr(T.n_agg + 1, 0), Eptr(T.n_agg + 1, 0);
    size_t maxA = 0;
    size_t mx_nd = 0, mx_np = 0, mx_nI = 0, mx_k = 0;
    for (int A = 0; A < T.n_agg; ++A) {
      const int npA = (int)(plan.pd_ptr[A + 1] - plan.pd_ptr[A]);
      const int nd = (int)(plan.dof_ptr[A + 1] - plan.dof_ptr[A]);
      const int nI = plan.n_int[A];
      const int k = C.h_lfptr[A + 1] - C.h_lfptr[A];
      Pptr[A + 1] = Pptr[A] + npA * plan.mA[A];
      Eptr[A + 1] = Eptr[A] + nI * k;
      mx_nd = std::max<size_t>(mx_nd, nd);
      mx_np = std::max<size_t>(mx_np, npA);
      mx_nI = std::max<size_t>(mx_nI, nI);
      mx_k = std::max<size_t>(mx_k, k);
      (void)maxA;
    }
    // the Jacobi tournament keeps (n+1)/2 rotation pairs in shared arrays of kBlock+1 entries
    require(mx_np <= 2 * kBlock, "aggregate with more than 512 pressure unknowns");
    T.h_Pptr = Pptr;
    T.h_Eptr = Eptr;
    T.Pptr.upload(Pptr, s);
    T.Eptr.upload(Eptr, s);
    T.P.alloc(Pptr.back());
    T.E.alloc(Eptr.back());
    T.trace.alloc(tf.n_flux);
    T.omega.alloc(tf.n_flux);
    T.trace.zero(s);
    T.omega.zero(s);
    T.eig.alloc(tf.n_p());
    // local view and per-level vectors of level l
    LocalView lv;
    const double *ones_l, *u_l, *vol_l;
    if (l == 0) {
      lv.level0 = 1;
      lv.cfptr = f.cfptr.p;
      lv.cfcode = f.cfcode.p;
      lv.TKi = f.TKi.p;
      lv.TLi = f.TLi.p;
      ones_l = ones0.p;
      u_l = f.vol.p;
      vol_l = f.vol.p;
    } else {
      CoarseLevel& Fl = *h.coarse[l - 1];
      lv = Fl.view();
      ones_l = Fl.ones.p;
      u_l = Fl.u.p;
      vol_l = Fl.vol.p;
    }
    DVec<int> bad;
    bad.alloc(4);
    bad.zero(s);
    PlanView pv = plan_view(T);
    const bool tr_on = trace_level() > 0;
    double t_a = wall_ms();
    if (tr_on) std::fprintf(stderr, "[spfas] setup level %d->%d host: uploads at %.1f ms\n", l, l + 1, t_a - t_level);
    // ---- phase A: PV traces
    int n_faces_c = 0;
    while (n_faces_c < C.nf && C.h_kind[n_faces_c] != FK_BUBBLE) ++n_faces_c;
    if (n_faces_c > 0 && !counting) {
      size_t mx_ns = 0, mx_npU = 0;
      for (int J = 0; J < n_faces_c; ++J) {
        const int A = C.h_c1[J], B = C.h_c2[J];
        const size_t ns = plan.n_int[A] + (B >= 0 ? plan.n_int[B] : 0) + (plan.fgrp_ptr[J + 1] - plan.fgrp_ptr[J]);
        const size_t npU = (plan.pd_ptr[A + 1] - plan.pd_ptr[A]) + (B >= 0 ? plan.pd_ptr[B + 1] - plan.pd_ptr[B] : 0);
        mx_ns = std::max(mx_ns, ns);
        mx_npU = std::max(mx_npU, npU);
      }
      ScratchA sa;
      sa.mu = l == 0 ? mx_ns : mx_ns * mx_ns;
      sa.du = l == 0 ? 4 * mx_ns : mx_npU * mx_ns;   // level 0: the incidence pairs of the fluxes
      sa.t = l == 0 ? 0 : mx_ns * mx_npU;
      sa.l = mx_npU * mx_npU;
      sa.y = mx_npU;
      sa.total = sa.mu + sa.du + sa.t + sa.l + sa.y + 8;
      const size_t slots = slots_for(sa.total, n_faces_c);
      DVec<double> scr;
      scr.alloc(slots * sa.total);
      // with fewer workgroups than interfaces, the largest (by the cube of
      // the local problem size) go first
      DVec<int> order;
      if (slots < (size_t)n_faces_c) {
        std::vector<double> cost(n_faces_c);
        for (int J = 0; J < n_faces_c; ++J) {
          const int A = C.h_c1[J], B = C.h_c2[J];
          const double ns = (double)(plan.n_int[A] + (B >= 0 ? plan.n_int[B] : 0) +
                                     (plan.fgrp_ptr[J + 1] - plan.fgrp_ptr[J]));
          cost[J] = ns * ns * ns;
        }
        std::vector<int> ord(n_faces_c);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        order.upload(ord, s);
      }
      hipLaunchKernelGGL(k_pv_trace, dim3((unsigned)slots), dim3(kBlock), 0, s, lv, pv, n_faces_c,
                         (const int*)order.p, C.c1.p, C.c2.p, ones_l, T.trace.p, scr.p, sa, bad.p);
      LAUNCHCHECK();
      HIPCHECK(hipStreamSynchronize(s));
      if (tr_on)
        std::fprintf(stderr, "[spfas] setup level %d->%d PV traces: %d interfaces, max ns %zu, max npU %zu, %zu "
                     "workgroups: %.1f ms\n", l, l + 1, n_faces_c, mx_ns, mx_npU, slots, wall_ms() - t_a);
    }
    const double t_b = wall_ms();
    // ---- phase B: per aggregate
    {
      ScratchB sb;
      sb.ma = l == 0 ? mx_nd : mx_nd * mx_nd;
      sb.da = mx_np * mx_nd;
      sb.ci = l == 0 ? 1 : mx_nI * mx_nI;
      sb.t = std::max<size_t>(1, mx_nI * mx_np);
      sb.l = mx_np * mx_np;
      sb.v = mx_np * mx_np;
      sb.pl = mx_nd * mx_k;
      sb.tmp = std::max(mx_nd, mx_np + 8) * std::max<size_t>(mx_k, 1) + 8;
      sb.vec = 3 * mx_np + std::max(mx_nd, mx_np) + 8;
      sb.ev = 3 * (size_t)(2 * kBlock) * kSubMax + 2 * kSubMax * kSubMax + kSubMax + 8 + 3 * mx_np + 8;
      sb.total = sb.ma + sb.da + sb.ci + sb.t + sb.l + sb.v + sb.pl + sb.tmp + sb.vec + sb.ev + 8;
      const size_t slots = slots_for(sb.total, T.n_agg);
      DVec<double> scr;
      scr.alloc(slots * sb.total);
      DVec<unsigned long long> phase_ns;
      if (tr_on) {
        phase_ns.alloc(8);
        phase_ns.zero(s);
      }
      CoarseOut co;
      co.lfptr = C.lfptr.p; co.lfidx = C.lfidx.p; co.c1 = C.c1.p; co.pptr = C.pptr.p; co.mptr = C.mptr.p;
      co.dptr = C.dptr.p; co.M = C.M.p; co.D = C.D.p; co.w = C.w.p; co.ones = C.ones.p; co.u = C.u.p;
      co.vol = C.vol.p;
      if (counting) T.lmax.alloc(T.n_agg);
      hipLaunchKernelGGL(k_agg_setup, dim3((unsigned)slots), dim3(kBlock), 0, s, lv, pv, T.n_agg, ones_l, u_l, vol_l,
                         T.trace.p, T.omega.p, T.Pptr.p, T.P.p, T.Eptr.p, T.E.p, T.eig.p,
                         counting ? T.lmax.p : nullptr, co, scr.p, sb, bad.p, tr_on ? phase_ns.p : nullptr);
      LAUNCHCHECK();
      HIPCHECK(hipStreamSynchronize(s));
      if (tr_on) {
        const std::vector<unsigned long long> ph = phase_ns.download(s);
        std::fprintf(stderr, "[spfas] setup level %d->%d aggregate phases (ms per workgroup): assemble %.2f, local "
                     "Laplacian %.2f, eigen %.2f, P_A %.2f, bubbles %.2f, traces/extensions %.2f, coarse M/D %.2f, "
                     "weights %.2f\n", l, l + 1, ph[0] * 1e-6 / slots, ph[1] * 1e-6 / slots, ph[2] * 1e-6 / slots,
                     ph[3] * 1e-6 / slots, ph[4] * 1e-6 / slots, ph[5] * 1e-6 / slots, ph[6] * 1e-6 / slots,
                     ph[7] * 1e-6 / slots);
      }
      if (tr_on)
        std::fprintf(stderr, "[spfas] setup level %d->%d aggregates: %d, max np %zu, max nd %zu, max nI %zu, %zu "
                     "workgroups: %.1f ms\n", l, l + 1, T.n_agg, mx_np, mx_nd, mx_nI, slots, wall_ms() - t_b);
    }
    if (tr_on) std::fprintf(stderr, "[spfas] setup level %d->%d: aggregates done at %.1f ms\n", l, l + 1, wall_ms() - t_level);
    std::vector<int> hb = bad.download(s);
    if (hb[0] != 0) {
      char buf[200];
      std::snprintf(buf, sizeof buf,
                    "local problem of the hierarchy setup is not positive definite (level %d, site %d, item %d, "
                    "pivot %d, %d failures)", l, hb[1], hb[2], hb[3], hb[0]);
      fail(SPFAS_ERR_INVALID, buf);
    }
    if (counting) {
      // m_A = #{lambda <= eig_threshold lambda_max}, clamped to [m_min, m]
      // and to the aggregate's unknowns (the provisional count computed
      // min(m, unknowns) eigenvalues, enough for the upper clamp)
      const std::vector<double> all = T.eig.download(s), lm = T.lmax.download(s);
      const std::vector<int64_t> npA = aggregate_unknowns(tf);
      std::vector<int64_t> mA(T.n_agg);
      bool same = true;
      for (int A = 0; A < T.n_agg; ++A) {
        int cnt = 0;
        for (int j = 0; j < plan.mA[A]; ++j) cnt += all[plan.pd_ptr[A] + j] <= h.copts.eig_threshold * lm[A];
        mA[A] = std::min<int64_t>(std::min(std::max(cnt, h.copts.m_min), h.copts.m), npA[A]);
        same = same && mA[A] == plan.mA[A];
      }
      if (tr_on) {
        std::vector<int> hist(h.copts.m + 1, 0);
        for (int A = 0; A < T.n_agg; ++A) ++hist[mA[A]];
        std::fprintf(stderr, "[spfas] setup level %d->%d eigenvector counts:", l, l + 1);
        for (int k = 1; k <= h.copts.m; ++k) std::fprintf(stderr, " %d:%d", k, hist[k]);
        std::fprintf(stderr, "\n");
      }
      counted[l] = 1;
      if (!same) h.rebuild_coarse_topology(l, mA);
      --l;   // this level again, on the final coarse topology
      continue;
    }
    {   // the mA smallest eigenvalues of every aggregate, ascending
      const std::vector<double> all = T.eig.download(s);
      std::vector<double>& ev = h.eigvals[l];
      ev.clear();
      for (int A = 0; A < T.n_agg; ++A)
        for (int j = 0; j < plan.mA[A]; ++j) ev.push_back(all[plan.pd_ptr[A] + j]);
    }
    // ---- prolongation helpers
    {
      std::vector<int> pd_agg(plan.pd_list.size()), pd_row(plan.pd_list.size());
      for (int A = 0; A < T.n_agg; ++A)
        for (int64_t q = plan.pd_ptr[A]; q < plan.pd_ptr[A + 1]; ++q) { pd_agg[q] = A; pd_row[q] = (int)(q - plan.pd_ptr[A]); }
      std::vector<int> int_agg, int_row, int_pos;
      for (int A = 0; A < T.n_agg; ++A)
        for (int r = 0; r < plan.n_int[A]; ++r) {
          int_agg.push_back(A);
          int_row.push_back(r);
          int_pos.push_back((int)(plan.dof_ptr[A] + r));
        }
      std::vector<int> grp_of(tf.n_flux, -1);
      for (int J = 0; J < C.nf; ++J)
        for (int64_t q = plan.fgrp_ptr[J]; q < plan.fgrp_ptr[J + 1]; ++q) grp_of[plan.fgrp_list[q]] = J;
      std::vector<int> bub0(T.n_agg, -1);
      for (int J = C.nf - 1; J >= 0; --J)
        if (C.h_kind[J] == FK_BUBBLE) bub0[C.h_c1[J]] = J;
      T.pd_agg.upload(pd_agg, s);
      T.pd_row.upload(pd_row, s);
      T.int_agg.upload(int_agg, s);
      T.int_row.upload(int_row, s);
      T.int_pos.upload(int_pos, s);
      T.grp_of.upload(grp_of, s);
      T.bub0.upload(bub0, s);
      T.n_int_total = (int)int_agg.size();
    }
    h.trans.push_back(std::move(tr));
    h.coarse.push_back(std::move(cl));
    HIPCHECK(hipStreamSynchronize(s));
    if (trace) std::fprintf(stderr, "[spfas] setup level %d->%d: %.1f ms\n", l, l + 1, wall_ms() - t_level);
  }
  // hot-path work buffers and the hybridised solvers of the coarse levels
  for (int l = 1; l < L; ++l) {
    const double t0 = wall_ms();
    setup_coarse_solver(h, l);
    if (trace) std::fprintf(stderr, "[spfas] setup level %d solver: %.1f ms\n", l, wall_ms() - t0);
  }
}

}  // namespace spfas
