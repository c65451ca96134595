// Coarse levels (l >= 1) and the transfers l -> l+1 (Section 3.1,
// Appendix A; Prop. 1).
//
// Every coarse level is stored in canonical order: cells = aggregates of the
// finer level; flux unknowns = interfaces (A < B), Dirichlet groups, bubbles.
// Cell c owns m_c pressure coefficients (pptr), a local flux list
// (lfptr/lfidx, ascending ids), the static local matrix M_c (k_c x k_c,
// row-major at mptr[c]), the local divergence D_c (m_c x k_c at dptr[c]) and
// the projector weights w_c (at pptr[c]).  Each flux unknown has one or two
// (cell, local index) contributors (fcell/floc).
#pragma once

#include <vector>

#include "common.hpp"
#include "sparse.hpp"

namespace spfas {

struct Hierarchy;

// Local matrices of a level as seen by the setup kernels: on level 0 they
// are diagonal and read from the face arrays; on coarse levels dense.
struct LocalView {
  int level0 = 0;
  const int* cfptr = nullptr;
  const int* cfcode = nullptr;
  const double* TKi = nullptr;
  const double* TLi = nullptr;
  const int* lfptr = nullptr;
  const int* lfidx = nullptr;
  const int* mptr = nullptr;
  const double* M = nullptr;
  const int* dptr = nullptr;
  const double* D = nullptr;
  const int* pptr = nullptr;
};

struct CoarseLevel {
  int n = 0, np = 0, nf = 0;
  std::vector<int> h_pptr, h_lfptr, h_lfidx, h_mptr, h_dptr, h_c1, h_c2;
  std::vector<int8_t> h_kind;
  DVec<int> pptr, lfptr, lfidx, mptr, dptr, c1, c2;
  DVec<int8_t> kind;
  DVec<double> M, D, w, ones, u, vol;
  DVec<double> zbar;              // kappa shift per cell of the current problem (when has_shift)
  bool has_shift = false;
  DVec<int> fcell, floc;          // [2*nf]
  int nsum = 0;                   // sum over cells of (k_c + m_c)
  DVec<int> zptr, invptr;         // offsets of local solution vectors / inverses
  // block elimination of the local saddle blocks with the static M_c^{-1}
  bool fast_local = false;
  DVec<int> gptr, sgptr;          // offsets of G_c = M_c^{-1} D_c^T and D_c G_c
  DVec<double> Minv, G, DG;
  // hybridisation: multipliers on interior interfaces
  int nl = 0;
  std::vector<int> h_lam_flux;    // multiplier -> flux id
  DVec<int> lam_flux;
  DVec<int> Hptr, Hcol, Hoc, Hoi, Hoj;   // off entries: contributor cell and local indices
  DVec<int8_t> Hos;                      // sign product of the off contributor
  DVec<double> Hdiag, Hoff, xi, lam;
  CsrView H;
  Amg amg;
  PrecReuse prec;
  Krylov kry;
  // nonlinear work
  DVec<double> x, dx, b, r, t, inv, z, div, x0, ax, zeros;
  LocalView view() const {
    LocalView v;
    v.level0 = 0;
    v.lfptr = lfptr.p; v.lfidx = lfidx.p; v.mptr = mptr.p; v.M = M.p; v.dptr = dptr.p; v.D = D.p; v.pptr = pptr.p;
    return v;
  }
};

struct TransferDev {
  int n_agg = 0;
  int nf_fine = 0, np_fine = 0;
  DVec<int> cell_ptr, cell_list, pd_ptr, pd_list, dof_ptr, dof_list, n_int, mA;
  DVec<int> fgrp_ptr, fgrp_list, grp_pos_A, grp_pos_B, smap_ptr, smap;
  DVec<int> Pptr, Eptr;
  DVec<double> P, E, trace, omega, eig;
  DVec<double> lmax;              // counting pass of the threshold rule: largest eigenvalue per aggregate
  // prolongation helpers
  DVec<int> pd_agg, pd_row;       // per entry of pd_list
  DVec<int> int_agg, int_row;     // per interior entry (int parts of dof_list, concatenated)
  DVec<int> int_pos;              // position of that entry in dof_list
  DVec<int> grp_of;               // per fine flux: coarse flux of its group, -1 if interior
  DVec<int> bub0;                 // per aggregate: first bubble id (coarse flux)
  int n_int_total = 0;
  std::vector<int> h_pd_ptr, h_Pptr, h_Eptr, h_mA, h_nint;
};

// Builds the device data of every coarse level and transfer of h.
void setup_coarse_levels(Hierarchy& h);

}  // namespace spfas
