// Fine-level (level 0) kernels; see fine.hip for the data layout.
#pragma once

#include "common.hpp"

namespace spfas {

// kappa of K(x, p) = K0(x) kappa(p - z(x)), z a per-cell shift:
// kind 0: exp(alpha psi) (Section 2, the model problem);
// kind 1: a / (a + |psi|^beta) (Example 3, Richards-type conductivity).
struct KappaFam {
  int kind = 0;
  double alpha = 0.0, a = 1.0, beta = 2.0;
};

struct FineView {
  int64_t n = 0, nf = 0;
  KappaFam kf;
  const double* z = nullptr;   // [n] shift per internal cell, nullptr: none
  const int* K = nullptr;
  const int* L = nullptr;
  const double* TKi = nullptr;
  const double* TLi = nullptr;
  const double* g = nullptr;
  const double* f = nullptr;
  const int* cfptr = nullptr;
  const int* cfcode = nullptr;
};

void launch_halftrans(int64_t nf, int dim, const int* fc, const double* area, const double* nrm,
                      const double* pt, const double* cen, const double* k0, double* TK, double* TL,
                      int* bad, hipStream_t s);
// Step lengths one multi-step residual launch evaluates.
constexpr int kMaxTrials = 4;
// returns the number of partial sums written
int launch_fine_resid(const FineView& v, const double* x, const double* dx, double s, double* r,
                      double* parts, hipStream_t st);
// sums of squares of r(x + s_t dx) for t < nt (nt <= kMaxTrials) in one pass;
// partials of trial t at parts[t G, (t+1) G); returns G
int launch_fine_resid_trials(const FineView& v, const double* x, const double* dx, const double* steps, int nt,
                             double* parts, hipStream_t st);
// S = D M^{-1} E (Picard: E = D^T) and its right-hand side in one cell
// pass, written into the SELL-64 slots of the level-0 matrix
// (sell_ptr/sell_val of its Sell64View) when sell_ptr is given, else into
// diag/off (DIA+CSR on the cell-face lists).
void launch_fine_linearize_cells(const FineView& v, bool newton, const double* x, const int* sell_ptr,
                                 double* sell_val, double* diag, double* off, double* rhs, hipStream_t s);
// mixed precision: SELL values and right-hand side stored in FP32 for the
// linear solves and in FP64 (sell_val64, rhs64) for the residual of the
// iterative refinement (the DIA+CSR values, when there is no SELL copy,
// are FP64 only)
void launch_fine_linearize_cells(const FineView& v, bool newton, const double* x, const int* sell_ptr,
                                 float* sell_val, double* sell_val64, double* diag, double* off, float* rhs,
                                 double* rhs64, hipStream_t s);
// b = (double) a, or b += (double) a when `add`
void launch_widen(int64_t n, const float* a, double* b, hipStream_t s, bool add = false);
int launch_fine_backsub(const FineView& v, bool newton, const double* x, double* dx, double* parts,
                        hipStream_t s);
void launch_fine_problem(const FineView& v, const int* cell_in, const int* flux_in, const double* vol,
                         const int* nptr, const int* nface, const double* narea, const double* src,
                         const double* gD, const double* gN, double* f, double* g, hipStream_t s);
void launch_gather(int64_t n, const int* map, const double* in, double* out, hipStream_t s);
void launch_scatter(int64_t n, const int* map, const double* in, double* out, hipStream_t s);
void launch_fill(int64_t n, double v, double* out, hipStream_t s);
void launch_neumann_flux(int64_t nn, const int* nface_in, const double* narea_in, const double* gN,
                         double* sig, hipStream_t s);

}  // namespace spfas
