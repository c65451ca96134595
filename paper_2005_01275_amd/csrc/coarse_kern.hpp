// Coarse-level kernels of the solve phase and the transfers (coarse.hip).
#pragma once

#include "coarse.hpp"
#include "fine.hpp"

namespace spfas {

struct Hierarchy;

// r = A^l(x + step dx) - b on a coarse level (Prop. 1 assembly); returns the
// number of partial sums of r.r written to parts.
int launch_coarse_resid(const CoarseLevel& C, const KappaFam& kf, const double* x, const double* dx, double step,
                        const double* b, double* r, double* parts, hipStream_t s);
// sums of squares of r(x + s_t dx) for t < nt (nt <= kMaxTrials) in one pass;
// partials of trial t at parts[t G, (t+1) G); returns G
int launch_coarse_resid_trials(const CoarseLevel& C, const KappaFam& kf, const double* x, const double* dx,
                               const double* steps, int nt, const double* b, double* parts, hipStream_t s);
// local saddle blocks [s_c M_c, E_c; D_c, 0], their inverses and the local
// solutions z_c = A_c^{-1} [-r_hat_c; -r_p,c] (algebraic hybridisation)
void launch_coarse_local(CoarseLevel& C, const KappaFam& kf, bool newton, const double* x, const double* r,
                         hipStream_t s);
void launch_H_assemble(CoarseLevel& C, hipStream_t s);
// dx from the multipliers; parts = per-block max |w_c . dp_c|; returns #parts
int launch_coarse_backsub(CoarseLevel& C, const double* lam, double* dx, double* parts, hipStream_t s);
// divergence D^l sigma per pressure unknown (level 0 uses the face lists)
void launch_div_coarse(const CoarseLevel& C, const double* sigma, double* div, hipStream_t s);
void launch_div_fine(int64_t n, const int* cfptr, const int* cfcode, const double* sigma, double* div,
                     hipStream_t s);
// out[A] = volume-weighted mean of the level-l cell field z_l over aggregate A
void launch_volume_mean(const TransferDev& T, const double* vol_l, const double* z_l, const double* vol_c,
                        double* out, hipStream_t s);
// transfers between level l (nf_l flux, np_l pressure) and level l+1
void launch_restrict(const TransferDev& T, const CoarseLevel& Cc, const double* rf, double* out, hipStream_t s);
void launch_project(const TransferDev& T, const CoarseLevel& Cc, const double* xf, const double* divf, double* out,
                    hipStream_t s);
void launch_prolong(const TransferDev& T, const CoarseLevel& Cc, const double* e, double* outf, hipStream_t s);

void setup_coarse_solver(Hierarchy& h, int l);

}  // namespace spfas
