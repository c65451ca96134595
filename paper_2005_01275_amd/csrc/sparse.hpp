// Linear solvers for the linearised systems of the smoothers: the fine-level
// eliminated system S dp = rhs (Section 3.4 reduced by the diagonal flux
// block) and the hybridised multiplier system H lambda = xi on coarse
// levels (Section 3.4, algebraic hybridisation).
//
// Matrix format ("DIA+CSR"): diagonal in its own array plus the
// off-diagonal entries in CSR (ptr/col/val).  The pattern is fixed at setup;
// values are rewritten by each linearisation.
//
// Preconditioner: unsmoothed-aggregation AMG.  Aggregates come from the
// strength of connection of the matrix values at setup (kappa = 1, Picard);
// coarse values are recomputed on the device after every linearisation as
// fixed-order sums of fine entries (P^T A P with piecewise-constant P), the
// coarsest level is factored by dense LU with partial pivoting.  Smoother:
// Jacobi with weights 1 / (|a_ii| + 0.5 sum_j |a_ij|).
//
// Krylov: PCG (symmetric Picard systems) and BiCGStab (Newton systems); all
// scalars stay on the device, the host reads the residual norm once per
// iteration to stop.
#pragma once

#include <memory>
#include <string>
#include <vector>

#include "common.hpp"

namespace spfas {

// Largest coarsest-level matrix inverted inside LDS (88^2 doubles < 64 KiB);
// AMG coarsening continues until the level is at most this size.
constexpr int kDenseLds = 88;
// Strength of connection of the aggregation: |a_ij| >= kStrength max_k |a_ik|.
constexpr double kStrength = 0.1;
// Levels with fewer rows than this run the group-per-row cycle kernels.
constexpr int kVecRows = 150000;

struct CsrView {
  int n = 0;
  const double* diag = nullptr;
  const int* ptr = nullptr;
  const int* col = nullptr;
  const double* val = nullptr;
};

// SELL-64 copy of a level matrix for the V-cycle kernels: rows in slices of
// 64 (one wavefront), each slice padded to its longest row and stored
// column-major, so entry k of row i sits at sptr[i / 64] + 64 k + i % 64.
// The diagonal is entry 0 of every row; padding entries have col = i and
// value 0.  Values are FP32 (the preconditioner's matrix only; every
// vector and every Galerkin product stays FP64).
struct SellView {
  int n = 0;
  const int* sptr = nullptr;   // [ceil(n/64) + 1]
  const int* col = nullptr;
  const float* val = nullptr;
};

// The same SELL-64 pattern with FP64 values (finest level of the fine
// solver, for the Krylov products).
struct Sell64View {
  int n = 0;
  const int* sptr = nullptr;
  const int* col = nullptr;
  const double* val = nullptr;
};

struct AmgLevel {
  int n = 0;
  // SELL-64 copy for the cycle (levels that have a coarser level)
  DVec<int> sptr, scol, smap;         // smap: CSR off index, -1 = diagonal, -2 = padding
  DVec<float> sval;
  DVec<double> sval64;                // level 0 only, when the Krylov products use SELL
  SellView sell;
  Sell64View sell64;
  long long sell_nnz = 0;             // stored nonzeros (diagonal + off), without padding
  bool vec = false;                   // small level: group-per-row kernels on the FP64 CSR, no SELL
  // matrix (level 0 refers to external storage through `view`)
  DVec<double> diag, val;
  DVec<int> ptr, col;
  CsrView view;
  DVec<double> invd;                  // smoother weights
  // aggregation to the next level
  DVec<int> agg;                      // [n]
  DVec<int> mptr, mem;                // members of each coarse node
  // Galerkin contributors of the next level's entries
  DVec<int> goff_ptr, goff_idx;       // coarse off entry -> fine off indices
  DVec<int> gdiag_ptr, gdiag_idx;     // coarse diag -> (idx << 1 | is_off)
  DVec<double> x, b, r, t;            // work vectors
};

struct KernelProf;
// Optional event timing of the finest-level launches of the Krylov solver
// (SpMV) and of the AMG cycle (two-sweep pre-smoothing, residual,
// prolongation + sweep, last sweep); the AMG computes its own byte counts.
struct ProfHook {
  KernelProf* prof = nullptr;
  int spmv_id = -1, spmv2_id = -1;
  double spmv_bytes = 0.0;
  int pre_id = -1, resid_id = -1, post1_id = -1, post2_id = -1;
};

struct Amg {
  std::vector<AmgLevel> lv;           // lv[0] is the fine matrix
  ProfHook hook;
  int nd = 0;                         // dense coarsest size
  DVec<double> lu;                    // [nd*nd]
  DVec<int> piv;                      // [nd]
  DVec<int> flag;                     // singular-pivot flag
  int cycles = 1;
  // host setup from the matrix pattern and setup values
  // sell64: also keep FP64 SELL values of level 0 (for Krylov::sell64)
  void setup(const CsrView& A0, hipStream_t s, bool sell64 = false, int dense_max = kDenseLds);
  void numeric(hipStream_t s);        // coarse values, weights, dense LU
  void apply(const double* b, double* x, hipStream_t s);   // x = B^{-1} b (one V-cycle)
  int n_levels() const { return (int)lv.size(); }
  std::string describe() const;       // "n/nnz" per level, for diagnostics
  // SPFAS_TRACE=2: event time of every level's down and up legs; level_times()
  // returns the sums since its last call and clears them
  std::shared_ptr<KernelProf> lvprof;
  std::string level_times();
};

struct Krylov {
  int n = 0;
  ProfHook hook;
  const Sell64View* sell64 = nullptr;  // when set (same matrix as A), products read it instead of A
  DVec<double> r, z, p, q, rh, v, s, t, y, w;
  DVec<double> parts, scal;
  double* hscal = nullptr;
  double* hlag = nullptr;             // pinned: p.Ap and r.r of the last two PCG iterations
  hipEvent_t ev[2] = {nullptr, nullptr};
  int iters = 0;
  bool failed = false;                // last solve met a non-finite value or a PCG breakdown (x returned as 0)
  bool converged = false;             // last solve reached its tolerance
  ~Krylov();
  void alloc(int n_);
  // returns the number of iterations; x is overwritten (zero initial guess)
  int pcg(const CsrView& A, Amg* M, const double* b, double* x, double rtol, int maxit, hipStream_t st);
  int bicgstab(const CsrView& A, Amg* M, const double* b, double* x, double rtol, int maxit, hipStream_t st);
};

// y = A x
void launch_spmv(const CsrView& A, const double* x, double* y, hipStream_t s);

}  // namespace spfas
