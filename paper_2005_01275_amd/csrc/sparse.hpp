// Linear solvers for the linearised systems of the smoothers: the fine-level
// eliminated system S dp = rhs (Section 3.4 reduced by the diagonal flux
// block) and the hybridised multiplier system H lambda = xi on coarse
// levels (Section 3.4, algebraic hybridisation).
//
// Matrix format ("DIA+CSR"): diagonal in its own array plus the
// off-diagonal entries in CSR (ptr/col/val).  The pattern is fixed at setup;
// values are rewritten by each linearisation.
//
// Preconditioners (both rebuilt numerically after every linearisation on a
// pattern and transfer fixed at setup from the matrix values at setup):
//  * classical AMG (level-0 eliminated system): PMIS coarsening,
//    extended+i interpolation P kept from setup, Galerkin coarse values
//    P^T A P recomputed on the device from per-entry product lists;
//    V(1,1) with one l1-Jacobi sweep on each side, fused into three kernels
//    per level (pre-sweep + residual, restriction, prolongation + sweep
//    through the stored A P);
//  * unsmoothed-aggregation AMG (hybridised coarse systems): piecewise-
//    constant P, V(2,2).
// Smoother weights 1 / (|a_ii| + 0.5 sum_j |a_ij|); the coarsest level is
// inverted densely.
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
// Aggregation-AMG levels with fewer rows than this run the group-per-row
// cycle kernels.
constexpr int kVecRows = 150000;
// Classical-AMG cycle operators with at least this many rows are stored as
// SELL-64 (one thread per row), smaller ones as CSR with a lane group per row.
// On the 60x220x85 hierarchy the 207,000-row level pads SELL-64 to about
// twice its entries and runs faster as CSR.
constexpr int kSellRows = 250000;
// Classical levels with at most this many rows (latency-bound launches)
// compute the restricted residual in the same launch as the residual, from
// G = P^T (I - A diag(w)) applied to the level's right-hand side.
constexpr int kFuseRows = 65536;

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

// The same pattern with FP32 values (level 0 in mixed precision), except
// that entry 0 of row i holds the row sum s_i = sum_j a_ij instead of the
// diagonal; products are formed as y_i = s_i x_i + sum_{j != i} a_ij (x_j -
// x_i).  Rounding to FP32 then perturbs each coupling and each row sum by a
// relative 2^-24, as a relative change of the coefficients would; a rounded
// diagonal would not, since on high-contrast systems it nearly cancels the
// couplings of its row.
struct Sell32View {
  int n = 0;
  const int* sptr = nullptr;
  const int* col = nullptr;
  const float* val = nullptr;
};

// Values of the classical cycle operators: FP16 (the operators A diag(w),
// P^T and P - diag(w) A P are scaled to O(1) entries; products and vectors
// stay FP64).
using cyc_t = _Float16;

// A sparse operator of the classical cycle with FP16 values: SELL-64
// (thread per row, `sell`) for large row counts, else CSR read by a lane
// group per row.  Padding slots of SELL have col = row and src = -1.
struct CycMat {
  int n = 0;
  bool sell = false;
  DVec<int> ptr, col;                 // SELL: slice offsets [ceil(n/64)+1]; CSR: row pointers [n+1]
  DVec<cyc_t> val;
  DVec<int> src;                      // per stored slot: source entry of the value, -1 = padding
  long long nnz = 0;                  // stored entries without padding
  int lanes = 8;                      // CSR: lanes per row of the cycle products
};

struct CycView {
  int n;
  const int* ptr;
  const int* col;
  const cyc_t* val;
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
  // classical interpolation to the next level (kept from setup) and the
  // product lists of A P and of the next level's entries
  DVec<double> pval;                  // P values, CSR order
  DVec<int> aplptr, apla, aplp;       // A P entry -> (A entry code, P entry) products
  DVec<int> appidx;                   // A P entry -> P entry at the same position, -1
  DVec<double> apv;                   // A P values
  DVec<int> clptr, clr, clq;          // next level's off entries then diagonal -> (P entry, A P entry)
  CycMat aw, rm, cm;                  // cycle operators A diag(w), R = P^T, P - diag(w) A P
  // fused down leg (n <= kFuseRows): G = P^T (I - A diag(w)) in FP16 and its
  // products: per entry the P entry of its P^T term (-1: none) and the list
  // of (P entry, A entry code) of its (P^T A) sum
  bool fused = false;
  CycMat gm;
  DVec<int> grt, glptr, glp, gla;
  DVec<double> x, b, r, t;            // work vectors (x, b, r: aggregation AMG)
  DVec<float> x32, b32, r32;          // classical cycle: FP32 vectors inside the cycle
};

// Reuse state of a preconditioner across the linearisations of one solve.
struct PrecReuse {
  bool valid = false;                 // values computed in this solve and the last solve did not fail
  int fresh = 0;                      // Krylov iterations right after the last recomputation
  int last = 0;                       // Krylov iterations of the last solve
  int age = 0;                        // linearisations since the last recomputation
};

struct KernelProf;
// Optional event timing of the finest-level launches of the Krylov solver
// (SpMV) and of the AMG cycle (smoothing + residual on the way down,
// restriction, prolongation + smoothing on the way up); the AMG computes
// its own byte counts.
struct ProfHook {
  KernelProf* prof = nullptr;
  int spmv_id = -1, spmv2_id = -1;
  double spmv_bytes = 0.0;
  int down_id = -1, restrict_id = -1, up_id = -1;
  // the same three phases summed over the levels below the finest
  int tail_down_id = -1, tail_restrict_id = -1, tail_up_id = -1;
};

struct Amg {
  std::vector<AmgLevel> lv;           // lv[0] is the fine matrix
  bool classical = false;             // classical levels (else aggregation)
  ProfHook hook;
  int nd = 0;                         // dense coarsest size
  DVec<double> lu;                    // [nd*nd]
  DVec<int> piv;                      // [nd]
  DVec<int> flag;                     // singular-pivot flag
  int cycles = 1;
  // level-0 values are written by the caller into the FP64 SELL copy
  // (sval64); the DIA+CSR arrays of `view` are refreshed from it only when
  // the preconditioner values are recomputed
  bool sell_source = false;
  void sell_to_csr(hipStream_t s);
  // host setup from the matrix pattern and setup values
  // sell64: also keep FP64 SELL values of level 0 (for Krylov::sell64)
  // classical: classical coarsening (falls back to aggregation when the first
  // classical step stalls)
  void setup(const CsrView& A0, hipStream_t s, bool sell64 = false, int dense_max = kDenseLds,
             bool classical = false);
  void numeric(hipStream_t s);        // coarse values, weights, dense LU
  void operator_values(hipStream_t s);   // only the FP64 SELL copy of level 0 (Krylov operator)
  void apply(const double* b, double* x, hipStream_t s);   // x = B^{-1} b (one V-cycle)
  void apply(const float* b, float* x, hipStream_t s);     // FP32 input and output (classical only)
  void numeric_classical(hipStream_t s);
  template <class T>
  void apply_classical(const T* b, T* x, hipStream_t s);
  void dense_numeric(hipStream_t s);
  int n_levels() const { return (int)lv.size(); }
  std::string describe() const;       // "n/nnz" per level, for diagnostics
  // SPFAS_TRACE=2: event time of every level's down and up legs; level_times()
  // returns the sums since its last call and clears them
  std::shared_ptr<KernelProf> lvprof;
  std::string level_times();
};

// SELL layout of the Krylov products for vectors of type T.
template <class T> struct KrylovSell;
template <> struct KrylovSell<double> { using type = Sell64View; };
template <> struct KrylovSell<float> { using type = Sell32View; };

// Krylov solvers with vectors of type T (FP64, or FP32 in mixed precision);
// dot products and scalars are FP64 either way.
template <class T>
struct KrylovT {
  using SellT = typename KrylovSell<T>::type;
  int n = 0;
  ProfHook hook;
  const SellT* sell = nullptr;        // when set (same matrix as A), products read it instead of A
  DVec<T> r, z, p, q, rh, v, s, t, y, w;
  DVec<double> parts, scal;
  // host-mapped values the host checks, written by the kernels: for PCG
  // p.Ap of the last two iterations, the b.b partials, the r.r partials of
  // the last two iterations; for BiCGStab b.b, then r.r, in the first slot
  double* hlag = nullptr;
  double* dlag = nullptr;             // device address of hlag
  hipEvent_t ev[2] = {nullptr, nullptr};
  int iters = 0;
  bool failed = false;                // last solve met a non-finite value or a PCG breakdown (x returned as 0)
  bool converged = false;             // last solve reached its tolerance
  KrylovT() = default;
  KrylovT(const KrylovT&) = delete;
  KrylovT& operator=(const KrylovT&) = delete;
  ~KrylovT();
  void alloc(int n_);
  // returns the number of iterations; x is overwritten (zero initial guess)
  // stall > 0: stop without convergence when ||r|| fell less than 2x over
  // the last `stall` iterations (for a caller with a fallback method)
  int pcg(const CsrView& A, Amg* M, const T* b, T* x, double rtol, int maxit, hipStream_t st, int stall = 0);
  int bicgstab(const CsrView& A, Amg* M, const T* b, T* x, double rtol, int maxit, hipStream_t st);
};
using Krylov = KrylovT<double>;
using Krylov32 = KrylovT<float>;

// y = A x
void launch_spmv(const CsrView& A, const double* x, double* y, hipStream_t s);
// r = b - A x (FP64 products, r stored in FP32), reading the SELL copy As
// of A when given; per-block partial sums of r.r then b.b in parts[0, 2G);
// returns G (at least 1, also for n = 0)
int launch_resid64(const CsrView& A, const Sell64View* As, const double* x, const double* b, float* r, double* parts,
                   hipStream_t s);

}  // namespace spfas
