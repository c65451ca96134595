// Nonlinear solvers (host control, device work): smoothing steps with the
// step cap and Alg. 1 backtracking, single-level Picard/Newton (Section
// 2.2) and the FAS V-cycle (Alg. 2).
#include "solve.hpp"

#include <algorithm>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <functional>
#include <vector>

#include "coarse_kern.hpp"
#include "kern.hpp"

namespace spfas {

// ------------------------------------------------------------------ small kernels

__global__ void __launch_bounds__(kBlock) k_axpy(int64_t n, double a, const double* __restrict__ x,
                                                 double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = fma(a, x[i], y[i]);   // the rounding of the trial points x + s dx in the residual kernels
}

__global__ void __launch_bounds__(kBlock) k_neu_flux(int64_t nn, const double* __restrict__ area,
                                                     const int* __restrict__ face, const double* __restrict__ gN,
                                                     double* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nn) out[face[i]] = gN ? -area[i] * gN[face[i]] : 0.0;
}

__global__ void __launch_bounds__(kBlock) k_copy_vec(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}

// y = x on the device (a kernel: cheaper than a copy engine transfer for
// the small coarse vectors)
static void launch_copy(int64_t n, const double* x, double* y, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_copy_vec, dim3(reduce_grid(n)), dim3(kBlock), 0, s, n, x, y);
  LAUNCHCHECK();
}

void launch_axpy(int64_t n, double a, const double* x, double* y, hipStream_t s) {
  if (!n) return;
  const int G = reduce_grid(n);
  hipLaunchKernelGGL(k_axpy, dim3(G), dim3(kBlock), 0, s, n, a, x, y);
  LAUNCHCHECK();
}

// ------------------------------------------------------------------ options

struct Opts {
  bool newton = true;
  double rtol = 1e-8, atol = 1e-10;
  int max_it = 50;
  int bt_nmax = 4;
  double bt_theta = 0.9;
  double cap = 0.0;            // <= 0: off
  int coarsest_max = 10;
  double lin_rtol = 1e-8;
  int lin_max_it = 500;
  int lin_max_it_coarse = 500;   // iteration limit of the coarse-level Krylov solves
  double lin_rtol_coarse = 0.0;  // <= 0: lin_rtol
  double lin_target = 0.0;       // inexact-Newton forcing on level 0; 0 = off
  double stop_tol = 0.0;         // outer stopping threshold of the running solve
  bool newton_pcg = false;       // PCG first on Newton systems, BiCGStab as fallback
  int amg_reuse = 0;             // linearisations that may reuse AMG values (0 = none, < 0 = no limit)
  double coarsest_atol = 1e-10;  // absolute floor of the coarsest level's test
  bool mixed = false;            // FP32 level-0 linear solves inside the FP64 residual and update
};

static Opts make_opts(const spfas_solve_opts& o, bool newton) {
  Opts r;
  r.newton = newton;
  r.rtol = o.rtol;
  r.atol = o.atol;
  r.max_it = o.max_it;
  r.bt_nmax = o.bt_nmax;
  r.bt_theta = o.bt_theta;
  r.cap = o.dp_cap;
  r.coarsest_max = o.coarsest_max_steps;
  r.lin_rtol = o.lin_rtol;
  r.lin_max_it = o.lin_max_it;
  r.lin_max_it_coarse = o.lin_max_it_coarse > 0 ? o.lin_max_it_coarse : o.lin_max_it;
  r.lin_rtol_coarse = o.lin_rtol_coarse > 0.0 ? o.lin_rtol_coarse : o.lin_rtol;
  r.lin_target = o.lin_target;
  r.newton_pcg = o.newton_pcg != 0;
  r.amg_reuse = o.amg_reuse;
  r.coarsest_atol = o.coarsest_atol >= 0.0 ? o.coarsest_atol : o.atol;
  require(o.precision == SPFAS_PREC_FP64 || o.precision == SPFAS_PREC_MIXED,
          "precision must be SPFAS_PREC_FP64 or SPFAS_PREC_MIXED");
  r.mixed = o.precision == SPFAS_PREC_MIXED;
  require(o.lin_target >= 0.0, "lin_target must be non-negative");
  require(r.max_it >= 0 && r.bt_nmax >= 0 && r.coarsest_max >= 0 && r.lin_max_it > 0, "negative iteration limits");
  require(r.bt_theta > 0.0 && r.bt_theta <= 1.0, "bt_theta must be in (0, 1]");
  require(r.rtol >= 0.0 && r.atol >= 0.0 && r.lin_rtol > 0.0, "tolerances must be non-negative");
  return r;
}

// Alg. 1 on a residual-norm function of the step length.  Returns the step
// taken and the residual norm there; `halvings` counts the halvings.
// A trial whose residual is not finite (kappa = exp(alpha p) overflowed)
// counts as +infinity, so it is never preferred to a finite one; when the
// trial finally chosen is still non-finite the step is rejected (0 returned,
// residual unchanged).
// `rn_batch`, when given, evaluates several step lengths in one pass: after a
// rejected full step it supplies the norms at 1/2, 1/4, ... (the same values
// the single evaluations would give), so the halvings need no further waits.
using NormBatch = std::function<void(const double*, int, double*)>;
static double backtrack(const std::function<double(double)>& rn_raw, double r_x, int nmax, double theta,
                        double& r_new, int& halvings, const NormBatch& rn_batch = nullptr) {
  auto fin = [](double v) { return std::isfinite(v) ? v : HUGE_VAL; };
  auto rn = [&](double s) { return fin(rn_raw(s)); };
  double s = 1.0;
  int n = 0;
  double r_s = rn(s);
  std::vector<double> pre;   // norms at 1/2, 1/4, ... from one batched evaluation
  if (rn_batch && r_s > r_x && nmax > 0) {
    const int k = std::min(nmax, kMaxTrials);
    std::vector<double> sl(k);
    double t = 1.0;
    for (int i = 0; i < k; ++i) sl[i] = (t *= 0.5);
    pre.resize(k);
    rn_batch(sl.data(), k, pre.data());
  }
  while (r_s > r_x && n < nmax) {
    const double r_half = n < (int)pre.size() ? fin(pre[n]) : rn(0.5 * s);
    if (r_half > theta * r_s) break;
    s *= 0.5;
    ++n;
    r_s = r_half;
  }
  halvings += n;
  if (r_s == HUGE_VAL) {
    r_new = r_x;
    return 0.0;
  }
  r_new = r_s;
  return s;
}

// PCG on a (non-symmetric) Newton system hands over to BiCGStab when ||r||
// fell less than 2x over this many iterations.
constexpr int kPcgStall = 5;

// Krylov solve of a linearised system: PCG for Picard (symmetric);
// BiCGStab for Newton, or PCG first with BiCGStab from scratch when PCG
// breaks down, stalls or does not converge; the limit counts the iterations
// of both.  `refine`: the first FP32 solve of mixed precision, where a
// stalled PCG (Picard or Newton) returns and the FP64-residual refinement
// goes on from its result.
template <class T>
static int krylov_solve(KrylovT<T>& kry, const CsrView& A, Amg* M, const T* b, T* x, double rtol, const Opts& o,
                        hipStream_t s, bool refine = false) {
  if (!o.newton && !refine) return kry.pcg(A, M, b, x, rtol, o.lin_max_it, s);
  if (!o.newton || o.newton_pcg) {
    const int it = kry.pcg(A, M, b, x, rtol, o.lin_max_it, s, kPcgStall);
    if (kry.converged || refine) return it;
    // the hand-over gets what is left of the solve's iteration limit
    const int left = o.lin_max_it - it;
    if (left <= 0) return it;
    const int it2 = kry.bicgstab(A, M, b, x, rtol, left, s);
    if (trace_level() > 0)
      std::fprintf(stderr, "[spfas] PCG stopped after %d iterations without convergence; BiCGStab %d\n", it, it2);
    return it + it2;
  }
  return kry.bicgstab(A, M, b, x, rtol, o.lin_max_it, s);
}

// Preconditioner values for the next linearised solve: recomputed unless
// they were computed at most amg_reuse linearisations ago (any number when
// amg_reuse < 0) and the last solve
// stayed within f + max(2, f/2) iterations (f: the count right after the
// last recomputation).  The operator copy the Krylov products read is
// refreshed either way.
static bool prec_refresh(Amg& amg, PrecReuse& pr, const Opts& o, hipStream_t s) {
  const bool aged = o.amg_reuse >= 0 && pr.age >= o.amg_reuse;
  const bool fresh = !pr.valid || aged || pr.last > pr.fresh + std::max(2, pr.fresh / 2);
  if (fresh) amg.numeric(s);
  else amg.operator_values(s);
  return fresh;
}

static void prec_record(PrecReuse& pr, bool fresh, int it, bool failed) {
  pr.last = it;
  if (fresh) {
    pr.fresh = it;
    pr.age = 0;
  } else {
    pr.age++;
  }
  pr.valid = !failed;
}

// SPFAS_TRACE=1 prints one line per smoothing step to stderr.
static bool trace_on() { return trace_level() > 0; }

// wall-clock milliseconds after draining the stream (trace output only)
static double trace_clock(hipStream_t s) {
  HIPCHECK(hipStreamSynchronize(s));
  return wall_ms();
}

static double check_finite(double v, const char* what) {
  if (!std::isfinite(v)) fail(SPFAS_ERR_NUMERIC, std::string("non-finite ") + what);
  return v;
}

// ------------------------------------------------------------------ fine level

void setup_fine_solver(Hierarchy& h) {
  FineWork& w = h.fw;
  FineDev& f = h.fine;
  hipStream_t s = h.stream;
  const int64_t n = f.n, nf = f.nf;
  w.x.alloc(nf + n);
  w.dx.alloc(nf + n);
  w.xt.alloc(nf + n);
  w.div.alloc(n);
  w.Sdiag.alloc(n);
  w.Soff.alloc(f.cfcode.n);
  w.rhs.alloc(n);
  w.S.n = (int)n;
  w.S.diag = w.Sdiag.p;
  w.S.ptr = f.cfptr.p;
  w.S.col = f.nb.p;
  w.S.val = w.Soff.p;
  // matrix of the aggregation: Picard at p = 0 (kappa = 1)
  w.x.zero(s);
  FineView v1 = f.view();
  v1.kf = KappaFam{};   // exp(0 psi) = 1
  v1.z = nullptr;
  launch_fine_linearize_cells(v1, false, w.x.p, nullptr, nullptr, w.Sdiag.p, w.Soff.p, w.rhs.p, s);
  HIPCHECK(hipStreamSynchronize(s));
  w.amg.setup(w.S, s, true, kDenseLds, true);
  if (trace_on()) std::fprintf(stderr, "[spfas] level 0 AMG: %s\n", w.amg.describe().c_str());
  // event timing hooks of the finest-level Krylov SpMV and AMG cycle kernels
  ProfHook hk;
  hk.prof = &h.prof;
  hk.spmv_id = SPFAS_PROF_FINE_SPMV;
  hk.spmv2_id = SPFAS_PROF_FINE_SPMV2;
  hk.spmv_bytes = 24.0 * nf + 32.0 * n;
  hk.down_id = SPFAS_PROF_FINE_AMG_DOWN;
  hk.restrict_id = SPFAS_PROF_FINE_AMG_RESTRICT;
  hk.up_id = SPFAS_PROF_FINE_AMG_UP;
  hk.tail_down_id = SPFAS_PROF_AMG_TAIL_DOWN;
  hk.tail_restrict_id = SPFAS_PROF_AMG_TAIL_RESTRICT;
  hk.tail_up_id = SPFAS_PROF_AMG_TAIL_UP;
  w.kry.hook = hk;
  w.amg.hook = hk;
  if (w.amg.lv[0].sval64.n) {   // S products read the SELL-64 copy: value + column per stored entry
    w.kry.sell = &w.amg.lv[0].sell64;
    w.kry.hook.spmv_bytes = 12.0 * (double)w.amg.lv[0].sell_nnz + 24.0 * n;
    // the linearisation writes S straight into that copy; its padding slots
    // stay zero
    w.amg.sell_source = true;
    w.amg.lv[0].sval64.zero(s);
  }
  // mixed precision (classical AMG only): FP32 twins of the SELL values,
  // the right-hand side, the correction and the Krylov vectors
  if (w.amg.classical) {
    w.rhs32.alloc(n);
    w.dp32.alloc(n);
    w.kry32.hook = w.kry.hook;
    if (w.amg.sell_source) {
      const AmgLevel& F0 = w.amg.lv[0];
      w.sval32.alloc(F0.sval64.n);
      w.sval32.zero(s);
      w.S32.n = F0.sell64.n;
      w.S32.sptr = F0.sell64.sptr;
      w.S32.col = F0.sell64.col;
      w.S32.val = w.sval32.p;
      w.kry32.sell = &w.S32;
      w.kry32.hook.spmv_bytes = 8.0 * (double)F0.sell_nnz + 12.0 * n;
    }
  }
  HIPCHECK(hipStreamSynchronize(s));
}

// ||r(x + s_t dx)|| for t < k in one pass (Alg. 1 halvings): the same values
// as fine_rnorm at each step
static void fine_rnorm_trials(Hierarchy& h, const double* x, const double* dx, const double* steps, int k,
                              double* out) {
  int G = 0;
  const double F = (double)h.fine.nf, N = (double)h.fine.n, I = (double)h.fine.cfcode.n;
  h.prof.run(SPFAS_PROF_FINE_RESID_TRIALS, 48.0 * F + 28.0 * N + 4.0 * I, h.stream, [&] {
    G = launch_fine_resid_trials(h.fine.view(), x, dx, steps, k, h.dpin, h.stream);
  });
  h.host_sums(G, k, out);
  for (int t = 0; t < k; ++t) out[t] = std::sqrt(out[t]);
}

static double fine_rnorm(Hierarchy& h, const double* x, const double* dx, double step) {
  int G = 0;
  // distinct data read: per face K, L, 1/T_K, 1/T_L, g, sigma (+ d sigma);
  // per cell p (+ dp), f, the list offset; 4 bytes per cell-face incidence
  const double F = (double)h.fine.nf, N = (double)h.fine.n, I = (double)h.fine.cfcode.n;
  const double bytes = dx ? 48.0 * F + 28.0 * N + 4.0 * I : 40.0 * F + 20.0 * N + 4.0 * I;
  h.prof.run(SPFAS_PROF_FINE_RESID, bytes, h.stream,
             [&] { G = launch_fine_resid(h.fine.view(), x, dx, step, nullptr, h.dpin, h.stream); });
  return std::sqrt(h.host_sum(G));   // may be non-finite inside Alg. 1 trials
}

// Refinement steps of a mixed-precision level-0 solve: the residual of the
// FP64 system S dp = rhs at the FP32 solution is formed in FP64 and, while
// it exceeds kRefineSlack eta ||rhs||, an FP32 solve of S c = r (tolerance
// eta ||rhs|| / ||r||, at most 0.5) adds its correction c to dp.  The slack
// accepts the FP32 solutions whose residual is near the target, where one
// more solve would cost more than the inexact step; FP32 vectors cannot
// hold a solution whose residual is below about 2^-24 ||S|| ||dp||, so on
// high-contrast systems the FP32 solve alone can end orders of magnitude
// above eta.  Returns the Krylov iterations it spent.
constexpr int kRefineMax = 3;
constexpr double kRefineSlack = 10.0;

static int mixed_refine(Hierarchy& h, const Opts& o, double eta, const Sell64View* sv, double* dp,
                        spfas_stats& st) {
  FineWork& w = h.fw;
  hipStream_t s = h.stream;
  const int64_t n = h.fine.n;
  int it = 0;
  for (int k = 0; k <= kRefineMax; ++k) {
    const int G = launch_resid64(w.S, sv, dp, w.rhs.p, w.rhs32.p, h.dpin, s);
    double rb[2];
    h.host_sums(G, 2, rb);
    if (trace_on())
      std::fprintf(stderr, "[spfas] level 0 mixed: refinement %d, ||r||/||b|| = %.3e (eta %.1e)\n", k,
                   std::sqrt(rb[0] / rb[1]), eta);
    // done (or a non-finite residual, which the back-substitution rejects)
    if (!(rb[0] > kRefineSlack * kRefineSlack * eta * eta * rb[1]) || k == kRefineMax) break;
    const double ec = std::min(0.5, std::max(eta, eta * std::sqrt(rb[1] / rb[0])));
    it += krylov_solve(w.kry32, w.S, &w.amg, w.rhs32.p, w.dp32.p, ec, o, s);
    st.refine_steps++;
    if (w.kry32.failed) break;   // keep the solution so far
    launch_widen(n, w.dp32.p, dp, s, true);
  }
  return it;
}

// One Picard or Newton step on level 0 (Section 3.3): solve the linearised
// system (flux block eliminated exactly, M is diagonal on level 0), cap,
// Alg. 1.  `r_x` = ||r(x)|| on entry; returns ||r|| after the step.
static double fine_smooth(Hierarchy& h, const Opts& o, double r_x, spfas_stats& st, bool* moved = nullptr) {
  if (moved) *moved = false;
  FineWork& w = h.fw;
  FineDev& f = h.fine;
  hipStream_t s = h.stream;
  const int64_t n = f.n, nf = f.nf;
  const double t0 = trace_on() ? trace_clock(s) : 0.0;
  // inputs K, L, 1/T_K, 1/T_L, g, sigma per face, p and f per cell, the cell-face
  // codes; outputs the values of S (diagonal + one per incidence) and rhs
  // one pass over the cells; with a SELL copy S goes straight into it.
  // Mixed precision: S (in the SELL layout) and the right-hand side are
  // stored in FP32 and FP64; the linear system is solved in FP32 and refined
  // against the FP64 system; the nonlinear residual, the back-substitution,
  // Alg. 1 and the update stay FP64, so each step corrects the FP64 defect
  // (defect correction).
  const bool mixed = o.mixed && w.amg.classical;
  const Sell64View* sv = w.amg.sell_source ? &w.amg.lv[0].sell64 : nullptr;
  h.prof.run(SPFAS_PROF_FINE_LINEARIZE, 40.0 * nf + 36.0 * n + 12.0 * (double)f.cfcode.n, s, [&] {
    if (mixed)
      launch_fine_linearize_cells(f.view(), o.newton, w.x.p, sv ? sv->sptr : nullptr, sv ? w.sval32.p : nullptr,
                                  sv ? const_cast<double*>(sv->val) : nullptr, w.Sdiag.p, w.Soff.p, w.rhs32.p,
                                  w.rhs.p, s);
    else
      launch_fine_linearize_cells(f.view(), o.newton, w.x.p, sv ? sv->sptr : nullptr,
                                  sv ? const_cast<double*>(sv->val) : nullptr, w.Sdiag.p, w.Soff.p, w.rhs.p, s);
  });
  const bool fresh = prec_refresh(w.amg, w.prec, o, s);
  double* dp = w.dx.p + nf;
  int it;
  double eta = o.lin_rtol;
  if (o.lin_target > 0.0 && o.stop_tol > 0.0 && r_x > 0.0)
    eta = std::max(eta, std::min(0.1, o.lin_target * o.stop_tol / r_x));
  bool failed;
  if (mixed) {
    it = krylov_solve(w.kry32, w.S, &w.amg, w.rhs32.p, w.dp32.p, eta, o, s, true);
    failed = w.kry32.failed;
    if (!failed) {
      launch_widen(n, w.dp32.p, dp, s);
      it += mixed_refine(h, o, eta, sv, dp, st);
    }
  } else {
    it = krylov_solve(w.kry, w.S, &w.amg, w.rhs.p, dp, eta, o, s);
    failed = w.kry.failed;
  }
  prec_record(w.prec, fresh, it, failed);
  st.lin_iters += it;
  double mx = HUGE_VAL;
  if (!failed) {
    const int G = launch_fine_backsub(f.view(), o.newton, w.x.p, w.dx.p, h.dpin, s);
    mx = h.host_max(G);
  }
  if (!std::isfinite(mx)) {   // non-finite linearisation or linear solve: the step is rejected
    st.rejected_steps++;
    st.smoothing_steps++;
    if (trace_on()) std::fprintf(stderr, "[spfas] level 0: step rejected (non-finite linear solve)\n");
    return r_x;
  }
  const double scale = (o.cap > 0.0 && mx > o.cap) ? o.cap / mx : 1.0;
  double r_new = r_x;
  const NormBatch batch = [&](const double* sl, int k, double* out) {
    double st_[kMaxTrials];
    for (int t = 0; t < k; ++t) st_[t] = sl[t] * scale;
    fine_rnorm_trials(h, w.x.p, w.dx.p, st_, k, out);
  };
  const double step = backtrack([&](double sl) { return fine_rnorm(h, w.x.p, w.dx.p, sl * scale); }, r_x,
                                o.bt_nmax, o.bt_theta, r_new, st.bt_halvings, batch);
  if (step > 0.0) launch_axpy(nf + n, step * scale, w.dx.p, w.x.p, s);
  if (moved) *moved = step > 0.0;
  st.smoothing_steps++;
  if (trace_on())
    std::fprintf(stderr, "[spfas] level 0 %s: krylov %d  |r| %.3e -> %.3e  cap %.3g  step %.4g  %.2f ms %s\n",
                 o.newton ? "newton" : "picard", it, r_x, r_new, scale, step, trace_clock(s) - t0,
                 w.amg.level_times().c_str());
  return r_new;
}

// ------------------------------------------------------------------ state I/O

static void load_state(Hierarchy& h, const double* p, const double* sig, bool dev, bool given) {
  FineDev& f = h.fine;
  hipStream_t s = h.stream;
  if (!given) {
    h.fw.x.zero(s);
    return;
  }
  DVec<double> pin, sin;
  const double *pd = p, *sd = sig;
  if (!dev) {
    pin.upload(p, h.n_cells_in, s);
    sin.upload(sig, h.n_faces_in, s);
    pd = pin.p;
    sd = sin.p;
  }
  launch_gather(f.nf, f.flux_in.p, sd, h.fw.x.p, s);
  launch_gather(f.n, f.cell_in.p, pd, h.fw.x.p + f.nf, s);
  HIPCHECK(hipStreamSynchronize(s));
}

static void store_state(Hierarchy& h, const spfas_problem& prob, double* p, double* sig, bool dev) {
  FineDev& f = h.fine;
  hipStream_t s = h.stream;
  DVec<double> po, so, gn;
  double *pd = p, *sd = sig;
  if (!dev) {
    po.alloc(h.n_cells_in);
    so.alloc(h.n_faces_in);
    pd = po.p;
    sd = so.p;
  }
  const double* gN = prob.g_neumann;
  if (gN && prob.mem == SPFAS_MEM_HOST) {
    gn.upload(prob.g_neumann, h.n_faces_in, s);
    gN = gn.p;
  }
  launch_scatter(f.nf, f.flux_in.p, h.fw.x.p, sd, s);
  launch_scatter(f.n, f.cell_in.p, h.fw.x.p + f.nf, pd, s);
  const int64_t nn = (int64_t)f.neu_in.n;
  if (nn) {
    hipLaunchKernelGGL(k_neu_flux, dim3(grid_for(nn, kBlock)), dim3(kBlock), 0, s, nn, f.neu_area.p, f.neu_in.p, gN,
                       sd);
    LAUNCHCHECK();
  }
  if (!dev) {
    HIPCHECK(hipMemcpyAsync(p, pd, h.n_cells_in * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(sig, sd, h.n_faces_in * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  HIPCHECK(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------ drivers

// every solve starts with freshly computed preconditioner values
static void prec_reset(Hierarchy& h) {
  h.fw.prec = PrecReuse();
  for (auto& c : h.coarse) c->prec = PrecReuse();
}

static int single_level(Hierarchy& h, const Opts& o_in, spfas_stats& st) {
  prec_reset(h);
  double r = check_finite(fine_rnorm(h, h.fw.x.p, nullptr, 0.0), "initial residual");
  st.r0 = r;
  const double tol = std::max(o_in.rtol * r, o_in.atol);
  Opts o = o_in;
  o.stop_tol = tol;
  int rc = SPFAS_NOT_CONVERGED;
  for (int it = 0;; ++it) {
    if (r <= tol) { rc = SPFAS_OK; break; }
    if (it >= o.max_it) break;
    r = check_finite(fine_smooth(h, o, r, st), "residual after a smoothing step (divergence)");
    st.iterations++;
  }
  st.r_final = r;
  return rc;
}

__global__ void __launch_bounds__(kBlock) k_sub(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                                                double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = a[i] - b[i];
}

static void launch_sub(int64_t n, const double* a, const double* b, double* out, hipStream_t s) {
  if (!n) return;
  hipLaunchKernelGGL(k_sub, dim3(reduce_grid(n)), dim3(kBlock), 0, s, n, a, b, out);
  LAUNCHCHECK();
}

// ------------------------------------------------------------------ coarse levels

static double coarse_rnorm(Hierarchy& h, int l, const double* x, const double* dx, double step) {
  CoarseLevel& C = *h.coarse[l - 1];
  const int G = launch_coarse_resid(C, h.fine.kf, x, dx, step, C.b.p, nullptr, h.dpin, h.stream);
  return std::sqrt(h.host_sum(G));   // may be non-finite inside Alg. 1 trials
}

// ||r(x + s_t dx)|| on coarse level l for t < k in one pass (same values as
// coarse_rnorm at each step)
static void coarse_rnorm_trials(Hierarchy& h, int l, const double* x, const double* dx, const double* steps, int k,
                                double* out) {
  CoarseLevel& C = *h.coarse[l - 1];
  const int G = launch_coarse_resid_trials(C, h.fine.kf, x, dx, steps, k, C.b.p, h.dpin, h.stream);
  h.host_sums(G, k, out);
  for (int t = 0; t < k; ++t) out[t] = std::sqrt(out[t]);
}

// One Picard or Newton step on coarse level l (Section 3.3) with the linear
// system solved by algebraic hybridisation (Section 3.4), the cap on the
// aggregate-average pressure change and Alg. 1.
static double coarse_smooth(Hierarchy& h, int l, const Opts& o, double r_x, spfas_stats& st, bool* moved = nullptr) {
  if (moved) *moved = false;
  CoarseLevel& C = *h.coarse[l - 1];
  hipStream_t s = h.stream;
  const KappaFam& kf = h.fine.kf;
  const double t0 = trace_on() ? trace_clock(s) : 0.0;
  launch_coarse_resid(C, kf, C.x.p, nullptr, 0.0, C.b.p, C.r.p, h.parts.p, s);
  launch_coarse_local(C, kf, o.newton, C.x.p, C.r.p, s);
  int it = 0;
  if (C.nl > 0) {
    launch_H_assemble(C, s);
    const bool fresh = prec_refresh(C.amg, C.prec, o, s);
    Opts oc = o;
    oc.lin_max_it = o.lin_max_it_coarse;
    it = krylov_solve(C.kry, C.H, &C.amg, C.xi.p, C.lam.p, o.lin_rtol_coarse, oc, s);
    prec_record(C.prec, fresh, it, C.kry.failed);
    st.lin_iters += it;
  }
  double mx = HUGE_VAL;
  if (!(C.nl > 0 && C.kry.failed)) {
    const int G = launch_coarse_backsub(C, C.lam.p, C.dx.p, h.dpin, s);
    mx = h.host_max(G);
  }
  if (!std::isfinite(mx)) {   // non-finite local or hybridised solve: the step is rejected
    st.rejected_steps++;
    st.smoothing_steps++;
    if (trace_on()) std::fprintf(stderr, "[spfas] level %d: step rejected (non-finite linear solve)\n", l);
    return r_x;
  }
  const double scale = (o.cap > 0.0 && mx > o.cap) ? o.cap / mx : 1.0;
  double r_new = r_x;
  const NormBatch batch = [&](const double* sl, int k, double* out) {
    double st_[kMaxTrials];
    for (int t = 0; t < k; ++t) st_[t] = sl[t] * scale;
    coarse_rnorm_trials(h, l, C.x.p, C.dx.p, st_, k, out);
  };
  const double step = backtrack([&](double sl) { return coarse_rnorm(h, l, C.x.p, C.dx.p, sl * scale); }, r_x,
                                o.bt_nmax, o.bt_theta, r_new, st.bt_halvings, batch);
  if (step > 0.0) launch_axpy(C.nf + C.np, step * scale, C.dx.p, C.x.p, s);
  if (moved) *moved = step > 0.0;
  st.smoothing_steps++;
  if (trace_on())
    std::fprintf(stderr, "[spfas] level %d %s: multipliers %d (AMG levels %d, dense %d) krylov %d  |r| %.3e -> "
                 "%.3e  cap %.3g  step %.4g  %.2f ms %s\n", l, o.newton ? "newton" : "picard", C.nl, C.amg.n_levels(),
                 C.amg.nd, it, r_x, r_new, scale, step, trace_clock(s) - t0, C.amg.level_times().c_str());
  return r_new;
}

// Coarsest level (Section 4): at most coarsest_max smoothing steps, fewer
// when the level residual meets rtol (relative to its value on entry) or
// atol.  A step Alg. 1 rejected (or whose linear solve was not finite)
// leaves the state unchanged, so the next one would repeat it: the loop ends
// there.  A step Alg. 1 accepted while the residual rose does not end it.
static void coarsest_solve(Hierarchy& h, int l, const Opts& o, spfas_stats& st) {
  double r = coarse_rnorm(h, l, h.coarse[l - 1]->x.p, nullptr, 0.0);
  const double tol = std::max(o.rtol * r, o.coarsest_atol);
  for (int i = 0; i < o.coarsest_max; ++i) {
    if (r <= tol) break;
    bool moved = false;
    r = coarse_smooth(h, l, o, r, st, &moved);
    if (!moved) break;
  }
}

// Alg. 2 on level l.  The state of level l lives in fw.x (l = 0) or
// coarse[l-1]->x; its right-hand side in coarse[l-1]->b (level 0 uses
// b^0 = -[g; f]).  Returns after pre-smoothing on level 0 when the fine
// residual already meets stop_tol.
// r_in >= 0: the residual norm of the level's state on entry (not
// recomputed).  Returns the residual norm of the state on return (NaN on
// the coarsest level, which does not track it).
static double nonlinear_mg(Hierarchy& h, int l, const Opts& o, spfas_stats& st, double stop_tol, bool& stopped,
                           double r_in = -1.0) {
  hipStream_t s = h.stream;
  const int L = h.n_levels;
  if (l == L - 1) {
    coarsest_solve(h, l, o, st);
    return std::nan("");
  }
  FineWork& w = h.fw;
  FineDev& f = h.fine;
  const KappaFam& kf = f.kf;
  double* x = l == 0 ? w.x.p : h.coarse[l - 1]->x.p;
  double* dx = l == 0 ? w.dx.p : h.coarse[l - 1]->dx.p;
  double* r = l == 0 ? w.xt.p : h.coarse[l - 1]->r.p;
  double* div = l == 0 ? w.div.p : h.coarse[l - 1]->div.p;
  const int64_t nfl = l == 0 ? f.nf : h.coarse[l - 1]->nf;
  const int64_t nl = l == 0 ? f.nf + f.n : h.coarse[l - 1]->nf + h.coarse[l - 1]->np;
  // pre-smoothing
  double r_x = r_in >= 0.0 ? r_in : l == 0 ? fine_rnorm(h, x, nullptr, 0.0) : coarse_rnorm(h, l, x, nullptr, 0.0);
  double r_s = l == 0 ? fine_smooth(h, o, r_x, st) : coarse_smooth(h, l, o, r_x, st);
  if (l == 0 && r_s <= stop_tol) {
    stopped = true;
    return r_s;
  }
  // residual, projection and coarse right-hand side b^{l+1} = A^{l+1}(Q x) - R r^l
  if (l == 0) {
    launch_fine_resid(f.view(), x, nullptr, 0.0, r, h.parts.p, s);
    launch_div_fine(f.n, f.cfptr.p, f.cfcode.p, x, div, s);
  } else {
    CoarseLevel& C = *h.coarse[l - 1];
    launch_coarse_resid(C, kf, x, nullptr, 0.0, C.b.p, r, h.parts.p, s);
    launch_div_coarse(C, x, div, s);
  }
  CoarseLevel& Cc = *h.coarse[l];
  TransferDev& T = *h.trans[l];
  const int64_t nc = Cc.nf + Cc.np;
  launch_project(T, Cc, x, div, Cc.x.p, s);
  launch_copy(nc, Cc.x.p, Cc.x0.p, s);
  launch_restrict(T, Cc, r, Cc.b.p, s);
  launch_coarse_resid(Cc, kf, Cc.x.p, nullptr, 0.0, Cc.zeros.p, Cc.ax.p, h.parts.p, s);
  launch_sub(nc, Cc.ax.p, Cc.b.p, Cc.b.p, s);
  nonlinear_mg(h, l + 1, o, st, 0.0, stopped);
  // coarse correction P(y - Q x) with Alg. 1 on level l
  launch_sub(nc, Cc.x.p, Cc.x0.p, Cc.dx.p, s);
  launch_prolong(T, Cc, Cc.dx.p, dx, s);
  double r_new = r_s;
  auto rn = [&](double sl) {
    return l == 0 ? fine_rnorm(h, x, dx, sl) : coarse_rnorm(h, l, x, dx, sl);
  };
  NormBatch batch;
  if (l == 0) batch = [&](const double* sl, int k, double* out) { fine_rnorm_trials(h, x, dx, sl, k, out); };
  else batch = [&](const double* sl, int k, double* out) { coarse_rnorm_trials(h, l, x, dx, sl, k, out); };
  const double step = backtrack(rn, r_s, o.bt_nmax, o.bt_theta, r_new, st.bt_halvings, batch);
  if (step > 0.0) launch_axpy(nl, step, dx, x, s);
  (void)nfl;
  // post-smoothing
  return l == 0 ? fine_smooth(h, o, r_new, st) : coarse_smooth(h, l, o, r_new, st);
}

int run_fas(Hierarchy& h, const Opts& o_in, spfas_stats& st) {
  prec_reset(h);
  double r = check_finite(fine_rnorm(h, h.fw.x.p, nullptr, 0.0), "initial residual");
  st.r0 = r;
  const double tol = std::max(o_in.rtol * r, o_in.atol);
  Opts o = o_in;
  o.stop_tol = tol;
  int rc = SPFAS_NOT_CONVERGED;
  for (int it = 0;; ++it) {
    if (r <= tol) { rc = SPFAS_OK; break; }
    if (it >= o.max_it) break;
    bool stopped = false;
    const double t0 = trace_on() ? trace_clock(h.stream) : 0.0;
    // the V-cycle starts from the norm of the last one and returns that of
    // its final state (the norm Alg. 1 or the smoother evaluated there)
    r = check_finite(nonlinear_mg(h, 0, o, st, tol, stopped, r), "residual after a V-cycle (divergence)");
    st.stopped_after_presmooth = stopped ? 1 : 0;
    if (trace_on())
      std::fprintf(stderr, "[spfas] V-cycle %d: |r| %.3e (rel %.3e)  %.2f ms\n", it + 1, r, r / st.r0,
                   trace_clock(h.stream) - t0);
    st.iterations++;
  }
  st.r_final = r;
  return rc;
}

// Nonlinear cascadic multigrid (Section 4.2, Table 4).  The right-hand
// sides are restricted level by level, b^{l+1} = R b^l, which is the FAS
// right-hand side A^{l+1}(Q x) - R r^l(x) at the zero state (A^l(0) = 0 on
// every level, so r^l(0) = -b^l).  The coarsest problem is solved from zero;
// each finer level starts from the prolongated solution of the level below
// and takes smoothing steps until ||r^l|| <= max(rtol ||b^l||, atol) or
// max_it steps; like the coarsest level of the V-cycle, a level also stops
// after a rejected step (state unchanged).  The return code reports the
// fine level's test.
static int run_cascadic(Hierarchy& h, const Opts& o_in, spfas_stats& st, int32_t* level_steps) {
  prec_reset(h);
  hipStream_t s = h.stream;
  const int L = h.n_levels;
  FineWork& w = h.fw;
  FineDev& f = h.fine;
  const KappaFam& kf = f.kf;
  auto state = [&](int l) { return l == 0 ? w.x.p : h.coarse[l - 1]->x.p; };
  auto size = [&](int l) -> int64_t {
    return l == 0 ? f.nf + f.n : h.coarse[l - 1]->nf + h.coarse[l - 1]->np;
  };
  auto rnorm = [&](int l) {
    return l == 0 ? fine_rnorm(h, w.x.p, nullptr, 0.0) : coarse_rnorm(h, l, state(l), nullptr, 0.0);
  };
  // zero states; ||b^l|| = ||r^l(0)|| and b^{l+1} = -R r^l(0)
  std::vector<double> bnorm(L);
  w.x.zero(s);
  for (int l = 0; l < L; ++l) {
    bnorm[l] = check_finite(rnorm(l), "right-hand side");
    if (l + 1 == L) break;
    CoarseLevel& Cc = *h.coarse[l];
    double* r = l == 0 ? w.xt.p : h.coarse[l - 1]->r.p;
    if (l == 0) {
      launch_fine_resid(f.view(), w.x.p, nullptr, 0.0, r, h.parts.p, s);
    } else {
      CoarseLevel& C = *h.coarse[l - 1];
      launch_coarse_resid(C, kf, C.x.p, nullptr, 0.0, C.b.p, r, h.parts.p, s);
    }
    launch_restrict(*h.trans[l], Cc, r, Cc.b.p, s);
    launch_sub(Cc.nf + Cc.np, Cc.zeros.p, Cc.b.p, Cc.b.p, s);
    Cc.x.zero(s);
  }
  st.r0 = bnorm[0];
  int rc = SPFAS_NOT_CONVERGED;
  for (int l = L - 1; l >= 0; --l) {
    if (l + 1 < L) {   // initial guess P x^{l+1}
      launch_fill(size(l), 0.0, state(l), s);
      launch_prolong(*h.trans[l], *h.coarse[l], state(l + 1), state(l), s);
    }
    Opts o = o_in;
    const double tol = std::max(o.rtol * bnorm[l], o.atol);
    o.stop_tol = tol;
    double r = check_finite(rnorm(l), "residual of the prolongated state");
    int k = 0;
    while (k < o.max_it && r > tol) {
      bool moved = false;
      r = l == 0 ? fine_smooth(h, o, r, st, &moved) : coarse_smooth(h, l, o, r, st, &moved);
      check_finite(r, "residual after a smoothing step (divergence)");
      ++k;
      if (!moved) break;
    }
    if (level_steps) level_steps[l] = k;
    if (trace_on()) std::fprintf(stderr, "[spfas] cascadic level %d: %d steps, |r| %.3e (tol %.3e)\n", l, k, r, tol);
    if (l == 0) {
      st.iterations = k;
      st.r_final = r;
      rc = r <= tol ? SPFAS_OK : SPFAS_NOT_CONVERGED;
    }
  }
  return rc;
}

int run_solve(Hierarchy& h, const spfas_problem& prob, const spfas_solve_opts& so, double* p, double* sigma, bool dev,
              SolveKind kind, spfas_stats& st, int32_t* level_steps) {
  const bool multilevel = kind == SolveKind::FAS || kind == SolveKind::CASCADIC;
  const bool newton = kind == SolveKind::NEWTON || (multilevel && so.smoother == SPFAS_NEWTON);
  require(!multilevel || so.smoother == SPFAS_NEWTON || so.smoother == SPFAS_PICARD,
          "smoother must be SPFAS_NEWTON or SPFAS_PICARD");
  require(kind != SolveKind::CASCADIC || so.x0_given == 0,
          "the cascadic solve starts from zero on the coarsest level: x0_given must be 0");
  Opts o = make_opts(so, newton);
  h.set_problem(prob);
  load_state(h, p, sigma, dev, so.x0_given != 0);
  int rc;
  if (kind == SolveKind::CASCADIC)
    rc = run_cascadic(h, o, st, level_steps);
  else if (kind == SolveKind::FAS && h.n_levels > 1)
    rc = run_fas(h, o, st);
  else
    rc = single_level(h, o, st);
  store_state(h, prob, p, sigma, dev);
  return rc;
}

}  // namespace spfas
