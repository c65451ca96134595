// The hierarchy handle: host topology of every level, device data of the
// fine level, the coarse levels and the transfers between them, and the
// solver state.  Built by spfas_setup_hierarchy, used by the solve entry
// points.
#pragma once

#include <memory>
#include <vector>

#include "coarse.hpp"
#include "common.hpp"
#include "fine.hpp"
#include "sparse.hpp"
#include "prof.hpp"
#include "topo.hpp"

namespace spfas {


struct FineDev {
  int64_t n = 0, nf = 0;
  DVec<int> K, L, cfptr, cfcode, nb;
  DVec<double> TKi, TLi, vol;
  DVec<int> cell_in, flux_in;             // internal -> input ids
  DVec<int> nptr, nface;                  // Neumann faces per internal cell (input face ids)
  DVec<double> narea;
  DVec<int> neu_in;                       // all Neumann faces (input ids)
  DVec<double> neu_area;
  DVec<double> f, g;                      // problem data of the current solve
  KappaFam kf;                            // kappa family of the current solve
  DVec<double> z;                         // its shift per internal cell (when has_shift)
  bool has_shift = false;
  FineView view() const {
    FineView v;
    v.n = n; v.nf = nf; v.kf = kf; v.z = has_shift ? z.p : nullptr;
    v.K = K.p; v.L = L.p; v.TKi = TKi.p; v.TLi = TLi.p; v.g = g.p; v.f = f.p;
    v.cfptr = cfptr.p; v.cfcode = cfcode.p;
    return v;
  }
};

// Work space of the fine-level smoother: state, step, eliminated system
// S dp = rhs (S shares the pattern of the cell->face lists), its AMG and
// Krylov workspaces.
struct FineWork {
  DVec<double> x, dx, xt;                 // [nf + n]; xt holds r(x) in the V-cycle
  DVec<double> div;                       // [n] D sigma (projection of bubbles)
  DVec<double> Sdiag, Soff, rhs;          // S = D M^{-1} E, right-hand side
  Amg amg;
  PrecReuse prec;
  Krylov kry;
  CsrView S;
  // mixed precision: FP32 copy of S in the SELL layout, FP32 right-hand
  // side and correction, FP32 Krylov vectors
  Krylov32 kry32;
  DVec<float> sval32, rhs32, dp32;
  Sell32View S32;
};

struct Hierarchy {
  // first member: destroyed after every buffer that returns memory to it
  AllocCtx mem;
  hipStream_t stream = nullptr;
  int device = -1;                        // device current at setup
  bool host_only = false;
  int dim = 0;
  int64_t n_cells_in = 0, n_faces_in = 0;
  int n_levels = 1;
  int m = 1;
  std::vector<Topo> topo;                 // canonical topology per level
  std::vector<TransferPlan> plans;        // host plans l -> l+1
  FineDev fine;
  FineWork fw;
  std::vector<std::unique_ptr<CoarseLevel>> coarse;   // levels 1..L-1
  std::vector<std::unique_ptr<TransferDev>> trans;    // transfers 0..L-2
  // host copies of hierarchy numbers for the parity hooks
  std::vector<std::vector<double>> eigvals;           // per transfer, concatenated
  // reduction scratch: partials that stay on the device, and partials the
  // host adds up, which the kernels write straight into coherent host-mapped
  // memory (hpin on the host, dpin its device address: no copy launch)
  DVec<double> parts;
  double* hpin = nullptr;
  double* dpin = nullptr;
  int launches = 0;
  KernelProf prof;                         // event timing of instrumented kernels

  // coarsening options of the setup (the threshold count rebuilds coarse
  // topologies level by level during setup_coarse_levels)
  spfas_coarsen_opts copts{};
  std::vector<int64_t> user_off;          // USER: offset of level l's ids in user_agg

  ~Hierarchy();
  void setup(const spfas_mesh& mesh, const spfas_coarsen_opts& o);
  // aggregates and renumbers topo[l] by the coarsening options
  void aggregate_level(int l);
  // replaces topo[l+1] by the coarse topology of topo[l] with mA[A]
  // eigenvectors per aggregate, aggregates and renumbers it when a coarser
  // level follows, and rebuilds topo[l+2] with the uniform provisional count
  void rebuild_coarse_topology(int l, const std::vector<int64_t>& mA);
  // stream of the current call, also handed to the allocator callbacks
  void use_stream(hipStream_t s) { stream = s; mem.stream = s; }
  void set_problem(const spfas_problem& prob);
  // fine residual in input order
  void eval_residual(const double* p, const double* sig, double* rp, double* rs, bool dev);
  // the same on device arrays, staging through a static device array
  // instead of allocating (noalloc.hip)
  void eval_residual_noalloc(const double* p, const double* sig, double* rp, double* rs);
  // wait for the stream, then the sum (max) of the n partials at dpin, in
  // index order
  double host_sum(int n);
  double host_max(int n);
  // k sums of n consecutive partials each (one wait)
  void host_sums(int n, int k, double* out);
};

// capacity of eval_residual_noalloc in level-0 unknowns (flux + cells)
size_t noalloc_max_unknowns();

}  // namespace spfas
