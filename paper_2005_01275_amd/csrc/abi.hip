// C ABI of the library (include/spfas.h).  Every entry point catches the
// library's exceptions and turns them into status codes plus a
// thread-local message.
#include <chrono>
#include <cstring>
#include <string>

#include "hier.hpp"
#include "solve.hpp"

using namespace spfas;

struct spfas_hierarchy {
  Hierarchy h;
};

static thread_local std::string g_last_error = "";

static int set_error(int code, const char* msg) {
  g_last_error = msg;
  return code;
}

template <class F>
static int guarded(F&& fn) {
  try {
    g_last_error.clear();
    return fn();
  } catch (const Error& e) {
    return set_error(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return set_error(SPFAS_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return set_error(SPFAS_ERR_INVALID, e.what());
  }
}

extern "C" {

int spfas_version(void) { return SPFAS_API_VERSION; }

const char* spfas_last_error(void) { return g_last_error.c_str(); }

void spfas_default_solve_opts(spfas_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->smoother = SPFAS_NEWTON;
  o->rtol = 1e-8;
  o->atol = 1e-10;
  o->max_it = 50;
  o->bt_nmax = 4;
  o->bt_theta = 0.9;
  o->dp_cap = 0.0;
  o->coarsest_max_steps = 10;
  o->lin_rtol = 1e-8;
  o->lin_max_it = 500;
  o->x0_given = 0;
  o->lin_rtol_coarse = 0.0;
  o->lin_target = 0.0;
  o->newton_pcg = 0;
  o->amg_reuse = 0;
  o->lin_max_it_coarse = 0;
  o->coarsest_atol = -1.0;
  o->precision = SPFAS_PREC_FP64;
}

int spfas_setup_hierarchy(const spfas_mesh* mesh, const spfas_coarsen_opts* opts, const spfas_allocator* allocator,
                          void* stream, spfas_hierarchy** out) {
  return guarded([&] {
    require(mesh && opts && out, "NULL argument");
    require(!allocator || (allocator->alloc && allocator->free), "allocator: both callbacks are needed");
    auto* H = new spfas_hierarchy();
    try {
      if (allocator) H->h.mem.user = *allocator;
      H->h.use_stream((hipStream_t)stream);
      AllocScope scope(&H->h.mem);
      H->h.setup(*mesh, *opts);
    } catch (...) {
      delete H;
      throw;
    }
    *out = H;
    return SPFAS_OK;
  });
}

int spfas_hierarchy_device_bytes(const spfas_hierarchy* h, int64_t* bytes, int64_t* peak) {
  return guarded([&] {
    require(h != nullptr, "NULL hierarchy");
    if (bytes) *bytes = h->h.mem.bytes.load();
    if (peak) *peak = h->h.mem.peak.load();
    return SPFAS_OK;
  });
}

int spfas_hierarchy_reset_peak(spfas_hierarchy* h) {
  return guarded([&] {
    require(h != nullptr, "NULL hierarchy");
    h->h.mem.peak.store(h->h.mem.bytes.load());
    return SPFAS_OK;
  });
}

void spfas_destroy(spfas_hierarchy* h) {
  if (!h) return;
  try {
    if (!h->h.host_only) (void)hipStreamSynchronize(h->h.stream);
    delete h;
  } catch (...) {
  }
}

static void need_device(const spfas_hierarchy* h) {
  require(h != nullptr, "NULL hierarchy");
  require(!h->h.host_only, "this handle was built with host_only and has no device data");
}

int spfas_eval_residual(spfas_hierarchy* h, const spfas_problem* prob, const double* p, const double* sigma,
                        double* r_p, double* r_sigma, int32_t mem, void* stream) {
  return guarded([&] {
    need_device(h);
    require(prob && p && sigma && r_p && r_sigma, "NULL argument");
    h->h.use_stream((hipStream_t)stream);
    AllocScope scope(&h->h.mem);
    h->h.set_problem(*prob);
    h->h.eval_residual(p, sigma, r_p, r_sigma, mem == SPFAS_MEM_DEVICE);
    return SPFAS_OK;
  });
}

int spfas_eval_residual_noalloc(spfas_hierarchy* h, const spfas_problem* prob, const double* p,
                                const double* sigma, double* r_p, double* r_sigma, void* stream) {
  return guarded([&] {
    need_device(h);
    require(prob && p && sigma && r_p && r_sigma, "NULL argument");
    require(prob->mem == SPFAS_MEM_DEVICE, "spfas_eval_residual_noalloc needs the problem data in device memory");
    require(prob->shift == nullptr, "spfas_eval_residual_noalloc takes no kappa shift (its buffer would be allocated)");
    const int64_t nu = h->h.fine.nf + h->h.fine.n;
    if ((size_t)nu > noalloc_max_unknowns())
      fail(SPFAS_ERR_INVALID, "spfas_eval_residual_noalloc: " + std::to_string(nu) +
                                  " level-0 unknowns exceed the scratch capacity of " +
                                  std::to_string(noalloc_max_unknowns()));
    h->h.use_stream((hipStream_t)stream);
    h->h.set_problem(*prob);
    h->h.eval_residual_noalloc(p, sigma, r_p, r_sigma);
    return SPFAS_OK;
  });
}

static int solve_common(spfas_hierarchy* h, const spfas_problem* prob, const spfas_solve_opts* opts, double* p,
                        double* sigma, int32_t state_mem, spfas_stats* stats, void* stream, SolveKind kind,
                        int32_t* level_steps = nullptr) {
  return guarded([&] {
    need_device(h);
    require(prob && opts && p && sigma, "NULL argument");
    h->h.use_stream((hipStream_t)stream);
    AllocScope scope(&h->h.mem);
    auto t0 = std::chrono::steady_clock::now();
    spfas_stats st;
    std::memset(&st, 0, sizeof st);
    int rc = run_solve(h->h, *prob, *opts, p, sigma, state_mem == SPFAS_MEM_DEVICE, kind, st, level_steps);
    auto t1 = std::chrono::steady_clock::now();
    st.solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    if (stats) *stats = st;
    if (rc == SPFAS_NOT_CONVERGED) g_last_error = "maximum number of iterations reached";
    return rc;
  });
}

int spfas_fas_solve(spfas_hierarchy* h, const spfas_problem* prob, const spfas_solve_opts* opts, double* p,
                    double* sigma, int32_t state_mem, spfas_stats* stats, void* stream) {
  return solve_common(h, prob, opts, p, sigma, state_mem, stats, stream, SolveKind::FAS);
}

int spfas_picard_solve(spfas_hierarchy* h, const spfas_problem* prob, const spfas_solve_opts* opts, double* p,
                       double* sigma, int32_t state_mem, spfas_stats* stats, void* stream) {
  return solve_common(h, prob, opts, p, sigma, state_mem, stats, stream, SolveKind::PICARD);
}

int spfas_newton_solve(spfas_hierarchy* h, const spfas_problem* prob, const spfas_solve_opts* opts, double* p,
                       double* sigma, int32_t state_mem, spfas_stats* stats, void* stream) {
  return solve_common(h, prob, opts, p, sigma, state_mem, stats, stream, SolveKind::NEWTON);
}

int spfas_cascadic_solve(spfas_hierarchy* h, const spfas_problem* prob, const spfas_solve_opts* opts, double* p,
                         double* sigma, int32_t state_mem, spfas_stats* stats, int32_t* level_steps, void* stream) {
  return solve_common(h, prob, opts, p, sigma, state_mem, stats, stream, SolveKind::CASCADIC, level_steps);
}

int spfas_level_sizes(const spfas_hierarchy* h, int32_t level, int64_t* n_cells, int64_t* n_p, int64_t* n_flux) {
  return guarded([&] {
    require(h != nullptr, "NULL hierarchy");
    require(level >= 0 && level < (int)h->h.topo.size(), "level out of range");
    const Topo& t = h->h.topo[level];
    if (n_cells) *n_cells = t.n_cells;
    if (n_p) *n_p = t.n_p();
    if (n_flux) *n_flux = t.n_flux;
    return SPFAS_OK;
  });
}

int spfas_get_aggregation(const spfas_hierarchy* h, int32_t level, int32_t* agg) {
  return guarded([&] {
    require(h != nullptr && agg != nullptr, "NULL argument");
    require(level >= 0 && level + 1 < (int)h->h.topo.size(), "level must be below the coarsest level");
    const Topo& t = h->h.topo[level];
    for (int64_t i = 0; i < t.n_cells; ++i) agg[i] = (int32_t)t.agg[i];
    return SPFAS_OK;
  });
}

int spfas_get_permutation(const spfas_hierarchy* h, int32_t level, int32_t* cell_order, int32_t* flux_order) {
  return guarded([&] {
    require(h != nullptr && cell_order != nullptr && flux_order != nullptr, "NULL argument");
    require(level >= 0 && level + 1 < (int)h->h.topo.size(), "level must be below the coarsest level");
    const Topo& t = h->h.topo[level];
    for (int64_t i = 0; i < t.n_cells; ++i) cell_order[i] = (int32_t)t.cell_order[i];
    for (int64_t i = 0; i < t.n_flux; ++i) flux_order[i] = (int32_t)t.flux_order[i];
    return SPFAS_OK;
  });
}

int spfas_get_level_operator(const spfas_hierarchy* h, int32_t level, int32_t what, double* out, size_t count) {
  return guarded([&] {
    need_device(h);
    require(out != nullptr, "NULL output");
    require(level >= 0 && level + 1 < h->h.n_levels, "level must be below the coarsest level");
    AllocScope scope(const_cast<AllocCtx*>(&h->h.mem));
    export_level_operator(h->h, level, what, out, count);
    return SPFAS_OK;
  });
}

int spfas_profile_enable(spfas_hierarchy* h, int32_t enable) {
  return guarded([&] {
    need_device(h);
    h->h.prof.reset();
    h->h.prof.on = enable != 0;
    return SPFAS_OK;
  });
}

int spfas_profile_read(spfas_hierarchy* h, int32_t which, int64_t* launches, double* total_ms, double* algo_bytes) {
  return guarded([&] {
    need_device(h);
    require(which >= 0 && which < SPFAS_PROF_COUNT, "unknown kernel id");
    h->h.prof.collect();
    if (launches) *launches = h->h.prof.launches[which];
    if (total_ms) *total_ms = h->h.prof.ms[which];
    if (algo_bytes) *algo_bytes = h->h.prof.bytes[which];
    return SPFAS_OK;
  });
}

}  // extern "C"
