// Serving runtime: continuous batching of solve requests over a cache of
// device-resident hierarchies (include/spfas.h, "Serving").
//
// A fixed set of worker threads, each with its own HIP stream, takes
// requests from one queue.  A request is admitted as soon as a worker is
// free and its model's hierarchy is cached and idle, or there is room under
// the device-memory budget to build it (idle hierarchies of other models
// are evicted, least recently used first, to make room).  Requests that
// cannot be admitted yet do not hold back later ones.  Each solve runs
// entirely on its worker's stream, so solves of different requests overlap
// on the GPU; a request's arithmetic does not depend on what else is in
// flight (its hierarchy is used by one solve at a time and every reduction
// has a fixed order), so its result is the same alone and in the mix.
//
// The server is a client of the library's own C ABI: hierarchies are built
// with spfas_setup_hierarchy and solved with the solve entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "common.hpp"

using namespace spfas;

namespace {

struct Instance {
  spfas_hierarchy* h = nullptr;
  bool busy = false;
  bool building = false;
  uint64_t last_used = 0;
  int64_t bytes = 0;              // device bytes reserved now (held, plus a running solve's temporaries)
  int64_t solve_extra = 0;        // measured temporaries of a solve beyond what the hierarchy holds
};

struct Model {
  int64_t id = 0;
  int32_t dim = 0;
  int64_t n_cells = 0, n_faces = 0;
  std::vector<double> vol, cen, k0, area, nrm, pt;
  std::vector<int32_t> fc;
  std::vector<int8_t> kind;
  spfas_coarsen_opts co{};
  std::vector<int32_t> user_agg;
  int64_t est_bytes = 0;          // device bytes of one instance (measured after the first build)
  bool measured = false;
  std::unique_ptr<Instance> inst;   // at most one cached hierarchy per model
  spfas_mesh mesh() const {
    spfas_mesh m;
    m.dim = dim;
    m.n_cells = n_cells;
    m.n_faces = n_faces;
    m.cell_volume = vol.data();
    m.cell_centroid = cen.data();
    m.cell_k0 = k0.data();
    m.face_cells = fc.data();
    m.face_area = area.data();
    m.face_normal = nrm.data();
    m.face_point = pt.data();
    m.face_kind = kind.data();
    return m;
  }
};

struct Request {
  int64_t ticket = 0;
  int64_t model = 0;
  int32_t kind = SPFAS_SOLVE_FAS;
  double alpha = 0.0;
  int32_t kappa_kind = SPFAS_KAPPA_EXP;
  double kappa_a = 1.0, kappa_beta = 2.0;
  std::vector<double> src, gd, gn, shift;
  bool has_gd = false, has_gn = false, has_shift = false;
  spfas_solve_opts opts{};
  std::vector<double> p, sigma;
  spfas_stats st{};
  int rc = SPFAS_OK;
  std::string err;
  double t_submit = 0, t_start = 0, t_solve = 0, t_end = 0;
  bool cache_hit = false;
  bool done = false;
};

}  // namespace

struct spfas_server {
  spfas_server_opts o{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::map<int64_t, std::unique_ptr<Model>> models;
  std::deque<Request*> queue;
  std::map<int64_t, std::unique_ptr<Request>> reqs;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  bool stop = false;
  int64_t next_model = 0, next_ticket = 0;
  uint64_t clock = 0;
  int64_t used = 0;                // device bytes reserved by cached instances
  spfas_server_counters cnt{};

  // Evicts idle instances (least recently used first) until `need` more
  // bytes fit under the budget; false if that is impossible now.
  bool make_room(int64_t need, const Model* keep) {
    while (used + need > o.hbm_budget) {
      Model* victim = nullptr;
      for (auto& kv : models) {
        Model* m = kv.second.get();
        if (m == keep || !m->inst || m->inst->busy) continue;
        if (!victim || m->inst->last_used < victim->inst->last_used) victim = m;
      }
      if (!victim) return false;
      used -= victim->inst->bytes;
      spfas_destroy(victim->inst->h);
      victim->inst.reset();
      cnt.evictions++;
    }
    return true;
  }

  // First admissible request in arrival order (caller holds the lock).  A
  // request whose model cannot fit under the budget even with every other
  // hierarchy evicted is completed at once with ERR_OOM.
  Request* admit() {
    for (auto it = queue.begin(); it != queue.end();) {
      Request* r = *it;
      Model* m = models.at(r->model).get();
      if (!m->inst && m->est_bytes > o.hbm_budget) {
        r->rc = SPFAS_ERR_OOM;
        r->err = "the model's hierarchy needs " + std::to_string(m->est_bytes) + " bytes, more than the budget of " +
                 std::to_string(o.hbm_budget);
        r->t_start = r->t_solve = r->t_end = wall_ms();
        r->done = true;
        cnt.completed++;
        it = queue.erase(it);
        cv_done.notify_all();
        continue;
      }
      if (m->inst) {
        if (m->inst->busy) { ++it; continue; }
        const int64_t extra = m->inst->solve_extra;
        if (extra > 0 && !make_room(extra, m)) { ++it; continue; }
        used += extra;
        m->inst->bytes += extra;
        m->inst->busy = true;
        r->cache_hit = true;
      } else {
        if (!make_room(m->est_bytes, m)) { ++it; continue; }
        m->inst = std::make_unique<Instance>();
        m->inst->busy = true;
        m->inst->building = true;
        m->inst->bytes = m->est_bytes;
        used += m->est_bytes;
        r->cache_hit = false;
      }
      queue.erase(it);
      return r;
    }
    return nullptr;
  }

  void work(int w) {
    hipStream_t s = streams[w];
    (void)hipSetDevice(o.device);
    // this worker's share of the host threads for the setups it runs
    tl_host_threads = std::max(1, kMaxHostThreads / std::max(1, o.n_slots));
    for (;;) {
      Request* r = nullptr;
      Model* m = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stop || (r = admit()) != nullptr; });
        if (!r) return;
        m = models.at(r->model).get();
        r->t_start = wall_ms();
      }
      Instance* in = m->inst.get();
      int rc = SPFAS_OK;
      std::string err;
      int64_t build_peak = 0;
      if (in->building) {
        const spfas_mesh mesh = m->mesh();
        spfas_hierarchy* h = nullptr;
        rc = spfas_setup_hierarchy(&mesh, &m->co, nullptr, (void*)s, &h);
        if (rc < 0) err = spfas_last_error();
        in->h = h;
        if (h) spfas_hierarchy_device_bytes(h, nullptr, &build_peak);
      }
      // the solve's own peak (the setup's scratch is gone by now)
      int64_t held0 = 0;
      if (in->h) {
        spfas_hierarchy_reset_peak(in->h);
        spfas_hierarchy_device_bytes(in->h, &held0, nullptr);
      }
      r->t_solve = wall_ms();
      if (rc >= 0) {
        spfas_problem pb;
        pb.alpha = r->alpha;
        pb.source = r->src.data();
        pb.g_dirichlet = r->has_gd ? r->gd.data() : nullptr;
        pb.g_neumann = r->has_gn ? r->gn.data() : nullptr;
        pb.mem = SPFAS_MEM_HOST;
        pb.kappa_kind = r->kappa_kind;
        pb.kappa_a = r->kappa_a;
        pb.kappa_beta = r->kappa_beta;
        pb.shift = r->has_shift ? r->shift.data() : nullptr;
        r->p.assign(m->n_cells, 0.0);
        r->sigma.assign(m->n_faces, 0.0);
        switch (r->kind) {
          case SPFAS_SOLVE_NEWTON:
            rc = spfas_newton_solve(in->h, &pb, &r->opts, r->p.data(), r->sigma.data(), SPFAS_MEM_HOST, &r->st, s);
            break;
          case SPFAS_SOLVE_PICARD:
            rc = spfas_picard_solve(in->h, &pb, &r->opts, r->p.data(), r->sigma.data(), SPFAS_MEM_HOST, &r->st, s);
            break;
          default:
            rc = spfas_fas_solve(in->h, &pb, &r->opts, r->p.data(), r->sigma.data(), SPFAS_MEM_HOST, &r->st, s);
        }
        if (rc != SPFAS_OK) err = spfas_last_error();
      }
      int64_t bytes = 0, peak = 0;
      if (in->h) spfas_hierarchy_device_bytes(in->h, &bytes, &peak);
      {
        std::lock_guard<std::mutex> lk(mu);
        if (in->building) {
          cnt.setups++;
          in->building = false;
        } else {
          cnt.cache_hits++;
        }
        if (!in->h) {   // the build failed: release the reservation
          used -= in->bytes;
          m->inst.reset();
        } else {
          // idle, the instance holds `bytes`; a later solve reserves its
          // temporaries on top, a rebuild the larger of the build's and the
          // solve's peaks
          used += bytes - in->bytes;
          in->bytes = bytes;
          in->solve_extra = std::max(in->solve_extra, std::max<int64_t>(0, peak - std::min(held0, bytes)));
          const int64_t need = std::max(build_peak, peak);
          if (!m->measured || need > m->est_bytes) m->est_bytes = need;
          m->measured = true;
          in->busy = false;
          in->last_used = ++clock;
        }
        cnt.peak_bytes = std::max(cnt.peak_bytes, used);
        r->rc = rc;
        r->err = err;
        r->t_end = wall_ms();
        r->done = true;
        cnt.completed++;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

static thread_local std::string g_server_error;

static int server_fail(int code, const std::string& msg) {
  g_server_error = msg;
  return code;
}

extern "C" {

const char* spfas_server_last_error(void) { return g_server_error.c_str(); }

int spfas_server_create(const spfas_server_opts* opts, spfas_server** out) {
  if (!opts || !out) return server_fail(SPFAS_ERR_INVALID, "NULL argument");
  if (opts->n_slots < 1 || opts->n_slots > 64) return server_fail(SPFAS_ERR_INVALID, "n_slots must be in [1, 64]");
  auto* S = new spfas_server();
  S->o = *opts;
  if (hipSetDevice(opts->device) != hipSuccess) {
    delete S;
    return server_fail(SPFAS_ERR_DEVICE, "hipSetDevice failed");
  }
  if (S->o.hbm_budget <= 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      delete S;
      return server_fail(SPFAS_ERR_DEVICE, "hipMemGetInfo failed");
    }
    S->o.hbm_budget = (int64_t)(0.8 * (double)fr);
  }
  for (int w = 0; w < opts->n_slots; ++w) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : S->streams) (void)hipStreamDestroy(x);
      delete S;
      return server_fail(SPFAS_ERR_DEVICE, "hipStreamCreate failed");
    }
    S->streams.push_back(s);
  }
  for (int w = 0; w < opts->n_slots; ++w) S->workers.emplace_back([S, w] { S->work(w); });
  *out = S;
  return SPFAS_OK;
}

int spfas_server_add_model(spfas_server* S, const spfas_mesh* mesh, const spfas_coarsen_opts* co, int64_t* model_id) {
  if (!S || !mesh || !co || !model_id) return server_fail(SPFAS_ERR_INVALID, "NULL argument");
  if (co->host_only) return server_fail(SPFAS_ERR_INVALID, "a served model needs device hierarchies (host_only = 0)");
  if (mesh->n_cells <= 0 || mesh->n_faces < 0 || (mesh->dim != 2 && mesh->dim != 3))
    return server_fail(SPFAS_ERR_INVALID, "malformed mesh sizes");
  auto m = std::make_unique<Model>();
  const int d = mesh->dim;
  const int64_t n = mesh->n_cells, nf = mesh->n_faces;
  m->dim = d;
  m->n_cells = n;
  m->n_faces = nf;
  m->vol.assign(mesh->cell_volume, mesh->cell_volume + n);
  m->cen.assign(mesh->cell_centroid, mesh->cell_centroid + n * d);
  m->k0.assign(mesh->cell_k0, mesh->cell_k0 + n * d * d);
  m->fc.assign(mesh->face_cells, mesh->face_cells + 2 * nf);
  m->area.assign(mesh->face_area, mesh->face_area + nf);
  m->nrm.assign(mesh->face_normal, mesh->face_normal + nf * d);
  m->pt.assign(mesh->face_point, mesh->face_point + nf * d);
  m->kind.assign(mesh->face_kind, mesh->face_kind + nf);
  m->co = *co;
  if (co->agg_kind == SPFAS_AGG_USER) {
    if (!co->user_agg || co->user_agg_len <= 0) return server_fail(SPFAS_ERR_INVALID, "USER aggregation without user_agg");
    m->user_agg.assign(co->user_agg, co->user_agg + co->user_agg_len);
    m->co.user_agg = m->user_agg.data();
  }
  // footprint until the first build measures it: a bound from the sizes
  // (about 3 KB per cell and 1 KB per face covers the hierarchies of the
  // box-aggregated meshes measured so far, plus fixed per-hierarchy buffers)
  m->est_bytes = 3072 * n + 1024 * nf + (16 << 20);
  std::lock_guard<std::mutex> lk(S->mu);
  m->id = S->next_model++;
  *model_id = m->id;
  S->models[m->id] = std::move(m);
  return SPFAS_OK;
}

int spfas_server_submit(spfas_server* S, int64_t model_id, const spfas_problem* prob, const spfas_solve_opts* opts,
                        int32_t kind, int64_t* ticket) {
  if (!S || !prob || !opts || !ticket) return server_fail(SPFAS_ERR_INVALID, "NULL argument");
  if (prob->mem != SPFAS_MEM_HOST) return server_fail(SPFAS_ERR_INVALID, "served problems are passed in host memory");
  if (!prob->source) return server_fail(SPFAS_ERR_INVALID, "problem.source must not be NULL");
  if (kind != SPFAS_SOLVE_FAS && kind != SPFAS_SOLVE_NEWTON && kind != SPFAS_SOLVE_PICARD)
    return server_fail(SPFAS_ERR_INVALID, "kind must be SPFAS_SOLVE_FAS, _NEWTON or _PICARD");
  if (opts->x0_given) return server_fail(SPFAS_ERR_INVALID, "served solves start from zero (x0_given must be 0)");
  auto r = std::make_unique<Request>();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->models.find(model_id);
    if (it == S->models.end()) return server_fail(SPFAS_ERR_INVALID, "unknown model id");
    const Model& m = *it->second;
    r->src.assign(prob->source, prob->source + m.n_cells);
    if (prob->g_dirichlet) { r->gd.assign(prob->g_dirichlet, prob->g_dirichlet + m.n_faces); r->has_gd = true; }
    if (prob->g_neumann) { r->gn.assign(prob->g_neumann, prob->g_neumann + m.n_faces); r->has_gn = true; }
    if (prob->shift) { r->shift.assign(prob->shift, prob->shift + m.n_cells); r->has_shift = true; }
    r->kappa_kind = prob->kappa_kind;
    r->kappa_a = prob->kappa_a;
    r->kappa_beta = prob->kappa_beta;
    r->model = model_id;
    r->kind = kind;
    r->alpha = prob->alpha;
    r->opts = *opts;
    r->ticket = S->next_ticket++;
    r->t_submit = wall_ms();
    *ticket = r->ticket;
    S->queue.push_back(r.get());
    S->reqs[r->ticket] = std::move(r);
    S->cnt.submitted++;
  }
  S->cv_work.notify_one();
  return SPFAS_OK;
}

int spfas_server_wait(spfas_server* S, int64_t ticket, double* p, double* sigma, spfas_stats* stats,
                      spfas_request_info* info) {
  if (!S) return server_fail(SPFAS_ERR_INVALID, "NULL server");
  std::unique_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return server_fail(SPFAS_ERR_INVALID, "unknown or already collected ticket");
    Request* rr = it->second.get();
    S->cv_done.wait(lk, [&] { return rr->done; });
    r = std::move(it->second);
    S->reqs.erase(it);
  }
  if (info) {
    info->queue_ms = r->t_start - r->t_submit;
    info->setup_ms = r->t_solve - r->t_start;
    info->solve_ms = r->t_end - r->t_solve;
    info->total_ms = r->t_end - r->t_submit;
    info->cache_hit = r->cache_hit ? 1 : 0;
  }
  if (r->rc < 0) return server_fail(r->rc, r->err);
  if (p) std::memcpy(p, r->p.data(), r->p.size() * sizeof(double));
  if (sigma) std::memcpy(sigma, r->sigma.data(), r->sigma.size() * sizeof(double));
  if (stats) *stats = r->st;
  if (r->rc == SPFAS_NOT_CONVERGED) g_server_error = r->err;
  return r->rc;
}

int spfas_server_counters_get(spfas_server* S, spfas_server_counters* c) {
  if (!S || !c) return server_fail(SPFAS_ERR_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  *c = S->cnt;
  c->cached_bytes = S->used;
  c->budget_bytes = S->o.hbm_budget;
  return SPFAS_OK;
}

void spfas_server_destroy(spfas_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto& t : S->workers) t.join();
  for (auto& kv : S->models)
    if (kv.second->inst && kv.second->inst->h) spfas_destroy(kv.second->inst->h);
  for (auto s : S->streams) (void)hipStreamDestroy(s);
  delete S;
}

}  // extern "C"
