// Hierarchy setup (host orchestration) and fine-level entry points.
#include "hier.hpp"

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <numeric>

#include "coarse.hpp"
#include "coarse_kern.hpp"
#include "kern.hpp"
#include "solve.hpp"
#include "sparse.hpp"

namespace spfas {

__global__ void k_invgather(int64_t n, const int* __restrict__ map, const double* __restrict__ T,
                            const int* __restrict__ L, int use_L, double* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (use_L && L[i] < 0) { out[i] = 0.0; return; }
  out[i] = 1.0 / T[map[i]];
}

Hierarchy::~Hierarchy() {
  coarse.clear();
  trans.clear();
  if (hpin) (void)hipHostFree(hpin);
}

double Hierarchy::host_sum(int n) {
  HIPCHECK(hipStreamSynchronize(stream));
  const volatile double* v = hpin;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += v[i];
  return s;
}

void Hierarchy::host_sums(int n, int k, double* out) {
  require((size_t)n * k <= (size_t)kMaxParts * 4, "too many partial sums");
  HIPCHECK(hipStreamSynchronize(stream));
  const volatile double* v = hpin;
  for (int t = 0; t < k; ++t) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += v[(size_t)t * n + i];
    out[t] = s;
  }
}

double Hierarchy::host_max(int n) {
  HIPCHECK(hipStreamSynchronize(stream));
  const volatile double* v = hpin;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s = std::max(s, (double)v[i]);
  return s;
}

static void validate_mesh(const spfas_mesh& M, const spfas_coarsen_opts& o) {
  require(M.dim == 2 || M.dim == 3, "mesh.dim must be 2 or 3");
  require(M.n_cells > 0, "mesh.n_cells must be positive");
  require(M.n_faces >= 0, "mesh.n_faces must be non-negative");
  require(M.n_cells < (int64_t)1 << 30 && M.n_faces < (int64_t)1 << 30, "mesh too large for 32-bit indices");
  require(M.cell_volume && M.cell_centroid && M.cell_k0 && M.face_cells && M.face_area && M.face_normal &&
              M.face_point && M.face_kind,
          "mesh arrays must not be NULL");
  require(o.n_levels >= 1 && o.n_levels <= 16, "n_levels must be in [1, 16]");
  require(o.m >= 1 && o.m <= 64, "m must be in [1, 64]");
  require(o.m_f == 0 || o.m_f == 1, "m_f must be 1 (one flux unknown per coarse interface; more are not built)");
  if (o.agg_kind == SPFAS_AGG_BOX)
    for (int a = 0; a < M.dim; ++a) require(o.box[a] >= 1, "box edges must be >= 1");
  int64_t ndir = 0;
  for (int64_t c = 0; c < M.n_cells; ++c)
    require(M.cell_volume[c] > 0.0 && std::isfinite(M.cell_volume[c]), "cell volumes must be positive");
  for (int64_t i = 0; i < M.n_cells * M.dim; ++i)
    require(std::isfinite(M.cell_centroid[i]), "cell centroids must be finite");
  for (int64_t f = 0; f < M.n_faces; ++f) {
    const int K = M.face_cells[2 * f], L = M.face_cells[2 * f + 1];
    const int k = M.face_kind[f];
    require(K >= 0 && K < M.n_cells, "face_cells: K out of range");
    require(L >= -1 && L < M.n_cells, "face_cells: L out of range");
    require(k >= 0 && k <= 2, "face_kind must be 0, 1 or 2");
    require((k == SPFAS_FACE_INTERIOR) == (L >= 0), "interior faces need L >= 0, boundary faces L = -1");
    require(L != K, "a face must join two different cells");
    require(M.face_area[f] > 0.0 && std::isfinite(M.face_area[f]), "face areas must be positive and finite");
    ndir += (k == SPFAS_FACE_DIRICHLET);
  }
  require(ndir > 0, "at least one Dirichlet face is required");
}

void Hierarchy::setup(const spfas_mesh& M, const spfas_coarsen_opts& o) {
  const double t_start = wall_ms();
  validate_mesh(M, o);
  dim = M.dim;
  n_cells_in = M.n_cells;
  n_faces_in = M.n_faces;
  n_levels = o.n_levels;
  m = o.m;
  host_only = o.host_only != 0;
  if (!host_only) HIPCHECK(hipGetDevice(&device));
  // ---------------- level-0 canonical topology
  topo.clear();
  topo.reserve(n_levels);   // references into topo stay valid below
  topo.emplace_back();
  Topo& t0 = topo[0];
  t0.n_cells = M.n_cells;
  t0.pptr.resize(M.n_cells + 1);
  std::iota(t0.pptr.begin(), t0.pptr.end(), 0);
  std::vector<int64_t> flux_face;
  for (int64_t f = 0; f < M.n_faces; ++f) {
    if (M.face_kind[f] == SPFAS_FACE_NEUMANN) continue;
    flux_face.push_back(f);
    t0.kind.push_back(M.face_kind[f] == SPFAS_FACE_DIRICHLET ? FK_DIRICHLET : FK_INTERIOR);
    t0.c1.push_back(M.face_cells[2 * f]);
    t0.c2.push_back(M.face_cells[2 * f + 1]);
  }
  t0.n_flux = (int64_t)flux_face.size();
  const bool trace = trace_level() > 0;
  auto stamp = [&](const char* what) {
    if (trace)
      std::fprintf(stderr, "[spfas] setup host: %s at %.1f ms\n", what, wall_ms() - t_start);
  };
  stamp("level-0 face lists");
  build_cell_lists(t0);
  stamp("cell lists");
  require(o.agg_kind == SPFAS_AGG_BOX || o.agg_kind == SPFAS_AGG_USER || o.agg_kind == SPFAS_AGG_GREEDY,
          "agg_kind must be SPFAS_AGG_BOX, SPFAS_AGG_USER or SPFAS_AGG_GREEDY");
  if (n_levels > 1 && o.agg_kind == SPFAS_AGG_BOX) {
    bool ok = lattice_from_centroids(M.dim, M.n_cells, M.cell_centroid, t0.lat_shape, t0.lat_index);
    require(ok, "box aggregation needs a Cartesian lattice of cell centroids");
  }
  stamp("lattice");
  // ---------------- coarse topologies, aggregation, renumbering
  copts = o;
  if (o.eig_threshold > 0.0) {
    require(std::isfinite(o.eig_threshold), "eig_threshold must be finite");
    require(o.m_min >= 1 && o.m_min <= o.m, "m_min must be in [1, m]");
    require(!host_only, "eig_threshold needs the device setup (not host_only)");
  }
  // with the threshold count the coarse topologies built here are
  // provisional (min(m, unknowns) per aggregate); setup_coarse_levels
  // replaces each before its numerics
  user_off.assign(n_levels, 0);
  for (int l = 0; l + 1 < n_levels; ++l) {
    if (l > 0) user_off[l] = user_off[l - 1] + topo[l - 1].n_cells;
    aggregate_level(l);
    stamp("aggregation, renumbering");
    Topo c = coarse_topology(topo[l], m);
    topo.push_back(std::move(c));
    stamp("coarse topology");
  }
  if (trace_level() > 0)
    std::fprintf(stderr, "[spfas] setup: host topology, aggregation, renumbering %.1f ms\n", wall_ms() - t_start);
  if (host_only) return;
  HIPCHECK(hipHostMalloc((void**)&hpin, kMaxParts * sizeof(double) * 4, hipHostMallocMapped | hipHostMallocCoherent));
  HIPCHECK(hipHostGetDevicePointer((void**)&dpin, hpin, 0));
  parts.alloc(kMaxParts * 4);
  // ---------------- level-0 device order
  const int64_t n = M.n_cells, nf = t0.n_flux;
  std::vector<int64_t> corder(n), forder(nf);
  if (n_levels > 1) {
    corder = t0.cell_order;
    forder = t0.flux_order;
  } else {
    std::iota(corder.begin(), corder.end(), 0);
    std::iota(forder.begin(), forder.end(), 0);
  }
  std::vector<int64_t> cpos(n), fpos(nf);
  for (int64_t i = 0; i < n; ++i) cpos[corder[i]] = i;
  for (int64_t i = 0; i < nf; ++i) fpos[forder[i]] = i;
  fine.n = n;
  fine.nf = nf;
  hipStream_t s = stream;
  {
    std::vector<int> cell_in(n), flux_in(nf), K(nf), L(nf);
    std::vector<double> vol(n);
    for (int64_t i = 0; i < n; ++i) { cell_in[i] = (int)corder[i]; vol[i] = M.cell_volume[corder[i]]; }
    for (int64_t i = 0; i < nf; ++i) {
      const int64_t j = forder[i];
      flux_in[i] = (int)flux_face[j];
      K[i] = (int)cpos[t0.c1[j]];
      L[i] = t0.c2[j] >= 0 ? (int)cpos[t0.c2[j]] : -1;
    }
    // cell -> face lists in internal order
    std::vector<int> cfptr(n + 1, 0);
    for (int64_t i = 0; i < nf; ++i) {
      cfptr[K[i] + 1]++;
      if (L[i] >= 0) cfptr[L[i] + 1]++;
    }
    for (int64_t c = 0; c < n; ++c) cfptr[c + 1] += cfptr[c];
    std::vector<int> cfcode(cfptr[n]), nb(cfptr[n]);
    std::vector<int> fill(cfptr.begin(), cfptr.end() - 1);
    for (int64_t i = 0; i < nf; ++i) {
      cfcode[fill[K[i]]] = (int)(i << 1);
      nb[fill[K[i]]++] = L[i] >= 0 ? L[i] : K[i];
      if (L[i] >= 0) {
        cfcode[fill[L[i]]] = (int)((i << 1) | 1);
        nb[fill[L[i]]++] = K[i];
      }
    }
    // Neumann faces per internal cell
    std::vector<int> nptr(n + 1, 0), nface, neu_in;
    std::vector<double> narea, neu_area;
    std::vector<std::vector<int>> per(n);
    for (int64_t f = 0; f < M.n_faces; ++f)
      if (M.face_kind[f] == SPFAS_FACE_NEUMANN) {
        per[cpos[M.face_cells[2 * f]]].push_back((int)f);
        neu_in.push_back((int)f);
        neu_area.push_back(M.face_area[f]);
      }
    for (int64_t c = 0; c < n; ++c) {
      for (int f : per[c]) { nface.push_back(f); narea.push_back(M.face_area[f]); }
      nptr[c + 1] = (int)nface.size();
    }
    fine.cell_in.upload(cell_in, s);
    fine.flux_in.upload(flux_in, s);
    fine.K.upload(K, s);
    fine.L.upload(L, s);
    fine.cfptr.upload(cfptr, s);
    fine.cfcode.upload(cfcode, s);
    fine.nb.upload(nb, s);
    fine.vol.upload(vol, s);
    fine.nptr.upload(nptr, s);
    fine.nface.upload(nface, s);
    fine.narea.upload(narea, s);
    fine.neu_in.upload(neu_in, s);
    fine.neu_area.upload(neu_area, s);
    HIPCHECK(hipStreamSynchronize(s));
  }
  // ---------------- half-transmissibilities (device, input order -> internal)
  {
    DVec<int> fc;
    DVec<double> area, nrm, pt, cen, k0, TK, TL;
    DVec<int> bad;
    cen.upload(M.cell_centroid, M.n_cells * dim, s);
    k0.upload(M.cell_k0, M.n_cells * dim * dim, s);
    bad.alloc(1);
    bad.zero(s);
    // evaluate on the non-Neumann faces only (the ones that carry a flux)
    std::vector<int> fcs(2 * nf);
    std::vector<double> ar(nf), nr(nf * dim), pp(nf * dim);
    for (int64_t j = 0; j < nf; ++j) {
      const int64_t f = flux_face[j];
      fcs[2 * j] = M.face_cells[2 * f];
      fcs[2 * j + 1] = M.face_cells[2 * f + 1];
      ar[j] = M.face_area[f];
      for (int a = 0; a < dim; ++a) { nr[j * dim + a] = M.face_normal[f * dim + a]; pp[j * dim + a] = M.face_point[f * dim + a]; }
    }
    fc.upload(fcs, s);
    area.upload(ar, s);
    nrm.upload(nr, s);
    pt.upload(pp, s);
    TK.alloc(nf);
    TL.alloc(nf);
    launch_halftrans(nf, dim, fc.p, area.p, nrm.p, pt.p, cen.p, k0.p, TK.p, TL.p, bad.p, s);
    std::vector<int> hb = bad.download(s);
    require(hb[0] == 0, "non-positive half-transmissibility (check normals, collocation points and K0)");
    // canonical flux id order -> internal
    std::vector<int> canon(nf);
    for (int64_t i = 0; i < nf; ++i) canon[i] = (int)forder[i];
    DVec<int> dcanon;
    dcanon.upload(canon, s);
    fine.TKi.alloc(nf);
    fine.TLi.alloc(nf);
    if (nf) {
      hipLaunchKernelGGL(k_invgather, dim3(grid_for(nf, kBlock)), dim3(kBlock), 0, s, nf, dcanon.p, TK.p,
                         fine.L.p, 0, fine.TKi.p);
      LAUNCHCHECK();
      hipLaunchKernelGGL(k_invgather, dim3(grid_for(nf, kBlock)), dim3(kBlock), 0, s, nf, dcanon.p, TL.p,
                         fine.L.p, 1, fine.TLi.p);
      LAUNCHCHECK();
    }
    HIPCHECK(hipStreamSynchronize(s));
  }
  fine.f.alloc(n);
  fine.g.alloc(nf);
  fine.f.zero(s);
  fine.g.zero(s);
  // ---------------- fine smoother (eliminated system and its AMG), coarse levels
  const bool tr_on = trace_level() > 0;
  double tp = wall_ms();
  setup_fine_solver(*this);
  if (tr_on) std::fprintf(stderr, "[spfas] setup: fine solver (S pattern, AMG) %.1f ms\n", wall_ms() - tp);
  tp = wall_ms();
  setup_coarse_levels(*this);
  if (tr_on) std::fprintf(stderr, "[spfas] setup: coarse levels %.1f ms\n", wall_ms() - tp);
  HIPCHECK(hipStreamSynchronize(s));
}

void Hierarchy::aggregate_level(int l) {
  const spfas_coarsen_opts& o = copts;
  if (o.agg_kind == SPFAS_AGG_USER) {
    require(user_off[l] + topo[l].n_cells <= o.user_agg_len, "user_agg is shorter than the cells of a coarsened level");
    user_aggregate(topo[l], o.user_agg + user_off[l], topo[l].n_cells);
  } else if (o.agg_kind == SPFAS_AGG_GREEDY) {
    greedy_aggregate(topo[l], l > 0 && o.greedy_size_coarse > 0 ? o.greedy_size_coarse : o.greedy_size);
  } else {
    box_aggregate(topo[l], o.box);
  }
  renumber(topo[l]);
}

void Hierarchy::rebuild_coarse_topology(int l, const std::vector<int64_t>& mA) {
  topo[l + 1] = coarse_topology(topo[l], mA);
  if (l + 2 < n_levels) {
    aggregate_level(l + 1);
    topo[l + 2] = coarse_topology(topo[l + 1], m);
  }
}

void Hierarchy::set_problem(const spfas_problem& P) {
  require(P.source != nullptr, "problem.source must not be NULL");
  require(std::isfinite(P.alpha), "problem.alpha must be finite");
  require(P.kappa_kind == SPFAS_KAPPA_EXP || P.kappa_kind == SPFAS_KAPPA_RICHARDS,
          "problem.kappa_kind must be SPFAS_KAPPA_EXP or SPFAS_KAPPA_RICHARDS");
  KappaFam kf;
  kf.kind = P.kappa_kind;
  kf.alpha = P.alpha;
  if (P.kappa_kind == SPFAS_KAPPA_RICHARDS) {
    require(std::isfinite(P.kappa_a) && P.kappa_a > 0.0, "problem.kappa_a must be finite and > 0");
    require(std::isfinite(P.kappa_beta) && P.kappa_beta >= 1.0, "problem.kappa_beta must be finite and >= 1");
    kf.a = P.kappa_a;
    kf.beta = P.kappa_beta;
  }
  fine.kf = kf;
  hipStream_t s = stream;
  const double *src = P.source, *gD = P.g_dirichlet, *gN = P.g_neumann, *sh = P.shift;
  DVec<double> hs, hd, hn, hz;
  if (P.mem == SPFAS_MEM_HOST) {
    hs.upload(P.source, n_cells_in, s);
    src = hs.p;
    if (gD) { hd.upload(P.g_dirichlet, n_faces_in, s); gD = hd.p; }
    if (gN) { hn.upload(P.g_neumann, n_faces_in, s); gN = hn.p; }
    if (sh) { hz.upload(P.shift, n_cells_in, s); sh = hz.p; }
  }
  launch_fine_problem(fine.view(), fine.cell_in.p, fine.flux_in.p, fine.vol.p, fine.nptr.p, fine.nface.p,
                      fine.narea.p, src, gD, gN, fine.f.p, fine.g.p, s);
  // shift of kappa: level 0 in internal order, coarse levels the volume
  // means over their level-0 cells (level by level: the mean of the finer
  // level's means weighted by the finer cells' volumes)
  fine.has_shift = sh != nullptr;
  for (auto& C : coarse) C->has_shift = fine.has_shift;
  if (sh) {
    if (fine.z.n != fine.n) fine.z.alloc(fine.n);
    launch_gather(fine.n, fine.cell_in.p, sh, fine.z.p, s);
    for (int l = 0; l + 1 < n_levels; ++l) {
      CoarseLevel& C = *coarse[l];
      if (C.zbar.n != C.n) C.zbar.alloc(C.n);
      const double* vol_l = l == 0 ? fine.vol.p : coarse[l - 1]->vol.p;
      const double* z_l = l == 0 ? fine.z.p : coarse[l - 1]->zbar.p;
      launch_volume_mean(*trans[l], vol_l, z_l, C.vol.p, C.zbar.p, s);
    }
  }
  HIPCHECK(hipStreamSynchronize(s));
}

void Hierarchy::eval_residual(const double* p, const double* sig, double* rp, double* rs, bool dev) {
  hipStream_t s = stream;
  const int64_t n = fine.n, nf = fine.nf;
  DVec<double> x, r, pin, sin, rpo, rso;
  x.alloc(nf + n);
  r.alloc(nf + n);
  const double *pd = p, *sd = sig;
  if (!dev) {
    pin.upload(p, n_cells_in, s);
    sin.upload(sig, n_faces_in, s);
    pd = pin.p;
    sd = sin.p;
  }
  launch_gather(nf, fine.flux_in.p, sd, x.p, s);
  launch_gather(n, fine.cell_in.p, pd, x.p + nf, s);
  launch_fine_resid(fine.view(), x.p, nullptr, 0.0, r.p, parts.p, s);
  double *rpd = rp, *rsd = rs;
  if (!dev) {
    rpo.alloc(n_cells_in);
    rso.alloc(n_faces_in);
    rpd = rpo.p;
    rsd = rso.p;
  }
  launch_fill(n_faces_in, 0.0, rsd, s);
  launch_scatter(nf, fine.flux_in.p, r.p, rsd, s);
  launch_scatter(n, fine.cell_in.p, r.p + nf, rpd, s);
  if (!dev) {
    HIPCHECK(hipMemcpyAsync(rp, rpd, n_cells_in * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHECK(hipMemcpyAsync(rs, rsd, n_faces_in * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  HIPCHECK(hipStreamSynchronize(s));
}

}  // namespace spfas
