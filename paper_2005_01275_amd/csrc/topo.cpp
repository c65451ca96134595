// Host-side integer structure of the hierarchy (see topo.hpp).
#include "topo.hpp"

#include <algorithm>
#include <atomic>
#include <climits>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <unordered_set>

#include "common.hpp"

namespace spfas {

bool lattice_from_centroids(int dim, int64_t n, const double* centroid, std::vector<int>& shape,
                            std::vector<int64_t>& index) {
  shape.assign(dim, 0);
  index.assign(n, 0);
  int64_t stride = 1;
  for (int a = 0; a < dim; ++a) {
    // distinct coordinate values along axis a, ascending (a lattice has few)
    std::unordered_set<double> seen_v;
    for (int64_t i = 0; i < n; ++i) {
      seen_v.insert(centroid[i * dim + a]);
      if ((int64_t)seen_v.size() > n) return false;
    }
    std::vector<double> u(seen_v.begin(), seen_v.end());
    std::sort(u.begin(), u.end());
    shape[a] = (int)u.size();
    parallel_ranges(n, [&](int64_t lo, int64_t hi) {
      for (int64_t i = lo; i < hi; ++i) {
        const int64_t r = std::lower_bound(u.begin(), u.end(), centroid[i * dim + a]) - u.begin();
        index[i] += r * stride;
      }
    });
    stride *= (int64_t)u.size();
  }
  if (stride != n) return false;
  std::vector<char> seen(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    if (seen[index[i]]) return false;
    seen[index[i]] = 1;
  }
  return true;
}

int box_blocks(int n, int a) {
  int nb = n / a, rem = n % a;
  if (rem == 0) return std::max(nb, 1);
  if (2 * rem < a) return std::max(nb, 1);
  return nb + 1;
}

void box_aggregate(Topo& t, const int box[3]) {
  const int dim = (int)t.lat_shape.size();
  t.agg.assign(t.n_cells, 0);
  t.agg_shape.assign(dim, 0);
  std::vector<int> nb(dim);
  for (int a = 0; a < dim; ++a) nb[a] = box_blocks(t.lat_shape[a], box[a]);
  for (int64_t c = 0; c < t.n_cells; ++c) {
    int64_t rem = t.lat_index[c], stride = 1, id = 0;
    for (int a = 0; a < dim; ++a) {
      int64_t coord = rem % t.lat_shape[a];
      rem /= t.lat_shape[a];
      int64_t blk = std::min<int64_t>(coord / box[a], nb[a] - 1);
      id += blk * stride;
      stride *= nb[a];
    }
    t.agg[c] = id;
  }
  t.agg_shape = nb;
  int64_t na = 1;
  for (int a = 0; a < dim; ++a) na *= nb[a];
  t.n_agg = na;
}

// Interior neighbours of each cell (ascending, without repeats), from the
// level's interior flux unknowns.
static void cell_neighbours(const Topo& t, std::vector<int64_t>& ptr, std::vector<int64_t>& nb) {
  const int64_t n = t.n_cells;
  // both cells of every interior flux, grouped by cell (flux order)
  std::vector<int64_t> deg(n + 1, 0);
  for (int64_t j = 0; j < t.n_flux; ++j)
    if (t.kind[j] == FK_INTERIOR && t.c2[j] >= 0) {
      deg[t.c1[j] + 1]++;
      deg[t.c2[j] + 1]++;
    }
  for (int64_t c = 0; c < n; ++c) deg[c + 1] += deg[c];
  std::unique_ptr<int64_t[]> raw(new int64_t[deg[n]]);   // every entry written below
  {
    std::vector<int64_t> fill(deg.begin(), deg.end() - 1);
    for (int64_t j = 0; j < t.n_flux; ++j)
      if (t.kind[j] == FK_INTERIOR && t.c2[j] >= 0) {
        raw[fill[t.c1[j]]++] = t.c2[j];
        raw[fill[t.c2[j]]++] = t.c1[j];
      }
  }
  // each row sorted without repeats (rows on host threads), then compacted
  ptr.assign(n + 1, 0);
  parallel_ranges(n, [&](int64_t lo, int64_t hi) {
    for (int64_t c = lo; c < hi; ++c) {
      int64_t *b = raw.get() + deg[c], *e = raw.get() + deg[c + 1];
      std::sort(b, e);
      ptr[c + 1] = std::unique(b, e) - b;
    }
  });
  for (int64_t c = 0; c < n; ++c) ptr[c + 1] += ptr[c];
  nb.resize(ptr[n]);
  parallel_ranges(n, [&](int64_t lo, int64_t hi) {
    for (int64_t c = lo; c < hi; ++c)
      std::copy(raw.get() + deg[c], raw.get() + deg[c] + (ptr[c + 1] - ptr[c]), nb.begin() + ptr[c]);
  });
}

void user_aggregate(Topo& t, const int32_t* agg, int64_t len) {
  require(agg != nullptr, "user_agg is NULL");
  require(len == t.n_cells, "user_agg is shorter than the cells of a coarsened level");
  int64_t na = 0;
  for (int64_t c = 0; c < t.n_cells; ++c) {
    require(agg[c] >= 0, "user_agg holds a negative aggregate id");
    na = std::max<int64_t>(na, (int64_t)agg[c] + 1);
  }
  require(na < t.n_cells || t.n_cells == 1, "user_agg does not coarsen the level");
  std::vector<int64_t> size(na, 0);
  for (int64_t c = 0; c < t.n_cells; ++c) size[agg[c]]++;
  for (int64_t A = 0; A < na; ++A) require(size[A] > 0, "user_agg leaves an aggregate id unused");
  // connectedness: union-find over interior faces inside one aggregate
  std::vector<int64_t> up(t.n_cells);
  std::iota(up.begin(), up.end(), 0);
  auto find = [&](int64_t x) {
    while (up[x] != x) x = up[x] = up[up[x]];
    return x;
  };
  for (int64_t j = 0; j < t.n_flux; ++j)
    if (t.kind[j] == FK_INTERIOR && t.c2[j] >= 0 && agg[t.c1[j]] == agg[t.c2[j]]) {
      const int64_t a = find(t.c1[j]), b = find(t.c2[j]);
      if (a != b) up[std::max(a, b)] = std::min(a, b);
    }
  std::vector<int64_t> root(na, -1);
  for (int64_t c = 0; c < t.n_cells; ++c) {
    const int64_t r = find(c);
    if (root[agg[c]] < 0) root[agg[c]] = r;
    else require(root[agg[c]] == r, "user_agg holds an aggregate that is not connected");
  }
  t.agg.assign(agg, agg + t.n_cells);
  t.n_agg = na;
  t.agg_shape.clear();
}

void greedy_aggregate(Topo& t, int target) {
  require(target >= 2, "greedy_size must be at least 2");
  const int64_t n = t.n_cells;
  std::vector<int64_t> nptr, nb;
  cell_neighbours(t, nptr, nb);
  // growth: seeds in ascending id, breadth first, neighbours in ascending id
  std::vector<int64_t> agg(n, -1), queue;
  std::vector<std::vector<int64_t>> members;
  for (int64_t s = 0; s < n; ++s) {
    if (agg[s] >= 0) continue;
    const int64_t A = (int64_t)members.size();
    members.emplace_back();
    auto& mem = members.back();
    agg[s] = A;
    mem.push_back(s);
    queue.assign(1, s);
    for (size_t head = 0; head < queue.size() && (int64_t)mem.size() < target; ++head) {
      const int64_t u = queue[head];
      for (int64_t k = nptr[u]; k < nptr[u + 1] && (int64_t)mem.size() < target; ++k) {
        const int64_t v = nb[k];
        if (agg[v] >= 0) continue;
        agg[v] = A;
        mem.push_back(v);
        queue.push_back(v);
      }
    }
  }
  const int64_t na0 = (int64_t)members.size();
  // fragments below target/2 join the neighbour sharing the most interior
  // faces (ties: lower id), in ascending id; labels stay original ids of
  // the surviving aggregates
  std::vector<int64_t> label(na0);
  std::iota(label.begin(), label.end(), 0);
  // original ids carrying each surviving label
  std::vector<std::vector<int64_t>> carried(na0);
  for (int64_t A = 0; A < na0; ++A) carried[A].assign(1, A);
  std::vector<char> alive(na0, 1);
  std::vector<int64_t> count(na0, 0), touched;
  for (int64_t A = 0; A < na0; ++A) {
    if (!alive[A] || 2 * (int64_t)members[A].size() >= target) continue;
    touched.clear();
    for (int64_t u : members[A])
      for (int64_t k = t.cfptr[u]; k < t.cfptr[u + 1]; ++k) {
        const int64_t j = t.cfidx[k];
        if (t.kind[j] != FK_INTERIOR || t.c2[j] < 0) continue;
        const int64_t v = t.c1[j] == u ? t.c2[j] : t.c1[j];
        const int64_t B = label[agg[v]];
        if (B == A) continue;
        if (count[B]++ == 0) touched.push_back(B);
      }
    int64_t best = -1;
    for (int64_t B : touched)
      if (best < 0 || count[B] > count[best] || (count[B] == count[best] && B < best)) best = B;
    for (int64_t B : touched) count[B] = 0;
    if (best < 0) continue;   // no neighbour: the fragment stays
    for (int64_t u : members[A]) members[best].push_back(u);
    members[A].clear();
    alive[A] = 0;
    for (int64_t X : carried[A]) label[X] = best;
    carried[best].insert(carried[best].end(), carried[A].begin(), carried[A].end());
    carried[A].clear();
  }
  // compact ids in ascending order of the surviving labels
  std::vector<int64_t> newid(na0, -1);
  int64_t na = 0;
  for (int64_t A = 0; A < na0; ++A)
    if (alive[A]) newid[A] = na++;
  t.agg.resize(n);
  for (int64_t c = 0; c < n; ++c) t.agg[c] = newid[label[agg[c]]];
  t.n_agg = na;
  t.agg_shape.clear();
}

void renumber(Topo& t) {
  const int64_t n = t.n_cells;
  // cells by aggregate, ascending id inside an aggregate (counting sort)
  t.cell_order.resize(n);
  {
    std::vector<int64_t> cnt(t.n_agg + 1, 0);
    for (int64_t i = 0; i < n; ++i) cnt[t.agg[i] + 1]++;
    for (int64_t a = 0; a < t.n_agg; ++a) cnt[a + 1] += cnt[a];
    for (int64_t i = 0; i < n; ++i) t.cell_order[cnt[t.agg[i]]++] = i;
  }
  std::vector<int64_t> pos(n);
  for (int64_t i = 0; i < n; ++i) pos[t.cell_order[i]] = i;
  const int64_t nf = t.n_flux;
  // Same order as sorting the whole key tuple (group, first aggregate,
  // second aggregate, bubble, lo, hi, id), in two passes: a counting sort on
  // the bucket (group, first aggregate), then a sort of each (small) bucket
  // on the remaining fields, which id makes a total order.
  const int64_t na = t.n_agg;
  struct Key { int64_t g2, kr, lo, hi, id; };
  // uninitialised: every entry is written by the threads below
  std::unique_ptr<Key[]> keys(new Key[nf]);
  std::unique_ptr<int64_t[]> bkt(new int64_t[nf]);
  parallel_ranges(nf, [&](int64_t jlo, int64_t jhi) {
    for (int64_t j = jlo; j < jhi; ++j) {
      const int64_t a = t.c1[j], b = t.c2[j];
      const int8_t k = t.kind[j];
      const int64_t a1 = t.agg[a];
      const int64_t a2 = b >= 0 ? t.agg[b] : -1;
      const bool inside = (k == FK_BUBBLE) || (k == FK_INTERIOR && a1 == a2);
      const bool cross = (k == FK_INTERIOR && a1 != a2);
      const int64_t g0 = inside ? 0 : (cross ? 1 : 2);
      const int64_t g1 = cross ? std::min(a1, a2) : a1;
      const int64_t p1 = pos[a];
      const int64_t p2 = b >= 0 ? pos[b] : p1;
      bkt[j] = g0 * na + g1;
      keys[j] = Key{cross ? std::max(a1, a2) : 0, (k == FK_BUBBLE) ? 1 : 0, std::min(p1, p2), std::max(p1, p2), j};
    }
  });
  std::vector<int64_t> bptr(3 * na + 1, 0);
  for (int64_t j = 0; j < nf; ++j) bptr[bkt[j] + 1]++;
  for (int64_t b = 0; b < 3 * na; ++b) bptr[b + 1] += bptr[b];
  std::unique_ptr<Key[]> sorted(new Key[nf]);
  {
    // scattered on host threads: the order inside a bucket is fixed by the sort below
    std::vector<std::atomic<int64_t>> fill(3 * na);
    for (int64_t b = 0; b < 3 * na; ++b) fill[b].store(bptr[b], std::memory_order_relaxed);
    parallel_ranges(nf, [&](int64_t jlo, int64_t jhi) {
      for (int64_t j = jlo; j < jhi; ++j) sorted[fill[bkt[j]].fetch_add(1, std::memory_order_relaxed)] = keys[j];
    });
  }
  t.flux_order.resize(nf);
  parallel_ranges(3 * na, [&](int64_t blo, int64_t bhi) {
    for (int64_t b = blo; b < bhi; ++b) {
      std::sort(sorted.get() + bptr[b], sorted.get() + bptr[b + 1], [](const Key& x, const Key& y) {
        return std::tie(x.g2, x.kr, x.lo, x.hi, x.id) < std::tie(y.g2, y.kr, y.lo, y.hi, y.id);
      });
      for (int64_t i = bptr[b]; i < bptr[b + 1]; ++i) t.flux_order[i] = sorted[i].id;
    }
  }, nf);
}

void build_cell_lists(Topo& t) {
  std::vector<int64_t> cnt(t.n_cells + 1, 0);
  for (int64_t j = 0; j < t.n_flux; ++j) {
    cnt[t.c1[j] + 1]++;
    if (t.c2[j] >= 0) cnt[t.c2[j] + 1]++;
  }
  for (int64_t c = 0; c < t.n_cells; ++c) cnt[c + 1] += cnt[c];
  t.cfptr = cnt;
  t.cfidx.assign(cnt.back(), 0);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t j = 0; j < t.n_flux; ++j) {   // ascending j -> lists sorted
    t.cfidx[fill[t.c1[j]]++] = j;
    if (t.c2[j] >= 0) t.cfidx[fill[t.c2[j]]++] = j;
  }
}

std::vector<int64_t> aggregate_unknowns(const Topo& f) {
  std::vector<int64_t> npA(f.n_agg, 0);
  for (int64_t i = 0; i < f.n_cells; ++i) npA[f.agg[i]] += f.pptr[i + 1] - f.pptr[i];
  for (int64_t A = 0; A < f.n_agg; ++A)
    if (npA[A] == 0) fail(SPFAS_ERR_INVALID, "empty aggregate");
  return npA;
}

Topo coarse_topology(const Topo& f, int m) {
  std::vector<int64_t> mA = aggregate_unknowns(f);
  for (auto& v : mA) v = std::min<int64_t>(m, v);
  return coarse_topology(f, mA);
}

Topo coarse_topology(const Topo& f, const std::vector<int64_t>& mA) {
  Topo c;
  const int64_t na = f.n_agg;
  c.n_cells = na;
  const std::vector<int64_t> npA = aggregate_unknowns(f);
  require((int64_t)mA.size() == na, "one eigenvector count per aggregate");
  c.pptr.assign(na + 1, 0);
  for (int64_t A = 0; A < na; ++A) {
    require(mA[A] >= 1 && mA[A] <= npA[A], "eigenvector count out of range");
    c.pptr[A + 1] = c.pptr[A] + mA[A];
  }
  std::vector<std::pair<int64_t, int64_t>> pairs;
  std::vector<char> hasdir(na, 0);
  for (int64_t j = 0; j < f.n_flux; ++j) {
    if (f.kind[j] == FK_INTERIOR) {
      int64_t a = f.agg[f.c1[j]], b = f.agg[f.c2[j]];
      if (a != b) pairs.emplace_back(std::min(a, b), std::max(a, b));
    } else if (f.kind[j] == FK_DIRICHLET) {
      hasdir[f.agg[f.c1[j]]] = 1;
    }
  }
  std::sort(pairs.begin(), pairs.end());
  pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
  int64_t nfc = 0;
  for (auto& pr : pairs) {
    c.kind.push_back(FK_INTERIOR);
    c.c1.push_back(pr.first);
    c.c2.push_back(pr.second);
    ++nfc;
  }
  for (int64_t A = 0; A < na; ++A)
    if (hasdir[A]) {
      c.kind.push_back(FK_DIRICHLET);
      c.c1.push_back(A);
      c.c2.push_back(-1);
      ++nfc;
    }
  for (int64_t A = 0; A < na; ++A)
    for (int64_t j = 1; j < mA[A]; ++j) {
      c.kind.push_back(FK_BUBBLE);
      c.c1.push_back(A);
      c.c2.push_back(-1);
      ++nfc;
    }
  c.n_flux = nfc;
  build_cell_lists(c);
  c.lat_shape = f.agg_shape;
  c.lat_index.resize(na);
  std::iota(c.lat_index.begin(), c.lat_index.end(), 0);
  return c;
}

TransferPlan make_plan(const Topo& f, const Topo& c, const std::vector<int64_t>& dev_cell,
                       const std::vector<int64_t>& dev_p, const std::vector<int64_t>& dev_flux,
                       const std::vector<int64_t>& dev_cfptr,
                       const std::vector<int64_t>& dev_cfidx) {
  TransferPlan P;
  const int64_t na = c.n_cells;
  P.n_agg = na;
  // Lists in CSR form by counting sorts, each filled in the order the plan
  // needs: cells of each aggregate by ascending canonical id; the fine
  // fluxes of each coarse face group and the interior fluxes int(A) of each
  // aggregate in the renumbered order of level l.
  auto csr = [](int64_t nb, const std::vector<int64_t>& key, std::vector<int64_t>& ptr) {
    ptr.assign(nb + 1, 0);
    for (int64_t k : key)
      if (k >= 0) ptr[k + 1]++;
    for (int64_t b = 0; b < nb; ++b) ptr[b + 1] += ptr[b];
  };
  std::vector<int64_t> mem_ptr, members;
  {
    std::vector<int64_t> key(f.agg.begin(), f.agg.end());
    csr(na, key, mem_ptr);
    members.resize(mem_ptr[na]);
    std::vector<int64_t> fill(mem_ptr.begin(), mem_ptr.end() - 1);
    for (int64_t i = 0; i < f.n_cells; ++i) members[fill[f.agg[i]]++] = i;
  }
  // coarse group of every fine flux (-1: none) and int(A) membership
  std::vector<int64_t> grp_of(f.n_flux, -1), int_of(f.n_flux, -1);
  {
    // map (a,b) pair -> coarse face id; Dirichlet A -> coarse id
    std::vector<int64_t> dir_id(na, -1);
    for (int64_t J = 0; J < c.n_flux; ++J)
      if (c.kind[J] == FK_DIRICHLET) dir_id[c.c1[J]] = J;
    // interior pairs are sorted by (lower, higher) aggregate: the pairs of
    // each lower aggregate form one range, searched linearly
    int64_t n_pairs = 0;
    while (n_pairs < c.n_flux && c.kind[n_pairs] == FK_INTERIOR) ++n_pairs;
    std::vector<int64_t> lo_ptr(na + 1, 0);
    for (int64_t J = 0; J < n_pairs; ++J) lo_ptr[c.c1[J] + 1]++;
    for (int64_t A = 0; A < na; ++A) lo_ptr[A + 1] += lo_ptr[A];
    std::atomic<bool> orphan{false};
    parallel_ranges(f.n_flux, [&](int64_t jlo, int64_t jhi) {
    for (int64_t j = jlo; j < jhi; ++j) {
      const int8_t k = f.kind[j];
      const int64_t a1 = f.agg[f.c1[j]];
      if (k == FK_BUBBLE) {
        int_of[j] = a1;
      } else if (k == FK_INTERIOR) {
        const int64_t a2 = f.agg[f.c2[j]];
        if (a1 == a2) {
          int_of[j] = a1;
          continue;
        }
        const int64_t lo = std::min(a1, a2), hi = std::max(a1, a2);
        int64_t J = lo_ptr[lo];
        while (J < lo_ptr[lo + 1] && c.c2[J] != hi) ++J;
        if (J == lo_ptr[lo + 1]) orphan = true;
        else grp_of[j] = J;
      } else if (k == FK_DIRICHLET) {
        grp_of[j] = dir_id[a1];
      }
    }
    });
    if (orphan) fail(SPFAS_ERR_INVALID, "fine face between aggregates without a coarse face");
  }
  std::vector<int64_t> grp_ptr, grp_list, int_ptr, int_list;
  csr(c.n_flux, grp_of, grp_ptr);
  csr(na, int_of, int_ptr);
  grp_list.resize(grp_ptr[c.n_flux]);
  int_list.resize(int_ptr[na]);
  {
    std::vector<int64_t> gfill(grp_ptr.begin(), grp_ptr.end() - 1), ifill(int_ptr.begin(), int_ptr.end() - 1);
    for (int64_t i = 0; i < f.n_flux; ++i) {   // renumbered order of level l
      const int64_t j = f.flux_order[i];
      if (grp_of[j] >= 0) grp_list[gfill[grp_of[j]]++] = j;
      if (int_of[j] >= 0) int_list[ifill[int_of[j]]++] = j;
    }
  }
  P.cell_ptr.assign(na + 1, 0);
  P.pd_ptr.assign(na + 1, 0);
  P.dof_ptr.assign(na + 1, 0);
  P.int_ptr.assign(na + 1, 0);
  P.n_int.assign(na, 0);
  P.mA.assign(na, 0);
  P.fgrp_ptr.assign(c.n_flux + 1, 0);
  P.grp_pos_A.assign(c.n_flux, -1);
  P.grp_pos_B.assign(c.n_flux, -1);
  P.fgrp_ptr = grp_ptr;
  P.fgrp_list.resize(grp_list.size());
  for (size_t q = 0; q < grp_list.size(); ++q) P.fgrp_list[q] = dev_flux[grp_list[q]];
  // device flux id -> canonical id (the device local lists are read in
  // device order, which is ascending device id within each cell)
  std::vector<int64_t> canon_of_dev(f.n_flux, -1);
  parallel_ranges(f.n_flux, [&](int64_t jlo, int64_t jhi) {
    for (int64_t j = jlo; j < jhi; ++j) canon_of_dev[dev_flux[j]] = j;
  });
  // list offsets of every aggregate (cells, p unknowns, dofs) and of every
  // member cell's scatter entries, so the aggregates fill their parts of
  // the lists on host threads
  P.cell_ptr = mem_ptr;
  P.int_ptr = int_ptr;
  const int64_t n_mem = mem_ptr[na];
  P.smap_ptr.assign(n_mem + 1, 0);
  for (int64_t A = 0; A < na; ++A) {
    int64_t npd = 0, nd = int_ptr[A + 1] - int_ptr[A];
    for (int64_t m = mem_ptr[A]; m < mem_ptr[A + 1]; ++m) {
      const int64_t cell = members[m];
      npd += f.pptr[cell + 1] - f.pptr[cell];
      P.smap_ptr[m + 1] = P.smap_ptr[m] + (f.cfptr[cell + 1] - f.cfptr[cell]);
    }
    for (int64_t q = c.cfptr[A]; q < c.cfptr[A + 1]; ++q) {
      const int64_t J = c.cfidx[q];
      if (c.kind[J] != FK_BUBBLE) nd += grp_ptr[J + 1] - grp_ptr[J];
    }
    P.pd_ptr[A + 1] = P.pd_ptr[A] + npd;
    P.dof_ptr[A + 1] = P.dof_ptr[A] + nd;
  }
  P.cell_list.resize(n_mem);
  P.pd_list.resize(P.pd_ptr[na]);
  P.dof_list.resize(P.dof_ptr[na]);
  P.smap.resize(P.smap_ptr[n_mem]);
  std::mutex err_mu;
  std::string err;   // first error of any thread, raised after the join
  parallel_ranges(na, [&](int64_t alo, int64_t ahi) {
    std::vector<int64_t> dofs;
    std::vector<std::pair<int64_t, int64_t>> pos;   // (flux, position in dofs(A)) sorted by flux
    try {
      for (int64_t A = alo; A < ahi; ++A) {
        P.mA[A] = (int32_t)(c.pptr[A + 1] - c.pptr[A]);
        int64_t pq = P.pd_ptr[A];
        for (int64_t m = mem_ptr[A]; m < mem_ptr[A + 1]; ++m) {
          const int64_t cell = members[m];
          P.cell_list[m] = dev_cell[cell];
          for (int64_t q = f.pptr[cell]; q < f.pptr[cell + 1]; ++q) P.pd_list[pq++] = dev_p[q];
        }
        // dofs(A): int(A), then the groups of A's coarse faces in A's local order
        dofs.assign(int_list.begin() + int_ptr[A], int_list.begin() + int_ptr[A + 1]);
        P.n_int[A] = (int32_t)(int_ptr[A + 1] - int_ptr[A]);
        for (int64_t q = c.cfptr[A]; q < c.cfptr[A + 1]; ++q) {
          const int64_t J = c.cfidx[q];
          if (c.kind[J] == FK_BUBBLE) continue;
          const int64_t off = (int64_t)dofs.size();
          if (c.c1[J] == A) P.grp_pos_A[J] = off; else P.grp_pos_B[J] = off;
          dofs.insert(dofs.end(), grp_list.begin() + grp_ptr[J], grp_list.begin() + grp_ptr[J + 1]);
        }
        pos.resize(dofs.size());
        for (size_t q = 0; q < dofs.size(); ++q) {
          pos[q] = {dofs[q], (int64_t)q};
          P.dof_list[P.dof_ptr[A] + q] = dev_flux[dofs[q]];
        }
        std::sort(pos.begin(), pos.end());
        for (int64_t m = mem_ptr[A]; m < mem_ptr[A + 1]; ++m) {
          const int64_t cell = members[m];
          const int64_t dc = dev_cell[cell];
          // the cell's fluxes in the device local order (ascending device id)
          const int64_t k = dev_cfptr[dc + 1] - dev_cfptr[dc];
          if (P.smap_ptr[m + 1] - P.smap_ptr[m] != k) fail(SPFAS_ERR_INVALID, "local flux list mismatch");
          int64_t prev = -1;
          for (int64_t q = 0; q < k; ++q) {
            const int64_t d = dev_cfidx[dev_cfptr[dc] + q];
            if (d <= prev || d < 0 || d >= f.n_flux) fail(SPFAS_ERR_INVALID, "device local order mismatch");
            prev = d;
            const int64_t j = canon_of_dev[d];
            if (f.c1[j] != cell && f.c2[j] != cell) fail(SPFAS_ERR_INVALID, "device local list holds a foreign flux");
            // the last position of j in dofs(A)
            auto it = std::upper_bound(pos.begin(), pos.end(), std::make_pair(j, INT64_MAX));
            if (it == pos.begin() || (it - 1)->first != j)
              fail(SPFAS_ERR_INVALID, "flux of an aggregate cell outside dofs(A)");
            P.smap[P.smap_ptr[m] + q] = (int32_t)(it - 1)->second;
          }
        }
      }
    } catch (const Error& e) {
      std::lock_guard<std::mutex> lk(err_mu);
      if (err.empty()) err = e.what();
    }
  }, f.n_flux);
  if (!err.empty()) fail(SPFAS_ERR_INVALID, err);
  return P;
}

}  // namespace spfas
