// Classical AMG setup on the host (see amg_host.hpp): PMIS coarsening
// (De Sterck, Yang, Heys 2006), extended+i interpolation (De Sterck,
// Falgout, Nolting, Yang 2008) with truncation, and the symbolic Galerkin
// products with their per-entry product lists.
#include "amg_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <thread>

namespace spfas {

namespace {

// Host threads for the row-parallel setup steps.
int host_threads() { return host_thread_limit(); }

// Below this many rows (or units of work) a step runs its chunks in order
// in the calling thread: thread start-up would cost more than it saves.
constexpr int kGrain = 16384;

// f(t, lo, hi) on nth contiguous, ordered chunks of [0, n), one thread each
// (in the calling thread, one after the other, when n is small; the chunks
// and so the results are the same).
template <class F>
void parallel_chunks(int n, int nth, F&& f) {
  const int per = (n + nth - 1) / nth;
  if (n < kGrain) {
    for (int t = 0; t < nth; ++t) {
      const int lo = std::min(n, t * per), hi = std::min(n, lo + per);
      f(t, lo, hi);
    }
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nth; ++t) {
    const int lo = std::min(n, t * per), hi = std::min(n, lo + per);
    th.emplace_back([&f, t, lo, hi] { f(t, lo, hi); });
  }
  for (auto& x : th) x.join();
}

// f(t) for t < nth, one thread each when `work` is large enough.
template <class F>
void per_chunk(int nth, size_t work, F&& f) {
  if (work < (size_t)kGrain) {
    for (int t = 0; t < nth; ++t) f(t);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nth; ++t) th.emplace_back([&f, t] { f(t); });
  for (auto& x : th) x.join();
}

// Exclusive prefix sums of per-chunk sizes: off[t] is where chunk t starts.
template <class Size>
std::vector<size_t> chunk_offsets(int nth, Size size) {
  std::vector<size_t> off(nth + 1, 0);
  for (int t = 0; t < nth; ++t) off[t + 1] = off[t] + size(t);
  return off;
}

// splitmix64 (Steele, Lea, Flood 2014): the PMIS tie-breaking measure
double unit_hash(uint64_t seed, uint64_t i) {
  uint64_t z = seed + 0x9E3779B97F4A7C15ULL * (i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

struct Strength {
  std::vector<int> ptr, col;     // strong dependences of each row
  std::vector<int> tptr, tcol;   // transpose: rows that depend strongly on each point
};

Strength strength(const HostCsr& A, double theta) {
  const int n = A.n, nth = host_threads();
  Strength S;
  // strong dependences of row i, in column order: counted, then written
  auto row = [&](int i, int* out) {
    double mx = 0.0;
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (A.col[k] != i) mx = std::max(mx, -A.val[k]);
    int c = 0;
    if (mx > 0.0)
      for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
        if (A.col[k] != i && -A.val[k] >= theta * mx) {
          if (out) out[c] = A.col[k];
          ++c;
        }
    return c;
  };
  S.ptr.assign(n + 1, 0);
  parallel_chunks(n, nth, [&](int, int lo, int hi) {
    for (int i = lo; i < hi; ++i) S.ptr[i + 1] = row(i, nullptr);
  });
  for (int i = 0; i < n; ++i) S.ptr[i + 1] += S.ptr[i];
  S.col.resize(S.ptr[n]);
  parallel_chunks(n, nth, [&](int, int lo, int hi) {
    for (int i = lo; i < hi; ++i) row(i, S.col.data() + S.ptr[i]);
  });
  S.tptr.assign(n + 1, 0);
  for (int j : S.col) S.tptr[j + 1]++;
  for (int i = 0; i < n; ++i) S.tptr[i + 1] += S.tptr[i];
  S.tcol.resize(S.col.size());
  std::vector<int> fill(S.tptr.begin(), S.tptr.end() - 1);
  for (int i = 0; i < n; ++i)
    for (int q = S.ptr[i]; q < S.ptr[i + 1]; ++q) S.tcol[fill[S.col[q]]++] = i;
  return S;
}

// state: 1 = C, -1 = F.  Each round's selection and F-marking read only the
// state of the previous step, so rows are split over host threads and the
// per-chunk lists joined in row order.
std::vector<int> pmis(const Strength& S, int n, uint64_t seed) {
  const int nth = host_threads();
  std::vector<double> lam(n);
  std::vector<int> state(n, 0);
  parallel_chunks(n, nth, [&](int, int lo, int hi) {
    for (int i = lo; i < hi; ++i) {
      const int ns = S.ptr[i + 1] - S.ptr[i], nt = S.tptr[i + 1] - S.tptr[i];
      lam[i] = nt + unit_hash(seed, (uint64_t)i);
      if (ns == 0 && nt == 0) state[i] = -1;   // isolated point: smoothing only
    }
  });
  std::vector<int> und;
  for (int i = 0; i < n; ++i)
    if (state[i] == 0) und.push_back(i);
  std::vector<char> newc(n, 0);
  std::vector<std::vector<int>> part(nth);
  auto join = [&](std::vector<int>& out) {
    const std::vector<size_t> off = chunk_offsets(nth, [&](int t) { return part[t].size(); });
    out.resize(off[nth]);
    per_chunk(nth, off[nth], [&](int t) { std::copy(part[t].begin(), part[t].end(), out.begin() + off[t]); });
  };
  std::vector<int> sel, rest;
  while (!und.empty()) {
    const int nu = (int)und.size();
    auto beats = [&](int j, int i) { return state[j] == 0 && (lam[j] > lam[i] || (lam[j] == lam[i] && j > i)); };
    parallel_chunks(nu, nth, [&](int t, int lo, int hi) {
      part[t].clear();
      for (int u = lo; u < hi; ++u) {
        const int i = und[u];
        bool mx = true;
        for (int q = S.ptr[i]; q < S.ptr[i + 1] && mx; ++q) mx = !beats(S.col[q], i);
        for (int q = S.tptr[i]; q < S.tptr[i + 1] && mx; ++q) mx = !beats(S.tcol[q], i);
        if (mx) part[t].push_back(i);
      }
    });
    join(sel);
    for (int i : sel) { state[i] = 1; newc[i] = 1; }
    parallel_chunks(nu, nth, [&](int t, int lo, int hi) {
      part[t].clear();
      for (int u = lo; u < hi; ++u) {
        const int i = und[u];
        if (state[i] != 0) continue;
        bool dep = false;
        for (int q = S.ptr[i]; q < S.ptr[i + 1] && !dep; ++q) dep = newc[S.col[q]];
        if (dep) state[i] = -1;
        else part[t].push_back(i);
      }
    });
    join(rest);
    for (int i : sel) newc[i] = 0;
    und.swap(rest);
  }
  return state;
}

}  // namespace

// Groups the products of one output row by column: columns ascending, each
// column's products in generation order; start[c] ends column c's products.
struct RowGrouper {
  struct Item { int key, a, b; };
  std::vector<Item> items, grouped;
  std::vector<int> mark, slot, cols, start;
  explicit RowGrouper(int ncols) : mark(ncols, -1), slot(ncols, 0) {}
  void group(int tag) {
    cols.clear();
    for (const Item& it : items)
      if (mark[it.key] != tag) { mark[it.key] = tag; cols.push_back(it.key); }
    std::sort(cols.begin(), cols.end());
    for (size_t c = 0; c < cols.size(); ++c) slot[cols[c]] = (int)c;
    start.assign(cols.size() + 1, 0);
    for (const Item& it : items) start[slot[it.key] + 1]++;
    for (size_t c = 0; c < cols.size(); ++c) start[c + 1] += start[c];
    grouped.resize(items.size());
    for (const Item& it : items) grouped[start[slot[it.key]]++] = it;
  }
};

// Per-chunk lists of the A P and P^T (A P) constructions.
struct ApChunk {
  std::vector<int> col, pidx, nprod, la, lp, rowlen;
  std::vector<double> val;
};
struct RapChunk {
  std::vector<int> col, nprod, r, q, dr, dq, rowlen, ndiag;
  std::vector<double> val;
};

bool classical_level(const HostCsr& A, double theta, uint64_t seed, ClassicalLevel& L) {
  const int n = A.n;
  L = ClassicalLevel();
  L.n = n;
  const Strength S = strength(A, theta);
  const std::vector<int> state = pmis(S, n, seed);
  std::vector<int> cidx(n, -1);
  int nc = 0;
  for (int i = 0; i < n; ++i)
    if (state[i] == 1) cidx[i] = nc++;
  if (nc == 0 || (long long)nc * 10 > (long long)n * 9) return false;
  L.nc = nc;

  // ---- extended+i interpolation, truncated (rows in contiguous chunks on
  // host threads, joined in row order)
  const int nth = host_threads();
  struct PChunk {
    std::vector<int> col, rowlen;
    std::vector<double> val;
  };
  std::vector<PChunk> pch(nth);
  parallel_chunks(n, nth, [&](int t, int lo, int hi) {
    PChunk& out = pch[t];
    std::vector<int> smark(n, -1), cmark(n, -1), cpos(n, 0);
    std::vector<int> hat;          // C-hat_i
    std::vector<double> w;         // accumulated numerators over C-hat_i
    std::vector<std::pair<int, double>> row;
    for (int i = lo; i < hi; ++i) {
      const size_t len0 = out.col.size();
      if (state[i] == 1) {
        out.col.push_back(cidx[i]);
        out.val.push_back(1.0);
        out.rowlen.push_back(1);
        continue;
      }
      hat.clear();
      for (int q = S.ptr[i]; q < S.ptr[i + 1]; ++q) smark[S.col[q]] = i;
      auto add_hat = [&](int j) {
        if (cmark[j] != i) { cmark[j] = i; cpos[j] = (int)hat.size(); hat.push_back(j); }
      };
      for (int q = S.ptr[i]; q < S.ptr[i + 1]; ++q) {
        const int k = S.col[q];
        if (state[k] == 1) add_hat(k);
        else
          for (int qq = S.ptr[k]; qq < S.ptr[k + 1]; ++qq)
            if (state[S.col[qq]] == 1) add_hat(S.col[qq]);
      }
      if (!hat.empty()) {
        w.assign(hat.size(), 0.0);
        double aii = A.diag[i];
        for (int q = A.ptr[i]; q < A.ptr[i + 1]; ++q) {
          const int j = A.col[q];
          const double a = A.val[q];
          if (j == i) { aii += a; continue; }
          if (cmark[j] == i) { w[cpos[j]] += a; continue; }
          if (smark[j] != i) { aii += a; continue; }   // weak neighbour: lumped into the diagonal
          // strong F neighbour k = j: distributed over C-hat_i and i with the
          // entries of row k of sign opposite to its diagonal
          const int k = j;
          const double sk = A.diag[k];
          auto bar = [&](double v) { return (v < 0.0) != (sk < 0.0) && v != 0.0 ? v : 0.0; };
          double den = 0.0;
          for (int qq = A.ptr[k]; qq < A.ptr[k + 1]; ++qq) {
            const int l = A.col[qq];
            if (l == i || cmark[l] == i) den += bar(A.val[qq]);
          }
          if (den == 0.0) { aii += a; continue; }
          for (int qq = A.ptr[k]; qq < A.ptr[k + 1]; ++qq) {
            const int l = A.col[qq];
            const double b = bar(A.val[qq]);
            if (b == 0.0) continue;
            if (l == i) aii += a * b / den;
            else if (cmark[l] == i) w[cpos[l]] += a * b / den;
          }
        }
        row.clear();
        if (aii != 0.0)
          for (size_t t = 0; t < hat.size(); ++t)
            if (w[t] != 0.0) row.emplace_back(cidx[hat[t]], -w[t] / aii);
        // truncation
        if (!row.empty()) {
          double sum = 0.0, mx = 0.0;
          for (auto& e : row) { sum += e.second; mx = std::max(mx, std::fabs(e.second)); }
          std::vector<std::pair<int, double>> kept;
          for (auto& e : row)
            if (std::fabs(e.second) >= kTruncRel * mx) kept.push_back(e);
          if ((int)kept.size() > kTruncMax) {
            std::stable_sort(kept.begin(), kept.end(), [](const std::pair<int, double>& a, const std::pair<int, double>& b) {
              return std::fabs(a.second) > std::fabs(b.second);
            });
            kept.resize(kTruncMax);
          }
          double ks = 0.0;
          for (auto& e : kept) ks += e.second;
          const double sc = ks != 0.0 ? sum / ks : 1.0;
          std::sort(kept.begin(), kept.end());
          for (auto& e : kept) {
            out.col.push_back(e.first);
            out.val.push_back(e.second * sc);
          }
        }
      }
      out.rowlen.push_back((int)(out.col.size() - len0));
    }
  });
  // The chunks are joined in row order by parallel copies to offsets from
  // per-chunk prefix sums (here and for the products below).
  const std::vector<size_t> row0 = chunk_offsets(nth, [&](int t) { return pch[t].rowlen.size(); });
  {
    const std::vector<size_t> eo = chunk_offsets(nth, [&](int t) { return pch[t].col.size(); });
    L.pptr.assign(n + 1, 0);
    L.pcol.resize(eo[nth]);
    L.pval.resize(eo[nth]);
    per_chunk(nth, eo[nth], [&](int t) {
      PChunk& ch = pch[t];
      std::copy(ch.col.begin(), ch.col.end(), L.pcol.begin() + eo[t]);
      std::copy(ch.val.begin(), ch.val.end(), L.pval.begin() + eo[t]);
      size_t e = eo[t];
      for (size_t r = 0; r < ch.rowlen.size(); ++r) L.pptr[row0[t] + r + 1] = (int)(e += ch.rowlen[r]);
      ch = PChunk();
    });
  }


  // ---- R = P^T
  L.rptr.assign(nc + 1, 0);
  for (int J : L.pcol) L.rptr[J + 1]++;
  for (int I = 0; I < nc; ++I) L.rptr[I + 1] += L.rptr[I];
  L.rcol.resize(L.pcol.size());
  L.rsrc.resize(L.pcol.size());
  {
    std::vector<int> fill(L.rptr.begin(), L.rptr.end() - 1);
    for (int i = 0; i < n; ++i)
      for (int p = L.pptr[i]; p < L.pptr[i + 1]; ++p) {
        const int e = fill[L.pcol[p]]++;
        L.rcol[e] = i;
        L.rsrc[e] = p;
      }
  }

  // Products of one output row are generated in a fixed order and grouped
  // by column: columns ascending, each column's products in generation order.
  // Rows are processed in contiguous chunks on host threads; every chunk
  // fills lists of its own and the chunks are joined in row order, so the
  // result does not depend on the number of threads.
  std::vector<ApChunk> apc(nth);
  parallel_chunks(n, nth, [&](int t, int lo, int hi) {
    ApChunk& ch = apc[t];
    {   // capacity: the chunk's products bound its entries (untouched capacity costs no memory)
      size_t np = 0;
      for (int i = lo; i < hi; ++i) {
        np += L.pptr[i + 1] - L.pptr[i];
        for (int q = A.ptr[i]; q < A.ptr[i + 1]; ++q) np += L.pptr[A.col[q] + 1] - L.pptr[A.col[q]];
      }
      ch.la.reserve(np);
      ch.lp.reserve(np);
      ch.col.reserve(np);
      ch.pidx.reserve(np);
      ch.nprod.reserve(np);
      ch.val.reserve(np);
      ch.rowlen.reserve(hi - lo);
    }
    RowGrouper g(nc);
    for (int i = lo; i < hi; ++i) {
      g.items.clear();
      for (int p = L.pptr[i]; p < L.pptr[i + 1]; ++p) g.items.push_back({L.pcol[p], dia_code(i), p});
      for (int q = A.ptr[i]; q < A.ptr[i + 1]; ++q) {
        const int j = A.col[q];
        for (int p = L.pptr[j]; p < L.pptr[j + 1]; ++p) g.items.push_back({L.pcol[p], off_code(q), p});
      }
      g.group(i);
      int k = 0;
      for (size_t c = 0; c < g.cols.size(); ++c) {
        const int J = g.cols[c];
        double v = 0.0;
        const int k0 = k;
        for (; k < g.start[c]; ++k) {
          const int code = g.grouped[k].a;
          v += ((code & 1) ? A.val[code >> 1] : A.diag[code >> 1]) * L.pval[g.grouped[k].b];
          ch.la.push_back(code);
          ch.lp.push_back(g.grouped[k].b);
        }
        int pidx = -1;
        for (int p = L.pptr[i]; p < L.pptr[i + 1]; ++p)
          if (L.pcol[p] == J) pidx = p;
        ch.col.push_back(J);
        ch.pidx.push_back(pidx);
        ch.nprod.push_back(k - k0);
        ch.val.push_back(v);
      }
      ch.rowlen.push_back((int)g.cols.size());
    }
  });
  // ---- A P: pattern, products, values (joined in row order)
  HostArray<double> apv;
  {
    const std::vector<size_t> eo = chunk_offsets(nth, [&](int t) { return apc[t].col.size(); });
    const std::vector<size_t> po = chunk_offsets(nth, [&](int t) { return apc[t].la.size(); });
    L.apptr.assign(n + 1, 0);
    L.apcol.resize(eo[nth]);
    L.appidx.resize(eo[nth]);
    apv.resize(eo[nth]);
    L.aplptr.resize(eo[nth] + 1);
    L.aplptr[0] = 0;
    L.apla.resize(po[nth]);
    L.aplp.resize(po[nth]);
    per_chunk(nth, po[nth], [&](int t) {
      ApChunk& ch = apc[t];
      std::copy(ch.col.begin(), ch.col.end(), L.apcol.begin() + eo[t]);
      std::copy(ch.pidx.begin(), ch.pidx.end(), L.appidx.data() + eo[t]);
      std::copy(ch.val.begin(), ch.val.end(), apv.data() + eo[t]);
      std::copy(ch.la.begin(), ch.la.end(), L.apla.data() + po[t]);
      std::copy(ch.lp.begin(), ch.lp.end(), L.aplp.data() + po[t]);
      size_t e = eo[t], q = po[t];
      for (size_t r = 0; r < ch.rowlen.size(); ++r) L.apptr[row0[t] + r + 1] = (int)(e += ch.rowlen[r]);
      for (size_t k = 0; k < ch.nprod.size(); ++k) L.aplptr[eo[t] + k + 1] = (int)(q += ch.nprod[k]);
      ch = ApChunk();
    });
  }

  // ---- P^T (A P): coarse pattern, products (off-diagonal entries, then the diagonal), values
  HostCsr& C = L.C;
  C.n = nc;
  C.diag.assign(nc, 0.0);
  C.ptr.assign(nc + 1, 0);
  std::vector<RapChunk> rpc(nth);
  parallel_chunks(nc, nth, [&](int t, int lo, int hi) {
    RapChunk& ch = rpc[t];
    {
      size_t np = 0;
      for (int I = lo; I < hi; ++I)
        for (int e = L.rptr[I]; e < L.rptr[I + 1]; ++e) np += L.apptr[L.rcol[e] + 1] - L.apptr[L.rcol[e]];
      for (auto* v : {&ch.col, &ch.nprod, &ch.r, &ch.q, &ch.dr, &ch.dq}) v->reserve(np);
      ch.val.reserve(np);
      ch.rowlen.reserve(hi - lo);
      ch.ndiag.reserve(hi - lo);
    }
    RowGrouper g(nc);
    for (int I = lo; I < hi; ++I) {
      g.items.clear();
      for (int e = L.rptr[I]; e < L.rptr[I + 1]; ++e) {
        const int i = L.rcol[e], p = L.rsrc[e];
        for (int q = L.apptr[i]; q < L.apptr[i + 1]; ++q) g.items.push_back({L.apcol[q], p, q});
      }
      g.group(I);
      int k = 0, noff = 0, ndg = 0;
      for (size_t c = 0; c < g.cols.size(); ++c) {
        const int J = g.cols[c];
        const bool dg = J == I;
        double v = 0.0;
        const int k0 = k;
        for (; k < g.start[c]; ++k) {
          v += L.pval[g.grouped[k].a] * apv[g.grouped[k].b];
          if (dg) { ch.dr.push_back(g.grouped[k].a); ch.dq.push_back(g.grouped[k].b); }
          else { ch.r.push_back(g.grouped[k].a); ch.q.push_back(g.grouped[k].b); }
        }
        if (dg) {
          C.diag[I] = v;   // rows are disjoint between chunks
          ndg += k - k0;
        } else {
          ch.col.push_back(J);
          ch.val.push_back(v);
          ch.nprod.push_back(k - k0);
          ++noff;
        }
      }
      ch.rowlen.push_back(noff);
      ch.ndiag.push_back(ndg);
    }
  });
  // products: the off-diagonal entries' lists in CSR order, then the
  // diagonal's lists row by row; clptr ends every entry's list
  {
    const std::vector<size_t> crow0 = chunk_offsets(nth, [&](int t) { return rpc[t].rowlen.size(); });
    const std::vector<size_t> eo = chunk_offsets(nth, [&](int t) { return rpc[t].col.size(); });
    const std::vector<size_t> po = chunk_offsets(nth, [&](int t) { return rpc[t].r.size(); });
    const std::vector<size_t> dof = chunk_offsets(nth, [&](int t) { return rpc[t].dr.size(); });
    const size_t ne = eo[nth], base = po[nth];
    C.col.resize(ne);
    C.val.resize(ne);
    L.clptr.resize(ne + 1 + nc);
    L.clptr[0] = 0;
    L.clr.resize(base + dof[nth]);
    L.clq.resize(base + dof[nth]);
    per_chunk(nth, base + dof[nth], [&](int t) {
      RapChunk& ch = rpc[t];
      std::copy(ch.col.begin(), ch.col.end(), C.col.begin() + eo[t]);
      std::copy(ch.val.begin(), ch.val.end(), C.val.begin() + eo[t]);
      std::copy(ch.r.begin(), ch.r.end(), L.clr.data() + po[t]);
      std::copy(ch.q.begin(), ch.q.end(), L.clq.data() + po[t]);
      std::copy(ch.dr.begin(), ch.dr.end(), L.clr.data() + base + dof[t]);
      std::copy(ch.dq.begin(), ch.dq.end(), L.clq.data() + base + dof[t]);
      size_t e = eo[t], q = po[t], d = base + dof[t];
      for (size_t k = 0; k < ch.nprod.size(); ++k) L.clptr[eo[t] + k + 1] = (int)(q += ch.nprod[k]);
      for (size_t r = 0; r < ch.rowlen.size(); ++r) {
        const size_t I = crow0[t] + r;
        C.ptr[I + 1] = (int)(e += ch.rowlen[r]);
        L.clptr[ne + 1 + I] = (int)(d += ch.ndiag[r]);
      }
      ch = RapChunk();
    });
  }
  return true;
}

}  // namespace spfas
