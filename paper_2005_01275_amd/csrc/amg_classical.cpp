// Classical AMG setup on the host (see amg_host.hpp): PMIS coarsening
// (De Sterck, Yang, Heys 2006), extended+i interpolation (De Sterck,
// Falgout, Nolting, Yang 2008) with truncation, and the symbolic Galerkin
// products with their per-entry product lists.
#include "amg_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>

namespace spfas {

namespace {

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
  const int n = A.n;
  Strength S;
  S.ptr.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    double mx = 0.0;
    for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
      if (A.col[k] != i) mx = std::max(mx, -A.val[k]);
    if (mx > 0.0)
      for (int k = A.ptr[i]; k < A.ptr[i + 1]; ++k)
        if (A.col[k] != i && -A.val[k] >= theta * mx) S.col.push_back(A.col[k]);
    S.ptr[i + 1] = (int)S.col.size();
  }
  S.tptr.assign(n + 1, 0);
  for (int j : S.col) S.tptr[j + 1]++;
  for (int i = 0; i < n; ++i) S.tptr[i + 1] += S.tptr[i];
  S.tcol.resize(S.col.size());
  std::vector<int> fill(S.tptr.begin(), S.tptr.end() - 1);
  for (int i = 0; i < n; ++i)
    for (int q = S.ptr[i]; q < S.ptr[i + 1]; ++q) S.tcol[fill[S.col[q]]++] = i;
  return S;
}

// state: 1 = C, -1 = F
std::vector<int> pmis(const Strength& S, int n, uint64_t seed) {
  std::vector<double> lam(n);
  std::vector<int> state(n, 0);
  for (int i = 0; i < n; ++i) {
    const int ns = S.ptr[i + 1] - S.ptr[i], nt = S.tptr[i + 1] - S.tptr[i];
    lam[i] = nt + unit_hash(seed, (uint64_t)i);
    if (ns == 0 && nt == 0) state[i] = -1;   // isolated point: smoothing only
  }
  std::vector<int> und;
  for (int i = 0; i < n; ++i)
    if (state[i] == 0) und.push_back(i);
  std::vector<char> newc(n, 0);
  while (!und.empty()) {
    auto beats = [&](int j, int i) { return state[j] == 0 && (lam[j] > lam[i] || (lam[j] == lam[i] && j > i)); };
    std::vector<int> sel;
    for (int i : und) {
      bool mx = true;
      for (int q = S.ptr[i]; q < S.ptr[i + 1] && mx; ++q) mx = !beats(S.col[q], i);
      for (int q = S.tptr[i]; q < S.tptr[i + 1] && mx; ++q) mx = !beats(S.tcol[q], i);
      if (mx) sel.push_back(i);
    }
    for (int i : sel) { state[i] = 1; newc[i] = 1; }
    std::vector<int> rest;
    for (int i : und) {
      if (state[i] != 0) continue;
      bool dep = false;
      for (int q = S.ptr[i]; q < S.ptr[i + 1] && !dep; ++q) dep = newc[S.col[q]];
      if (dep) state[i] = -1;
      else rest.push_back(i);
    }
    for (int i : sel) newc[i] = 0;
    und.swap(rest);
  }
  return state;
}

}  // namespace

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

  // ---- extended+i interpolation, truncated
  L.pptr.assign(n + 1, 0);
  std::vector<int> smark(n, -1), cmark(n, -1), cpos(n, 0);
  std::vector<int> hat;          // C-hat_i
  std::vector<double> w;         // accumulated numerators over C-hat_i
  std::vector<std::pair<int, double>> row;
  for (int i = 0; i < n; ++i) {
    if (state[i] == 1) {
      L.pcol.push_back(cidx[i]);
      L.pval.push_back(1.0);
      L.pptr[i + 1] = (int)L.pcol.size();
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
          L.pcol.push_back(e.first);
          L.pval.push_back(e.second * sc);
        }
      }
    }
    L.pptr[i + 1] = (int)L.pcol.size();
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
  struct Item { int key, a, b; };
  std::vector<Item> items, grouped;
  std::vector<int> mark(nc, -1), slot(nc, 0), cols, start;
  auto group_row = [&](int tag) {
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
    // start[c] is now the end of column c's products
  };

  // ---- A P: pattern, products, values (for the next level's setup)
  L.apptr.assign(n + 1, 0);
  L.aplptr.assign(1, 0);
  std::vector<double> apv;
  for (int i = 0; i < n; ++i) {
    items.clear();
    for (int p = L.pptr[i]; p < L.pptr[i + 1]; ++p) items.push_back({L.pcol[p], dia_code(i), p});
    for (int q = A.ptr[i]; q < A.ptr[i + 1]; ++q) {
      const int j = A.col[q];
      for (int p = L.pptr[j]; p < L.pptr[j + 1]; ++p) items.push_back({L.pcol[p], off_code(q), p});
    }
    group_row(i);
    int t = 0;
    for (size_t c = 0; c < cols.size(); ++c) {
      const int J = cols[c];
      double v = 0.0;
      for (; t < start[c]; ++t) {
        const int code = grouped[t].a;
        v += ((code & 1) ? A.val[code >> 1] : A.diag[code >> 1]) * L.pval[grouped[t].b];
        L.apla.push_back(code);
        L.aplp.push_back(grouped[t].b);
      }
      int pidx = -1;
      for (int p = L.pptr[i]; p < L.pptr[i + 1]; ++p)
        if (L.pcol[p] == J) pidx = p;
      L.apcol.push_back(J);
      L.appidx.push_back(pidx);
      L.aplptr.push_back((int)L.apla.size());
      apv.push_back(v);
    }
    L.apptr[i + 1] = (int)L.apcol.size();
  }

  // ---- P^T (A P): coarse pattern, products (off-diagonal entries, then the diagonal), values
  std::fill(mark.begin(), mark.end(), -1);
  HostCsr& C = L.C;
  C.n = nc;
  C.diag.assign(nc, 0.0);
  C.ptr.assign(nc + 1, 0);
  std::vector<int> dptr(nc + 1, 0), dr, dq;
  L.clptr.assign(1, 0);
  for (int I = 0; I < nc; ++I) {
    items.clear();
    for (int e = L.rptr[I]; e < L.rptr[I + 1]; ++e) {
      const int i = L.rcol[e], p = L.rsrc[e];
      for (int q = L.apptr[i]; q < L.apptr[i + 1]; ++q) items.push_back({L.apcol[q], p, q});
    }
    group_row(I);
    int t = 0;
    for (size_t c = 0; c < cols.size(); ++c) {
      const int J = cols[c];
      const bool dg = J == I;
      double v = 0.0;
      for (; t < start[c]; ++t) {
        v += L.pval[grouped[t].a] * apv[grouped[t].b];
        if (dg) { dr.push_back(grouped[t].a); dq.push_back(grouped[t].b); }
        else { L.clr.push_back(grouped[t].a); L.clq.push_back(grouped[t].b); }
      }
      if (dg) {
        C.diag[I] = v;
      } else {
        C.col.push_back(J);
        C.val.push_back(v);
        L.clptr.push_back((int)L.clr.size());
      }
    }
    C.ptr[I + 1] = (int)C.col.size();
    dptr[I + 1] = (int)dr.size();
  }
  const int base = (int)L.clr.size();
  for (int I = 0; I < nc; ++I) L.clptr.push_back(base + dptr[I + 1]);
  L.clr.insert(L.clr.end(), dr.begin(), dr.end());
  L.clq.insert(L.clq.end(), dq.begin(), dq.end());
  return true;
}

}  // namespace spfas
