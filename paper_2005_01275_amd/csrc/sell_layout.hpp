// Host-side SELL-64 layouts of the AMG operators: rows in slices of 64, each
// slice as wide as its longest row, slot (slice, k, lane) at
// ptr[slice] + 64 k + lane, so a wave reads slot k of its 64 rows in one
// coalesced access.  Slices are independent and laid out on host threads.
#pragma once

#include <climits>
#include <vector>

#include "common.hpp"

namespace spfas {

// Slice offsets for rows of `len(i)` stored entries (each slice at least one wide).
template <class Len>
std::vector<int> sell_slice_ptr(int n, Len len, const char* what) {
  const int ns = (n + 63) / 64;
  std::vector<int> width(ns, 1);
  parallel_ranges(
      ns,
      [&](int64_t lo, int64_t hi) {
        for (int64_t sl = lo; sl < hi; ++sl)
          for (int i = (int)sl * 64; i < std::min(n, (int)sl * 64 + 64); ++i) width[sl] = std::max(width[sl], len(i));
      },
      n);
  std::vector<int> sptr(ns + 1, 0);
  long long off = 0;
  for (int sl = 0; sl < ns; ++sl) {
    off += 64LL * width[sl];
    require(off < INT_MAX, what);
    sptr[sl + 1] = (int)off;
  }
  return sptr;
}

// SELL layout of a level's DIA+CSR matrix with the diagonal first in every
// row: columns (padding repeats the row's own index) and the source of every
// slot (-1 - i: diagonal of row i; q: off-diagonal entry q; pad: padding and
// lanes past the last row, whose column is 0).
inline void sell_matrix_layout(int n, const std::vector<int>& ptr, const std::vector<int>& colin, int pad,
                               std::vector<int>& sptr, std::vector<int>& col, std::vector<int>& map) {
  sptr = sell_slice_ptr(n, [&](int i) { return 1 + ptr[i + 1] - ptr[i]; }, "AMG level too large for 32-bit SELL offsets");
  const int ns = (n + 63) / 64;
  col.assign(sptr[ns], 0);
  map.assign(sptr[ns], pad);
  parallel_ranges(ns, [&](int64_t lo, int64_t hi) {
    for (int64_t sl = lo; sl < hi; ++sl) {
      const int width = (sptr[sl + 1] - sptr[sl]) / 64;
      for (int lane = 0; lane < 64; ++lane) {
        const int i = (int)sl * 64 + lane;
        const int base = sptr[sl] + lane;
        if (i >= n) continue;   // lanes past the last row are never read
        col[base] = i;
        map[base] = -1 - i;
        int k = 1;
        for (int q = ptr[i]; q < ptr[i + 1]; ++q, ++k) {
          col[base + 64 * k] = colin[q];
          map[base + 64 * k] = q;
        }
        for (; k < width; ++k) col[base + 64 * k] = i;
      }
    }
  }, (int64_t)col.size());
}

// SELL layout of CSR rows with a source code per entry: padding slots read
// the row's first column (0 for an empty row) with source -1; lanes past the
// last row hold column 0, source -1.
inline void sell_cyc_layout(int n, const std::vector<int>& ptr, const std::vector<int>& col,
                            const std::vector<int>& src, std::vector<int>& sptr, std::vector<int>& scol,
                            std::vector<int>& ssrc) {
  sptr = sell_slice_ptr(n, [&](int i) { return ptr[i + 1] - ptr[i]; }, "AMG operator too large for 32-bit SELL offsets");
  const int ns = (n + 63) / 64;
  scol.assign(sptr[ns], 0);
  ssrc.assign(sptr[ns], -1);
  parallel_ranges(ns, [&](int64_t lo, int64_t hi) {
    for (int64_t sl = lo; sl < hi; ++sl) {
      const int width = (sptr[sl + 1] - sptr[sl]) / 64;
      for (int lane = 0; lane < 64; ++lane) {
        const int i = (int)sl * 64 + lane;
        if (i >= n) continue;
        const int pad = ptr[i + 1] > ptr[i] ? col[ptr[i]] : 0;
        for (int k = 0; k < width; ++k) {
          const int slot = sptr[sl] + 64 * k + lane;
          if (ptr[i] + k < ptr[i + 1]) {
            scol[slot] = col[ptr[i] + k];
            ssrc[slot] = src[ptr[i] + k];
          } else {
            scol[slot] = pad;
          }
        }
      }
    }
  }, (int64_t)scol.size());
}

// CSR rows of A diag(w) for a DIA+CSR matrix: every row as [diagonal,
// off-diagonal entries], with the entry codes of the product lists.
inline void aw_rows(int n, const std::vector<int>& ptr, const std::vector<int>& colin, std::vector<int>& p,
                    std::vector<int>& c, std::vector<int>& src, int (*dia)(int), int (*off)(int)) {
  p.assign(n + 1, 0);
  for (int i = 0; i <= n; ++i) p[i] = i + ptr[i];
  c.resize(p[n]);
  src.resize(p[n]);
  parallel_ranges(n, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      int e = p[i];
      c[e] = (int)i;
      src[e++] = dia((int)i);
      for (int k = ptr[i]; k < ptr[i + 1]; ++k, ++e) {
        c[e] = colin[k];
        src[e] = off(k);
      }
    }
  }, (int64_t)c.size());
}

}  // namespace spfas
