// Host-side AMG setup structures (no device code).
//
// Classical AMG for the level-0 eliminated system: PMIS coarsening on the
// strong negative couplings, extended+i interpolation with truncation, and
// Galerkin coarse operators P^T A P.  The interpolation is computed once from
// the setup matrix and kept; the device recomputes A P and P^T (A P) after
// every linearisation from the product lists built here.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <memory>
#include <thread>
#include <vector>

namespace spfas {

// Host threads one setup step may use: at most 16, and at most
// tl_host_threads when a caller sets it (a serving worker takes its share,
// so that setups running side by side do not oversubscribe the host).
constexpr int kMaxHostThreads = 16;
inline thread_local int tl_host_threads = 0;
inline int host_thread_limit() {
  const int hc = (int)std::max(1u, std::thread::hardware_concurrency());
  const int lim = std::min(kMaxHostThreads, hc);
  return tl_host_threads > 0 ? std::min(lim, tl_host_threads) : lim;
}

// DIA+CSR matrix on the host: diagonal separately, off-diagonal entries in CSR.
struct HostCsr {
  int n = 0;
  std::vector<double> diag, val;
  std::vector<int> ptr, col;
};

// Entry codes of a DIA+CSR matrix in product lists: (i << 1) for the
// diagonal of row i, (k << 1) | 1 for off-diagonal entry k.
inline int dia_code(int i) { return i << 1; }
inline int off_code(int k) { return (k << 1) | 1; }

// Host array whose resize leaves the elements uninitialised: the product
// lists are written in full by the threads that fill them, which then also
// take the first-touch page faults in parallel.
template <class T>
struct HostArray {
  std::unique_ptr<T[]> a;
  size_t n = 0;
  void resize(size_t m) {
    a.reset(m ? new T[m] : nullptr);
    n = m;
  }
  size_t size() const { return n; }
  T* data() { return a.get(); }
  const T* data() const { return a.get(); }
  T& operator[](size_t i) { return a[i]; }
  const T& operator[](size_t i) const { return a[i]; }
};

struct ClassicalLevel {
  int n = 0, nc = 0;
  // interpolation P (n x nc), CSR with ascending columns in each row
  std::vector<int> pptr, pcol;
  std::vector<double> pval;
  // R = P^T (nc x n), CSR; rsrc[e] = P entry of R entry e
  std::vector<int> rptr, rcol, rsrc;
  // A P (n x nc): CSR pattern with ascending columns; products per entry
  // (A entry code, P entry); appidx[e] = P entry at the same position or -1
  std::vector<int> apptr, apcol;
  HostArray<int> aplptr, apla, aplp, appidx;
  // next level: DIA+CSR matrix and products per entry, off-diagonal entries
  // first (in CSR order) then the diagonal: (P entry, A P entry)
  HostCsr C;
  HostArray<int> clptr, clr, clq;
};

// Strength of connection of the classical coarsening: j is a strong
// dependence of i when -a_ij >= theta * max_k (-a_ik) > 0.
constexpr double kClassicalStrength = 0.25;
// Truncation of interpolation rows: drop |w| < kTruncRel * max |w|, keep at
// most kTruncMax entries, rescale to the row sum before truncation.
constexpr double kTruncRel = 0.2;
constexpr int kTruncMax = 4;

// One coarsening step of A.  Returns false when the coarsening stalls (no
// C-point or more than 90 % of the points kept); `seed` fixes the PMIS
// tie-breaking measure.
bool classical_level(const HostCsr& A, double theta, uint64_t seed, ClassicalLevel& L);

}  // namespace spfas
