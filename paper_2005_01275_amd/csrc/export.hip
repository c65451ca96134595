// Parity hooks: copies of hierarchy operators in canonical order
// (include/spfas.h, spfas_get_level_operator).
#include <algorithm>
#include <cstring>

#include "hier.hpp"
#include "solve.hpp"

namespace spfas {

void export_level_operator(const Hierarchy& h, int l, int what, double* out, size_t count) {
  require(l >= 0 && l + 1 < h.n_levels, "level must be below the coarsest level");
  hipStream_t s = h.stream;
  const TransferDev& T = *h.trans[l];
  const CoarseLevel& C = *h.coarse[l];
  const Topo& tf = h.topo[l];
  auto need = [&](size_t n) {
    if (count != n) {
      char buf[160];
      std::snprintf(buf, sizeof buf, "operator %d of level %d has %zu entries, %zu given", what, l, n, count);
      fail(SPFAS_ERR_INVALID, buf);
    }
  };
  // level-l device flux id -> canonical flux id
  std::vector<int64_t> canon_flux(tf.n_flux);
  if (l == 0)
    for (int64_t i = 0; i < tf.n_flux; ++i) canon_flux[i] = tf.flux_order[i];
  else
    for (int64_t i = 0; i < tf.n_flux; ++i) canon_flux[i] = i;
  switch (what) {
    case SPFAS_OP_EIGVALS: {
      need(h.eigvals[l].size());
      std::copy(h.eigvals[l].begin(), h.eigvals[l].end(), out);
      break;
    }
    case SPFAS_OP_PP: {
      std::vector<double> P = T.P.download(s);
      need(P.size());
      std::copy(P.begin(), P.end(), out);
      break;
    }
    case SPFAS_OP_MLOC: {
      std::vector<double> M = C.M.download(s);
      need(M.size());
      std::copy(M.begin(), M.end(), out);
      break;
    }
    case SPFAS_OP_DLOC: {
      std::vector<double> D = C.D.download(s);
      need(D.size());
      std::copy(D.begin(), D.end(), out);
      break;
    }
    case SPFAS_OP_MCOUNT: {
      need((size_t)C.n);
      for (int A = 0; A < C.n; ++A) out[A] = (double)(C.h_pptr[A + 1] - C.h_pptr[A]);
      break;
    }
    case SPFAS_OP_W: {
      std::vector<double> w = C.w.download(s);
      need(w.size());
      std::copy(w.begin(), w.end(), out);
      break;
    }
    case SPFAS_OP_PSIGMA: {
      const size_t nf = tf.n_flux, nc = C.nf;
      need(nf * nc);
      std::memset(out, 0, nf * nc * sizeof(double));
      std::vector<double> E = T.E.download(s), tr = T.trace.download(s);
      std::vector<int> dof_ptr = T.dof_ptr.download(s), dof_list = T.dof_list.download(s);
      std::vector<int> grp_of = T.grp_of.download(s);
      for (int A = 0; A < T.n_agg; ++A) {
        const int kA = C.h_lfptr[A + 1] - C.h_lfptr[A];
        for (int r = 0; r < T.h_nint[A]; ++r)
          for (int k = 0; k < kA; ++k)
            out[canon_flux[dof_list[dof_ptr[A] + r]] * nc + C.h_lfidx[C.h_lfptr[A] + k]] = E[T.h_Eptr[A] + r * kA + k];
      }
      for (size_t j = 0; j < nf; ++j)
        if (grp_of[j] >= 0) out[canon_flux[j] * nc + grp_of[j]] = tr[j];
      break;
    }
    case SPFAS_OP_QSIGMA: {
      const size_t nf = tf.n_flux, nc = C.nf;
      need(nf * nc);
      std::memset(out, 0, nf * nc * sizeof(double));
      std::vector<double> om = T.omega.download(s), P = T.P.download(s);
      std::vector<int> grp_of = T.grp_of.download(s), pd_list = T.pd_list.download(s);
      std::vector<int> cell_list = T.cell_list.download(s), cell_ptr = T.cell_ptr.download(s);
      for (size_t j = 0; j < nf; ++j)
        if (grp_of[j] >= 0) out[(size_t)grp_of[j] * nf + canon_flux[j]] = om[j];
      // bubble rows: v_j^T D^l restricted to the aggregate (local matrices of level l)
      std::vector<double> Dl;
      std::vector<int> dptr, lfptr, lfidx, pptr;
      std::vector<int> cfptr, cfcode;
      if (l == 0) {
        cfptr = h.fine.cfptr.download(s);
        cfcode = h.fine.cfcode.download(s);
      } else {
        const CoarseLevel& F = *h.coarse[l - 1];
        Dl = F.D.download(s);
        dptr = F.h_dptr;
        lfptr = F.h_lfptr;
        lfidx = F.h_lfidx;
        pptr = F.h_pptr;
      }
      for (int A = 0; A < T.n_agg; ++A) {
        const int mA = T.h_mA[A];
        if (mA < 2) continue;
        int bub0 = -1;
        for (int q = C.h_lfptr[A]; q < C.h_lfptr[A + 1]; ++q)
          if (C.h_kind[C.h_lfidx[q]] == FK_BUBBLE) { bub0 = C.h_lfidx[q]; break; }
        int row = 0;
        for (int ci = cell_ptr[A]; ci < cell_ptr[A + 1]; ++ci) {
          const int c = cell_list[ci];
          if (l == 0) {
            for (int k = cfptr[c]; k < cfptr[c + 1]; ++k) {
              const int code = cfcode[k];
              const double d = (code & 1) ? 1.0 : -1.0;
              for (int j = 1; j < mA; ++j)
                out[(size_t)(bub0 + j - 1) * nf + canon_flux[code >> 1]] += P[T.h_Pptr[A] + row * mA + j] * d;
            }
            row += 1;
          } else {
            const int k = lfptr[c + 1] - lfptr[c], m = pptr[c + 1] - pptr[c];
            for (int r = 0; r < m; ++r)
              for (int i = 0; i < k; ++i)
                for (int j = 1; j < mA; ++j)
                  out[(size_t)(bub0 + j - 1) * nf + canon_flux[lfidx[lfptr[c] + i]]] +=
                      P[T.h_Pptr[A] + (row + r) * mA + j] * Dl[dptr[c] + r * k + i];
            row += m;
          }
        }
      }
      break;
    }
    default:
      fail(SPFAS_ERR_INVALID, "unknown operator code");
  }
}

}  // namespace spfas
