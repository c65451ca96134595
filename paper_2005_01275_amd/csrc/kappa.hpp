// Device evaluation of the kappa families of KappaFam (fine.hpp): only
// 1/kappa and its derivative enter the method (Prop. 1, Props. 2-3).
#pragma once

#include "fine.hpp"

namespace spfas {

// psi = p - z_c (no shift: p itself, bit for bit)
__device__ inline double kap_psi(const double* z, double p, int64_t c) { return z ? p - z[c] : p; }

__device__ inline double kap_inv(const KappaFam& k, double psi) {
  if (k.kind == 0) return exp(-k.alpha * psi);
  return 1.0 + pow(fabs(psi), k.beta) / k.a;
}

// d(1/kappa)/d psi, given kinv = kap_inv(k, psi)
__device__ inline double kap_dinv(const KappaFam& k, double psi, double kinv) {
  if (k.kind == 0) return -k.alpha * kinv;
  return psi == 0.0 ? 0.0 : copysign(k.beta * pow(fabs(psi), k.beta - 1.0) / k.a, psi);
}

}  // namespace spfas
