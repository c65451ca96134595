// Nonlinear solvers: FAS V-cycle (Alg. 2), nonlinear cascadic multigrid,
// single-level Picard/Newton, smoothing with the step cap and backtracking
// (Alg. 1).
#pragma once

#include "hier.hpp"

namespace spfas {

enum class SolveKind { FAS, PICARD, NEWTON, CASCADIC };

// level_steps (CASCADIC only, may be null): smoothing steps per level
int run_solve(Hierarchy& h, const spfas_problem& prob, const spfas_solve_opts& o, double* p, double* sigma,
              bool dev, SolveKind kind, spfas_stats& st, int32_t* level_steps = nullptr);

void export_level_operator(const Hierarchy& h, int level, int what, double* out, size_t count);

// device work space of the fine smoother and the AMG of its eliminated system
void setup_fine_solver(Hierarchy& h);

}  // namespace spfas
