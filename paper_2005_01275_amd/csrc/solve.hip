#include "solve.hpp"
namespace spfas {
int run_solve(Hierarchy&, const spfas_problem&, const spfas_solve_opts&, double*, double*, bool, SolveKind,
              spfas_stats&) {
  fail(SPFAS_ERR_INVALID, "not built yet");
}
void export_level_operator(const Hierarchy&, int, int, double*, size_t) { fail(SPFAS_ERR_INVALID, "not built yet"); }
}
