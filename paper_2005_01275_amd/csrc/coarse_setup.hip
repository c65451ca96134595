#include "coarse.hpp"
#include "hier.hpp"
namespace spfas {
void setup_coarse_levels(Hierarchy&) {}
}
