// Coarse levels (l >= 1) and transfers between levels.
#pragma once

#include "common.hpp"

namespace spfas {

struct Hierarchy;
struct CoarseLevel {};
struct TransferDev {};

// Builds the device data of every coarse level and transfer of h.
void setup_coarse_levels(Hierarchy& h);

}  // namespace spfas
