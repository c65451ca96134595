#pragma once
namespace spfas {
struct SparseSolver {};
}
