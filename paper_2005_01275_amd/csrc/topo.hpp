// Host-side integer structure of the hierarchy: lattice recovery, box
// aggregation, renumbering and the coarse topology (Section 3.1 and
// Appendix A: aggregates of cells, coarse interfaces between aggregates,
// bubbles).  No floating-point arithmetic of the method happens here.
#pragma once

#include <cstdint>
#include <vector>

namespace spfas {

enum FluxKind : int8_t { FK_INTERIOR = 0, FK_DIRICHLET = 1, FK_BUBBLE = 2 };

// One level in canonical order (level 0: input order of cells and of the
// non-Neumann faces; coarse levels: aggregate ids and coarse flux ids).
struct Topo {
  int64_t n_cells = 0;
  std::vector<int64_t> pptr;     // [n_cells+1] pressure unknowns of each cell
  int64_t n_flux = 0;
  std::vector<int8_t> kind;      // [n_flux]
  std::vector<int64_t> c1, c2;   // [n_flux] owning cells; c2 = -1 if one cell
  std::vector<int64_t> cfptr;    // [n_cells+1] local flux lists, ascending ids
  std::vector<int64_t> cfidx;
  std::vector<int> lat_shape;    // lattice of the level (box aggregation)
  std::vector<int64_t> lat_index;
  // filled when the level is coarsened
  std::vector<int64_t> agg;      // [n_cells] aggregate id
  int64_t n_agg = 0;
  std::vector<int> agg_shape;
  std::vector<int64_t> cell_order, flux_order;   // renumbered position -> id
  int64_t n_p() const { return pptr.empty() ? 0 : pptr.back(); }
};

// Lattice from centroids: per axis the rank of the coordinate among the
// distinct values.  Returns false if the cells do not fill the lattice
// exactly once.
bool lattice_from_centroids(int dim, int64_t n, const double* centroid, std::vector<int>& shape,
                            std::vector<int64_t>& index);

int box_blocks(int n, int a);
void box_aggregate(Topo& t, const int box[3]);
// aggregation given by the caller (validated: ids dense, aggregates connected)
void user_aggregate(Topo& t, const int32_t* agg, int64_t len);
// greedy graph aggregation of about `target` cells (rule in include/spfas.h)
void greedy_aggregate(Topo& t, int target);
void renumber(Topo& t);
void build_cell_lists(Topo& t);  // cfptr/cfidx from c1/c2
// Coarse topology from an aggregated level; m = eigenvectors per aggregate.
Topo coarse_topology(const Topo& fine, int m);   // min(m, unknowns of A) eigenvectors per aggregate A
Topo coarse_topology(const Topo& fine, const std::vector<int64_t>& mA);   // mA[A] per aggregate
// pressure unknowns of each aggregate of an aggregated level
std::vector<int64_t> aggregate_unknowns(const Topo& fine);

// Per-transfer index plan, level l (device numbering `dev_cell`/`dev_p`/
// `dev_flux` = canonical id -> device index) to level l+1 (canonical).
struct TransferPlan {
  int64_t n_agg = 0;
  std::vector<int64_t> cell_ptr, cell_list;  // per aggregate: level-l device cells
  std::vector<int64_t> pd_ptr, pd_list;      // per aggregate: level-l device p unknowns
  std::vector<int64_t> int_ptr;              // int(A) = dof_list[dof_ptr[A] .. dof_ptr[A]+nint]
  std::vector<int64_t> dof_ptr, dof_list;    // dofs(A): int(A) then boundary groups in A's
                                             // coarse-local order (interfaces, Dirichlet)
  std::vector<int32_t> n_int;                // |int(A)|
  std::vector<int32_t> mA;
  std::vector<int64_t> fgrp_ptr, fgrp_list;  // per coarse flux: level-l device flux ids (faces)
  std::vector<int64_t> grp_pos_A;            // per coarse flux (face): offset of its group in dofs(c1)
  std::vector<int64_t> grp_pos_B;            // ... in dofs(c2) (-1 if none)
  // scatter map: for each aggregate A, each cell of A (cell_list order), each
  // local flux of that cell (device local order): position in dofs(A)
  std::vector<int64_t> smap_ptr;             // [cell_list.size()+1]
  std::vector<int32_t> smap;
};

// `dev_cfptr/dev_cfidx`: the level-l device local flux lists indexed by
// device cell id (device flux ids, device local order).
TransferPlan make_plan(const Topo& fine, const Topo& coarse, const std::vector<int64_t>& dev_cell,
                       const std::vector<int64_t>& dev_p, const std::vector<int64_t>& dev_flux,
                       const std::vector<int64_t>& dev_cfptr,
                       const std::vector<int64_t>& dev_cfidx);

}  // namespace spfas
