// Locally refined meshes (octree leaves over n^3 Cartesian cells of the unit
// cube) with hanging nodes: host construction of the conforming equal-order
// Q_k space (k = 1, 2) and of the sparse maps from global unknowns to
// cell-local nodal values (the constraint matrices C_e of eq. (transfer),
// Sec. 2; locally refined meshes of Sec. 5).  Internal to the library.
//
// Node positions are integer points of the lattice of spacing
// 1 / (k n 2^L), L the finest level (the GLL nodes of k <= 2 are equispaced),
// so positions shared by several cells are found exactly.  A position that
// lies in the closed box of a coarser leaf without being one of its nodes is a
// hanging node: its value is that leaf's interpolant there, and a master node
// that is itself hanging is expanded in turn.  All other positions are the
// unknowns, numbered in lexicographic order of their position (x fastest).
#pragma once

#include <cstdint>
#include <vector>

#include "hp.h"

namespace mfs {

struct AmrSpaceHost {
  int n = 0, L = 0, k = 0;
  int64_t ncells = 0;
  int64_t R = 0;                 // lattice extent: positions 0..R per axis
  int64_t N = 0, nhanging = 0;   // unknowns, hanging positions
  std::vector<int64_t> tpos;     // [N][3] lattice positions of the unknowns
  std::vector<int> level;        // per cell
  std::vector<int> idx;          // per cell, [3]
  // maps in the form the E-vector kernels take: deg (all k), N, row_base,
  // row_ptr, col, val, dirichlet, owner_cell, owner_local
  HpSpaceHost V;
  std::vector<double> Xcell;     // [ncells][8][3] corner coordinates, x fastest

  // validates the leaves (levels, index ranges, a partition of the cube) and
  // builds everything above; throws mfs::Error(MFS_EINVAL) on bad input
  void build(int n, int L, int64_t ncells, const int *level, const int *idx, int k);
  // greedy colouring of the unknowns (needs the row maps): no two unknowns
  // that appear in one cell's rows share a colour
  std::vector<int> colours(int *ncolours) const;
};

// Global coarsening: every family of eight leaves replaced by its parent;
// cells listed by level, then lexicographically (x fastest) within a level.
void amr_coarsen(int n, const std::vector<int> &level, const std::vector<int> &idx, std::vector<int> &level_c,
                 std::vector<int> &idx_c);

// Cell relation between a mesh and its global coarsening: parent[f] = coarse
// cell holding fine cell f, octant[f] = child position (bit a: upper half
// along axis a) or 8 when the cell is unchanged; cptr/child list the fine
// cells of every coarse cell (CSR, ascending fine ids).
struct AmrTransferHost {
  std::vector<int> parent, child;
  std::vector<uint8_t> octant;
  std::vector<int64_t> cptr;
};
AmrTransferHost amr_transfer(int n, const std::vector<int> &lf, const std::vector<int> &xf,
                             const std::vector<int> &lc, const std::vector<int> &xc);
// for every unknown of the coarse space, the unknown of the fine space at the
// same position (each coarse unknown is one)
std::vector<int64_t> amr_injection(const AmrSpaceHost &fine, const AmrSpaceHost &coarse);

// Parallel efficiency of the multigrid levels of a refined mesh on P
// processes (partitions along the Morton curve): out = {eta_w, eta_v} of the
// global-coarsening levels, then of the local-smoothing levels
void amr_mg_metrics(int n, const std::vector<int> &level, const std::vector<int> &idx, int P, double out[4]);

}  // namespace mfs
