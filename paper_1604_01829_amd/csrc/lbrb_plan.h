// lbrb_plan.h -- host-only planners of the library: the compact fluid-row tables of a boundary
// mask, the node tiles of a replica, the moving-wall link list, the spatial order of a
// raspberry's beads and the excluded-volume site grids.  Plain C++ (no HIP call), so the same
// source builds into the library and, for the sanitizer checks, into a host program with g++.
#ifndef LBRB_PLAN_H
#define LBRB_PLAN_H

#include <stdint.h>

#include <vector>

#include "lbrb_layout.h"
#include "lbrb_walls.h"

namespace lbrb {

inline int64_t pad_nodes(int64_t n) { return (n + kNodeBlock - 1) / kNodeBlock * kNodeBlock; }

// excluded-volume grids: coarse cells per axis at most, fine flag cells at most 2 wide
constexpr int kMaxCellsPerAxis = 32;
constexpr double kFineCell = 2.0;
int cells_per_axis_cap(int n);
int fine_per_axis(int n);

// The fluid rows of one replica's boundary mask (nx*ny*nz wall ids, x fastest, 0 = fluid;
// Sec. 1.1 bounce-back nodes).  A (y,z) row stores the span from its first to its last fluid
// node; the boundary nodes inside the span are holes.
struct MaskRows {
    std::vector<RowDesc> rows;      // the rows with fluid, in (z, y) order
    std::vector<RowDesc> info;      // one per (y, z) at y + ny z; len 0 for a row without fluid
    std::vector<uint8_t> holes;     // per stored node: the wall id of a hole, else 0
    int64_t stored = 0;             // stored nodes: fluid nodes and holes
    int64_t n_holes = 0;
    bool any_solid = false;
};
MaskRows compress_mask(int nx, int ny, int nz, const uint8_t* mask);

// The node tiles of replica r (kNodeBlock stored nodes each, the last one ragged), appended to
// T.  For a masked replica, rows and rowinfo are the library's row tables (the replica's
// entries from R.row_base on) and each tile gets the range of rows[] that covers it.
void append_tiles(const ReplicaDesc& R, int32_t r, const RowDesc* rows, const RowDesc* rowinfo,
                  std::vector<NodeTile>& T);

// Moving-wall links of one replica: every stored fluid node x and direction i whose neighbour
// x - c_i (periodic) is a boundary node of a wall k with c_i . u_k != 0 (Ladd's moving
// bounce-back).  R, info (the rows per (y,z)) and mask (wall ids) are in storage coordinates:
// when R.swap the box's axes x and z are exchanged, so c_i steps by (c_iz, c_iy, c_ix) there.
// uwall holds three velocities per wall id (empty: no moving walls).  Sorted by the population
// slot they update.
std::vector<WallLink> build_links(const ReplicaDesc& R, const uint8_t* mask, const RowDesc* info,
                                  const std::vector<double>& uwall, double rho0);

// Morton (Z-order) ranking of n body-frame offsets on a half-lattice-unit grid (stable)
std::vector<int32_t> spatial_order(const double* offs, int32_t n);

// Excluded-volume site tables of the replicas, concatenated.
struct WcaTables {
    std::vector<int32_t> nb_start;  // per coarse cell: first entry in nb_sites; one extra end
    std::vector<WallSite> nb_sites; // each coarse cell's neighbourhood, the site records in place
    std::vector<WallSite> sites;    // the sites binned by coarse cell
    std::vector<uint8_t> near;      // fine cells whose centre lies within reach of a site
};
// The grids of one replica of side lengths dims with static sites `sites_in` and body sites of
// radius ev_r (< 0: no body sites): fills W's grid fields and appends to t.  The coarse cells
// are at least one interaction range wide (with a margin), so a site within range of a point
// lies in the point's cell or an adjacent one.  Returns false if a side is shorter than twice
// the largest range (the minimum image would be ambiguous).
bool wca_grid(const int dims[3], double ev_r, const std::vector<WallSite>& sites_in, WcaRep& W,
              WcaTables& t);

}  // namespace lbrb

#endif
