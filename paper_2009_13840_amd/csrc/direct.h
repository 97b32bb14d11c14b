// Sparse direct solver of the coarsest level (the paper's 2D coarse solver is a
// direct factorisation, Section 5.2): host-side symbolic phase.
//
// Ordering: nested dissection of the cells by recursive coordinate bisection.
// A face belongs to the front of the node where its two cells are separated (a
// leaf for faces inside it or on the boundary).  The coarsest operator is a
// saddle-point matrix (velocity faces, cell pressures), so a pressure may only be
// eliminated once enough velocity unknowns before it make the leading block
// nonsingular: within every set of cells connected through faces already
// eliminated, one pressure is held back and passed to the parent front; the one
// left at the root is the constant-pressure null space, which is pinned to zero
// (the solution is then made orthogonal to that null vector, which gives the
// bordered system's solution) or, when the operator is nonsingular, eliminated
// last; a batch of disjoint problems leaves one per member, each member's null
// space.  Within a front the faces come first, then the pressures placed there.
//
// The numeric phase (k_direct.hip) eliminates each front's own unknowns with the
// sweep operator, so that the stored front holds -F11^{-1}, F11^{-1} F12,
// F21 F11^{-1} and the update F22 - F21 F11^{-1} F12 that its parent assembles:
// the solves are then dense products, one launch per tree height each way.
#pragma once

#include <cstdint>
#include <vector>

#include "internal.h"

namespace hho {

constexpr int kNdLeafCells = 8;   // cells of a leaf of the dissection
constexpr int kNdSmall = 128;     // fronts of at most this many unknowns are eliminated in LDS
constexpr int kNdPanel = 64;      // pivots per panel of a larger front
constexpr int kNdTile = 64;       // rows and columns of a tile of a larger front
constexpr int kNdChunk = 64;      // rows of a front per block of the panel kernel
constexpr int kNdSolveRows = 32;  // rows of a front per block of the solve kernels (two waves of 16)

struct NdHost {
  int nfront = 0, nheight = 0;
  std::vector<int32_t> m, nfs;               // [nfront] unknowns of the front, of which eliminated there
  std::vector<int64_t> off, voff, dofoff;    // [nfront+1] front matrix (m*m), solve vector (m), unknown list
  std::vector<int32_t> dof;                  // [dofoff[nfront]] unknown at each front position
  std::vector<int32_t> cmap;                 // [2*dofoff[nfront]] position in child 0/1's update part, or -1
  std::vector<int32_t> child;                // [2*nfront] children, -1 if none
  std::vector<int64_t> soff;                 // [nfront] panel scratch offset (fronts of the larger heights)
  std::vector<int64_t> src, dst;             // operator entry (bsr | cpl | spp concatenated) -> front entry
  std::vector<int32_t> hfront, hptr;         // fronts by height
  std::vector<int32_t> tiles, tptr;          // (front, row, col) tiles (col <= row) of each larger height
  std::vector<int32_t> chunks, cptr;         // (front, first row) chunks of kNdChunk rows, every height
  std::vector<int32_t> schunks, scptr;       // the same with kNdSolveRows rows (solve kernels)
  std::vector<uint8_t> big;                  // [nheight] height eliminated by panels
  std::vector<int32_t> hmaxnfs, hmaxm;       // [nheight]
  int64_t total = 0, vtotal = 0, stotal = 0; // doubles of the fronts, solve vectors, panel scratch
  std::vector<int64_t> pins;                 // per member: the unknown fixed to zero, or -1
  std::vector<int64_t> segp;                 // [members+1] cell ranges of the members (one member: all cells)
  std::vector<int32_t> cseg;                 // [cells] member of every cell
  int maxm = 0;
  int64_t factor_entries = 0;                // stored entries used by the solves (sum of m^2 - up^2)
};

// The symbolic phase for the coarsest level of degree 0: d*p unknowns per face
// (face-major), t per cell after the faces; bsr blocks of size bs (v-cond: p, the
// block acting on every component; v&p-cond: d*p), cpl per (cell-face entry,
// face unknown, cell unknown), spp per cell (v-cond only).  pin: the operator has
// the constant-pressure null space (pure Dirichlet), one per member of a batch.
// seg_cell_ptr: the members' cell ranges of a batch (empty: one problem).
void nd_symbolic(const hho_mesh *mesh, int d, int p, int t, int cond, bool pin, const std::vector<int32_t> &rowptr,
                 const std::vector<int32_t> &col, const std::vector<int64_t> &seg_cell_ptr, NdHost *H);

}  // namespace hho
