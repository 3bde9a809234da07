// Gather and scatter of the bond updates of a larger unit cell (k_cell.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace ntu {

constexpr int CELL_GROUP_MAX = 48;

// One launch group: n independent bond updates, for bond k the cell sites of
// its eight cluster roles [X, Y, L, TX, BX, TY, BY, Rn] and whether it is
// vertical (its tensors then turned a quarter turn clockwise).
struct CellGroup {
  int n;
  int site[CELL_GROUP_MAX][8];
  int vert[CELL_GROUP_MAX];
};

// work (role r, bond k at (r n + k) nsite) <- the cell's site tensors, turned
// for vertical bonds; nsite = p D^4
hipError_t launch_cell_gather(bool cplx, const void* cell, void* work, int p, int D, const CellGroup& g,
                              hipStream_t st);
// the cell's X and Y sites of every bond <- roles 0 and 1 of work, turned
// back counter-clockwise for vertical bonds
hipError_t launch_cell_scatter(bool cplx, void* cell, const void* work, int p, int D, const CellGroup& g,
                               hipStream_t st);

}  // namespace ntu
