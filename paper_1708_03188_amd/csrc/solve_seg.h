#pragma once
#include "kernels.h"

namespace sgm {
// Galerkin solves with each (column, parity) chain split over K lanes of
// R rows each (R = 16, the default, or 8; K a power of two <= kSegMaxLanes).
constexpr int kSegRows = 16;
constexpr int kSegMaxLanes = 16;

// Lanes per chain for chains of at most nmax rows at R rows per lane; 0 if too
// long (or R is not 8 or 16).
int seg_lanes(int nmax, int R = kSegRows);
// Doubles of the boundary-state table of a plan.
size_t seg_table_doubles(int kind, int K, int ncols);
// Fill the table (w state of the elimination at every segment boundary);
// depends on the plan and alpha only.
hipError_t launch_seg_table(double* tab, const ChebDev& cd, const ColGeom& g, int kind, int K, int R, double alpha,
                            hipStream_t s);
// Solve in -> out (in may equal out) with a table filled for the same alpha.
hipError_t launch_solve_seg(const double2* in, double2* out, const double* tab, const ChebDev& cd, const ColGeom& g,
                            int kind, int K, int R, double alpha, hipStream_t s);
}  // namespace sgm
