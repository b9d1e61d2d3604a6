#pragma once
#include "kernels.h"

namespace sgm {
// Galerkin solves with one lane per (column, parity) chain; `scratch` holds
// 2 doubles per spectral element (the plan workspace).  in may equal out.
hipError_t launch_solve_chain(const double2* in, double2* out, double* scratch, const ChebDev& cd, const ColGeom& g,
                              int kind, double alpha, hipStream_t s);
}  // namespace sgm
