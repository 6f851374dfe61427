// build_mc.hpp -- launcher of the factored Monte Carlo entry kernel.
#pragma once

#include "impact_internal.hpp"

namespace impact {

// Entries of every row under correlated noise: the factored kernel (one
// workgroup per row, shared exp tables per chunk of points) when the grid has
// at most 5 dimensions and at most 16 candidate means per cell, else the
// direct kernel (launch_mc_entries).  gA (n_samples x (d + 1) doubles) and
// gmax (d doubles) are its temporaries.
hipError_t launch_mc_rows(const SysParams* sys, int32_t d, int64_t n_rows, int64_t n_ent,
                          const int32_t* win, const int64_t* row_off, double2* ent,
                          hipStream_t st, int32_t G, double* gA, double* gmax);

}  // namespace impact
