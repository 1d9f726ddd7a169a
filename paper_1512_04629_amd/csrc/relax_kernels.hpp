// Hybrid Gauss-Seidel relaxation (the relaxation of the paper's experiments,
// Section 5): Gauss-Seidel inside contiguous blocks of rows, Jacobi across
// them.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace amg355 {

// One sweep: for each block of `block` consecutive rows, rows are visited in
// ascending (forward) or descending (backward) order and
//   xnew_i = (b_i - sum_{j != i} a_ij y_j) / a_ii,
// the terms subtracted in ascending column order, y_j the new value of a row
// of the same block visited before row i and xold_j otherwise.  Every row of
// xnew is written; xnew and xold must not overlap.  mean_row (entries per
// row) only sizes the chunks of the staged form.
void launch_hybrid_gs(bool forward, int n, const int32_t* rp, const int32_t* ci, const double* v,
                      const double* b, const double* xold, double* xnew, int block, double mean_row,
                      hipStream_t st);

}  // namespace amg355
