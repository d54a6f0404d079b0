// Small dense FP64 kernels on the host for the randomised partial SVD
// (Section 6): an orthonormal basis of a tall block of columns, and the SVD
// of a tall matrix with few columns.  Column-major storage throughout.
#pragma once

#include <cstdint>
#include <vector>

namespace svt {

// Z (rows x cols, leading dimension rows) <- an orthonormal basis of its
// column span, by modified Gram-Schmidt applied twice to every column (a
// column that vanishes against the earlier ones is left zero).
void orth_columns(double *Z, int64_t rows, int cols);

// W (rows x cols, rows >= cols) = Vw diag(sigma) Uw^T by one-sided Jacobi
// rotations on W's columns (Hestenes; each rotation in Rutishauser's form),
// until every pair of columns is orthogonal to machine precision.  sigma is
// sorted in decreasing order; Vw is rows x cols (the normalised columns,
// zero where sigma is zero), Uw cols x cols orthogonal.  Returns false if
// the sweeps did not settle.
bool jacobi_svd_tall(const double *W, int64_t rows, int cols, std::vector<double> &sigma, std::vector<double> &Vw,
                     std::vector<double> &Uw);

}  // namespace svt
