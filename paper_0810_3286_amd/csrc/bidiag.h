// SVD of a small upper-bidiagonal matrix on the host (FP64).
//
// B (k x k) has diagonal d[0..k-1] and superdiagonal e[0..k-2].  The
// bidiagonalisation of the sparse iterate produces B; its singular values are
// the Ritz values and its singular vectors combine the Lanczos bases into Ritz
// vectors.
#pragma once

#include <vector>

namespace svt {

struct BidiagSVD {
  std::vector<double> sigma;   // k values, descending
  std::vector<double> P;       // left vectors, k x k column-major (if requested),
                               // formed as B q_i / sigma_i (zero for sigma_i = 0)
  std::vector<double> Q;       // right vectors, k x k column-major (if requested)
  std::vector<double> p_last;  // last row of P (always computed), k entries
};

// Implicit-shift QR (Golub-Kahan step with a Wilkinson shift, zero-diagonal
// deflation by Givens chasing).  With vectors = false only sigma and the last
// row of P are formed (O(k^2) work); with vectors = true also Q (accumulated)
// and P (from Q).
// Returns false for non-finite input or if the sweep cap (30 k + 1000) is hit.
bool bidiag_svd(const std::vector<double> &d, const std::vector<double> &e, bool vectors,
                BidiagSVD &out);

}  // namespace svt
