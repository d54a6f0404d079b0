// SVD of a small upper-bidiagonal matrix on the host (FP64).
//
// B (k x k) has diagonal d[0..k-1] and superdiagonal e[0..k-2].  The
// bidiagonalisation of the sparse iterate produces B; its singular values are
// the Ritz values and its singular vectors combine the Lanczos bases into Ritz
// vectors.
#pragma once

#include <vector>

namespace svt {

// One right rotation of the QR iteration: columns (a, b) of Q become
// (c q_a + s q_b, -s q_a + c q_b).
struct BidiagRot {
  int a, b;
  double c, s;
};

struct BidiagSVD {
  std::vector<double> sigma;   // k values, descending
  std::vector<double> p_last;  // last row of P (always computed), k entries
  int nvec = 0;                // columns in P and Q
  std::vector<double> P;       // first nvec left vectors, k x nvec column-major,
                               // formed as B q_i / sigma_i (zero for sigma_i = 0)
  std::vector<double> Q;       // first nvec right vectors, k x nvec column-major
  // for bidiag_vectors: the right rotations in order, and the unsorted
  // position and sign of each sorted value
  std::vector<BidiagRot> rots;
  std::vector<int> src;
  std::vector<signed char> sgn;
};

// Implicit-shift QR (Golub-Kahan step with a Wilkinson shift, zero-diagonal
// deflation by Givens chasing): sigma, the last row of P and the log of right
// rotations (O(k^2) work).  Returns false for non-finite input or if the
// sweep cap (30 k + 1000) is hit.
bool bidiag_svd(const std::vector<double> &d, const std::vector<double> &e, BidiagSVD &out);

// The first nvec singular vector pairs of the same B from out's rotation log
// (out from bidiag_svd on d, e): q_i = H_1 ... H_n e_src(i) applied to a unit
// vector (O(nvec) per rotation), p_i = B q_i / sigma_i.
void bidiag_vectors(const std::vector<double> &d, const std::vector<double> &e, int nvec, BidiagSVD &out);

// Both: with vectors, all k pairs.
bool bidiag_svd(const std::vector<double> &d, const std::vector<double> &e, bool vectors,
                BidiagSVD &out);

}  // namespace svt
