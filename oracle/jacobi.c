/*
 * Test infrastructure, not product code: only the tests, the smoke check and
 * the CPU-baseline leg of the benchmark may load this library.
 *
 * One-sided Jacobi SVD (Hestenes, 1958), the dense full SVD the oracle uses to
 * evaluate the singular value shrinkage operator D_tau of Section 2.1
 * (eq. (2.2)): D_tau needs the singular values and vectors of the iterate.
 *
 * Method: orthogonalise the columns of A (m x n, m >= n) by plane rotations
 * applied from the right, A <- A J, accumulating V <- V J, sweeping the pairs
 * (p, q), p < q, in cyclic-by-row order.  A pair is left alone when its
 * columns are already orthogonal to working precision,
 *     |a_p . a_q| <= tol * ||a_p|| ||a_q||.
 * The sweeps stop after one in which no pair was rotated.  Then the column
 * norms are the singular values, the normalised columns are the left singular
 * vectors and V holds the right singular vectors.  Results are sorted by
 * decreasing singular value.
 *
 * The rotation for a pair zeroes the off-diagonal entry of the 2 x 2 Gram
 * matrix [[alpha, gamma], [gamma, beta]] (alpha = |a_p|^2, beta = |a_q|^2,
 * gamma = a_p . a_q): with zeta = (beta - alpha) / (2 gamma) the smaller root
 * t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)) of t^2 + 2 zeta t - 1 = 0 gives
 * c = 1 / sqrt(1 + t^2), s = c t, and the new columns are
 *     a_p' = c a_p - s a_q,   a_q' = s a_p + c a_q.
 * (Rutishauser's form of the Jacobi angle; the smaller root keeps the
 * rotation angle at most pi/4, which makes the cyclic method converge.)
 *
 * Everything is double precision; no blocking or reordering beyond the plain
 * cyclic order.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Inner product with eight interleaved partial sums (a fixed summation order
 * that the compiler can vectorise without reassociating). */
static double dot(int m, const double *restrict x, const double *restrict y) {
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int i = 0;
  for (; i + 8 <= m; i += 8)
    for (int l = 0; l < 8; ++l) acc[l] += x[i + l] * y[i + l];
  double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  for (; i < m; ++i) s += x[i] * y[i];
  return s;
}

static void rotate(int m, double *restrict x, double *restrict y, double c, double s) {
  for (int i = 0; i < m; ++i) {
    const double xi = x[i], yi = y[i];
    x[i] = c * xi - s * yi;
    y[i] = s * xi + c * yi;
  }
}

/*
 * A: m x n column-major (leading dimension m), m >= n >= 1; overwritten by U
 *    (m x n, orthonormal columns for nonzero singular values, zero columns
 *    otherwise).
 * V: n x n column-major output (right singular vectors).
 * sigma: n outputs, descending.
 * tol: orthogonality threshold (1e-15 is the oracle's setting).
 * max_sweeps: cap; returns the number of sweeps used, or -1 if the cap was hit.
 */
int oracle_jacobi_svd(int m, int n, double *A, double *V, double *sigma,
                      double tol, int max_sweeps) {
  if (m < n || n < 1) return -2;
  memset(V, 0, sizeof(double) * (size_t)n * (size_t)n);
  for (int j = 0; j < n; ++j) V[(size_t)j * n + j] = 1.0;

  int sweeps = 0;
  for (;;) {
    long rotations = 0;
    for (int p = 0; p < n - 1; ++p) {
      double *ap = A + (size_t)p * m;
      for (int q = p + 1; q < n; ++q) {
        double *aq = A + (size_t)q * m;
        const double alpha = dot(m, ap, ap);
        const double beta = dot(m, aq, aq);
        const double gamma = dot(m, ap, aq);
        if (gamma == 0.0 || fabs(gamma) <= tol * sqrt(alpha) * sqrt(beta)) continue;
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double s = c * t;
        rotate(m, ap, aq, c, s);
        rotate(n, V + (size_t)p * n, V + (size_t)q * n, c, s);
        ++rotations;
      }
    }
    ++sweeps;
    if (rotations == 0) break;
    if (sweeps >= max_sweeps) return -1;
  }

  /* singular values are the column norms; normalise the columns */
  for (int j = 0; j < n; ++j) {
    double *aj = A + (size_t)j * m;
    const double nrm = sqrt(dot(m, aj, aj));
    sigma[j] = nrm;
    if (nrm > 1e-300) {
      for (int i = 0; i < m; ++i) aj[i] /= nrm;
    } else {
      sigma[j] = 0.0;
      for (int i = 0; i < m; ++i) aj[i] = 0.0;
    }
  }

  /* sort descending (selection sort on indices; n is small enough) */
  double *tmp = (double *)malloc(sizeof(double) * (size_t)(m > n ? m : n));
  if (!tmp) return -3;
  for (int j = 0; j < n; ++j) {
    int best = j;
    for (int k = j + 1; k < n; ++k)
      if (sigma[k] > sigma[best]) best = k;
    if (best != j) {
      const double s = sigma[j]; sigma[j] = sigma[best]; sigma[best] = s;
      memcpy(tmp, A + (size_t)j * m, sizeof(double) * m);
      memcpy(A + (size_t)j * m, A + (size_t)best * m, sizeof(double) * m);
      memcpy(A + (size_t)best * m, tmp, sizeof(double) * m);
      memcpy(tmp, V + (size_t)j * n, sizeof(double) * n);
      memcpy(V + (size_t)j * n, V + (size_t)best * n, sizeof(double) * n);
      memcpy(V + (size_t)best * n, tmp, sizeof(double) * n);
    }
  }
  free(tmp);
  return sweeps;
}
