#include "dense_host.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace svt {

namespace {

double dot(const double *a, const double *b, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

}  // namespace

void orth_columns(double *Z, int64_t rows, int cols) {
  for (int j = 0; j < cols; ++j) {
    double *zj = Z + (int64_t)j * rows;
    const double before = std::sqrt(dot(zj, zj, rows));
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < j; ++i) {
        const double *qi = Z + (int64_t)i * rows;
        const double c = dot(qi, zj, rows);
        for (int64_t t = 0; t < rows; ++t) zj[t] -= c * qi[t];
      }
    const double nrm = std::sqrt(dot(zj, zj, rows));
    // a column left with no more than rounding of what it had lies in the
    // span of the earlier ones
    const bool keep = nrm > 0.0 && nrm > 1e-13 * before;
    const double inv = keep ? 1.0 / nrm : 0.0;
    for (int64_t t = 0; t < rows; ++t) zj[t] *= inv;
  }
}

bool jacobi_svd_tall(const double *W, int64_t rows, int cols, std::vector<double> &sigma, std::vector<double> &Vw,
                     std::vector<double> &Uw) {
  std::vector<double> A(W, W + rows * (int64_t)cols);
  std::vector<double> U((size_t)cols * cols, 0.0);
  for (int j = 0; j < cols; ++j) U[(size_t)j * cols + j] = 1.0;
  const double eps = 1e-15;
  bool settled = false;
  for (int sweep = 0; sweep < 60 && !settled; ++sweep) {
    settled = true;
    for (int p = 0; p < cols - 1; ++p)
      for (int q = p + 1; q < cols; ++q) {
        double *ap = A.data() + (int64_t)p * rows, *aq = A.data() + (int64_t)q * rows;
        const double alpha = dot(ap, ap, rows), beta = dot(aq, aq, rows), gamma = dot(ap, aq, rows);
        if (gamma == 0.0 || std::fabs(gamma) <= eps * std::sqrt(alpha * beta)) continue;
        settled = false;
        const double zeta = (beta - alpha) / (2.0 * gamma);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int64_t i = 0; i < rows; ++i) {
          const double x = ap[i], y = aq[i];
          ap[i] = c * x - s * y;
          aq[i] = s * x + c * y;
        }
        double *up = U.data() + (size_t)p * cols, *uq = U.data() + (size_t)q * cols;
        for (int i = 0; i < cols; ++i) {
          const double x = up[i], y = uq[i];
          up[i] = c * x - s * y;
          uq[i] = s * x + c * y;
        }
      }
  }
  std::vector<double> nrm(cols);
  for (int j = 0; j < cols; ++j) {
    const double *aj = A.data() + (int64_t)j * rows;
    nrm[(size_t)j] = std::sqrt(dot(aj, aj, rows));
  }
  std::vector<int> order(cols);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nrm[(size_t)a] > nrm[(size_t)b]; });
  sigma.assign(cols, 0.0);
  Vw.assign((size_t)rows * cols, 0.0);
  Uw.assign((size_t)cols * cols, 0.0);
  for (int k = 0; k < cols; ++k) {
    const int j = order[(size_t)k];
    const double sg = nrm[(size_t)j];
    sigma[(size_t)k] = sg;
    const double *aj = A.data() + (int64_t)j * rows;
    double *vk = Vw.data() + (int64_t)k * rows;
    if (sg > 0.0)
      for (int64_t i = 0; i < rows; ++i) vk[i] = aj[i] / sg;
    std::copy(U.begin() + (size_t)j * cols, U.begin() + (size_t)(j + 1) * cols, Uw.begin() + (size_t)k * cols);
  }
  return settled;
}

}  // namespace svt
